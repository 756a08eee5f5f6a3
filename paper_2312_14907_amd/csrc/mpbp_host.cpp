// mpbp_host.cpp - the C-ABI of include/mpbp.h: plan creation and validation, the
// integer tables of the shift and projection operators of eq. (2), workspace
// ownership, and the enqueueing of the device kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/mpbp.h"
#include "mpbp_kernels.hpp"
#include "mpbp_launch.hpp"
#include "mpbp_plain.hpp"
#include "mpbp_unwrap.hpp"

using mpbp::PeakDev;

namespace {

thread_local std::string g_err;

mpbp_status fail(mpbp_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

mpbp_status hip_fail(hipError_t e, const char* what) {
  return fail(MPBP_ERR_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// MPBP_TRACE=1 in the environment: one line per plan choice on stderr (geometry, size
// classes and their launch parameters, workspace, autotuner and cache choices, graph
// captures).
bool trace_on() {
  static const bool on = [] {
    const char* v = std::getenv("MPBP_TRACE");
    return v && *v && std::strcmp(v, "0") != 0;
  }();
  return on;
}

void trace(const char* fmt, ...) {
  if (!trace_on()) return;
  char buf[768];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  std::fprintf(stderr, "mpbp: %s\n", buf);
  std::fflush(stderr);
}

bool supported_det(int d) {
  return d == 32 || d == 64 || d == 96 || d == 128 || d == 150 || d == 192 || d == 256;
}

constexpr int kMaxPeaks = 16;
constexpr int kMaxLds = 160 * 1024;
constexpr size_t kMaxGraphs = 8;   // captured full-batch calls kept per plan
constexpr int kRedParts = 1024;    // block partials of mpbp_norm2

// What a captured full-batch call depends on besides the plan: the call kind, the
// caller's buffer addresses and the launch options.  A replay reads and writes the
// buffers at these addresses, so equal keys mean equal work.
struct GraphKey {
  int kind = 0;                    // 0: mpbp_forward, 1: mpbp_loss_grad
  int xcd = 0;
  const void* ptr[11] = {};
  bool operator==(const GraphKey& o) const {
    return kind == o.kind && xcd == o.xcd && std::memcmp(ptr, o.ptr, sizeof(ptr)) == 0;
  }
};

struct GraphEntry {
  GraphKey key;
  hipGraphExec_t exec = nullptr;
  uint64_t used = 0;
};

// The fixed device workspace of mpbp_loss_grad_static (callers that cannot allocate).
// One copy per GPU, at its own address on each: host code never uses the array's name
// as an address, only the pointer hipGetSymbolAddress returns with that device current.
constexpr size_t kStaticScratchBytes = size_t(MPBP_STATIC_SCRATCH_BYTES);
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxScratchDevices] = {};   // per device, set once at plan creation

}  // namespace

static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

// Look up this device's copy of the array (the device must be current).  Called by
// mpbp_plan_create for device plans, once per device.
mpbp_status scratch_setup(int device) {
  if (device >= kMaxScratchDevices) return MPBP_OK;   // the static variant then reports it
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return MPBP_OK;
  void* ptr = nullptr;
  hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !ptr) return hip_fail(e != hipSuccess ? e : hipErrorInvalidSymbol, "hipGetSymbolAddress(scratch)");
  g_scratch[device] = ptr;
  return MPBP_OK;
}

void* scratch_of(int device) {
  if (device < 0 || device >= kMaxScratchDevices) return nullptr;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  return g_scratch[device];
}

}  // namespace

struct mpbp_plan_t {
  int device = -1;
  int nz = 0, ny = 0, nx = 0, np = 0, M = 0;
  long long nvox = 0;
  long long tied = 0;              // ny * nx under MPBP_Z_TIED, else 0
  int probe3 = 0;                  // MPBP_PROBE_3D: probe [M][nz][np][np]
  int linear = 0;                  // MPBP_SHEAR_LINEAR: fractional exit-beam offsets
  std::vector<float> shw;          // [M][nz][2] their fractions (MPBP_SHEAR_LINEAR)
  int mapped = 0;                  // MPBP_DETECTOR_MAP: R interpolates in each detector frame
  std::vector<float> mapz;         // [M][nz][2] window centre of slice z, footprint coordinates
  std::vector<int32_t> color_list; // the frames grouped by colour (no two frames of one
  std::vector<int32_t> color_off;  // peak and colour overlap), and each colour's offset
  int64_t F = 0, ylen = 0;
  std::vector<mpbp_peak> peaks;
  std::vector<PeakDev> pdev;
  std::vector<int32_t> scan;     // [F][2]
  std::vector<int32_t> shear;    // [M][nz][2]
  std::vector<int64_t> y_off;    // [M+1]
  std::vector<int32_t> peak_of;  // [F]
  std::vector<int32_t> order;    // processing order of the full batch
  // Frames of one detector size D and smallest footprint bound `key`, with the launch
  // parameters in use (compiled footprint bound FB >= key, projection depth G, XCD order).
  struct SizeClass {
    int D, key, begin, count;
    int fy, fx;                        // largest footprint over the class's peaks
    int FB, G, xcd;                    // G: object slices in flight per lane of the projection
    int lds_fwd, lds_grad;             // dynamic LDS of the frame kernel
    double tuned_us;                   // autotuned launch time (0: not tuned)
  };
  std::vector<SizeClass> classes;      // full batch: frames of one detector size, in `order`
  std::vector<SizeClass> sub_classes;  // the same for the last staged minibatch (capacity reserved)
  std::vector<unsigned char> seen;     // [F] duplicate check of a staged list (sized once)
  int grad_batch = mpbp::kDefaultGradBatch;
  int runs = 1;                        // project and back-project per run of equal exit-beam
                                       // offset where it applies (one probe, rounded offsets)
  std::vector<int32_t> zrun;           // [M][nz] run of each slice
  std::vector<int32_t> roff;           // [M][nz][2] footprint offset of run k
  int lds_runs = 0;
  int grad_tile = mpbp::kDefaultGradTileX;
  double grad_tuned_us = 0.0;
  std::string tune_source = "default";
  std::string tune_report;             // candidates timed by the last mpbp_autotune
  int lds_fwd = 0, lds_grad_frame = 0, lds_grad = 0;
  int lds_project[9] = {0};        // projection kernel, per projection depth
  int maxspan_y = 0, maxspan_x = 0;
  int max_cand = 0;
  // gradient tile grids, per compiled tile width: origin (<= 0) and tile counts
  struct GradTiling { int tx, ox, oy, nx, ny; };
  std::vector<GradTiling> tilings;
  int max_tiles = 0;
  int max_parts = 0;                   // alpha partials: per tile, or per chain-rule workgroup
  int acc_pix = 0;                     // projection accumulator: largest fy * fx (multiple of 4)
  int n_runs = 0;                      // runs over all peaks
  long long slots_cplx = 0;
  // options
  int path = 0, graph = 1, xcd = 1;
  // device buffers
  PeakDev* d_peaks = nullptr;
  int* d_scan = nullptr;
  int* d_peak_of = nullptr;
  int* d_shear = nullptr;
  int* d_zrun = nullptr;           // [M][nz] (the run gather of the gradient kernel)
  int* d_roff = nullptr;           // [M][nz][2]
  float* d_shw = nullptr;          // [M][nz][2] fractional offsets (MPBP_SHEAR_LINEAR)
  float* d_mapz = nullptr;         // [M][nz][2] (MPBP_DETECTOR_MAP)
  int* d_color_list = nullptr;     // [F] (MPBP_DETECTOR_MAP)
  int* d_order = nullptr;          // full-batch processing order
  int* d_list = nullptr;           // caller's list (subset calls)
  int* d_list_sorted = nullptr;    // the caller's list grouped by detector size
  unsigned char* d_active = nullptr;     // per-frame minibatch mask (subset calls)
  unsigned char* d_active_all = nullptr; // all ones
  unsigned* d_dbg = nullptr;       // status word of the device bounds checks (debug library)
  float* d_obj = nullptr;
  float* d_slots = nullptr;        // exit waves (k_project -> k_frames)
  float* d_gslots = nullptr;       // footprint gradients (k_frames -> the back-projection)
  double* d_floss = nullptr;
  double* d_apart = nullptr;
  double* d_red = nullptr;         // sum-of-squares partials (kRedParts)
  float* d_tw = nullptr;           // twiddle tables of all peaks
  const float* d_bg = nullptr;     // caller's background b of eq. (2) (mpbp_set_background)
  std::vector<float> tw;
  int* h_list = nullptr;           // pinned staging of the caller's list
  hipEvent_t staged = nullptr;
  bool staged_pending = false;
  mpbp::PlainWork plain;
  // stage timing (MPBP_OPT_PROFILE)
  int profile = 0;
  std::vector<hipEvent_t> ev_pool;
  std::vector<std::pair<int, std::pair<hipEvent_t, hipEvent_t>>> ev_pending;
  size_t ev_used = 0;
  double stage_ms[MPBP_NUM_STAGES] = {0};
  int64_t stage_n[MPBP_NUM_STAGES] = {0};
  // unwrap projector workspace (allocated by the first mpbp_unwrap_project call)
  mpbp::UnwrapArgs uw{};
  void* d_uw = nullptr;
  int* h_uw_err = nullptr;         // pinned copy of the device consistency flag
  // captured full-batch calls (MPBP_OPT_GRAPH)
  std::vector<GraphEntry> graphs;
  uint64_t graph_clock = 0;
  hipStream_t cap = nullptr;              // capture stream
  std::vector<hipStream_t> forks;         // one per extra size class
  std::vector<hipEvent_t> joins;
  hipEvent_t fork_ev = nullptr;
};

namespace {

template <typename T>
hipError_t dalloc(T** p, size_t n) {
  return hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T));
}

void clear_graphs(mpbp_plan_t* p) {
  if (p->graphs.empty()) return;
  (void)hipDeviceSynchronize();
  for (auto& g : p->graphs) (void)hipGraphExecDestroy(g.exec);
  p->graphs.clear();
}

void free_device(mpbp_plan_t* p) {
  if (p->device < 0) return;
  (void)hipSetDevice(p->device);
  (void)hipDeviceSynchronize();
  clear_graphs(p);
  for (hipStream_t f : p->forks) (void)hipStreamDestroy(f);
  for (hipEvent_t e : p->joins) (void)hipEventDestroy(e);
  if (p->fork_ev) (void)hipEventDestroy(p->fork_ev);
  if (p->cap) (void)hipStreamDestroy(p->cap);
  (void)hipFree(p->d_peaks);
  (void)hipFree(p->d_scan);
  (void)hipFree(p->d_peak_of);
  (void)hipFree(p->d_shear);
  (void)hipFree(p->d_zrun);
  (void)hipFree(p->d_roff);
  (void)hipFree(p->d_shw);
  (void)hipFree(p->d_mapz);
  (void)hipFree(p->d_color_list);
  (void)hipFree(p->d_order);
  (void)hipFree(p->d_list);
  (void)hipFree(p->d_list_sorted);
  (void)hipFree(p->d_active);
  (void)hipFree(p->d_active_all);
  (void)hipFree(p->d_dbg);
  (void)hipFree(p->d_obj);
  (void)hipFree(p->d_slots);
  (void)hipFree(p->d_gslots);
  (void)hipFree(p->d_floss);
  (void)hipFree(p->d_apart);
  (void)hipFree(p->d_red);
  (void)hipFree(p->d_tw);
  for (hipEvent_t e : p->ev_pool) (void)hipEventDestroy(e);
  if (p->h_list) (void)hipHostFree(p->h_list);
  if (p->staged) (void)hipEventDestroy(p->staged);
  mpbp::plain_free(&p->plain);
  (void)hipFree(p->d_uw);
  if (p->h_uw_err) (void)hipHostFree(p->h_uw_err);
}

// MPBP_DETECTOR_MAP: the peak's map M and its inverse, the footprint (the bounding box,
// over the slices, of the images of the support's corners (-1, -1) .. (n, n) taken
// relative to the window centre c + n/2, moved by the slice offset (z - nz/2) t, and
// rounded outwards: the interpolation reaches one sample beyond the support), and each
// slice's window centre in footprint coordinates (mapz [nz][2]).
mpbp_status map_footprint(const mpbp_peak& k, int m, int np, int nz, int zref, PeakDev& d, float* mapz) {
  const double* M = k.map;
  for (int i = 0; i < 4; ++i)
    if (!std::isfinite(M[i]) || std::fabs(M[i]) > 1e3)
      return fail(MPBP_ERR_INVALID, "peak %d: detector map not finite or above 1e3", m);
  const double det = M[0] * M[3] - M[1] * M[2];
  if (!(std::fabs(det) > 1e-6)) return fail(MPBP_ERR_INVALID, "peak %d: detector map is singular", m);
  const double inv[4] = {M[3] / det, -M[1] / det, -M[2] / det, M[0] / det};
  const double centre = (double)((k.det - np) / 2) + 0.5 * np;
  double lo[2] = {1e300, 1e300}, hi[2] = {-1e300, -1e300};
  for (int z = 0; z < nz; ++z) {
    const double oy = (double)(z - zref) * k.shear[0], ox = (double)(z - zref) * k.shear[1];
    for (double ca : {-1.0, (double)np})
      for (double cb : {-1.0, (double)np}) {
        const double ya = ca - 0.5 * np, yb = cb - 0.5 * np;
        const double q[2] = {M[0] * ya + M[1] * yb + centre + oy, M[2] * ya + M[3] * yb + centre + ox};
        for (int c = 0; c < 2; ++c) {
          lo[c] = std::min(lo[c], q[c]);
          hi[c] = std::max(hi[c], q[c]);
        }
      }
  }
  const double qlo[2] = {std::floor(lo[0]), std::floor(lo[1])}, qhi[2] = {std::ceil(hi[0]), std::ceil(hi[1])};
  for (int c = 0; c < 2; ++c)
    if (qlo[c] < 0 || qhi[c] > k.det - 1)
      return fail(MPBP_ERR_FOOTPRINT, "peak %d: mapped support leaves the %dx%d window", m, k.det, k.det);
  d.r0 = (int)qlo[0];
  d.c0 = (int)qlo[1];
  d.fy = (int)(qhi[0] - qlo[0]) + 1;
  d.fx = (int)(qhi[1] - qlo[1]) + 1;
  d.spany = std::max(0, d.fy - np);
  d.spanx = std::max(0, d.fx - np);
  for (int i = 0; i < 4; ++i) {
    d.mm[i] = (float)M[i];
    d.mi[i] = (float)inv[i];
  }
  for (int z = 0; z < nz; ++z) {
    mapz[2 * z] = (float)(centre + (double)(z - zref) * k.shear[0] - d.r0);
    mapz[2 * z + 1] = (float)(centre + (double)(z - zref) * k.shear[1] - d.c0);
  }
  return MPBP_OK;
}

// Build tables and per-peak constants on the host; validate the problem.
mpbp_status build_tables(const mpbp_problem* pr, mpbp_plan_t* p) {
  if (!pr) return fail(MPBP_ERR_INVALID, "problem is NULL");
  if (pr->flags & ~(uint32_t)(MPBP_Z_TIED | MPBP_PROBE_3D | MPBP_SHEAR_LINEAR | MPBP_DETECTOR_MAP))
    return fail(MPBP_ERR_INVALID,
                "unknown flags 0x%x (MPBP_Z_TIED, MPBP_PROBE_3D, MPBP_SHEAR_LINEAR and MPBP_DETECTOR_MAP are defined)",
                pr->flags);
  if ((pr->flags & MPBP_DETECTOR_MAP) && (pr->flags & MPBP_SHEAR_LINEAR))
    return fail(MPBP_ERR_INVALID, "MPBP_DETECTOR_MAP already interpolates the exit-beam offsets: "
                "MPBP_SHEAR_LINEAR does not apply");
  if (pr->nz < 1 || pr->ny < 1 || pr->nx < 1)
    return fail(MPBP_ERR_SHAPE, "object grid must be positive (nz=%d ny=%d nx=%d)", pr->nz, pr->ny, pr->nx);
  if (pr->probe_n < 1) return fail(MPBP_ERR_SHAPE, "probe_n must be positive (%d)", pr->probe_n);
  if (pr->probe_n * pr->probe_n > mpbp::kProjE * mpbp::kFrameThreads)
    return fail(MPBP_ERR_UNSUPPORTED, "probe_n %d above the supported 32", pr->probe_n);
  if (pr->n_peaks < 1 || pr->n_peaks > kMaxPeaks)
    return fail(MPBP_ERR_SHAPE, "n_peaks must be in [1, %d] (got %d)", kMaxPeaks, pr->n_peaks);
  if (!pr->peaks) return fail(MPBP_ERR_INVALID, "peaks is NULL");
  const long long nvox = (long long)pr->nz * pr->ny * pr->nx;
  if (nvox * pr->n_peaks > (1LL << 40)) return fail(MPBP_ERR_SHAPE, "object grid too large");
  if (3 * nvox >= (1LL << 32)) return fail(MPBP_ERR_UNSUPPORTED, "3 * nz * ny * nx must be below 2^32");
  if (pr->nz > 4096) return fail(MPBP_ERR_SHAPE, "nz too large (%d)", pr->nz);

  p->nz = pr->nz; p->ny = pr->ny; p->nx = pr->nx; p->np = pr->probe_n; p->M = pr->n_peaks;
  p->nvox = nvox;
  p->tied = (pr->flags & MPBP_Z_TIED) ? (long long)pr->ny * pr->nx : 0;
  p->probe3 = (pr->flags & MPBP_PROBE_3D) ? 1 : 0;
  p->linear = (pr->flags & MPBP_SHEAR_LINEAR) ? 1 : 0;
  p->mapped = (pr->flags & MPBP_DETECTOR_MAP) ? 1 : 0;
  p->mapz.assign((size_t)pr->n_peaks * pr->nz * 2, 0.f);
  p->peaks.assign(pr->peaks, pr->peaks + pr->n_peaks);
  p->pdev.assign(p->M, PeakDev{});
  p->shear.assign((size_t)p->M * p->nz * 2, 0);
  p->shw.assign((size_t)p->M * p->nz * 2, 0.f);
  p->zrun.assign((size_t)p->M * p->nz, 0);
  p->roff.assign((size_t)p->M * p->nz * 2, 0);
  p->y_off.assign(p->M + 1, 0);
  p->scan.clear();
  p->peak_of.clear();
  p->tw.clear();
  p->acc_pix = 0;
  const int np = p->np;
  const int zref = p->nz / 2;
  long long slot = 0;
  int n_runs = 0;
  for (int m = 0; m < p->M; ++m) {
    const mpbp_peak& k = p->peaks[m];
    for (int c = 0; c < 3; ++c)
      if (!std::isfinite(k.g[c])) return fail(MPBP_ERR_INVALID, "peak %d: G not finite", m);
    for (int c = 0; c < 2; ++c)
      if (!std::isfinite(k.shear[c]) || std::fabs(k.shear[c]) > 1e6)
        return fail(MPBP_ERR_INVALID, "peak %d: shear not finite", m);
    if (!supported_det(k.det))
      return fail(MPBP_ERR_SHAPE, "peak %d: detector size %d not in {32,64,96,128,150,192,256}", m, k.det);
    if (np > k.det) return fail(MPBP_ERR_FOOTPRINT, "peak %d: probe support %d > window %d", m, np, k.det);
    if (k.scan_n[0] < 1 || k.scan_n[1] < 1)
      return fail(MPBP_ERR_SHAPE, "peak %d: raster must be positive (%d x %d)", m, k.scan_n[0], k.scan_n[1]);
    if (k.scan_step[0] < 1 || k.scan_step[1] < 1)
      return fail(MPBP_ERR_SHAPE, "peak %d: raster step must be positive", m);
    if ((long long)k.scan_n[0] * k.scan_n[1] > (1LL << 24))
      return fail(MPBP_ERR_SHAPE, "peak %d: raster too large", m);
    // shear offsets s_m(z) = round-half-away((z - nz/2) * t_m); under MPBP_SHEAR_LINEAR
    // the floor of (z - nz/2) * t_m and its fraction (the slice also reaches s + 1)
    int lo[2] = {1 << 30, 1 << 30}, hi[2] = {-(1 << 30), -(1 << 30)};
    for (int z = 0; z < p->nz; ++z) {
      for (int c = 0; c < 2; ++c) {
        const double t = (double)(z - zref) * k.shear[c];
        const double v = p->linear ? std::floor(t) : std::round(t);
        int s = (int)v;
        p->shear[((size_t)m * p->nz + z) * 2 + c] = s;
        if (p->linear) p->shw[((size_t)m * p->nz + z) * 2 + c] = (float)(t - v);
        lo[c] = std::min(lo[c], s);
        hi[c] = std::max(hi[c], s + p->linear);
      }
    }
    const int cw = (k.det - np) / 2;
    for (int c = 0; c < 2 && !p->mapped; ++c)
      if (cw + lo[c] < 0 || cw + np - 1 + hi[c] > k.det - 1)
        return fail(MPBP_ERR_FOOTPRINT, "peak %d: sheared support leaves the %dx%d window", m, k.det, k.det);
    PeakDev& d = p->pdev[m];
    d.D = k.det;
    d.L = mpbp::frame_chunk_len(k.det);
    d.R = k.det / d.L;
    d.c = cw;
    d.miny = lo[0]; d.minx = lo[1];
    d.spany = hi[0] - lo[0]; d.spanx = hi[1] - lo[1];
    d.r0 = cw + lo[0]; d.c0 = cw + lo[1];
    d.fy = np + d.spany; d.fx = np + d.spanx;
    if (p->mapped) {
      const mpbp_status st = map_footprint(k, m, np, p->nz, zref, d, &p->mapz[(size_t)m * p->nz * 2]);
      if (st != MPBP_OK) return st;
    }
    // runs of consecutive slices with equal offsets, and each run's footprint offset
    for (int z = 0, k = -1; z < p->nz; ++z) {
      const int* sz = &p->shear[((size_t)m * p->nz + z) * 2];
      if (z == 0 || sz[0] != sz[-2] || sz[1] != sz[-1]) {
        ++k;
        p->roff[((size_t)m * p->nz + k) * 2] = sz[0] - lo[0];
        p->roff[((size_t)m * p->nz + k) * 2 + 1] = sz[1] - lo[1];
      }
      p->zrun[(size_t)m * p->nz + z] = k;
      d.nruns = k + 1;
    }
    if (p->mapped) {
      // the detector-map back-projection sums the frames per slice into the objects'
      // buffer, [M][nz][ny][nx]: its chain rule reads slice z of peak m as "run" m nz + z
      for (int z = 0; z < p->nz; ++z) p->zrun[(size_t)m * p->nz + z] = z;
      d.nruns = p->nz;
    }
    d.run_base = n_runs;
    n_runs += d.nruns;
    p->n_runs = n_runs;
    if (d.fy * d.fx > mpbp::kProjMaxPix)
      return fail(MPBP_ERR_UNSUPPORTED, "peak %d: footprint %dx%d above %d pixels", m, d.fy, d.fx,
                  mpbp::kProjMaxPix);
    p->acc_pix = std::max(p->acc_pix, (d.fy * d.fx + 3) & ~3);
    d.fxp = d.fx | 1;
    d.rows = k.scan_n[0]; d.cols = k.scan_n[1];
    d.nfr = d.rows * d.cols;
    d.sy = k.scan_step[0]; d.sx = k.scan_step[1];
    d.oy = k.scan_origin[0]; d.ox = k.scan_origin[1];
    d.frame_base = (int)p->F;
    d.y_off = p->y_off[m];
    d.slot_off = slot;
    d.gx = (float)k.g[0]; d.gy = (float)k.g[1]; d.gz = (float)k.g[2];
    d.tw_off = (long long)(p->tw.size() / 2);
    mpbp::frame_twiddles(d.D, d.fy, p->tw);
    d.lds_bytes = mpbp::frame_lds_bytes(d.D, d.fy, d.fx, d.fxp, true);
    if (d.lds_bytes > kMaxLds)
      return fail(MPBP_ERR_UNSUPPORTED, "peak %d: footprint %dx%d needs %d B of LDS", m, d.fy, d.fx, d.lds_bytes);
    p->lds_grad_frame = std::max(p->lds_grad_frame, d.lds_bytes);
    p->lds_fwd = std::max(p->lds_fwd, mpbp::frame_lds_bytes(d.D, d.fy, d.fx, d.fxp, false));
    p->maxspan_y = std::max(p->maxspan_y, d.spany);
    p->maxspan_x = std::max(p->maxspan_x, d.spanx);
    slot += (long long)d.nfr * d.fy * d.fx;
    for (int iy = 0; iy < d.rows; ++iy)
      for (int ix = 0; ix < d.cols; ++ix) {
        p->scan.push_back(d.oy + iy * d.sy);
        p->scan.push_back(d.ox + ix * d.sx);
        p->peak_of.push_back(m);
      }
    p->F += d.nfr;
    if (p->F > (1LL << 30)) return fail(MPBP_ERR_SHAPE, "too many frames");
    p->y_off[m + 1] = p->y_off[m] + (int64_t)d.nfr * k.det * k.det;
  }
  p->ylen = p->y_off[p->M];
  p->slots_cplx = slot;
  p->max_cand = 0;
  p->tilings.clear();
  p->max_tiles = 0;
  for (int tx : mpbp::kGradTileXs) {
    const int ty = mpbp::kGradTile / tx;
    for (const auto& d : p->pdev) {
      const int cy = std::min(d.rows, (ty + np - 2) / d.sy + 2);
      const int cx = std::min(d.cols, (tx + np - 2) / d.sx + 2);
      p->max_cand = std::max(p->max_cand, cy * cx);
    }
    // The 8 x 8 grid is aligned with the first peak's raster (tile edges on its frame
    // edges), so that with an 8-voxel step every voxel of a tile has the same frames;
    // the 16 x 4 grid starts at the object's corner.
    mpbp_plan_t::GradTiling t{tx, 0, 0, 0, 0};
    if (tx == 8) {
      const int rx = ((p->pdev[0].ox % tx) + tx) % tx, ry = ((p->pdev[0].oy % ty) + ty) % ty;
      t.ox = rx ? rx - tx : 0;
      t.oy = ry ? ry - ty : 0;
    }
    t.nx = (p->nx - t.ox + tx - 1) / tx;
    t.ny = (p->ny - t.oy + ty - 1) / ty;
    p->tilings.push_back(t);
    p->max_tiles = std::max(p->max_tiles, t.nx * t.ny);
  }
  p->lds_grad = mpbp::grad_lds_bytes(np, p->nz, p->maxspan_y, p->maxspan_x, p->max_cand, p->tied != 0, false);
  p->lds_runs = mpbp::grad_lds_bytes(np, p->nz, p->maxspan_y, p->maxspan_x, p->max_cand, p->tied != 0, true);
  for (int G : mpbp::kSlabDepths) p->lds_project[G] = mpbp::project_lds_bytes(np, G, p->nz, p->acc_pix);
  if (p->lds_project[mpbp::kDefaultSlab] > kMaxLds)
    return fail(MPBP_ERR_UNSUPPORTED, "projection needs %d B of LDS", p->lds_project[mpbp::kDefaultSlab]);
  if (p->lds_grad > kMaxLds || p->lds_runs > kMaxLds)
    return fail(MPBP_ERR_UNSUPPORTED, "gradient kernel needs %d B of LDS", std::max(p->lds_grad, p->lds_runs));
  // Full-batch processing order: larger windows first (they cost most), each peak's
  // frames in tiles of its raster.
  std::vector<int> pk(p->M);
  for (int m = 0; m < p->M; ++m) pk[m] = m;
  auto fb = [&](int m) {
    const PeakDev& d = p->pdev[m];
    return mpbp::frame_bound(d.D, std::max(d.fy, d.fx));
  };
  std::stable_sort(pk.begin(), pk.end(), [&](int a, int b) {
    if (p->pdev[a].D != p->pdev[b].D) return p->pdev[a].D > p->pdev[b].D;
    return fb(a) < fb(b);
  });
  p->order.clear();
  p->classes.clear();
  for (int m : pk) {
    const PeakDev& d = p->pdev[m];
    if (p->classes.empty() || p->classes.back().D != d.D || p->classes.back().key != fb(m)) {
      mpbp_plan_t::SizeClass c{};
      c.D = d.D;
      c.key = fb(m);
      c.begin = (int)p->order.size();
      c.FB = c.key;
      c.G = mpbp::kDefaultSlab;
      c.xcd = p->xcd;
      p->classes.push_back(c);
    }
    auto& c = p->classes.back();
    c.count += d.nfr;
    c.fy = std::max(c.fy, d.fy);
    c.fx = std::max(c.fx, d.fx);
    c.lds_fwd = std::max(c.lds_fwd, mpbp::frame_lds_bytes(d.D, d.fy, d.fx, d.fxp, false));
    c.lds_grad = std::max(c.lds_grad, mpbp::frame_lds_bytes(d.D, d.fy, d.fx, d.fxp, true));
    // frames in square tiles of the raster, tiles in row-major order: a run of
    // consecutive frames reads a compact patch of the object (it stays in the XCD's L2
    // while its neighbours are projected)
    constexpr int kOrderTile = 16;
    for (int ty = 0; ty < d.rows; ty += kOrderTile)
      for (int tx = 0; tx < d.cols; tx += kOrderTile)
        for (int iy = ty; iy < std::min(ty + kOrderTile, d.rows); ++iy)
          for (int ix = tx; ix < std::min(tx + kOrderTile, d.cols); ++ix)
            p->order.push_back(d.frame_base + iy * d.cols + ix);
  }
  p->seen.assign(p->F, 0);
  // MPBP_DETECTOR_MAP: the frames' colours for the back-projection.  Frame (iy, ix) of a
  // peak takes colour (iy mod cy) cx + (ix mod cx), cy = ceil(np / sy), cx = ceil(np / sx):
  // two frames of one peak and colour lie at least np apart along a raster axis, so their
  // windows do not overlap and one launch per colour adds each voxel's frames one at a
  // time, in colour order.
  p->color_list.clear();
  p->color_off.clear();
  if (p->mapped) {
    int nc = 0;
    for (const auto& d : p->pdev) nc = std::max(nc, ((np + d.sy - 1) / d.sy) * ((np + d.sx - 1) / d.sx));
    std::vector<std::vector<int32_t>> by((size_t)nc);
    for (const auto& d : p->pdev) {
      const int cy = (np + d.sy - 1) / d.sy, cx = (np + d.sx - 1) / d.sx;
      for (int iy = 0; iy < d.rows; ++iy)
        for (int ix = 0; ix < d.cols; ++ix) by[(size_t)((iy % cy) * cx + ix % cx)].push_back(d.frame_base + iy * d.cols + ix);
    }
    p->color_off.assign((size_t)nc + 1, 0);
    for (int c = 0; c < nc; ++c) {
      p->color_off[c + 1] = p->color_off[c] + (int)by[c].size();
      p->color_list.insert(p->color_list.end(), by[c].begin(), by[c].end());
    }
  }
  {
    const long long lanes = (long long)p->ny * p->nx * (p->tied ? 1 : (p->nz + mpbp::kBpZ - 1) / mpbp::kBpZ);
    p->max_parts = std::max<long long>(p->max_tiles, (lanes + mpbp::kBpThreads - 1) / mpbp::kBpThreads);
  }
  p->sub_classes.reserve(p->classes.size());
  return MPBP_OK;
}

mpbp_status ensure_capture_streams(mpbp_plan p);

mpbp_status alloc_device(mpbp_plan_t* p) {
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  e = mpbp::prepare_kernels();
  if (e != hipSuccess) return hip_fail(e, "kernel attributes");
#define ALLOC(ptr, n)                                                           \
  do {                                                                          \
    e = dalloc(&(ptr), (n));                                                    \
    if (e != hipSuccess) return fail(MPBP_ERR_NOMEM, "hipMalloc %s (%zu elements): %s", #ptr, \
                                     (size_t)(n), hipGetErrorString(e));        \
  } while (0)
  ALLOC(p->d_peaks, p->M);
  ALLOC(p->d_scan, p->F * 2);
  ALLOC(p->d_peak_of, p->F);
  ALLOC(p->d_shear, (size_t)p->M * p->nz * 2);
  ALLOC(p->d_shw, (size_t)p->M * p->nz * 2);
  ALLOC(p->d_mapz, (size_t)p->M * p->nz * 2);
  ALLOC(p->d_color_list, std::max<int64_t>(p->F, 1));
  ALLOC(p->d_zrun, (size_t)p->M * p->nz);
  ALLOC(p->d_roff, (size_t)p->M * p->nz * 2);
  ALLOC(p->d_order, p->F);
  ALLOC(p->d_list, p->F);
  ALLOC(p->d_list_sorted, p->F);
  ALLOC(p->d_active, p->F);
  ALLOC(p->d_active_all, p->F);
  ALLOC(p->d_dbg, 1);
  ALLOC(p->d_obj, (size_t)p->M * p->nvox * 2);
  ALLOC(p->d_slots, (size_t)p->slots_cplx * 2);
  ALLOC(p->d_gslots, (size_t)p->slots_cplx * 2);
  ALLOC(p->d_floss, p->F);
  ALLOC(p->d_apart, (size_t)p->max_parts * p->M);
  ALLOC(p->d_red, kRedParts);
  ALLOC(p->d_tw, p->tw.size());
#undef ALLOC
  e = hipHostMalloc((void**)&p->h_list, std::max<int64_t>(2 * p->F, 1) * sizeof(int), hipHostMallocDefault);
  if (e != hipSuccess) return fail(MPBP_ERR_NOMEM, "hipHostMalloc: %s", hipGetErrorString(e));
  e = hipEventCreateWithFlags(&p->staged, hipEventDisableTiming);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  e = hipMemcpy(p->d_peaks, p->pdev.data(), p->M * sizeof(PeakDev), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_scan, p->scan.data(), p->scan.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_peak_of, p->peak_of.data(), p->peak_of.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_shear, p->shear.data(), p->shear.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_shw, p->shw.data(), p->shw.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_mapz, p->mapz.data(), p->mapz.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e == hipSuccess && !p->color_list.empty())
    e = hipMemcpy(p->d_color_list, p->color_list.data(), p->color_list.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_zrun, p->zrun.data(), p->zrun.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_roff, p->roff.data(), p->roff.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_order, p->order.data(), p->order.size() * sizeof(int), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(p->d_tw, p->tw.data(), p->tw.size() * sizeof(float), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy tables");
  if (e == hipSuccess) e = hipMemset(p->d_dbg, 0, sizeof(unsigned));
  std::vector<unsigned char> ones(p->F, 1);
  e = hipMemcpy(p->d_active_all, ones.data(), p->F, hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy mask");
  e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "hipDeviceSynchronize");
  // the fork streams of concurrent size classes (direct launches and graph captures)
  return ensure_capture_streams(p);
}

// Validate and stage a caller's frame list; returns the number of listed frames.
mpbp_status stage_frames(mpbp_plan_t* p, const int32_t* frames, int64_t n, hipStream_t s,
                         bool need_mask, int* n_out) {
  if (!frames) {
    *n_out = (int)p->F;
    return MPBP_OK;
  }
  if (n < 0 || n > p->F) return fail(MPBP_ERR_INVALID, "n_frames %lld out of range [0, %lld]", (long long)n, (long long)p->F);
  // (no allocation here: the flags and the class list were sized at plan creation)
  std::fill(p->seen.begin(), p->seen.end(), (unsigned char)0);
  for (int64_t i = 0; i < n; ++i) {
    int f = frames[i];
    if (f < 0 || f >= p->F) return fail(MPBP_ERR_INVALID, "frame id %d out of range", f);
    if (p->seen[f]) return fail(MPBP_ERR_INVALID, "duplicate frame id %d", f);
    p->seen[f] = 1;
  }
  hipError_t e;
  if (p->staged_pending) {
    e = hipEventSynchronize(p->staged);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
  }
  std::memcpy(p->h_list, frames, (size_t)n * sizeof(int));
  // grouped by detector size in the order of the full-batch classes
  int* sorted = p->h_list + p->F;
  int pos = 0;
  p->sub_classes.clear();
  for (const auto& c : p->classes) {
    mpbp_plan_t::SizeClass sc = c;
    sc.begin = pos;
    for (int64_t i = 0; i < n; ++i)
      if (p->pdev[p->peak_of[frames[i]]].D == c.D &&
          mpbp::frame_bound(c.D, std::max(p->pdev[p->peak_of[frames[i]]].fy,
                                          p->pdev[p->peak_of[frames[i]]].fx)) == c.key)
        sorted[pos++] = frames[i];
    sc.count = pos - sc.begin;
    p->sub_classes.push_back(sc);
  }
  if (n > 0) {
    e = hipMemcpyAsync(p->d_list, p->h_list, (size_t)n * sizeof(int), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
      e = hipMemcpyAsync(p->d_list_sorted, sorted, (size_t)n * sizeof(int), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync frame list");
  }
  e = hipEventRecord(p->staged, s);
  if (e != hipSuccess) return hip_fail(e, "hipEventRecord");
  p->staged_pending = true;
  if (need_mask) {
    e = mpbp::launch_mark_active(p->d_active, p->F, p->d_list, (int)n, s);
    if (e != hipSuccess) return hip_fail(e, "mask kernel");
  }
  *n_out = (int)n;
  return MPBP_OK;
}

mpbp_status check_plan(mpbp_plan p) {
  if (!p) return fail(MPBP_ERR_INVALID, "plan is NULL");
  if (p->device < 0) return fail(MPBP_ERR_DEVICE, "host-only plan: compute calls need a device plan");
  hipError_t e = hipSetDevice(p->device);
  if (e != hipSuccess) return hip_fail(e, "hipSetDevice");
  return MPBP_OK;
}

// Stage timer: records an event pair around the enclosed launches when profiling.
struct StageTimer {
  mpbp_plan_t* p;
  int stage;
  hipStream_t s;
  hipEvent_t a = nullptr, b = nullptr;
  StageTimer(mpbp_plan_t* p_, int stage_, hipStream_t s_, bool on = true) : p(p_), stage(stage_), s(s_) {
    if (!on || !(p->profile == 1 || (p->profile == 2 && stage == MPBP_STAGE_FRAMES))) return;
    while (p->ev_pool.size() < p->ev_used + 2) {
      hipEvent_t e;
      if (hipEventCreate(&e) != hipSuccess) return;
      p->ev_pool.push_back(e);
    }
    a = p->ev_pool[p->ev_used];
    b = p->ev_pool[p->ev_used + 1];
    p->ev_used += 2;
    (void)hipEventRecord(a, s);
  }
  ~StageTimer() {
    if (!a) return;
    (void)hipEventRecord(b, s);
    p->ev_pending.push_back({stage, {a, b}});
  }
};

// Enqueue the per-frame kernel for every detector-size class of the call.  The classes
// after the first run on fork streams joined back into `s` (under graph capture the
// graph then holds them as parallel nodes): the classes write disjoint slots and frame
// losses.
// Each class runs the projection kernel (exit waves into the frames' slots), then the
// frame kernel.  Profiled direct launches instead run every class's projection first,
// then every class's frame kernel, each group under its stage timer (the classes of a
// group side by side).  The plan creates the fork streams with its device buffers.
hipError_t enqueue_frames(mpbp_plan p, const mpbp::FrameArgs& base, bool subset, bool grad, hipStream_t s,
                          bool branch = false, bool timed = true) {
  const auto& cls = subset ? p->sub_classes : p->classes;
  const int* list = subset ? p->d_list_sorted : p->d_order;
  auto class_args = [&](const mpbp_plan_t::SizeClass& c) {
    mpbp::FrameArgs a = base;
    a.list = list + c.begin;
    a.n_list = c.count;
    a.xcd = c.xcd;
    return a;
  };
  hipError_t e = hipSuccess;
  if (!branch && p->profile && timed) {
    // Profiled direct launches: every class's projection, then every class's frame
    // kernel, each stage under its timer.  With more than one class, the classes of a
    // stage run concurrently on the plan's fork streams, joined back into `s` before the
    // next stage (the GPU then fills one class's last partial wave of workgroups with
    // another's).
    int live = 0;
    for (const auto& c : cls) live += c.count > 0;
    const bool fork = live > 1 && p->forks.size() + 1 >= (size_t)live && p->joins.size() >= p->forks.size();
    auto stage = [&](int which, auto&& launch) {
      StageTimer t(p, which, s, timed);
      if (!fork) {
        for (const auto& c : cls)
          if (c.count && e == hipSuccess) e = launch(c, s);
        return;
      }
      if (e == hipSuccess) e = hipEventRecord(p->fork_ev, s);
      size_t k = 0;
      bool first = true;
      for (const auto& c : cls) {
        if (c.count == 0 || e != hipSuccess) continue;
        hipStream_t t2 = first ? s : p->forks[k];
        if (!first) e = hipStreamWaitEvent(t2, p->fork_ev, 0);
        if (e == hipSuccess) e = launch(c, t2);
        if (!first) {
          if (e == hipSuccess) e = hipEventRecord(p->joins[k], t2);
          if (e == hipSuccess) e = hipStreamWaitEvent(s, p->joins[k], 0);
          ++k;
        }
        first = false;
      }
    };
    stage(MPBP_STAGE_PROJECT, [&](const mpbp_plan_t::SizeClass& c, hipStream_t t2) {
      return mpbp::launch_project(c.G, class_args(c), p->lds_project[c.G], t2);
    });
    stage(MPBP_STAGE_FRAMES, [&](const mpbp_plan_t::SizeClass& c, hipStream_t t2) {
      return mpbp::launch_frames(c.D, c.FB, class_args(c), grad ? c.lds_grad : c.lds_fwd, t2);
    });
    return e;
  }
  // Otherwise (graph captures, unprofiled direct launches) each class's projection and
  // frame kernel form one chain on its own fork stream, so one class's projection
  // overlaps another's frame kernel.
  e = hipEventRecord(p->fork_ev, s);
  size_t k = 0;
  bool first = true;
  for (const auto& c : cls) {
    if (c.count == 0) continue;
    const mpbp::FrameArgs a = class_args(c);
    hipStream_t t = s;
    if (!first) {
      t = p->forks[k];
      if (e == hipSuccess) e = hipStreamWaitEvent(t, p->fork_ev, 0);
    }
    if (e == hipSuccess) e = mpbp::launch_project(c.G, a, p->lds_project[c.G], t);
    if (e == hipSuccess) e = mpbp::launch_frames(c.D, c.FB, a, grad ? c.lds_grad : c.lds_fwd, t);
    if (!first) {
      if (e == hipSuccess) e = hipEventRecord(p->joins[k], t);
      if (e == hipSuccess) e = hipStreamWaitEvent(s, p->joins[k], 0);
      ++k;
    }
    first = false;
    if (e != hipSuccess) return e;
  }
  return e;
}

// The per-call device workspace of the fused path: per-peak objects, exit-wave and
// gradient footprint slots, per-frame losses, per-tile alpha partials.  Normally the
// plan's own buffers; mpbp_loss_grad_static carves it from the library's fixed array.
struct Work {
  float* obj;
  float* slots;
  float* gslots;
  double* floss;
  double* apart;
};

Work plan_work(mpbp_plan p) { return {p->d_obj, p->d_slots, p->d_gslots, p->d_floss, p->d_apart}; }

// Projection and back-projection per run of equal exit-beam offset (one probe for all
// slices, rounded offsets): the objects are then stored as run sums.
bool uses_runs(const mpbp_plan_t* p) { return p->runs && !p->probe3 && !p->linear && !p->mapped; }

// The objects of eq. (1)/(3) into the workspace: per slice, or summed over each run.
hipError_t launch_objects(mpbp_plan p, const Work& w, const float* u, const float* chi, const float* alpha,
                          hipStream_t s) {
  if (uses_runs(p))
    return mpbp::launch_runsum(u, chi, alpha, p->d_peaks, p->M, p->nz, (long long)p->ny * p->nx, p->tied != 0,
                               p->d_zrun, w.obj, s);
  return mpbp::launch_object(u, chi, alpha, p->d_peaks, p->M, p->nvox, p->tied, w.obj, s);
}

mpbp::FrameArgs frame_args(mpbp_plan p, const Work& w, const float* y, const int* list, int n, float* mi,
                           int grad) {
  mpbp::FrameArgs a{};
  a.obj = w.obj;
  a.y = y;
  a.bg = p->d_bg;
  a.list = list;
  a.n_list = n;
  a.scan = p->d_scan;
  a.peak_of = p->d_peak_of;
  a.peaks = p->d_peaks;
  a.shear = p->d_shear;
  a.slots = w.slots;
  a.gslots = w.gslots;
  a.floss = w.floss;
  a.tw = p->d_tw;
  a.mi = mi;
  a.nz = p->nz; a.ny = p->ny; a.nx = p->nx; a.np = p->np;
  a.grad = grad;
  a.xcd = p->xcd;
  a.probe3 = p->probe3;
  a.shw = p->linear ? p->d_shw : nullptr;
  a.runs = uses_runs(p);
  a.acc_pix = p->acc_pix;
  a.n_runs = p->n_runs;
  a.dbg = p->d_dbg;
  a.roff = reinterpret_cast<const int2*>(p->d_roff);
  a.mapz = p->mapped ? reinterpret_cast<const float2*>(p->d_mapz) : nullptr;
  return a;
}

const mpbp_plan_t::GradTiling& grad_tiling(mpbp_plan p) {
  for (const auto& t : p->tilings)
    if (t.tx == p->grad_tile) return t;
  return p->tilings.front();
}

// Alpha partials the gradient launch leaves: one per voxel tile, or one per workgroup of
// the run chain rule.
int bp_parts(mpbp_plan p) {
  const long long lanes = (long long)p->ny * p->nx * (p->tied ? 1 : (p->nz + mpbp::kBpZ - 1) / mpbp::kBpZ);
  return (int)((lanes + mpbp::kBpThreads - 1) / mpbp::kBpThreads);
}

int grad_parts(mpbp_plan p) {
  if (p->mapped || uses_runs(p)) return bp_parts(p);
  return grad_tiling(p).nx * grad_tiling(p).ny;
}

mpbp::GradArgs grad_args(mpbp_plan p, const Work& w, const float* u, const float* chi, const float* alpha,
                         const float* probe, bool subset, float* grad_u, float* grad_chi) {
  mpbp::GradArgs g{};
  g.slots = w.gslots;
  g.active = subset ? p->d_active : p->d_active_all;
  g.all_active = subset ? 0 : 1;
  g.probe = probe;
  g.u = u; g.chi = chi; g.alpha = alpha;
  g.shear = p->d_shear;
  g.peaks = p->d_peaks;
  g.n_peaks = p->M;
  g.nz = p->nz; g.ny = p->ny; g.nx = p->nx; g.np = p->np;
  const auto& tl = grad_tiling(p);
  g.tiles_x = tl.nx; g.tiles_y = tl.ny;
  g.tile_ox = tl.ox; g.tile_oy = tl.oy;
  g.maxspan_y = p->maxspan_y; g.maxspan_x = p->maxspan_x;
  g.max_cand = p->max_cand;
  g.tied = p->tied != 0;
  g.probe3 = p->probe3;
  g.shw = p->linear ? p->d_shw : nullptr;
  g.runs = p->runs;
  g.rs = w.obj;          // the run sums' buffer: the forward projection is done with it
  g.nlat = (long long)p->ny * p->nx;
  g.n_runs = p->n_runs;
  g.dbg = p->d_dbg;
  g.zrun = p->d_zrun;
  g.roff = reinterpret_cast<const int2*>(p->d_roff);
  g.mapz = p->mapped ? reinterpret_cast<const float2*>(p->d_mapz) : nullptr;
  g.peak_of = p->d_peak_of;
  g.scan = p->d_scan;
  g.color_list = p->d_color_list;
  g.color_off = p->color_off.data();
  g.n_colors = p->color_off.empty() ? 0 : (int)p->color_off.size() - 1;
  g.map_pix = p->acc_pix;
  g.grad_u = grad_u; g.grad_chi = grad_chi;
  g.alpha_part = w.apart;
  return g;
}

// The batched fused path's launches of one mpbp_forward call.  `what` names the stage
// that failed.
hipError_t enqueue_forward(mpbp_plan p, const float* u, const float* chi, const float* alpha,
                           const float* probe, const float* y, const int* list, int n, bool subset,
                           float* model_intensity, hipStream_t s, bool branch, const char** what) {
  hipError_t e;
  const Work w = plan_work(p);
  {
    StageTimer t(p, MPBP_STAGE_OBJECT, s);
    e = launch_objects(p, w, u, chi, alpha, s);
  }
  if (e != hipSuccess) return *what = "object kernel", e;
  mpbp::FrameArgs a = frame_args(p, w, y, list, n, model_intensity, 0);
  a.probe = probe;
  e = enqueue_frames(p, a, subset, false, s, branch);
  if (e != hipSuccess) return *what = "frame kernel", e;
  return hipSuccess;
}

// The batched fused path's launches of one mpbp_loss_grad call, finalize excluded.
hipError_t enqueue_loss_grad(mpbp_plan p, const Work& w, const float* u, const float* chi, const float* alpha,
                             const float* probe, const float* y, const int* list, int n, bool subset,
                             float* grad_u, float* grad_chi, hipStream_t s, bool branch,
                             const char** what, bool timed = true) {
  hipError_t e;
  {
    StageTimer t(p, MPBP_STAGE_OBJECT, s, timed);
    e = launch_objects(p, w, u, chi, alpha, s);
  }
  if (e != hipSuccess) return *what = "object kernel", e;
  mpbp::FrameArgs a = frame_args(p, w, y, list, n, nullptr, 1);
  a.probe = probe;
  e = enqueue_frames(p, a, subset, true, s, branch, timed);
  if (e != hipSuccess) return *what = "frame kernel", e;
  const mpbp::GradArgs g = grad_args(p, w, u, chi, alpha, probe, subset, grad_u, grad_chi);
  {
    StageTimer t(p, MPBP_STAGE_GRAD, s, timed);
    e = mpbp::launch_grad(p->grad_batch, p->grad_tile, g, mpbp::grad_uses_runs(g) ? p->lds_runs : p->lds_grad, s);
  }
  if (e != hipSuccess) return *what = "gradient kernel", e;
  return hipSuccess;
}

// Full-batch fused calls are replayed from captured graphs unless profiling (which
// times each stage with events) or the plain path is selected.
bool use_graph(mpbp_plan p, const int32_t* frames) {
  return p->graph && !p->profile && p->path == 0 && frames == nullptr;
}

mpbp_status ensure_capture_streams(mpbp_plan p) {
  hipError_t e = hipSuccess;
  if (!p->cap) e = hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking);
  if (e == hipSuccess && !p->fork_ev) e = hipEventCreateWithFlags(&p->fork_ev, hipEventDisableTiming);
  const size_t need = p->classes.empty() ? 0 : p->classes.size() - 1;
  while (e == hipSuccess && p->forks.size() < need) {
    hipStream_t f = nullptr;
    hipEvent_t j = nullptr;
    e = hipStreamCreateWithFlags(&f, hipStreamNonBlocking);
    if (e != hipSuccess) break;
    p->forks.push_back(f);
    e = hipEventCreateWithFlags(&j, hipEventDisableTiming);
    if (e != hipSuccess) break;
    p->joins.push_back(j);
  }
  if (p->joins.size() < p->forks.size()) e = hipErrorOutOfMemory;
  return e == hipSuccess ? MPBP_OK : hip_fail(e, "capture streams");
}

// Replay the graph captured for `key`, capturing it first (from `enqueue`, run on the
// plan's capture stream) if it is not cached.  The least recently used graph is
// dropped beyond kMaxGraphs (after a device synchronisation).
template <class Enqueue>
mpbp_status run_graph(mpbp_plan p, const GraphKey& key, hipStream_t s, Enqueue&& enqueue) {
  hipError_t e;
  for (auto& g : p->graphs) {
    if (g.key == key) {
      g.used = ++p->graph_clock;
      e = hipGraphLaunch(g.exec, s);
      return e == hipSuccess ? MPBP_OK : hip_fail(e, "hipGraphLaunch");
    }
  }
  mpbp_status st = ensure_capture_streams(p);
  if (st != MPBP_OK) return st;
  e = hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return hip_fail(e, "hipStreamBeginCapture");
  const char* what = "capture";
  const hipError_t le = enqueue(p->cap, &what);
  hipGraph_t graph = nullptr;
  e = hipStreamEndCapture(p->cap, &graph);
  if (le != hipSuccess || e != hipSuccess) {
    if (graph) (void)hipGraphDestroy(graph);
    return le != hipSuccess ? hip_fail(le, what) : hip_fail(e, "hipStreamEndCapture");
  }
  hipGraphExec_t exec = nullptr;
  e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  if (e != hipSuccess) return hip_fail(e, "hipGraphInstantiate");
  if (p->graphs.size() >= kMaxGraphs) {
    auto old = std::min_element(p->graphs.begin(), p->graphs.end(),
                                [](const GraphEntry& a, const GraphEntry& b) { return a.used < b.used; });
    (void)hipDeviceSynchronize();
    (void)hipGraphExecDestroy(old->exec);
    p->graphs.erase(old);
  }
  p->graphs.push_back({key, exec, ++p->graph_clock});
  trace("plan %p: captured a %s graph (%zu kept)", (void*)p, key.kind ? "loss_grad" : "forward", p->graphs.size());
  e = hipGraphLaunch(exec, s);
  return e == hipSuccess ? MPBP_OK : hip_fail(e, "hipGraphLaunch");
}

// ---- launch-parameter tuning ----------------------------------------------------

// Compiled footprint bounds a class may use (>= its smallest bound), and whether a
// variant fits the LDS of a CU.
std::vector<int> class_bounds(const mpbp_plan_t::SizeClass& c) {
  std::vector<int> out;
  for (int fb : {32, 48, 64, c.D})
    if (fb >= c.key && std::find(out.begin(), out.end(), fb) == out.end()) {
      bool any = false;
      any = mpbp::frame_instance(c.D, fb);
      if (any) out.push_back(fb);
    }
  return out;
}

bool variant_ok(const mpbp_plan_t* p, const mpbp_plan_t::SizeClass& c, int fb, int G) {
  return fb >= c.key && (G == 2 || G == 4 || G == 8) && mpbp::frame_instance(c.D, fb) && c.lds_grad > 0 &&
         c.lds_grad <= kMaxLds && c.lds_fwd <= kMaxLds && p->lds_project[G] <= kMaxLds;
}

std::string device_arch(int device) {
  hipDeviceProp_t prop;
  if (hipGetDeviceProperties(&prop, device) != hipSuccess) return "unknown";
  std::string a = prop.gcnArchName;
  return a.substr(0, a.find(':'));
}

std::string frames_key(const mpbp_plan_t* p, const mpbp_plan_t::SizeClass& c, const std::string& arch) {
  char buf[192];
  snprintf(buf, sizeof(buf), "frames %s D=%d key=%d fy=%d fx=%d np=%d nz=%d", arch.c_str(), c.D, c.key, c.fy,
           c.fx, p->np, p->nz);
  return buf;
}

std::string grad_key(const mpbp_plan_t* p, const std::string& arch) {
  char buf[192];
  snprintf(buf, sizeof(buf), "grad %s nz=%d ny=%d nx=%d np=%d M=%d spany=%d spanx=%d", arch.c_str(), p->nz,
           p->ny, p->nx, p->np, p->M, p->maxspan_y, p->maxspan_x);
  return buf;
}

// The tuning cache is a text file named by MPBP_TUNE_CACHE: one line per tuned kernel,
// "<key> | <parameters>", keyed by GPU architecture and the shapes the kernel's speed
// depends on.
std::vector<std::pair<std::string, std::string>> read_cache(const char* path) {
  std::vector<std::pair<std::string, std::string>> out;
  FILE* f = std::fopen(path, "r");
  if (!f) return out;
  char line[512];
  while (std::fgets(line, sizeof(line), f)) {
    std::string l(line);
    while (!l.empty() && (l.back() == '\n' || l.back() == '\r')) l.pop_back();
    const size_t bar = l.find(" | ");
    if (bar != std::string::npos) out.push_back({l.substr(0, bar), l.substr(bar + 3)});
  }
  std::fclose(f);
  return out;
}

void load_tuning(mpbp_plan_t* p) {
  const char* path = std::getenv("MPBP_TUNE_CACHE");
  if (!path || !*path) return;
  const auto entries = read_cache(path);
  if (entries.empty()) return;
  const std::string arch = device_arch(p->device);
  bool used = false;
  for (auto& c : p->classes) {
    const std::string k = frames_key(p, c, arch);
    for (const auto& e : entries) {
      int fb = 0, G = 0, xcd = 0;
      double us = 0.0;
      if (e.first == k && std::sscanf(e.second.c_str(), "FB=%d G=%d xcd=%d us=%lf", &fb, &G, &xcd, &us) == 4 &&
          variant_ok(p, c, fb, G) && (xcd == 0 || xcd == 1)) {
        c.FB = fb; c.G = G; c.xcd = xcd; c.tuned_us = us;
        used = true;
      }
    }
  }
  const std::string gk = grad_key(p, arch);
  for (const auto& e : entries) {
    int b = 0, tx = 0;
    double us = 0.0;
    if (e.first == gk && std::sscanf(e.second.c_str(), "batch=%d tile=%d us=%lf", &b, &tx, &us) == 3 &&
        (b == 1 || b == 2 || b == 4 || b == 8 || b == 16) && (tx == 16 || tx == 8)) {
      p->grad_batch = b;
      p->grad_tile = tx;
      p->grad_tuned_us = us;
      used = true;
    }
  }
  if (used) {
    p->tune_source = "cache";
    trace("plan %p: launch parameters from the tuning cache %s", (void*)p, path);
  }
}

void save_tuning(const mpbp_plan_t* p) {
  const char* path = std::getenv("MPBP_TUNE_CACHE");
  if (!path || !*path) return;
  auto entries = read_cache(path);
  const std::string arch = device_arch(p->device);
  auto put = [&](const std::string& k, const std::string& v) {
    for (auto& e : entries)
      if (e.first == k) {
        e.second = v;
        return;
      }
    entries.push_back({k, v});
  };
  char buf[128];
  for (const auto& c : p->classes) {
    if (c.count == 0) continue;
    snprintf(buf, sizeof(buf), "FB=%d G=%d xcd=%d us=%.2f", c.FB, c.G, c.xcd, c.tuned_us);
    put(frames_key(p, c, arch), buf);
  }
  snprintf(buf, sizeof(buf), "batch=%d tile=%d us=%.2f", p->grad_batch, p->grad_tile, p->grad_tuned_us);
  put(grad_key(p, arch), buf);
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return;
  for (const auto& e : entries) std::fprintf(f, "%s | %s\n", e.first.c_str(), e.second.c_str());
  std::fclose(f);
  (void)std::rename(tmp.c_str(), path);
}


// ---- the unwrap projector (eqs. (9)-(10)) ----

// Moore-Penrose inverse H^+ (M x 3) of H (3 x M, column m = G_m), in double:
// H^+ = H^T (H H^T)^+, with the pseudo-inverse of the symmetric 3 x 3 matrix H H^T from
// its eigen-decomposition by cyclic Jacobi rotations; eigenvalues below 1e-12 of the
// largest count as zero (coplanar Bragg vectors: the component no peak sees is kept).
void bragg_pinv(const std::vector<mpbp_peak>& pk, double hp[][3]) {
  double A[3][3] = {{0}}, V[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  for (const auto& p : pk)
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) A[a][b] += p.g[a] * p.g[b];
  for (int sweep = 0; sweep < 64; ++sweep) {
    const double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
    const double dia = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
    if (off <= 1e-32 * dia) break;
    for (int p = 0; p < 2; ++p)
      for (int q = p + 1; q < 3; ++q) {
        if (A[p][q] == 0.0) continue;
        // rotation in the (p, q) plane that zeroes A[p][q]
        const double th = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
        const double t = (th >= 0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int k = 0; k < 3; ++k) {          // A <- A J
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - s * akq;
          A[k][q] = s * akp + c * akq;
        }
        for (int k = 0; k < 3; ++k) {          // A <- J^T A
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - s * aqk;
          A[q][k] = s * apk + c * aqk;
        }
        for (int k = 0; k < 3; ++k) {          // V <- V J
          const double vkp = V[k][p], vkq = V[k][q];
          V[k][p] = c * vkp - s * vkq;
          V[k][q] = s * vkp + c * vkq;
        }
      }
  }
  double lmax = 0.0;
  for (int k = 0; k < 3; ++k) lmax = std::max(lmax, std::fabs(A[k][k]));
  double Ai[3][3] = {{0}};
  for (int k = 0; k < 3; ++k) {
    if (!(A[k][k] > 1e-12 * lmax)) continue;
    const double il = 1.0 / A[k][k];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Ai[a][b] += il * V[a][k] * V[b][k];
  }
  for (size_t m = 0; m < pk.size(); ++m)
    for (int c = 0; c < 3; ++c) {
      double v = 0.0;
      for (int a = 0; a < 3; ++a) v += pk[m].g[a] * Ai[a][c];
      hp[m][c] = v;
    }
}

// Allocate the projector's workspace on first use.
mpbp_status ensure_unwrap(mpbp_plan_t* p) {
  if (p->d_uw) return MPBP_OK;
  mpbp::UnwrapArgs& A = p->uw;
  A = mpbp::UnwrapArgs{};
  A.M = p->M;
  A.S = p->tied ? 1 : p->nz;
  A.ny = p->ny;
  A.nx = p->nx;
  A.np = (long long)p->ny * p->nx;
  A.nmaps = (long long)A.M * A.S;
  A.npix = A.nmaps * A.np;
  A.rounds = mpbp::unwrap_rounds(A.np);
  if (2 * A.np >= (1LL << 31)) return fail(MPBP_ERR_SHAPE, "unwrap: ny * nx too large (%lld)", A.np);
  double hp[kMaxPeaks][3];
  bragg_pinv(p->peaks, hp);
  for (int m = 0; m < A.M; ++m)
    for (int c = 0; c < 3; ++c) {
      A.g[m][c] = (float)p->peaks[m].g[c];
      A.coef[m][c] = (float)(2.0 * M_PI * hp[m][c]);
    }
  // one allocation: 8-byte arrays first
  const long long n = A.npix;
  size_t bytes = 0;
  auto take = [&](size_t b) { size_t o = bytes; bytes += (b + 255) & ~(size_t)255; return o; };
  const size_t o_best = take(8 * n), o_sums = take(8 * A.nmaps), o_psi = take(4 * n), o_q = take(4 * n),
               o_rel = take(4 * n), o_par = take(4 * n), o_pot = take(4 * n), o_hk = take(4 * n),
               o_hpot = take(4 * n), o_hooks = take(4 * 64 * (size_t)A.rounds), o_err = take(4);
  hipError_t e = hipMalloc(&p->d_uw, bytes);
  if (e != hipSuccess) {
    p->d_uw = nullptr;
    return fail(MPBP_ERR_NOMEM, "unwrap workspace (%zu bytes): %s", bytes, hipGetErrorString(e));
  }
  e = hipHostMalloc((void**)&p->h_uw_err, sizeof(int), hipHostMallocDefault);
  if (e != hipSuccess) {
    (void)hipFree(p->d_uw);
    p->d_uw = nullptr;
    p->h_uw_err = nullptr;
    return fail(MPBP_ERR_NOMEM, "unwrap status word: %s", hipGetErrorString(e));
  }
  char* b = (char*)p->d_uw;
  A.best = (unsigned long long*)(b + o_best);
  A.sums = (long long*)(b + o_sums);
  A.psi = (float*)(b + o_psi);
  A.q = (int*)(b + o_q);
  A.rel = (float*)(b + o_rel);
  A.par = (int*)(b + o_par);
  A.pot = (int*)(b + o_pot);
  A.hk = (int*)(b + o_hk);
  A.hpot = (int*)(b + o_hpot);
  A.hooks = (int*)(b + o_hooks);
  A.err = (int*)(b + o_err);
  return MPBP_OK;
}

}  // namespace

extern "C" {

// The debug library (MPBP_DEBUG) waits for each compute call and reports a device-side
// bounds check that fired; the release library returns at once.
static mpbp_status debug_check(mpbp_plan_t* p, hipStream_t s, mpbp_status st) {
#ifdef MPBP_DEBUG
  if (st != MPBP_OK) return st;
  unsigned bits = 0;
  hipError_t e = hipStreamSynchronize(s);
  if (e == hipSuccess) e = hipMemcpy(&bits, p->d_dbg, sizeof(bits), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "debug status word");
  if (bits) {
    (void)hipMemset(p->d_dbg, 0, sizeof(unsigned));
    return fail(MPBP_ERR_INTERNAL, "device bounds check failed (bits 0x%x: 1 accumulator, 2 object, 4 slot, "
                "8 frame list, 16 run sums)", bits);
  }
  return MPBP_OK;
#else
  (void)p;
  (void)s;
  return st;
#endif
}

// The plan's choices, under MPBP_TRACE.
static void trace_plan(const mpbp_plan_t* p, const char* when) {
  if (!trace_on()) return;
  trace("plan %p (%s): grid %dx%dx%d, probe %d, %d peaks, %lld frames, flags%s%s%s%s; device %d", (void*)p, when,
        p->nz, p->ny, p->nx, p->np, p->M, (long long)p->F, p->tied ? " z-tied" : "", p->probe3 ? " probe-3d" : "",
        p->linear ? " shear-linear" : "", p->mapped ? " detector-map" : "", p->device);
  for (int m = 0; m < p->M; ++m) {
    const PeakDev& d = p->pdev[m];
    trace("  peak %d: D %d, footprint %dx%d at (%d, %d), %d runs of equal offset over %d slices, raster %dx%d", m,
          d.D, d.fy, d.fx, d.r0, d.c0, d.nruns, p->nz, d.rows, d.cols);
    if (p->mapped)
      trace("    detector map [%g %g; %g %g]", d.mm[0], d.mm[1], d.mm[2], d.mm[3]);
  }
  if (p->mapped && !p->color_off.empty()) {
    int lo = 1 << 30, hi = 0;
    for (size_t c = 0; c + 1 < p->color_off.size(); ++c) {
      lo = std::min(lo, p->color_off[c + 1] - p->color_off[c]);
      hi = std::max(hi, p->color_off[c + 1] - p->color_off[c]);
    }
    trace("  back-projection: %zu colours of non-overlapping frames, %d to %d frames each, %d in all",
          p->color_off.size() - 1, lo, hi, p->color_off.back());
  }
  for (size_t k = 0; k < p->classes.size(); ++k) {
    const auto& c = p->classes[k];
    trace("  class %zu: D %d, %d frames, footprint bound %d (smallest %d), projection depth %d, xcd order %d%s", k,
          c.D, c.count, c.FB, c.key, c.G, c.xcd, c.tuned_us > 0 ? " (tuned)" : "");
  }
  const bool runs = uses_runs(p);
  char bp[96];
  if (p->mapped)
    snprintf(bp, sizeof(bp), "per colour of frames, then the chain rule per voxel");
  else
    snprintf(bp, sizeof(bp), "%s, batch %d, tile %d", runs ? "per run (gather + chain rule)" : "per slice",
             p->grad_batch, p->grad_tile);
  trace("  path: %s; objects %s; back-projection %s; tuning source %s", p->path ? "plain" : "batched fused",
        runs ? "summed per run" : "per slice", bp, p->tune_source.c_str());
  const int lds_bp = p->mapped ? (p->np * p->np + p->acc_pix) * (int)sizeof(float) * 2 : runs ? p->lds_runs : p->lds_grad;
  const int W = p->np + 2;   // the detector-map projection's bordered window
  const int lds_pr = p->mapped ? p->nz * 8 + (p->np * p->np + 2 * W * W) * 8 : p->lds_project[mpbp::kDefaultSlab];
  trace("  LDS bytes: frame kernel %d, projection %d, back-projection %d; projection accumulator %d pixels",
        p->lds_grad_frame, lds_pr, lds_bp, p->acc_pix);
  if (p->device >= 0)
    trace("  device workspace: objects %zu B, two footprint slots of %zu B each, %d alpha partials per peak",
          sizeof(float) * 2 * (size_t)p->M * (size_t)p->nvox, sizeof(float) * 2 * (size_t)p->slots_cplx, p->max_parts);
}

mpbp_status mpbp_plan_create(const mpbp_problem* problem, int device, mpbp_plan* out) {
  if (!out) return fail(MPBP_ERR_INVALID, "out is NULL");
  *out = nullptr;
  mpbp_plan_t* p = new (std::nothrow) mpbp_plan_t();
  if (!p) return fail(MPBP_ERR_NOMEM, "host allocation failed");
  mpbp_status st = build_tables(problem, p);
  if (st != MPBP_OK) {
    delete p;
    return st;
  }
  if (device >= 0) {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || device >= n) {
      delete p;
      return fail(MPBP_ERR_DEVICE, "device %d not available (%d devices)", device, e == hipSuccess ? n : 0);
    }
    p->device = device;
    st = alloc_device(p);
    if (st != MPBP_OK) {
      std::string msg = g_err;
      free_device(p);
      delete p;
      g_err = msg;
      return st;
    }
    st = scratch_setup(device);
    if (st != MPBP_OK) {
      std::string msg = g_err;
      free_device(p);
      delete p;
      g_err = msg;
      return st;
    }
    load_tuning(p);
  } else if (device != -1) {
    delete p;
    return fail(MPBP_ERR_INVALID, "device must be >= 0, or -1 for a host-only plan");
  }
  g_err.clear();
  trace_plan(p, "created");
  *out = p;
  return MPBP_OK;
}

void mpbp_plan_destroy(mpbp_plan plan) {
  if (!plan) return;
  free_device(plan);
  delete plan;
}

int64_t mpbp_num_frames(mpbp_plan plan) { return plan ? plan->F : -1; }

int64_t mpbp_intensity_size(mpbp_plan plan) { return plan ? plan->ylen : -1; }

mpbp_status mpbp_tables(mpbp_plan plan, int32_t* scan_yx, int32_t* shear_yx, int64_t* y_off) {
  if (!plan) return fail(MPBP_ERR_INVALID, "plan is NULL");
  if (scan_yx) std::memcpy(scan_yx, plan->scan.data(), plan->scan.size() * sizeof(int32_t));
  if (shear_yx) std::memcpy(shear_yx, plan->shear.data(), plan->shear.size() * sizeof(int32_t));
  if (y_off) std::memcpy(y_off, plan->y_off.data(), plan->y_off.size() * sizeof(int64_t));
  return MPBP_OK;
}

mpbp_status mpbp_forward(mpbp_plan plan, const float* u, const float* chi, const float* alpha,
                         const void* probe, const float* y, const int32_t* frames, int64_t n_frames,
                         double* loss, float* frame_loss, float* model_intensity, void* stream) {
  mpbp_status st = check_plan(plan);
  if (st != MPBP_OK) return st;
  if (!u || !chi || !alpha || !probe) return fail(MPBP_ERR_INVALID, "u, chi, alpha and probe are required");
  if ((loss || frame_loss) && !y) return fail(MPBP_ERR_INVALID, "y is required for loss / frame_loss");
  hipStream_t s = (hipStream_t)stream;
  int n = 0;
  st = stage_frames(plan, frames, n_frames, s, false, &n);
  if (st != MPBP_OK) return st;
  const int* list = frames ? plan->d_list : plan->d_order;
  const int* out_list = frames ? plan->d_list : nullptr;
  hipError_t e;
  if (plan->path == 1) {
    StageTimer t(plan, MPBP_STAGE_PLAIN, s);
    plan->plain.bg = plan->d_bg;
    plan->plain.probe3 = plan->probe3;
    plan->plain.shw = plan->linear ? plan->d_shw : nullptr;
    e = mpbp::plain_forward(&plan->plain, plan->pdev.data(), plan->d_peaks, plan->M, plan->nz, plan->ny,
                            plan->nx, plan->np, plan->d_shear, plan->scan.data(), plan->peak_of.data(),
                            frames, frames ? n : (int)plan->F, u, chi, alpha, (const float*)probe, y,
                            model_intensity, plan->d_obj, plan->d_floss, plan->tied, s);
    if (e != hipSuccess) return hip_fail(e, "plain path");
  } else if (use_graph(plan, frames)) {
    GraphKey key;
    key.kind = 0;
    key.xcd = plan->xcd;
    const void* ptrs[] = {u, chi, alpha, probe, y, loss, frame_loss, model_intensity, plan->d_bg};
    std::copy(std::begin(ptrs), std::end(ptrs), key.ptr);
    return debug_check(plan, s, run_graph(plan, key, s, [&](hipStream_t cs, const char** what) {
      hipError_t le = enqueue_forward(plan, u, chi, alpha, (const float*)probe, y, list, n, false,
                                      model_intensity, cs, true, what);
      if (le == hipSuccess && (loss || frame_loss)) {
        le = mpbp::launch_finalize(plan->d_floss, out_list, n, loss, frame_loss, nullptr, 0, plan->M,
                                   nullptr, cs);
        if (le != hipSuccess) *what = "finalize kernel";
      }
      return le;
    }));
  } else {
    const char* what = "";
    e = enqueue_forward(plan, u, chi, alpha, (const float*)probe, y, list, n, frames != nullptr,
                        model_intensity, s, false, &what);
    if (e != hipSuccess) return hip_fail(e, what);
  }
  if (loss || frame_loss) {
    StageTimer t(plan, MPBP_STAGE_FINALIZE, s);
    e = mpbp::launch_finalize(plan->d_floss, out_list, n, loss, frame_loss, nullptr, 0, plan->M, nullptr, s);
    if (e != hipSuccess) return hip_fail(e, "finalize kernel");
  }
  return debug_check(plan, s, MPBP_OK);
}

mpbp_status mpbp_loss_grad(mpbp_plan plan, const float* u, const float* chi, const float* alpha,
                           const void* probe, const float* y, const int32_t* frames, int64_t n_frames,
                           double* loss, float* frame_loss, float* grad_u, float* grad_chi,
                           float* grad_alpha, void* stream) {
  mpbp_status st = check_plan(plan);
  if (st != MPBP_OK) return st;
  if (!u || !chi || !alpha || !probe || !y)
    return fail(MPBP_ERR_INVALID, "u, chi, alpha, probe and y are required");
  if (!grad_u || !grad_chi || !grad_alpha) return fail(MPBP_ERR_INVALID, "grad_u, grad_chi and grad_alpha are required");
  hipStream_t s = (hipStream_t)stream;
  int n = 0;
  st = stage_frames(plan, frames, n_frames, s, plan->path == 0, &n);
  if (st != MPBP_OK) return st;
  const int* list = frames ? plan->d_list : plan->d_order;
  const int* out_list = frames ? plan->d_list : nullptr;
  hipError_t e;
  int n_part = grad_parts(plan);
  const double* apart = plan->d_apart;
  if (plan->path == 1) {
    StageTimer t(plan, MPBP_STAGE_PLAIN, s);
    plan->plain.bg = plan->d_bg;
    plan->plain.probe3 = plan->probe3;
    plan->plain.shw = plan->linear ? plan->d_shw : nullptr;
    e = mpbp::plain_loss_grad(&plan->plain, plan->pdev.data(), plan->d_peaks, plan->M, plan->nz, plan->ny,
                              plan->nx, plan->np, plan->d_shear, plan->scan.data(), plan->peak_of.data(),
                              frames, frames ? n : (int)plan->F, u, chi, alpha, (const float*)probe, y,
                              plan->d_obj, plan->d_floss, grad_u, grad_chi, &apart, &n_part, plan->tied, s);
    if (e != hipSuccess) return hip_fail(e, "plain path");
  } else if (use_graph(plan, frames)) {
    GraphKey key;
    key.kind = 1;
    key.xcd = plan->xcd;
    const void* ptrs[] = {u, chi, alpha, probe, y, loss, frame_loss, grad_u, grad_chi, grad_alpha, plan->d_bg};
    std::copy(std::begin(ptrs), std::end(ptrs), key.ptr);
    return debug_check(plan, s, run_graph(plan, key, s, [&](hipStream_t cs, const char** what) {
      hipError_t le = enqueue_loss_grad(plan, plan_work(plan), u, chi, alpha, (const float*)probe, y, list, n,
                                        false, grad_u, grad_chi, cs, true, what);
      if (le == hipSuccess) {
        le = mpbp::launch_finalize(plan->d_floss, out_list, n, loss, frame_loss, apart, n_part, plan->M,
                                   grad_alpha, cs);
        if (le != hipSuccess) *what = "finalize kernel";
      }
      return le;
    }));
  } else {
    const char* what = "";
    e = enqueue_loss_grad(plan, plan_work(plan), u, chi, alpha, (const float*)probe, y, list, n,
                          frames != nullptr, grad_u, grad_chi, s, false, &what);
    if (e != hipSuccess) return hip_fail(e, what);
  }
  {
    StageTimer t(plan, MPBP_STAGE_FINALIZE, s);
    e = mpbp::launch_finalize(plan->d_floss, out_list, n, loss, frame_loss, apart, n_part, plan->M,
                              grad_alpha, s);
  }
  if (e != hipSuccess) return hip_fail(e, "finalize kernel");
  return debug_check(plan, s, MPBP_OK);
}

// Layout of the fused path's workspace in the fixed array: objects, exit-wave slots,
// gradient slots, frame losses, alpha partials, each starting on a 256-byte boundary.
// Returns the bytes needed.
static size_t static_work(mpbp_plan p, char* base, Work* w) {
  size_t off = 0;
  auto take = [&](size_t bytes) {
    char* q = base ? base + off : nullptr;
    off += (bytes + 255) & ~size_t(255);
    return q;
  };
  Work t;
  t.obj = (float*)take(sizeof(float) * 2 * (size_t)p->M * (size_t)p->nvox);
  t.slots = (float*)take(sizeof(float) * 2 * (size_t)p->slots_cplx);
  t.gslots = (float*)take(sizeof(float) * 2 * (size_t)p->slots_cplx);
  t.floss = (double*)take(sizeof(double) * (size_t)p->F);
  t.apart = (double*)take(sizeof(double) * (size_t)p->max_parts * p->M);
  if (w) *w = t;
  return off;
}

mpbp_status mpbp_loss_grad_static(mpbp_plan plan, const float* u, const float* chi, const float* alpha,
                                  const void* probe, const float* y, const int32_t* frames, int64_t n_frames,
                                  double* loss, float* frame_loss, float* grad_u, float* grad_chi,
                                  float* grad_alpha, void* stream) {
  mpbp_status st = check_plan(plan);
  if (st != MPBP_OK) return st;
  if (!u || !chi || !alpha || !probe || !y)
    return fail(MPBP_ERR_INVALID, "u, chi, alpha, probe and y are required");
  if (!grad_u || !grad_chi || !grad_alpha) return fail(MPBP_ERR_INVALID, "grad_u, grad_chi and grad_alpha are required");
  const size_t need = static_work(plan, nullptr, nullptr);
  if (need > kStaticScratchBytes)
    return fail(MPBP_ERR_UNSUPPORTED, "the workload needs %zu bytes of workspace; the static workspace holds %zu",
                need, kStaticScratchBytes);
  char* base = (char*)scratch_of(plan->device);
  if (!base) return fail(MPBP_ERR_DEVICE, "no static workspace on device %d", plan->device);
  Work w;
  static_work(plan, base, &w);
  hipStream_t s = (hipStream_t)stream;
  int n = 0;
  st = stage_frames(plan, frames, n_frames, s, true, &n);
  if (st != MPBP_OK) return st;
  const int* list = frames ? plan->d_list : plan->d_order;
  const int* out_list = frames ? plan->d_list : nullptr;
  const char* what = "";
  hipError_t e = enqueue_loss_grad(plan, w, u, chi, alpha, (const float*)probe, y, list, n, frames != nullptr,
                                   grad_u, grad_chi, s, false, &what, false);
  if (e != hipSuccess) return hip_fail(e, what);
  const int n_part = grad_parts(plan);
  e = mpbp::launch_finalize(w.floss, out_list, n, loss, frame_loss, w.apart, n_part, plan->M, grad_alpha, s);
  if (e != hipSuccess) return hip_fail(e, "finalize kernel");
  return debug_check(plan, s, MPBP_OK);
}

mpbp_status mpbp_step(mpbp_plan plan, float* u, float* chi, float* alpha, const float* grad_u,
                      const float* grad_chi, const float* grad_alpha, const float* eta, void* stream) {
  mpbp_status st = check_plan(plan);
  if (st != MPBP_OK) return st;
  if (!u || !chi || !alpha || !grad_u || !grad_chi || !grad_alpha || !eta)
    return fail(MPBP_ERR_INVALID, "all pointers are required");
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(eta[i])) return fail(MPBP_ERR_INVALID, "eta[%d] not finite", i);
  hipStream_t s = (hipStream_t)stream;
  const long long nf = plan->tied ? plan->tied : plan->nvox;   // field elements
  hipError_t e = mpbp::launch_step(u, grad_u, 3 * nf, eta[0], s);
  if (e == hipSuccess) e = mpbp::launch_step(chi, grad_chi, nf, eta[1], s);
  if (e == hipSuccess) e = mpbp::launch_step(alpha, grad_alpha, plan->M, eta[2], s);
  if (e != hipSuccess) return hip_fail(e, "step kernel");
  return MPBP_OK;
}

mpbp_status mpbp_adam_step(mpbp_plan plan, const mpbp_adam* cfg, int64_t t, float* u, float* chi,
                           float* alpha, float* chi_log, float* alpha_log, float* state,
                           const float* grad_u, const float* grad_chi, const float* grad_alpha,
                           void* stream) {
  mpbp_status st = check_plan(plan);
  if (st != MPBP_OK) return st;
  if (!cfg) return fail(MPBP_ERR_INVALID, "cfg is NULL");
  if (!u || !chi || !alpha || !state) return fail(MPBP_ERR_INVALID, "u, chi, alpha and state are required");
  if (t > 0 && (!grad_u || !grad_chi || !grad_alpha)) return fail(MPBP_ERR_INVALID, "the gradients are required");
  if (cfg->log_params != 0 && cfg->log_params != 1) return fail(MPBP_ERR_INVALID, "log_params must be 0 or 1");
  if (cfg->log_params && (!chi_log || !alpha_log))
    return fail(MPBP_ERR_INVALID, "chi_log and alpha_log are required with log_params");
  if (t < 0) return fail(MPBP_ERR_INVALID, "t must be >= 0 (got %lld)", (long long)t);
  if (t == 0) {
    const long long nf0 = plan->tied ? plan->tied : plan->nvox;
    hipStream_t s0 = (hipStream_t)stream;
    hipError_t e0 = mpbp::launch_fill(state, 2 * (4 * nf0 + plan->M), 0.f, s0);
    if (e0 == hipSuccess && cfg->log_params) e0 = mpbp::launch_exp(chi, chi_log, nf0, s0);
    if (e0 == hipSuccess && cfg->log_params) e0 = mpbp::launch_exp(alpha, alpha_log, plan->M, s0);
    if (e0 != hipSuccess) return hip_fail(e0, "adam initialisation");
    return MPBP_OK;
  }
  for (int i = 0; i < 3; ++i)
    if (!std::isfinite(cfg->lr[i]) || cfg->lr[i] < 0.f) return fail(MPBP_ERR_INVALID, "lr[%d] invalid", i);
  if (!(cfg->beta1 >= 0.f && cfg->beta1 < 1.f) || !(cfg->beta2 >= 0.f && cfg->beta2 < 1.f) ||
      !(cfg->eps > 0.f) || !std::isfinite(cfg->eps))
    return fail(MPBP_ERR_INVALID, "beta1, beta2 must be in [0, 1) and eps > 0");
  if (cfg->fixed_alpha < -1 || cfg->fixed_alpha >= plan->M)
    return fail(MPBP_ERR_INVALID, "fixed_alpha %d out of range", cfg->fixed_alpha);
  const long long nf = plan->tied ? plan->tied : plan->nvox;
  const float c1 = (float)(1.0 - std::pow((double)cfg->beta1, (double)t));
  const float c2 = (float)(1.0 - std::pow((double)cfg->beta2, (double)t));
  if (!(c1 > 0.f) || !(c2 > 0.f)) return fail(MPBP_ERR_INVALID, "bias corrections vanish (beta = 0 and t too small?)");
  // state: first moments of (u, chi, alpha), then second moments
  float* m = state;
  float* v = state + 4 * nf + plan->M;
  hipStream_t s = (hipStream_t)stream;
  const int lg = cfg->log_params;
  hipError_t e = mpbp::launch_adam(u, nullptr, m, v, grad_u, 3 * nf, cfg->lr[0], cfg->beta1, cfg->beta2,
                                   cfg->eps, c1, c2, 0, 0, -1, s);
  if (e == hipSuccess)
    e = mpbp::launch_adam(lg ? chi_log : chi, lg ? chi : nullptr, m + 3 * nf, v + 3 * nf, grad_chi, nf, cfg->lr[1],
                          cfg->beta1, cfg->beta2, cfg->eps, c1, c2, lg, 1, -1, s);
  if (e == hipSuccess)
    e = mpbp::launch_adam(lg ? alpha_log : alpha, lg ? alpha : nullptr, m + 4 * nf, v + 4 * nf, grad_alpha, plan->M,
                          cfg->lr[2], cfg->beta1, cfg->beta2, cfg->eps, c1, c2, lg, 1, cfg->fixed_alpha, s);
  if (e != hipSuccess) return hip_fail(e, "adam kernel");
  return MPBP_OK;
}

mpbp_status mpbp_unwrap_project(mpbp_plan plan, float* u, int32_t* wraps, void* stream) {
  mpbp_status st = check_plan(plan);
  if (st != MPBP_OK) return st;
  if (!u) return fail(MPBP_ERR_INVALID, "u is required");
  st = ensure_unwrap(plan);
  if (st != MPBP_OK) return st;
  hipStream_t s = (hipStream_t)stream;
  hipError_t e = mpbp::launch_unwrap(u, wraps, plan->uw, s);
  if (e == hipSuccess) e = hipMemcpyAsync(plan->h_uw_err, plan->uw.err, sizeof(int), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return hip_fail(e, "unwrap projector");
  if (*plan->h_uw_err != 0)
    return fail(MPBP_ERR_INTERNAL, "unwrap projector: merge consistency check %d failed", *plan->h_uw_err);
  return MPBP_OK;
}

mpbp_status mpbp_norm2(mpbp_plan plan, const float* a, int64_t n, double* out, void* stream) {
  mpbp_status st = check_plan(plan);
  if (st != MPBP_OK) return st;
  if (!a || !out || n < 0) return fail(MPBP_ERR_INVALID, "a and out are required and n >= 0");
  hipError_t e = mpbp::launch_norm2(a, n, plan->d_red, kRedParts, out, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "norm kernel");
  return MPBP_OK;
}

mpbp_status mpbp_set_background(mpbp_plan plan, const float* b) {
  if (!plan) return fail(MPBP_ERR_INVALID, "plan is NULL");
  plan->d_bg = b;   // graphs are keyed by it
  return MPBP_OK;
}

mpbp_status mpbp_set_option(mpbp_plan plan, int option, int64_t value) {
  if (!plan) return fail(MPBP_ERR_INVALID, "plan is NULL");
  switch (option) {
    case MPBP_OPT_PATH:
      if (value != 0 && value != 1) return fail(MPBP_ERR_INVALID, "path must be 0 or 1");
      if (value == 1 && plan->mapped)
        return fail(MPBP_ERR_UNSUPPORTED, "the plain path has no detector-map projection (MPBP_DETECTOR_MAP)");
      plan->path = (int)value;
      return MPBP_OK;
    case MPBP_OPT_GRAPH:
      if (value != 0 && value != 1) return fail(MPBP_ERR_INVALID, "graph must be 0 or 1");
      plan->graph = (int)value;
      if (!value && plan->device >= 0) {
        (void)hipSetDevice(plan->device);
        clear_graphs(plan);
      }
      return MPBP_OK;
    case MPBP_OPT_XCD_ORDER:
      if (value != 0 && value != 1) return fail(MPBP_ERR_INVALID, "xcd order must be 0 or 1");
      plan->xcd = (int)value;
      for (auto& c : plan->classes) c.xcd = (int)value;
      if (plan->device >= 0) {
        (void)hipSetDevice(plan->device);
        clear_graphs(plan);
      }
      return MPBP_OK;
    case MPBP_OPT_PROFILE:
      if (value < 0 || value > 2) return fail(MPBP_ERR_INVALID, "profile must be 0, 1 or 2");
      plan->profile = (int)value;
      return MPBP_OK;
    case MPBP_OPT_GRAD_BATCH:
      if (value != 1 && value != 2 && value != 4 && value != 8 && value != 16)
        return fail(MPBP_ERR_INVALID, "grad batch must be 1, 2, 4, 8 or 16");
      plan->grad_batch = (int)value;
      plan->tune_source = "manual";
      if (plan->device >= 0) {
        (void)hipSetDevice(plan->device);
        clear_graphs(plan);
      }
      return MPBP_OK;
    case MPBP_OPT_RUNS:
      if (value != 0 && value != 1) return fail(MPBP_ERR_INVALID, "runs must be 0 or 1");
      plan->runs = (int)value;
      if (plan->device >= 0) {
        (void)hipSetDevice(plan->device);
        clear_graphs(plan);
      }
      return MPBP_OK;
    case MPBP_OPT_GRAD_TILE:
      if (value != 16 && value != 8) return fail(MPBP_ERR_INVALID, "grad tile must be 16 or 8");
      plan->grad_tile = (int)value;
      plan->tune_source = "manual";
      if (plan->device >= 0) {
        (void)hipSetDevice(plan->device);
        clear_graphs(plan);
      }
      return MPBP_OK;
    default:
      return fail(MPBP_ERR_INVALID, "unknown option %d", option);
  }
}

mpbp_status mpbp_get_option(mpbp_plan plan, int option, int64_t* value) {
  if (!plan || !value) return fail(MPBP_ERR_INVALID, "plan and value are required");
  switch (option) {
    case MPBP_OPT_PATH: *value = plan->path; return MPBP_OK;
    case MPBP_OPT_GRAPH: *value = plan->graph; return MPBP_OK;
    case MPBP_OPT_XCD_ORDER: *value = plan->xcd; return MPBP_OK;
    case MPBP_OPT_PROFILE: *value = plan->profile; return MPBP_OK;
    case MPBP_OPT_GRAD_BATCH: *value = plan->grad_batch; return MPBP_OK;
    case MPBP_OPT_GRAD_TILE: *value = plan->grad_tile; return MPBP_OK;
    case MPBP_OPT_RUNS: *value = plan->runs; return MPBP_OK;
    default: return fail(MPBP_ERR_INVALID, "unknown option %d", option);
  }
}

mpbp_status mpbp_stage_times(mpbp_plan plan, double* ms, int64_t* counts) {
  if (!plan) return fail(MPBP_ERR_INVALID, "plan is NULL");
  if (plan->device >= 0) (void)hipSetDevice(plan->device);
  for (auto& pe : plan->ev_pending) {
    hipError_t e = hipEventSynchronize(pe.second.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventSynchronize");
    float t = 0.f;
    e = hipEventElapsedTime(&t, pe.second.first, pe.second.second);
    if (e != hipSuccess) return hip_fail(e, "hipEventElapsedTime");
    plan->stage_ms[pe.first] += t;
    plan->stage_n[pe.first] += 1;
  }
  plan->ev_pending.clear();
  plan->ev_used = 0;
  for (int i = 0; i < MPBP_NUM_STAGES; ++i) {
    if (ms) ms[i] = plan->stage_ms[i];
    if (counts) counts[i] = plan->stage_n[i];
    plan->stage_ms[i] = 0.0;
    plan->stage_n[i] = 0;
  }
  return MPBP_OK;
}

mpbp_status mpbp_autotune(mpbp_plan plan, const float* u, const float* chi, const float* alpha,
                          const void* probe, const float* y, void* stream) {
  mpbp_status st = check_plan(plan);
  if (st != MPBP_OK) return st;
  if (!u || !chi || !alpha || !probe || !y) return fail(MPBP_ERR_INVALID, "u, chi, alpha, probe and y are required");
  hipStream_t s = (hipStream_t)stream;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  float* gbuf = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
  auto cleanup = [&]() {
    (void)hipStreamSynchronize(s);
    if (gbuf) (void)hipFree(gbuf);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
  };
  // one warm-up launch, then the mean of `reps` launches
  auto time_us = [&](auto&& launch, int reps, double* us) -> hipError_t {
    hipError_t r = launch();
    if (r == hipSuccess) r = hipEventRecord(e0, s);
    for (int i = 0; i < reps && r == hipSuccess; ++i) r = launch();
    if (r == hipSuccess) r = hipEventRecord(e1, s);
    if (r == hipSuccess) r = hipEventSynchronize(e1);
    float ms = 0.f;
    if (r == hipSuccess) r = hipEventElapsedTime(&ms, e0, e1);
    *us = 1e3 * (double)ms / reps;
    return r;
  };
  const long long nf = plan->tied ? plan->tied : plan->nvox;   // field elements
  e = hipMalloc((void**)&gbuf, (size_t)4 * nf * sizeof(float));
  if (e != hipSuccess) {
    cleanup();
    return fail(MPBP_ERR_NOMEM, "hipMalloc gradient scratch: %s", hipGetErrorString(e));
  }
  e = launch_objects(plan, plan_work(plan), u, chi, alpha, s);
  std::string rep = "[";
  char buf[160];
  // The projection and the frame kernel are separate launches: the projection depth G is
  // tuned on the projection alone, then the footprint bound FB on projection (at its
  // best G) plus frame kernel, for each XCD order.  Every candidate is timed in two
  // rounds and keeps its faster round (the first launches of a run are slowed by the
  // clock ramp).
  for (size_t ci = 0; ci < plan->classes.size() && e == hipSuccess; ++ci) {
    auto& c = plan->classes[ci];
    if (c.count == 0) continue;
    mpbp::FrameArgs a = frame_args(plan, plan_work(plan), y, plan->d_order + c.begin, c.count, nullptr, 1);
    a.probe = (const float*)probe;
    auto run_pf = [&](int G, int fb, int xcd) {
      a.xcd = xcd;
      hipError_t r = mpbp::launch_project(G, a, plan->lds_project[G], s);
      return r == hipSuccess && fb > 0 ? mpbp::launch_frames(c.D, fb, a, c.lds_grad, s) : r;
    };
    for (int w = 0; w < 3 && e == hipSuccess; ++w) e = run_pf(c.G, c.FB, c.xcd);   // clock warm-up
    double best = 1e300;
    int bfb = c.FB, bg = c.G, bx = c.xcd;
    for (int xcd = 0; xcd < 2 && e == hipSuccess; ++xcd) {
      double gbest = 1e300;
      int g_at = c.G;
      for (int G : mpbp::kSlabDepths) {
        if (e != hipSuccess || !variant_ok(plan, c, c.FB, G)) continue;
        double us = 1e300;
        for (int round = 0; round < 2 && e == hipSuccess; ++round) {
          double t = 0.0;
          e = time_us([&]() { return run_pf(G, 0, xcd); }, 3, &t);
          us = t < us ? t : us;
        }
        snprintf(buf, sizeof(buf), "%s{\"class\": %zu, \"kernel\": \"project\", \"G\": %d, \"xcd\": %d, \"us\": %.2f}",
                 rep.size() > 1 ? ", " : "", ci, G, xcd, us);
        rep += buf;
        if (e == hipSuccess && us < gbest) {
          gbest = us;
          g_at = G;
        }
      }
      for (int fb : class_bounds(c)) {
        if (e != hipSuccess || !variant_ok(plan, c, fb, g_at)) continue;
        double us = 1e300;
        for (int round = 0; round < 2 && e == hipSuccess; ++round) {
          double t = 0.0;
          e = time_us([&]() { return run_pf(g_at, fb, xcd); }, 3, &t);
          us = t < us ? t : us;
        }
        snprintf(buf, sizeof(buf), "%s{\"class\": %zu, \"FB\": %d, \"G\": %d, \"xcd\": %d, \"us\": %.2f}",
                 rep.size() > 1 ? ", " : "", ci, fb, g_at, xcd, us);
        rep += buf;
        if (e == hipSuccess && us < best) {
          best = us;
          bfb = fb; bg = g_at; bx = xcd;
        }
      }
    }
    c.FB = bfb; c.G = bg; c.xcd = bx; c.tuned_us = best;
  }
  if (e == hipSuccess) {
    // the gradient kernel, on the footprint gradients the frame launches left in the slots
    double best = 1e300;
    int bb = plan->grad_batch, bt = plan->grad_tile;
    for (int TX : mpbp::kGradTileXs) {
      plan->grad_tile = TX;
      const mpbp::GradArgs g = grad_args(plan, plan_work(plan), u, chi, alpha, (const float*)probe, false, gbuf, gbuf + 3 * nf);
      const bool runs = mpbp::grad_uses_runs(g);
      const std::vector<int> batches = runs ? std::vector<int>(std::begin(mpbp::kGradRunBatches), std::end(mpbp::kGradRunBatches))
                                            : std::vector<int>(std::begin(mpbp::kGradBatches), std::end(mpbp::kGradBatches));
      for (int B : batches) {
        if (e != hipSuccess) break;
        // the detector-map back-projection has no batch or tile width: time it once
        if (g.mapz && (TX != mpbp::kGradTileXs[0] || B != batches[0])) continue;
        double us = 1e300;
        for (int round = 0; round < 2 && e == hipSuccess; ++round) {
          double t = 0.0;
          e = time_us([&]() { return mpbp::launch_grad(B, TX, g, runs ? plan->lds_runs : plan->lds_grad, s); }, 3, &t);
          us = t < us ? t : us;
        }
        snprintf(buf, sizeof(buf), "%s{\"grad_batch\": %d, \"grad_tile\": %d, \"us\": %.2f}",
                 rep.size() > 1 ? ", " : "", B, TX, us);
        rep += buf;
        if (e == hipSuccess && us < best) {
          best = us;
          bb = B;
          bt = TX;
        }
      }
    }
    plan->grad_batch = bb;
    plan->grad_tile = bt;
    plan->grad_tuned_us = best;
  }
  cleanup();
  if (e != hipSuccess) return hip_fail(e, "autotune");
  plan->tune_report = rep + "]";
  plan->tune_source = "autotune";
  trace_plan(plan, "autotuned");
  clear_graphs(plan);
  save_tuning(plan);
  return MPBP_OK;
}

mpbp_status mpbp_set_variant(mpbp_plan plan, int size_class, int footprint_bound, int slab, int xcd_order) {
  if (!plan) return fail(MPBP_ERR_INVALID, "plan is NULL");
  if (size_class < 0 || size_class >= (int)plan->classes.size())
    return fail(MPBP_ERR_INVALID, "size class %d out of range [0, %zu)", size_class, plan->classes.size());
  auto& c = plan->classes[size_class];
  if (xcd_order != 0 && xcd_order != 1) return fail(MPBP_ERR_INVALID, "xcd_order must be 0 or 1");
  if (!variant_ok(plan, c, footprint_bound, slab))
    return fail(MPBP_ERR_UNSUPPORTED, "no compiled frame kernel for D=%d with footprint bound %d >= %d and projection depth %d",
                c.D, footprint_bound, c.key, slab);
  c.FB = footprint_bound;
  c.G = slab;
  c.xcd = xcd_order;
  c.tuned_us = 0.0;
  plan->tune_source = "manual";
  if (plan->device >= 0) {
    (void)hipSetDevice(plan->device);
    clear_graphs(plan);
  }
  return MPBP_OK;
}

mpbp_status mpbp_tuning(mpbp_plan plan, char* buf, int64_t cap, int64_t* len) {
  if (!plan) return fail(MPBP_ERR_INVALID, "plan is NULL");
  std::string out = "{\"source\": \"" + plan->tune_source + "\", \"grad_batch\": " +
                    std::to_string(plan->grad_batch) + ", \"grad_tile\": " + std::to_string(plan->grad_tile) +
                    ", \"runs\": " + std::to_string(plan->runs) +
                    ", \"classes\": [";
  char tmp[256];
  for (size_t i = 0; i < plan->classes.size(); ++i) {
    const auto& c = plan->classes[i];
    snprintf(tmp, sizeof(tmp),
             "%s{\"D\": %d, \"key\": %d, \"frames\": %d, \"fy\": %d, \"fx\": %d, \"FB\": %d, \"G\": %d, "
             "\"xcd\": %d, \"us\": %.2f}",
             i ? ", " : "", c.D, c.key, c.count, c.fy, c.fx, c.FB, c.G, c.xcd, c.tuned_us);
    out += tmp;
  }
  snprintf(tmp, sizeof(tmp), "], \"grad_us\": %.2f, \"candidates\": ", plan->grad_tuned_us);
  out += tmp;
  out += plan->tune_report.empty() ? "[]" : plan->tune_report;
  out += "}";
  if (len) *len = (int64_t)out.size() + 1;
  if (buf && cap > 0) {
    const size_t n = std::min<size_t>((size_t)cap - 1, out.size());
    std::memcpy(buf, out.data(), n);
    buf[n] = 0;
    if ((int64_t)out.size() + 1 > cap) return fail(MPBP_ERR_INVALID, "buffer too small (%zu bytes needed)", out.size() + 1);
  }
  return MPBP_OK;
}

const char* mpbp_last_error(void) { return g_err.c_str(); }

}  // extern "C"
