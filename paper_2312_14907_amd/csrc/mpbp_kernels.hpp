// mpbp_kernels.hpp - device-side data structures shared by the kernels and the host.
#pragma once
#include <stdint.h>

namespace mpbp {

// Device-side bounds checks of the projection and the back-projection, compiled in with
// MPBP_DEBUG (the debug library): an index outside its buffer sets a bit of the plan's
// status word (*dbg) and the access is skipped; the host reads the word after the call.
enum { kDbgAccumulator = 1, kDbgObject = 2, kDbgSlot = 4, kDbgFrameList = 8, kDbgRunSum = 16 };
#ifdef MPBP_DEBUG
#define MPBP_CHECK(dbg, cond, bit) ((cond) ? true : (atomicOr((dbg), (unsigned)(bit)), false))
#else
#define MPBP_CHECK(dbg, cond, bit) true
#endif

// Per-peak constants, built on the host from the plan's tables.
struct PeakDev {
  int D;            // detector / exit-wave window
  int R;            // number of residue chunks of the detector rows (D = R * L)
  int L;            // rows per chunk
  int c;            // window offset of the probe support: (D - Np) / 2
  int miny, minx;   // minimum shear over z
  int spany, spanx; // max - min shear
  int r0, c0;       // footprint origin in the window: c + min shear
  int fy, fx;       // footprint: Np + span
  int fxp;          // padded row stride of the chunk buffer (complex)
  int nfr;          // frames of this peak
  int frame_base;   // global id of this peak's frame 0
  int rows, cols;   // raster
  int sy, sx;       // raster step
  int oy, ox;       // raster origin
  long long y_off;  // element offset of this peak's frames in y
  long long slot_off;  // complex offset of frame 0's footprint slot in the workspace
  float gx, gy, gz; // Bragg vector (rad/nm)
  int lds_bytes;    // dynamic LDS the frame kernel needs for this peak
  long long tw_off; // complex offset of this peak's twiddle tables (D + L + R * fy)
  int nruns;        // runs of consecutive slices with equal exit-beam offset
  int run_base;     // index of this peak's first run over all peaks
  // MPBP_DETECTOR_MAP: the 2 x 2 map M of probe-window coordinates to exit-wave pixels
  // (row-major) and its inverse
  float mm[4], mi[4];
};

struct FrameArgs {
  const float* obj;        // complex64 [M][nz][ny][nx] (interleaved); with runs: the run
                           // sums [sum of nruns over peaks][ny][nx] (launch_runsum)
  const float* probe;      // complex64 [M][np][np]
  const float* y;          // ragged intensities (may be null)
  const float* bg;         // background b of eq. (2), ragged like y (may be null)
  const int* list;         // global frame ids to process
  int n_list;
  const int* scan;         // [F][2] (py, px)
  const int* peak_of;      // [F]
  const PeakDev* peaks;    // [M]
  const int* shear;        // [M][nz][2]
  float* slots;            // complex64 exit waves, one F_y x F_x slot per frame (written
                           // by the projection, read by k_frames)
  float* gslots;           // complex64 footprint gradients in the same slot layout (written
                           // by k_frames, read by the back-projection)
  double* floss;           // per-frame loss, indexed by global frame id
  const float* tw;         // complex64 twiddle tables of all peaks
  float* mi;               // model intensity (ragged like y) or null
  int nz, ny, nx, np;
  int grad;                // 1: also compute the footprint gradient
  int xcd;                 // XCD-aware block order
  int probe3;              // 1: probe is [M][nz][np][np] (a 3D illumination volume)
  const float* shw;        // [M][nz][2] fractional exit-beam offsets (null: rounded offsets)
  int runs;                // 1: project from the run sums (one probe, rounded offsets)
  int acc_pix;             // LDS footprint accumulator of the projection: the plan's largest
                           // fy * fx, rounded up to a multiple of 4
  int n_runs;              // runs over all peaks (the run sums' planes)
  unsigned* dbg;           // status word of the bounds checks (MPBP_DEBUG)
  const int2* roff;        // [M][nz] footprint offset (s_y - min s_y, s_x - min s_x) of run k
  const float2* mapz;      // MPBP_DETECTOR_MAP: [M][nz] exit-wave point of the probe window's
                           // centre for slice z, in footprint coordinates (null: no map)
};

struct GradArgs {
  const float* slots;      // complex64 footprint gradients
  const unsigned char* active;  // [F] 1 if the frame is in the minibatch
  int all_active;          // 1: every frame is (full batch): the flags are not read
  const float* probe;
  const float* u;
  const float* chi;
  const float* alpha;
  const int* shear;
  const PeakDev* peaks;
  int n_peaks;
  int nz, ny, nx, np;
  int tiles_x, tiles_y;
  int tile_ox, tile_oy;      // origin of the tile grid (<= 0)
  int maxspan_y, maxspan_x;  // largest shear span over peaks
  int max_cand;              // largest number of frames of one peak meeting one tile
  int tied;                  // 1: u, chi and their gradients per lateral pixel (z-sums)
  int probe3;                // 1: probe is [M][nz][np][np] (a 3D illumination volume)
  const float* shw;          // [M][nz][2] fractional exit-beam offsets (null: rounded offsets)
  int runs;                  // 1: back-project per run of equal offsets (k_bp_gather, k_bp_chain)
                             // where it applies
  float* rs;                 // complex64 [sum of nruns][ny][nx]: the frame sums per run
  long long nlat;            // ny * nx
  int n_runs;                // runs over all peaks
  unsigned* dbg;             // status word of the bounds checks (MPBP_DEBUG)
  const int* zrun;           // [M][nz] run of each slice (consecutive slices of equal offset)
  const int2* roff;          // [M][nz] footprint offset (s_y - min s_y, s_x - min s_x) of run k
  const float2* mapz;        // MPBP_DETECTOR_MAP: as FrameArgs::mapz (null: no map)
  const int* peak_of;        // [F]
  const int* scan;           // [F][2] (py, px)
  const int* color_list;     // MPBP_DETECTOR_MAP: the frames grouped by colour (no two
                             // frames of one peak and colour overlap)
  const int* color_off;      // (host) [n_colors + 1] offset of each colour in color_list
  int n_colors;
  int map_pix;               // the plan's largest footprint fy * fx (multiple of 4)
  float* grad_u;
  float* grad_chi;
  double* alpha_part;      // [n_blocks][M]
};

constexpr int kFrameThreads = 256;
constexpr int kSlabDepths[] = {2, 4, 8};   // compiled projection depths (object slices in flight per lane)
constexpr int kDefaultSlab = 4;
constexpr int kProjE = 4;     // probe pixels per lane in the projection (probe_n^2 <= 4 * 256)
constexpr int kProjMaxPix = 16384;   // largest footprint fy * fx of the projection (128 KB of LDS)
constexpr int kGradTile = 64, kGradTZ = 8;              // 64 voxels of a slice x 8 slice groups
constexpr int kGradThreads = kGradTile * kGradTZ;        // 512 threads
constexpr int kGradTileXs[] = {16, 8};                   // compiled tile widths (16 x 4, 8 x 8)
constexpr int kDefaultGradTileX = 16;
constexpr int kGradZB = 32;                             // z per pass of the grad kernel
constexpr int kGradZPer = kGradZB / kGradTZ;            // z per thread per pass
constexpr int kGradBatches[] = {1, 2, 4};               // compiled batch sizes of the per-slice walk
constexpr int kGradRunBatches[] = {4, 8, 16};           // compiled batch sizes of the run gather
constexpr int kBpThreads = 256;                         // workgroup of k_bp_gather and k_bp_chain
constexpr int kBpZ = 4;                                 // slices per lane of k_bp_chain
constexpr int kBpRunGroup = 3;                          // runs per wavefront per pass of k_bp_gather
constexpr int kDefaultGradBatch = 8;
constexpr int kMaxPeaksDev = 16;
constexpr int kMapThreads = 256;                        // workgroup of the detector-map kernels

}  // namespace mpbp
