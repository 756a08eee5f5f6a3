// mpbp_map.hip - R with a detector-frame map (MPBP_DETECTOR_MAP).  Section 2: each Bragg
// peak's exit wave lives in that peak's detector frame, which is turned against the
// object's frame and sampled at a pixel size of its own.  Slice z's probe-window point
// (a, b) lands on the exit-wave point
//   q = M_m ((a, b) - n/2) + centre_m + (z - nz/2) t_m,
// each exit-wave pixel takes the bilinear interpolation of the illuminated slice P_z O_z
// (zero off the probe support and off the object) at its pre-image, and the slices are
// summed.
//   k_project_map  one workgroup per frame: each illuminated slice is staged on the probe
//                  window in LDS (with a zero border; the next slice's object values load
//                  while this slice is summed), and each lane sums, over the slices, the
//                  four taps around its footprint pixels' pre-images (a gather: no two
//                  lanes write one pixel)
//   k_bp_map_color the adjoint, per colour of frames (frames of one peak and colour do
//                  not overlap): one workgroup per frame stages its footprint gradient in
//                  LDS; for each slice and window point, the footprint pixels whose
//                  pre-image lies within one sample of the point, with the same tent
//                  weights, times conj(P_z), are added to the slice's frame sum G_{m,z}.
//                  The colours run in order, so every sum has a fixed order; k_bp_chain
//                  then applies the chain rule of eq. (1)/(3) per voxel.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpbp_chain.hpp"
#include "mpbp_dft.hpp"
#include "mpbp_frame.hpp"
#include "mpbp_kernels.hpp"
#include "mpbp_launch.hpp"

namespace mpbp {

// Pre-image, in probe-window coordinates, of footprint pixel (qy, qx) for a slice whose
// window centre lands on c (footprint coordinates): p = M^-1 (q - c) + n/2.  Both
// kernels evaluate it with these operations, so the back-projection's weights are the
// projection's.
__device__ __forceinline__ float2 preimage(const PeakDev& pk, float2 c, float h, int qy, int qx) {
  const float ry = (float)qy - c.x, rx = (float)qx - c.y;
  return make_float2(fmaf(pk.mi[0], ry, fmaf(pk.mi[1], rx, h)), fmaf(pk.mi[2], ry, fmaf(pk.mi[3], rx, h)));
}

// Footprint pixels a lane sums in registers per pass over the slices (a footprint of
// more than kMapThreads * kMapQ pixels takes several passes).
constexpr int kMapQ = 16;
// Probe-window points per lane (probe_n^2 <= kMapThreads * kMapE): the projection stages
// them, the back-projection sums them.
constexpr int kMapE = 4;

template <bool P3>
__global__ __launch_bounds__(kMapThreads) void k_project_map(FrameArgs A) {
  extern __shared__ cplx smem[];
  const int idx = frame_block_index(blockIdx.x, gridDim.x, A.xcd);
  if (idx >= A.n_list) return;
  const int fid = A.list[idx];
  const int m = A.peak_of[fid];
  const PeakDev pk = A.peaks[m];
  const int np = A.np, nz = A.nz, fy = pk.fy, fx = pk.fx;
  const int py = A.scan[2 * fid], px = A.scan[2 * fid + 1];
  const int j = fid - pk.frame_base;
  cplx* slot = reinterpret_cast<cplx*>(A.slots) + pk.slot_off + (long long)j * fy * fx;
  const long long plane = (long long)A.ny * A.nx;
  const cplx* O = reinterpret_cast<const cplx*>(A.obj) + (long long)m * nz * plane;
  const cplx* probe = reinterpret_cast<const cplx*>(A.probe) + (long long)m * (P3 ? nz : 1) * np * np;
  // LDS: the slices' window centres, the probe, and two buffers of an illuminated slice
  // on the probe window with a zero border of one sample (W x W, W = np + 2): a tap off
  // the support or off the object reads an exact zero, so the interpolation needs no
  // bounds checks
  const int W = np + 2;
  float2* cz = reinterpret_cast<float2*>(smem);   // [nz]
  cplx* Ps = smem + nz;                           // [np][np]
  cplx* ill = Ps + np * np;                       // [2][W][W]
  const int tid = threadIdx.x;
  for (int z = tid; z < nz; z += kMapThreads) cz[z] = A.mapz[(long long)m * nz + z];
  if (!P3)
    for (int k = tid; k < np * np; k += kMapThreads) Ps[k] = probe[k];
  for (int k = tid; k < 2 * W * W; k += kMapThreads) ill[k] = {0.f, 0.f};
  // the lane's window points: their place in a staging buffer (-1: none) and their
  // object pixel (-1: off the object, staged as zero)
  int sidx[kMapE];
  long long goff[kMapE];
#pragma unroll
  for (int i = 0; i < kMapE; ++i) {
    const int e = tid + kMapThreads * i, a = e / np, b = e - (e / np) * np;
    const int oy = py + a, ox = px + b;
    sidx[i] = e < np * np ? (a + 1) * W + b + 1 : -1;
    goff[i] = e < np * np && (unsigned)oy < (unsigned)A.ny && (unsigned)ox < (unsigned)A.nx
                  ? (long long)oy * A.nx + ox : -1;
  }
  cplx ov[kMapE];   // the next slice's object values, in flight during this slice's taps
  auto fetch = [&](int z) {
    const cplx* Oz = O + (long long)z * plane;
#pragma unroll
    for (int i = 0; i < kMapE; ++i) ov[i] = goff[i] >= 0 ? Oz[goff[i]] : cplx{0.f, 0.f};
  };
  __syncthreads();
  const float h = 0.5f * (float)np;
  const int npix = fy * fx;
  for (int q0 = 0; q0 < npix; q0 += kMapThreads * kMapQ) {
    cplx acc[kMapQ];
#pragma unroll
    for (int i = 0; i < kMapQ; ++i) acc[i] = {0.f, 0.f};
    fetch(0);
    for (int z = 0; z < nz; ++z) {
      // stage P_z O_z of this frame's window (its interior; the border stays zero).  The
      // other buffer still serves the previous slice: one barrier per slice suffices.
      cplx* buf = ill + (z & 1) * W * W;
      const cplx* Pz = P3 ? probe + (long long)z * np * np : Ps;
#pragma unroll
      for (int i = 0; i < kMapE; ++i)
        if (sidx[i] >= 0) buf[sidx[i]] = goff[i] >= 0 ? cmul(Pz[tid + kMapThreads * i], ov[i]) : cplx{0.f, 0.f};
      __syncthreads();
      if (z + 1 < nz) fetch(z + 1);
      const float2 c = cz[z];
#pragma unroll
      for (int i = 0; i < kMapQ; ++i) {
        const int q = q0 + tid + kMapThreads * i;
        if (q < npix) {
          const int qy = q / fx, qx = q - (q / fx) * fx;
          const float2 p = preimage(pk, c, h, qy, qx);
          if (p.x > -1.f && p.x < (float)np && p.y > -1.f && p.y < (float)np) {
            const float y0 = floorf(p.x), x0 = floorf(p.y);
            // the four taps lie in the bordered window: y0, x0 in [-1, np - 1]
            if (!MPBP_CHECK(A.dbg, y0 >= -1.f && y0 <= (float)(np - 1) && x0 >= -1.f && x0 <= (float)(np - 1),
                            kDbgSlot))
              continue;
            const float ty = p.x - y0, tx = p.y - x0;
            const cplx* t = buf + ((int)y0 + 1) * W + (int)x0 + 1;   // tap (y0, x0)
            const cplx v00 = t[0], v01 = t[1], v10 = t[W], v11 = t[W + 1];
            // bilinear: along x, then along y
            const cplx top = {fmaf(tx, v01.x - v00.x, v00.x), fmaf(tx, v01.y - v00.y, v00.y)};
            const cplx bot = {fmaf(tx, v11.x - v10.x, v10.x), fmaf(tx, v11.y - v10.y, v10.y)};
            acc[i] = {acc[i].x + fmaf(ty, bot.x - top.x, top.x), acc[i].y + fmaf(ty, bot.y - top.y, top.y)};
          }
        }
      }
    }
#pragma unroll
    for (int i = 0; i < kMapQ; ++i) {
      const int q = q0 + tid + kMapThreads * i;
      if (q < npix) slot[q] = acc[i];
    }
    __syncthreads();   // the next pass restages the slices
  }
}

// Footprint pixels q whose pre-image p(q) lies within one sample of window point (a, b):
// the rows are the image of the 2 x 2 square around (a, b); in each row both tent
// conditions |p - (a, b)| < 1 are linear in q_x and give an interval.  The intervals are
// widened by kMapSlack (pixels) against the rounding of their ends, and each pixel's
// weight is then the projection's (its pre-image and tents): a pixel of weight zero adds
// nothing.
constexpr float kMapSlack = 1e-3f;

__device__ __forceinline__ cplx map_gather(const PeakDev& pk, const cplx* __restrict__ gs, float2 c, float h,
                                           float hy, float inv1, float inv3, int a, int b) {
  const float fa = (float)a, fb = (float)b;
  const float qcy = fmaf(pk.mm[0], fa - h, fmaf(pk.mm[1], fb - h, c.x));
  const int qy_lo = max(0, (int)ceilf(qcy - hy - kMapSlack));
  const int qy_hi = min(pk.fy - 1, (int)floorf(qcy + hy + kMapSlack));
  cplx s = {0.f, 0.f};
  for (int qy = qy_lo; qy <= qy_hi; ++qy) {
    const float ry = (float)qy - c.x;
    // p_y - a = by + mi1 (q_x - c_x), p_x - b = bx + mi3 (q_x - c_x), with q_x - c_x = t
    const float by = fmaf(pk.mi[0], ry, h - fa), bx = fmaf(pk.mi[2], ry, h - fb);
    float lo = -1e30f, hi = 1e30f;
    if (inv1 != 0.f) {
      const float t0 = (-1.f - by) * inv1, t1 = (1.f - by) * inv1;
      lo = fmaxf(lo, fminf(t0, t1));
      hi = fminf(hi, fmaxf(t0, t1));
    } else if (fabsf(by) >= 1.f) {
      continue;
    }
    if (inv3 != 0.f) {
      const float t0 = (-1.f - bx) * inv3, t1 = (1.f - bx) * inv3;
      lo = fmaxf(lo, fminf(t0, t1));
      hi = fminf(hi, fmaxf(t0, t1));
    } else if (fabsf(bx) >= 1.f) {
      continue;
    }
    const int qx_lo = max(0, (int)ceilf(fmaxf(lo + c.y - kMapSlack, -1.f)));
    const int qx_hi = min(pk.fx - 1, (int)floorf(fminf(hi + c.y + kMapSlack, (float)pk.fx)));
    for (int qx = qx_lo; qx <= qx_hi; ++qx) {
      const float2 p = preimage(pk, c, h, qy, qx);
      const float wy = 1.f - fabsf(p.x - fa), wx = 1.f - fabsf(p.y - fb);
      if (wy > 0.f && wx > 0.f) s = cadd(s, cscale(gs[qy * pk.fx + qx], wy * wx));
    }
  }
  return s;
}

// map_gather for a map whose inverse has no zero in its second column (mi1, mi3 != 0):
// along a row the tent arguments p - (a, b) and both interval ends change by fixed steps,
// so they are carried from pixel to pixel and from row to row instead of being formed
// anew (pixels of non-positive weight that the slack lets in take weight zero).
__device__ __forceinline__ cplx map_gather_steps(const PeakDev& pk, const cplx* __restrict__ gs, float2 c, float h,
                                                 float hy, float inv1, float inv3, int a, int b) {
  const float fa = (float)a, fb = (float)b;
  const float qcy = fmaf(pk.mm[0], fa - h, fmaf(pk.mm[1], fb - h, c.x));
  const int qy_lo = max(0, (int)ceilf(qcy - hy - kMapSlack));
  const int qy_hi = min(pk.fy - 1, (int)floorf(qcy + hy + kMapSlack));
  const float ry = (float)qy_lo - c.x;
  float by = fmaf(pk.mi[0], ry, h - fa), bx = fmaf(pk.mi[2], ry, h - fb);
  // ends, in t = q_x - c_x, of the intervals of |by + mi1 t| < 1 and |bx + mi3 t| < 1
  const float sg1 = inv1 > 0.f ? 1.f : -1.f, sg3 = inv3 > 0.f ? 1.f : -1.f;
  float loy = (-sg1 - by) * inv1, hiy = (sg1 - by) * inv1;
  float lox = (-sg3 - bx) * inv3, hix = (sg3 - bx) * inv3;
  const float sty = -pk.mi[0] * inv1, stx = -pk.mi[2] * inv3;   // their change per row
  cplx s = {0.f, 0.f};
  const cplx* row = gs + qy_lo * pk.fx;
  for (int qy = qy_lo; qy <= qy_hi; ++qy) {
    const float lo = fmaxf(loy, lox) + c.y, hi = fminf(hiy, hix) + c.y;
    const int qx_lo = max(0, (int)ceilf(fmaxf(lo - kMapSlack, -1.f)));
    const int qx_hi = min(pk.fx - 1, (int)floorf(fminf(hi + kMapSlack, (float)pk.fx)));
    float dy = fmaf(pk.mi[1], (float)qx_lo - c.y, by), dx = fmaf(pk.mi[3], (float)qx_lo - c.y, bx);
    for (int qx = qx_lo; qx <= qx_hi; ++qx) {
      const float w = fmaxf(1.f - fabsf(dy), 0.f) * fmaxf(1.f - fabsf(dx), 0.f);
      const cplx v = row[qx];
      s.x = fmaf(w, v.x, s.x);
      s.y = fmaf(w, v.y, s.y);
      dy += pk.mi[1];
      dx += pk.mi[3];
    }
    by += pk.mi[0];
    bx += pk.mi[2];
    loy += sty; hiy += sty;
    lox += stx; hix += stx;
    row += pk.fx;
  }
  return s;
}

// Back-projection of the frames of one colour (list[0 .. n)): one workgroup per frame
// stages the frame's footprint gradient in LDS and, for every slice z and window point
// (a, b), adds conj(P_z[a, b]) times the tent-weighted sum of its pixels (map_gather) to
// G_{m,z} at object pixel (p_y + a, p_x + b) (read, add, write: the colour's frames of one
// peak do not overlap).  G is complex64 [M][nz][ny][nx] in A.rs.
template <bool P3>
__global__ __launch_bounds__(kMapThreads) void k_bp_map_color(GradArgs A, const int* __restrict__ list, int n) {
  extern __shared__ cplx smem[];
  if ((int)blockIdx.x >= n) return;
  const int fid = list[blockIdx.x];
  if (!A.all_active && !A.active[fid]) return;
  const int m = A.peak_of[fid];
  const PeakDev pk = uniform_peak(A.peaks + m);
  const int np = A.np, nz = A.nz;
  const int py = A.scan[2 * fid], px = A.scan[2 * fid + 1];
  const int npix = pk.fy * pk.fx;
  if (!MPBP_CHECK(A.dbg, npix <= A.map_pix && m >= 0 && m < A.n_peaks, kDbgSlot)) return;   // LDS holds map_pix
  const cplx* g = reinterpret_cast<const cplx*>(A.slots) + pk.slot_off + (long long)(fid - pk.frame_base) * npix;
  const cplx* probe = reinterpret_cast<const cplx*>(A.probe) + (long long)m * (P3 ? nz : 1) * np * np;
  cplx* Ps = smem;             // [np][np] (one probe for all slices)
  cplx* gs = smem + np * np;   // [fy][fx]
  const int tid = threadIdx.x;
  if (!P3)
    for (int k = tid; k < np * np; k += kMapThreads) Ps[k] = probe[k];
  for (int k = tid; k < npix; k += kMapThreads) gs[k] = g[k];
  __syncthreads();
  const float h = 0.5f * (float)np;
  const float hy = fabsf(pk.mm[0]) + fabsf(pk.mm[1]);
  const float inv1 = pk.mi[1] != 0.f ? 1.f / pk.mi[1] : 0.f;
  const float inv3 = pk.mi[3] != 0.f ? 1.f / pk.mi[3] : 0.f;
  const bool steps = inv1 != 0.f && inv3 != 0.f;   // uniform
  cplx* G = reinterpret_cast<cplx*>(A.rs) + (long long)m * nz * A.nlat;
  int a[kMapE], b[kMapE];
  long long off[kMapE];   // object pixel of window point e (-1: off the window or the grid)
#pragma unroll
  for (int i = 0; i < kMapE; ++i) {
    const int e = tid + kMapThreads * i;
    a[i] = e / np;
    b[i] = e - a[i] * np;
    const int oy = py + a[i], ox = px + b[i];
    const bool in = e < np * np && (unsigned)oy < (unsigned)A.ny && (unsigned)ox < (unsigned)A.nx;
    off[i] = in ? (long long)oy * A.nx + ox : -1;
  }
  for (int z = 0; z < nz; ++z) {
    const float2 c = A.mapz[(long long)m * nz + z];
    const cplx* Pz = P3 ? probe + (long long)z * np * np : Ps;
    cplx* Gz = G + (long long)z * A.nlat;
    cplx old[kMapE];
#pragma unroll
    for (int i = 0; i < kMapE; ++i) old[i] = off[i] >= 0 ? Gz[off[i]] : cplx{0.f, 0.f};
#pragma unroll
    for (int i = 0; i < kMapE; ++i) {
      if (off[i] >= 0) {
        const cplx s = steps ? map_gather_steps(pk, gs, c, h, hy, inv1, inv3, a[i], b[i])
                             : map_gather(pk, gs, c, h, hy, inv1, inv3, a[i], b[i]);
        Gz[off[i]] = cmulc_acc(old[i], s, Pz[a[i] * np + b[i]]);
      }
    }
  }
}

hipError_t prepare_map_kernels() {
  hipError_t e = hipFuncSetAttribute((const void*)k_bp_map_color<false>, hipFuncAttributeMaxDynamicSharedMemorySize,
                                     160 * 1024);
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_bp_map_color<true>, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  return e;
}

hipError_t launch_project_map(const FrameArgs& a, hipStream_t s) {
  const unsigned grid = a.xcd ? (unsigned)(((a.n_list + 7) / 8) * 8) : (unsigned)a.n_list;
  if (grid == 0) return hipSuccess;
  const size_t W = (size_t)a.np + 2;
  const size_t lds = (size_t)a.nz * sizeof(float2) + ((size_t)a.np * a.np + 2 * W * W) * sizeof(cplx);
  if (a.probe3)
    k_project_map<true><<<dim3(grid), dim3(kMapThreads), lds, s>>>(a);
  else
    k_project_map<false><<<dim3(grid), dim3(kMapThreads), lds, s>>>(a);
  return hipGetLastError();
}

// G = 0, one launch of k_bp_map_color per colour (in colour order: each object pixel
// adds its frames in a fixed order), then the chain rule per voxel (k_bp_chain, with
// slice z of peak m as run m nz + z).
hipError_t launch_grad_map(const GradArgs& a, hipStream_t s) {
  static_assert((kProjMaxPix + kMapThreads * kMapE) * sizeof(cplx) <= 160 * 1024, "k_bp_map_color's LDS");
  if (!a.color_off || a.n_colors < 1 || a.np * a.np > kMapThreads * kMapE || a.map_pix > kProjMaxPix)
    return hipErrorInvalidValue;
  hipError_t e = launch_fill(a.rs, 2LL * a.n_peaks * a.nz * a.nlat, 0.f, s);
  const size_t lds = ((size_t)a.np * a.np + (size_t)a.map_pix) * sizeof(cplx);
  for (int c = 0; c < a.n_colors && e == hipSuccess; ++c) {
    const int n = a.color_off[c + 1] - a.color_off[c];
    if (n <= 0) continue;
    const int* list = a.color_list + a.color_off[c];
    if (a.probe3)
      k_bp_map_color<true><<<dim3((unsigned)n), dim3(kMapThreads), lds, s>>>(a, list, n);
    else
      k_bp_map_color<false><<<dim3((unsigned)n), dim3(kMapThreads), lds, s>>>(a, list, n);
    e = hipGetLastError();
  }
  if (e != hipSuccess) return e;
  return launch_bp_chain(a, s);
}

}  // namespace mpbp
