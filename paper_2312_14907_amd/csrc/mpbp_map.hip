// mpbp_map.hip - R with a detector-frame map (MPBP_DETECTOR_MAP).  Section 2: each Bragg
// peak's exit wave lives in that peak's detector frame, which is turned against the
// object's frame and sampled at a pixel size of its own.  Slice z's probe-window point
// (a, b) lands on the exit-wave point
//   q = M_m ((a, b) - n/2) + centre_m + (z - nz/2) t_m,
// each exit-wave pixel takes the bilinear interpolation of the illuminated slice P_z O_z
// (zero off the probe support and off the object) at its pre-image, and the slices are
// summed.
//   k_project_map  one workgroup per frame: each lane owns footprint pixels and sums, over
//                  the slices, the four taps around the pixel's pre-image (a gather: no
//                  two lanes write one pixel, so no accumulator in LDS)
//   k_grad_map     one lane per voxel (per lateral pixel when z-tied): for each covering
//                  frame of the minibatch, the footprint pixels whose pre-image lies
//                  within one sample of the voxel's probe-window point, with the same tent
//                  weights (the adjoint of the interpolation), times conj(P_z); then the
//                  chain rule of eq. (1)/(3).  Every sum runs in a fixed order.
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
  float2* cz = reinterpret_cast<float2*>(smem);   // [nz] window centre of each slice
  cplx* Ps = smem + nz;                           // [np][np] (one probe for all slices)
  for (int z = threadIdx.x; z < nz; z += kMapThreads) cz[z] = A.mapz[(long long)m * nz + z];
  if (!P3)
    for (int k = threadIdx.x; k < np * np; k += kMapThreads) Ps[k] = probe[k];
  __syncthreads();
  // taps (a, b) are live inside the probe support and over the object grid
  const int a0 = max(0, -py), a1 = min(np, A.ny - py);
  const int b0 = max(0, -px), b1 = min(np, A.nx - px);
  const float h = 0.5f * (float)np;
  for (int q = threadIdx.x; q < fy * fx; q += kMapThreads) {
    const int qy = q / fx, qx = q - (q / fx) * fx;
    cplx acc = {0.f, 0.f};
    for (int z = 0; z < nz; ++z) {
      const float2 p = preimage(pk, cz[z], h, qy, qx);
      if (!(p.x > -1.f && p.x < (float)np && p.y > -1.f && p.y < (float)np)) continue;
      const float y0 = floorf(p.x), x0 = floorf(p.y);
      const float ty = p.x - y0, tx = p.y - x0;
      const int iy = (int)y0, ix = (int)x0;
      const cplx* Oz = O + (long long)z * plane;
      const cplx* Pz = P3 ? probe + (long long)z * np * np : Ps;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int a = iy + (t >> 1), b = ix + (t & 1);
        if (a >= a0 && a < a1 && b >= b0 && b < b1) {
          const float w = ((t >> 1) ? ty : 1.f - ty) * ((t & 1) ? tx : 1.f - tx);
          const cplx v = cmul(Pz[a * np + b], Oz[(long long)(py + a) * A.nx + (px + b)]);
          acc = cadd(acc, cscale(v, w));
        }
      }
    }
    slot[q] = acc;
  }
}

template <bool P3>
__global__ __launch_bounds__(kMapThreads) void k_grad_map(GradArgs A) {
  __shared__ float red[kMapThreads / 64];
  __shared__ double apl[kMaxPeaksDev];
  const int tid = threadIdx.x;
  const int np = A.np, nz = A.nz;
  const long long nlat = (long long)A.ny * A.nx;
  const long long nvox = nlat * nz;
  const long long task = (long long)blockIdx.x * kMapThreads + tid;
  const bool live = task < (A.tied ? nlat : nvox);
  const long long lat = live ? task % nlat : 0;
  const int zlo = (A.tied || !live) ? 0 : (int)(task / nlat);
  const int zhi = !live ? 0 : A.tied ? nz : zlo + 1;
  const int y = (int)(lat / A.nx), x = (int)(lat - (lat / A.nx) * A.nx);
  const long long fstride = A.tied ? nlat : nvox;   // field component stride
  const float h = 0.5f * (float)np;
  const cplx* slots = reinterpret_cast<const cplx*>(A.slots);
  if (tid < kMaxPeaksDev) apl[tid] = 0.0;
  float gux = 0.f, guy = 0.f, guz = 0.f, gch = 0.f;
  for (int m = 0; m < A.n_peaks; ++m) {
    const PeakDev pk = uniform_peak(A.peaks + m);
    const cplx* probe = reinterpret_cast<const cplx*>(A.probe) + (long long)m * (P3 ? nz : 1) * np * np;
    const float al = A.alpha[m];
    // frames whose window covers (y, x): window origin p with p <= (y, x) < p + np
    const int iy_lo = max(0, -floordiv(-(y - np + 1 - pk.oy), pk.sy));
    const int iy_hi = min(pk.rows - 1, floordiv(y - pk.oy, pk.sy));
    const int ix_lo = max(0, -floordiv(-(x - np + 1 - pk.ox), pk.sx));
    const int ix_hi = min(pk.cols - 1, floordiv(x - pk.ox, pk.sx));
    // exit-wave pixels within one sample of a point: the image of a 2 x 2 square
    const float hy = fabsf(pk.mm[0]) + fabsf(pk.mm[1]), hx = fabsf(pk.mm[2]) + fabsf(pk.mm[3]);
    float ap = 0.f;
    for (int z = zlo; z < zhi; ++z) {
      const float2 c = A.mapz[(long long)m * nz + z];
      const cplx* Pz = probe + (P3 ? (long long)z * np * np : 0);
      cplx acc = {0.f, 0.f};
      for (int iy = iy_lo; iy <= iy_hi; ++iy)
        for (int ix = ix_lo; ix <= ix_hi; ++ix) {
          const int f = iy * pk.cols + ix;
          if (!A.all_active && !A.active[pk.frame_base + f]) continue;
          const int a = y - (pk.oy + iy * pk.sy), b = x - (pk.ox + ix * pk.sx);
          const float ca = (float)a - h, cb = (float)b - h;
          const float qcy = fmaf(pk.mm[0], ca, fmaf(pk.mm[1], cb, c.x));
          const float qcx = fmaf(pk.mm[2], ca, fmaf(pk.mm[3], cb, c.y));
          const int qy0 = (int)floorf(qcy - hy), qx0 = (int)floorf(qcx - hx);
          const cplx* g = slots + pk.slot_off + (long long)f * pk.fy * pk.fx;
          cplx s = {0.f, 0.f};
          for (int dy = 0; dy < pk.ncy; ++dy) {
            const int qy = qy0 + dy;
            if ((unsigned)qy >= (unsigned)pk.fy) continue;
            for (int dx = 0; dx < pk.ncx; ++dx) {
              const int qx = qx0 + dx;
              if ((unsigned)qx >= (unsigned)pk.fx) continue;
              const float2 p = preimage(pk, c, h, qy, qx);
              const float wy = 1.f - fabsf(p.x - (float)a), wx = 1.f - fabsf(p.y - (float)b);
              if (wy > 0.f && wx > 0.f) s = cadd(s, cscale(g[qy * pk.fx + qx], wy * wx));
            }
          }
          acc = cmulc_acc(acc, s, Pz[a * np + b]);   // conj(P_z) times the weighted sum
        }
      const long long v = A.tied ? lat : (long long)z * nlat + lat;
      chain_voxel(pk, acc, A.u[v], A.u[fstride + v], A.u[2 * fstride + v], A.chi[v], al, gux, guy, guz, gch, ap);
    }
    const float apb = block_sum_f(ap, red);
    if (tid == 0) apl[m] += (double)apb;
  }
  if (live) {
    const long long v = A.tied ? lat : (long long)zlo * nlat + lat;
    A.grad_u[v] = gux;
    A.grad_u[fstride + v] = guy;
    A.grad_u[2 * fstride + v] = guz;
    A.grad_chi[v] = gch;
  }
  __syncthreads();
  if (tid < A.n_peaks) A.alpha_part[(long long)blockIdx.x * A.n_peaks + tid] = apl[tid];
}

static unsigned map_blocks(long long n) { return (unsigned)((n + kMapThreads - 1) / kMapThreads); }

hipError_t launch_project_map(const FrameArgs& a, hipStream_t s) {
  const unsigned grid = a.xcd ? (unsigned)(((a.n_list + 7) / 8) * 8) : (unsigned)a.n_list;
  if (grid == 0) return hipSuccess;
  const size_t lds = (size_t)a.nz * sizeof(float2) + (size_t)a.np * a.np * sizeof(cplx);
  if (a.probe3)
    k_project_map<true><<<dim3(grid), dim3(kMapThreads), lds, s>>>(a);
  else
    k_project_map<false><<<dim3(grid), dim3(kMapThreads), lds, s>>>(a);
  return hipGetLastError();
}

int grad_map_partials(const GradArgs& a) {
  const long long nlat = (long long)a.ny * a.nx;
  return (int)map_blocks(a.tied ? nlat : nlat * a.nz);
}

hipError_t launch_grad_map(const GradArgs& a, hipStream_t s) {
  const unsigned grid = (unsigned)grad_map_partials(a);
  if (a.probe3)
    k_grad_map<true><<<dim3(grid), dim3(kMapThreads), 0, s>>>(a);
  else
    k_grad_map<false><<<dim3(grid), dim3(kMapThreads), 0, s>>>(a);
  return hipGetLastError();
}

}  // namespace mpbp
