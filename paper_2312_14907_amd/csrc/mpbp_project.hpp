// mpbp_project.hpp - the per-frame projection kernel (one workgroup per frame):
// eq. (2) R diag(P) S O, the exit wave on the frame's footprint, written to the frame's
// slot for the frame kernel.  A kernel of its own: it needs little LDS and few
// registers, so many workgroups share a CU and hide the latency of the object reads,
// which the FFT-heavy frame kernel (two workgroups per CU) cannot.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpbp_frame.hpp"

namespace mpbp {

// G: object slices in flight per lane (the slices are loaded in blocks of G).
//
// eq. (2) R diag(P) S O on the footprint: psi[q] = sum_z (P O_z)[q - s(z) + min s].
// Consecutive slices with equal shear offset (runs, uniform) are summed in registers;
// at the end of a run each lane adds its probe pixels of the run's sum into the
// footprint accumulator in LDS at the run's offset.  Within one run every footprint
// pixel receives at most one value, so no two lanes collide; a barrier separates runs,
// which keeps the order of every sum fixed.
// P3: the probe varies along z (probe [M][nz][np][np]); P_z O_z is formed per slice
// before the run sums.  LIN: fractional exit-beam offsets (A.shw): a slice reaches the
// offsets s0 + (dy, dx), dy, dx in {0, 1}, with bilinear weights; a run (equal s0)
// keeps four weighted sums, and its additions go out one tap at a time (a barrier
// between taps: within a tap no two lanes meet).
template <int G, bool P3, bool LIN>
__device__ void project_body(const FrameArgs& A, const PeakDev& pk, int fid, cplx* sm) {
  constexpr int NT = kFrameThreads;
  const int tid = threadIdx.x;
  const int np = A.np, nz = A.nz;
  const int fy = pk.fy, fx = pk.fx;
  const int m = A.peak_of[fid];
  const int py = A.scan[2 * fid], px = A.scan[2 * fid + 1];
  const int j = fid - pk.frame_base;
  const long long pstride = P3 ? (long long)np * np : 0;   // probe slice stride
  const cplx* probe = reinterpret_cast<const cplx*>(A.probe) + (long long)m * (P3 ? nz : 1) * np * np;
  cplx* slot = reinterpret_cast<cplx*>(A.slots) + pk.slot_off + (long long)j * fy * fx;
  const cplx* O = reinterpret_cast<const cplx*>(A.obj) + (long long)m * nz * A.ny * A.nx;
  const int* shz = A.shear + 2 * m * nz;   // uniform: scalar loads
  const int np2 = np * np;
  cplx* acc = sm;                          // [fy][fx] footprint accumulator
  // per-slice footprint offsets (and interpolation fractions) in LDS: the slice loop
  // then reads nothing from device memory but the object, and the waits for the
  // object loads issued G slices ahead cover those loads alone
  int* sho = reinterpret_cast<int*>(acc + A.acc_pix);                                 // [nz]
  float2* shf = reinterpret_cast<float2*>(sho + ((nz + 3) & ~3));                     // [nz] (LIN)
  for (int p = tid; p < fy * fx; p += NT) acc[p] = {0.f, 0.f};
  for (int z = tid; z < nz; z += NT) {
    sho[z] = (shz[2 * z] - pk.miny) * fx + (shz[2 * z + 1] - pk.minx);
    if constexpr (LIN) shf[z] = make_float2(A.shw[2 * (m * nz + z)], A.shw[2 * (m * nz + z) + 1]);
  }
  __syncthreads();

  // lane's probe pixels e = tid + NT i: probe value (0 off the object), object offset,
  // and footprint offset at zero shear
  cplx pv[kProjE];
  unsigned off[kProjE];   // byte offset in a slice: a 32-bit lane offset from a uniform base
  int fo[kProjE], pe[kProjE];
  bool pok[kProjE];
#pragma unroll
  for (int i = 0; i < kProjE; ++i) {
    const int e = tid + NT * i;
    const int a = e / np, b = e - (e / np) * np;
    const int oy = py + a, ox = px + b;
    const bool ok = e < np2 && (unsigned)oy < (unsigned)A.ny && (unsigned)ox < (unsigned)A.nx;
    pv[i] = ok ? probe[e < np2 ? e : 0] : cplx{0.f, 0.f};
    pe[i] = e < np2 ? e : 0;
    pok[i] = ok;
    off[i] = ok ? (unsigned)(oy * A.nx + ox) * (unsigned)sizeof(cplx) : 0u;
    fo[i] = a * fx + b;
  }
  // Object reads: a uniform slice base plus the lane's 32-bit byte offset.  The slice
  // index passes through readfirstlane, which hides the affine recurrence from the
  // compiler's strength reduction; otherwise it keeps one 64-bit pointer per load live
  // across the loop and spills them.
  const long long plane = (long long)A.ny * A.nx;
  auto load = [&](cplx (&o)[kProjE], cplx (&q)[P3 ? kProjE : 1], int z) {
    const int zz = __builtin_amdgcn_readfirstlane(z < nz ? z : nz - 1);
    const char* Oz = reinterpret_cast<const char*>(O + (long long)zz * plane);
#pragma unroll
    for (int i = 0; i < kProjE; ++i) o[i] = *reinterpret_cast<const cplx*>(Oz + off[i]);
    if constexpr (P3) {
      const cplx* Pz = probe + (long long)zz * pstride;
#pragma unroll
      for (int i = 0; i < kProjE; ++i) q[i] = pok[i] ? Pz[pe[i]] : cplx{0.f, 0.f};
    }
  };
  // footprint offset of slice z's pixel (0, 0): (s_y - min s_y) fx + (s_x - min s_x)
  auto shift = [&](int z) { return __builtin_amdgcn_readfirstlane(sho[z]); };
  constexpr int NW = LIN ? 4 : 1;   // weighted sums per run (taps)
  cplx w[NW][kProjE];
  auto flush = [&](int d) {
#pragma unroll
    for (int tp = 0; tp < NW; ++tp) {
      const int to = d + (tp >> 1) * fx + (tp & 1);   // tap (dy, dx) = (tp / 2, tp % 2)
      __syncthreads();   // zeroing, or the previous additions, are complete
#pragma unroll
      for (int i = 0; i < kProjE; ++i) {
        if ((i + 1) * NT <= np2 || tid + NT * i < np2) {   // uniform when every lane has a pixel
          if (MPBP_CHECK(A.dbg, (unsigned)(fo[i] + to) < (unsigned)(fy * fx), kDbgAccumulator)) {
            cplx* q = acc + fo[i] + to;
            *q = cadd(*q, w[tp][i]);
          }
        }
      }
    }
  };
  // add slice z's P O (v) into the run's sums
  auto accumulate = [&](const cplx (&v)[kProjE], int z, bool first) {
    if constexpr (LIN) {
      const float2 f = shf[z];
      const float ry = f.x, rx = f.y;   // fractions
      const float wt[4] = {(1.f - ry) * (1.f - rx), (1.f - ry) * rx, ry * (1.f - rx), ry * rx};
#pragma unroll
      for (int tp = 0; tp < 4; ++tp)
#pragma unroll
        for (int i = 0; i < kProjE; ++i) {
          const cplx t = cscale(v[i], wt[tp]);
          w[tp][i] = first ? t : cadd(w[tp][i], t);
        }
    } else {
#pragma unroll
      for (int i = 0; i < kProjE; ++i) w[0][i] = first ? v[i] : cadd(w[0][i], v[i]);
    }
  };
  // Slices go in blocks of G: all G slices' loads are issued, then consumed in order.
  // Nothing loaded is carried across the loop's back-edge, so the compiler waits for
  // exactly the loads each slice uses (with a prefetch carried across iterations it
  // copied the buffers at the back-edge and waited for every load there); a frame
  // costs nz / G memory latencies.
  int cur = shift(0);
#pragma unroll
  for (int tp = 0; tp < NW; ++tp)
#pragma unroll
    for (int i = 0; i < kProjE; ++i) w[tp][i] = {0.f, 0.f};
  for (int z0 = 0; z0 < nz; z0 += G) {
    cplx buf[G][kProjE], pbuf[G][P3 ? kProjE : 1];
#pragma unroll
    for (int g = 0; g < G; ++g) load(buf[g], pbuf[g], z0 + g);   // clamped past nz
#pragma unroll
    for (int g = 0; g < G; ++g) {
      const int z = z0 + g;
      if (z < nz) {   // uniform
        cplx v[kProjE];
#pragma unroll
        for (int i = 0; i < kProjE; ++i) v[i] = cmul(P3 ? pbuf[g][P3 ? i : 0] : pv[i], buf[g][i]);
        const int d = shift(z);
        if (d != cur) {   // uniform: a new run
          flush(cur);
          cur = d;
          accumulate(v, z, true);
        } else {
          accumulate(v, z, false);
        }
      }
    }
  }
  flush(cur);
  __syncthreads();
  for (int p = tid; p < fy * fx; p += NT) slot[p] = acc[p];
}

// The projection from the run sums (one probe for all slices, rounded offsets):
//   psi = sum_k shift_{s_k}( P . S_k[window] )
// with S_k from launch_runsum.  A frame reads its window of each run's sum (about a
// third of the slices at the workloads' shears), G runs' loads in flight per lane; each
// run's P . S_k is added into the LDS footprint accumulator at the run's offset (a
// barrier per run: within one run no two lanes meet).
template <int G>
__device__ void project_runs_body(const FrameArgs& A, const PeakDev& pk, int fid, cplx* sm) {
  constexpr int NT = kFrameThreads;
  const int tid = threadIdx.x;
  const int np = A.np, nz = A.nz;
  const int fy = pk.fy, fx = pk.fx;
  const int m = A.peak_of[fid];
  const int py = A.scan[2 * fid], px = A.scan[2 * fid + 1];
  const int j = fid - pk.frame_base;
  const cplx* probe = reinterpret_cast<const cplx*>(A.probe) + (long long)m * np * np;
  cplx* slot = reinterpret_cast<cplx*>(A.slots) + pk.slot_off + (long long)j * fy * fx;
  const long long plane = (long long)A.ny * A.nx;
  const cplx* S = reinterpret_cast<const cplx*>(A.obj) + (long long)pk.run_base * plane;
  const int np2 = np * np;
  const int nr = pk.nruns;
  cplx* acc = sm;                                                     // [fy][fx]
  int* sho = reinterpret_cast<int*>(acc + A.acc_pix);                 // [nruns] footprint offsets
  for (int p = tid; p < fy * fx; p += NT) acc[p] = {0.f, 0.f};
  for (int k = tid; k < nr; k += NT) {
    const int2 ro = A.roff[m * nz + k];
    sho[k] = ro.x * fx + ro.y;
  }
  cplx pv[kProjE];
  unsigned off[kProjE];
  int fo[kProjE];
#pragma unroll
  for (int i = 0; i < kProjE; ++i) {
    const int e = tid + NT * i;
    const int a = e / np, b = e - (e / np) * np;
    const int oy = py + a, ox = px + b;
    const bool ok = e < np2 && (unsigned)oy < (unsigned)A.ny && (unsigned)ox < (unsigned)A.nx;
    pv[i] = ok ? probe[e < np2 ? e : 0] : cplx{0.f, 0.f};
    off[i] = ok ? (unsigned)(oy * A.nx + ox) * (unsigned)sizeof(cplx) : 0u;
    fo[i] = a * fx + b;
  }
  __syncthreads();
  for (int k0 = 0; k0 < nr; k0 += G) {
    cplx buf[G][kProjE];
#pragma unroll
    for (int g = 0; g < G; ++g) {   // run index clamped past the last run
      int k = __builtin_amdgcn_readfirstlane(k0 + g < nr ? k0 + g : nr - 1);
      if (!MPBP_CHECK(A.dbg, k >= 0 && pk.run_base + k < A.n_runs, kDbgRunSum)) k = 0;
      const char* Sk = reinterpret_cast<const char*>(S + (long long)k * plane);
#pragma unroll
      for (int i = 0; i < kProjE; ++i) buf[g][i] = *reinterpret_cast<const cplx*>(Sk + off[i]);
    }
#pragma unroll
    for (int g = 0; g < G; ++g) {
      if (k0 + g < nr) {   // uniform
        const int d = __builtin_amdgcn_readfirstlane(sho[k0 + g]);
        __syncthreads();   // zeroing, or the previous run's additions, are complete
#pragma unroll
        for (int i = 0; i < kProjE; ++i) {
          if ((i + 1) * NT <= np2 || tid + NT * i < np2) {   // uniform when every lane has a pixel
            if (MPBP_CHECK(A.dbg, (unsigned)(fo[i] + d) < (unsigned)(fy * fx), kDbgAccumulator)) {
              cplx* q = acc + fo[i] + d;
              *q = cadd(*q, cmul(pv[i], buf[g][i]));
            }
          }
        }
      }
    }
  }
  __syncthreads();
  for (int p = tid; p < fy * fx; p += NT) slot[p] = acc[p];
}

// Occupancy target: the fewer slices in flight, the fewer registers, the more
// workgroups per CU.
template <int G, bool LIN> struct ProjectWaves {
  static constexpr int value = LIN ? (G <= 2 ? 5 : G <= 4 ? 4 : 3) : (G <= 2 ? 8 : G <= 4 ? 6 : 4);
};

template <int G, bool P3, bool LIN>
__global__ __launch_bounds__(kFrameThreads) __attribute__((amdgpu_waves_per_eu(ProjectWaves<G, LIN>::value)))
void k_project(FrameArgs A) {
  extern __shared__ cplx smem[];
  const int idx = frame_block_index(blockIdx.x, gridDim.x, A.xcd);
  if (idx >= A.n_list) return;
  const int fid = A.list[idx];
  const PeakDev pk = A.peaks[A.peak_of[fid]];
  project_body<G, P3, LIN>(A, pk, fid, smem);
}

}  // namespace mpbp

namespace mpbp {

template <int G>
__global__ __launch_bounds__(kFrameThreads) __attribute__((amdgpu_waves_per_eu(ProjectWaves<G, false>::value)))
void k_project_runs(FrameArgs A) {
  extern __shared__ cplx smem[];
  const int idx = frame_block_index(blockIdx.x, gridDim.x, A.xcd);
  if (idx >= A.n_list) return;
  const int fid = A.list[idx];
  const PeakDev pk = A.peaks[A.peak_of[fid]];
  project_runs_body<G>(A, pk, fid, smem);
}

}  // namespace mpbp
