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

// G: object slices staged per step (the slab depth).
template <int G>
__device__ void project_body(const FrameArgs& A, const PeakDev& pk, int fid, cplx* sm) {
  constexpr int NT = kFrameThreads;
  const int tid = threadIdx.x;
  const int np = A.np, nz = A.nz;
  const int fy = pk.fy, fx = pk.fx;
  const int m = A.peak_of[fid];
  const int py = A.scan[2 * fid], px = A.scan[2 * fid + 1];
  const int j = fid - pk.frame_base;
  const cplx* probe = reinterpret_cast<const cplx*>(A.probe) + (long long)m * np * np;
  cplx* slot = reinterpret_cast<cplx*>(A.slots) + pk.slot_off + (long long)j * fy * fx;
  const cplx* O = reinterpret_cast<const cplx*>(A.obj) + (long long)m * nz * A.ny * A.nx;
  // The illuminated slices W_z = P * O[z, window], summed over runs of slices with equal
  // shear offset within each group of G slices, are staged in LDS; each lane then
  // gathers its footprint pixels
  //   psi[q] += W_z[q + min shear - s(z)]   (zero outside the probe support).
  // A staged slice is (np + 1) x (np + 1) with a zero last row and column: offsets
  // outside the support are clamped onto them, so the gather has no tests or branches.
  {
    const int np1 = np + 1;
    const int sw = np1 * np1;
    const int np2 = np * np;
    cplx* Wb = sm;
    const int* shz = A.shear + 2 * m * nz;   // uniform: scalar loads
    for (int k = tid; k < G * (2 * np + 1); k += NT) {
      const int g = k / (2 * np + 1), e = k - g * (2 * np + 1);
      Wb[g * sw + (e <= np ? np * np1 + e : (e - np - 1) * np1 + np)] = {0.f, 0.f};
    }
    cplx pv[kProjE];
    int off[kProjE], wo[kProjE];
#pragma unroll
    for (int i = 0; i < kProjE; ++i) {
      const int e = tid + NT * i;
      const int a = e / np, b = e - (e / np) * np;
      const int oy = py + a, ox = px + b;
      const bool ok = e < np2 && (unsigned)oy < (unsigned)A.ny && (unsigned)ox < (unsigned)A.nx;
      pv[i] = ok ? probe[e < np2 ? e : 0] : cplx{0.f, 0.f};
      off[i] = ok ? oy * A.nx + ox : 0;
      wo[i] = e < np2 ? a * np1 + b : -1;
    }
    const long long plane = (long long)A.ny * A.nx;
    // Object values of two groups of G slices are in flight: group k + 2 is requested
    // while group k is used (the loads are L2 round trips that one group's work does
    // not cover).
    auto load_group = [&](cplx (&on)[G][kProjE], int z0) {
#pragma unroll
      for (int g = 0; g < G; ++g) {
        const int z = z0 + g < nz ? z0 + g : nz - 1;
        const cplx* Oz = O + (long long)z * plane;
#pragma unroll
        for (int i = 0; i < kProjE; ++i) on[g][i] = Oz[off[i]];
      }
    };
    cplx onA[G][kProjE], onB[G][kProjE];
    load_group(onA, 0);
    load_group(onB, G);
    // Footprint pixel q = (qy, qx) of slice z reads staged element (qy + min s_y -
    // s_y(z), qx + min s_x - s_x(z)), each coordinate clamped to np (the zero border).
    // Both coordinates travel as one pair of 16-bit lanes: one packed subtract, one
    // packed clamp and one dot product (row * (np + 1) * 8 + column * 8 + slot base)
    // give the byte address of the element.
    u16x2 pq[kProjPix];
    cplx acc[kProjPix];
#pragma unroll
    for (int h = 0; h < kProjPix; ++h) {
      const int p = tid + NT * h;
      const int qy = p / fx;
      pq[h] = u16x2{(unsigned short)(p - qy * fx + pk.minx), (unsigned short)(qy + pk.miny)};
      acc[h] = {0.f, 0.f};
    }
    const u16x2 lim = {(unsigned short)np, (unsigned short)np};
    const u16x2 wts = {(unsigned short)sizeof(cplx), (unsigned short)(np1 * sizeof(cplx))};
    const unsigned wb_lds = (unsigned)(size_t)(const lds_cplx*)Wb;   // LDS byte address of slot 0
    u16x2* slot_shift = reinterpret_cast<u16x2*>(Wb + G * sw);      // shear of each staged slot
    auto stage = [&](const cplx (&w)[kProjE], int sl) {
#pragma unroll
      for (int i = 0; i < kProjE; ++i) {
        if ((i + 1) * NT <= np2)   // uniform: every lane holds a probe pixel
          Wb[sl * sw + wo[i]] = w[i];
        else if (wo[i] >= 0)
          Wb[sl * sw + wo[i]] = w[i];
      }
    };
    // One group: slices with equal shear offset (runs, uniform) are summed in registers
    // and staged once, then every footprint pixel gathers from the staged slots.
    auto step = [&](cplx (&on)[G][kProjE], int z0) {
      __syncthreads();   // the previous group's gather is done with the slots
      int nsl = 0;
      int cy = shz[2 * z0], cx = shz[2 * z0 + 1];
      cplx w[kProjE];
#pragma unroll
      for (int i = 0; i < kProjE; ++i) w[i] = cmul(pv[i], on[0][i]);
#pragma unroll
      for (int g = 1; g < G; ++g) {
        const int z = z0 + g;
        if (z < nz) {   // uniform
          const int sy = shz[2 * z], sx = shz[2 * z + 1];
          if (sy != cy || sx != cx) {   // uniform: a new run
            stage(w, nsl);
            if (tid == 0) slot_shift[nsl] = u16x2{(unsigned short)cx, (unsigned short)cy};
            ++nsl;
            cy = sy;
            cx = sx;
#pragma unroll
            for (int i = 0; i < kProjE; ++i) w[i] = cmul(pv[i], on[g][i]);
          } else {
#pragma unroll
            for (int i = 0; i < kProjE; ++i) w[i] = cadd(w[i], cmul(pv[i], on[g][i]));
          }
        }
      }
      stage(w, nsl);
      if (tid == 0) slot_shift[nsl] = u16x2{(unsigned short)cx, (unsigned short)cy};
      ++nsl;
      load_group(on, z0 + 2 * G);
      __syncthreads();
      for (int k = 0; k < nsl; ++k) {   // uniform trip count
        const u16x2 sh = slot_shift[k];
        const unsigned base = wb_lds + (unsigned)(k * sw * sizeof(cplx));
#pragma unroll
        for (int h = 0; h < kProjPix; ++h) {
          const u16x2 d = __builtin_elementwise_min(pq[h] - sh, lim);
          const lds_cplx* q = (const lds_cplx*)(size_t)__builtin_amdgcn_udot2(d, wts, base, false);
          acc[h] = cadd(acc[h], cplx{q->x, q->y});
        }
      }
    };
    for (int z0 = 0; z0 < nz; z0 += 2 * G) {
      step(onA, z0);
      if (z0 + G < nz) step(onB, z0 + G);   // uniform
    }
#pragma unroll
    for (int h = 0; h < kProjPix; ++h)
      if (tid + NT * h < fy * fx) slot[tid + NT * h] = acc[h];
  }

}

// Occupancy target: the shallower the slab, the less LDS and the fewer registers, the
// more workgroups per CU.
template <int G> struct ProjectWaves { static constexpr int value = G <= 2 ? 5 : G <= 4 ? 4 : 2; };

template <int G>
__global__ __launch_bounds__(kFrameThreads) __attribute__((amdgpu_waves_per_eu(ProjectWaves<G>::value)))
void k_project(FrameArgs A) {
  extern __shared__ cplx smem[];
  const int idx = frame_block_index(blockIdx.x, gridDim.x, A.xcd);
  if (idx >= A.n_list) return;
  const int fid = A.list[idx];
  const PeakDev pk = A.peaks[A.peak_of[fid]];
  project_body<G>(A, pk, fid, smem);
}

}  // namespace mpbp
