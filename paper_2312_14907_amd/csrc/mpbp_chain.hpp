// mpbp_chain.hpp - device helpers shared by the back-projection kernels: the chain rule
// of one voxel through eq. (1)/(3), written out so that every kernel rounds it alike,
// block sums, and the uniform read of a peak record.
#pragma once
#include <hip/hip_runtime.h>

#include "mpbp_dft.hpp"
#include "mpbp_kernels.hpp"
#include "mpbp_phase.hpp"

namespace mpbp {

__device__ __forceinline__ int floordiv(int a, int b) {  // b > 0
  int q = a / b;
  return (a % b != 0 && a < 0) ? q - 1 : q;
}

__device__ __forceinline__ float block_sum_f(float v, float* red) {
  for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
  __syncthreads();
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  float s = 0.f;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) s += red[w];
  __syncthreads();
  return s;
}

// acc + a conj(b) with the two fused multiply-adds per component written out, so that
// every instance of the gradient kernel rounds the frame sums the same way (left to the
// compiler, the contraction into FMAs differs between instances).
__device__ __forceinline__ cplx cmulc_acc(cplx acc, cplx a, cplx b) {
  return {fmaf(a.x, b.x, fmaf(a.y, b.y, acc.x)), fmaf(a.y, b.x, fmaf(-a.x, b.y, acc.y))};
}

// Chain rule of one voxel and peak through O_m = alpha_m chi exp(i phi), phi = G_m . u,
// for the frame sum g of conj(P) g_psi: adds G_m Im(g conj(O)) to du, alpha_m Re(conj(g)
// e^{i phi}) to dchi and chi Re(conj(g) e^{i phi}) to the alpha partial.  Every
// product and sum is written out, so every gradient kernel rounds it identically.
__device__ __forceinline__ void chain_voxel(const PeakDev& pk, cplx g, float ux, float uy, float uz, float ch,
                                            float al, float& gux, float& guy, float& guz, float& gch, float& ap) {
  const float phi = fmaf(pk.gz, uz, fmaf(pk.gy, uy, pk.gx * ux));   // as k_object
  float s, c;
  phase_sincos(phi, s, c);                                          // as k_object
  const float re = fmaf(g.y, s, g.x * c);                           // Re(conj(g) e^{i phi})
  const float dphi = (al * ch) * fmaf(g.y, c, -(g.x * s));          // Im(g conj(O))
  gux = fmaf(pk.gx, dphi, gux);
  guy = fmaf(pk.gy, dphi, guy);
  guz = fmaf(pk.gz, dphi, guz);
  gch = fmaf(al, re, gch);
  ap = fmaf(ch, re, ap);
}

// The peak record is the same for every lane: read it once and pass each word through
// readfirstlane, so that the raster walk and the slot bases derived from it live in
// scalar registers (a plain load from the table leaves them in vector registers, since
// the compiler cannot prove the table unchanged by the kernel's own stores).
__device__ __forceinline__ PeakDev uniform_peak(const PeakDev* p) {
  static_assert(sizeof(PeakDev) % 4 == 0, "PeakDev is read as 32-bit words");
  constexpr int kWords = sizeof(PeakDev) / 4;
  int w[kWords];
  __builtin_memcpy(w, p, sizeof(PeakDev));
#pragma unroll
  for (int i = 0; i < kWords; ++i) w[i] = __builtin_amdgcn_readfirstlane(w[i]);
  PeakDev pk;
  __builtin_memcpy(&pk, w, sizeof(PeakDev));
  return pk;
}

}  // namespace mpbp
