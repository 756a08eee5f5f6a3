// mpbp_plain.hpp - the plain GPU path: one launch per stage per (peak, scan position),
// full D x D exit waves in device memory, no fusion.  It computes the same quantities
// as the batched fused path and serves as its speed and correctness baseline.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpbp_kernels.hpp"

namespace mpbp {

struct PlainWork {
  int device = -1;
  float* psi = nullptr;     // complex64 [Dmax][Dmax]
  float* gobj = nullptr;    // complex64 [M][nvox]
  double* lpart = nullptr;  // [Dmax] per-row loss partials
  double* apart = nullptr;  // [blocks][M] alpha-gradient partials
  long long gobj_len = 0;
  long long apart_len = 0;
  int dmax = 0;
  const float* bg = nullptr;   // background b of eq. (2), ragged like y (set by the plan)
  int probe3 = 0;              // 1: probe [M][nz][np][np] (set by the plan)
  const float* shw = nullptr;  // [M][nz][2] fractional exit-beam offsets or null (set by the plan)
};

void plain_free(PlainWork* w);

hipError_t plain_forward(PlainWork* w, const PeakDev* hpeaks, const PeakDev* dpeaks, int M, int nz,
                         int ny, int nx, int np, const int* dshear, const int32_t* hscan,
                         const int32_t* hpeak_of, const int32_t* frames, int n, const float* u,
                         const float* chi, const float* alpha, const float* probe, const float* y,
                         float* mi, float* obj, double* floss, long long tied, hipStream_t s);

hipError_t plain_loss_grad(PlainWork* w, const PeakDev* hpeaks, const PeakDev* dpeaks, int M, int nz,
                           int ny, int nx, int np, const int* dshear, const int32_t* hscan,
                           const int32_t* hpeak_of, const int32_t* frames, int n, const float* u,
                           const float* chi, const float* alpha, const float* probe, const float* y,
                           float* obj, double* floss, float* grad_u, float* grad_chi,
                           const double** apart, int* n_part, long long tied, hipStream_t s);

}  // namespace mpbp
