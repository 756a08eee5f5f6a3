// mpbp_phase.hpp - sin and cos of the phase G_m . u of eq. (1)/(3) in FP32, shared by
// every kernel that forms the objects O_m = alpha_m chi e^{i G_m . u} or differentiates
// them, so that all of them round the phase alike.
//
// Method: the additive argument reduction of Cody and Waite (Software Manual for the
// Elementary Functions, 1980): j = rint(2 phi / pi), and r = phi - j pi/2 with pi/2 split
// into three floats (the float nearest pi/2, then the floats nearest the two remainders)
// subtracted by fused multiply-adds; then the Taylor series of sin (to r^9) and cos (to
// r^10) on |r| <= pi/4, whose truncation stays below 2e-9, and the quadrant j mod 4.
// The absolute error is about one unit in the last place of 1 for |phi| up to 2e4 rad (a
// float phase itself carries |phi| 6e-8 of rounding); beyond that the reduction loses
// accuracy gradually.  No branch: every lane runs the same instructions.
#pragma once
#include <hip/hip_runtime.h>

namespace mpbp {

__device__ __forceinline__ void phase_sincos(float phi, float& s, float& c) {
  constexpr float kTwoOverPi = 0.6366197466850281f;
  constexpr float kHalfPi1 = 1.5707963705062866f;       // float nearest pi/2
  constexpr float kHalfPi2 = -4.371138828673793e-08f;   // float nearest pi/2 - kHalfPi1
  constexpr float kHalfPi3 = -1.7151245100058819e-15f;  // float nearest the rest
  const float j = __builtin_rintf(phi * kTwoOverPi);
  float r = fmaf(-j, kHalfPi1, phi);
  r = fmaf(-j, kHalfPi2, r);
  r = fmaf(-j, kHalfPi3, r);
  const float r2 = r * r;
  // sin r = r + r^3 (-1/3! + r^2 (1/5! + r^2 (-1/7! + r^2 / 9!)))
  float ps = fmaf(r2, 1.f / 362880.f, -1.f / 5040.f);
  ps = fmaf(r2, ps, 1.f / 120.f);
  ps = fmaf(r2, ps, -1.f / 6.f);
  const float sn = fmaf(r * r2, ps, r);
  // cos r = 1 + r^2 (-1/2! + r^2 (1/4! + r^2 (-1/6! + r^2 (1/8! - r^2 / 10!))))
  float pc = fmaf(r2, -1.f / 3628800.f, 1.f / 40320.f);
  pc = fmaf(r2, pc, -1.f / 720.f);
  pc = fmaf(r2, pc, 1.f / 24.f);
  pc = fmaf(r2, pc, -0.5f);
  const float cs = fmaf(r2, pc, 1.f);
  // quadrant: phi = r + q pi/2, q = j mod 4 (two's complement keeps it in 0..3)
  const int q = (int)j & 3;
  const float a = (q & 1) ? cs : sn, b = (q & 1) ? sn : cs;
  s = (q & 2) ? -a : a;
  c = ((q + 1) & 2) ? -b : b;
}

}  // namespace mpbp
