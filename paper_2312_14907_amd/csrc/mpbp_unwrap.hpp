// mpbp_unwrap.hpp - arguments and launcher of the phase-unwrap projector kernels.
#pragma once
#include <hip/hip_runtime.h>

namespace mpbp {

constexpr int kUnwrapMaxPeaks = 16;

// Device workspace and geometry of one projector call.  Per-map arrays hold
// nmaps = M * S maps of np = ny * nx pixels, map g = m * S + s.
struct UnwrapArgs {
  int M, S, ny, nx;
  long long np;                // pixels per map
  long long nmaps;
  long long npix;              // nmaps * np
  int rounds;                  // Boruvka rounds launched (unwrap_rounds(np))
  float g[kUnwrapMaxPeaks][3];     // Bragg vectors G_m (rad/nm), float32
  float coef[kUnwrapMaxPeaks][3];  // 2 pi H^+[m][c]: displacement of one 2 pi wrap of map m
  float* psi;                  // wrapped phase
  int* q;                      // rint(Phi / 2 pi) of the wrap
  float* rel;                  // pixel reliability
  int* par;                    // current root (local index)
  int* pot;                    // wrap count relative to the root
  int* hk;                     // root hooked onto this round (itself if none)
  int* hpot;                   // wrap count of a hooked root relative to its new parent
  unsigned long long* best;    // best outgoing edge key of a root this round (0: none)
  int* hooks;                  // [rounds][64] flags: a root hooked in this round
  long long* sums;             // [nmaps] sum of (q - pot)
  int* err;                    // 0, or a failed consistency check
};

// Boruvka rounds needed for maps of np pixels.
int unwrap_rounds(long long np);
// Pi_U in place on u ([3][S][ny][nx] float32); wraps (may be null) receives the integer
// N of every map pixel.  The caller checks *A.err after the stream completes.
hipError_t launch_unwrap(float* u, int* wraps, const UnwrapArgs& A, hipStream_t s);

}  // namespace mpbp
