// mpbp_frame.hpp - the per-frame kernel (one workgroup per frame): eq. (2) forward model,
// eq. (4) modulus residual and the adjoint back to the exit-wave footprint.  Included
// by one translation unit per detector size, which instantiates the kernel for that
// size's footprint bounds and slab depths.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mpbp_dft.hpp"
#include "mpbp_kernels.hpp"

namespace mpbp {

typedef unsigned short u16x2 __attribute__((ext_vector_type(2)));
typedef __attribute__((address_space(3))) const cplx lds_cplx;   // LDS-addressed complex

// ------------------------------------------------------------------- frame kernel ---
template <int D> struct ColLen { static constexpr int L = 64; };
template <> struct ColLen<32> { static constexpr int L = 32; };
template <> struct ColLen<96> { static constexpr int L = 96; };
template <> struct ColLen<150> { static constexpr int L = 50; };

__device__ __forceinline__ int frame_block_index(int b, int n, int xcd) {
  if (!xcd) return b;
  // Blocks are dispatched round-robin over the 8 XCDs: give XCD k the contiguous run
  // of frames [k * per, (k + 1) * per) so overlapping windows share that XCD's L2.
  int per = n >> 3;
  return (b & 7) * per + (b >> 3);
}

// FB bounds the footprint (fy, fx <= FB).  The footprint is placed at the window's
// origin: |Psi| does not depend on where the exit wave sits inside the window (a
// translation only multiplies Psi by a phase ramp), and the residual r Psi/|Psi| carries
// the same ramp, which the inverse transform undoes.  With the footprint at the origin,
// only the first ceil(FB / Q) inputs of each lane are nonzero and only those outputs are
// needed, so the compiler drops the rest of the first and last DFT stages.
// BG: the model intensity carries the background b of eq. (2) (A.bg, ragged like y).
template <int D, int FB, bool BG>
__device__ void frame_body(const FrameArgs& A, const PeakDev& pk, int fid, cplx* sm) {
  using RC = LineCfg<D>;
  constexpr int RP = RC::P, RQ = RC::Q, RT = RC::TPL;
  constexpr int RV = RP > RQ ? RP : RQ;
  constexpr int L = ColLen<D>::L;
  constexpr int R = D / L;
  using CC = LineCfg<L>;
  constexpr int CP = CC::P, CQ = CC::Q, CT = CC::TPL;
  constexpr int CV = CP > CQ ? CP : CQ;
  constexpr int NT = kFrameThreads;
  constexpr int RLINES = NT / RT;
  constexpr int CLINES = NT / CT;
  constexpr int EXL = RQ * (RP + 1);  // exchange buffer per row line (floats: one part at a time)
  constexpr int NAR = (FB + RQ - 1) / RQ < RP ? (FB + RQ - 1) / RQ : RP;  // live row inputs
  // lane t takes part in a pass of Q (or P) lanes; true for every lane when Q == TPL.
  // When P is a multiple of TPL, each lane of the second row pass owns RJ = P / TPL
  // columns c = t + TPL j (every lane busy in both passes).
  static_assert(RQ <= RT && (RP <= RT || RP % RT == 0), "row line configuration");
  constexpr int RJ = RP > RT ? RP / RT : 1;
  auto rowq = [](int t) { return RQ == RT || t < RQ; };
  auto rowp = [](int t) { return RP >= RT || t < RP; };
  auto colq = [](int t) { return CQ == CT || t < CQ; };
  auto colp = [](int t) { return CP == CT || t < CP; };
  constexpr int NAC = (FB + CQ - 1) / CQ < CP ? (FB + CQ - 1) / CQ : CP;  // live column inputs

  const int tid = threadIdx.x;
  const int fy = pk.fy, fx = pk.fx, fxp = pk.fxp;
  // chunk row k starts at k * fxp + k / 8: the skew spreads the column pass's lanes
  // (8 rows apart) over the LDS banks
  auto TRI = [fxp](int k) { return k * fxp + (k >> 3); };
  const int j = fid - pk.frame_base;

  // LDS layout (complex units):
  //   tw2  [D]      row twiddles, tw2[c * RQ + t] = w_D^{t c} (lane-contiguous)
  //   twc  [L]      column twiddles, twc[c * CQ + t] = w_L^{t c}
  //   ftw  [R][fy]  residue-fold twiddles w_D^{rr r}
  //   Tr   [L][fxp] chunk of the column-transformed footprint, row k at k*fxp + k/8
  //   exch          per-line exchange buffers
  // The exit wave and the footprint gradient stay in device memory (the frame's slots;
  // they are L2-resident while the frame runs): without them the kernel fits three
  // workgroups per CU instead of two.
  cplx* tw2 = sm;
  cplx* twc = tw2 + D;
  cplx* ftw = twc + L;
  cplx* Tr = ftw + R * fy;
  cplx* exch = Tr + L * fxp + L / 8;

  {
    const cplx* tsrc = reinterpret_cast<const cplx*>(A.tw) + pk.tw_off;
    for (int k = tid; k < D + L + R * fy; k += NT) tw2[k] = tsrc[k];
  }

  // ---- the exit wave on the footprint, left in the frame's slot by k_project, and the
  // slot of its gradient (each lane of the adjoint column pass owns the same elements
  // in every chunk, so its read-modify-writes need no barrier) ----
  const long long so = pk.slot_off + (long long)j * fy * fx;
  const cplx* psi = reinterpret_cast<const cplx*>(A.slots) + so;
  cplx* gacc = A.grad ? reinterpret_cast<cplx*>(A.gslots) + so : nullptr;
  __syncthreads();

  const bool has_y = A.y != nullptr;
  const float* yf = has_y ? A.y + pk.y_off + (long long)j * D * D : nullptr;
  float* mif = A.mi ? A.mi + pk.y_off + (long long)j * D * D : nullptr;
  const float* bgf = BG ? A.bg + pk.y_off + (long long)j * D * D : nullptr;
  const float invD = 1.0f / (float)D;
  const float invD2 = invD * invD;
  double lsum = 0.0;

  // Intensities are prefetched one row-iteration ahead (across chunk boundaries) so the
  // HBM latency overlaps the transforms of the current rows.
  const int rline = tid / RT, rt = tid % RT;
  // a lane's detector pixels of a row: columns t + RT j + RP d (j < RJ, d < RQ), in
  // slot j RQ + d
  constexpr int RY = RJ * RQ;
  constexpr bool kAhead = RJ == 1;   // intensities prefetched one row iteration ahead
  float ynext[RY], bnext[BG ? RY : 1], yalt[RY], balt[BG ? RY : 1];
  if (kAhead && has_y && rowp(rt)) {
    const float* yr = yf + (long long)(R * rline) * D;
#pragma unroll
    for (int j = 0; j < RJ; ++j)
#pragma unroll
      for (int d = 0; d < RQ; ++d) ynext[j * RQ + d] = __builtin_nontemporal_load(yr + rt + RT * j + RP * d);
  }
  if constexpr (BG) {
    if (kAhead && rowp(rt)) {
      const float* br = bgf + (long long)(R * rline) * D;
#pragma unroll
      for (int j = 0; j < RJ; ++j)
#pragma unroll
        for (int d = 0; d < RQ; ++d) bnext[j * RQ + d] = __builtin_nontemporal_load(br + rt + RT * j + RP * d);
    }
  }

  for (int r = 0; r < R; ++r) {
    // ---- column pass: rows k = R k' + r of the y-direction DFT of the footprint ----
    {
      const int line = tid / CT, t = tid % CT;
      for (int col0 = 0; col0 < fx; col0 += CLINES) {
        const int col = col0 + line;
        const bool on = col < fx;
        cplx v[CV];
        if (on && colq(t)) {
          // the live inputs' loads go out together (clamped addresses, masked by a
          // multiply): as selects, the compiler put each in a branch of its own and
          // waited for it before issuing the next
          cplx pin[NAC];
          if constexpr (FB <= L) {
#pragma unroll
            for (int a = 0; a < NAC; ++a) {
              const int rr = t + CQ * a;
              pin[a] = psi[(rr < fy ? rr : 0) * fx + col];
            }
          }
#pragma unroll
          for (int a = 0; a < CP; ++a) {
            // footprint rows rr = t + CQ a (mod L)
            cplx s = {0.f, 0.f};
            if (a < NAC) {
              if constexpr (FB <= L) {
                const int rr = t + CQ * a;
                const cplx tv = ftw[r * fy + (rr < fy ? rr : 0)];
                s = cscale(cmul(pin[a < NAC ? a : 0], tv), rr < fy ? 1.0f : 0.0f);
              } else {
                for (int rr = t + CQ * a; rr < fy; rr += L)
                  s = cadd(s, cmul(psi[rr * fx + col], ftw[r * fy + rr]));
              }
            }
            v[a] = s;
          }
          DFT<CP, false>::run(v);
#pragma unroll
          for (int c = 0; c < CP; ++c)   // twiddle w^0 = 1 for c = 0
            Tr[TRI(c + CP * t) + col] = c == 0 ? v[0] : cmul(v[c], twc[c * CQ + t]);
        }
        wave_sync();
        if (on && colp(t)) {
#pragma unroll
          for (int b = 0; b < CQ; ++b) v[b] = Tr[TRI(t + CP * b) + col];
          DFT<CQ, false>::run(v);
#pragma unroll
          for (int d = 0; d < CQ; ++d) Tr[TRI(t + CP * d) + col] = v[d];
        }
        wave_sync();
      }
    }
    __syncthreads();

    // ---- row pass: x-direction DFT, modulus residual (eq. (4)), inverse DFT ----
    // The exchange between the two passes moves real parts, then imaginary parts,
    // through a per-line float buffer (all lanes of a line are in one wavefront).
    {
      const int line = tid / RT, t = tid % RT;
      float* ex = reinterpret_cast<float*>(exch) + line * EXL;
      // One row iteration: the intensities (and background) of its rows are in yv (bv);
      // those of the next iteration are prefetched into ynx (bnx).  With several columns
      // per lane (RJ > 1) the prefetch would hold twice the registers: the rows'
      // intensities are then loaded at the start of the iteration instead, ahead of the
      // first pass, and yv, ynx (bv, bnx) are not used.
      auto row_iter = [&](int k0, const float (&yv)[RY], float (&ynx)[RY], const float (&bv)[BG ? RY : 1],
                          float (&bnx)[BG ? RY : 1]) __attribute__((always_inline)) {
        const int kp = k0 + line;
        const int k = R * kp + r;
        // chunk rows beyond L (when L is not a multiple of the lines per pass) have no work
        const bool lok = (L % RLINES == 0) || kp < L;
        float yl[kAhead ? 1 : RY], bl[BG && !kAhead ? RY : 1];
        if constexpr (!kAhead) {
          if (has_y && rowp(t) && lok) {
            const float* yr = yf + (long long)k * D;
#pragma unroll
            for (int j = 0; j < RJ; ++j)
#pragma unroll
              for (int d = 0; d < RQ; ++d) yl[j * RQ + d] = __builtin_nontemporal_load(yr + t + RT * j + RP * d);
          }
          if constexpr (BG) {
            if (rowp(t) && lok) {
              const float* br = bgf + (long long)k * D;
#pragma unroll
              for (int j = 0; j < RJ; ++j)
#pragma unroll
                for (int d = 0; d < RQ; ++d) bl[j * RQ + d] = __builtin_nontemporal_load(br + t + RT * j + RP * d);
            }
          }
        }
        const float* yc = kAhead ? yv : yl;
        const float* bc = kAhead ? bv : bl;
        if constexpr (kAhead) {
          const int nk0 = k0 + RLINES < L ? k0 + RLINES : 0;
          const int nr = k0 + RLINES < L ? r : r + 1;
          const bool nok = (L % RLINES == 0) || nk0 + line < L;
          if (has_y && rowp(t) && nr < R && nok) {
            const float* yr = yf + (long long)(R * (nk0 + line) + nr) * D;
#pragma unroll
            for (int j = 0; j < RJ; ++j)
#pragma unroll
              for (int d = 0; d < RQ; ++d) ynx[j * RQ + d] = __builtin_nontemporal_load(yr + t + RT * j + RP * d);
          }
          if constexpr (BG) {
            if (rowp(t) && nr < R && nok) {
              const float* br = bgf + (long long)(R * (nk0 + line) + nr) * D;
#pragma unroll
              for (int j = 0; j < RJ; ++j)
#pragma unroll
                for (int d = 0; d < RQ; ++d) bnx[j * RQ + d] = __builtin_nontemporal_load(br + t + RT * j + RP * d);
            }
          }
        }
        if (!lok) return;   // (uniform per line; the line's prefetch above is done)
        cplx v[RV];
        if (rowq(t)) {
#pragma unroll
          for (int a = 0; a < RP; ++a) {
            const int cc = t + RQ * a;
            if (a < NAR) {
              const cplx tv = Tr[TRI(kp) + (cc < fx ? cc : 0)];
              v[a] = cc < fx ? tv : cplx{0.f, 0.f};
            } else {
              v[a] = {0.f, 0.f};
            }
          }
          DFT<RP, false>::run(v);
#pragma unroll
          for (int c = 0; c < RP; ++c) {
            if (c > 0) v[c] = cmul(v[c], tw2[c * RQ + t]);   // w^0 = 1
            ex[t * (RP + 1) + c] = v[c].x;
          }
        }
        // second pass: column c = t + RT j of the line's exchange, its Q values in
        // v[j RQ .. j RQ + RQ); X[c + P d] ends in v[j RQ + d]
        wave_sync();
        float re[RY];
        if (rowp(t)) {
#pragma unroll
          for (int j = 0; j < RJ; ++j)
#pragma unroll
            for (int b = 0; b < RQ; ++b) re[j * RQ + b] = ex[b * (RP + 1) + t + RT * j];
        }
        wave_sync();
        if (rowq(t)) {
#pragma unroll
          for (int c = 0; c < RP; ++c) ex[t * (RP + 1) + c] = v[c].y;
        }
        wave_sync();
        if (rowp(t)) {
#pragma unroll
          for (int j = 0; j < RJ; ++j) {
#pragma unroll
            for (int b = 0; b < RQ; ++b) v[j * RQ + b] = {re[j * RQ + b], ex[b * (RP + 1) + t + RT * j]};
            DFT<RQ, false>::run(v + j * RQ);
          }
          if (mif) {
#pragma unroll
            for (int j = 0; j < RJ; ++j)
#pragma unroll
              for (int d = 0; d < RQ; ++d) {
                const int e = j * RQ + d;
                const float i2 = fmaf(v[e].x, v[e].x, v[e].y * v[e].y) * invD2;
                mif[(long long)k * D + t + RT * j + RP * d] = BG ? i2 + bc[BG ? e : 0] : i2;
              }
          }
          if (has_y) {
            float rowl = 0.f;
#pragma unroll
            for (int e = 0; e < RY; ++e) {
              const cplx X = v[e];
              const float s2 = fmaf(X.x, X.x, X.y * X.y);
              if constexpr (BG) {
                // I = |Psi|^2 + b; r = sqrt(I) - sqrt(y); gradient r Psi / sqrt(I), Psi = X / D.
                const float I = fmaf(s2, invD2, bc[BG ? e : 0]);
                const float ri = __builtin_amdgcn_rsqf(I + 1.17549435e-38f);
                const float res = fmaf(I, ri, -__builtin_amdgcn_sqrtf(yc[e]));
                rowl = fmaf(res, res, rowl);
                v[e] = cscale(X, res * ri * invD);
              } else {
                // X = D Psi.  r = |Psi| - sqrt(y); gradient r X / |X|.  The reciprocal
                // square root is taken of |X|^2 + FLT_MIN: finite where X = 0 (there the
                // modulus and the gradient come out exactly 0), absorbed for |X|^2 above
                // about 1e-31.
                const float rinv = __builtin_amdgcn_rsqf(s2 + 1.17549435e-38f);
                const float res = fmaf(s2 * rinv, invD, -__builtin_amdgcn_sqrtf(yc[e]));
                rowl = fmaf(res, res, rowl);
                v[e] = cscale(X, res * rinv);
              }
            }
            lsum += 0.5 * (double)rowl;
          }
        }
        if (A.grad) {
          wave_sync();
          if (rowp(t)) {
#pragma unroll
            for (int j = 0; j < RJ; ++j) {
              DFT<RQ, true>::run(v + j * RQ);
#pragma unroll
              for (int b = 0; b < RQ; ++b) ex[b * (RP + 1) + t + RT * j] = v[j * RQ + b].x;
            }
          }
          wave_sync();
          float rex[RP];
          if (rowq(t)) {
#pragma unroll
            for (int c = 0; c < RP; ++c) rex[c] = ex[t * (RP + 1) + c];
          }
          wave_sync();
          if (rowp(t)) {
#pragma unroll
            for (int j = 0; j < RJ; ++j)
#pragma unroll
              for (int b = 0; b < RQ; ++b) ex[b * (RP + 1) + t + RT * j] = v[j * RQ + b].y;
          }
          wave_sync();
          if (rowq(t)) {
#pragma unroll
            for (int c = 0; c < RP; ++c) {
              const cplx x = {rex[c], ex[t * (RP + 1) + c]};
              v[c] = c == 0 ? x : cmulc(x, tw2[c * RQ + t]);
            }
            DFT<RP, true>::run(v);
#pragma unroll
            for (int a = 0; a < NAR; ++a) {
              const int cc = t + RQ * a;
              if (cc < fx) Tr[TRI(kp) + cc] = v[a];
            }
          }
        }
        wave_sync();
            };
      // With an even number of iterations per chunk the two buffers trade places and no
      // copies are needed; otherwise the prefetched values are copied once per iteration.
      constexpr int NIT = (L + RLINES - 1) / RLINES;
      if constexpr (NIT % 2 == 0) {
        for (int k0 = 0; k0 < L; k0 += 2 * RLINES) {
          row_iter(k0, ynext, yalt, bnext, balt);
          row_iter(k0 + RLINES, yalt, ynext, balt, bnext);
        }
      } else {
        for (int k0 = 0; k0 < L; k0 += RLINES) {
          float yv[RY], bv[BG ? RY : 1];
#pragma unroll
          for (int d = 0; d < RY; ++d) yv[d] = ynext[d];
          if constexpr (BG) {
#pragma unroll
            for (int d = 0; d < RY; ++d) bv[d] = bnext[d];
          }
          row_iter(k0, yv, ynext, bv, bnext);
        }
      }
    }
    __syncthreads();

    // ---- adjoint column pass: accumulate this chunk's share of the footprint gradient ----
    if (A.grad) {
      const int line = tid / CT, t = tid % CT;
      for (int col0 = 0; col0 < fx; col0 += CLINES) {
        const int col = col0 + line;
        const bool on = col < fx;
        cplx v[CV];
        if (on && colp(t)) {
#pragma unroll
          for (int d = 0; d < CQ; ++d) v[d] = Tr[TRI(t + CP * d) + col];
          DFT<CQ, true>::run(v);
#pragma unroll
          for (int b = 0; b < CQ; ++b) Tr[TRI(t + CP * b) + col] = v[b];
        }
        wave_sync();
        if (on && colq(t)) {
#pragma unroll
          for (int c = 0; c < CP; ++c) {
            const cplx x = Tr[TRI(c + CP * t) + col];
            v[c] = c == 0 ? x : cmulc(x, twc[c * CQ + t]);
          }
          DFT<CP, true>::run(v);
          if constexpr (FB <= L) {
            cplx gv[NAC], tv[NAC];
            // chunk 0 starts the sums; the last chunk applies the 1/D of the orthonormal
            // transforms
            const float sc = r == R - 1 ? invD : 1.0f;
#pragma unroll
            for (int a = 0; a < NAC; ++a) {
              const int rr = t + CQ * a;
              const int rc = rr < fy ? rr : 0;
              gv[a] = r > 0 ? gacc[rc * fx + col] : cplx{0.f, 0.f};
              tv[a] = ftw[r * fy + rc];
            }
#pragma unroll
            for (int a = 0; a < NAC; ++a) {
              const int rr = t + CQ * a;
              if (rr < fy) gacc[rr * fx + col] = cscale(cadd(gv[a], cmulc(v[a], tv[a])), sc);
            }
          } else {
#pragma unroll
            for (int a = 0; a < NAC; ++a) {
              for (int rr = t + CQ * a; rr < fy; rr += L) {
                cplx* g = gacc + rr * fx + col;
                const cplx prev = r > 0 ? *g : cplx{0.f, 0.f};
                *g = cscale(cadd(prev, cmulc(v[a], ftw[r * fy + rr])), r == R - 1 ? invD : 1.0f);
              }
            }
          }
        }
        wave_sync();
      }
      __syncthreads();
    }
  }


  if (has_y) {
    // workgroup sum of the per-lane losses (fixed order)
    for (int off = 32; off > 0; off >>= 1) lsum += __shfl_xor(lsum, off);
    __syncthreads();
    double* red = reinterpret_cast<double*>(exch);
    if ((tid & 63) == 0) red[tid >> 6] = lsum;
    __syncthreads();
    if (tid == 0) {
      double s = 0.0;
      for (int w = 0; w < NT / 64; ++w) s += red[w];
      A.floss[fid] = s;
    }
  }
}

// One instance per detector size D and footprint bound FB; the frames of a size class
// form one launch.
template <int D, int FB, bool BG>
__global__ __launch_bounds__(kFrameThreads) void k_frames(FrameArgs A) {
  extern __shared__ cplx smem[];
  const int idx = frame_block_index(blockIdx.x, gridDim.x, A.xcd);
  if (idx >= A.n_list) return;
  const int fid = A.list[idx];
  const PeakDev pk = A.peaks[A.peak_of[fid]];
  frame_body<D, FB, BG>(A, pk, fid, smem);
}

// Launch / prepare one instance (with and without background).  op 0: launch over
// a.n_list frames (the background variant when a.bg is set); op 1: allow both variants
// the full LDS of a CU on the current device; op 2: report that the instance exists.
template <int D, int FB>
hipError_t frame_instance_op(int op, const FrameArgs* a, int lds_bytes, hipStream_t s) {
  if (op == 1) {
    hipError_t e = hipFuncSetAttribute((const void*)k_frames<D, FB, false>,
                                       hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
    if (e == hipSuccess)
      e = hipFuncSetAttribute((const void*)k_frames<D, FB, true>, hipFuncAttributeMaxDynamicSharedMemorySize,
                              160 * 1024);
    return e;
  }
  if (op == 2) return hipSuccess;
  const unsigned grid = a->xcd ? (unsigned)(((a->n_list + 7) / 8) * 8) : (unsigned)a->n_list;
  if (grid == 0) return hipSuccess;
  if (a->bg)
    k_frames<D, FB, true><<<dim3(grid), dim3(kFrameThreads), lds_bytes, s>>>(*a);
  else
    k_frames<D, FB, false><<<dim3(grid), dim3(kFrameThreads), lds_bytes, s>>>(*a);
  return hipGetLastError();
}

// Dispatch over the compiled footprint bounds FBs...
template <int D, int... FBs>
hipError_t frame_dispatch(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s) {
  hipError_t e = hipErrorInvalidValue;
  bool done = false;
  auto one = [&](auto fb_) {
    constexpr int F = decltype(fb_)::value;
    if (!done && fb == F) {
      e = frame_instance_op<D, F>(op, a, lds_bytes, s);
      done = true;
    }
  };
  (one(std::integral_constant<int, FBs>{}), ...);
  return e;
}

}  // namespace mpbp
