// mpbp_device.hip - HIP kernels (gfx950) of the MPBP objective-and-gradient path.
//
//   k_object   eq. (1)/(3): O_m = alpha_m chi exp(i G_m . u) for every voxel and peak
//   k_frames   one workgroup per frame (m, j): eq. (2) forward model, eq. (4) residual,
//              and the adjoint back to the exit-wave footprint
//   k_grad     gather back-projection of the footprint gradients over all frames that
//              cover a voxel tile, then the chain rule to df/du, df/dchi, df/dalpha
//   k_finalize deterministic FP64 sums of the per-frame losses and alpha partials
//   k_step     p <- p - eta g
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <cmath>
#include <vector>

#include "mpbp_dft.hpp"
#include "mpbp_kernels.hpp"
#include "mpbp_launch.hpp"

namespace mpbp {

// ------------------------------------------------------------------ object build ---
__global__ __launch_bounds__(256) void k_object(const float* __restrict__ u,
                                                const float* __restrict__ chi,
                                                const float* __restrict__ alpha,
                                                const PeakDev* __restrict__ peaks, int n_peaks,
                                                long long nvox, float* __restrict__ obj) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  float ux = u[v], uy = u[nvox + v], uz = u[2 * nvox + v];
  float ch = chi[v];
  for (int m = 0; m < n_peaks; ++m) {
    float phi = peaks[m].gx * ux + peaks[m].gy * uy + peaks[m].gz * uz;
    float s, c;
    sincosf(phi, &s, &c);
    float a = alpha[m] * ch;
    float2* o = reinterpret_cast<float2*>(obj) + (long long)m * nvox + v;
    *o = make_float2(a * c, a * s);
  }
}

// ------------------------------------------------------------------- frame kernel ---
template <int D> struct ColLen { static constexpr int L = 64; };
template <> struct ColLen<32> { static constexpr int L = 32; };
template <> struct ColLen<96> { static constexpr int L = 96; };

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
template <int D, int FB>
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
  // lane t takes part in a pass of Q (or P) lanes; true for every lane when Q == TPL
  auto rowq = [](int t) { return RQ == RT || t < RQ; };
  auto rowp = [](int t) { return RP == RT || t < RP; };
  auto colq = [](int t) { return CQ == CT || t < CQ; };
  auto colp = [](int t) { return CP == CT || t < CP; };
  constexpr int NAC = (FB + CQ - 1) / CQ < CP ? (FB + CQ - 1) / CQ : CP;  // live column inputs

  const int tid = threadIdx.x;
  const int np = A.np, nz = A.nz;
  const int fy = pk.fy, fx = pk.fx, fxp = pk.fxp;
  // chunk row k starts at k * fxp + k / 8: the skew spreads the column pass's lanes
  // (8 rows apart) over the LDS banks
  auto TRI = [fxp](int k) { return k * fxp + (k >> 3); };
  const int m = A.peak_of[fid];
  const int py = A.scan[2 * fid], px = A.scan[2 * fid + 1];
  const int j = fid - pk.frame_base;

  // LDS layout (complex units):
  //   tw2  [D]      row twiddles, tw2[c * RQ + t] = w_D^{t c} (lane-contiguous)
  //   twc  [L]      column twiddles, twc[c * CQ + t] = w_L^{t c}
  //   ftw  [R][fy]  residue-fold twiddles w_D^{rr r}
  //   psi  [fy][fx] exit wave on the footprint
  //   gacc [fy][fx] footprint gradient
  //   Tr   [L][fxp] chunk of the column-transformed footprint, row k at k*fxp + k/8
  //   exch          per-line exchange buffers (with Tr: staged slices during the projection)
  //   sh   [nz]     shear offsets
  cplx* tw2 = sm;
  cplx* twc = tw2 + D;
  cplx* ftw = twc + L;
  cplx* psi = ftw + R * fy;
  cplx* gacc = psi + fy * fx;
  cplx* Tr = gacc + (A.grad ? fy * fx : 0);
  cplx* exch = Tr + L * fxp + L / 8;
  // the exchange area also holds (with the chunk buffer before it) kProjG staged slices
  const int exch_min = kProjG * (np + 1) * (np + 1) - (L * fxp + L / 8);
  const int exch_sz = (RLINES * EXL + 1) / 2 > exch_min ? (RLINES * EXL + 1) / 2 : exch_min;
  int2* sh = reinterpret_cast<int2*>(exch + exch_sz);

  {
    const cplx* tsrc = reinterpret_cast<const cplx*>(A.tw) + pk.tw_off;
    for (int k = tid; k < D + L + R * fy; k += NT) tw2[k] = tsrc[k];
  }
  const cplx* probe = reinterpret_cast<const cplx*>(A.probe) + (long long)m * np * np;
  for (int z = tid; z < nz; z += NT) {
    const int* s = A.shear + 2 * (m * nz + z);
    sh[z] = make_int2(s[0], s[1]);
  }
  if (A.grad)
    for (int k = tid; k < fy * fx; k += NT) gacc[k] = {0.f, 0.f};
  __syncthreads();

  // ---- eq. (2): R diag(P) S O -> exit wave on the footprint (gather over slices) ----
  cplx* slot = reinterpret_cast<cplx*>(A.slots) + pk.slot_off + (long long)j * fy * fx;
  const cplx* O = reinterpret_cast<const cplx*>(A.obj) + (long long)m * nz * A.ny * A.nx;
  // The illuminated slices W_z = P * O[z, window] are staged kProjG at a time in the
  // chunk / exchange area (idle during the projection), the next group's object values
  // already in flight in registers; each lane then gathers its footprint pixels
  //   psi[q] += W_z[q + min shear - s(z)]   (zero outside the probe support).
  // A staged slice is (np + 1) x (np + 1) with a zero last row and column: offsets
  // outside the support are clamped onto them, so the gather has no tests or branches.
  {
    const int np1 = np + 1;
    const int sw = np1 * np1;
    const int np2 = np * np;
    cplx* Wb = Tr;
    const int* shz = A.shear + 2 * m * nz;   // uniform: scalar loads
    for (int k = tid; k < kProjG * (2 * np + 1); k += NT) {
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
    cplx on[kProjG][kProjE];
#pragma unroll
    for (int g = 0; g < kProjG; ++g) {
      const cplx* Oz = O + (long long)(g < nz ? g : 0) * plane;
#pragma unroll
      for (int i = 0; i < kProjE; ++i) on[g][i] = Oz[off[i]];
    }
    int pby[kProjPix], pbx[kProjPix];
    cplx acc[kProjPix];
#pragma unroll
    for (int h = 0; h < kProjPix; ++h) {
      const int p = tid + NT * h;
      const int qy = p / fx;
      pby[h] = qy + pk.miny;
      pbx[h] = p - qy * fx + pk.minx;
      acc[h] = {0.f, 0.f};
    }
    for (int z0 = 0; z0 < nz; z0 += kProjG) {
      __syncthreads();
#pragma unroll
      for (int g = 0; g < kProjG; ++g)
#pragma unroll
        for (int i = 0; i < kProjE; ++i)
          if (wo[i] >= 0) Wb[g * sw + wo[i]] = (z0 + g < nz) ? cmul(pv[i], on[g][i]) : cplx{0.f, 0.f};
#pragma unroll
      for (int g = 0; g < kProjG; ++g) {
        const int z = z0 + kProjG + g;
        const cplx* Oz = O + (long long)(z < nz ? z : 0) * plane;
#pragma unroll
        for (int i = 0; i < kProjE; ++i) on[g][i] = Oz[off[i]];
      }
      int ssy[kProjG], ssx[kProjG];
#pragma unroll
      for (int g = 0; g < kProjG; ++g) {
        const int z = z0 + g < nz ? z0 + g : 0;
        ssy[g] = shz[2 * z];
        ssx[g] = shz[2 * z + 1];
      }
      __syncthreads();
#pragma unroll
      for (int h = 0; h < kProjPix; ++h) {
        cplx w[kProjG];
#pragma unroll
        for (int g = 0; g < kProjG; ++g) {
          const unsigned a = min((unsigned)(pby[h] - ssy[g]), (unsigned)np);
          const unsigned b = min((unsigned)(pbx[h] - ssx[g]), (unsigned)np);
          w[g] = Wb[g * sw + (int)(a * np1 + b)];
        }
#pragma unroll
        for (int g = 0; g < kProjG; ++g) acc[h] = cadd(acc[h], w[g]);
      }
    }
#pragma unroll
    for (int h = 0; h < kProjPix; ++h)
      if (tid + NT * h < fy * fx) psi[tid + NT * h] = acc[h];
  }
  __syncthreads();

  const bool has_y = A.y != nullptr;
  const float* yf = has_y ? A.y + pk.y_off + (long long)j * D * D : nullptr;
  float* mif = A.mi ? A.mi + pk.y_off + (long long)j * D * D : nullptr;
  const float invD = 1.0f / (float)D;
  const float invD2 = invD * invD;
  double lsum = 0.0;

  // Intensities are prefetched one row-iteration ahead (across chunk boundaries) so the
  // HBM latency overlaps the transforms of the current rows.
  const int rline = tid / RT, rt = tid % RT;
  float ynext[RQ];
  if (has_y && rowp(rt)) {
    const float* yr = yf + (long long)(R * rline) * D;
#pragma unroll
    for (int d = 0; d < RQ; ++d) ynext[d] = __builtin_nontemporal_load(yr + rt + RP * d);
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
#pragma unroll
          for (int a = 0; a < CP; ++a) {
            // footprint rows rr = t + CQ a (mod L)
            cplx s = {0.f, 0.f};
            if (a < NAC) {
              if constexpr (FB <= L) {
                const int rr = t + CQ * a;
                const bool ok = rr < fy;
                const cplx pv = psi[(ok ? rr : 0) * fx + col];
                const cplx tv = ftw[r * fy + (ok ? rr : 0)];
                s = ok ? cmul(pv, tv) : cplx{0.f, 0.f};
              } else {
                for (int rr = t + CQ * a; rr < fy; rr += L)
                  s = cadd(s, cmul(psi[rr * fx + col], ftw[r * fy + rr]));
              }
            }
            v[a] = s;
          }
          DFT<CP, false>::run(v);
#pragma unroll
          for (int c = 0; c < CP; ++c) Tr[TRI(c + CP * t) + col] = cmul(v[c], twc[c * CQ + t]);
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
      for (int k0 = 0; k0 < L; k0 += RLINES) {
        const int kp = k0 + line;
        const int k = R * kp + r;
        float yv[RQ];
#pragma unroll
        for (int d = 0; d < RQ; ++d) yv[d] = ynext[d];
        {
          const int nk0 = k0 + RLINES < L ? k0 + RLINES : 0;
          const int nr = k0 + RLINES < L ? r : r + 1;
          if (has_y && rowp(t) && nr < R) {
            const float* yr = yf + (long long)(R * (nk0 + line) + nr) * D;
#pragma unroll
            for (int d = 0; d < RQ; ++d) ynext[d] = __builtin_nontemporal_load(yr + t + RP * d);
          }
        }
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
            v[c] = cmul(v[c], tw2[c * RQ + t]);
            ex[t * (RP + 1) + c] = v[c].x;
          }
        }
        wave_sync();
        float re[RQ];
        if (rowp(t)) {
#pragma unroll
          for (int b = 0; b < RQ; ++b) re[b] = ex[b * (RP + 1) + t];
        }
        wave_sync();
        if (rowq(t)) {
#pragma unroll
          for (int c = 0; c < RP; ++c) ex[t * (RP + 1) + c] = v[c].y;
        }
        wave_sync();
        if (rowp(t)) {
#pragma unroll
          for (int b = 0; b < RQ; ++b) v[b] = {re[b], ex[b * (RP + 1) + t]};
          DFT<RQ, false>::run(v);
          float rowl = 0.f;
#pragma unroll
          for (int d = 0; d < RQ; ++d) {
            // X = D Psi.  r = |Psi| - sqrt(y); gradient r X / |X| (0 where |X|^2 is
            // below the smallest normal float, i.e. Psi = 0 in this precision).
            const cplx X = v[d];
            const float s2 = X.x * X.x + X.y * X.y;
            if (mif) mif[(long long)k * D + t + RP * d] = s2 * invD2;
            if (has_y) {
              const bool nzr = s2 >= 1.17549435e-38f;
              const float rinv = __builtin_amdgcn_rsqf(nzr ? s2 : 1.0f);
              const float A = nzr ? s2 * rinv * invD : 0.f;
              const float res = A - __builtin_amdgcn_sqrtf(yv[d]);
              rowl = fmaf(0.5f * res, res, rowl);
              v[d] = cscale(X, nzr ? res * rinv : 0.f);
            }
          }
          lsum += (double)rowl;
        }
        if (A.grad) {
          wave_sync();
          if (rowp(t)) {
            DFT<RQ, true>::run(v);
#pragma unroll
            for (int b = 0; b < RQ; ++b) ex[b * (RP + 1) + t] = v[b].x;
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
            for (int b = 0; b < RQ; ++b) ex[b * (RP + 1) + t] = v[b].y;
          }
          wave_sync();
          if (rowq(t)) {
#pragma unroll
            for (int c = 0; c < RP; ++c) v[c] = cmulc(cplx{rex[c], ex[t * (RP + 1) + c]}, tw2[c * RQ + t]);
            DFT<RP, true>::run(v);
#pragma unroll
            for (int a = 0; a < NAR; ++a) {
              const int cc = t + RQ * a;
              if (cc < fx) Tr[TRI(kp) + cc] = v[a];
            }
          }
        }
        wave_sync();
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
          for (int c = 0; c < CP; ++c) v[c] = cmulc(Tr[TRI(c + CP * t) + col], twc[c * CQ + t]);
          DFT<CP, true>::run(v);
          if constexpr (FB <= L) {
            cplx gv[NAC], tv[NAC];
#pragma unroll
            for (int a = 0; a < NAC; ++a) {
              const int rr = t + CQ * a;
              const int rc = rr < fy ? rr : 0;
              gv[a] = gacc[rc * fx + col];
              tv[a] = ftw[r * fy + rc];
            }
#pragma unroll
            for (int a = 0; a < NAC; ++a) {
              const int rr = t + CQ * a;
              if (rr < fy) gacc[rr * fx + col] = cadd(gv[a], cmulc(v[a], tv[a]));
            }
          } else {
#pragma unroll
            for (int a = 0; a < NAC; ++a) {
              for (int rr = t + CQ * a; rr < fy; rr += L) {
                cplx* g = gacc + rr * fx + col;
                *g = cadd(*g, cmulc(v[a], ftw[r * fy + rr]));
              }
            }
          }
        }
        wave_sync();
      }
      __syncthreads();
    }
  }

  if (A.grad) {
    for (int p = tid; p < fy * fx; p += NT) slot[p] = cscale(gacc[p], invD);
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

// One instance per detector size: the frames of a size class form one launch.
template <int D, int FB>
__global__ __launch_bounds__(kFrameThreads) void k_frames(FrameArgs A) {
  extern __shared__ cplx smem[];
  const int idx = frame_block_index(blockIdx.x, gridDim.x, A.xcd);
  if (idx >= A.n_list) return;
  const int fid = A.list[idx];
  const PeakDev pk = A.peaks[A.peak_of[fid]];
  frame_body<D, FB>(A, pk, fid, smem);
}

// -------------------------------------------- gather back-projection + chain rule ---
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

__global__ __launch_bounds__(kGradThreads, 4) void k_grad(GradArgs A) {
  extern __shared__ cplx smem[];
  const int np = A.np, nz = A.nz;
  const int RW = kGradTX + A.maxspan_x;
  const int RS = (kGradTY + A.maxspan_y) * RW;       // one staged region (complex)
  cplx* Ps = smem;                                   // np * np
  int2* sh = reinterpret_cast<int2*>(Ps + np * np);  // nz
  double* apl = reinterpret_cast<double*>(sh + nz);  // alpha partials
  float* red = reinterpret_cast<float*>(apl + kMaxPeaksDev);       // block reduction
  unsigned char* actf = reinterpret_cast<unsigned char*>(red + 16);  // candidate frames' flags

  const int tid = threadIdx.x;
  const int tx = tid % kGradTX, ty = (tid / kGradTX) % kGradTY, tz = tid / (kGradTX * kGradTY);
  // Tiles are handed out so that each XCD (blocks are dispatched round-robin over the
  // 8 XCDs) walks a contiguous band of tile rows: neighbouring tiles read the same
  // frames' footprints, which then stay in that XCD's L2.
  const int tile = frame_block_index(blockIdx.x, gridDim.x, 1);
  if (tile >= A.tiles_x * A.tiles_y) return;
  const int bx = tile % A.tiles_x, by = tile / A.tiles_x;
  const int x0 = bx * kGradTX, y0 = by * kGradTY;
  const int x = x0 + tx, y = y0 + ty;
  const bool inb = x < A.nx && y < A.ny;
  const long long nvox = (long long)nz * A.ny * A.nx;
  // this thread's element positions in a staged region (row-major with stride RW)
  const int e0r = tid / RW, e0c = tid - e0r * RW;
  const int e1 = tid + kGradThreads;
  const int e1r = e1 / RW, e1c = e1 - e1r * RW;
  if (tid < kMaxPeaksDev) apl[tid] = 0.0;

  for (int zb = 0; zb < nz; zb += kGradZB) {
    float gux[kGradZPer], guy[kGradZPer], guz[kGradZPer], gch[kGradZPer];
#pragma unroll
    for (int i = 0; i < kGradZPer; ++i) gux[i] = guy[i] = guz[i] = gch[i] = 0.f;

    for (int m = 0; m < A.n_peaks; ++m) {
      const PeakDev pk = A.peaks[m];
      // Frames of this peak whose windows meet the tile: a rectangle of the raster.
      const int iy_lo = max(0, -floordiv(-(y0 - np + 1 - pk.oy), pk.sy));
      const int iy_hi = min(pk.rows - 1, floordiv(y0 + kGradTY - 1 - pk.oy, pk.sy));
      const int ix_lo = max(0, -floordiv(-(x0 - np + 1 - pk.ox), pk.sx));
      const int ix_hi = min(pk.cols - 1, floordiv(x0 + kGradTX - 1 - pk.ox, pk.sx));
      const int ncx = ix_hi - ix_lo + 1;
      const int ncand = (iy_hi >= iy_lo && ncx > 0) ? (iy_hi - iy_lo + 1) * ncx : 0;
      __syncthreads();
      const cplx* probe = reinterpret_cast<const cplx*>(A.probe) + (long long)m * np * np;
      for (int k = tid; k < np * np; k += kGradThreads) Ps[k] = probe[k];
      for (int z = tid; z < nz; z += kGradThreads) {
        const int* s = A.shear + 2 * (m * nz + z);
        sh[z] = make_int2(s[0], s[1]);
      }
      // minibatch flags of the candidate frames, loaded in parallel
      for (int c = tid; c < ncand; c += kGradThreads) {
        const int cy = iy_lo + c / ncx, cx = ix_lo + c % ncx;
        actf[c] = A.active[pk.frame_base + cy * pk.cols + cx];
      }
      cplx acc[kGradZPer];
#pragma unroll
      for (int i = 0; i < kGradZPer; ++i) acc[i] = {0.f, 0.f};
      __syncthreads();

      // this lane's slices: shear offsets in registers
      int zsy[kGradZPer], zsx[kGradZPer];
#pragma unroll
      for (int i = 0; i < kGradZPer; ++i) {
        const int z = zb + tz + kGradTZ * i;
        zsy[i] = sh[z < nz ? z : 0].x - pk.miny;
        zsx[i] = sh[z < nz ? z : 0].y - pk.minx;
      }
      // Frames of the minibatch, kGradBatch at a time (uniform walk, scalar results).
      // Each lane reads its footprint-gradient values straight from the frame's slot:
      // a wavefront covers a 4 x 16 voxel patch at one slice, so its reads are rows.
      const cplx* slots = reinterpret_cast<const cplx*>(A.slots);
      int iy = iy_lo, ix = ix_lo, ci = 0;
      while (iy <= iy_hi) {
        int nb = 0;
        int fpy[kGradBatch], fpx[kGradBatch];
        long long fso[kGradBatch];
#pragma unroll
        for (int k = 0; k < kGradBatch; ++k) {
          fpy[k] = fpx[k] = 0;
          fso[k] = 0;
          while (nb == k && iy <= iy_hi) {
            const int cy = iy, cx = ix;
            if (++ix > ix_hi) { ix = ix_lo; ++iy; }
            const int act = __builtin_amdgcn_readfirstlane((int)actf[ci]);
            ++ci;
            if (!act) continue;
            fpy[k] = pk.oy + cy * pk.sy;
            fpx[k] = pk.ox + cx * pk.sx;
            fso[k] = pk.slot_off + (long long)(cy * pk.cols + cx) * pk.fy * pk.fx;
            nb = k + 1;
          }
        }
        if (nb == 0) break;
        cplx gv[kGradBatch][kGradZPer], pv[kGradBatch];
#pragma unroll
        for (int k = 0; k < kGradBatch; ++k) {
          const int a = y - fpy[k], b = x - fpx[k];
          const bool inw = k < nb && inb && (unsigned)a < (unsigned)np && (unsigned)b < (unsigned)np;
          const int ac = inw ? a : 0, bc = inw ? b : 0;
          const cplx pr = Ps[ac * np + bc];
          pv[k] = inw ? pr : cplx{0.f, 0.f};
          const cplx* sl = slots + fso[k];
#pragma unroll
          for (int i = 0; i < kGradZPer; ++i) gv[k][i] = sl[(ac + zsy[i]) * pk.fx + bc + zsx[i]];
        }
#pragma unroll
        for (int k = 0; k < kGradBatch; ++k)
#pragma unroll
          for (int i = 0; i < kGradZPer; ++i) acc[i] = cadd(acc[i], cmulc(gv[k][i], pv[k]));   // conj(P) g_psi
      }
      // chain rule through O_m = alpha_m chi exp(i G_m . u); 32-bit voxel offsets from
      // uniform bases (the plan limits 3 * nvox to 2^32)
      float ap = 0.f;
      if (inb) {
        const float al = A.alpha[m];
        const unsigned nv = (unsigned)nvox;
#pragma unroll
        for (int i = 0; i < kGradZPer; ++i) {
          const int z = zb + tz + kGradTZ * i;
          if (z < nz) {
            const unsigned v = ((unsigned)z * (unsigned)A.ny + (unsigned)y) * (unsigned)A.nx + (unsigned)x;
            const float ux = A.u[v], uy = A.u[nv + v], uzv = A.u[2u * nv + v];
            const float ch = A.chi[v];
            const float phi = pk.gx * ux + pk.gy * uy + pk.gz * uzv;
            float s, c;
            __sincosf(phi, &s, &c);
            const cplx g = acc[i];
            const float re = g.x * c + g.y * s;                 // Re(conj(g) e^{i phi})
            const float dphi = al * ch * (g.y * c - g.x * s);   // Im(g conj(O))
            gux[i] += pk.gx * dphi;
            guy[i] += pk.gy * dphi;
            guz[i] += pk.gz * dphi;
            gch[i] += al * re;
            ap += ch * re;
          }
        }
      }
      const float apb = block_sum_f(ap, red);
      if (tid == 0) apl[m] += (double)apb;
    }
    if (inb) {
      const unsigned nv = (unsigned)nvox;
#pragma unroll
      for (int i = 0; i < kGradZPer; ++i) {
        const int z = zb + tz + kGradTZ * i;
        if (z < nz) {
          const unsigned v = ((unsigned)z * (unsigned)A.ny + (unsigned)y) * (unsigned)A.nx + (unsigned)x;
          A.grad_u[v] = gux[i];
          A.grad_u[nv + v] = guy[i];
          A.grad_u[2u * nv + v] = guz[i];
          A.grad_chi[v] = gch[i];
        }
      }
    }
  }
  __syncthreads();
  if (tid < A.n_peaks) A.alpha_part[(long long)tile * A.n_peaks + tid] = apl[tid];
}

// --------------------------------------------------------------------- finalize ---
__global__ __launch_bounds__(256) void k_finalize(const double* __restrict__ floss,
                                                  const int* __restrict__ out_list, int n_out,
                                                  double* loss, float* frame_loss,
                                                  const double* __restrict__ apart, int n_part,
                                                  int n_peaks, float* grad_alpha) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  if (loss || frame_loss) {
    double s = 0.0;
    for (int i = tid; i < n_out; i += 256) {
      double v = floss[out_list ? out_list[i] : i];
      s += v;
      if (frame_loss) frame_loss[i] = (float)v;
    }
    red[tid] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0 && loss) *loss = red[0];
    __syncthreads();
  }
  if (grad_alpha) {
    for (int m = 0; m < n_peaks; ++m) {
      double s = 0.0;
      for (int i = tid; i < n_part; i += 256) s += apart[(long long)i * n_peaks + m];
      red[tid] = s;
      __syncthreads();
      for (int w = 128; w > 0; w >>= 1) {
        if (tid < w) red[tid] += red[tid + w];
        __syncthreads();
      }
      if (tid == 0) grad_alpha[m] = (float)red[0];
      __syncthreads();
    }
  }
}

__global__ __launch_bounds__(256) void k_step(float* __restrict__ p, const float* __restrict__ g,
                                              long long n, float eta) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = p[i] - eta * g[i];
}

__global__ __launch_bounds__(256) void k_fill_u8(unsigned char* p, long long n, unsigned char v) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

__global__ __launch_bounds__(256) void k_mark_active(unsigned char* act, const int* list, int n) {
  int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) act[list[i]] = 1;
}

// ------------------------------------------------------------------ host launchers ---
static inline unsigned nblk(long long n, int t) { return (unsigned)((n + t - 1) / t); }

hipError_t launch_object(const float* u, const float* chi, const float* alpha, const PeakDev* peaks,
                         int n_peaks, long long nvox, float* obj, hipStream_t s) {
  k_object<<<dim3(nblk(nvox, 256)), dim3(256), 0, s>>>(u, chi, alpha, peaks, n_peaks, nvox, obj);
  return hipGetLastError();
}

template <int D, int FB>
static hipError_t launch_frames_d(const FrameArgs& a, int lds_bytes, hipStream_t s) {
  const unsigned grid = a.xcd ? (unsigned)(((a.n_list + 7) / 8) * 8) : (unsigned)a.n_list;
  if (grid == 0) return hipSuccess;
  k_frames<D, FB><<<dim3(grid), dim3(kFrameThreads), lds_bytes, s>>>(a);
  return hipGetLastError();
}

int frame_bound(int D, int f) {
  if (D == 32) return 32;
  if (f <= 48) return 48;
  if (f <= 64) return 64;
  return D;
}

// Every compiled (D, FB) instance of the frame kernel.
#define MPBP_FRAME_INSTANCES(X)             \
  X(32, 32)                                 \
  X(64, 48) X(64, 64)                       \
  X(96, 48) X(96, 64) X(96, 96)             \
  X(128, 48) X(128, 64) X(128, 128)         \
  X(192, 48) X(192, 64) X(192, 192)         \
  X(256, 48) X(256, 64) X(256, 256)

hipError_t launch_frames(int D, int FB, const FrameArgs& a, int lds_bytes, hipStream_t s) {
#define MPBP_CASE(d, fb) \
  if (D == d && FB == fb) return launch_frames_d<d, fb>(a, lds_bytes, s);
  MPBP_FRAME_INSTANCES(MPBP_CASE)
#undef MPBP_CASE
  return hipErrorInvalidValue;
}

bool frame_instance(int D, int FB) {
#define MPBP_CASE(d, fb) \
  if (D == d && FB == fb) return true;
  MPBP_FRAME_INSTANCES(MPBP_CASE)
#undef MPBP_CASE
  return false;
}

hipError_t prepare_kernels() {
  hipError_t e = hipSuccess;
#define MPBP_CASE(d, fb)                                                                     \
  if (e == hipSuccess)                                                                       \
    e = hipFuncSetAttribute((const void*)k_frames<d, fb>,                                    \
                            hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  MPBP_FRAME_INSTANCES(MPBP_CASE)
#undef MPBP_CASE
  if (e == hipSuccess)
    e = hipFuncSetAttribute((const void*)k_grad, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
  return e;
}

hipError_t launch_grad(const GradArgs& a, int lds_bytes, hipStream_t s) {
  const unsigned grid = (unsigned)(((a.tiles_x * a.tiles_y + 7) / 8) * 8);
  k_grad<<<dim3(grid), dim3(kGradThreads), lds_bytes, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_finalize(const double* floss, const int* out_list, int n_out, double* loss,
                           float* frame_loss, const double* apart, int n_part, int n_peaks,
                           float* grad_alpha, hipStream_t s) {
  k_finalize<<<dim3(1), dim3(256), 0, s>>>(floss, out_list, n_out, loss, frame_loss, apart, n_part, n_peaks, grad_alpha);
  return hipGetLastError();
}

hipError_t launch_step(float* p, const float* g, long long n, float eta, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_step<<<dim3(nblk(n, 256)), dim3(256), 0, s>>>(p, g, n, eta);
  return hipGetLastError();
}

hipError_t launch_mark_active(unsigned char* act, long long n_frames, const int* list, int n,
                              hipStream_t s) {
  k_fill_u8<<<dim3(nblk(n_frames, 256)), dim3(256), 0, s>>>(act, n_frames, (unsigned char)0);
  if (n > 0) k_mark_active<<<dim3(nblk(n, 256)), dim3(256), 0, s>>>(act, list, n);
  return hipGetLastError();
}

}  // namespace mpbp

namespace mpbp {

template <int D>
static int lds_for(int fy, int fx, int fxp, int np, int nz, bool grad) {
  using RC = LineCfg<D>;
  constexpr int L = ColLen<D>::L;
  constexpr int RLINES = kFrameThreads / RC::TPL;
  constexpr int EXL = RC::Q * (RC::P + 1);
  const long long exch_min = (long long)kProjG * (np + 1) * (np + 1) - ((long long)L * fxp + L / 8);
  const long long exch = (RLINES * EXL + 1) / 2 > exch_min ? (RLINES * EXL + 1) / 2 : exch_min;
  const long long cpx = D + L + (long long)(D / L) * fy + (long long)fy * fx +
                        (grad ? (long long)fy * fx : 0) + (long long)L * fxp + L / 8 + exch;
  return (int)(cpx * 8 + (long long)nz * 8);
}

int frame_lds_bytes(int D, int fy, int fx, int fxp, int np, int nz, bool grad) {
  switch (D) {
    case 32: return lds_for<32>(fy, fx, fxp, np, nz, grad);
    case 64: return lds_for<64>(fy, fx, fxp, np, nz, grad);
    case 96: return lds_for<96>(fy, fx, fxp, np, nz, grad);
    case 128: return lds_for<128>(fy, fx, fxp, np, nz, grad);
    case 192: return lds_for<192>(fy, fx, fxp, np, nz, grad);
    case 256: return lds_for<256>(fy, fx, fxp, np, nz, grad);
    default: return -1;
  }
}

template <int D>
static void twiddles_for(int fy, std::vector<float>& out) {
  using RC = LineCfg<D>;
  constexpr int L = ColLen<D>::L;
  constexpr int R = D / L;
  using CC = LineCfg<L>;
  auto w = [&](long long k, int n) {   // exp(-2 pi i k / n), in double
    const double a = -2.0 * M_PI * (double)(k % n) / (double)n;
    out.push_back((float)std::cos(a));
    out.push_back((float)std::sin(a));
  };
  for (int c = 0; c < RC::P; ++c)
    for (int t = 0; t < RC::Q; ++t) w((long long)t * c, D);
  for (int c = 0; c < CC::P; ++c)
    for (int t = 0; t < CC::Q; ++t) w((long long)t * c, L);
  for (int r = 0; r < R; ++r)
    for (int rr = 0; rr < fy; ++rr) w((long long)rr * r, D);
}

bool frame_twiddles(int D, int fy, std::vector<float>& out) {
  switch (D) {
    case 32: twiddles_for<32>(fy, out); return true;
    case 64: twiddles_for<64>(fy, out); return true;
    case 96: twiddles_for<96>(fy, out); return true;
    case 128: twiddles_for<128>(fy, out); return true;
    case 192: twiddles_for<192>(fy, out); return true;
    case 256: twiddles_for<256>(fy, out); return true;
    default: return false;
  }
}

int frame_chunk_len(int D) {
  switch (D) {
    case 32: return ColLen<32>::L;
    case 64: return ColLen<64>::L;
    case 96: return ColLen<96>::L;
    case 128: return ColLen<128>::L;
    case 192: return ColLen<192>::L;
    case 256: return ColLen<256>::L;
    default: return -1;
  }
}

int grad_lds_bytes(int np, int nz, int maxspan_y, int maxspan_x, int max_cand) {
  (void)maxspan_y;
  (void)maxspan_x;
  return np * np * 8 + nz * 8 + kMaxPeaksDev * 8 + 64 + max_cand;
}

}  // namespace mpbp
