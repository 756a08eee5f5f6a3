// mpbp_device.hip - HIP kernels (gfx950) of the MPBP objective-and-gradient path, and
// the host launchers of every kernel of the fused path.
//
//   k_object    eq. (1)/(3): O_m = alpha_m chi exp(i G_m . u) for every voxel and peak
//   k_runsum    the same objects summed over each run of consecutive slices with equal
//               exit-beam offset (one probe for all slices, rounded offsets)
//   (k_project_runs, k_project: mpbp_project.hpp; k_frames: mpbp_frame.hpp, one
//    instance file per detector size; k_project_map, k_bp_map_color: mpbp_map.hip)
//   k_grad      per-slice gather back-projection of the footprint gradients over all
//               frames that cover a voxel tile, then the chain rule to df/du, df/dchi,
//               df/dalpha (3D probes, interpolated offsets)
//   k_bp_gather, k_bp_chain  the same per run: frame sums per run, then the chain rule
//   k_finalize  deterministic FP64 sums of the per-frame losses and alpha partials
//   k_step     p <- p - eta g
//   k_adam     one Adam update (Kingma and Ba), optionally of a log-parameter (eq. (8))
//   k_norm2    deterministic FP64 sum of squares (two passes)
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <vector>

#include "mpbp_dft.hpp"
#include "mpbp_frame.hpp"
#include "mpbp_project.hpp"
#include "mpbp_chain.hpp"
#include "mpbp_phase.hpp"
#include "mpbp_kernels.hpp"
#include "mpbp_launch.hpp"

namespace mpbp {

// ------------------------------------------------------------------ object build ---
// tied > 0: u and chi are given per lateral pixel ([3][1][ny][nx], [1][ny][nx], with
// tied = ny * nx) and hold for every slice.
__global__ __launch_bounds__(256) void k_object(const float* __restrict__ u,
                                                const float* __restrict__ chi,
                                                const float* __restrict__ alpha,
                                                const PeakDev* __restrict__ peaks, int n_peaks,
                                                long long nvox, long long tied, float* __restrict__ obj) {
  long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (v >= nvox) return;
  const long long vi = tied ? v % tied : v;
  const long long us = tied ? tied : nvox;
  float ux = u[vi], uy = u[us + vi], uz = u[2 * us + vi];
  float ch = chi[vi];
  for (int m = 0; m < n_peaks; ++m) {
    // G . u with explicit FMAs: the gradient kernel forms the same phase bit for bit
    float phi = fmaf(peaks[m].gz, uz, fmaf(peaks[m].gy, uy, peaks[m].gx * ux));
    float s, c;
    phase_sincos(phi, s, c);
    float a = alpha[m] * ch;
    float2* o = reinterpret_cast<float2*>(obj) + (long long)m * nvox + v;
    *o = make_float2(a * c, a * s);
  }
}

// --------------------------------------------------------- run-summed objects ---
// With one probe for all slices and rounded exit-beam offsets, eq. (2)'s projection
// regroups over runs k of consecutive slices with equal offset s_k:
//   R diag(P) S O = sum_k shift_{s_k}( P . S_k[window] ),  S_k = sum_{z in run k} O_z,
// and S_k does not depend on the frame.  This kernel forms every S_k of every peak once
// (in place of the per-slice objects): one lane per lateral pixel walks z, forms
// O_m(z) = alpha_m chi e^{i G_m . u} (as k_object) and adds it to peak m's running sum,
// kept in LDS, which is stored at the last slice of each run.  Output: complex64
// [run_base_m + k][ny][nx].
__global__ __launch_bounds__(256) void k_runsum(const float* __restrict__ u, const float* __restrict__ chi,
                                                const float* __restrict__ alpha,
                                                const PeakDev* __restrict__ peaks, int n_peaks, int nz,
                                                long long nlat, int tied, const int* __restrict__ zrun,
                                                float* __restrict__ rsum) {
  __shared__ float2 acc[kMaxPeaksDev][256];
  const int tid = threadIdx.x;
  const long long p = (long long)blockIdx.x * 256 + tid;
  if (p >= nlat) return;   // (no barriers below: each lane's sums are its own)
  const long long us = tied ? nlat : (long long)nz * nlat;   // field component stride
  constexpr int ZB = 4;   // slices whose fields are loaded together
  for (int z0 = 0; z0 < nz; z0 += ZB) {
    float fu[ZB][3], fc[ZB];
#pragma unroll
    for (int i = 0; i < ZB; ++i) {
      const long long vi = tied ? p : (long long)min(z0 + i, nz - 1) * nlat + p;
      fu[i][0] = u[vi];
      fu[i][1] = u[us + vi];
      fu[i][2] = u[2 * us + vi];
      fc[i] = chi[vi];
    }
#pragma unroll
    for (int i = 0; i < ZB; ++i) {
    const int z = z0 + i;
    if (z >= nz) break;   // uniform
    const float ux = fu[i][0], uy = fu[i][1], uz = fu[i][2];
    const float ch = fc[i];
    for (int m = 0; m < n_peaks; ++m) {
      const float gx = peaks[m].gx, gy = peaks[m].gy, gz = peaks[m].gz;
      const float phi = fmaf(gz, uz, fmaf(gy, uy, gx * ux));   // as k_object
      float s, c;
      phase_sincos(phi, s, c);
      const float a = alpha[m] * ch;
      const float2 o = make_float2(a * c, a * s);
      const int* zr = zrun + m * nz;
      const int k = zr[z];
      const bool first = z == 0 || zr[z - 1] != k;    // uniform
      const bool last = z == nz - 1 || zr[z + 1] != k;
      const float2 cur = first ? o : make_float2(acc[m][tid].x + o.x, acc[m][tid].y + o.y);
      if (last)
        reinterpret_cast<float2*>(rsum)[(long long)(peaks[m].run_base + k) * nlat + p] = cur;
      else
        acc[m][tid] = cur;
    }
    }
  }
}

// -------------------------------------------- gather back-projection + chain rule ---
// B: frames whose footprint gradients are read per step of the frame walk.  TX: tile
// width (TX x TY voxels per slice, TX * TY = 64: one wavefront per slice).  The tile
// grid starts at (tile_oy, tile_ox) <= 0, so that a grid aligned with a raster of step
// TX x TY gives every voxel of a tile the same covering frames.
// P3: the probe varies along z (probe [M][nz][np][np]): conj(P_z) is read per frame and
// slice from the probe volume (L2-resident) instead of the per-peak probe in LDS.
// LIN: fractional exit-beam offsets (A.shw): a voxel's footprint gradient is the
// bilinearly weighted sum of four footprint pixels (the adjoint of the projection's taps).
template <int B, int TX, bool P3, bool LIN>
__global__ __launch_bounds__(kGradThreads, 4) void k_grad(GradArgs A) {
  constexpr int TY = kGradTile / TX;
  extern __shared__ cplx smem[];
  const int np = A.np, nz = A.nz;
  cplx* Ps = smem;                                   // np * np
  int2* sh = reinterpret_cast<int2*>(Ps + np * np);  // nz
  double* apl = reinterpret_cast<double*>(sh + nz);  // alpha partials
  float* red = reinterpret_cast<float*>(apl + kMaxPeaksDev);       // block reduction
  unsigned char* actf = reinterpret_cast<unsigned char*>(red + 16);  // candidate frames' flags
  // z-tied: per-thread partial z-sums, reduced over the slice groups at the end
  float* zred = reinterpret_cast<float*>(actf + ((A.max_cand + 15) & ~15));
  float tgu[3] = {0.f, 0.f, 0.f}, tgc = 0.f;

  const int tid = threadIdx.x;
  const int tx = tid % TX, ty = (tid / TX) % TY, tz = tid / kGradTile;
  // Tiles are handed out so that each XCD (blocks are dispatched round-robin over the
  // 8 XCDs) walks a contiguous band of tile rows: neighbouring tiles read the same
  // frames' footprints, which then stay in that XCD's L2.
  const int tile = frame_block_index(blockIdx.x, gridDim.x, 1);
  if (tile >= A.tiles_x * A.tiles_y) return;
  const int bx = tile % A.tiles_x, by = tile / A.tiles_x;
  const int x0 = A.tile_ox + bx * TX, y0 = A.tile_oy + by * TY;
  const int x = x0 + tx, y = y0 + ty;
  const bool inb = (unsigned)x < (unsigned)A.nx && (unsigned)y < (unsigned)A.ny;
  const long long nvox = (long long)nz * A.ny * A.nx;
  const unsigned lat = (unsigned)(y * A.nx + x);                 // lateral pixel
  const unsigned fstride = A.tied ? (unsigned)(A.ny * A.nx) : (unsigned)nvox;   // field component stride
  if (tid < kMaxPeaksDev) apl[tid] = 0.0;

  for (int zb = 0; zb < nz; zb += kGradZB) {
    float gux[kGradZPer], guy[kGradZPer], guz[kGradZPer], gch[kGradZPer];
#pragma unroll
    for (int i = 0; i < kGradZPer; ++i) gux[i] = guy[i] = guz[i] = gch[i] = 0.f;

    for (int m = 0; m < A.n_peaks; ++m) {
      const PeakDev pk = uniform_peak(A.peaks + m);
      // Frames of this peak whose windows meet the tile: a rectangle of the raster.
      const int iy_lo = max(0, -floordiv(-(y0 - np + 1 - pk.oy), pk.sy));
      const int iy_hi = min(pk.rows - 1, floordiv(y0 + TY - 1 - pk.oy, pk.sy));
      const int ix_lo = max(0, -floordiv(-(x0 - np + 1 - pk.ox), pk.sx));
      const int ix_hi = min(pk.cols - 1, floordiv(x0 + TX - 1 - pk.ox, pk.sx));
      const int ncx = ix_hi - ix_lo + 1;
      const int ncand = (iy_hi >= iy_lo && ncx > 0) ? (iy_hi - iy_lo + 1) * ncx : 0;
      __syncthreads();
      const cplx* probe = reinterpret_cast<const cplx*>(A.probe) + (long long)m * (P3 ? nz : 1) * np * np;
      if (!P3)
        for (int k = tid; k < np * np; k += kGradThreads) Ps[k] = probe[k];
      for (int z = tid; z < nz; z += kGradThreads) {
        const int* s = A.shear + 2 * (m * nz + z);
        sh[z] = make_int2(s[0], s[1]);
      }
      // minibatch flags of the candidate frames, loaded in parallel
      for (int c = tid; c < (A.all_active ? 0 : ncand); c += kGradThreads) {
        const int cy = iy_lo + c / ncx, cx = ix_lo + c % ncx;
        actf[c] = A.active[pk.frame_base + cy * pk.cols + cx];
      }
      cplx acc[kGradZPer];
#pragma unroll
      for (int i = 0; i < kGradZPer; ++i) acc[i] = {0.f, 0.f};
      __syncthreads();

      // this lane's slices: shear offsets (and tap weights) in registers.  With integer
      // offsets and one probe for all slices, a slice whose offset equals the previous
      // slice's reads the same footprint pixel with the same probe value: its sum over
      // the frames is the previous slice's, so it skips the walk (same[i], uniform per
      // wavefront: the lanes of one wavefront share their slices).
      constexpr bool kRuns = !LIN && !P3;
      int zsy[kGradZPer], zsx[kGradZPer];
      bool same[kGradZPer];
      float zw[kGradZPer][LIN ? 4 : 1];
#pragma unroll
      for (int i = 0; i < kGradZPer; ++i) {
        const int z = zb + tz * kGradZPer + i;
        zsy[i] = sh[z < nz ? z : 0].x - pk.miny;
        zsx[i] = sh[z < nz ? z : 0].y - pk.minx;
        same[i] = __builtin_amdgcn_readfirstlane(
                      (int)(kRuns && i > 0 && z < nz && zsy[i] == zsy[i - 1] && zsx[i] == zsx[i - 1])) != 0;
        if constexpr (LIN) {
          const int zc = z < nz ? z : 0;
          const float ry = A.shw[2 * (m * nz + zc)], rx = A.shw[2 * (m * nz + zc) + 1];
          zw[i][0] = (1.f - ry) * (1.f - rx);
          zw[i][LIN ? 1 : 0] = (1.f - ry) * rx;
          zw[i][LIN ? 2 : 0] = ry * (1.f - rx);
          zw[i][LIN ? 3 : 0] = ry * rx;
        }
      }
      // Frames of the minibatch, B at a time (uniform walk, scalar results).
      // Each lane reads its footprint-gradient values straight from the frame's slot:
      // a wavefront covers a 4 x 16 voxel patch at one slice, so its reads are rows.
      const cplx* slots = reinterpret_cast<const cplx*>(A.slots);
      // one batch of nb (<= B) frames: window origins (fpy, fpx) and slot offsets fso
      auto batch = [&](int nb, const int (&fpy)[B], const int (&fpx)[B], const long long (&fso)[B])
                       __attribute__((always_inline)) {
          cplx gv[B][kGradZPer], pv[B], pz[B][P3 ? kGradZPer : 1];
#pragma unroll
          for (int k = 0; k < B; ++k) {
            const int a = y - fpy[k], b = x - fpx[k];
            const bool inw = k < nb && inb && (unsigned)a < (unsigned)np && (unsigned)b < (unsigned)np;
            const int ac = inw ? a : 0, bc = inw ? b : 0;
            if constexpr (P3) {
#pragma unroll
              for (int i = 0; i < kGradZPer; ++i) {
                const int z = zb + tz * kGradZPer + i;
                const cplx pr = probe[(long long)(z < nz ? z : 0) * np * np + ac * np + bc];
                pz[k][i] = inw ? pr : cplx{0.f, 0.f};
              }
            } else {
              const cplx pr = Ps[ac * np + bc];
              pv[k] = inw ? pr : cplx{0.f, 0.f};
            }
            // uniform slot base + 32-bit lane offset (a slot holds fewer than 2^29 values)
            const char* sl = reinterpret_cast<const char*>(slots + fso[k]);
#pragma unroll
            for (int i = 0; i < kGradZPer; ++i) {
              if (same[i]) continue;
              const unsigned off = (unsigned)((ac + zsy[i]) * pk.fx + bc + zsx[i]) * (unsigned)sizeof(cplx);
              const bool okq = MPBP_CHECK(
                  A.dbg, off / sizeof(cplx) + (LIN ? pk.fx + 1 : 0) < (unsigned)(pk.fy * pk.fx), kDbgSlot);
              const cplx* q = reinterpret_cast<const cplx*>(okq ? sl + off : sl);
              if constexpr (LIN) {
                const cplx q00 = q[0], q01 = q[1], q10 = q[pk.fx], q11 = q[pk.fx + 1];
                gv[k][i] = cadd(cadd(cscale(q00, zw[i][0]), cscale(q01, zw[i][LIN ? 1 : 0])),
                                cadd(cscale(q10, zw[i][LIN ? 2 : 0]), cscale(q11, zw[i][LIN ? 3 : 0])));
              } else {
                gv[k][i] = q[0];
              }
            }
          }
#pragma unroll
          for (int k = 0; k < B; ++k)
#pragma unroll
            for (int i = 0; i < kGradZPer; ++i)   // conj(P) g_psi
              if (!same[i]) acc[i] = cmulc_acc(acc[i], gv[k][i], P3 ? pz[k][P3 ? i : 0] : pv[k]);
      };
      if (A.all_active) {
        // full batch: every covering frame, row by row, B consecutive columns per batch;
        // window origins and slot offsets advance by additions (scalar registers)
        const long long fyfx = (long long)pk.fy * pk.fx;
        int wy = pk.oy + iy_lo * pk.sy;
        long long srow = pk.slot_off + (long long)(iy_lo * pk.cols + ix_lo) * fyfx;
        for (int cy = iy_lo; cy <= iy_hi; ++cy) {
          int wx = pk.ox + ix_lo * pk.sx;
          long long so = srow;
          for (int cx = ix_lo; cx <= ix_hi; cx += B) {
            const int nb = min(B, ix_hi - cx + 1);
            int fpy[B], fpx[B];
            long long fso[B];
#pragma unroll
            for (int k = 0; k < B; ++k) {   // past the row's end: the batch's first slot
              fpy[k] = wy;
              fpx[k] = wx + k * pk.sx;
              fso[k] = k < nb ? so + k * fyfx : so;
            }
            batch(nb, fpy, fpx, fso);
            wx += B * pk.sx;
            so += B * fyfx;
          }
          wy += pk.sy;
          srow += (long long)pk.cols * fyfx;
        }
      } else {
        // minibatch: skip the frames whose flag is clear
        int iy = iy_lo, ix = ix_lo, ci = 0;
        while (ix_lo <= ix_hi && iy <= iy_hi) {
          int nb = 0;
          int fpy[B], fpx[B];
          long long fso[B];
#pragma unroll
          for (int k = 0; k < B; ++k) {
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
          batch(nb, fpy, fpx, fso);
        }
      }
#pragma unroll
      for (int i = 1; i < kGradZPer; ++i)
        if (same[i]) acc[i] = acc[i - 1];
      // chain rule through O_m = alpha_m chi exp(i G_m . u); 32-bit voxel offsets from
      // uniform bases (the plan limits 3 * nvox to 2^32)
      float ap = 0.f;
      if (inb) {
        const float al = A.alpha[m];
        const unsigned nv = (unsigned)nvox;
#pragma unroll
        for (int i = 0; i < kGradZPer; ++i) {
          const int z = zb + tz * kGradZPer + i;
          if (z < nz) {
            const unsigned v = ((unsigned)z * (unsigned)A.ny + (unsigned)y) * (unsigned)A.nx + (unsigned)x;
            const unsigned vf = A.tied ? lat : v;
            const float ux = A.u[vf], uy = A.u[fstride + vf], uzv = A.u[2u * fstride + vf];
            chain_voxel(pk, acc[i], ux, uy, uzv, A.chi[vf], al, gux[i], guy[i], guz[i], gch[i], ap);
          }
        }
      }
      const float apb = block_sum_f(ap, red);
      if (tid == 0) apl[m] += (double)apb;
    }
    if (inb && A.tied) {
#pragma unroll
      for (int i = 0; i < kGradZPer; ++i) {
        tgu[0] += gux[i];
        tgu[1] += guy[i];
        tgu[2] += guz[i];
        tgc += gch[i];
      }
    } else if (inb) {
      const unsigned nv = (unsigned)nvox;
#pragma unroll
      for (int i = 0; i < kGradZPer; ++i) {
        const int z = zb + tz * kGradZPer + i;
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
  if (A.tied) {
    // z-sums: add the kGradTZ slice groups of each lateral pixel in a fixed order
    const int xy = tid % kGradTile;
    zred[0 * kGradThreads + tid] = tgu[0];
    zred[1 * kGradThreads + tid] = tgu[1];
    zred[2 * kGradThreads + tid] = tgu[2];
    zred[3 * kGradThreads + tid] = tgc;
    __syncthreads();
    if (tz == 0 && inb) {
      float s[4] = {0.f, 0.f, 0.f, 0.f};
      for (int g = 0; g < kGradTZ; ++g)
#pragma unroll
        for (int c = 0; c < 4; ++c) s[c] += zred[c * kGradThreads + g * kGradTile + xy];
      A.grad_u[lat] = s[0];
      A.grad_u[fstride + lat] = s[1];
      A.grad_u[2u * fstride + lat] = s[2];
      A.grad_chi[lat] = s[3];
    }
  }
  if (tid < A.n_peaks) A.alpha_part[(long long)tile * A.n_peaks + tid] = apl[tid];
}

// ------------------------------------ back-projection over runs of slices ---
// With one probe for all slices and rounded exit-beam offsets (neither MPBP_PROBE_3D nor
// MPBP_SHEAR_LINEAR), the slices of a run (consecutive slices with equal offset) read
// the same footprint pixel of every frame with the same probe value: the frame sum
//   G_{m,k}[y][x] = sum_f conj(P_m[y - py_f][x - px_f]) g_psi,f[y - py_f + o_k][x - px_f + o_k']
// serves every slice of run k.  Two kernels:
//   k_bp_gather  one workgroup per (peak, voxel tile): the frames of the minibatch that
//                meet the tile are listed in LDS (raster order), and each wavefront sums
//                them for the tile's 64 pixels and one run at a time, B frames' loads in
//                flight per lane; the sums go to G (the run sums' buffer, which the
//                forward projection no longer needs).
//   k_bp_chain   one lane per lateral pixel walks the slices: the chain rule through
//                O_m = alpha_m chi e^{i G_m . u} on G_{m, run of z}, gradients written per
//                voxel (z-summed when tied), alpha partials per workgroup.
// The frames are summed in raster order with the fused multiply-adds of k_grad and the
// chain rule is k_grad's (chain_voxel, peaks in order): df/du and df/dchi come out
// bitwise equal to the per-slice walk; the alpha partials group the voxels differently.
struct GradCand {
  int fpy, fpx;
  long long so;
};

template <int B, int TX>
__global__ __launch_bounds__(kBpThreads) void k_bp_gather(GradArgs A) {
  constexpr int TY = kGradTile / TX;
  extern __shared__ cplx smem[];
  const int np = A.np, nz = A.nz;
  cplx* Ps = smem;                                                     // np * np
  GradCand* cand = reinterpret_cast<GradCand*>(Ps + np * np);          // [max_cand]
  int* ncand_s = reinterpret_cast<int*>(cand + A.max_cand);
  const int tid = threadIdx.x;
  const int lane = tid % kGradTile, wv = tid / kGradTile;
  const int ntiles = A.tiles_x * A.tiles_y;
  // XCD k takes a contiguous range of (peak, tile): neighbouring tiles read the same
  // frames' footprints, which then stay in that XCD's L2
  const int bid = frame_block_index(blockIdx.x, gridDim.x, 1);
  if (bid >= ntiles * A.n_peaks) return;
  const int m = bid / ntiles, tile = bid % ntiles;
  const int bx = tile % A.tiles_x, by = tile / A.tiles_x;
  const int x0 = A.tile_ox + bx * TX, y0 = A.tile_oy + by * TY;
  const int x = x0 + lane % TX, y = y0 + lane / TX;
  const bool inb = (unsigned)x < (unsigned)A.nx && (unsigned)y < (unsigned)A.ny;
  const PeakDev pk = uniform_peak(A.peaks + m);
  const int iy_lo = max(0, -floordiv(-(y0 - np + 1 - pk.oy), pk.sy));
  const int iy_hi = min(pk.rows - 1, floordiv(y0 + TY - 1 - pk.oy, pk.sy));
  const int ix_lo = max(0, -floordiv(-(x0 - np + 1 - pk.ox), pk.sx));
  const int ix_hi = min(pk.cols - 1, floordiv(x0 + TX - 1 - pk.ox, pk.sx));
  const int ncx = ix_hi - ix_lo + 1;
  const int ncand = (iy_hi >= iy_lo && ncx > 0) ? (iy_hi - iy_lo + 1) * ncx : 0;
  const cplx* probe = reinterpret_cast<const cplx*>(A.probe) + (long long)m * np * np;
  for (int k = tid; k < np * np; k += kBpThreads) Ps[k] = probe[k];
  // the frames of the minibatch meeting the tile, in raster order (wavefront 0: flags,
  // ballot, prefix count)
  if (tid < 64) {
    int base = 0;
    for (int c0 = 0; c0 < ncand; c0 += 64) {
      const int c = c0 + tid;
      const int cy = iy_lo + c / (ncx > 0 ? ncx : 1), cx = ix_lo + c % (ncx > 0 ? ncx : 1);
      const bool act = c < ncand && (A.all_active || A.active[pk.frame_base + cy * pk.cols + cx]);
      const unsigned long long mask = __ballot(act);
      const int pos = base + (int)__builtin_amdgcn_mbcnt_hi((unsigned)(mask >> 32),
                                                            __builtin_amdgcn_mbcnt_lo((unsigned)mask, 0u));
      if (act && MPBP_CHECK(A.dbg, pos < A.max_cand, kDbgFrameList))
        cand[pos] = {pk.oy + cy * pk.sy, pk.ox + cx * pk.sx,
                     pk.slot_off + (long long)(cy * pk.cols + cx) * pk.fy * pk.fx};
      base += __popcll(mask);
    }
    if (tid == 0) *ncand_s = base;
  }
  __syncthreads();
  const int nact = min(__builtin_amdgcn_readfirstlane(*ncand_s), A.max_cand);
  const cplx* slots = reinterpret_cast<const cplx*>(A.slots);
  cplx* G = reinterpret_cast<cplx*>(A.rs) + (long long)pk.run_base * A.nlat + (long long)(inb ? y : 0) * A.nx + (inb ? x : 0);
  // Wavefront wv sums runs wv, wv + 4, ..., up to kBpRunGroup of them per pass over the
  // frame list: a frame's window position, probe value and footprint offset are worked
  // out once and serve each of those runs, which differ only by the run's offset.
  constexpr int NW = kBpThreads / kGradTile;
  const int lane_p = y * np + x, lane_f = y * pk.fx + x;
  for (int run0 = wv; run0 < pk.nruns; run0 += NW * kBpRunGroup) {
    int rof[kBpRunGroup];   // footprint offset of each run of the group (uniform)
#pragma unroll
    for (int g = 0; g < kBpRunGroup; ++g) {
      const int run = run0 + NW * g;
      const int2 ro = A.roff[m * nz + (run < pk.nruns ? run : run0)];
      rof[g] = __builtin_amdgcn_readfirstlane(ro.x * pk.fx + ro.y);
    }
    cplx acc[kBpRunGroup];
#pragma unroll
    for (int g = 0; g < kBpRunGroup; ++g) acc[g] = {0.f, 0.f};
    for (int c0 = 0; c0 < nact; c0 += B) {
      // one LDS read brings the batch's B list entries (lane l holds entry c0 + l mod B;
      // past the list: the batch's first entry), then each is taken from its lane
      const int cl = c0 + lane % B < nact ? c0 + lane % B : c0;
      const GradCand mine = cand[cl];
      const unsigned so_lo = (unsigned)mine.so, so_hi = (unsigned)((unsigned long long)mine.so >> 32);
      cplx pv[B];
      unsigned off[B];   // byte offset of (y, x)'s footprint pixel at zero run offset
      const char* sl[B];
#pragma unroll
      for (int k = 0; k < B; ++k) {
        const int fpy = __builtin_amdgcn_readlane(mine.fpy, k);
        const int fpx = __builtin_amdgcn_readlane(mine.fpx, k);
        const long long so = (long long)(((unsigned long long)__builtin_amdgcn_readlane(so_hi, k) << 32) |
                                         (unsigned)__builtin_amdgcn_readlane(so_lo, k));
        const int a = y - fpy, b = x - fpx;
        const bool inw = inb && (unsigned)a < (unsigned)np && (unsigned)b < (unsigned)np;
        // (a, b) = (y, x) - window origin: the probe index and the footprint offset are
        // the lane's own value at origin 0 minus a uniform one
        const int pi = inw ? lane_p - (fpy * np + fpx) : 0;
        const cplx pr = Ps[pi];
        pv[k] = inw ? pr : cplx{0.f, 0.f};
        sl[k] = reinterpret_cast<const char*>(slots + so);
        off[k] = inw ? (unsigned)(lane_f - (fpy * pk.fx + fpx)) : 0u;
      }
#pragma unroll
      for (int g = 0; g < kBpRunGroup; ++g) {
        if (run0 + NW * g < pk.nruns) {   // uniform
          cplx gv[B];
#pragma unroll
          for (int k = 0; k < B; ++k) {
            const unsigned o = off[k] + (unsigned)rof[g];
            const bool okg = MPBP_CHECK(A.dbg, o < (unsigned)(pk.fy * pk.fx), kDbgSlot);
            gv[k] = *reinterpret_cast<const cplx*>(sl[k] + (okg ? o : 0u) * (unsigned)sizeof(cplx));
          }
#pragma unroll
          for (int k = 0; k < B; ++k)
            if (c0 + k < nact) acc[g] = cmulc_acc(acc[g], gv[k], pv[k]);   // conj(P) g_psi
        }
      }
    }
#pragma unroll
    for (int g = 0; g < kBpRunGroup; ++g) {
      const int run = run0 + NW * g;
      if (run < pk.nruns && inb && MPBP_CHECK(A.dbg, pk.run_base + run < A.n_runs, kDbgRunSum))
        G[(long long)run * A.nlat] = acc[g];
    }
  }
}

// One lane per lateral pixel and chunk of kBpZ slices (per lateral pixel and every slice
// when tied: the z-sum stays in the lane).
__global__ __launch_bounds__(kBpThreads) void k_bp_chain(GradArgs A) {
  __shared__ float red[kBpThreads / 64];
  const int tid = threadIdx.x;
  const long long t = (long long)blockIdx.x * kBpThreads + tid;
  const int nz = A.nz;
  const long long p = A.tied ? t : t % A.nlat;
  const int z0 = A.tied ? 0 : (int)(t / A.nlat) * kBpZ;
  const int z1 = A.tied ? nz : min(z0 + kBpZ, nz);
  const bool on = A.tied ? t < A.nlat : z0 < nz;
  const long long nvox = (long long)nz * A.nlat;
  const long long us = A.tied ? A.nlat : nvox;    // field component stride
  const cplx* G = reinterpret_cast<const cplx*>(A.rs);
  float ap[kMaxPeaksDev];
  float tg[4] = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
  for (int m = 0; m < kMaxPeaksDev; ++m) ap[m] = 0.f;
  if (on && !A.tied) {
    // kBpZ slices: every load is issued before the first store (the compiler cannot move
    // loads across the gradient stores, which might alias the fields as far as it knows)
    float fu[kBpZ][3], fc[kBpZ], gu[kBpZ][3], gc[kBpZ];
#pragma unroll
    for (int i = 0; i < kBpZ; ++i) {
      const long long vi = (long long)min(z0 + i, nz - 1) * A.nlat + p;
      fu[i][0] = A.u[vi];
      fu[i][1] = A.u[us + vi];
      fu[i][2] = A.u[2 * us + vi];
      fc[i] = A.chi[vi];
      gu[i][0] = gu[i][1] = gu[i][2] = gc[i] = 0.f;
    }
#pragma unroll
    for (int m = 0; m < kMaxPeaksDev; ++m) {
      if (m < A.n_peaks) {   // uniform
        const PeakDev pk = uniform_peak(A.peaks + m);
        cplx g[kBpZ];
#pragma unroll
        for (int i = 0; i < kBpZ; ++i) {
          int k = A.zrun[m * nz + min(z0 + i, nz - 1)];
          if (!MPBP_CHECK(A.dbg, k >= 0 && pk.run_base + k < A.n_runs, kDbgRunSum)) k = -pk.run_base;
          g[i] = G[(long long)(pk.run_base + k) * A.nlat + p];
        }
        const float al = A.alpha[m];
#pragma unroll
        for (int i = 0; i < kBpZ; ++i)
          if (z0 + i < z1)
            chain_voxel(pk, g[i], fu[i][0], fu[i][1], fu[i][2], fc[i], al, gu[i][0], gu[i][1], gu[i][2], gc[i], ap[m]);
      }
    }
#pragma unroll
    for (int i = 0; i < kBpZ; ++i) {
      if (z0 + i < z1) {
        const long long vi = (long long)(z0 + i) * A.nlat + p;
        A.grad_u[vi] = gu[i][0];
        A.grad_u[nvox + vi] = gu[i][1];
        A.grad_u[2 * nvox + vi] = gu[i][2];
        A.grad_chi[vi] = gc[i];
      }
    }
  } else if (on) {   // z-tied: every slice of the lateral pixel, summed in the lane
    for (int z = z0; z < z1; ++z) {
      const long long vi = A.tied ? p : (long long)z * A.nlat + p;
      const float ux = A.u[vi], uy = A.u[us + vi], uz = A.u[2 * us + vi], ch = A.chi[vi];
      float gux = 0.f, guy = 0.f, guz = 0.f, gch = 0.f;
#pragma unroll
      for (int m = 0; m < kMaxPeaksDev; ++m) {
        if (m < A.n_peaks) {   // uniform
          const PeakDev pk = uniform_peak(A.peaks + m);
          int k = A.zrun[m * nz + z];
          if (!MPBP_CHECK(A.dbg, k >= 0 && pk.run_base + k < A.n_runs, kDbgRunSum)) k = -pk.run_base;
          const cplx g = G[(long long)(pk.run_base + k) * A.nlat + p];
          chain_voxel(pk, g, ux, uy, uz, ch, A.alpha[m], gux, guy, guz, gch, ap[m]);
        }
      }
      if (A.tied) {
        tg[0] += gux;
        tg[1] += guy;
        tg[2] += guz;
        tg[3] += gch;
      } else {
        A.grad_u[vi] = gux;
        A.grad_u[nvox + vi] = guy;
        A.grad_u[2 * nvox + vi] = guz;
        A.grad_chi[vi] = gch;
      }
    }
    if (A.tied) {
      A.grad_u[p] = tg[0];
      A.grad_u[A.nlat + p] = tg[1];
      A.grad_u[2 * A.nlat + p] = tg[2];
      A.grad_chi[p] = tg[3];
    }
  }
  // alpha partials of this workgroup, one sum per peak (fixed order)
  for (int m = 0; m < A.n_peaks; ++m) {
    float v = 0.f;
#pragma unroll
    for (int q = 0; q < kMaxPeaksDev; ++q)
      if (q == m) v = ap[q];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off);
    __syncthreads();
    if ((tid & 63) == 0) red[tid >> 6] = v;
    __syncthreads();
    if (tid == 0) {
      double t = 0.0;
      for (int w = 0; w < kBpThreads / 64; ++w) t += (double)red[w];
      A.alpha_part[(long long)blockIdx.x * A.n_peaks + m] = t;
    }
  }
}

// --------------------------------------------------------------------- finalize ---
// One workgroup of 1024 lanes.  Each lane reads its values in batches of kFinBatch
// independent loads (a loop of one load per add would wait a full memory latency per
// value), adds them in index order, and the lanes' partials are combined in a fixed
// order: the sums are deterministic.
constexpr int kFinThreads = 1024;
constexpr int kFinBatch = 8;
constexpr int kFinPeaks = 4;

__device__ __forceinline__ double fin_block_sum(double s, double* red) {
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  double t = 0.0;
  for (int w = 0; w < kFinThreads / 64; ++w) t += red[w];
  __syncthreads();
  return t;
}

__global__ __launch_bounds__(kFinThreads) void k_finalize(const double* __restrict__ floss,
                                                          const int* __restrict__ out_list, int n_out,
                                                          double* __restrict__ loss,
                                                          float* __restrict__ frame_loss,
                                                          const double* __restrict__ apart, int n_part,
                                                          int n_peaks, float* __restrict__ grad_alpha) {
  __shared__ double red[kFinThreads / 64];
  const int tid = threadIdx.x;
  if (loss || frame_loss) {
    double s = 0.0;
    for (int i0 = 0; i0 < n_out; i0 += kFinBatch * kFinThreads) {
      double v[kFinBatch];
#pragma unroll
      for (int u = 0; u < kFinBatch; ++u) {
        const int i = i0 + u * kFinThreads + tid;
        v[u] = i < n_out ? floss[out_list ? out_list[i] : i] : 0.0;
      }
#pragma unroll
      for (int u = 0; u < kFinBatch; ++u) {
        const int i = i0 + u * kFinThreads + tid;
        s += v[u];
        if (frame_loss && i < n_out) frame_loss[i] = (float)v[u];
      }
    }
    const double t = fin_block_sum(s, red);
    if (tid == 0 && loss) *loss = t;
  }
  if (grad_alpha) {
    // kFinPeaks peaks per pass over the partials (a partial's peaks are adjacent), each
    // peak's values added in the same order as alone
    for (int m0 = 0; m0 < n_peaks; m0 += kFinPeaks) {
      double s[kFinPeaks];
#pragma unroll
      for (int j = 0; j < kFinPeaks; ++j) s[j] = 0.0;
      for (int i0 = 0; i0 < n_part; i0 += kFinBatch * kFinThreads) {
        double v[kFinBatch][kFinPeaks];
#pragma unroll
        for (int u = 0; u < kFinBatch; ++u) {
          const int i = i0 + u * kFinThreads + tid;
#pragma unroll
          for (int j = 0; j < kFinPeaks; ++j)
            v[u][j] = i < n_part && m0 + j < n_peaks ? apart[(long long)i * n_peaks + m0 + j] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < kFinBatch; ++u)
#pragma unroll
          for (int j = 0; j < kFinPeaks; ++j) s[j] += v[u][j];
      }
#pragma unroll
      for (int j = 0; j < kFinPeaks; ++j) {
        if (m0 + j < n_peaks) {   // uniform
          const double t = fin_block_sum(s[j], red);
          if (tid == 0) grad_alpha[m0 + j] = (float)t;
        }
      }
    }
  }
}

__global__ __launch_bounds__(256) void k_step(float* __restrict__ p, const float* __restrict__ g,
                                              long long n, float eta) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = p[i] - eta * g[i];
}

// Adam on n parameters p with gradient g of f with respect to the model variable.
// log_mode: p is the log of the model variable x = exp(p) (eq. (8)); the gradient is
// taken to p by df/dp = x df/dx, and x is rewritten from the updated p.  Otherwise p is
// the model variable and, with project, is clamped at 0 after the step.  c1 = 1 - b1^t,
// c2 = 1 - b2^t (bias corrections).  Element `fixed` (or none if < 0) is left alone.
__global__ __launch_bounds__(256) void k_adam(float* __restrict__ p, float* __restrict__ x,
                                              float* __restrict__ m, float* __restrict__ v,
                                              const float* __restrict__ g, long long n, float lr,
                                              float b1, float b2, float eps, float c1, float c2,
                                              int log_mode, int project, long long fixed) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || i == fixed) return;
  float gi = g[i];
  if (log_mode) gi *= x[i];
  const float mi = b1 * m[i] + (1.f - b1) * gi;
  const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
  m[i] = mi;
  v[i] = vi;
  float pi = p[i] - lr * (mi / c1) / (sqrtf(vi / c2) + eps);
  if (log_mode) {
    x[i] = expf(pi);
  } else if (project) {
    pi = fmaxf(pi, 0.f);
  }
  p[i] = pi;
}

// x = exp(xlog) (eq. (8)), and a plain fill (graph-safe zeroing of optimiser state).
__global__ __launch_bounds__(256) void k_exp(float* __restrict__ x, const float* __restrict__ xlog, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = expf(xlog[i]);
}

__global__ __launch_bounds__(256) void k_fill_f32(float* __restrict__ p, long long n, float v) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// Sum of squares: per-block FP64 partials in a fixed order, then one block adds them.
__global__ __launch_bounds__(256) void k_norm2_part(const float* __restrict__ a, long long n,
                                                    double* __restrict__ part) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (long long i = (long long)blockIdx.x * 256 + tid; i < n; i += (long long)gridDim.x * 256) {
    const double q = (double)a[i];
    s += q * q;
  }
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) part[blockIdx.x] = red[0];
}

__global__ __launch_bounds__(256) void k_norm2_final(const double* __restrict__ part, int n_part,
                                                     double* __restrict__ out) {
  __shared__ double red[256];
  const int tid = threadIdx.x;
  double s = 0.0;
  for (int i = tid; i < n_part; i += 256) s += part[i];
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) *out = red[0];
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
                         int n_peaks, long long nvox, long long tied, float* obj, hipStream_t s) {
  k_object<<<dim3(nblk(nvox, 256)), dim3(256), 0, s>>>(u, chi, alpha, peaks, n_peaks, nvox, tied, obj);
  return hipGetLastError();
}

hipError_t launch_runsum(const float* u, const float* chi, const float* alpha, const PeakDev* peaks, int n_peaks,
                         int nz, long long nlat, int tied, const int* zrun, float* rsum, hipStream_t s) {
  k_runsum<<<dim3(nblk(nlat, 256)), dim3(256), 0, s>>>(u, chi, alpha, peaks, n_peaks, nz, nlat, tied, zrun, rsum);
  return hipGetLastError();
}

int frame_bound(int D, int f) {
  if (D == 32) return 32;
  if (f <= 48) return 48;
  if (f <= 64) return 64;
  return D;
}

// One translation unit per detector size instantiates the frame kernel (mpbp_frames_<D>.hip).
hipError_t frames_d32(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s);
hipError_t frames_d64(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s);
hipError_t frames_d96(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s);
hipError_t frames_d128(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s);
hipError_t frames_d192(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s);
hipError_t frames_d256(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s);
hipError_t frames_d150(int op, int fb, const FrameArgs* a, int lds_bytes, hipStream_t s);

static hipError_t frames_op(int op, int D, int FB, const FrameArgs* a, int lds_bytes, hipStream_t s) {
  switch (D) {
    case 32: return frames_d32(op, FB, a, lds_bytes, s);
    case 64: return frames_d64(op, FB, a, lds_bytes, s);
    case 96: return frames_d96(op, FB, a, lds_bytes, s);
    case 128: return frames_d128(op, FB, a, lds_bytes, s);
    case 192: return frames_d192(op, FB, a, lds_bytes, s);
    case 256: return frames_d256(op, FB, a, lds_bytes, s);
    case 150: return frames_d150(op, FB, a, lds_bytes, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_frames(int D, int FB, const FrameArgs& a, int lds_bytes, hipStream_t s) {
  return frames_op(0, D, FB, &a, lds_bytes, s);
}

bool frame_instance(int D, int FB) { return frames_op(2, D, FB, nullptr, 0, nullptr) == hipSuccess; }

hipError_t launch_project(int G, const FrameArgs& a, int lds_bytes, hipStream_t s) {
  if (a.mapz) return launch_project_map(a, s);
  const unsigned grid = a.xcd ? (unsigned)(((a.n_list + 7) / 8) * 8) : (unsigned)a.n_list;
  if (grid == 0) return hipSuccess;
#define MPBP_PROJ(g)                                                                          \
  case g:                                                                                     \
    if (a.probe3 && a.shw)                                                                    \
      k_project<g, true, true><<<dim3(grid), dim3(kFrameThreads), lds_bytes, s>>>(a);         \
    else if (a.probe3)                                                                        \
      k_project<g, true, false><<<dim3(grid), dim3(kFrameThreads), lds_bytes, s>>>(a);        \
    else if (a.shw)                                                                           \
      k_project<g, false, true><<<dim3(grid), dim3(kFrameThreads), lds_bytes, s>>>(a);        \
    else                                                                                      \
      k_project<g, false, false><<<dim3(grid), dim3(kFrameThreads), lds_bytes, s>>>(a);       \
    break;
  if (a.runs && !a.probe3 && !a.shw) {
    switch (G) {
      case 2: k_project_runs<2><<<dim3(grid), dim3(kFrameThreads), lds_bytes, s>>>(a); break;
      case 4: k_project_runs<4><<<dim3(grid), dim3(kFrameThreads), lds_bytes, s>>>(a); break;
      case 8: k_project_runs<8><<<dim3(grid), dim3(kFrameThreads), lds_bytes, s>>>(a); break;
      default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
  }
  switch (G) {
    MPBP_PROJ(2)
    MPBP_PROJ(4)
    MPBP_PROJ(8)
    default: return hipErrorInvalidValue;
  }
#undef MPBP_PROJ
  return hipGetLastError();
}

// the footprint accumulator (acc_pix pixels, a multiple of 4), then the per-slice offset
// and fraction tables
int project_lds_bytes(int np, int G, int nz, int acc_pix) {
  (void)np;
  (void)G;
  return acc_pix * (int)sizeof(cplx) + ((nz + 3) & ~3) * 4 + nz * 8;
}

static const int kDets[] = {32, 64, 96, 128, 150, 192, 256};

#define MPBP_GRAD_INSTANCES(X) X(1, 16) X(2, 16) X(4, 16) X(1, 8) X(2, 8) X(4, 8)
#define MPBP_GRAD_RUN_INSTANCES(X) X(4, 16) X(8, 16) X(16, 16) X(4, 8) X(8, 8) X(16, 8)

template <int B, int TX, bool P3, bool LIN>
static hipError_t grad_set_lds() {
  return hipFuncSetAttribute((const void*)k_grad<B, TX, P3, LIN>, hipFuncAttributeMaxDynamicSharedMemorySize,
                             160 * 1024);
}

hipError_t prepare_kernels() {
  hipError_t e = hipSuccess;
  for (int D : kDets)
    for (int FB : {32, 48, 64, D})
      if (e == hipSuccess && frame_instance(D, FB)) e = frames_op(1, D, FB, nullptr, 0, nullptr);
  const void* projs[] = {
      (const void*)k_project<2, false, false>, (const void*)k_project<4, false, false>,
      (const void*)k_project<8, false, false>, (const void*)k_project<2, true, false>,
      (const void*)k_project<4, true, false>,  (const void*)k_project<8, true, false>,
      (const void*)k_project<2, false, true>,  (const void*)k_project<4, false, true>,
      (const void*)k_project<8, false, true>,  (const void*)k_project<2, true, true>,
      (const void*)k_project<4, true, true>,   (const void*)k_project<8, true, true>,
      (const void*)k_project_runs<2>,          (const void*)k_project_runs<4>,
      (const void*)k_project_runs<8>};
  for (const void* f : projs)
    if (e == hipSuccess) e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024);
#define MPBP_CASE(b, tx)                                                                        \
  if (e == hipSuccess)                                                                          \
    e = grad_set_lds<b, tx, false, false>();                                                    \
  if (e == hipSuccess) e = grad_set_lds<b, tx, true, false>();                                  \
  if (e == hipSuccess) e = grad_set_lds<b, tx, false, true>();                                  \
  if (e == hipSuccess) e = grad_set_lds<b, tx, true, true>();
  MPBP_GRAD_INSTANCES(MPBP_CASE)
#undef MPBP_CASE
#define MPBP_CASE(b, tx)                                                                                   \
  if (e == hipSuccess)                                                                                     \
    e = hipFuncSetAttribute((const void*)k_bp_gather<b, tx>, hipFuncAttributeMaxDynamicSharedMemorySize,  \
                            160 * 1024);
  MPBP_GRAD_RUN_INSTANCES(MPBP_CASE)
#undef MPBP_CASE
  if (e == hipSuccess) e = prepare_map_kernels();
  return e;
}

bool grad_uses_runs(const GradArgs& a) { return a.runs && !a.probe3 && !a.shw && !a.mapz; }

int grad_partials(const GradArgs& a) {
  if (!grad_uses_runs(a) && !a.mapz) return a.tiles_x * a.tiles_y;
  return (int)nblk(a.tied ? a.nlat : a.nlat * ((a.nz + kBpZ - 1) / kBpZ), kBpThreads);
}

int grad_effective_batch(int batch, bool runs) {
  return runs ? std::min(std::max(batch, 4), 16) : std::min(batch, 4);
}

hipError_t launch_bp_chain(const GradArgs& a, hipStream_t s) {
  k_bp_chain<<<dim3(grad_partials(a)), dim3(kBpThreads), 0, s>>>(a);
  return hipGetLastError();
}

hipError_t launch_grad(int batch, int tile_x, const GradArgs& a, int lds_bytes, hipStream_t s) {
  if (a.mapz) return launch_grad_map(a, s);
  const unsigned grid = (unsigned)(((a.tiles_x * a.tiles_y + 7) / 8) * 8);
  if (grad_uses_runs(a)) {
    const int b = grad_effective_batch(batch, true);
    const unsigned ggrid = (unsigned)(((a.tiles_x * a.tiles_y * a.n_peaks + 7) / 8) * 8);
    hipError_t e = hipErrorInvalidValue;
#define MPBP_CASE(bb, tx)                                                                     \
    if (b == bb && tile_x == tx) {                                                            \
      k_bp_gather<bb, tx><<<dim3(ggrid), dim3(kBpThreads), lds_bytes, s>>>(a);                \
      e = hipGetLastError();                                                                  \
    }
    MPBP_GRAD_RUN_INSTANCES(MPBP_CASE)
#undef MPBP_CASE
    if (e != hipSuccess) return e;
    return launch_bp_chain(a, s);
  }
  batch = grad_effective_batch(batch, false);
#define MPBP_CASE(b, tx)                                                       \
  if (batch == b && tile_x == tx) {                                            \
    if (a.probe3 && a.shw)                                                              \
      k_grad<b, tx, true, true><<<dim3(grid), dim3(kGradThreads), lds_bytes, s>>>(a);     \
    else if (a.probe3)                                                                  \
      k_grad<b, tx, true, false><<<dim3(grid), dim3(kGradThreads), lds_bytes, s>>>(a);    \
    else if (a.shw)                                                                     \
      k_grad<b, tx, false, true><<<dim3(grid), dim3(kGradThreads), lds_bytes, s>>>(a);    \
    else                                                                                \
      k_grad<b, tx, false, false><<<dim3(grid), dim3(kGradThreads), lds_bytes, s>>>(a);   \
    return hipGetLastError();                                                  \
  }
  MPBP_GRAD_INSTANCES(MPBP_CASE)
#undef MPBP_CASE
  return hipErrorInvalidValue;
}

hipError_t launch_finalize(const double* floss, const int* out_list, int n_out, double* loss,
                           float* frame_loss, const double* apart, int n_part, int n_peaks,
                           float* grad_alpha, hipStream_t s) {
  k_finalize<<<dim3(1), dim3(kFinThreads), 0, s>>>(floss, out_list, n_out, loss, frame_loss, apart, n_part, n_peaks, grad_alpha);
  return hipGetLastError();
}

hipError_t launch_step(float* p, const float* g, long long n, float eta, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_step<<<dim3(nblk(n, 256)), dim3(256), 0, s>>>(p, g, n, eta);
  return hipGetLastError();
}

hipError_t launch_adam(float* p, float* x, float* m, float* v, const float* g, long long n, float lr,
                       float b1, float b2, float eps, float c1, float c2, int log_mode, int project,
                       long long fixed, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_adam<<<dim3(nblk(n, 256)), dim3(256), 0, s>>>(p, x, m, v, g, n, lr, b1, b2, eps, c1, c2, log_mode, project,
                                                  fixed);
  return hipGetLastError();
}

hipError_t launch_exp(float* x, const float* xlog, long long n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_exp<<<dim3(nblk(n, 256)), dim3(256), 0, s>>>(x, xlog, n);
  return hipGetLastError();
}

hipError_t launch_fill(float* p, long long n, float v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  k_fill_f32<<<dim3(nblk(n, 256)), dim3(256), 0, s>>>(p, n, v);
  return hipGetLastError();
}

hipError_t launch_norm2(const float* a, long long n, double* part, int max_part, double* out, hipStream_t s) {
  const int nb = (int)std::min<long long>(std::max<long long>(nblk(n, 256), 1), max_part);
  k_norm2_part<<<dim3(nb), dim3(256), 0, s>>>(a, n, part);
  k_norm2_final<<<dim3(1), dim3(256), 0, s>>>(part, nb, out);
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
static int lds_for(int fy, int fx, int fxp, bool grad) {
  using RC = LineCfg<D>;
  constexpr int L = ColLen<D>::L;
  constexpr int RLINES = kFrameThreads / RC::TPL;
  constexpr int EXL = RC::Q * (RC::P + 1);
  const long long exch = (RLINES * EXL + 1) / 2;
  (void)fx;
  (void)grad;   // the exit wave and its gradient stay in the slots
  const long long cpx = D + L + (long long)(D / L) * fy + (long long)L * fxp + L / 8 + exch;
  return (int)(cpx * 8);
}

int frame_lds_bytes(int D, int fy, int fx, int fxp, bool grad) {
  switch (D) {
    case 32: return lds_for<32>(fy, fx, fxp, grad);
    case 64: return lds_for<64>(fy, fx, fxp, grad);
    case 96: return lds_for<96>(fy, fx, fxp, grad);
    case 128: return lds_for<128>(fy, fx, fxp, grad);
    case 192: return lds_for<192>(fy, fx, fxp, grad);
    case 256: return lds_for<256>(fy, fx, fxp, grad);
    case 150: return lds_for<150>(fy, fx, fxp, grad);
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
    case 150: twiddles_for<150>(fy, out); return true;
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
    case 150: return ColLen<150>::L;
    default: return -1;
  }
}

int grad_lds_bytes(int np, int nz, int maxspan_y, int maxspan_x, int max_cand, bool tied, bool runs) {
  (void)maxspan_y;
  (void)maxspan_x;
  if (runs)   // k_bp_gather: the probe, the frame list, its length
    return np * np * 8 + max_cand * (int)sizeof(GradCand) + 16;
  return np * np * 8 + nz * 8 + kMaxPeaksDev * 8 + 64 + ((max_cand + 15) & ~15) +
         (tied ? 4 * kGradThreads * 4 : 0);
}

}  // namespace mpbp
