// mpbp_plain.hip - the plain path: for every listed frame, separate launches for the
// projection, the two 1D passes of the forward DFT, the modulus residual, the two
// passes of the inverse DFT and the back-projection, with the D x D exit wave in device
// memory.  Line transforms are mixed-radix (2, 3, 5) Stockham FFTs in LDS (Govindaraju
// et al., SC 2008), one workgroup per line.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "mpbp_dft.hpp"
#include "mpbp_launch.hpp"
#include "mpbp_plain.hpp"
#include "mpbp_phase.hpp"

namespace mpbp {

__global__ __launch_bounds__(256) void k_pl_project(const float* __restrict__ obj,
                                                    const float* __restrict__ probe,
                                                    const int* __restrict__ shear,
                                                    const PeakDev* __restrict__ peaks, int m, int py,
                                                    int px, int nz, int ny, int nx, int np, int probe3,
                                                    const float* __restrict__ shw,
                                                    float* __restrict__ psi) {
  const PeakDev pk = peaks[m];
  const int D = pk.D;
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= D * D) return;
  const int wy = p / D, wx = p - wy * D;
  const cplx* O = reinterpret_cast<const cplx*>(obj) + (long long)m * nz * ny * nx;
  const long long pz = probe3 ? (long long)np * np : 0;   // probe slice stride
  const cplx* P0 = reinterpret_cast<const cplx*>(probe) + (long long)m * (probe3 ? nz : 1) * np * np;
  cplx acc = {0.f, 0.f};
  for (int z = 0; z < nz; ++z) {
    const cplx* P = P0 + z * pz;
    // taps (dy, dx): one of weight 1 for rounded offsets, four bilinear ones otherwise
    const float ry = shw ? shw[2 * (m * nz + z)] : 0.f, rx = shw ? shw[2 * (m * nz + z) + 1] : 0.f;
    for (int tp = 0; tp < (shw ? 4 : 1); ++tp) {
      const int dy = tp >> 1, dx = tp & 1;
      const float wt = (dy ? ry : 1.f - ry) * (dx ? rx : 1.f - rx);
      const int a = wy - pk.c - shear[2 * (m * nz + z)] - dy;
      const int b = wx - pk.c - shear[2 * (m * nz + z) + 1] - dx;
      if ((unsigned)a < (unsigned)np && (unsigned)b < (unsigned)np) {
        const int oy = py + a, ox = px + b;
        if ((unsigned)oy < (unsigned)ny && (unsigned)ox < (unsigned)nx) {
          const cplx t = cmul(P[a * np + b], O[((long long)z * ny + oy) * nx + ox]);
          acc = cadd(acc, shw ? cscale(t, wt) : t);
        }
      }
    }
  }
  reinterpret_cast<cplx*>(psi)[p] = acc;
}

// One line of D points per workgroup: x[line * line_stride + i * elem_stride].
__global__ __launch_bounds__(256) void k_pl_fft(float* __restrict__ buf, int D, int line_stride,
                                                int elem_stride, int inv) {
  __shared__ cplx a[256], b[256];
  cplx* base = reinterpret_cast<cplx*>(buf) + (long long)blockIdx.x * line_stride;
  const int tid = threadIdx.x;
  for (int i = tid; i < D; i += blockDim.x) a[i] = base[(long long)i * elem_stride];
  __syncthreads();
  cplx* src = a;
  cplx* dst = b;
  int rem = D;
  for (int ns = 1; ns < D;) {
    const int R = (rem % 5 == 0) ? 5 : (rem % 3 == 0) ? 3 : 2;
    const int nb = D / R;
    for (int j = tid; j < nb; j += blockDim.x) {
      const int k = j % ns;
      cplx v[5];
      for (int r = 0; r < R; ++r) {
        cplx x = src[j + r * nb];
        double s, c;
        sincospi((inv ? 2.0 : -2.0) * (double)(k * r) / (double)(ns * R), &s, &c);
        v[r] = cmul(x, cplx{(float)c, (float)s});
      }
      if (R == 5) {
        if (inv) DFT<5, true>::run(v); else DFT<5, false>::run(v);
      } else if (R == 3) {
        if (inv) DFT<3, true>::run(v); else DFT<3, false>::run(v);
      } else {
        DFT<2, false>::run(v);
      }
      const int d0 = (j / ns) * ns * R + k;
      for (int r = 0; r < R; ++r) dst[d0 + r * ns] = v[r];
    }
    __syncthreads();
    cplx* t = src;
    src = dst;
    dst = t;
    ns *= R;
    rem /= R;
  }
  for (int i = tid; i < D; i += blockDim.x) base[(long long)i * elem_stride] = src[i];
}

// Modulus residual of eq. (4) on one frame, in place; per-row loss partials.
__global__ __launch_bounds__(256) void k_pl_residual(float* __restrict__ psi,
                                                     const float* __restrict__ y,
                                                     const float* __restrict__ bg, int D,
                                                     double* __restrict__ lpart,
                                                     float* __restrict__ mi, int grad) {
  __shared__ double red[256];
  const int row = blockIdx.x, tid = threadIdx.x;
  const float invD = 1.0f / (float)D;
  double s = 0.0;
  for (int c = tid; c < D; c += blockDim.x) {
    cplx* X = reinterpret_cast<cplx*>(psi) + (long long)row * D + c;
    float a2 = (X->x * X->x + X->y * X->y) * invD * invD;   // model intensity of eq. (2)
    if (bg) a2 += bg[(long long)row * D + c];
    if (mi) mi[(long long)row * D + c] = a2;
    if (y) {
      const float A = sqrtf(a2);
      const float r = A - sqrtf(y[(long long)row * D + c]);
      s += 0.5 * (double)r * (double)r;
      if (grad) {
        const float coef = A > 0.f ? r / A * invD : 0.f;
        *X = cscale(*X, coef);
      }
    }
  }
  red[tid] = s;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if (tid < w) red[tid] += red[tid + w];
    __syncthreads();
  }
  if (tid == 0) lpart[row] = red[0];
}

__global__ void k_pl_sum(const double* __restrict__ lpart, int n, double* out) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    double s = 0.0;
    for (int i = 0; i < n; ++i) s += lpart[i];
    *out = s;
  }
}

// Adjoint of the projection for one frame: g_O[z, py+a, px+b] += conj(P) g_psi / D.
__global__ __launch_bounds__(256) void k_pl_backproject(const float* __restrict__ psi,
                                                        const float* __restrict__ probe,
                                                        const int* __restrict__ shear,
                                                        const PeakDev* __restrict__ peaks, int m,
                                                        int py, int px, int nz, int ny, int nx,
                                                        int np, int probe3, const float* __restrict__ shw,
                                                        float* __restrict__ gobj) {
  const PeakDev pk = peaks[m];
  const int D = pk.D;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nz * np * np) return;
  const int z = i / (np * np);
  const int ab = i - z * np * np;
  const int a = ab / np, b = ab - a * np;
  const int oy = py + a, ox = px + b;
  if ((unsigned)oy >= (unsigned)ny || (unsigned)ox >= (unsigned)nx) return;
  const int wy = a + pk.c + shear[2 * (m * nz + z)];
  const int wx = b + pk.c + shear[2 * (m * nz + z) + 1];
  const cplx* ps = reinterpret_cast<const cplx*>(psi);
  cplx g = ps[wy * D + wx];
  if (shw) {   // the adjoint of the four bilinear taps
    const float ry = shw[2 * (m * nz + z)], rx = shw[2 * (m * nz + z) + 1];
    g = cadd(cadd(cscale(g, (1.f - ry) * (1.f - rx)), cscale(ps[wy * D + wx + 1], (1.f - ry) * rx)),
             cadd(cscale(ps[(wy + 1) * D + wx], ry * (1.f - rx)), cscale(ps[(wy + 1) * D + wx + 1], ry * rx)));
  }
  const cplx p = reinterpret_cast<const cplx*>(probe)[((long long)m * (probe3 ? nz : 1) + (probe3 ? z : 0)) * np * np + ab];
  cplx* dst = reinterpret_cast<cplx*>(gobj) + (long long)m * nz * ny * nx + ((long long)z * ny + oy) * nx + ox;
  const float invD = 1.0f / (float)D;
  *dst = cadd(*dst, cscale(cmulc(g, p), invD));
}

__global__ __launch_bounds__(256) void k_pl_zero(float* __restrict__ p, long long n) {
  long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.f;
}

// Chain rule from g_O,m to df/du, df/dchi and per-block df/dalpha partials.  One
// thread per voxel, or (tied = ny * nx) per lateral pixel, summing over the slices.
__global__ __launch_bounds__(256) void k_pl_chain(const float* __restrict__ gobj,
                                                  const float* __restrict__ u,
                                                  const float* __restrict__ chi,
                                                  const float* __restrict__ alpha,
                                                  const PeakDev* __restrict__ peaks, int M,
                                                  long long nvox, long long tied,
                                                  float* __restrict__ grad_u,
                                                  float* __restrict__ grad_chi,
                                                  double* __restrict__ apart) {
  __shared__ double red[256];
  const long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int tid = threadIdx.x;
  const long long nf = tied ? tied : nvox;      // field elements (and component stride)
  const long long nslices = tied ? nvox / tied : 1;
  const bool on = v < nf;
  float gx = 0.f, gy = 0.f, gz = 0.f, gc = 0.f;
  float ux = 0.f, uy = 0.f, uz = 0.f, ch = 0.f;
  if (on) {
    ux = u[v]; uy = u[nf + v]; uz = u[2 * nf + v]; ch = chi[v];
  }
  for (int m = 0; m < M; ++m) {
    double ap = 0.0;
    if (on) {
      const PeakDev pk = peaks[m];
      const float phi = fmaf(pk.gz, uz, fmaf(pk.gy, uy, pk.gx * ux));   // as k_object
      float s, c;
      phase_sincos(phi, s, c);
      const float al = alpha[m];
      for (long long k = 0; k < nslices; ++k) {
        const cplx g = reinterpret_cast<const cplx*>(gobj)[(long long)m * nvox + k * nf + v];
        const float re = g.x * c + g.y * s;
        const float dphi = al * ch * (g.y * c - g.x * s);
        gx += pk.gx * dphi;
        gy += pk.gy * dphi;
        gz += pk.gz * dphi;
        gc += al * re;
        ap += (double)(ch * re);
      }
    }
    red[tid] = ap;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if (tid < w) red[tid] += red[tid + w];
      __syncthreads();
    }
    if (tid == 0) apart[(long long)blockIdx.x * M + m] = red[0];
    __syncthreads();
  }
  if (on) {
    grad_u[v] = gx;
    grad_u[nf + v] = gy;
    grad_u[2 * nf + v] = gz;
    grad_chi[v] = gc;
  }
}

void plain_free(PlainWork* w) {
  if (w->device >= 0) {
    (void)hipFree(w->psi);
    (void)hipFree(w->gobj);
    (void)hipFree(w->lpart);
    (void)hipFree(w->apart);
  }
  *w = PlainWork{};
}

static hipError_t plain_ensure(PlainWork* w, const PeakDev* hp, int M, long long nvox, bool grad) {
  int dmax = 0;
  for (int m = 0; m < M; ++m) dmax = std::max(dmax, hp[m].D);
  hipError_t e = hipSuccess;
  int dev = 0;
  (void)hipGetDevice(&dev);
  w->device = dev;
  if (w->dmax < dmax) {
    (void)hipFree(w->psi);
    (void)hipFree(w->lpart);
    e = hipMalloc((void**)&w->psi, (size_t)dmax * dmax * 8);
    if (e == hipSuccess) e = hipMalloc((void**)&w->lpart, (size_t)dmax * sizeof(double));
    if (e != hipSuccess) return e;
    w->dmax = dmax;
  }
  if (grad && w->gobj_len < (long long)M * nvox) {
    (void)hipFree(w->gobj);
    (void)hipFree(w->apart);
    e = hipMalloc((void**)&w->gobj, (size_t)M * nvox * 8);
    long long nb = (nvox + 255) / 256;
    if (e == hipSuccess) e = hipMalloc((void**)&w->apart, (size_t)nb * M * sizeof(double));
    if (e != hipSuccess) return e;
    w->gobj_len = (long long)M * nvox;
    w->apart_len = nb * M;
  }
  return e;
}

static hipError_t plain_frames(PlainWork* w, const PeakDev* hp, const PeakDev* dp, int nz, int ny,
                               int nx, int np, const int* dshear, const int32_t* hscan,
                               const int32_t* hpeak_of, const int32_t* frames, int n,
                               const float* probe, const float* y, float* mi, const float* obj,
                               double* floss, bool grad, hipStream_t s) {
  for (int i = 0; i < n; ++i) {
    const int fid = frames ? frames[i] : i;
    const int m = hpeak_of[fid];
    const PeakDev& pk = hp[m];
    const int D = pk.D;
    const int py = hscan[2 * fid], px = hscan[2 * fid + 1];
    const long long yo = pk.y_off + (long long)(fid - pk.frame_base) * D * D;
    k_pl_project<<<dim3((D * D + 255) / 256), dim3(256), 0, s>>>(obj, probe, dshear, dp, m, py, px, nz, ny, nx, np,
                                                                 w->probe3, w->shw, w->psi);
    k_pl_fft<<<dim3(D), dim3(128), 0, s>>>(w->psi, D, D, 1, 0);
    k_pl_fft<<<dim3(D), dim3(128), 0, s>>>(w->psi, D, 1, D, 0);
    k_pl_residual<<<dim3(D), dim3(256), 0, s>>>(w->psi, y ? y + yo : nullptr, w->bg ? w->bg + yo : nullptr, D,
                                                 w->lpart, mi ? mi + yo : nullptr, grad ? 1 : 0);
    if (y) k_pl_sum<<<dim3(1), dim3(64), 0, s>>>(w->lpart, D, floss + fid);
    if (grad) {
      k_pl_fft<<<dim3(D), dim3(128), 0, s>>>(w->psi, D, D, 1, 1);
      k_pl_fft<<<dim3(D), dim3(128), 0, s>>>(w->psi, D, 1, D, 1);
      k_pl_backproject<<<dim3((nz * np * np + 255) / 256), dim3(256), 0, s>>>(w->psi, probe, dshear, dp, m, py, px, nz,
                                                                              ny, nx, np, w->probe3, w->shw, w->gobj);
    }
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t plain_forward(PlainWork* w, const PeakDev* hpeaks, const PeakDev* dpeaks, int M, int nz,
                         int ny, int nx, int np, const int* dshear, const int32_t* hscan,
                         const int32_t* hpeak_of, const int32_t* frames, int n, const float* u,
                         const float* chi, const float* alpha, const float* probe, const float* y,
                         float* mi, float* obj, double* floss, long long tied, hipStream_t s) {
  const long long nvox = (long long)nz * ny * nx;
  hipError_t e = plain_ensure(w, hpeaks, M, nvox, false);
  if (e != hipSuccess) return e;
  e = launch_object(u, chi, alpha, dpeaks, M, nvox, tied, obj, s);
  if (e != hipSuccess) return e;
  return plain_frames(w, hpeaks, dpeaks, nz, ny, nx, np, dshear, hscan, hpeak_of, frames, n, probe, y,
                      mi, obj, floss, false, s);
}

hipError_t plain_loss_grad(PlainWork* w, const PeakDev* hpeaks, const PeakDev* dpeaks, int M, int nz,
                           int ny, int nx, int np, const int* dshear, const int32_t* hscan,
                           const int32_t* hpeak_of, const int32_t* frames, int n, const float* u,
                           const float* chi, const float* alpha, const float* probe, const float* y,
                           float* obj, double* floss, float* grad_u, float* grad_chi,
                           const double** apart, int* n_part, long long tied, hipStream_t s) {
  const long long nvox = (long long)nz * ny * nx;
  hipError_t e = plain_ensure(w, hpeaks, M, nvox, true);
  if (e != hipSuccess) return e;
  e = launch_object(u, chi, alpha, dpeaks, M, nvox, tied, obj, s);
  if (e != hipSuccess) return e;
  k_pl_zero<<<dim3((unsigned)((2 * M * nvox + 255) / 256)), dim3(256), 0, s>>>(w->gobj, 2 * M * nvox);
  e = plain_frames(w, hpeaks, dpeaks, nz, ny, nx, np, dshear, hscan, hpeak_of, frames, n, probe, y,
                   nullptr, obj, floss, true, s);
  if (e != hipSuccess) return e;
  const unsigned nb = (unsigned)(((tied ? tied : nvox) + 255) / 256);
  k_pl_chain<<<dim3(nb), dim3(256), 0, s>>>(w->gobj, u, chi, alpha, dpeaks, M, nvox, tied, grad_u, grad_chi,
                                            w->apart);
  *apart = w->apart;
  *n_part = (int)nb;
  return hipGetLastError();
}

}  // namespace mpbp
