// mpbp_unwrap.hip - the phase-unwrap projector Pi_U of eq. (10) (section 3.3, the last
// step of each iteration of Algorithm 1) on the GPU.
//
// Phase maps Phi_m = G_m . u (eq. (9)), one map per peak m and slice s, are wrapped and
// unwrapped in 2D by reliability-guided merging (Herraez et al., Appl. Opt. 41, 7437,
// 2002): pixel reliability 1/D from the second differences of the wrapped phase, edges
// between 4-neighbours ranked by the summed reliability of their two pixels, groups
// joined from the most reliable edge down.  The groups a sequential pass joins are the
// edges of the maximum spanning tree of that (total) edge order, and the unwrapped
// phase is the wrapped phase integrated along that tree.  The tree is unique, so it is
// built here in parallel by Boruvka rounds: every component takes its best outgoing
// edge and hooks onto the component across it.  Each pixel carries its wrap count
// relative to its component's root (a weighted union-find): hooking root a onto root b
// records n(a) - n(b), and a walk from every pixel to its new root sums those offsets.
//
// Every float decision (wrap counts, reliabilities, edge keys) is taken in float32 with
// each operation rounded separately in a fixed order (no contraction), so the integer
// results are those of any implementation that follows the same steps.
//
// Layout: map g = m * S + s (S = nz, or 1 for fields tied along z), pixel i = y * nx + x;
// per-map arrays are [nmaps][ny * nx].  Parent indices are local to the map.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mpbp_unwrap.hpp"

#pragma clang fp contract(off)

namespace mpbp {

namespace {

constexpr float kTwoPi = 6.28318530717958647692f;
constexpr int kUwThreads = 256;
constexpr int kHookSlots = 64;     // per-round "a root hooked" flags, one per block mod 64

// True if round r hooked anything (any of its flag slots set).
__device__ __forceinline__ bool round_hooked(const int* hooks, int r) {
  const int* h = hooks + r * kHookSlots;
  int any = 0;
#pragma unroll 8
  for (int k = 0; k < kHookSlots; ++k) any |= h[k];
  return any != 0;
}

// atomicMax, skipped when the slot already holds a key at least as large (keys only
// grow during a launch, so a stale read can only cause an unneeded atomic)
__device__ __forceinline__ void offer(unsigned long long* slot, unsigned long long k) {
  if (*(volatile unsigned long long*)slot < k) atomicMax(slot, k);
}

// MurmurHash3's 32-bit finalizer and its inverse (every step is a bijection): the
// tie-break of equal edge keys.
__host__ __device__ constexpr uint32_t fmix32(uint32_t x) {
  x ^= x >> 16;
  x *= 0x85ebca6bu;
  x ^= x >> 13;
  x *= 0xc2b2ae35u;
  x ^= x >> 16;
  return x;
}
// Multiplicative inverse of an odd number modulo 2^32 (Newton's iteration).
__host__ __device__ constexpr uint32_t inv_odd(uint32_t a) {
  uint32_t x = a;                  // correct to 3 bits
  for (int i = 0; i < 5; ++i) x *= 2u - a * x;
  return x;
}
__host__ __device__ constexpr uint32_t fmix32_inv(uint32_t x) {
  x ^= x >> 16;
  x *= inv_odd(0xc2b2ae35u);
  x ^= (x >> 13) ^ (x >> 26);
  x *= inv_odd(0x85ebca6bu);
  x ^= x >> 16;
  return x;
}
static_assert(fmix32_inv(fmix32(0u)) == 0u, "fmix32 inverse");
static_assert(fmix32_inv(fmix32(1u)) == 1u, "fmix32 inverse");
static_assert(fmix32_inv(fmix32(123456789u)) == 123456789u, "fmix32 inverse");
static_assert(fmix32_inv(fmix32(0xfffffffeu)) == 0xfffffffeu, "fmix32 inverse");
static_assert(fmix32(fmix32_inv(0xdeadbeefu)) == 0xdeadbeefu, "fmix32 inverse");

// Wrap: psi = phi - 2 pi rint(phi / 2 pi); the rint (halves to even) is returned in q.
__device__ __forceinline__ float wrap_phase(float phi, float* q) {
  const float qf = rintf(phi / kTwoPi);
  *q = qf;
  return phi - qf * kTwoPi;
}
__device__ __forceinline__ float gamma(float d) {
  float q;
  return wrap_phase(d, &q);
}

// Edge key of a map: ((bits of the summed reliability) + 1) << 32 | ~fmix32(edge): the
// larger key is the more reliable edge, equal sums go to the smaller hash.  Never 0.
__device__ __forceinline__ unsigned long long edge_key(float rsum, uint32_t e) {
  return ((unsigned long long)(__float_as_uint(rsum) + 1u) << 32) | (unsigned long long)(~fmix32(e));
}

__device__ __forceinline__ void edge_ends(uint32_t e, int ny, int nx, int* p, int* q) {
  const uint32_t nh = (uint32_t)ny * (uint32_t)(nx - 1);
  if (e < nh) {
    const int row = (int)(e / (uint32_t)(nx - 1)), col = (int)(e - (uint32_t)row * (uint32_t)(nx - 1));
    *p = row * nx + col;
    *q = *p + 1;
  } else {
    *p = (int)(e - nh);
    *q = *p + nx;
  }
}

// ---- phases, wrap, and the union-find state of every map pixel ----
__global__ __launch_bounds__(kUwThreads) void k_uw_wrap(const float* __restrict__ u, UnwrapArgs A) {
  const long long t = (long long)blockIdx.x * kUwThreads + threadIdx.x;
  if (t < (long long)A.rounds * kHookSlots) A.hooks[t] = 0;
  if (t < A.nmaps) A.sums[t] = 0;
  if (t == 0) *A.err = 0;
  const long long lat = (long long)A.S * A.np;   // pixels of one component of u
  if (t >= lat) return;
  const int s = (int)(t / A.np);
  const int i = (int)(t - (long long)s * A.np);
  const float u0 = u[t], u1 = u[lat + t], u2 = u[2 * lat + t];
  for (int m = 0; m < A.M; ++m) {
    const float phi = (A.g[m][0] * u0 + A.g[m][1] * u1) + A.g[m][2] * u2;
    float qf;
    const float psi = wrap_phase(phi, &qf);
    const long long x = (long long)(m * A.S + s) * A.np + i;
    A.psi[x] = psi;
    A.q[x] = (int)qf;
    A.par[x] = i;
    A.pot[x] = 0;
    A.hk[x] = i;
    A.hpot[x] = 0;
    A.best[x] = 0ull;
  }
}

// ---- reliability: 1 / sqrt(H^2 + V^2 + D1^2 + D2^2); 0 on the border ----
__global__ __launch_bounds__(kUwThreads) void k_uw_reliability(UnwrapArgs A) {
  const long long x = (long long)blockIdx.x * kUwThreads + threadIdx.x;
  if (x >= A.npix) return;
  const long long g = x / A.np;
  const int i = (int)(x - g * A.np);
  const int row = i / A.nx, col = i - (i / A.nx) * A.nx;
  if (row == 0 || col == 0 || row == A.ny - 1 || col == A.nx - 1) {
    A.rel[x] = 0.f;
    return;
  }
  const float* p = A.psi + x;
  const int w = A.nx;
  const float c = p[0];
  auto second = [&](float a, float b) { return gamma(a - c) - gamma(c - b); };
  const float H = second(p[-1], p[1]);
  const float V = second(p[-w], p[w]);
  const float D1 = second(p[-w - 1], p[w + 1]);
  const float D2 = second(p[-w + 1], p[w - 1]);
  const float s2 = ((H * H + V * V) + D1 * D1) + D2 * D2;
  A.rel[x] = 1.0f / sqrtf(s2);
}

// ---- Boruvka round r: every root collects its best outgoing edge ----
__global__ __launch_bounds__(kUwThreads) void k_uw_best(UnwrapArgs A, int r) {
  if (r > 0 && !round_hooked(A.hooks, r - 1)) return;
  const long long x = (long long)blockIdx.x * kUwThreads + threadIdx.x;
  if (x >= A.npix) return;
  const long long g = x / A.np;
  const long long base = g * A.np;
  const int i = (int)(x - base);
  const int row = i / A.nx, col = i - (i / A.nx) * A.nx;
  const int rx = A.par[x];
  const float relx = A.rel[x];
  if (col < A.nx - 1) {
    const int ry = A.par[x + 1];
    if (ry != rx) {
      const uint32_t e = (uint32_t)row * (uint32_t)(A.nx - 1) + (uint32_t)col;
      const unsigned long long k = edge_key(relx + A.rel[x + 1], e);
      offer(A.best + base + rx, k);
      offer(A.best + base + ry, k);
    }
  }
  if (row < A.ny - 1) {
    const int ry = A.par[x + A.nx];
    if (ry != rx) {
      const uint32_t e = (uint32_t)A.ny * (uint32_t)(A.nx - 1) + (uint32_t)i;
      const unsigned long long k = edge_key(relx + A.rel[x + A.nx], e);
      offer(A.best + base + rx, k);
      offer(A.best + base + ry, k);
    }
  }
}

// ---- Boruvka round r: every root hooks onto the root across its best edge ----
// Two roots that chose the same edge would hook onto each other; the smaller index stays
// a root.  With a total edge order no other cycle can form.
__global__ __launch_bounds__(kUwThreads) void k_uw_hook(UnwrapArgs A, int r) {
  if (r > 0 && !round_hooked(A.hooks, r - 1)) return;
  const long long x = (long long)blockIdx.x * kUwThreads + threadIdx.x;
  bool hooked = false;
  if (x < A.npix) {
    const long long g = x / A.np;
    const long long base = g * A.np;
    const int i = (int)(x - base);
    const unsigned long long k = A.best[x];
    if (A.par[x] == i && k != 0ull) {
      const uint32_t e = fmix32_inv(~(uint32_t)(k & 0xffffffffull));
      const uint32_t n_edges = (uint32_t)A.ny * (uint32_t)(A.nx - 1) + (uint32_t)(A.ny - 1) * (uint32_t)A.nx;
      int p = 0, q = 0;
      if (e < n_edges) edge_ends(e, A.ny, A.nx, &p, &q);
      const int rp = A.par[base + p], rq = A.par[base + q];
      if (e >= n_edges) {
        *A.err = 3;               // not an edge of this map
      } else if (rp != i && rq != i) {
        *A.err = 1;               // the best edge of a root must touch its component
      } else {
        const int other = rp == i ? rq : rp;
        if (!(A.best[base + other] == k && i < other)) {
          // wrap count of the edge: the unwrapped phase steps by psi_q - psi_p - 2 pi w
          const float d = A.psi[base + q] - A.psi[base + p];
          const int w = (int)rintf(d / kTwoPi);
          const int pp = A.pot[base + p], pq = A.pot[base + q];
          A.hk[x] = other;
          A.hpot[x] = rp == i ? pq - pp + w : pp - pq - w;   // n(this root) - n(other)
          hooked = true;
        }
      }
    }
  }
  // one flag store per block that hooked, spread over the round's slots
  if (__syncthreads_or(hooked) && threadIdx.x == 0) A.hooks[r * kHookSlots + (blockIdx.x & (kHookSlots - 1))] = 1;
}

// ---- Boruvka round r: every pixel walks to its new root, summing the offsets ----
__global__ __launch_bounds__(kUwThreads) void k_uw_walk(UnwrapArgs A, int r) {
  if (!round_hooked(A.hooks, r)) return;
  const long long x = (long long)blockIdx.x * kUwThreads + threadIdx.x;
  if (x >= A.npix) return;
  const long long base = (x / A.np) * A.np;
  A.best[x] = 0ull;
  int cur = A.par[x];
  int acc = A.pot[x];
  for (long long step = 0;; ++step) {
    const int nxt = A.hk[base + cur];
    if (nxt == cur) break;
    if (step >= A.np) {           // longer than the map: a cycle (never with a total order)
      *A.err = 2;
      break;
    }
    acc += A.hpot[base + cur];
    cur = nxt;
  }
  A.par[x] = cur;
  A.pot[x] = acc;
}

// ---- per map: sum of (q - n), n the wrap count relative to the map's root ----
__global__ __launch_bounds__(kUwThreads) void k_uw_sum(UnwrapArgs A) {
  __shared__ long long red[kUwThreads / 64];
  const long long g = blockIdx.y;
  const long long base = g * A.np;
  long long s = 0;
  for (long long i = (long long)blockIdx.x * kUwThreads + threadIdx.x; i < A.np;
       i += (long long)gridDim.x * kUwThreads)
    s += (long long)A.q[base + i] - (long long)A.pot[base + i];
  for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    long long t = 0;
    for (int w = 0; w < kUwThreads / 64; ++w) t += red[w];
    atomicAdd((unsigned long long*)(A.sums + g), (unsigned long long)t);
  }
}

// floor((2 s + n) / (2 n)) for n > 0: the mean s / n rounded, halves up
__device__ __forceinline__ long long round_mean(long long s, long long n) {
  const long long a = 2 * s + n, b = 2 * n;
  long long qv = a / b;
  if ((a % b != 0) && (a < 0)) --qv;
  return qv;
}

// ---- N = n + k - q per map pixel, and u += 2 pi sum_m N_m H^+[m] ----
__global__ __launch_bounds__(kUwThreads) void k_uw_apply(float* __restrict__ u, int* __restrict__ wraps,
                                                         UnwrapArgs A) {
  const long long t = (long long)blockIdx.x * kUwThreads + threadIdx.x;
  const long long lat = (long long)A.S * A.np;
  if (t >= lat) return;
  const int s = (int)(t / A.np);
  const int i = (int)(t - (long long)s * A.np);
  float du0 = 0.f, du1 = 0.f, du2 = 0.f;
  bool any = false;
  for (int m = 0; m < A.M; ++m) {
    const long long g = (long long)m * A.S + s;
    const long long x = g * A.np + i;
    const long long k = round_mean(A.sums[g], A.np);
    const int N = (int)((long long)A.pot[x] + k - (long long)A.q[x]);
    if (wraps) wraps[x] = N;
    if (N != 0) {
      const float fN = (float)N;
      du0 += fN * A.coef[m][0];
      du1 += fN * A.coef[m][1];
      du2 += fN * A.coef[m][2];
      any = true;
    }
  }
  if (any) {
    u[t] += du0;
    u[lat + t] += du1;
    u[2 * lat + t] += du2;
  }
}

inline unsigned blocks_for(long long n) { return (unsigned)((n + kUwThreads - 1) / kUwThreads); }

}  // namespace

int unwrap_rounds(long long np) {
  int b = 0;
  while ((1LL << b) < np) ++b;
  return b + 1;                    // Boruvka at least halves the components of a map per round
}

hipError_t launch_unwrap(float* u, int* wraps, const UnwrapArgs& A, hipStream_t s) {
  const long long lat = (long long)A.S * A.np;
  long long nw = lat > (long long)A.rounds * kHookSlots ? lat : (long long)A.rounds * kHookSlots;
  nw = nw > A.nmaps ? nw : A.nmaps;
  k_uw_wrap<<<blocks_for(nw), kUwThreads, 0, s>>>(u, A);
  k_uw_reliability<<<blocks_for(A.npix), kUwThreads, 0, s>>>(A);
  for (int r = 0; r < A.rounds; ++r) {
    k_uw_best<<<blocks_for(A.npix), kUwThreads, 0, s>>>(A, r);
    k_uw_hook<<<blocks_for(A.npix), kUwThreads, 0, s>>>(A, r);
    k_uw_walk<<<blocks_for(A.npix), kUwThreads, 0, s>>>(A, r);
  }
  long long bx = (A.np + kUwThreads - 1) / kUwThreads;
  if (bx > 256) bx = 256;
  k_uw_sum<<<dim3((unsigned)bx, (unsigned)A.nmaps), kUwThreads, 0, s>>>(A);
  k_uw_apply<<<blocks_for(lat), kUwThreads, 0, s>>>(u, wraps, A);
  return hipGetLastError();
}

}  // namespace mpbp
