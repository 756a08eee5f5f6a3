// mpbp_dft.hpp - register-resident small DFTs and lane-cooperative line FFTs for gfx950.
//
// The far-field operator F of eq. (2) is a 2D DFT of the exit wave; every detector
// size used here factors as D = P * Q with P, Q in {4, 5, 8, 10, 12, 15, 16}.  A line of D points
// is transformed by a group of lanes of one wavefront with the four-step
// decomposition (n = b + Q a, k = c + P d):
//
//   X[c + P d] = sum_b w_Q^{b d} [ w_D^{b c} sum_a x[b + Q a] w_P^{a c} ]
//
// pass 1: lane b holds x[b + Q a] (a < P) in registers and does a P-point DFT, then
//         the twiddle w_D^{b c};
// pass 2: after an exchange through LDS, lane c holds the Q values of column c and
//         does a Q-point DFT; lane c ends with X[c + P d] (d < Q).
// The inverse runs the adjoint sequence, starting from the pass-2 layout, so the
// modulus residual of eq. (4) can be applied between the two without moving data.
#pragma once
#include <hip/hip_runtime.h>
#include <utility>

namespace mpbp {

struct cplx {
  float x, y;
};

__device__ __forceinline__ cplx cadd(cplx a, cplx b) { return {a.x + b.x, a.y + b.y}; }
__device__ __forceinline__ cplx csub(cplx a, cplx b) { return {a.x - b.x, a.y - b.y}; }
__device__ __forceinline__ cplx cmul(cplx a, cplx b) {
  return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x};
}
// a * conj(b)
__device__ __forceinline__ cplx cmulc(cplx a, cplx b) {
  return {a.x * b.x + a.y * b.y, a.y * b.x - a.x * b.y};
}
__device__ __forceinline__ cplx cscale(cplx a, float s) { return {a.x * s, a.y * s}; }

// cos and sin of 2 pi k / 48, k = 0..47 (all DFT sizes used divide 48).
__device__ constexpr double kCos48[48] = {
    1, 0.99144486137381038, 0.96592582628906831, 0.92387953251128674, 0.86602540378443871,
    0.79335334029123517, 0.70710678118654757, 0.60876142900872066, 0.50000000000000011,
    0.38268343236508984, 0.25881904510252074, 0.13052619222005171, 0, -0.1305261922200516,
    -0.25881904510252063, -0.3826834323650895, -0.49999999999999978, -0.60876142900872066,
    -0.70710678118654746, -0.79335334029123505, -0.86602540378443871, -0.92387953251128674,
    -0.9659258262890682, -0.99144486137381038, -1, -0.99144486137381038, -0.96592582628906831,
    -0.92387953251128685, -0.86602540378443882, -0.79335334029123517, -0.70710678118654791,
    -0.60876142900872088, -0.50000000000000044, -0.3826834323650895, -0.25881904510252063,
    -0.13052619222005163, 0, 0.13052619222005127, 0.2588190451025203, 0.38268343236508917,
    0.50000000000000011, 0.60876142900871988, 0.70710678118654735, 0.79335334029123494,
    0.86602540378443837, 0.92387953251128685, 0.96592582628906809, 0.99144486137381038};
__device__ constexpr double kSin48[48] = {
    0, 0.13052619222005157, 0.25881904510252074, 0.38268343236508978, 0.49999999999999994,
    0.60876142900872066, 0.70710678118654746, 0.79335334029123517, 0.8660254037844386,
    0.92387953251128674, 0.96592582628906831, 0.99144486137381038, 1, 0.99144486137381038,
    0.96592582628906831, 0.92387953251128685, 0.86602540378443871, 0.79335334029123517,
    0.70710678118654757, 0.60876142900872088, 0.49999999999999994, 0.38268343236508989,
    0.25881904510252102, 0.13052619222005199, 0, -0.13052619222005177, -0.25881904510252079,
    -0.38268343236508967, -0.49999999999999972, -0.60876142900872066, -0.70710678118654713,
    -0.79335334029123494, -0.86602540378443837, -0.92387953251128685, -0.96592582628906831,
    -0.99144486137381038, -1, -0.99144486137381049, -0.96592582628906842, -0.92387953251128696,
    -0.8660254037844386, -0.79335334029123572, -0.70710678118654768, -0.60876142900872088,
    -0.50000000000000044, -0.38268343236508956, -0.25881904510252157, -0.13052619222005168};

// cos and sin of 2 pi k / n for any n, in double at compile time: the turn fraction k / n
// is reduced to a quadrant exactly (integer arithmetic), then Taylor series on [0, pi/2).
constexpr double kPiD = 3.14159265358979323846264338327950288;
constexpr double taylor_sin(double x) {
  double t = x, s = x;
  for (int i = 1; i < 16; ++i) {
    t *= -x * x / ((2.0 * i) * (2.0 * i + 1.0));
    s += t;
  }
  return s;
}
constexpr double taylor_cos(double x) {
  double t = 1.0, s = 1.0;
  for (int i = 1; i < 16; ++i) {
    t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}
constexpr double cos_turn(long k, long n) {
  k = ((k % n) + n) % n;
  const long q = (4 * k) / n, r = 4 * k - q * n;      // quadrant, remainder
  const double t = (double)r / (double)n * (kPiD / 2.0);
  return q == 0 ? taylor_cos(t) : q == 1 ? -taylor_sin(t) : q == 2 ? -taylor_cos(t) : taylor_sin(t);
}
constexpr double sin_turn(long k, long n) {
  k = ((k % n) + n) % n;
  const long q = (4 * k) / n, r = 4 * k - q * n;
  const double t = (double)r / (double)n * (kPiD / 2.0);
  return q == 0 ? taylor_sin(t) : q == 1 ? taylor_cos(t) : q == 2 ? -taylor_sin(t) : -taylor_cos(t);
}

// Multiply by w_N^K = exp(-+2 pi i K / N) (minus for the forward transform), with the
// multiples of pi/4 done without general multiplies.
template <int N, int K, bool INV>
__device__ __forceinline__ cplx twc(cplx a) {
  constexpr int k = ((K % N) + N) % N;
  if constexpr (k == 0) {
    return a;
  } else if constexpr (2 * k == N) {
    return {-a.x, -a.y};
  } else if constexpr (4 * k == N) {         // forward: -i ; inverse: +i
    if constexpr (INV) return {-a.y, a.x};
    else return {a.y, -a.x};
  } else if constexpr (4 * k == 3 * N) {     // forward: +i ; inverse: -i
    if constexpr (INV) return {a.y, -a.x};
    else return {-a.y, a.x};
  } else if constexpr (8 * k == N || 8 * k == 3 * N || 8 * k == 5 * N || 8 * k == 7 * N) {
    constexpr float h = 0.70710678118654752f;
    constexpr int o = (8 * k) / N;           // odd multiple of pi/4
    // exp(-+ i pi o / 4) = h * (sx + i sy)
    constexpr float sx = (o == 1 || o == 7) ? 1.f : -1.f;
    constexpr float sy0 = (o == 1 || o == 3) ? -1.f : 1.f;   // forward sign of sin
    constexpr float sy = INV ? -sy0 : sy0;
    return {h * (sx * a.x - sy * a.y), h * (sx * a.y + sy * a.x)};
  } else if constexpr (48 % N == 0) {
    constexpr int idx = k * (48 / N);
    constexpr float c = (float)kCos48[idx];
    constexpr float s = INV ? (float)kSin48[idx] : -(float)kSin48[idx];
    return {a.x * c - a.y * s, a.x * s + a.y * c};
  } else {
    constexpr float c = (float)cos_turn(k, N);
    constexpr float s = INV ? (float)sin_turn(k, N) : -(float)sin_turn(k, N);
    return {a.x * c - a.y * s, a.x * s + a.y * c};
  }
}

template <int... I, typename F>
__device__ __forceinline__ void static_for_impl(std::integer_sequence<int, I...>, F&& f) {
  (f(std::integral_constant<int, I>{}), ...);
}
template <int N, typename F>
__device__ __forceinline__ void static_for(F&& f) {
  static_for_impl(std::make_integer_sequence<int, N>{}, f);
}

template <int N, bool INV>
struct DFT;

template <bool INV>
struct DFT<1, INV> {
  __device__ __forceinline__ static void run(cplx*) {}
};

template <bool INV>
struct DFT<2, INV> {
  __device__ __forceinline__ static void run(cplx* x) {
    cplx a = x[0], b = x[1];
    x[0] = cadd(a, b);
    x[1] = csub(a, b);
  }
};

template <bool INV>
struct DFT<3, INV> {
  __device__ __forceinline__ static void run(cplx* x) {
    constexpr float h = 0.86602540378443865f;  // sqrt(3)/2
    cplx t = cadd(x[1], x[2]);
    cplx d = csub(x[1], x[2]);
    cplx m = {x[0].x - 0.5f * t.x, x[0].y - 0.5f * t.y};
    // forward: j = -i h d ; inverse: +i h d
    cplx j = INV ? cplx{-h * d.y, h * d.x} : cplx{h * d.y, -h * d.x};
    x[0] = cadd(x[0], t);
    x[1] = cadd(m, j);
    x[2] = csub(m, j);
  }
};

// X_k = sum_n x_n w^{n k}, w = exp(-+2 pi i / 5), from the pair sums x1 + x4, x2 + x3
// and differences x1 - x4, x2 - x3 (w^4 = conj(w), w^3 = conj(w^2)).
template <bool INV>
struct DFT<5, INV> {
  __device__ __forceinline__ static void run(cplx* x) {
    constexpr float c1 = (float)cos_turn(1, 5), c2 = (float)cos_turn(2, 5);
    constexpr float s1 = (float)sin_turn(1, 5), s2 = (float)sin_turn(2, 5);
    const cplx t1 = cadd(x[1], x[4]), t2 = cadd(x[2], x[3]);
    const cplx t3 = csub(x[1], x[4]), t4 = csub(x[2], x[3]);
    const cplx m1 = {x[0].x + c1 * t1.x + c2 * t2.x, x[0].y + c1 * t1.y + c2 * t2.y};
    const cplx m2 = {x[0].x + c2 * t1.x + c1 * t2.x, x[0].y + c2 * t1.y + c1 * t2.y};
    const cplx n1 = {s1 * t3.x + s2 * t4.x, s1 * t3.y + s2 * t4.y};
    const cplx n2 = {s2 * t3.x - s1 * t4.x, s2 * t3.y - s1 * t4.y};
    // forward: X1 = m1 - i n1, X4 = m1 + i n1, X2 = m2 - i n2, X3 = m2 + i n2
    const cplx j1 = INV ? cplx{-n1.y, n1.x} : cplx{n1.y, -n1.x};
    const cplx j2 = INV ? cplx{-n2.y, n2.x} : cplx{n2.y, -n2.x};
    x[0] = cadd(x[0], cadd(t1, t2));
    x[1] = cadd(m1, j1);
    x[4] = csub(m1, j1);
    x[2] = cadd(m2, j2);
    x[3] = csub(m2, j2);
  }
};

template <bool INV>
struct DFT<4, INV> {
  __device__ __forceinline__ static void run(cplx* x) {
    cplx a = cadd(x[0], x[2]), b = csub(x[0], x[2]);
    cplx c = cadd(x[1], x[3]), d = csub(x[1], x[3]);
    cplx jd = INV ? cplx{-d.y, d.x} : cplx{d.y, -d.x};   // -+ i d
    x[0] = cadd(a, c);
    x[2] = csub(a, c);
    x[1] = cadd(b, jd);
    x[3] = csub(b, jd);
  }
};

// Composite sizes by the four-step formula above, entirely in registers.
template <int P, int Q, bool INV>
__device__ __forceinline__ void dft_pq(cplx* x) {
  constexpr int N = P * Q;
  cplx y[Q][P];
  static_for<Q>([&](auto b_) {
    constexpr int b = decltype(b_)::value;
    cplx t[P];
#pragma unroll
    for (int a = 0; a < P; ++a) t[a] = x[b + Q * a];
    DFT<P, INV>::run(t);
    static_for<P>([&](auto c_) {
      constexpr int c = decltype(c_)::value;
      y[b][c] = twc<N, b * c, INV>(t[c]);
    });
  });
#pragma unroll
  for (int c = 0; c < P; ++c) {
    cplx t[Q];
#pragma unroll
    for (int b = 0; b < Q; ++b) t[b] = y[b][c];
    DFT<Q, INV>::run(t);
#pragma unroll
    for (int d = 0; d < Q; ++d) x[c + P * d] = t[d];
  }
}

template <bool INV> struct DFT<6, INV>  { __device__ __forceinline__ static void run(cplx* x) { dft_pq<3, 2, INV>(x); } };
template <bool INV> struct DFT<8, INV>  { __device__ __forceinline__ static void run(cplx* x) { dft_pq<4, 2, INV>(x); } };
template <bool INV> struct DFT<12, INV> { __device__ __forceinline__ static void run(cplx* x) { dft_pq<4, 3, INV>(x); } };
template <bool INV> struct DFT<16, INV> { __device__ __forceinline__ static void run(cplx* x) { dft_pq<4, 4, INV>(x); } };
template <bool INV> struct DFT<10, INV> { __device__ __forceinline__ static void run(cplx* x) { dft_pq<5, 2, INV>(x); } };
template <bool INV> struct DFT<15, INV> { __device__ __forceinline__ static void run(cplx* x) { dft_pq<5, 3, INV>(x); } };

// Line configuration: D = P * Q; TPL lanes per line, a power of two >= Q, and >= P or a
// divisor of P (then each lane of the second pass takes P / TPL of the P columns, so no
// lane idles in either pass).
template <int D> struct LineCfg;
template <> struct LineCfg<32>  { static constexpr int P = 8,  Q = 4,  TPL = 8;  };
template <> struct LineCfg<64>  { static constexpr int P = 8,  Q = 8,  TPL = 8;  };
template <> struct LineCfg<96>  { static constexpr int P = 12, Q = 8,  TPL = 16; };
template <> struct LineCfg<128> { static constexpr int P = 16, Q = 8,  TPL = 8;  };
template <> struct LineCfg<192> { static constexpr int P = 16, Q = 12, TPL = 16; };
template <> struct LineCfg<256> { static constexpr int P = 16, Q = 16, TPL = 16; };
template <> struct LineCfg<50>  { static constexpr int P = 10, Q = 5,  TPL = 16; };
template <> struct LineCfg<150> { static constexpr int P = 10, Q = 15, TPL = 16; };

// Order LDS traffic between lanes of one wavefront (all lanes of a line live in one
// wavefront, so no workgroup barrier is needed for the exchange).
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

}  // namespace mpbp
