// Device arithmetic of the governor: counter-based draws, the two plants,
// the RK4 step, constraint margins and ordered reduction keys.
#pragma once

#include <math.h>

#include "rg_internal.hpp"

namespace rg {

// ---------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds of two 32x32
// multiplies whose high halves are XORed with the other counter words and the
// round key; the key advances by the golden-ratio / sqrt(3) Weyl constants.
// ---------------------------------------------------------------------------
struct Words {
  uint32_t v[4];
};

__device__ __forceinline__ Words philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                          uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int round = 0; round < 10; ++round) {
    // one 32 x 32 -> 64-bit product per multiplier (v_mad_u64_u32) instead of
    // separate low and high multiplies
    const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
    const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
    const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
    const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
    const uint32_t y0 = hi1 ^ c1 ^ k0;
    const uint32_t y2 = hi0 ^ c3 ^ k1;
    c0 = y0;
    c1 = lo1;
    c2 = y2;
    c3 = lo0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  Words w;
  w.v[0] = c0;
  w.v[1] = c1;
  w.v[2] = c2;
  w.v[3] = c3;
  return w;
}

// Canonical box draw: u = top 24 bits * 2^-24 (exact in binary32), then one
// correctly rounded binary32 FMA span * u + lo.
__device__ __forceinline__ float box_draw(uint32_t word, float lo32, float span32) {
  const float u = (float)(word >> 8) * 0x1p-24f;
  return __fmaf_rn(span32, u, lo32);
}

// ---------------------------------------------------------------------------
// Ordered keys: unsigned integers whose order is the order of the floats, so
// a device-wide minimum is a single integer atomicMin (exact and order-free).
// ---------------------------------------------------------------------------
__host__ __device__ __forceinline__ uint32_t ord32(float f) {
  uint32_t b;
  __builtin_memcpy(&b, &f, 4);
  return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__host__ __device__ __forceinline__ float unord32(uint32_t o) {
  const uint32_t b = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  float f;
  __builtin_memcpy(&f, &b, 4);
  return f;
}
__host__ __device__ __forceinline__ unsigned long long ord64(double d) {
  unsigned long long b;
  __builtin_memcpy(&b, &d, 8);
  return (b >> 63) ? ~b : (b | 0x8000000000000000ull);
}
__host__ __device__ __forceinline__ double unord64(unsigned long long o) {
  const unsigned long long b = (o >> 63) ? (o & 0x7fffffffffffffffull) : ~o;
  double d;
  __builtin_memcpy(&d, &b, 8);
  return d;
}

// Margin reduction key of one lane: FP32 rollouts carry the scenario index in
// the low word (ties resolve to the lowest scenario); FP64 rollouts use the
// full ordered double.
__device__ __forceinline__ unsigned long long lane_key(float m, int k) {
  return ((unsigned long long)ord32(m) << 32) | (uint32_t)k;
}
__device__ __forceinline__ unsigned long long lane_key(double m, int) { return ord64(m); }
__device__ __forceinline__ double key_margin(unsigned long long key, int precision) {
  return precision == 0 ? (double)unord32((uint32_t)(key >> 32)) : unord64(key);
}

template <class T>
__device__ __forceinline__ T t_inf() {
  return (T)INFINITY;
}

// FP32 rollouts: tanh from the hardware base-2 exponential and reciprocal,
// tanh(z) = 1 - 2 / (1 + e^{2z}), branch-free and with no sign handling (e^{2z}
// overflows to +inf for large z, giving 1, and underflows to 0 for very
// negative z, giving -1); absolute error a few 2^-24 (relative error grows
// only where |tanh z| is itself below 1e-6); square root from the hardware
// instruction (1 ulp).  FP64 paths use the FP64 tanh below.
__device__ __forceinline__ float t_tanh(float z) {
  const float e = __builtin_amdgcn_exp2f(z * 2.8853900817779268f);  // 2 log2(e) z
  const float r = __builtin_amdgcn_rcpf(e + 1.0f);
  return __builtin_fmaf(-2.0f, r, 1.0f);
}
// tanh(x - xbar) with the shift folded into the exponent: nk = -2 log2(e) xbar
// (rounded once), so e^{2(x - xbar)} = 2^{fma(2 log2(e), x, nk)}; same error
// terms as t_tanh plus the rounding of nk (a few 2^-24 |xbar| in the exponent).
__device__ __forceinline__ float t_tanh_shift(float x, float nk) {
  const float e = __builtin_amdgcn_exp2f(__builtin_fmaf(2.8853900817779268f, x, nk));
  const float r = __builtin_amdgcn_rcpf(e + 1.0f);
  return __builtin_fmaf(-2.0f, r, 1.0f);
}
// FP64 tanh of the FP64 rollouts and steady-state solves (written here, not
// the library's): tanh|z| = t / (t + 2) with t = expm1(2|z|), which has no
// cancellation at small |z|, carrying the sign of z; 1 once 2|z| >= 40 (then
// 1 - tanh|z| < 2^-56).  expm1(x), 0 <= x <= 40: Cody-Waite reduction
// x = k ln2 + r with |r| <= ln2 / 2 and ln 2 split into a 32-bit head (k ln2_head
// is exact) and its remainder; expm1(r) = r p(r) with p the Taylor series of
// expm1(r) / r to degree 12 (truncation below 2^-56 relative on that interval),
// its tail evaluated in Estrin's scheme (dependent depth 6 instead of Horner's
// 12: the FP64 rechecks are bound by this latency); then
// expm1(x) = 2^k expm1(r) + (2^k - 1).
// Branch-free: arguments at or beyond 40 (and NaN) run the same arithmetic on
// 40 and are replaced at the end.  Within 3 ulp of tanh over the arguments the
// rollouts meet (checked against an extended-precision reference in the tests).
__device__ __forceinline__ double t_tanh(double z) {
  const double ax = 2.0 * fabs(z);
  const double x = fmin(ax, 40.0);
  constexpr double kLn2Head = 0x1.62e42ff0p-1;         // ln 2 to 32 significant bits
  constexpr double kLn2Tail = -0x1.718432a1b0e26p-35;  // ln 2 - kLn2Head
  constexpr double kInvLn2 = 0x1.71547652b82fep+0;
  const double k = rint(x * kInvLn2);
  double r = fma(-k, kLn2Head, x);
  r = fma(-k, kLn2Tail, r);
  // p(r) = sum_n r^n / (n + 1)!, n = 0..12, as 1 + r (1/2 + r s(r)) with the
  // tail s (degree 10) in Estrin's scheme: its rounding errors enter p scaled
  // by r^2, and the two outer steps round as Horner's last two do
  const double r2 = r * r, r4 = r2 * r2, r8 = r4 * r4;
  const double e1 = fma(1.0 / 24.0, r, 1.0 / 6.0);
  const double e2 = fma(1.0 / 720.0, r, 1.0 / 120.0);
  const double e3 = fma(1.0 / 40320.0, r, 1.0 / 5040.0);
  const double e4 = fma(1.0 / 3628800.0, r, 1.0 / 362880.0);
  const double e5 = fma(1.0 / 479001600.0, r, 1.0 / 39916800.0);
  const double f1 = fma(e2, r2, e1);
  const double f2 = fma(e4, r2, e3);
  const double f3 = fma(1.0 / 6227020800.0, r2, e5);
  const double g1 = fma(f2, r4, f1);
  const double sr = fma(f3, r8, g1);
  const double p = fma(fma(sr, r, 0.5), r, 1.0);
  const double em = p * r;  // expm1(r)
  const double two_k = ldexp(1.0, (int)k);
  const double t = fma(two_k, em, two_k - 1.0);
  const double th = copysign(t / (t + 2.0), z);
  const double sat = ax == ax ? copysign(1.0, z) : z;
  return ax < 40.0 ? th : sat;
}
__device__ __forceinline__ float t_sqrt(float z) { return __builtin_amdgcn_sqrtf(z); }
__device__ __forceinline__ double t_sqrt(double z) { return sqrt(z); }
__device__ __forceinline__ float t_fma(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double t_fma(double a, double b, double c) { return __builtin_fma(a, b, c); }

// ---------------------------------------------------------------------------
// Plants.  Coef holds the uniform coefficients (kernel arguments, so scalar
// registers); Lane holds what is fixed for one rollout (set-point, sampled
// coefficients).  force() is the part of the derivative that is constant over
// one RK4 step.
// ---------------------------------------------------------------------------
template <int KIND, class T>
struct Plant;

// LQ4: xdot = A x + B v + G (x.*x) + E w,  y = C x.
template <class T>
struct Plant<1, T> {
  static constexpr int n = 4, nw = 2, ny = 2, nth = 0;
  struct Coef {
    T A[16], B[4], G[16], E[8], C[8];
  };
  struct Lane {
    T bv[4];
  };
  __host__ __device__ static const T* nominal_theta(const Coef&) { return nullptr; }
  static void load(Coef& c, const double* s) {
    for (int i = 0; i < 16; ++i) c.A[i] = (T)s[i];
    for (int i = 0; i < 4; ++i) c.B[i] = (T)s[16 + i];
    for (int i = 0; i < 16; ++i) c.G[i] = (T)s[20 + i];
    for (int i = 0; i < 8; ++i) c.E[i] = (T)s[36 + i];
    for (int i = 0; i < 8; ++i) c.C[i] = (T)s[44 + i];
  }
  __device__ static void lane_init(const Coef& c, const T*, T v, Lane& L) {
#pragma unroll
    for (int i = 0; i < 4; ++i) L.bv[i] = c.B[i] * v;
  }
  __device__ static void force(const Coef& c, const Lane& L, const T* w, T* s) {
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] = t_fma(c.E[2 * i + 1], w[1], t_fma(c.E[2 * i], w[0], L.bv[i]));
  }
  __device__ static void force0(const Coef&, const Lane& L, T* s) {
#pragma unroll
    for (int i = 0; i < 4; ++i) s[i] = L.bv[i];
  }
  __device__ static void deriv(const Coef& c, const Lane&, const T* s, const T* x, T* xd) {
    T q[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) q[j] = x[j] * x[j];
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      T a = s[i];
#pragma unroll
      for (int j = 0; j < 4; ++j) a = t_fma(c.A[4 * i + j], x[j], a);
#pragma unroll
      for (int j = 0; j < 4; ++j) a = t_fma(c.G[4 * i + j], q[j], a);
      xd[i] = a;
    }
  }
  __device__ static void post(const Coef& c, const T* w, T* x) {
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = x[i] + (c.E[2 * i] * w[0] + c.E[2 * i + 1] * w[1]);
  }
  __device__ static void output(const Coef& c, const Lane&, const T* x, T* y) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      T a = c.C[4 * i] * x[0];
#pragma unroll
      for (int j = 1; j < 4; ++j) a = t_fma(c.C[4 * i + j], x[j], a);
      y[i] = a;
    }
  }
  // Reverse mode: xb = J(x)^T al, vb += al . df/dv (df/dtheta: none).
  __device__ static void vjp(const Coef& c, const Lane&, const T* x, const T* al, T* xb,
                             double& vb, double*) {
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      T acc = 0;
#pragma unroll
      for (int i = 0; i < 4; ++i) acc = t_fma(t_fma(2 * c.G[4 * i + j], x[j], c.A[4 * i + j]), al[i], acc);
      xb[j] = acc;
    }
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 4; ++i) s += (double)al[i] * (double)c.B[i];
    vb += s;
  }
  // Forward mode: out = J(x) dx + df/dv (a unit change of the set-point).
  __device__ static void jvp(const Coef& c, const Lane&, const T* x, const T* dx, T* out) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      T a = c.B[i];
#pragma unroll
      for (int j = 0; j < 4; ++j) a = t_fma(t_fma(2 * c.G[4 * i + j], x[j], c.A[4 * i + j]), dx[j], a);
      out[i] = a;
    }
  }
  // dy = (dh/dx) dx.
  __device__ static void output_tan(const Coef& c, const T*, const T* dx, T* dy) {
#pragma unroll
    for (int i = 0; i < 2; ++i) {
      T a = c.C[4 * i] * dx[0];
#pragma unroll
      for (int j = 1; j < 4; ++j) a = t_fma(c.C[4 * i + j], dx[j], a);
      dy[i] = a;
    }
  }
  // dm/dx of the margin row m = g_r - F_r h(x) (F row given).
  __device__ static void out_grad(const Coef& c, const T* Fr, const T*, T* gx) {
#pragma unroll
    for (int j = 0; j < 4; ++j) gx[j] = -(Fr[0] * c.C[j] + Fr[1] * c.C[4 + j]);
  }
  // Equilibrium helpers (FP64 only): initial guess solves A x = -B v.
  __device__ static void eq_guess(const Coef& c, T v, T* x, T* J) {
#pragma unroll
    for (int i = 0; i < 16; ++i) J[i] = c.A[i];
#pragma unroll
    for (int i = 0; i < 4; ++i) x[i] = -(c.B[i] * v);
  }
  __device__ static bool eq_guess_needs_solve() { return true; }
  __device__ static void dfdv(const Coef& c, const T*, T* fv) {
#pragma unroll
    for (int i = 0; i < 4; ++i) fv[i] = c.B[i];
  }
  __device__ static void jacobian(const Coef& c, const T* x, T, T* J) {
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) J[4 * i + j] = c.A[4 * i + j] + 2 * c.G[4 * i + j] * x[j];
  }
};

// FC9: volumes p1..p6 (x0..x5) fed by compressor speed w1 (x6), auxiliary
// speed w2 (x7), demand state w3 (x8):  z = x - xbar, p7 = p_amb,
//   q0 = c_q0 w1,  q_l = k_l sqrt(max(p_l - p_{l+1}, 0)),
//   xdot_i = -a_i z_i + (W tanh z)_i + w_i + phi_i,
//   phi_l = q_{l-1} - q_l (l = 1..6), phi_7 = b1 v - mu1 w1 (p1 - p1ref),
//   phi_8 = b2 v w1, phi_9 = b3 v - mu2 (w3 - 1) v;
//   y = (c_q0 w1 / (d0 + d1 w3), p1, w1).
template <class T>
struct Plant<2, T> {
  static constexpr int n = 9, nw = 9, ny = 3, nth = 20;
  struct Coef {
    T W[81], xbar[9], thnom[20];
    T c_q0, p_amb, d0, d1, p1ref;
    T nkxbar[9];  // -2 log2(e) xbar (FP32 tanh with the shift in its exponent)
  };
  struct Lane {
    T a[9], kq[6], b[3], mu[2];
    T v;
    T axb[9];    // a_i xbar_i: -a_i (x_i - xbar_i) = -a_i x_i + a_i xbar_i, the constant
                 // part carried in the step forcing s_i
    const T* W;  // the coupling matrix the derivative reads (c.W, or a copy in registers)
  };
  __host__ __device__ static const T* nominal_theta(const Coef& c) { return c.thnom; }
  static void load(Coef& c, const double* s) {
    for (int i = 0; i < 81; ++i) c.W[i] = (T)s[i];
    for (int i = 0; i < 9; ++i) c.xbar[i] = (T)s[81 + i];
    for (int i = 0; i < 20; ++i) c.thnom[i] = (T)s[90 + i];
    c.c_q0 = (T)s[110];
    c.p_amb = (T)s[111];
    c.d0 = (T)s[112];
    c.d1 = (T)s[113];
    c.p1ref = (T)s[114];
    for (int i = 0; i < 9; ++i) c.nkxbar[i] = (T)(-2.8853900817779268 * s[81 + i]);
  }
  __device__ static void lane_init(const Coef& c, const T* th, T v, Lane& L) {
#pragma unroll
    for (int i = 0; i < 9; ++i) L.a[i] = th[i];
#pragma unroll
    for (int i = 0; i < 6; ++i) L.kq[i] = th[9 + i];
#pragma unroll
    for (int i = 0; i < 3; ++i) L.b[i] = th[15 + i];
    L.mu[0] = th[18];
    L.mu[1] = th[19];
    L.v = v;
#pragma unroll
    for (int i = 0; i < 9; ++i) L.axb[i] = L.a[i] * c.xbar[i];
    L.W = c.W;
  }
  // Step forcing of component i: w_i + a_i xbar_i (the derivative takes
  // -a_i x_i, so the sum is w_i - a_i (x_i - xbar_i))
  __device__ static void force(const Coef&, const Lane& L, const T* w, T* s) {
#pragma unroll
    for (int i = 0; i < 9; ++i) s[i] = w[i] + L.axb[i];
  }
  __device__ static void force0(const Coef&, const Lane& L, T* s) {
#pragma unroll
    for (int i = 0; i < 9; ++i) s[i] = L.axb[i];
  }
  // tanh(x_j - xbar_j): FP32 with the shift in the exponent, FP64 on the difference
  __device__ static T tanh_at(T x, T xbar, T nkxbar) {
    if constexpr (sizeof(T) == 4) return t_tanh_shift(x, nkxbar);
    else return t_tanh(x - xbar);
  }
  // Component i of the derivative from the pieces of the evaluation point:
  // x_i (si carries a_i xbar_i), the vector tz = tanh(x - xbar), the orifice
  // flows q_i = qa qb and q_{i+1} = qk qr as factor pairs (i < 6), and the
  // states x0, x6, x8.  Every
  // product-sum is an explicit fma and nothing here is contracted, so the
  // one-lane derivative below and the FP64 recheck that gives each component
  // its own lane round alike.
  __device__ static T comp(int i, T ai, const T* wrow, T si, T xi, const T* tz, T qa, T qb,
                           T qk, T qr, T x0, T x6, T x8, const Lane& L, T p1ref) {
#pragma clang fp contract(off)
    // phi_i = A B + C D in one form for every row (i < 6: q_i - q_{i+1};
    // 6: b1 v - mu1 w1 (p1 - p1ref); 7: b2 v w1; 8: b3 v - mu2 (w3 - 1) v);
    // every candidate is computed and then selected (no branch where i varies
    // over the lanes).  The sum runs s_i + C D, - a_i x_i, the coupling
    // terms, + A B: one fma per term.
    const T a6 = -(L.mu[0] * x6), b6 = x0 - p1ref;
    const T a7 = L.b[1] * L.v;
    const T a8 = -(L.mu[1] * (x8 - (T)1));
    const bool lo = i < 6, r6 = i == 6, r7 = i == 7;
    const T A = lo ? qa : (r6 ? a6 : (r7 ? a7 : a8));
    const T B = lo ? qb : (r6 ? b6 : (r7 ? x6 : L.v));
    const T C = lo ? -qk : (r6 ? L.b[0] : L.b[2]);
    const T D = lo ? qr : L.v;
    T a = r7 ? si : t_fma(C, D, si);
    a = t_fma(-ai, xi, a);
#pragma unroll
    for (int j = 0; j < 9; ++j) a = t_fma(wrow[j], tz[j], a);
    return t_fma(A, B, a);
  }
  // Square-root factor of the orifice flow q_{l+1}: sqrt(max(p_l - p_{l+1}, 0))
  // with p_7 = p_amb.
  __device__ static T orifice(T pl, T pn) {
    const T dp = pl - pn;
    return t_sqrt(dp > (T)0 ? dp : (T)0);
  }
  __device__ static void deriv(const Coef& c, const Lane& L, const T* s, const T* x, T* xd) {
    T tz[9], r[6];
#pragma unroll
    for (int j = 0; j < 9; ++j) tz[j] = tanh_at(x[j], c.xbar[j], c.nkxbar[j]);
#pragma unroll
    for (int l = 0; l < 6; ++l) r[l] = orifice(x[l], (l < 5) ? x[l + 1] : c.p_amb);
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      const T qa = i == 0 ? c.c_q0 : (i < 6 ? L.kq[i > 0 ? i - 1 : 0] : (T)0);
      const T qb = i == 0 ? x[6] : (i < 6 ? r[i > 0 ? i - 1 : 0] : (T)0);
      const T qk = i < 6 ? L.kq[i < 6 ? i : 0] : (T)0;
      const T qr = i < 6 ? r[i < 6 ? i : 0] : (T)0;
      xd[i] = comp(i, L.a[i], &L.W[9 * i], s[i], x[i], tz, qa, qb, qk, qr, x[0], x[6], x[8], L,
                   c.p1ref);
    }
  }
  __device__ static void post(const Coef&, const T* w, T* x) {
#pragma unroll
    for (int i = 0; i < 9; ++i) x[i] = x[i] + w[i];
  }
  __device__ static void output(const Coef& c, const Lane&, const T* x, T* y) {
    y[0] = c.c_q0 * x[6] / t_fma(c.d1, x[8], c.d0);
    y[1] = x[0];
    y[2] = x[6];
  }
  // Reverse mode: xb = J(x)^T al, vb += al . df/dv, tb += al . df/dtheta
  // (theta = the lane's coefficients a, k, b, mu).
  __device__ static void vjp(const Coef& c, const Lane& L, const T* x, const T* al, T* xb,
                             double& vb, double* tb) {
    T z[9], tz[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      z[j] = x[j] - c.xbar[j];
      tz[j] = tanh_at(x[j], c.xbar[j], c.nkxbar[j]);
    }
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      T acc = 0;
#pragma unroll
      for (int i = 0; i < 9; ++i) acc = t_fma(L.W[9 * i + j], al[i], acc);
      xb[j] = t_fma(-L.a[j], al[j], acc * (1 - tz[j] * tz[j]));
      tb[j] += -(double)al[j] * (double)z[j];
    }
    // orifice flows q_{l+1} = k_l sqrt(max(dp_l, 0)): -in phi_l, +in phi_{l+1}
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      const T dn = (l < 5) ? x[l + 1] : c.p_amb;
      const T dp = x[l] - dn;
      const T sq = dp > (T)0 ? t_sqrt(dp) : (T)0;
      const T d = dp > (T)0 ? L.kq[l] / (2 * sq) : (T)0;
      const T beta = (l < 5) ? al[l + 1] - al[l] : -al[l];
      xb[l] += beta * d;
      if (l < 5) xb[l + 1] -= beta * d;
      tb[9 + l] += (double)beta * (double)sq;
    }
    xb[6] += al[0] * c.c_q0;  // q0 in phi_1
    // phi_7 = b1 v - mu1 w1 (p1 - p1ref)
    xb[6] -= al[6] * L.mu[0] * (x[0] - c.p1ref);
    xb[0] -= al[6] * L.mu[0] * x[6];
    // phi_8 = b2 v w1
    xb[6] += al[7] * L.b[1] * L.v;
    // phi_9 = b3 v - mu2 (w3 - 1) v
    xb[8] -= al[8] * L.mu[1] * L.v;
    const double v = (double)L.v;
    vb += (double)al[6] * (double)L.b[0] + (double)al[7] * (double)L.b[1] * (double)x[6] +
          (double)al[8] * ((double)L.b[2] - (double)L.mu[1] * ((double)x[8] - 1.0));
    tb[15] += (double)al[6] * v;
    tb[16] += (double)al[7] * v * (double)x[6];
    tb[17] += (double)al[8] * v;
    tb[18] += -(double)al[6] * (double)x[6] * ((double)x[0] - (double)c.p1ref);
    tb[19] += -(double)al[8] * ((double)x[8] - 1.0) * v;
  }
  // Forward mode: out = J(x) dx + df/dv (a unit change of the set-point), with
  // the lane's coefficients; the orifice flow has derivative 0 where the
  // valve is closed (p_l <= p_{l+1}).
  __device__ static void jvp(const Coef& c, const Lane& L, const T* x, const T* dx, T* out) {
    T sd[9], dq[7];
#pragma unroll
    for (int j = 0; j < 9; ++j) {
      const T tz = tanh_at(x[j], c.xbar[j], c.nkxbar[j]);
      sd[j] = (1 - tz * tz) * dx[j];
    }
    dq[0] = c.c_q0 * dx[6];
#pragma unroll
    for (int l = 0; l < 6; ++l) {
      const T dn = (l < 5) ? x[l + 1] : c.p_amb;
      const T dp = x[l] - dn;
      const T ddp = (l < 5) ? dx[l] - dx[l + 1] : dx[l];
      dq[l + 1] = dp > (T)0 ? L.kq[l] / (2 * t_sqrt(dp)) * ddp : (T)0;
    }
#pragma unroll
    for (int i = 0; i < 9; ++i) {
      T a = -L.a[i] * dx[i];
#pragma unroll
      for (int j = 0; j < 9; ++j) a = t_fma(L.W[9 * i + j], sd[j], a);
      T dphi;
      if (i < 6) dphi = dq[i] - dq[i + 1];
      else if (i == 6) dphi = L.b[0] - L.mu[0] * (dx[6] * (x[0] - c.p1ref) + x[6] * dx[0]);
      else if (i == 7) dphi = L.b[1] * (x[6] + L.v * dx[6]);
      else dphi = L.b[2] - L.mu[1] * ((x[8] - (T)1) + L.v * dx[8]);
      out[i] = a + dphi;
    }
  }
  // dy = (dh/dx) dx.
  __device__ static void output_tan(const Coef& c, const T* x, const T* dx, T* dy) {
    const T den = t_fma(c.d1, x[8], c.d0);
    dy[0] = c.c_q0 * (dx[6] * den - x[6] * c.d1 * dx[8]) / (den * den);
    dy[1] = dx[0];
    dy[2] = dx[6];
  }
  __device__ static void out_grad(const Coef& c, const T* Fr, const T* x, T* gx) {
#pragma unroll
    for (int j = 0; j < 9; ++j) gx[j] = 0;
    const T den = t_fma(c.d1, x[8], c.d0);
    gx[6] = -(Fr[0] * c.c_q0 / den + Fr[2]);
    gx[8] = Fr[0] * c.c_q0 * x[6] * c.d1 / (den * den);
    gx[0] = -Fr[1];
  }
  // df/dv and df/dtheta at nominal theta (FP64, steady-state sensitivities).
  __device__ static void dfdv(const Coef& c, const T* x, T* fv) {
    const T* b = c.thnom + 15;
    const T* mu = c.thnom + 18;
#pragma unroll
    for (int i = 0; i < 9; ++i) fv[i] = 0;
    fv[6] = b[0];
    fv[7] = b[1] * x[6];
    fv[8] = b[2] - mu[1] * (x[8] - 1);
  }
  __device__ static void eq_guess(const Coef& c, T, T* x, T*) {
#pragma unroll
    for (int i = 0; i < 9; ++i) x[i] = c.xbar[i];
  }
  __device__ static bool eq_guess_needs_solve() { return false; }
  // df/dx at nominal theta, w = 0.
  __device__ static void jacobian(const Coef& c, const T* x, T v, T* J) {
    const T* a = c.thnom;
    const T* kq = c.thnom + 9;
    const T* b = c.thnom + 15;
    const T* mu = c.thnom + 18;
    for (int j = 0; j < 9; ++j) {
      const T tj = t_tanh(x[j] - c.xbar[j]);
      const T dj = 1 - tj * tj;
      for (int i = 0; i < 9; ++i) J[9 * i + j] = c.W[9 * i + j] * dj;
    }
    for (int i = 0; i < 9; ++i) J[9 * i + i] -= a[i];
    J[0 * 9 + 6] += c.c_q0;  // q0 enters phi_1
    for (int l = 0; l < 6; ++l) {
      const T dn = (l < 5) ? x[l + 1] : c.p_amb;
      const T dp = x[l] - dn;
      const T d = dp > 0 ? kq[l] / (2 * t_sqrt(dp)) : (T)0;  // dq_{l+1}/dp_l
      J[9 * l + l] -= d;
      if (l < 5) {
        J[9 * l + l + 1] += d;
        J[9 * (l + 1) + l] += d;
        J[9 * (l + 1) + l + 1] -= d;
      }
    }
    J[9 * 6 + 6] -= mu[0] * (x[0] - c.p1ref);
    J[9 * 6 + 0] -= mu[0] * x[6];
    J[9 * 7 + 6] += b[1] * v;
    J[9 * 8 + 8] -= mu[1] * v;
  }
};

// ---------------------------------------------------------------------------
// Classical RK4 step with the step forcing s held: the stage increments are
// accumulated as k1 + 2 k2 + 2 k3 + k4.
// ---------------------------------------------------------------------------
template <int KIND, class T>
__device__ __forceinline__ void rk4_step(const typename Plant<KIND, T>::Coef& c,
                                         const typename Plant<KIND, T>::Lane& L, const T* s,
                                         T h, T hh, T h6, T* x) {
  using P = Plant<KIND, T>;
  T k[P::n], acc[P::n], xs[P::n];
  P::deriv(c, L, s, x, k);
#pragma unroll
  for (int i = 0; i < P::n; ++i) {
    acc[i] = k[i];
    xs[i] = t_fma(hh, k[i], x[i]);
  }
  P::deriv(c, L, s, xs, k);
#pragma unroll
  for (int i = 0; i < P::n; ++i) {
    acc[i] = t_fma((T)2, k[i], acc[i]);
    xs[i] = t_fma(hh, k[i], x[i]);
  }
  P::deriv(c, L, s, xs, k);
#pragma unroll
  for (int i = 0; i < P::n; ++i) {
    acc[i] = t_fma((T)2, k[i], acc[i]);
    xs[i] = t_fma(h, k[i], x[i]);
  }
  P::deriv(c, L, s, xs, k);
#pragma unroll
  for (int i = 0; i < P::n; ++i) x[i] = t_fma(h6, acc[i] + k[i], x[i]);
}

// One RK4 step of the state together with its forward tangent dx (the
// derivative with respect to the set-point): the state update has the same
// operations, in the same order, as rk4_step.
template <int KIND, class T>
__device__ __forceinline__ void rk4_step_tan(const typename Plant<KIND, T>::Coef& c,
                                             const typename Plant<KIND, T>::Lane& L, const T* s,
                                             T h, T hh, T h6, T* x, T* dx) {
  using P = Plant<KIND, T>;
  constexpr int n = P::n;
  T k[n], acc[n], xs[n], d[n], dacc[n], dxs[n];
  P::deriv(c, L, s, x, k);
  P::jvp(c, L, x, dx, d);
#pragma unroll
  for (int i = 0; i < n; ++i) {
    acc[i] = k[i];
    xs[i] = t_fma(hh, k[i], x[i]);
    dacc[i] = d[i];
    dxs[i] = t_fma(hh, d[i], dx[i]);
  }
  P::deriv(c, L, s, xs, k);
  P::jvp(c, L, xs, dxs, d);
#pragma unroll
  for (int i = 0; i < n; ++i) {
    acc[i] = t_fma((T)2, k[i], acc[i]);
    xs[i] = t_fma(hh, k[i], x[i]);
    dacc[i] = t_fma((T)2, d[i], dacc[i]);
    dxs[i] = t_fma(hh, d[i], dx[i]);
  }
  P::deriv(c, L, s, xs, k);
  P::jvp(c, L, xs, dxs, d);
#pragma unroll
  for (int i = 0; i < n; ++i) {
    acc[i] = t_fma((T)2, k[i], acc[i]);
    xs[i] = t_fma(h, k[i], x[i]);
    dacc[i] = t_fma((T)2, d[i], dacc[i]);
    dxs[i] = t_fma(h, d[i], dx[i]);
  }
  P::deriv(c, L, s, xs, k);
  P::jvp(c, L, xs, dxs, d);
#pragma unroll
  for (int i = 0; i < n; ++i) {
    x[i] = t_fma(h6, acc[i] + k[i], x[i]);
    dx[i] = t_fma(h6, dacc[i] + d[i], dx[i]);
  }
}

// Reverse sweep of one RK4 step at x with forcing s: lam <- (dPhi/dx)^T lam,
// vb += lam . dPhi/dv, tb += lam . dPhi/dtheta.  Stage states are recomputed.
template <int KIND, class T>
__device__ __forceinline__ void rk4_vjp(const typename Plant<KIND, T>::Coef& c,
                                        const typename Plant<KIND, T>::Lane& L, const T* s,
                                        T h, T hh, T h6, const T* x, T* lam, double& vb,
                                        double* tb) {
  using P = Plant<KIND, T>;
  constexpr int n = P::n;
  T x2[n], x3[n], x4[n], k[n];
  P::deriv(c, L, s, x, k);
#pragma unroll
  for (int i = 0; i < n; ++i) x2[i] = t_fma(hh, k[i], x[i]);
  P::deriv(c, L, s, x2, k);
#pragma unroll
  for (int i = 0; i < n; ++i) x3[i] = t_fma(hh, k[i], x[i]);
  P::deriv(c, L, s, x3, k);
#pragma unroll
  for (int i = 0; i < n; ++i) x4[i] = t_fma(h, k[i], x[i]);
  T a[n], u[n], acc[n];
  // k4 = f(x4), weight h/6
#pragma unroll
  for (int i = 0; i < n; ++i) a[i] = h6 * lam[i];
  P::vjp(c, L, x4, a, u, vb, tb);
#pragma unroll
  for (int i = 0; i < n; ++i) {
    acc[i] = u[i];
    a[i] = t_fma(h, u[i], 2 * h6 * lam[i]);  // adjoint of k3: 2h/6 lam + h u4
  }
  P::vjp(c, L, x3, a, u, vb, tb);
#pragma unroll
  for (int i = 0; i < n; ++i) {
    acc[i] += u[i];
    a[i] = t_fma(hh, u[i], 2 * h6 * lam[i]);  // adjoint of k2
  }
  P::vjp(c, L, x2, a, u, vb, tb);
#pragma unroll
  for (int i = 0; i < n; ++i) {
    acc[i] += u[i];
    a[i] = t_fma(hh, u[i], h6 * lam[i]);  // adjoint of k1
  }
  P::vjp(c, L, x, a, u, vb, tb);
#pragma unroll
  for (int i = 0; i < n; ++i) lam[i] = lam[i] + (acc[i] + u[i]);
}

// Margin over kNC padded rows (padding rows: F = 0, g = +inf).
// Margin and its minimising row.
template <int NY, class T>
__device__ __forceinline__ T margin_rows_arg(const T* F, const T* g, const T* y, int& rarg) {
  T best = t_inf<T>();
  rarg = 0;
#pragma unroll
  for (int r = 0; r < kNC; ++r) {
    T fy = F[r * NY] * y[0];
#pragma unroll
    for (int i = 1; i < NY; ++i) fy = t_fma(F[r * NY + i], y[i], fy);
    const T m = g[r] - fy;
    if (m < best || m != m) {
      best = m;
      rarg = r;
    }
  }
  return best;
}

template <int NY, class T>
__device__ __forceinline__ T margin_rows(const T* F, const T* g, const T* y) {
  T best = t_inf<T>();
#pragma unroll
  for (int r = 0; r < kNC; ++r) {
    T fy = F[r * NY] * y[0];
#pragma unroll
    for (int i = 1; i < NY; ++i) fy = t_fma(F[r * NY + i], y[i], fy);
    const T m = g[r] - fy;
    best = (m < best || m != m) ? m : best;  // a NaN row stays NaN (caller maps it to -inf)
  }
  return best;
}

}  // namespace rg
