// Device helpers shared by the gedmg kernels: reference-element shape data,
// softplus pairs in delta form, wavefront helpers.
#pragma once

#include <hip/hip_runtime.h>

namespace gedmg {

constexpr double kInvSqrt3 = 0.57735026918962576451;

// Reference coordinate (+-1) of local node a along axis d (Q4 counter-clockwise,
// Hex8 bottom face then top face).
__device__ __forceinline__ double ref_coord(int a, int d) {
  const int r = a & 3;
  if (d == 0) return (r == 1 || r == 2) ? 1.0 : -1.0;
  if (d == 1) return (r >= 2) ? 1.0 : -1.0;
  return (a >= 4) ? 1.0 : -1.0;
}

// Shape value and natural derivatives of node a at Gauss point q (the point on
// the ray to node q, natural coordinates +-1/sqrt(3)).
template <int DIM>
__device__ __forceinline__ void shape_at(int a, int q, double& N, double dN[DIM]) {
  double f[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) f[d] = 0.5 * (1.0 + ref_coord(a, d) * ref_coord(q, d) * kInvSqrt3);
  N = 1.0;
#pragma unroll
  for (int d = 0; d < DIM; ++d) N *= f[d];
#pragma unroll
  for (int k = 0; k < DIM; ++k) {
    double p = 0.5 * ref_coord(a, k);
#pragma unroll
    for (int d = 0; d < DIM; ++d)
      if (d != k) p *= f[d];
    dN[k] = p;
  }
}

// ------------------------------------------------------------------ FP64 math
// Elementary functions for the network activations, written for the argument
// ranges the kernels use.
//   exp(t), expm1(t) for t <= 700: Cody-Waite reduction t = n ln2 + r with
//     |r| <= ln2/2 (ln2 split so that n * kLn2Hi is exact), Taylor series of
//     expm1(r) through r^13/13! (truncation below 2^-60 relative), scaling by
//     2^n; expm1 adds 2^n - 1, exact for the n that occur.
//   log1p(y) for y in (-0.5, 1]: log1p(y) = 2 atanh(s), s = y / (2 + y),
//     |s| <= 1/3, atanh series in s^2 through s^32 / 33.
//   reciprocals: hardware estimate refined by two Newton steps.
// Errors stay within 2 ulp on these ranges; NaN inputs propagate.
constexpr double kInvLn2 = 1.4426950408889634;
constexpr double kLn2Hi = 6.93147180369123816490e-01;
constexpr double kLn2Lo = 1.90821492927058770002e-10;

__device__ __forceinline__ double rcp_d(double b) {
  double r = __builtin_amdgcn_rcp(b);
  r = fma(r, fma(-b, r, 1.0), r);
  r = fma(r, fma(-b, r, 1.0), r);
  return r;
}

__device__ __forceinline__ double div_d(double a, double b) {
  const double r = rcp_d(b);
  const double q = a * r;
  return fma(r, fma(-b, q, a), q);
}

// Reduced argument and expm1 of it; n such that t = n ln2 + r.  Valid for
// t <= 700 (arguments below -800 are clamped; the results are then 0 / -1).
__device__ __forceinline__ double expm1_reduced(double t, double& n) {
  t = (t < -800.0) ? -800.0 : ((t > 700.0) ? 700.0 : t);
  n = rint(t * kInvLn2);
  const double r = fma(-n, kLn2Lo, fma(-n, kLn2Hi, t));
  constexpr double c13 = 1.0 / 6227020800.0, c12 = 1.0 / 479001600.0, c11 = 1.0 / 39916800.0,
                   c10 = 1.0 / 3628800.0, c9 = 1.0 / 362880.0, c8 = 1.0 / 40320.0, c7 = 1.0 / 5040.0,
                   c6 = 1.0 / 720.0, c5 = 1.0 / 120.0, c4 = 1.0 / 24.0, c3 = 1.0 / 6.0, c2 = 0.5;
  double p = fma(c13, r, c12);
  p = fma(p, r, c11);
  p = fma(p, r, c10);
  p = fma(p, r, c9);
  p = fma(p, r, c8);
  p = fma(p, r, c7);
  p = fma(p, r, c6);
  p = fma(p, r, c5);
  p = fma(p, r, c4);
  p = fma(p, r, c3);
  p = fma(p, r, c2);
  return fma(r * r, p, r);
}

__device__ __forceinline__ double exp_d(double t) {
  double n;
  const double q = expm1_reduced(t, n);
  return ldexp(1.0 + q, (int)n);
}

__device__ __forceinline__ double log1p_small(double y) {
  const double s = div_d(y, 2.0 + y);
  const double z = s * s;
  double p = fma(1.0 / 33.0, z, 1.0 / 31.0);
  p = fma(p, z, 1.0 / 29.0);
  p = fma(p, z, 1.0 / 27.0);
  p = fma(p, z, 1.0 / 25.0);
  p = fma(p, z, 1.0 / 23.0);
  p = fma(p, z, 1.0 / 21.0);
  p = fma(p, z, 1.0 / 19.0);
  p = fma(p, z, 1.0 / 17.0);
  p = fma(p, z, 1.0 / 15.0);
  p = fma(p, z, 1.0 / 13.0);
  p = fma(p, z, 1.0 / 11.0);
  p = fma(p, z, 1.0 / 9.0);
  p = fma(p, z, 1.0 / 7.0);
  p = fma(p, z, 1.0 / 5.0);
  p = fma(p, z, 1.0 / 3.0);
  const double ts = 2.0 * s;
  return fma(ts * z, p, ts);
}

// Increment form of the activations (used by the energy-network jets):
// softplus(a0 + d) - softplus(a0) and the logistic pair (s, 1 - s) at
// a = a0 + d, from s0 = logistic(a0) and sb0 = logistic(-a0), without branches.
// For a <= 0 the increment is log(w) with w = sb0 + s0 e^d = 1 + s0 expm1(d);
// for a > 0, by softplus(a) = a + softplus(-a), it is d + log(w) with
// w = s0 + sb0 e^-d.  Choosing the form by the sign of a keeps the increment
// free of cancellation (the logarithm carries the whole increment where the
// network is in its flat half), w is a sum of non-negative terms, and the
// logistic pair is (s0 e^d / w, sb0 / w) or (s0 / w, sb0 e^-d / w).  The
// split also keeps the result exact where |d| exceeds the exponent range: with
// a0 and a both large and positive (reference pre-activations of thousands
// occur in deep networks with large weights), sb0 underflows and the a > 0
// form returns d + log(s0) exactly, where the a <= 0 form alone would saturate.

// ---- table-driven variants, after the published methods of P. T. P. Tang
// ("Table-driven implementation of the exponential function in IEEE
// floating-point arithmetic", ACM TOMS 15(2), 1989, and "Table-driven
// implementation of the logarithm function in IEEE floating-point arithmetic",
// ACM TOMS 16(4), 1990): argument reduction against a table of 2^(j/64)
// (exponential) or of reciprocals of interval centres (logarithm), then a short
// polynomial.  The caller stages the kMathTabDoubles-entry table (exp: 64 x
// (Thi, Tlo); log: 64 x (1/c, log c hi, log c lo, 0); built on the host by
// build_math_tables) in LDS.
// exp / expm1: t = (64 n + j) ln2/64 + r with |r| <= ln2/128 (ln2/64 split so
// that the products with the integer multiple are exact), 2^(j/64) = Thi + Tlo
// from the table, expm1(r) by its Taylor series through r^6 (truncation below
// 1e-17 relative).  E = e^t = 2^n (Thi + tmp) and M = e^t - 1 =
// 2^n ((Thi - 2^-n) + tmp) with tmp = Thi expm1(r) + Tlo; Thi - 2^-n is exact
// (or dominated by the power of two), so M keeps relative precision at t -> 0.
// log1p: w = 2^e z with z in [0.6875, 1.375) by integer arithmetic on the high
// word; 64 intervals of z with 1/c_i from the table (exactly 1 on the two
// intervals next to 1), r = z / c_i - 1 by one fused rounding, |r| <= 1/64,
// log1p(r) by its series through r^9; log w = e ln2 + log c_i + log1p(r).  For
// y > -1/2 the argument is w = 1 + y with the exact rounding error of that sum
// added as err / w, so small |y| keep relative precision; otherwise an
// accurate w from the caller.  Table indices are masked to 0..63 whatever the
// input; NaN inputs propagate.
constexpr double kTabC1 = 0x1.62e42fefa0000p-7, kTabC2 = 0x1.cf79abc9e3b3ap-46;  // ln2/64
constexpr double kTabInv = 0x1.71547652b82fep+6;                                 // 64/ln2
constexpr double kLn2Hi32 = 0x1.62e42fee00000p-1, kLn2Lo32 = 0x1.a39ef35793c76p-33;

__device__ __forceinline__ void exp_expm1_tab(double t, const double* __restrict__ et, double& E, double& M) {
  t = fma(0.0, t, fmin(fmax(t, -700.0), 700.0));  // clamp; a NaN t stays NaN
  const double kk = rint(t * kTabInv);
  const int ki = (int)kk;
  const double r = fma(-kk, kTabC2, fma(-kk, kTabC1, t));
  const int j = ki & 63, n = ki >> 6;
  double q = fma(r, 1.0 / 720.0, 1.0 / 120.0);
  q = fma(q, r, 1.0 / 24.0);
  q = fma(q, r, 1.0 / 6.0);
  q = fma(q, r, 0.5);
  const double em = fma(r * r, q, r);
  const double thi = et[2 * j], tlo = et[2 * j + 1];
  const double tmp = fma(thi, em, tlo);
  E = ldexp(thi + tmp, n);
  M = ldexp((thi - ldexp(1.0, -n)) + tmp, n);
}

__device__ __forceinline__ double log1p_tab(double y, double wacc, double winv, const double* __restrict__ lt) {
  const bool small = y > -0.5;
  const double ws = 1.0 + y;
  const double w = small ? ws : wacc;
  const double err = small ? y - (ws - 1.0) : 0.0;
  const int hi = __double2hiint(w);
  const int tmp = hi - 0x3FE60000;
  const int e = tmp >> 20;
  const int i = (tmp >> 14) & 63;
  const double z = __hiloint2double(hi - (e << 20), __double2loint(w));
  const double invc = lt[4 * i], lhi = lt[4 * i + 1], llo = lt[4 * i + 2];
  const double r = fma(z, invc, -1.0);
  double q = fma(r, 1.0 / 9.0, -1.0 / 8.0);
  q = fma(q, r, 1.0 / 7.0);
  q = fma(q, r, -1.0 / 6.0);
  q = fma(q, r, 1.0 / 5.0);
  q = fma(q, r, -0.25);
  q = fma(q, r, 1.0 / 3.0);
  q = fma(q, r, -0.5);
  const double ed = (double)e;
  const double res = fma(ed, kLn2Hi32, lhi) + (fma(r * r, q, r) + fma(err, winv, fma(ed, kLn2Lo32, llo)));
  return fma(0.0, y, res);  // keeps a NaN y
}

// The increment form above with the table-driven exp / log1p.
__device__ __forceinline__ double delta_softplus_tab(double d, double a0, double s0, double sb0, double& s,
                                                     double& sb, const double* __restrict__ et,
                                                     const double* __restrict__ lt) {
  const bool fa = a0 + d <= 0.0;
  double E, M;
  exp_expm1_tab(fa ? d : -d, et, E, M);
  const double p = fa ? s0 : sb0, c = fa ? sb0 : s0;
  const double w = fma(p, E, c);
  // one Newton step on the hardware estimate (11 ulp): the reciprocal only
  // scales the logistic pair, the increment does not depend on it
  double inv = __builtin_amdgcn_rcp(w);
  inv = fma(inv, fma(-w, inv, 1.0), inv);
  const double sp = p * E * inv, sc = c * inv;
  s = fa ? sp : sc;
  sb = fa ? sc : sp;
  return (fa ? 0.0 : d) + log1p_tab(p * M, w, inv, lt);
}

// FP32 version for the mixed-precision jets (same forms, hardware exp / log /
// reciprocal; expm1 and log1p of small arguments by their Taylor / atanh
// series, so small increments keep relative precision).
__device__ __forceinline__ float delta_softplus(float d, float a0, float s0, float sb0, float& s, float& sb) {
  const bool fa = a0 + d <= 0.0f;
  const float t = fa ? d : -d;
  const float E = __expf(t);
  const float Ms =
      t * (1.0f + t * (0.5f + t * (1.0f / 6 + t * (1.0f / 24 + t * (1.0f / 120 + t * (1.0f / 720 + t * (1.0f / 5040)))))));
  const float M = (fabsf(t) < 0.25f) ? Ms : E - 1.0f;
  const float p = fa ? s0 : sb0, c = fa ? sb0 : s0;
  const float w = fmaf(p, E, c);
  const float inv = __builtin_amdgcn_rcpf(w);
  const float sp = p * E * inv, sc = c * inv;
  s = fa ? sp : sc;
  sb = fa ? sc : sp;
  const float y = p * M;
  const float u = y * __builtin_amdgcn_rcpf(2.0f + y);
  const float z = u * u;
  const float Ls = 2.0f * u * (1.0f + z * (1.0f / 3 + z * (1.0f / 5 + z * (1.0f / 7 + z * (1.0f / 9)))));
  const float Lg = (fabsf(y) < 0.25f) ? Ls : __logf(w);
  return (fa ? 0.0f : d) + Lg;
}

// Plain softplus and logistic (yield network, evaluated directly).
__device__ __forceinline__ double softplus_d(double a, double& s) {
  const double e = exp_d(-fabs(a));
  const double inv = rcp_d(1.0 + e);
  s = (a >= 0.0) ? inv : e * inv;
  return fmax(a, 0.0) + log1p_small(e);
}

// Make LDS writes of this wavefront visible to its own later reads, and keep
// the compiler from moving memory operations across this point.  No s_barrier:
// safe inside divergent control flow.
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Cross-lane move of a double within rows of the wavefront (DPP, no LDS).
template <int CTRL>
__device__ __forceinline__ double dpp_mov(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_mov_dpp((int)(b & 0xffffffffll), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// Sum over aligned groups of 8 lanes with DPP: swap neighbours (quad_perm
// 1,0,3,2), swap pairs (quad_perm 2,3,0,1), then add the mirrored half-row
// (the other quad of the 8).  Every lane of the group gets the same bits
// (each addition pairs two equal-shape partial sums, which commute).
__device__ __forceinline__ double group8_sum(double v) {
  v += dpp_mov<0xB1>(v);
  v += dpp_mov<0x4E>(v);
  v += dpp_mov<0x141>(v);
  return v;
}

}  // namespace gedmg
