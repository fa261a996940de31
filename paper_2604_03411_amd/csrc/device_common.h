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

// softplus(a0 + d) - softplus(a0) and the logistic pair (s, 1 - s) at a0 + d,
// from a0 and s0 = logistic(a0), sb0 = logistic(-a0).  For increments that
// keep 1 + y above 1/2 the expm1/log1p form is used (relative precision of
// small increments, no overflow); larger increments (|d| of order one or more)
// take the direct difference, which then loses nothing.
template <typename T>
__device__ __forceinline__ T softplus_pair(T a, T& s, T& sb) {
  const T e = exp(-fabs(a));
  const T inv = T(1) / (T(1) + e);
  s = (a >= T(0)) ? inv : e * inv;
  sb = (a >= T(0)) ? e * inv : inv;
  return fmax(a, T(0)) + log1p(e);
}

template <typename T>
__device__ __forceinline__ T delta_softplus(T d, T a0, T s0, T sb0, T& s, T& sb) {
  const bool neg = d <= T(0);
  const T e = expm1(neg ? d : -d);
  const T y = (neg ? s0 : sb0) * e;
  if (y > T(-0.5)) {
    const T inv = T(1) / (T(1) + y);
    if (neg) {
      s = s0 * (T(1) + e) * inv;
      sb = sb0 * inv;
      return log1p(y);
    }
    s = s0 * inv;
    sb = sb0 * (T(1) + e) * inv;
    return d + log1p(y);
  }
  T s_ref, sb_ref;
  const T za = softplus_pair<T>(a0 + d, s, sb);
  return za - softplus_pair<T>(a0, s_ref, sb_ref);
}

// Plain softplus and logistic (yield network, evaluated directly).
__device__ __forceinline__ double softplus_d(double a, double& s) {
  const double e = exp(-fabs(a));
  const double inv = 1.0 / (1.0 + e);
  s = (a >= 0.0) ? inv : e * inv;
  return fmax(a, 0.0) + log1p(e);
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
