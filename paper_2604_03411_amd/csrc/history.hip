// Local damage update (Sec. 3.2, Eq. dd_7): at every quadrature point the
// history variable kappa solves h(kappa) = N^(q(kappa)) - kappa = 0 when the
// trial state yields, with the driving force of Eqs. q_q_loc_q_nloc /
// ostwald_potential,
//   q(kappa) = psi_e + (gamma beta / eta) (phi - kappa) / f_d(kappa),
// f_d(kappa) = exp(-eta <kappa - kappa_d>) (Eq. degradation_function), and
// kappa = kappa_n otherwise.  The consistent tangent also needs the two
// sensitivities of the solution, d kappa / d psi_e and d kappa / d phi.
//
// One lane per quadrature point: the inputs are per-point scalars (psi_e from
// the energy jet and the invariant J - 1, phi interpolated by the quadrature-
// input kernel, kappa_n), so the yield network (Eq. Gq_NN) is evaluated whole
// in each lane and its neurons are independent instruction streams; the
// weights are wave-uniform and come through the scalar cache.
#include "device_common.h"
#include "gedmg_internal.h"

namespace gedmg {

// softplus(a) = max(a, 0) + log1p(e^-|a|) and the logistic s(a), with the
// table-driven exp and log1p (tables staged in LDS by the kernel); the argument
// of log1p is in (0, 1], where it keeps relative precision.
__device__ __forceinline__ double softplus_tab(double a, double& s, const double* __restrict__ et,
                                               const double* __restrict__ lt) {
  double E, M;
  exp_expm1_tab(-fabs(a), et, E, M);
  const double w = 1.0 + E;
  const double inv = rcp_d(w);
  s = (a >= 0.0) ? inv : E * inv;
  return fmax(a, 0.0) + log1p_tab(E, w, inv, lt);
}

// N^(q) - N^(0) and dN^/dq of the packed single-input yield network (input-
// convex layers with a skip connection from q, softplus activations).
template <int H, int L>
__device__ __forceinline__ double yield_eval_lane(const double* __restrict__ net, double yN0, double q,
                                                  double& dN, const double* __restrict__ et,
                                                  const double* __restrict__ lt) {
  if constexpr (L == 0) {  // closed-form model: G(q) = q (Eq. ostwald_potential)
    dN = 1.0;
    return q;
  } else {
    const int stride = H * H + 2 * H;  // Wz, Wx, b of one hidden layer
    const int owz = 2 * H + (L - 1) * stride;
    double pN = 0.0, pD = 0.0;
    if constexpr (L == 1) {
      // a single hidden layer: all of its weights fit in registers, and the
      // unrolled form lets the neurons' instruction streams interleave
      double z[H], zt[H];
#pragma unroll
      for (int n = 0; n < H; ++n) {
        const double w = net[n];
        double s;
        z[n] = softplus_tab(fma(w, q, net[H + n]), s, et, lt);
        zt[n] = s * w;
      }
#pragma unroll
      for (int n = 0; n < H; ++n) {
        pN = fma(net[owz + n], z[n], pN);
        pD = fma(net[owz + n], zt[n], pD);
      }
    } else {
      double z[H], zt[H];
#pragma unroll
      for (int n = 0; n < H; ++n) {
        const double w = net[n];
        double s;
        z[n] = softplus_tab(fma(w, q, net[H + n]), s, et, lt);
        zt[n] = s * w;
      }
#pragma unroll
      for (int k = 1; k < L - 1; ++k) {
        const double* Wz = net + 2 * H + (k - 1) * stride;
        const double* Wx = Wz + H * H;
        const double* b = Wx + H;
        double zn[H], ztn[H];
#pragma unroll
        for (int n = 0; n < H; ++n) {
          double acc = fma(Wx[n], q, b[n]);
          double acct = Wx[n];
#pragma unroll
          for (int m = 0; m < H; ++m) {
            acc = fma(Wz[n * H + m], z[m], acc);
            acct = fma(Wz[n * H + m], zt[m], acct);
          }
          double s;
          zn[n] = softplus_tab(acc, s, et, lt);
          ztn[n] = s * acct;
        }
#pragma unroll
        for (int n = 0; n < H; ++n) {
          z[n] = zn[n];
          zt[n] = ztn[n];
        }
      }
      // last hidden layer: one neuron per iteration of a rolled loop, so its
      // weight row is loaded when needed rather than held in registers, and its
      // activation goes straight into the output sums
      const double* Wz = net + 2 * H + (L - 2) * stride;
      const double* Wx = Wz + H * H;
      const double* b = Wx + H;
#pragma unroll 1
      for (int n = 0; n < H; ++n) {
        double acc = fma(Wx[n], q, b[n]);
        double acct = Wx[n];
#pragma unroll
        for (int m = 0; m < H; ++m) {
          acc = fma(Wz[n * H + m], z[m], acc);
          acct = fma(Wz[n * H + m], zt[m], acct);
        }
        double s;
        const double zv = softplus_tab(acc, s, et, lt);
        pN = fma(net[owz + n], zv, pN);
        pD = fma(net[owz + n], s * acct, pD);
      }
    }
    const double wx = net[owz + H];
    dN = pD + wx;
    return pN + wx * q + net[owz + H + 1] - yN0;
  }
}

// The same network in FP32 with the hardware exponential, logarithm and
// reciprocal (relative error about 1e-6): the model the FP32 pre-solve iterates on.
template <int H, int L>
__device__ __forceinline__ float yield_eval_lane_f32(const double* __restrict__ net, float yN0, float q,
                                                     float& dN) {
  const int stride = H * H + 2 * H;
  const int owz = 2 * H + (L - 1) * stride;
  auto sp = [](float t, float& s) {
    const float e = __expf(-fabsf(t));
    const float inv = __builtin_amdgcn_rcpf(1.0f + e);
    s = (t >= 0.0f) ? inv : e * inv;
    return fmaxf(t, 0.0f) + __logf(1.0f + e);
  };
  float pN = 0.0f, pD = 0.0f;
  if constexpr (L == 1) {
    float z[H], zt[H];
#pragma unroll
    for (int n = 0; n < H; ++n) {
      const float w = (float)net[n];
      float s;
      z[n] = sp(fmaf(w, q, (float)net[H + n]), s);
      zt[n] = s * w;
    }
#pragma unroll
    for (int n = 0; n < H; ++n) {
      pN = fmaf((float)net[owz + n], z[n], pN);
      pD = fmaf((float)net[owz + n], zt[n], pD);
    }
  } else {
    float z[H], zt[H];
#pragma unroll
    for (int n = 0; n < H; ++n) {
      const float w = (float)net[n];
      float s;
      z[n] = sp(fmaf(w, q, (float)net[H + n]), s);
      zt[n] = s * w;
    }
#pragma unroll
    for (int k = 1; k < L - 1; ++k) {
      const double* Wz = net + 2 * H + (k - 1) * stride;
      const double* Wx = Wz + H * H;
      const double* b = Wx + H;
      float zn[H], ztn[H];
#pragma unroll
      for (int n = 0; n < H; ++n) {
        float acc = fmaf((float)Wx[n], q, (float)b[n]);
        float acct = (float)Wx[n];
#pragma unroll
        for (int m = 0; m < H; ++m) {
          acc = fmaf((float)Wz[n * H + m], z[m], acc);
          acct = fmaf((float)Wz[n * H + m], zt[m], acct);
        }
        float s;
        zn[n] = sp(acc, s);
        ztn[n] = s * acct;
      }
#pragma unroll
      for (int n = 0; n < H; ++n) {
        z[n] = zn[n];
        zt[n] = ztn[n];
      }
    }
    const double* Wz = net + 2 * H + (L - 2) * stride;
    const double* Wx = Wz + H * H;
    const double* b = Wx + H;
#pragma unroll 1
    for (int n = 0; n < H; ++n) {
      float acc = fmaf((float)Wx[n], q, (float)b[n]);
      float acct = (float)Wx[n];
#pragma unroll
      for (int m = 0; m < H; ++m) {
        acc = fmaf((float)Wz[n * H + m], z[m], acc);
        acct = fmaf((float)Wz[n * H + m], zt[m], acct);
      }
      float s;
      const float zv = sp(acc, s);
      pN = fmaf((float)net[owz + n], zv, pN);
      pD = fmaf((float)net[owz + n], s * acct, pD);
    }
  }
  const float wx = (float)net[owz + H];
  dN = pD + wx;
  return pN + wx * q + (float)net[owz + H + 1] - yN0;
}

// FP32 pre-solve iterations (not counted against max_local).
constexpr int kF32Iters = 12;
// Acceptance of the FP64 local Newton iteration: a correction |dk| below
// kAcceptRel max(1, |k|) is applied without a further network evaluation (the
// error of k + dk is the curvature times dk^2, far below rounding); the
// bracket [lo, hi] counts as closed below kBracketRel max(1, |k|).
constexpr double kAcceptRel = 1e-13;
constexpr double kBracketRel = 1e-15;

template <int YH, int YL>
__global__ __launch_bounds__(256, YL <= 2 ? 2 : 1) void history_kernel(HistArgs a) {
  __shared__ double mt[kMathTabDoubles];  // exp table [64][2], then log table [64][4]
  for (int i = threadIdx.x; i < kMathTabDoubles; i += blockDim.x) mt[i] = a.mtab[i];
  __syncthreads();
  const double* et = mt;
  const double* lt = mt + 128;
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.nq) return;
  const Material M = a.m;
  if (a.frozen) {  // staggered scheme: the history stays at kappa_n during the global solve
    a.kappa_out[g] = a.kappa_n[g];
    a.sens[g * 2] = 0.0;
    a.sens[g * 2 + 1] = 0.0;
    return;
  }
  // psi_e at the point (Eq. dd_0): mu (N(x) - N(0) - n0 x3) + lam (J + 1/J - 2)^2
  const double x3 = a.x[g * 3 + 2];
  const double Jd = 1.0 + x3;
  const double vol = Jd + rcp_d(Jd) - 2.0;
  const double psi_e = M.mu * (a.jet[g * 10] - a.n0 * x3) + M.lam * vol * vol;
  const double phi = a.phiq[g];
  const double kn = a.kappa_n[g];

  const double gbe = M.gamma * M.beta / M.eta;  // q = psi_e + gbe (phi - kappa) / f_d(kappa)
  double kap = kn, dNy = 0.0;
  const double q0 = psi_e + gbe * (phi - kn) * exp_d(M.eta * fmax(kn - M.kd, 0.0));
  double d0;
  const double h0 = yield_eval_lane<YH, YL>(a.ynet, a.yN0, q0, d0, et, lt) - kn;
  dNy = d0;
  const bool yielded = h0 > 0.0;
  if (yielded) {
    // Bracket [lo, hi] with h(lo) > 0 >= h(hi): h(kappa_n) = h0 > 0, and on
    // kappa >= phi the driving force is at most psi_e, so h <= N^(psi_e) - kappa
    // there and any top >= max(kappa_n, phi, N^(psi_e)) closes the bracket.
    double lo = kn, hi, k = kn, h = h0;
    if constexpr (YL == 1) {
      // Single hidden layer: N^(psi_e) from the FP32 network with a margin far
      // above its error, and the root first located by safeguarded Newton on the
      // FP32 model; the FP64 iteration below starts there and decides convergence.
      const float psif = (float)psi_e, phif = (float)phi, gbef = (float)gbe;
      const float etaf = (float)M.eta, kdf = (float)M.kd, yN0f = (float)a.yN0;
      float dtopf;
      const float topf = yield_eval_lane_f32<YH, YL>(a.ynet, yN0f, psif, dtopf);
      const double top = (double)topf + 1e-4 * (1.0 + fabs((double)topf));
      hi = fmax(fmax(kn, phi), top);
      float lof = (float)lo, hif = (float)hi, kf = (float)kn;
      for (int it = 0; it < kF32Iters; ++it) {
        const float invf = __expf(fminf(etaf * fmaxf(kf - kdf, 0.0f), 80.0f));
        const float qf = psif + gbef * (phif - kf) * invf;
        float dNf;
        const float hf = yield_eval_lane_f32<YH, YL>(a.ynet, yN0f, qf, dNf) - kf;
        if (hf > 0.0f) lof = kf; else hif = kf;
        const float dqf = gbef * invf * (-1.0f + ((kf > kdf) ? etaf * (phif - kf) : 0.0f));
        float kn1 = kf - hf * __builtin_amdgcn_rcpf(dNf * dqf - 1.0f);
        if (!(kn1 > lof && kn1 < hif)) kn1 = 0.5f * (lof + hif);
        const bool done = fabsf(kn1 - kf) <= 1e-6f * fmaxf(1.0f, fabsf(kf));
        kf = kn1;
        if (done) break;
      }
      const double ks = (double)kf;
      if (ks > lo && ks < hi) {
        k = ks;
        const double qk = psi_e + gbe * (phi - k) * exp_d(M.eta * fmax(k - M.kd, 0.0));
        h = yield_eval_lane<YH, YL>(a.ynet, a.yN0, qk, dNy, et, lt) - k;
        if (h > 0.0) lo = k; else hi = k;
      }
    } else {
      // At kappa = phi the driving force is psi_e, so one evaluation gives both
      // h(phi) = N^(psi_e) - phi and the bracket top; with a large penalty the
      // root sits just above phi: start there when the yield condition still
      // holds at phi.
      double dtop;
      const double top = yield_eval_lane<YH, YL>(a.ynet, a.yN0, psi_e, dtop, et, lt);
      hi = fmax(fmax(kn, phi), top);
      if (phi > kn) {
        if (top - phi > 0.0) {
          lo = phi;
          k = phi;
          h = top - phi;
          dNy = dtop;
        } else {
          hi = phi;
        }
      }
    }
    bool conv = false;
    // Step sizes of the last two iterations: a Newton step longer than half the
    // step before the last one is replaced by bisection, so the bracket at
    // least halves every second iteration even when h is dominated by rounding
    // near the root (there the Newton corrections are noise).
    double step1 = hi - lo, step2 = hi - lo;
    double inv_f = exp_d(M.eta * fmax(k - M.kd, 0.0));  // 1 / f_d(k)
    for (int it = 0; it < a.max_local; ++it) {
      // Newton correction from the current iterate; the convergence test comes
      // before the bracket safeguard so that a root reached on the bracket's end
      // is accepted rather than bisected away from.
      const double dq = gbe * inv_f * (-1.0 + ((k > M.kd) ? M.eta * (phi - k) : 0.0));
      const double dk = div_d(-h, dNy * dq - 1.0);
      const double bracket_tol = kBracketRel * fmax(1.0, fabs(k));
      if (fabs(dk) <= kAcceptRel * fmax(1.0, fabs(k))) {
        k = fmin(fmax(k + dk, lo), hi);
        conv = true;
        break;
      }
      double kn1 = k + dk;
      step2 = step1;
      if (!(kn1 > lo && kn1 < hi) || 2.0 * fabs(dk) > step2) {
        kn1 = 0.5 * (lo + hi);
        step1 = 0.5 * (hi - lo);
      } else {
        step1 = fabs(dk);
      }
      k = kn1;
      inv_f = exp_d(M.eta * fmax(k - M.kd, 0.0));
      const double qk = psi_e + gbe * (phi - k) * inv_f;
      h = yield_eval_lane<YH, YL>(a.ynet, a.yN0, qk, dNy, et, lt) - k;
      if (h > 0.0) lo = k; else hi = k;
      if (h == 0.0 || !(hi - lo > bracket_tol)) { conv = true; break; }
    }
    if (!conv) a.status[0] = GEDMG_E_LOCAL_NOCONV;
    kap = k;
  }
  // Sensitivities of the local solution (implicit function theorem on h = 0):
  // d kappa / d psi_e = -N^' / h_kappa and d kappa / d phi = -N^' q_phi / h_kappa,
  // with h_kappa = N^' q_kappa - 1; both vanish on the elastic branch.
  double rhoF = 0.0, kphi = 0.0;
  if (yielded) {
    const double inv_f = exp_d(M.eta * fmax(kap - M.kd, 0.0));
    const double dq = gbe * inv_f * (-1.0 + ((kap > M.kd) ? M.eta * (phi - kap) : 0.0));
    const double ihk = rcp_d(dNy * dq - 1.0);
    rhoF = -dNy * ihk;
    kphi = -dNy * gbe * inv_f * ihk;
  }
  a.kappa_out[g] = kap;
  a.sens[g * 2] = rhoF;
  a.sens[g * 2 + 1] = kphi;
}

hipError_t launch_history(const HistArgs& a, int yH, hipStream_t s) {
  const int blocks = (int)((a.nq + 255) / 256);
  if (blocks == 0) return hipSuccess;
  const dim3 g(blocks), b(256);
  if (a.yL == 0) hipLaunchKernelGGL((history_kernel<0, 0>), g, b, 0, s, a);
  else if (yH == 16 && a.yL == 1) hipLaunchKernelGGL((history_kernel<16, 1>), g, b, 0, s, a);
  else if (yH == 16 && a.yL == 2) hipLaunchKernelGGL((history_kernel<16, 2>), g, b, 0, s, a);
  else if (yH == 16 && a.yL == 3) hipLaunchKernelGGL((history_kernel<16, 3>), g, b, 0, s, a);
  else if (yH == 32 && a.yL == 1) hipLaunchKernelGGL((history_kernel<32, 1>), g, b, 0, s, a);
  else if (yH == 32 && a.yL == 2) hipLaunchKernelGGL((history_kernel<32, 2>), g, b, 0, s, a);
  else if (yH == 32 && a.yL == 3) hipLaunchKernelGGL((history_kernel<32, 3>), g, b, 0, s, a);
  else return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace gedmg
