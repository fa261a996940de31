// Closed-form constitutive model of Sec. 4.1: the compressible Neo-Hooke
// energy psi_NH = mu/2 (I1 - 3) - mu ln J + lambda/2 (ln J)^2 written as a
// function of the network inputs x = (I1G - 3, I2G - 3, J - 1) with
// I1 = J^(2/3) (x1 + 3) and J = 1 + x3, so that it drops into the slot of the
// energy network: the kernel writes the same jet row (value, gradient and
// Hessian in x), and the element and history kernels run unchanged with unit
// energy scale and no separate volumetric term.  The value vanishes at x = 0
// and so does its x3 slope (mu - mu = 0), which is the stress normality of the
// reference state.
//   N       = mu/2 (a (x1 + 3) - 3) - mu ln J + lambda/2 (ln J)^2,  a = J^(2/3)
//   N_1     = mu/2 a,  N_2 = 0
//   N_3     = mu/3 (x1 + 3) a / J - mu / J + lambda ln J / J
//   N_13    = mu/3 a / J,  N_11 = N_22 = N_12 = N_23 = 0
//   N_33    = -mu/9 (x1 + 3) a / J^2 + mu / J^2 + lambda (1 - ln J) / J^2
#include "gedmg_internal.h"

namespace gedmg {

__global__ __launch_bounds__(256) void closed_form_jet_kernel(JetArgs a) {
  const long g = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= a.nq) return;
  const double x1 = a.x[g * 3], x3 = a.x[g * 3 + 2];
  const double mu = a.cf_mu, lam = a.cf_lam;
  const double J = 1.0 + x3;
  const double iJ = 1.0 / J;
  const double cj = cbrt(J);
  const double aJ = cj * cj;  // J^(2/3)
  const double lnJ = log1p(x3);
  const double i1 = x1 + 3.0;
  double* o = a.jet + g * 10;
  // mu/2 (a i1 - 3) = mu/2 (a x1 + 3 (a - 1)); a - 1 = expm1(2/3 ln J) keeps
  // the increment's relative precision near J = 1
  o[0] = 0.5 * mu * (aJ * x1 + 3.0 * expm1((2.0 / 3.0) * lnJ)) - mu * lnJ + 0.5 * lam * lnJ * lnJ;
  o[1] = 0.5 * mu * aJ;
  o[2] = 0.0;
  o[3] = (mu / 3.0) * i1 * aJ * iJ - mu * iJ + lam * lnJ * iJ;
  o[4] = 0.0;
  o[5] = 0.0;
  o[6] = (-(mu / 9.0) * i1 * aJ + mu + lam * (1.0 - lnJ)) * iJ * iJ;
  o[7] = 0.0;
  o[8] = (mu / 3.0) * aJ * iJ;
  o[9] = 0.0;
}

hipError_t launch_closed_form_jet(const JetArgs& a, hipStream_t s) {
  const int blocks = (int)((a.nq + 255) / 256);
  if (blocks == 0) return hipSuccess;
  hipLaunchKernelGGL(closed_form_jet_kernel, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

}  // namespace gedmg
