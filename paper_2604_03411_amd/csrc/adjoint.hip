// Load-path adjoint: gradient of L = sum_n (reaction_n - target_n)^2 with
// respect to the raw parameters of both networks, through the converged
// monolithic load path.  The paper motivates differentiating through the
// solver for design and inverse problems (Sec. 5); this is the discrete
// adjoint of the monolithic scheme of Sec. 3.2.
//
// With abar_n = dL_{>n}/dkappa_n per quadrature point, for n = N..1:
//   K_T^T lambda = d/dU [ell_n + abar_n . kappa_n]                on free dofs
//   dL/dtheta  += d/dtheta      [ell_n + abar_n . kappa_n - lambda . R]
//   abar_{n-1}  = d/dkappa_{n-1} [ell_n + abar_n . kappa_n - lambda . R]
// where R is the residual written as a function of (U_n, kappa_{n-1}, theta)
// through the history update kappa_n = kappa(z, kappa_{n-1}).
//
// Per quadrature point, with the cotangent c of R (c = 2 (r_n - t_n) on the
// reaction dofs, -lambda on the free dofs) and zeta = Jw B c_e:
//   s = zeta . dP/dkappa + abar_n = f_d' zeta_F . psi_e,F - beta_d zeta_phi + abar_n
//   yielded (kappa_n > kappa_{n-1}): dkappa = -dh/h_kappa, abar_{n-1} = 0
//   elastic:                         dkappa = dkappa_{n-1}, abar_{n-1} = s
// and the parameters receive the vector-Jacobian products of
//   c0 N(x) + omega . grad_x N(x)     energy network, omega_i = mu_e f_d zeta_F . dx_i/dF,
//                                     c0 = mu_e N^_kappa'(q) (-s / h_kappa)
//   c_y N_kappa(q)                    yield network, c_y = -s / h_kappa
// plus the reference-state terms N(0), dN/dx_3(0) (energy) and N_kappa(0)
// (yield), which are one extra row at zero input with the summed cotangents.
//
// Everything is deterministic (per-colour element order, fixed-order sums), so
// a segment recomputed from its checkpoint reproduces the forward states bit
// for bit and the checkpointed gradient equals the store-all gradient.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <vector>

#include "device_common.h"
#include "gedmg_internal.h"

namespace gedmg {
namespace {

constexpr int kMaxYieldWidth = 32;
constexpr int kChunks = 64;  // row chunks of the parameter-gradient reduction
constexpr int kRefinePasses = 2;  // iterative refinement of each adjoint solve

template <int DIM>
struct ATr;
template <>
struct ATr<3> { static constexpr int NEN = 8, NQP = 8, ND = 4; };
template <>
struct ATr<2> { static constexpr int NEN = 4, NQP = 4, ND = 3; };

struct AdjQpArgs {
  const double* X;
  const int32_t* conn;
  const int32_t* perm;
  int e_begin, e_end;
  const double* u;
  const double* phi;
  const double* kappa_prev;  // [nq] kappa_{n-1}
  const double* kappa_cur;   // [nq] kappa_n at (U_n, kappa_{n-1})
  const double* jet;         // [nq][10] FP64 energy jets at U_n
  const double* ynet;        // packed yield network
  const double* abar;        // [nq] abar_n
  const double* cR;          // [ndof] cotangent of R (mode 1)
  double* gU;                // [ndof] += sum_q abar_q B^T dkappa/dz (mode 0)
  double* abar_prev;         // [nq] (mode 1)
  double* erow;              // [nq][7] x(3), omega(3), c0 (mode 1)
  double* yrow;              // [nq][2] q, c_y (mode 1)
  int n_nodes;
  Material m;
  double n0, yN0;
  int yH, yL, mode;
};

// Yield network N_kappa(q) - N_kappa(0) and dN/dq, one thread.
__device__ double yield_serial(const double* __restrict__ net, int H, int L, double yN0, double q, double& dN) {
  const NetLayout lay = make_layout_hd(1, H, L, 1);
  double z[kMaxYieldWidth], zt[kMaxYieldWidth];
  for (int n = 0; n < H; ++n) {
    double s;
    const double w = net[lay.W0 + n];
    z[n] = softplus_d(w * q + net[lay.b0 + n], s);
    zt[n] = s * w;
  }
  for (int k = 1; k < L; ++k) {
    double z2[kMaxYieldWidth], zt2[kMaxYieldWidth];
    for (int n = 0; n < H; ++n) {
      const double wx = net[lay.Wx[k] + n];
      double a = wx * q + net[lay.b[k] + n], at = wx;
      for (int m = 0; m < H; ++m) {
        const double w = net[lay.Wz[k] + n * H + m];
        a = fma(w, z[m], a);
        at = fma(w, zt[m], at);
      }
      double s;
      z2[n] = softplus_d(a, s);
      zt2[n] = s * at;
    }
    for (int n = 0; n < H; ++n) {
      z[n] = z2[n];
      zt[n] = zt2[n];
    }
  }
  double N = net[lay.bout] + net[lay.wx] * q, D = net[lay.wx];
  for (int n = 0; n < H; ++n) {
    N = fma(net[lay.wz + n], z[n], N);
    D = fma(net[lay.wz + n], zt[n], D);
  }
  dN = D;
  return N - yN0;
}

// One thread per element of a colour.  mode 0: gU += sum_q abar_q B^T kappa_z
// (elements of one colour share no node, so the read-modify-write is race
// free).  mode 1: per-point cotangents, abar_{n-1} and the network rows.
template <int DIM>
__global__ __launch_bounds__(64) void adj_qp_kernel(AdjQpArgs a) {
  using T = ATr<DIM>;
  const int pe = a.e_begin + blockIdx.x * blockDim.x + threadIdx.x;
  if (pe >= a.e_end) return;
  const int e = a.perm[pe];
  const Material M = a.m;
  int nodes[T::NEN];
  double Xe[T::NEN][DIM], ue[T::NEN][DIM], phie[T::NEN];
  for (int n = 0; n < T::NEN; ++n) {
    nodes[n] = a.conn[(long)e * T::NEN + n];
    for (int d = 0; d < DIM; ++d) {
      Xe[n][d] = a.X[(long)d * a.n_nodes + nodes[n]];
      ue[n][d] = a.u[(long)d * a.n_nodes + nodes[n]];
    }
    phie[n] = a.phi[nodes[n]];
  }
  double gloc[T::NEN][T::ND];
  for (int n = 0; n < T::NEN; ++n)
    for (int c = 0; c < T::ND; ++c) gloc[n][c] = 0.0;
  const double gb = M.gamma * M.beta;
  for (int q = 0; q < T::NQP; ++q) {
    const long qg = (long)e * T::NQP + q;
    const double kn = a.kappa_prev[qg], kap = a.kappa_cur[qg];
    const bool yielded = kap > kn;
    if (a.mode == 0 && (!yielded || a.abar[qg] == 0.0)) continue;
    // reference gradients and the Jacobian of the isoparametric map
    double Nv[T::NEN], dN[T::NEN][DIM], Jx[DIM][DIM];
    for (int d = 0; d < DIM; ++d)
      for (int k = 0; k < DIM; ++k) Jx[d][k] = 0.0;
    for (int n = 0; n < T::NEN; ++n) {
      shape_at<DIM>(n, q, Nv[n], dN[n]);
      for (int d = 0; d < DIM; ++d)
        for (int k = 0; k < DIM; ++k) Jx[d][k] += Xe[n][d] * dN[n][k];
    }
    double Ji[DIM][DIM], det;
    if constexpr (DIM == 2) {
      det = Jx[0][0] * Jx[1][1] - Jx[0][1] * Jx[1][0];
      const double id = 1.0 / det;
      Ji[0][0] = Jx[1][1] * id;
      Ji[0][1] = -Jx[0][1] * id;
      Ji[1][0] = -Jx[1][0] * id;
      Ji[1][1] = Jx[0][0] * id;
    } else {
      const double c00 = Jx[1][1] * Jx[2][2] - Jx[1][2] * Jx[2][1];
      const double c01 = Jx[1][2] * Jx[2][0] - Jx[1][0] * Jx[2][2];
      const double c02 = Jx[1][0] * Jx[2][1] - Jx[1][1] * Jx[2][0];
      det = Jx[0][0] * c00 + Jx[0][1] * c01 + Jx[0][2] * c02;
      const double id = 1.0 / det;
      Ji[0][0] = c00 * id;
      Ji[1][0] = c01 * id;
      Ji[2][0] = c02 * id;
      Ji[0][1] = (Jx[0][2] * Jx[2][1] - Jx[0][1] * Jx[2][2]) * id;
      Ji[1][1] = (Jx[0][0] * Jx[2][2] - Jx[0][2] * Jx[2][0]) * id;
      Ji[2][1] = (Jx[0][1] * Jx[2][0] - Jx[0][0] * Jx[2][1]) * id;
      Ji[0][2] = (Jx[0][1] * Jx[1][2] - Jx[0][2] * Jx[1][1]) * id;
      Ji[1][2] = (Jx[0][2] * Jx[1][0] - Jx[0][0] * Jx[1][2]) * id;
      Ji[2][2] = (Jx[0][0] * Jx[1][1] - Jx[0][1] * Jx[1][0]) * id;
    }
    // spatial gradients G[n][d] = dN_n/dX_d (component 2 zero in plane strain)
    double G[T::NEN][3];
    for (int n = 0; n < T::NEN; ++n)
      for (int d = 0; d < 3; ++d) {
        double g = 0.0;
        if (d < DIM)
          for (int k = 0; k < DIM; ++k) g += Ji[k][d] * dN[n][k];
        G[n][d] = g;
      }
    double F[9] = {1, 0, 0, 0, 1, 0, 0, 0, 1}, phi = 0.0;
    for (int n = 0; n < T::NEN; ++n) {
      for (int i = 0; i < DIM; ++i)
        for (int d = 0; d < DIM; ++d) F[i * 3 + d] += ue[n][i] * G[n][d];
      phi += phie[n] * Nv[n];
    }
    // cofactor A = dJ/dF, C = F^T F, invariants, Q = dI2/dF
    double A[9];
    A[0] = F[4] * F[8] - F[5] * F[7];
    A[1] = F[5] * F[6] - F[3] * F[8];
    A[2] = F[3] * F[7] - F[4] * F[6];
    A[3] = F[2] * F[7] - F[1] * F[8];
    A[4] = F[0] * F[8] - F[2] * F[6];
    A[5] = F[1] * F[6] - F[0] * F[7];
    A[6] = F[1] * F[5] - F[2] * F[4];
    A[7] = F[2] * F[3] - F[0] * F[5];
    A[8] = F[0] * F[4] - F[1] * F[3];
    const double J = F[0] * A[0] + F[1] * A[1] + F[2] * A[2];
    const double iJ = 1.0 / J;
    double C[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) C[i * 3 + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
    const double I1 = C[0] + C[4] + C[8];
    double CC = 0.0;
    for (int t = 0; t < 9; ++t) CC += C[t] * C[t];
    const double I2 = 0.5 * (I1 * I1 - CC);
    double Q[9];
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j)
        Q[i * 3 + j] =
            2.0 * (I1 * F[i * 3 + j] - (F[i * 3] * C[j] + F[i * 3 + 1] * C[3 + j] + F[i * 3 + 2] * C[6 + j]));
    const double cj = cbrt(J);
    const double Jm23 = 1.0 / (cj * cj), Jm53 = Jm23 * iJ, Jm4 = iJ * iJ * iJ * iJ, Jm5 = Jm4 * iJ;
    // dx_1/dF, dx_2/dF (dx_3/dF = A)
    double x1F[9], x2F[9];
    for (int r = 0; r < 9; ++r) {
      x1F[r] = 2.0 * Jm23 * F[r] - (2.0 / 3.0) * I1 * Jm53 * A[r];
      x2F[r] = (1.0 / 3.0) * I2 * I2 * Jm4 * Q[r] - (4.0 / 9.0) * I2 * I2 * I2 * Jm5 * A[r];
    }
    // psi_e,F = mu_e (dN/dx_i - n0 delta_i3) dx_i/dF + lambda_e 2 v (1 - J^-2) A, v = J + 1/J - 2
    const double* jt = a.jet + qg * 10;
    const double m0 = jt[1], m1 = jt[2], m2 = jt[3] - a.n0;
    const double vol = J + iJ - 2.0;
    const double pv1 = 2.0 * vol * (1.0 - iJ * iJ);
    const double x3 = J - 1.0;
    double psiF[9];
    for (int r = 0; r < 9; ++r) psiF[r] = M.mu * (m0 * x1F[r] + m1 * x2F[r] + m2 * A[r]) + M.lam * pv1 * A[r];
    const double psi_e = M.mu * (jt[0] - a.n0 * x3) + M.lam * vol * vol;
    // history sensitivities at the converged kappa_n (Eqs. Gq_NN, dd_7)
    const double f = exp_d(-M.eta * fmax(kap - M.kd, 0.0));
    const double fp = (kap > M.kd) ? -M.eta * f : 0.0;
    const double qk = psi_e + gb * (phi - kap) / (M.eta * f);
    double hk = -1.0, dNy = 0.0;
    if (yielded) {
      (void)yield_serial(a.ynet, a.yH, a.yL, a.yN0, qk, dNy);
      const double dq = gb / (M.eta * f) * (-1.0 + ((kap > M.kd) ? M.eta * (phi - kap) : 0.0));
      hk = dNy * dq - 1.0;
    }
    if (a.mode == 0) {
      // kappa_F = -N^' psi_e,F / h_kappa, kappa_phi = -N^' gamma beta / (eta f) / h_kappa
      const double ab = a.abar[qg];
      const double rhoF = -dNy / hk;
      const double kphi = -dNy * gb / (M.eta * f) / hk;
      for (int n = 0; n < T::NEN; ++n) {
        for (int i = 0; i < DIM; ++i) {
          double t = 0.0;
          for (int d = 0; d < DIM; ++d) t += psiF[i * 3 + d] * G[n][d];
          gloc[n][i] += ab * rhoF * t;
        }
        gloc[n][DIM] += ab * kphi * Nv[n];
      }
      continue;
    }
    // mode 1: zeta = Jw B c_e (Gauss weights 1)
    double zF[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, zphi = 0.0;
    for (int n = 0; n < T::NEN; ++n) {
      const double* cr = a.cR + (long)nodes[n] * T::ND;
      for (int i = 0; i < DIM; ++i)
        for (int d = 0; d < DIM; ++d) zF[i * 3 + d] += det * cr[i] * G[n][d];
      zphi += det * cr[DIM] * Nv[n];
    }
    double zpsi = 0.0, t0 = 0.0, t1 = 0.0, t2 = 0.0;
    for (int r = 0; r < 9; ++r) {
      zpsi += zF[r] * psiF[r];
      t0 += zF[r] * x1F[r];
      t1 += zF[r] * x2F[r];
      t2 += zF[r] * A[r];
    }
    const double s = fp * zpsi - M.beta * zphi + a.abar[qg];
    double c0 = 0.0, cy = 0.0;
    if (yielded) {
      cy = -s / hk;
      c0 = M.mu * dNy * cy;
    }
    a.abar_prev[qg] = yielded ? 0.0 : s;
    double* er = a.erow + qg * 7;
    er[0] = I1 * Jm23 - 3.0;
    er[1] = I2 * I2 * I2 / (9.0 * J * J * J * J) - 3.0;
    er[2] = x3;
    er[3] = M.mu * f * t0;
    er[4] = M.mu * f * t1;
    er[5] = M.mu * f * t2;
    er[6] = c0;
    a.yrow[qg * 2] = qk;
    a.yrow[qg * 2 + 1] = cy;
  }
  if (a.mode == 0) {
    for (int n = 0; n < T::NEN; ++n)
      for (int c = 0; c < T::ND; ++c) a.gU[(long)nodes[n] * T::ND + c] += gloc[n][c];
  }
}

// Reference-state row: N(0) receives -sum c0, dN/dx_3(0) receives
// -sum (c0 x_3 + omega_3), N_kappa(0) receives -sum c_y.  Fixed-order sums:
// 256 block partials, then one thread per quantity.
__global__ void ref_partial_kernel(const double* erow, const double* yrow, long nq, double* part) {
  __shared__ double sh[3][256];
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < nq; i += (long)gridDim.x * blockDim.x) {
    const double* e = erow + i * 7;
    s0 -= e[6];
    s1 -= e[6] * e[2] + e[5];
    s2 -= yrow[i * 2 + 1];
  }
  sh[0][threadIdx.x] = s0;
  sh[1][threadIdx.x] = s1;
  sh[2][threadIdx.x] = s2;
  __syncthreads();
  if (threadIdx.x < 3) {
    double t = 0.0;
    for (int j = 0; j < (int)blockDim.x; ++j) t += sh[threadIdx.x][j];
    part[threadIdx.x * gridDim.x + blockIdx.x] = t;
  }
}

__global__ void ref_rows_kernel(const double* part, int nb, double* erow_ref, double* yrow_ref) {
  if (threadIdx.x != 0) return;
  double t[3];
  for (int k = 0; k < 3; ++k) {
    double s = 0.0;
    for (int b = 0; b < nb; ++b) s += part[k * nb + b];
    t[k] = s;
  }
  for (int k = 0; k < 5; ++k) erow_ref[k] = 0.0;
  erow_ref[5] = t[1];
  erow_ref[6] = t[0];
  yrow_ref[0] = 0.0;
  yrow_ref[1] = t[2];
}

// Energy network, one row per thread: forward value and tangent in direction
// omega, then the reverse pass of y = c0 N(x) + omega . grad_x N(x).
// state [row][L][4][H]: z, t (tangent), then abar and tbar (adjoints of the
// pre-activation and of its tangent), which overwrite a and at.
__global__ void energy_vjp_kernel(const double* __restrict__ net, NetLayout lay, const double* rows, int nrow,
                                  double* state) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrow) return;
  const int H = lay.H, L = lay.L;
  const double* x = rows + (long)r * 7;
  const double* om = x + 3;
  const double c0 = x[6];
  double* st = state + (long)r * L * 4 * H;
  for (int n = 0; n < H; ++n) {
    const double* w = net + lay.W0 + n * 3;
    const double a0 = w[0] * x[0] + w[1] * x[1] + w[2] * x[2] + net[lay.b0 + n];
    const double at = w[0] * om[0] + w[1] * om[1] + w[2] * om[2];
    double s;
    st[n] = softplus_d(a0, s);
    st[H + n] = s * at;
    st[2 * H + n] = a0;
    st[3 * H + n] = at;
  }
  for (int k = 1; k < L; ++k) {
    const double* sp = st + (k - 1) * 4 * H;
    double* sk = st + k * 4 * H;
    for (int n = 0; n < H; ++n) {
      const double* wz = net + lay.Wz[k] + n * H;
      const double* wx = net + lay.Wx[k] + n * 3;
      double a0 = wx[0] * x[0] + wx[1] * x[1] + wx[2] * x[2] + net[lay.b[k] + n];
      double at = wx[0] * om[0] + wx[1] * om[1] + wx[2] * om[2];
      for (int m = 0; m < H; ++m) {
        a0 = fma(wz[m], sp[m], a0);
        at = fma(wz[m], sp[H + m], at);
      }
      double s;
      sk[n] = softplus_d(a0, s);
      sk[H + n] = s * at;
      sk[2 * H + n] = a0;
      sk[3 * H + n] = at;
    }
  }
  for (int k = L - 1; k >= 0; --k) {
    double* sk = st + k * 4 * H;
    const double* sn = st + (k + 1) * 4 * H;  // read only for k < L - 1: abar, tbar of layer k + 1
    for (int n = 0; n < H; ++n) {
      double zb, tb;
      if (k == L - 1) {
        zb = c0 * net[lay.wz + n];
        tb = net[lay.wz + n];
      } else {
        zb = 0.0;
        tb = 0.0;
        for (int m = 0; m < H; ++m) {
          const double w = net[lay.Wz[k + 1] + m * H + n];
          zb = fma(w, sn[2 * H + m], zb);
          tb = fma(w, sn[3 * H + m], tb);
        }
      }
      double s;
      (void)softplus_d(sk[2 * H + n], s);
      const double at = sk[3 * H + n];
      sk[2 * H + n] = zb * s + tb * s * (1.0 - s) * at;
      sk[3 * H + n] = tb * s;
    }
  }
}

// Yield network, one row per thread: y = c_y N_kappa(q).
// state [row][L][2][H]: z, then abar (overwrites the pre-activation).
__global__ void yield_vjp_kernel(const double* __restrict__ net, NetLayout lay, const double* rows, int nrow,
                                 double* state) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrow) return;
  const int H = lay.H, L = lay.L;
  const double q = rows[(long)r * 2], cy = rows[(long)r * 2 + 1];
  double* st = state + (long)r * L * 2 * H;
  for (int n = 0; n < H; ++n) {
    const double a0 = net[lay.W0 + n] * q + net[lay.b0 + n];
    double s;
    st[n] = softplus_d(a0, s);
    st[H + n] = a0;
  }
  for (int k = 1; k < L; ++k) {
    const double* sp = st + (k - 1) * 2 * H;
    double* sk = st + k * 2 * H;
    for (int n = 0; n < H; ++n) {
      double a0 = net[lay.Wx[k] + n] * q + net[lay.b[k] + n];
      for (int m = 0; m < H; ++m) a0 = fma(net[lay.Wz[k] + n * H + m], sp[m], a0);
      double s;
      sk[n] = softplus_d(a0, s);
      sk[H + n] = a0;
    }
  }
  for (int k = L - 1; k >= 0; --k) {
    double* sk = st + k * 2 * H;
    const double* sn = st + (k + 1) * 2 * H;
    for (int n = 0; n < H; ++n) {
      double zb;
      if (k == L - 1) {
        zb = cy * net[lay.wz + n];
      } else {
        zb = 0.0;
        for (int m = 0; m < H; ++m) zb = fma(net[lay.Wz[k + 1] + m * H + n], sn[H + m], zb);
      }
      double s;
      (void)softplus_d(sk[H + n], s);
      sk[H + n] = zb * s;
    }
  }
}

// Which array of a packed layout a parameter index falls in.
struct ParamRef {
  int kind;  // 0 W0, 1 b0, 2 Wz, 3 Wx, 4 b, 5 wz, 6 wx, 7 b_out
  int k, n, m;
};

__device__ ParamRef decode_param(const NetLayout& lay, int p) {
  const int H = lay.H, ni = lay.n_in;
  ParamRef r{7, 0, 0, 0};
  if (p < lay.b0) {
    r = ParamRef{0, 0, p / ni, p % ni};
  } else if (p < lay.b0 + H) {
    r = ParamRef{1, 0, p - lay.b0, 0};
  } else if (p >= lay.wz) {
    if (p < lay.wz + H)
      r = ParamRef{5, 0, p - lay.wz, 0};
    else if (p < lay.wx + ni)
      r = ParamRef{6, 0, 0, p - lay.wx};
  } else {
    for (int k = 1; k < lay.L; ++k) {
      if (p >= lay.Wz[k] && p < lay.Wz[k] + H * H)
        r = ParamRef{2, k, (p - lay.Wz[k]) / H, (p - lay.Wz[k]) % H};
      else if (p >= lay.Wx[k] && p < lay.Wx[k] + H * ni)
        r = ParamRef{3, k, (p - lay.Wx[k]) / ni, (p - lay.Wx[k]) % ni};
      else if (p >= lay.b[k] && p < lay.b[k] + H)
        r = ParamRef{4, k, p - lay.b[k], 0};
    }
  }
  return r;
}

// Partial gradients of the effective energy weights over a chunk of rows:
// part[chunk][param].  The output bias cancels exactly in N(x) - N(0).
__global__ void energy_grad_kernel(NetLayout lay, const double* rows, const double* state, int nrow,
                                   double* part) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = lay.n_raw;
  if (p >= np) return;
  const int ch = blockIdx.y, nch = gridDim.y;
  const int r0 = (int)((long)nrow * ch / nch), r1 = (int)((long)nrow * (ch + 1) / nch);
  const int H = lay.H, S = lay.L * 4 * H;
  const ParamRef pr = decode_param(lay, p);
  double acc = 0.0;
  if (pr.kind != 7) {
    for (int r = r0; r < r1; ++r) {
      const double* x = rows + (long)r * 7;
      const double* st = state + (long)r * S;
      const double* sk = st + pr.k * 4 * H;
      switch (pr.kind) {
        case 0:
        case 3: acc += sk[2 * H + pr.n] * x[pr.m] + sk[3 * H + pr.n] * x[3 + pr.m]; break;
        case 1:
        case 4: acc += sk[2 * H + pr.n]; break;
        case 2: {
          const double* sp = sk - 4 * H;
          acc += sk[2 * H + pr.n] * sp[pr.m] + sk[3 * H + pr.n] * sp[H + pr.m];
          break;
        }
        case 5: {
          const double* sl = st + (lay.L - 1) * 4 * H;
          acc += x[6] * sl[pr.n] + sl[H + pr.n];
          break;
        }
        case 6: acc += x[6] * x[pr.m] + x[3 + pr.m]; break;
        default: break;
      }
    }
  }
  part[(long)ch * np + p] = acc;
}

__global__ void yield_grad_kernel(NetLayout lay, const double* rows, const double* state, int nrow,
                                  double* part) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int np = lay.n_raw;
  if (p >= np) return;
  const int ch = blockIdx.y, nch = gridDim.y;
  const int r0 = (int)((long)nrow * ch / nch), r1 = (int)((long)nrow * (ch + 1) / nch);
  const int H = lay.H, S = lay.L * 2 * H;
  const ParamRef pr = decode_param(lay, p);
  double acc = 0.0;
  if (pr.kind != 7) {
    for (int r = r0; r < r1; ++r) {
      const double q = rows[(long)r * 2], cy = rows[(long)r * 2 + 1];
      const double* st = state + (long)r * S;
      const double* sk = st + pr.k * 2 * H;
      switch (pr.kind) {
        case 0:
        case 3: acc += sk[H + pr.n] * q; break;
        case 1:
        case 4: acc += sk[H + pr.n]; break;
        case 2: acc += sk[H + pr.n] * (sk - 2 * H)[pr.m]; break;
        case 5: acc += cy * st[(lay.L - 1) * 2 * H + pr.n]; break;
        case 6: acc += cy * q; break;
        default: break;
      }
    }
  }
  part[(long)ch * np + p] = acc;
}

__global__ void chunk_sum_kernel(const double* part, int nch, int np, double* out) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  double s = 0.0;
  for (int c = 0; c < nch; ++c) s += part[(long)c * np + p];
  out[p] += s;
}

__global__ void transpose_values_kernel(const double* K, const int32_t* permT, double* KT, long nnz) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nnz) KT[i] = K[permT[i]];
}

// e = indicator of the reaction dofs (distinct, in range: checked on the host).
__global__ void indicator_kernel(double* e, const int32_t* rd, int nr) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nr) e[rd[i]] = 1.0;
}

// b = gU + cr * y (the solver ignores prescribed rows)
__global__ void adj_rhs_kernel(const double* gU, const double* y, double cr, double* b, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = gU[i] + cr * y[i];
}

// cR = cr e - lambda (lambda is zero on prescribed dofs)
__global__ void adj_cot_kernel(const double* lam, const double* e, double cr, double* cR, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) cR[i] = cr * e[i] - lam[i];
}

double softplus_prime_h(double t) {
  const double e = std::exp(-std::fabs(t));
  return t >= 0 ? 1.0 / (1.0 + e) : e / (1.0 + e);
}

// Chain rule from effective (packed) to raw parameters.
void raw_chain(const NetLayout& lay, const double* raw, const double* geff, double* graw) {
  const int H = lay.H, ni = lay.n_in;
  auto pass = [&](double t, int i) { return ((lay.mask >> i) & 1) ? softplus_prime_h(t) : 1.0; };
  for (int p = 0; p < lay.n_raw; ++p) graw[p] = geff[p];
  for (int r = 0; r < H; ++r)
    for (int i = 0; i < ni; ++i) graw[lay.W0 + r * ni + i] *= pass(raw[lay.W0 + r * ni + i], i);
  for (int k = 1; k < lay.L; ++k) {
    for (int t = 0; t < H * H; ++t) graw[lay.Wz[k] + t] *= softplus_prime_h(raw[lay.Wz[k] + t]);
    for (int r = 0; r < H; ++r)
      for (int i = 0; i < ni; ++i) graw[lay.Wx[k] + r * ni + i] *= pass(raw[lay.Wx[k] + r * ni + i], i);
  }
  for (int r = 0; r < H; ++r) graw[lay.wz + r] *= softplus_prime_h(raw[lay.wz + r]);
  for (int i = 0; i < ni; ++i) graw[lay.wx + i] *= pass(raw[lay.wx + i], i);
}

#define AH(expr)                                                      \
  do {                                                                \
    hipError_t e_ = (expr);                                           \
    if (e_ != hipSuccess) {                                           \
      c->err = std::string(#expr) + ": " + hipGetErrorString(e_);     \
      return GEDMG_E_HIP;                                             \
    }                                                                 \
  } while (0)

// Device buffers of one adjoint call, freed on every return path.
struct Buffers {
  std::vector<void*> owned;
  gedmg_ctx* c;
  explicit Buffers(gedmg_ctx* ctx) : c(ctx) {}
  ~Buffers() {
    (void)hipStreamSynchronize(c->stream);
    for (void* p : owned) (void)hipFree(p);
  }
  template <typename T>
  bool get(T** p, size_t n) {
    if (hipMalloc((void**)p, sizeof(T) * std::max<size_t>(n, 1)) != hipSuccess) {
      *p = nullptr;
      return false;
    }
    owned.push_back(*p);
    return true;
  }
};

inline dim3 grid1(long n, int b = 256) { return dim3((unsigned)((n + b - 1) / b)); }

}  // namespace
}  // namespace gedmg

using namespace gedmg;

extern "C" int gedmg_adjoint(gedmg_ctx* c, int32_t n_steps, const gedmg_dirichlet* bc_per_step,
                             const double* predictor_du, const int32_t* reaction_dofs, int32_t n_reaction,
                             const double* targets, int32_t checkpoint_every, const gedmg_solver_opts* opts_in,
                             double* u, double* phi, double* kappa, double* loss, double* grad_energy,
                             double* grad_yield, gedmg_adjoint_report* rep) {
  if (!c) return GEDMG_E_ARG;
  if (n_steps <= 0 || !bc_per_step || !reaction_dofs || n_reaction <= 0 || !targets || !u || !phi ||
      !kappa || !loss || !grad_energy || !grad_yield) {
    c->err = "null or inconsistent adjoint argument";
    return GEDMG_E_ARG;
  }
  if (c->closed_energy || c->closed_yield) {
    c->err = "the adjoint differentiates network parameters; the closed-form model has none";
    return GEDMG_E_SHAPE;
  }
  if (c->ylay.H > kMaxYieldWidth) {
    c->err = "yield-network width above 32 is not supported by the adjoint";
    return GEDMG_E_SHAPE;
  }
  gedmg_solver_opts o = default_solver_opts();
  if (opts_in) o = *opts_in;
  gedmg_adjoint_report local{};
  gedmg_adjoint_report& R = rep ? *rep : local;
  R = gedmg_adjoint_report{};
  const int ce = (checkpoint_every <= 0 || checkpoint_every > n_steps) ? n_steps : checkpoint_every;
  const long ndof = c->ndof, nq = (long)c->n_elems * c->nqp, nn = c->n_nodes, nu = (long)c->dim * nn;
  const int nseg = (n_steps + ce - 1) / ce;
  const NetLayout& le = c->elay;
  const NetLayout& ly = c->ylay;

  // reaction dofs must be distinct and in range (checked on the host)
  {
    std::vector<int32_t> rd(n_reaction);
    AH(hipMemcpy(rd.data(), reaction_dofs, sizeof(int32_t) * n_reaction, hipMemcpyDeviceToHost));
    std::sort(rd.begin(), rd.end());
    if (rd.front() < 0 || rd.back() >= ndof || std::adjacent_find(rd.begin(), rd.end()) != rd.end()) {
      c->err = "reaction dofs must be distinct and in range";
      return GEDMG_E_ARG;
    }
  }
  std::vector<double> tgt(n_steps), reac(n_steps, 0.0);
  AH(hipMemcpy(tgt.data(), targets, sizeof(double) * n_steps, hipMemcpyDeviceToHost));

  Buffers B(c);
  double *ck_u, *ck_p, *ck_k, *seg_u, *seg_p, *seg_k, *end_u, *end_p, *end_k, *K, *KT, *Rv, *kt;
  double *e_react, *y, *gU, *b, *lam, *cR, *abar, *abarp, *erow, *yrow, *est, *yst, *part, *rpart, *ge, *gy;
  int32_t* permT;
  const int npmax = std::max(le.n_raw, ly.n_raw);
  if (!B.get(&ck_u, nu * nseg) || !B.get(&ck_p, nn * nseg) || !B.get(&ck_k, nq * nseg) ||
      !B.get(&seg_u, nu * ce) || !B.get(&seg_p, nn * ce) || !B.get(&seg_k, nq * (ce + 1)) ||
      !B.get(&end_u, nu) || !B.get(&end_p, nn) || !B.get(&end_k, nq) || !B.get(&K, c->nnz) ||
      !B.get(&KT, c->nnz) || !B.get(&permT, c->nnz) || !B.get(&Rv, ndof) || !B.get(&kt, nq) ||
      !B.get(&e_react, ndof) || !B.get(&y, ndof) || !B.get(&gU, ndof) || !B.get(&b, ndof) ||
      !B.get(&lam, ndof) || !B.get(&cR, ndof) || !B.get(&abar, nq) || !B.get(&abarp, nq) ||
      !B.get(&erow, (nq + 1) * 7) || !B.get(&yrow, (nq + 1) * 2) ||
      !B.get(&est, (nq + 1) * le.L * 4 * le.H) || !B.get(&yst, (nq + 1) * ly.L * 2 * ly.H) ||
      !B.get(&part, (size_t)kChunks * npmax) || !B.get(&rpart, 3 * 256) || !B.get(&ge, le.n_raw) ||
      !B.get(&gy, ly.n_raw)) {
    c->err = "device allocation for the adjoint failed";
    return GEDMG_E_NOMEM;
  }
  // value permutation of the transposed matrix (the node-block pattern is
  // structurally symmetric and its column indices are sorted per row)
  {
    std::vector<int32_t> rp(ndof + 1), cl(c->nnz), pt(c->nnz);
    AH(hipMemcpy(rp.data(), c->drowptr, sizeof(int32_t) * (ndof + 1), hipMemcpyDeviceToHost));
    AH(hipMemcpy(cl.data(), c->dcol, sizeof(int32_t) * c->nnz, hipMemcpyDeviceToHost));
    for (long r = 0; r < ndof; ++r)
      for (int j = rp[r]; j < rp[r + 1]; ++j) {
        const int cc = cl[j];
        const int32_t* beg = cl.data() + rp[cc];
        const int32_t* end = cl.data() + rp[cc + 1];
        const int32_t* it = std::lower_bound(beg, end, (int32_t)r);
        if (it == end || *it != r) {
          c->err = "CSR pattern is not structurally symmetric";
          return GEDMG_E_SHAPE;
        }
        pt[j] = (int32_t)(it - cl.data());
      }
    AH(hipMemcpyAsync(permT, pt.data(), sizeof(int32_t) * c->nnz, hipMemcpyHostToDevice, c->stream));
    AH(hipStreamSynchronize(c->stream));
  }
  AH(hipMemsetAsync(e_react, 0, sizeof(double) * ndof, c->stream));
  hipLaunchKernelGGL(indicator_kernel, grid1(n_reaction), dim3(256), 0, c->stream, e_react, reaction_dofs,
                     n_reaction);
  AH(hipGetLastError());

  int newton_its = 0, krylov_its = 0;
  // one converged load step from the current (u, phi, kappa)
  auto step = [&](int n) -> int {
    gedmg_newton_report nr{};
    const int rc = gedmg_newton_step(c, &bc_per_step[n - 1], &o, GEDMG_FP64,
                                     predictor_du ? predictor_du + (long)(n - 1) * nu : nullptr, u, phi, kappa,
                                     reaction_dofs, n_reaction, &nr);
    newton_its += nr.newton_iters;
    krylov_its += nr.krylov_iters_total;
    if (rc) return rc;
    reac[n - 1] = nr.reaction;
    return GEDMG_OK;
  };
  auto copy = [&](double* dst, const double* src, long n) {
    return hipMemcpyAsync(dst, src, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream);
  };
  // states of a segment: seg_k[j] = kappa before its step j, seg_u/p[j] after it
  auto store_seg = [&](int j) -> int {
    AH(copy(seg_u + j * nu, u, nu));
    AH(copy(seg_p + j * nn, phi, nn));
    AH(copy(seg_k + (j + 1) * nq, kappa, nq));
    return GEDMG_OK;
  };

  const auto t0 = std::chrono::steady_clock::now();
  int rc;
  // forward: checkpoint at the start of every segment; the last segment's
  // states are kept as they are produced (it is reversed first)
  for (int n = 1; n <= n_steps; ++n) {
    const int sg = (n - 1) / ce, j = (n - 1) % ce;
    if (j == 0) {
      AH(copy(ck_u + sg * nu, u, nu));
      AH(copy(ck_p + sg * nn, phi, nn));
      AH(copy(ck_k + sg * nq, kappa, nq));
      R.n_checkpoints++;
      if (sg == nseg - 1) AH(copy(seg_k, kappa, nq));
    }
    if ((rc = step(n))) return rc;
    if (sg == nseg - 1 && (rc = store_seg(j))) return rc;
  }
  AH(copy(end_u, u, nu));
  AH(copy(end_p, phi, nn));
  AH(copy(end_k, kappa, nq));
  double L = 0.0;
  for (int n = 0; n < n_steps; ++n) L += (reac[n] - tgt[n]) * (reac[n] - tgt[n]);
  AH(hipStreamSynchronize(c->stream));
  const auto t1 = std::chrono::steady_clock::now();
  double t_recompute = 0.0;

  AH(hipMemsetAsync(abar, 0, sizeof(double) * nq, c->stream));
  AH(hipMemsetAsync(ge, 0, sizeof(double) * le.n_raw, c->stream));
  AH(hipMemsetAsync(gy, 0, sizeof(double) * ly.n_raw, c->stream));
  AdjQpArgs aa{};
  aa.X = c->dX;
  aa.conn = c->dconn;
  aa.perm = c->dperm;
  aa.jet = c->djet;
  aa.ynet = c->dynet;
  aa.abar = abar;
  aa.cR = cR;
  aa.gU = gU;
  aa.abar_prev = abarp;
  aa.erow = erow;
  aa.yrow = yrow;
  aa.n_nodes = c->n_nodes;
  aa.m = c->mat;
  aa.n0 = c->eref.n0;
  aa.yN0 = c->yref.N0;
  aa.yH = ly.H;
  aa.yL = ly.L;
  auto run_qp = [&](int mode) -> int {
    aa.mode = mode;
    if (mode == 0) {
      for (size_t k = 0; k + 1 < c->color_begin.size(); ++k) {
        aa.e_begin = c->color_begin[k];
        aa.e_end = c->color_begin[k + 1];
        const int ne = aa.e_end - aa.e_begin;
        if (ne <= 0) continue;
        if (c->dim == 3)
          hipLaunchKernelGGL(adj_qp_kernel<3>, grid1(ne, 64), dim3(64), 0, c->stream, aa);
        else
          hipLaunchKernelGGL(adj_qp_kernel<2>, grid1(ne, 64), dim3(64), 0, c->stream, aa);
      }
    } else {
      aa.e_begin = 0;
      aa.e_end = c->n_elems;
      if (c->dim == 3)
        hipLaunchKernelGGL(adj_qp_kernel<3>, grid1(c->n_elems, 64), dim3(64), 0, c->stream, aa);
      else
        hipLaunchKernelGGL(adj_qp_kernel<2>, grid1(c->n_elems, 64), dim3(64), 0, c->stream, aa);
    }
    AH(hipGetLastError());
    return GEDMG_OK;
  };
  const int nrow = (int)(nq + 1);

  for (int sg = nseg - 1; sg >= 0; --sg) {
    const int s0 = sg * ce + 1, s1 = std::min(n_steps, s0 + ce - 1);
    if (sg != nseg - 1) {
      // recompute the segment from its checkpoint (bitwise the forward states)
      const auto tr0 = std::chrono::steady_clock::now();
      AH(copy(u, ck_u + sg * nu, nu));
      AH(copy(phi, ck_p + sg * nn, nn));
      AH(copy(kappa, ck_k + sg * nq, nq));
      AH(copy(seg_k, kappa, nq));
      for (int n = s0; n <= s1; ++n) {
        if ((rc = step(n))) return rc;
        if ((rc = store_seg(n - s0))) return rc;
        R.recomputed_steps++;
      }
      AH(hipStreamSynchronize(c->stream));
      t_recompute += std::chrono::duration<double>(std::chrono::steady_clock::now() - tr0).count();
    }
    for (int n = s1; n >= s0; --n) {
      const int j = n - s0;
      const double* Un = seg_u + j * nu;
      const double* Pn = seg_p + j * nn;
      const double* Kp = seg_k + j * nq;
      // FP64 tangent, kappa_n and jets at (U_n, kappa_{n-1})
      if ((rc = gedmg_assemble(c, Un, Pn, Kp, GEDMG_FP64, Rv, K, kt))) return rc;
      hipLaunchKernelGGL(transpose_values_kernel, grid1(c->nnz), dim3(256), 0, c->stream, K, permT, KT, c->nnz);
      AH(hipGetLastError());
      // y = K^T e: derivative of the reaction sum with respect to U
      if ((rc = solver_spmv(c, KT, e_react, y))) return rc;
      const double cr = 2.0 * (reac[n - 1] - tgt[n - 1]);
      aa.u = Un;
      aa.phi = Pn;
      aa.kappa_prev = Kp;
      aa.kappa_cur = kt;
      AH(hipMemsetAsync(gU, 0, sizeof(double) * ndof, c->stream));
      if ((rc = run_qp(0))) return rc;
      hipLaunchKernelGGL(adj_rhs_kernel, grid1(ndof), dim3(256), 0, c->stream, gU, y, cr, b, ndof);
      AH(hipGetLastError());
      int its = 0;
      if ((rc = solver_solve_free(c, KT, &bc_per_step[n - 1], b, lam, o.max_krylov, o.krylov_rtol,
                                  kRefinePasses, &its)))
        return rc;
      krylov_its += its;
      hipLaunchKernelGGL(adj_cot_kernel, grid1(ndof), dim3(256), 0, c->stream, lam, e_react, cr, cR, ndof);
      if ((rc = run_qp(1))) return rc;
      hipLaunchKernelGGL(ref_partial_kernel, dim3(256), dim3(256), 0, c->stream, erow, yrow, nq, rpart);
      hipLaunchKernelGGL(ref_rows_kernel, dim3(1), dim3(64), 0, c->stream, rpart, 256, erow + nq * 7,
                         yrow + nq * 2);
      hipLaunchKernelGGL(energy_vjp_kernel, grid1(nrow, 64), dim3(64), 0, c->stream, c->denet, le, erow, nrow,
                         est);
      hipLaunchKernelGGL(yield_vjp_kernel, grid1(nrow, 64), dim3(64), 0, c->stream, c->dynet, ly, yrow, nrow,
                         yst);
      hipLaunchKernelGGL(energy_grad_kernel, dim3((le.n_raw + 63) / 64, kChunks), dim3(64), 0, c->stream, le,
                         erow, est, nrow, part);
      hipLaunchKernelGGL(chunk_sum_kernel, grid1(le.n_raw), dim3(256), 0, c->stream, part, kChunks, le.n_raw, ge);
      hipLaunchKernelGGL(yield_grad_kernel, dim3((ly.n_raw + 63) / 64, kChunks), dim3(64), 0, c->stream, ly,
                         yrow, yst, nrow, part);
      hipLaunchKernelGGL(chunk_sum_kernel, grid1(ly.n_raw), dim3(256), 0, c->stream, part, kChunks, ly.n_raw, gy);
      AH(hipGetLastError());
      AH(copy(abar, abarp, nq));
    }
  }
  if ((rc = gedmg_status(c))) return rc;
  // leave the caller's state at the end of the load path
  AH(copy(u, end_u, nu));
  AH(copy(phi, end_p, nn));
  AH(copy(kappa, end_k, nq));
  std::vector<double> he(le.n_raw), hy(ly.n_raw);
  AH(hipMemcpyAsync(he.data(), ge, sizeof(double) * le.n_raw, hipMemcpyDeviceToHost, c->stream));
  AH(hipMemcpyAsync(hy.data(), gy, sizeof(double) * ly.n_raw, hipMemcpyDeviceToHost, c->stream));
  AH(hipStreamSynchronize(c->stream));
  raw_chain(le, c->eraw.data(), he.data(), grad_energy);
  raw_chain(ly, c->yraw.data(), hy.data(), grad_yield);
  *loss = L;
  const auto t2 = std::chrono::steady_clock::now();
  R.newton_iters_total = newton_its;
  R.krylov_iters_total = krylov_its;
  R.t_forward_s = std::chrono::duration<double>(t1 - t0).count();
  R.t_recompute_s = t_recompute;
  R.t_reverse_s = std::chrono::duration<double>(t2 - t1).count() - t_recompute;
  return GEDMG_OK;
}
