// Quadrature inputs, element residual / consistent tangent and the atomic-free
// coloured scatter into CSR (Sec. 3.1 residual, Sec. 3.2 monolithic scheme,
// Sec. 4.2 constitutive model).  The local damage update runs before the
// element kernel, one lane per quadrature point; the element kernel takes the
// updated history and its two sensitivities from there.
//
// One wavefront owns 8 quadrature points: one Hex8 element, or two Q4
// elements.  Each quadrature point is served by a group of 8 lanes: the lanes
// reduce the element gather and split the consistent tangent's rows; the whole
// wavefront then integrates K_e = sum_q Jw B^T D B column-parallel and writes
// its rows into CSR with plain stores, read-modify-write after the first
// writer of a block (elements of one colour share no node).
#include "device_common.h"
#include "gedmg_internal.h"

namespace gedmg {

template <int DIM>
struct Tr;
template <>
struct Tr<3> {
  static constexpr int NEN = 8, NQP = 8, ND = 4, NZ = 13, NDOFE = 32, EPW = 1;
};
template <>
struct Tr<2> {
  static constexpr int NEN = 4, NQP = 4, ND = 3, NZ = 7, NDOFE = 12, EPW = 2;
};

// 3-D z index of the local z index (2-D keeps the in-plane entries of the
// plane-strain 3-D state: F11 F12 F21 F22 phi g1 g2).
template <int DIM>
__device__ __forceinline__ int z3(int z) {
  if (DIM == 3) return z;
  return z < 4 ? (z >> 1) * 3 + (z & 1) : z + 5;  // 0 1 3 4 | 9 10 11
}

// ------------------------------------------------------------------ kinematics
// F = I + sum_a u_a (x) grad N_a at qp q of element e (one thread); x inputs of
// the energy network: (J^-2/3 I1 - 3, I2^3/(9 J^4) - 3, J - 1)  (Eq. dd_0).
template <int DIM>
__global__ __launch_bounds__(256) void qp_inputs_kernel(KinArgs a) {
  using T = Tr<DIM>;
  const long gid = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (gid >= (long)a.n_elems * T::NQP) return;
  const int e = (int)(gid / T::NQP), q = (int)(gid % T::NQP);
  double Jx[DIM][DIM] = {};
  double dNs[T::NEN][DIM];
  int nodes[T::NEN];
  double phiq = 0.0;
#pragma unroll
  for (int n = 0; n < T::NEN; ++n) {
    nodes[n] = a.conn[(long)e * T::NEN + n];
    double Nv;
    shape_at<DIM>(n, q, Nv, dNs[n]);
    phiq = fma(Nv, a.phi[nodes[n]], phiq);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      const double xd = a.X[(long)d * a.n_nodes + nodes[n]];
#pragma unroll
      for (int k = 0; k < DIM; ++k) Jx[d][k] += xd * dNs[n][k];
    }
  }
  double Ji[DIM][DIM];
  if (DIM == 2) {
    const double det = Jx[0][0] * Jx[1][1] - Jx[0][1] * Jx[1][0];
    Ji[0][0] = Jx[1][1] / det; Ji[0][1] = -Jx[0][1] / det;
    Ji[1][0] = -Jx[1][0] / det; Ji[1][1] = Jx[0][0] / det;
  } else {
    const double c00 = Jx[1][1] * Jx[2][2] - Jx[1][2] * Jx[2][1];
    const double c01 = Jx[1][2] * Jx[2][0] - Jx[1][0] * Jx[2][2];
    const double c02 = Jx[1][0] * Jx[2][1] - Jx[1][1] * Jx[2][0];
    const double det = Jx[0][0] * c00 + Jx[0][1] * c01 + Jx[0][2] * c02;
    const double id = 1.0 / det;
    double (*M)[DIM] = Jx;
    Ji[0][0] = c00 * id;
    Ji[1][0] = c01 * id;
    Ji[2][0] = c02 * id;
    Ji[0][1] = (M[0][2] * M[2][1] - M[0][1] * M[2][2]) * id;
    Ji[1][1] = (M[0][0] * M[2][2] - M[0][2] * M[2][0]) * id;
    Ji[2][1] = (M[0][1] * M[2][0] - M[0][0] * M[2][1]) * id;
    Ji[0][2] = (M[0][1] * M[1][2] - M[0][2] * M[1][1]) * id;
    Ji[1][2] = (M[0][2] * M[1][0] - M[0][0] * M[1][2]) * id;
    Ji[2][2] = (M[0][0] * M[1][1] - M[0][1] * M[1][0]) * id;
  }
  double F[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
#pragma unroll
  for (int n = 0; n < T::NEN; ++n) {
    double G[DIM];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      G[d] = 0.0;
#pragma unroll
      for (int k = 0; k < DIM; ++k) G[d] += Ji[k][d] * dNs[n][k];
    }
#pragma unroll
    for (int i = 0; i < DIM; ++i) {
      const double ui = a.u[(long)i * a.n_nodes + nodes[n]];
#pragma unroll
      for (int d = 0; d < DIM; ++d) F[i][d] += ui * G[d];
    }
  }
  double C[3][3];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[i][j] = F[0][i] * F[0][j] + F[1][i] * F[1][j] + F[2][i] * F[2][j];
  const double I1 = C[0][0] + C[1][1] + C[2][2];
  double CC = 0.0;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) CC += C[i][j] * C[i][j];
  const double I2 = 0.5 * (I1 * I1 - CC);
  const double J = F[0][0] * (F[1][1] * F[2][2] - F[1][2] * F[2][1]) -
                   F[0][1] * (F[1][0] * F[2][2] - F[1][2] * F[2][0]) +
                   F[0][2] * (F[1][0] * F[2][1] - F[1][1] * F[2][0]);
  if (!(J > 0.0)) a.status[0] = GEDMG_E_JNONPOS;
  const double cj = cbrt(J);
  const double J2 = J * J;
  a.x[gid * 3 + 0] = I1 / (cj * cj) - 3.0;
  a.x[gid * 3 + 1] = I2 * I2 * I2 / (9.0 * J2 * J2) - 3.0;
  a.x[gid * 3 + 2] = J - 1.0;
  a.phiq[gid] = phiq;
}

// ------------------------------------------------------------------ per-qp state
// Per-quadrature-point quantities the consistent tangent is built from (one
// copy per 8-lane group in LDS; the lanes of the group write identical values).
// Everything else the tangent needs (C, b, F^-1, C^-1 slices, dx/dF columns,
// dpsi_e/dF) is rebuilt from these with a few multiply-adds per row.
struct Qp {
  double F[9], A[9], Q[9];   // F, cof F = dJ/dF, dI2/dF = 2 (I1 F - F C)
  double v[3], w[3];         // C^-1 grad phi, F C^-1 grad phi
  double Hn[6];              // network Hessian (xx, yy, zz, xy, xz, yz)
  double J, I1, I2, Jm23, Jm53, Jm83, Jm4, Jm5, Jm6;
  double m[3];               // dN/dx - n0 e3
  double pv1, pv2;           // psi_vol', psi_vol''
  double f, fp, rhoF, kphi;  // f_d, f_d', d kappa/dF = rhoF psi_e,F, d kappa/d phi
  double C[9], b[9], Ci[9];  // F^T F, F F^T, C^-1 (3-D rows only)
};

// Row r (3-D z index) of the consistent tangent D = dPz/dz (Pz = (P, dPsi/dphi,
// Y_vec), z = (F, phi, grad phi)), for the local columns of DIM:
//   D_FF  = f_d psi_e,FF + grad-term_FF + f_d' rhoF psi_e,F (x) psi_e,F
//   D_Fphi = f_d' psi_e,F kappa_phi,   D_Fg = -c_d (F^-T_iL v_J + w_i C^-1_JL)
//   D_phiF = -beta_d rhoF psi_e,F,     D_phiphi = beta_d (1 - kappa_phi)
//   D_gF = -c_d (F^-1_Jk v_L + w_k C^-1_LJ),  D_gg = c_d C^-1
// with psi_e,FF = mu [x_F^T H x_F + m1 x1_FF + m2 x2_FF + m3 J_FF]
//                + lambda [psi_vol'' A (x) A + psi_vol' J_FF]
// written with the second derivatives of I1G, I2G and J (A = cof F):
//   J_FF = (A_iJ A_kL - A_iL A_kJ)/J
//   x1_FF = 2 J^-2/3 dd - 4/3 J^-5/3 (F A + A F) + 10/9 I1 J^-8/3 A A - 2/3 I1 J^-5/3 J_FF
//   x2_FF = 2/3 I2 J^-4 Q Q - 4/3 I2^2 J^-5 (Q A + A Q) + 1/3 I2^2 J^-4 I2_FF
//           + 20/9 I2^3 J^-6 A A - 4/9 I2^3 J^-5 J_FF
//   I2_FF = 2 (2 F F + I1 dd - d_ik C_JL - F_iL F_kJ - b_ik d_JL)
// and the gradient-energy term c_d (F^-T_Li w_k v_J + w_i w_k C^-1_JL + w_i v_L F^-1_Jk).
template <int DIM>
__device__ __forceinline__ void d_row(const Qp& __restrict__ s, const Material& M, int r, double* out) {
  using T = Tr<DIM>;
  double F[9], A[9], Q[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) {
    F[t] = s.F[t];
    A[t] = s.A[t];
    Q[t] = s.Q[t];
  }
  const double iJ = 1.0 / s.J;
  const double m0 = s.m[0], m1 = s.m[1], m2 = s.m[2];
  const double I22 = s.I2 * s.I2, I23 = I22 * s.I2;
  const double a1 = 2.0 * s.Jm23, b1 = -(2.0 / 3.0) * s.I1 * s.Jm53;      // x1_F = a1 F + b1 A
  const double a2 = (1.0 / 3.0) * I22 * s.Jm4, b2 = -(4.0 / 9.0) * I23 * s.Jm5;  // x2_F = a2 Q + b2 A
  auto psiF = [&](int c) {
    const double x1 = a1 * F[c] + b1 * A[c], x2 = a2 * Q[c] + b2 * A[c];
    return M.mu * (m0 * x1 + m1 * x2 + m2 * A[c]) + M.lam * s.pv1 * A[c];
  };
  if (r < 9) {
    const int i = r / 3, J = r % 3;
    const double c_d1 = M.mu * m0 * a1;
    const double c_FA = -M.mu * m0 * (4.0 / 3.0) * s.Jm53;
    const double c_AA = M.mu * (m0 * (10.0 / 9.0) * s.I1 * s.Jm83 + m1 * (20.0 / 9.0) * I23 * s.Jm6) +
                        M.lam * s.pv2;
    const double c_J = M.mu * (-m0 * (2.0 / 3.0) * s.I1 * s.Jm53 - m1 * (4.0 / 9.0) * I23 * s.Jm5 + m2) +
                       M.lam * s.pv1;
    const double c_QQ = M.mu * m1 * (2.0 / 3.0) * s.I2 * s.Jm4;
    const double c_QA = -M.mu * m1 * (4.0 / 3.0) * I22 * s.Jm5;
    const double c_I2 = M.mu * m1 * (1.0 / 3.0) * I22 * s.Jm4;
    const double Ar = A[r], Fr = F[r], Qr = Q[r], pr = psiF(r);
    // H x_F for this row
    const double x1r = a1 * Fr + b1 * Ar, x2r = a2 * Qr + b2 * Ar;
    const double* Hn = s.Hn;
    const double h0 = Hn[0] * x1r + Hn[3] * x2r + Hn[4] * Ar;
    const double h1 = Hn[3] * x1r + Hn[1] * x2r + Hn[5] * Ar;
    const double h2 = Hn[4] * x1r + Hn[5] * x2r + Hn[2] * Ar;
    // row slices of C, b, F^-1 and C^-1
    double CJ[3], bi[3], FiLi[3], FiJk[3], CiJ[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      CJ[t] = F[J] * F[t] + F[3 + J] * F[3 + t] + F[6 + J] * F[6 + t];
      bi[t] = F[i * 3] * F[t * 3] + F[i * 3 + 1] * F[t * 3 + 1] + F[i * 3 + 2] * F[t * 3 + 2];
      FiLi[t] = A[i * 3 + t] * iJ;   // F^-1_{t i}
      FiJk[t] = A[t * 3 + J] * iJ;   // F^-1_{J t}
      CiJ[t] = (A[J] * A[t] + A[3 + J] * A[3 + t] + A[6 + J] * A[6 + t]) * iJ * iJ;
    }
    const double wi = s.w[i], vJ = s.v[J];
    const double rank1 = s.fp * s.rhoF * pr;
#pragma unroll
    for (int cz = 0; cz < T::NZ; ++cz) {
      const int c = z3<DIM>(cz);
      double v;
      if (c < 9) {
        const int k = c / 3, L = c % 3;
        const double Ac = A[c], Fc = F[c], Qc = Q[c];
        const double dik = (i == k) ? 1.0 : 0.0, dJL = (J == L) ? 1.0 : 0.0;
        const double JFF = (Ar * Ac - A[i * 3 + L] * A[k * 3 + J]) * iJ;
        const double I2FF = 2.0 * (2.0 * Fr * Fc + s.I1 * dik * dJL - dik * CJ[L] -
                                   F[i * 3 + L] * F[k * 3 + J] - bi[k] * dJL);
        const double x1c = a1 * Fc + b1 * Ac, x2c = a2 * Qc + b2 * Ac;
        const double psiFF = M.mu * (h0 * x1c + h1 * x2c + h2 * Ac) + c_d1 * dik * dJL +
                             c_FA * (Fr * Ac + Ar * Fc) + c_AA * Ar * Ac + c_J * JFF + c_QQ * Qr * Qc +
                             c_QA * (Qr * Ac + Ar * Qc) + c_I2 * I2FF;
        const double grad = M.c * (FiLi[L] * s.w[k] * vJ + wi * s.w[k] * CiJ[L] + wi * s.v[L] * FiJk[k]);
        v = s.f * psiFF + grad + rank1 * psiF(c);
      } else if (c == 9) {
        v = s.fp * pr * s.kphi;
      } else {
        const int L = c - 10;
        v = -M.c * (FiLi[L] * vJ + wi * CiJ[L]);
      }
      out[cz] = v;
    }
    return;
  }
  if (r == 9) {
    const double bk = -M.beta * s.rhoF;
#pragma unroll
    for (int cz = 0; cz < T::NZ; ++cz) {
      const int c = z3<DIM>(cz);
      out[cz] = (c < 9) ? bk * psiF(c) : (c == 9 ? M.beta * (1.0 - s.kphi) : 0.0);
    }
    return;
  }
  const int Jp = r - 10;
  double FiJk[3], CiJ[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    FiJk[t] = A[t * 3 + Jp] * iJ;
    CiJ[t] = (A[Jp] * A[t] + A[3 + Jp] * A[3 + t] + A[6 + Jp] * A[6 + t]) * iJ * iJ;
  }
#pragma unroll
  for (int cz = 0; cz < T::NZ; ++cz) {
    const int c = z3<DIM>(cz);
    double v;
    if (c < 9) {
      const int k = c / 3, L = c % 3;
      v = -M.c * (FiJk[k] * s.v[L] + s.w[k] * CiJ[L]);
    } else if (c == 9) {
      v = 0.0;
    } else {
      v = M.c * CiJ[c - 10];
    }
    out[cz] = v;
  }
}

// Hex8 rows of D, the same quantities as d_row regrouped.  Every outer-product
// part of D_FF lies in span{F, A, Q} (x1_F = a1 F + b1 A, x2_F = a2 Q + b2 A,
// x3_F = A, psi_e,F = pF F + pA A + pQ Q), so with B_r = (F_r, A_r, Q_r)
//   D_FF(r, c) = B_r S B_c^T + kA A_iL A_kJ + kF (F_iL F_kJ + d_ik C_JL + b_ik d_JL)
//              + dd d_ik d_JL + w_k g1_L + v_L g2_k,       r = (i, J), c = (k, L),
// with one symmetric 3x3 S per point (network Hessian term, the F/A/Q outer
// products of J_FF, x1_FF, x2_FF, I2_FF and f_d' rhoF psi_e,F (x) psi_e,F),
// g1_L = c_d (F^-1_Li v_J + w_i C^-1_JL) and g2_k = c_d w_i F^-1_Jk.  A lane
// owns one row r; the row's slices of A, F, C, b and C^-1 come from LDS
// (dynamic index), the column operands are compile-time register indices.
// D_FF is symmetric, so row 8 of the F block is the transpose of column 8.
struct HexRowCoef {
  double S[3][3];
  double kA, kF, dd, pF, pA, pQ, fpk, iJ, cd;
};

__device__ __forceinline__ HexRowCoef hex_row_coef(const Qp& __restrict__ s, const Material& M) {
  HexRowCoef h;
  const double iJ = 1.0 / s.J;
  const double m0 = s.m[0], m1 = s.m[1], m2 = s.m[2];
  const double I22 = s.I2 * s.I2, I23 = I22 * s.I2;
  const double a1 = 2.0 * s.Jm23, b1 = -(2.0 / 3.0) * s.I1 * s.Jm53;
  const double a2 = (1.0 / 3.0) * I22 * s.Jm4, b2 = -(4.0 / 9.0) * I23 * s.Jm5;
  const double c_d1 = M.mu * m0 * a1;
  const double c_FA = -M.mu * m0 * (4.0 / 3.0) * s.Jm53;
  const double c_AA = M.mu * (m0 * (10.0 / 9.0) * s.I1 * s.Jm83 + m1 * (20.0 / 9.0) * I23 * s.Jm6) +
                      M.lam * s.pv2;
  const double c_J = M.mu * (-m0 * (2.0 / 3.0) * s.I1 * s.Jm53 - m1 * (4.0 / 9.0) * I23 * s.Jm5 + m2) +
                     M.lam * s.pv1;
  const double c_QQ = M.mu * m1 * (2.0 / 3.0) * s.I2 * s.Jm4;
  const double c_QA = -M.mu * m1 * (4.0 / 3.0) * I22 * s.Jm5;
  const double c_I2 = M.mu * m1 * (1.0 / 3.0) * I22 * s.Jm4;
  // T: rows x1_F, x2_F, x3_F in the basis (F, A, Q); S1 = mu T^T Hn T
  const double T[3][3] = {{a1, b1, 0.0}, {0.0, b2, a2}, {0.0, 1.0, 0.0}};
  const double Hm[3][3] = {{s.Hn[0], s.Hn[3], s.Hn[4]}, {s.Hn[3], s.Hn[1], s.Hn[5]}, {s.Hn[4], s.Hn[5], s.Hn[2]}};
  double HT[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) HT[a][b] = Hm[a][0] * T[0][b] + Hm[a][1] * T[1][b] + Hm[a][2] * T[2][b];
  double S0[3][3];
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) S0[a][b] = M.mu * (T[0][a] * HT[0][b] + T[1][a] * HT[1][b] + T[2][a] * HT[2][b]);
  S0[0][0] += 4.0 * c_I2;
  S0[0][1] += c_FA;
  S0[1][0] += c_FA;
  S0[1][1] += c_AA + c_J * iJ;
  S0[1][2] += c_QA;
  S0[2][1] += c_QA;
  S0[2][2] += c_QQ;
  h.pF = M.mu * m0 * a1;
  h.pA = M.mu * (m0 * b1 + m1 * b2 + m2) + M.lam * s.pv1;
  h.pQ = M.mu * m1 * a2;
  const double p[3] = {h.pF, h.pA, h.pQ};
  const double r1 = s.fp * s.rhoF;
#pragma unroll
  for (int a = 0; a < 3; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) h.S[a][b] = s.f * S0[a][b] + r1 * p[a] * p[b];
  h.kA = -s.f * c_J * iJ;
  h.kF = -2.0 * s.f * c_I2;
  h.dd = s.f * (c_d1 + 2.0 * c_I2 * s.I1);
  h.fpk = s.fp * s.kphi;
  h.iJ = iJ;
  h.cd = M.c;
  return h;
}

// F-block row r (0..8) of D for the F columns CB..8 and the phi / grad-phi
// columns; with MIRROR the column-8 entry is also stored as D[8][r].
template <int CB, bool MIRROR>
__device__ __forceinline__ void hex_f_row(const Qp& __restrict__ s, const HexRowCoef& h, int r,
                                          const double (&F)[9], const double (&A)[9], const double (&Q)[9],
                                          const double (&w)[3], const double (&v)[3], double (*D)[13]) {
  const int i = r / 3, J = r - 3 * (r / 3);
  const double Fr = s.F[r], Ar = s.A[r], Qr = s.Q[r];
  double Ai[3], AJ[3], Fi[3], FJ[3], CJ[3], bi[3], CiJ[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    Ai[t] = s.A[i * 3 + t];
    AJ[t] = s.A[t * 3 + J];
    Fi[t] = s.F[i * 3 + t];
    FJ[t] = s.F[t * 3 + J];
    CJ[t] = s.C[J * 3 + t];
    bi[t] = s.b[i * 3 + t];
    CiJ[t] = s.Ci[J * 3 + t];
  }
  const double wi = s.w[i], vJ = s.v[J];
  double u[3];
#pragma unroll
  for (int b = 0; b < 3; ++b) u[b] = Fr * h.S[0][b] + Ar * h.S[1][b] + Qr * h.S[2][b];
  double rA[3], rF[3], rC[3], rb[3], g1[3], g2[3], dik[3], dJL[3];
  const double cvJ = h.cd * vJ * h.iJ, cwi = h.cd * wi;
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    rA[t] = h.kA * Ai[t];
    rF[t] = h.kF * Fi[t];
    rC[t] = h.kF * CJ[t];
    rb[t] = h.kF * bi[t];
    g1[t] = cvJ * Ai[t] + cwi * CiJ[t];
    g2[t] = cwi * h.iJ * AJ[t];
    dik[t] = (i == t) ? 1.0 : 0.0;
    dJL[t] = (J == t) ? 1.0 : 0.0;
  }
#pragma unroll
  for (int c = CB; c < 9; ++c) {
    const int k = c / 3, L = c % 3;
    double x = u[0] * F[c] + u[1] * A[c] + u[2] * Q[c];
    x += rA[L] * AJ[k] + rF[L] * FJ[k];
    x += dik[k] * (rC[L] + dJL[L] * h.dd) + dJL[L] * rb[k];
    x += w[k] * g1[L] + v[L] * g2[k];
    D[r][c] = x;
    if (MIRROR && c == 8) D[8][r] = x;
  }
  D[r][9] = h.fpk * (h.pF * Fr + h.pA * Ar + h.pQ * Qr);
#pragma unroll
  for (int L = 0; L < 3; ++L) D[r][10 + L] = -g1[L];
}

// phi row (r = 9) and grad-phi rows (r = 10..12) in one form, so the four
// lanes run without divergence:
//   D(r, c) = al . (F_c, A_c, Q_c) + be_k v_L + w_k ga_L   (F columns c = (k, L))
// phi row: al = -beta rhoF psi_e,F coefficients, be = ga = 0;
// grad row Jp: al = 0, be_k = -c_d F^-1_{Jp k}, ga_L = -c_d C^-1_{L Jp}.
__device__ __forceinline__ void hex_pg_row(const Qp& __restrict__ s, const Material& M, const HexRowCoef& h,
                                           int r, const double (&F)[9], const double (&A)[9],
                                           const double (&Q)[9], const double (&w)[3], const double (&v)[3],
                                           double (*D)[13]) {
  const bool pr = r == 9;
  const int Jp = pr ? 0 : r - 10;
  const double bk = -M.beta * s.rhoF;
  const double al0 = pr ? bk * h.pF : 0.0, al1 = pr ? bk * h.pA : 0.0, al2 = pr ? bk * h.pQ : 0.0;
  double be[3], ga[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    be[t] = pr ? 0.0 : -h.cd * h.iJ * s.A[t * 3 + Jp];
    ga[t] = pr ? 0.0 : s.Ci[Jp * 3 + t];
  }
#pragma unroll
  for (int c = 0; c < 9; ++c) {
    const int k = c / 3, L = c % 3;
    D[r][c] = al0 * F[c] + al1 * A[c] + al2 * Q[c] + be[k] * v[L] - h.cd * w[k] * ga[L];
  }
  D[r][9] = pr ? M.beta * (1.0 - s.kphi) : 0.0;
#pragma unroll
  for (int L = 0; L < 3; ++L) D[r][10 + L] = pr ? 0.0 : h.cd * ga[L];
}

// ------------------------------------------------------------------ element kernel
typedef double d2_t __attribute__((ext_vector_type(2)));

template <int DIM>
struct alignas(16) ElemLds {
  using T = Tr<DIM>;
  double G[8][T::NEN][3];  // grad N per qp
  double N[8][T::NEN];
  double Jw[8];
  double Pz[8][T::NZ];
  double D[8][T::NZ][T::NZ];
  Qp qs[8];                // per-group state for the tangent rows
};

template <int DIM, bool TANGENT>
__global__ __launch_bounds__(64) void element_kernel(ElemArgs a) {
  using T = Tr<DIM>;
  __shared__ ElemLds<DIM> S;
  const int lane = threadIdx.x;
  const int g = lane >> 3, sub = lane & 7;
  const int es = (DIM == 3) ? 0 : (g >> 2);        // element slot of this group
  const int q = (DIM == 3) ? g : (g & 3);           // qp within the element
  const int slot_base = a.e_begin + blockIdx.x * T::EPW;
  const int pe = slot_base + es;
  const bool valid = pe < a.e_end;
  const int e = valid ? a.perm[pe] : 0;
  const Material M = a.m;
  const long qg = (long)e * T::NQP + q;

  // ---------------- gather and kinematics (lane sub serves node sub)
  const bool has_node = valid && sub < T::NEN;
  int node = 0;
  if (has_node) node = a.conn_s[(long)pe * T::NEN + sub];
  // Loads that do not depend on the connectivity, issued before the gather
  // chain so that their latency overlaps it: this point's jet row, updated
  // history and its sensitivities, the node coordinates, and (Hex8 tangent)
  // the CSR segments this lane writes at the end.
  d2_t jv[5] = {}, sens = {};
  double kap = 0.0;
  if (valid) {
    const d2_t* jr = reinterpret_cast<const d2_t*>(a.jet + qg * 10);
#pragma unroll
    for (int t = 0; t < 5; ++t) jv[t] = jr[t];
    kap = a.kappa[qg];
    sens = reinterpret_cast<const d2_t*>(a.sens)[qg];
  }
  constexpr int SPL = (DIM == 3 && TANGENT) ? T::NDOFE * T::NEN / 64 : 1;  // segments per lane
  uint32_t segv[SPL];
#pragma unroll
  for (int t = 0; t < SPL; ++t) segv[t] = 0u;
  if (DIM == 3 && TANGENT && valid) {
#pragma unroll
    for (int t = 0; t < SPL; ++t) segv[t] = (uint32_t)a.seg[(long)slot_base * (T::NDOFE * T::NEN) + lane + 64 * t];
  }
  double Xn[DIM] = {}, un[DIM] = {}, phin = 0.0, Nv = 0.0, dN[DIM] = {};
  if (has_node) {
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      Xn[d] = a.Xs[((long)pe * DIM + d) * T::NEN + sub];
      un[d] = a.u[(long)d * a.n_nodes + node];
    }
    phin = a.phi[node];
    shape_at<DIM>(sub, q, Nv, dN);
  }
  // The residual entries this wave updates at the end (lane dl owns element
  // dof dl: node dl / ND, component dl % ND); the node comes from the lane of
  // the first group of the element slot that gathered it.
  const int r_slot = (DIM == 3) ? 0 : (lane >> 5);
  const int r_dl = (DIM == 3) ? lane : (lane & 31);
  const bool r_own = r_dl < T::NDOFE && (slot_base + r_slot < a.e_end);
  const int r_node = __shfl(node, r_slot * 32 + r_dl / T::ND, 64);
  const long r_idx = (long)r_node * T::ND + r_dl % T::ND;
  const double r_old = r_own ? a.R[r_idx] : 0.0;
  double Jx[DIM][DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d)
#pragma unroll
    for (int k = 0; k < DIM; ++k) Jx[d][k] = group8_sum(Xn[d] * dN[k]);
  double Ji[DIM][DIM], detJx;
  if (DIM == 2) {
    detJx = Jx[0][0] * Jx[1][1] - Jx[0][1] * Jx[1][0];
    Ji[0][0] = Jx[1][1] / detJx; Ji[0][1] = -Jx[0][1] / detJx;
    Ji[1][0] = -Jx[1][0] / detJx; Ji[1][1] = Jx[0][0] / detJx;
  } else {
    double (*X)[DIM] = Jx;
    const double c00 = X[1][1] * X[2][2] - X[1][2] * X[2][1];
    const double c01 = X[1][2] * X[2][0] - X[1][0] * X[2][2];
    const double c02 = X[1][0] * X[2][1] - X[1][1] * X[2][0];
    detJx = X[0][0] * c00 + X[0][1] * c01 + X[0][2] * c02;
    const double id = 1.0 / detJx;
    Ji[0][0] = c00 * id; Ji[1][0] = c01 * id; Ji[2][0] = c02 * id;
    Ji[0][1] = (X[0][2] * X[2][1] - X[0][1] * X[2][2]) * id;
    Ji[1][1] = (X[0][0] * X[2][2] - X[0][2] * X[2][0]) * id;
    Ji[2][1] = (X[0][1] * X[2][0] - X[0][0] * X[2][1]) * id;
    Ji[0][2] = (X[0][1] * X[1][2] - X[0][2] * X[1][1]) * id;
    Ji[1][2] = (X[0][2] * X[1][0] - X[0][0] * X[1][2]) * id;
    Ji[2][2] = (X[0][0] * X[1][1] - X[0][1] * X[1][0]) * id;
  }
  double G[DIM];
#pragma unroll
  for (int d = 0; d < DIM; ++d) {
    G[d] = 0.0;
#pragma unroll
    for (int k = 0; k < DIM; ++k) G[d] += Ji[k][d] * dN[k];
  }
  if (has_node) {
#pragma unroll
    for (int d = 0; d < 3; ++d) S.G[g][sub][d] = (d < DIM) ? G[d] : 0.0;
    S.N[g][sub] = Nv;
  }
  if (sub == 0) S.Jw[g] = detJx;

  // The group's state is built in LDS; the 8 lanes write identical values.
  Qp& s = S.qs[g];
  {
    double Fr[9];
#pragma unroll
    for (int i = 0; i < 9; ++i) Fr[i] = (i % 4 == 0) ? 1.0 : 0.0;
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int d = 0; d < DIM; ++d) Fr[i * 3 + d] += group8_sum(un[i] * G[d]);
#pragma unroll
    for (int i = 0; i < 9; ++i) s.F[i] = Fr[i];
  }
  const double phi = group8_sum(phin * Nv);
  double gphi[3] = {0.0, 0.0, 0.0};
#pragma unroll
  for (int d = 0; d < DIM; ++d) gphi[d] = group8_sum(phin * G[d]);

  // ---------------- invariants and their first derivatives (all 8 lanes)
  double F[9];
#pragma unroll
  for (int t = 0; t < 9; ++t) F[t] = s.F[t];
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
  const double Jd = F[0] * A[0] + F[1] * A[1] + F[2] * A[2];
  if (valid && !(Jd > 0.0)) a.status[0] = GEDMG_E_JNONPOS;
  const double iJ = 1.0 / Jd;
  double C[9], Q[9];
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) C[i * 3 + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
  const double I1 = C[0] + C[4] + C[8];
  double CC = 0.0;
#pragma unroll
  for (int t = 0; t < 9; ++t) CC += C[t] * C[t];
  const double I2 = 0.5 * (I1 * I1 - CC);
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double FC = F[i * 3] * C[j] + F[i * 3 + 1] * C[3 + j] + F[i * 3 + 2] * C[6 + j];
      Q[i * 3 + j] = 2.0 * (I1 * F[i * 3 + j] - FC);
    }
  const double cj = cbrt(Jd);
  const double Jm23 = 1.0 / (cj * cj), Jm53 = Jm23 * iJ;
  const double Jm4 = iJ * iJ * iJ * iJ, Jm5 = Jm4 * iJ;
  const double x3 = Jd - 1.0;
  const double I22 = I2 * I2;
  // v = C^-1 grad phi (C^-1 = A^T A / J^2), w = F v
  double v[3], w[3];
#pragma unroll
  for (int i = 0; i < 3; ++i) {
    double t = 0.0;
#pragma unroll
    for (int j = 0; j < 3; ++j)
      t += (A[i] * A[j] + A[3 + i] * A[3 + j] + A[6 + i] * A[6 + j]) * gphi[j];
    v[i] = t * iJ * iJ;
  }
#pragma unroll
  for (int i = 0; i < 3; ++i) w[i] = F[i * 3] * v[0] + F[i * 3 + 1] * v[1] + F[i * 3 + 2] * v[2];

  // ---------------- energy from the network jet
  const double jt[10] = {jv[0][0], jv[0][1], jv[1][0], jv[1][1], jv[2][0],
                         jv[2][1], jv[3][0], jv[3][1], jv[4][0], jv[4][1]};
  const double dNx = jt[0];
  const double m0 = jt[1], m1 = jt[2], m2 = jt[3] - a.n0;
  const double vol = Jd + iJ - 2.0;
  const double pv1 = 2.0 * vol * (1.0 - iJ * iJ);
  const double psi_e = M.mu * (dNx - a.n0 * x3) + M.lam * vol * vol;
  double psiF[9];
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    const double x1 = 2.0 * Jm23 * F[r] - (2.0 / 3.0) * I1 * Jm53 * A[r];
    const double x2 = (1.0 / 3.0) * I22 * Jm4 * Q[r] - (4.0 / 9.0) * I22 * I2 * Jm5 * A[r];
    psiF[r] = M.mu * (m0 * x1 + m1 * x2 + m2 * A[r]) + M.lam * pv1 * A[r];
  }
  if (TANGENT) {
#pragma unroll
    for (int t = 0; t < 9; ++t) {
      s.A[t] = A[t];
      s.Q[t] = Q[t];
    }
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      s.v[t] = v[t];
      s.w[t] = w[t];
    }
#pragma unroll
    for (int t = 0; t < 6; ++t) s.Hn[t] = jt[4 + t];
    s.J = Jd; s.I1 = I1; s.I2 = I2;
    s.Jm23 = Jm23; s.Jm53 = Jm53; s.Jm83 = Jm53 * iJ; s.Jm4 = Jm4; s.Jm5 = Jm5; s.Jm6 = Jm5 * iJ;
    s.m[0] = m0; s.m[1] = m1; s.m[2] = m2;
    s.pv1 = pv1;
    s.pv2 = 2.0 * (1.0 - iJ * iJ) * (1.0 - iJ * iJ) + 4.0 * vol * iJ * iJ * iJ;
    if constexpr (DIM == 3) {
#pragma unroll
      for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
          s.C[i * 3 + j] = C[i * 3 + j];
          s.b[i * 3 + j] = F[i * 3] * F[j * 3] + F[i * 3 + 1] * F[j * 3 + 1] + F[i * 3 + 2] * F[j * 3 + 2];
          s.Ci[i * 3 + j] = (A[i] * A[j] + A[3 + i] * A[3 + j] + A[6 + i] * A[6 + j]) * iJ * iJ;
        }
    }
  }

  // ---------------- updated history (Eq. dd_7) and its sensitivities
  const double rhoF = sens[0], kphi = sens[1];
  const double fkap = exp_d(-M.eta * fmax(kap - M.kd, 0.0));
  const double fpkap = (kap > M.kd) ? -M.eta * fkap : 0.0;
  if (TANGENT) {
    s.f = fkap; s.fp = fpkap; s.rhoF = rhoF; s.kphi = kphi;
  }

  // ---------------- conjugates Pz = (P, dPsi/dphi, Y_vec) and the tangent
  if (sub == 0) {
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) S.Pz[g][i * DIM + j] = fkap * psiF[i * 3 + j] - M.c * w[i] * v[j];
    S.Pz[g][DIM * DIM] = M.beta * (phi - kap);
#pragma unroll
    for (int j = 0; j < DIM; ++j) S.Pz[g][DIM * DIM + 1 + j] = M.c * v[j];
  }
  if (TANGENT) {
    wave_lds_sync();
    if constexpr (DIM == 3) {
      // F rows 0..7 on lanes 0..7 (column 8 mirrored into row 8); then row 8's
      // remaining entries on lane 0 and the phi / grad-phi rows 9..12 on lanes 1..4
      const Qp& sq = S.qs[g];
      const HexRowCoef h = hex_row_coef(sq, M);
      double Fc[9], Ac[9], Qc[9], wc[3], vc[3];
#pragma unroll
      for (int t = 0; t < 9; ++t) {
        Fc[t] = sq.F[t];
        Ac[t] = sq.A[t];
        Qc[t] = sq.Q[t];
      }
#pragma unroll
      for (int t = 0; t < 3; ++t) {
        wc[t] = sq.w[t];
        vc[t] = sq.v[t];
      }
      hex_f_row<0, true>(sq, h, sub, Fc, Ac, Qc, wc, vc, S.D[g]);
      if (sub == 0) hex_f_row<8, false>(sq, h, 8, Fc, Ac, Qc, wc, vc, S.D[g]);
      else if (sub <= 4) hex_pg_row(sq, M, h, 8 + sub, Fc, Ac, Qc, wc, vc, S.D[g]);
    } else {
      // 2-D: row sub (< 7) per lane
      double dr[T::NZ];
      if (sub < T::NZ) {
        d_row<DIM>(S.qs[g], M, z3<DIM>(sub), dr);
#pragma unroll
        for (int c = 0; c < T::NZ; ++c) S.D[g][sub][c] = dr[c];
      }
    }
  }
  __syncthreads();

  // ---------------- element residual: lanes own element dofs
  // (Hex8: the two halves of the wavefront integrate points 0..3 and 4..7 of
  // the same 32 dofs and are summed with one lane exchange)
  if constexpr (DIM == 3) {
    const int dl = lane & 31, hq = lane >> 5;
    const int an = dl / T::ND, cc = dl % T::ND;
    double acc = 0.0;
#pragma unroll 1
    for (int qq = 0; qq < 4; ++qq) {
      const int gq = hq * 4 + qq;
      double t;
      if (cc < DIM) {
        t = 0.0;
#pragma unroll
        for (int J = 0; J < DIM; ++J) t += S.G[gq][an][J] * S.Pz[gq][cc * DIM + J];
      } else {
        const int zp = DIM * DIM;
        t = S.N[gq][an] * S.Pz[gq][zp];
#pragma unroll
        for (int J = 0; J < DIM; ++J) t += S.G[gq][an][J] * S.Pz[gq][zp + 1 + J];
      }
      acc += S.Jw[gq] * t;
    }
    acc += __shfl_xor(acc, 32, 64);
    if (r_own) a.R[r_idx] = r_old + acc;
  } else {
    const int eslot = r_slot;
    const int dl = r_dl;
    if (r_own) {
      const int an = dl / T::ND, cc = dl % T::ND;
      double acc = 0.0;
#pragma unroll 1
    for (int qq = 0; qq < T::NQP; ++qq) {
        const int gq = eslot * 4 + qq;
        double t;
        if (cc < DIM) {
          t = 0.0;
#pragma unroll
          for (int J = 0; J < DIM; ++J) t += S.G[gq][an][J] * S.Pz[gq][cc * DIM + J];
        } else {
          const int zp = DIM * DIM;
          t = S.N[gq][an] * S.Pz[gq][zp];
#pragma unroll
          for (int J = 0; J < DIM; ++J) t += S.G[gq][an][J] * S.Pz[gq][zp + 1 + J];
        }
        acc += S.Jw[gq] * t;
      }
      a.R[r_idx] = r_old + acc;
    }
  }
  if (!TANGENT) return;

  // ---------------- element tangent and its CSR scatter
  if constexpr (DIM == 3) {
    // Hex8.  Lane (h, col): column col = (bnode, kc) of K_e and the rows
    // (an, 2h), (an, 2h + 1) of every element node an.  Per qp the half h
    // needs T = Jw D B[:, col] only at the z its rows touch: h = 0 (rows of
    // u1, u2) the z of F rows 1 and 2 (0..5), h = 1 (rows of u3 and phi)
    // z = 6..12; slot 3 of half 0 is a zero so both halves run one formula:
    //   K[(an, 2h)]     += G_an . T[0..2]
    //   K[(an, 2h + 1)] += N_an T[3] + G_an . T[4..6]
    const int h = lane >> 5, col = lane & 31;
    const int bnode = col >> 2, kc = col & 3;
    // the segments this lane writes afterwards (offsets loaded in the
    // prologue): issue their old values now, so the loads complete while the
    // tangent is integrated
    long soff[SPL];
    bool sfirst[SPL];
    d2_t old0[SPL], old1[SPL];
#pragma unroll
    for (int t = 0; t < SPL; ++t) {
      soff[t] = (long)(segv[t] & 0x7fffffffu);
      sfirst[t] = (segv[t] >> 31) != 0u;
    }
#pragma unroll
    for (int t = 0; t < SPL; ++t) {
      old0[t] = d2_t{0.0, 0.0};
      old1[t] = d2_t{0.0, 0.0};
      if (!sfirst[t]) {
        const d2_t* k2 = reinterpret_cast<const d2_t*>(a.K + soff[t]);
        old0[t] = k2[0];
        old1[t] = k2[1];
      }
    }
    // column operand: D offsets and weights of B[:, col]
    int o[4];
    if (kc < 3) {
      o[0] = 3 * kc; o[1] = 3 * kc + 1; o[2] = 3 * kc + 2; o[3] = 3 * kc + 2;
    } else {
      o[0] = 9; o[1] = 10; o[2] = 11; o[3] = 12;
    }
    int zs[7];
#pragma unroll
    for (int j = 0; j < 7; ++j) zs[j] = h ? 6 + j : (j < 3 ? j : (j == 3 ? 0 : j - 1));
    const double m3 = h ? 1.0 : 0.0;
    double Kacc[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) Kacc[t] = 0.0;
#pragma unroll 2
    for (int gq = 0; gq < T::NQP; ++gq) {
      const double jw = S.Jw[gq];
      double w[4];
      if (kc < 3) {
        w[0] = S.G[gq][bnode][0]; w[1] = S.G[gq][bnode][1]; w[2] = S.G[gq][bnode][2]; w[3] = 0.0;
      } else {
        w[0] = S.N[gq][bnode]; w[1] = S.G[gq][bnode][0]; w[2] = S.G[gq][bnode][1]; w[3] = S.G[gq][bnode][2];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i) w[i] *= jw;
      double Tz[7];
#pragma unroll
      for (int j = 0; j < 7; ++j) {
        const double* Dz = S.D[gq][zs[j]];
        Tz[j] = Dz[o[0]] * w[0] + Dz[o[1]] * w[1] + Dz[o[2]] * w[2] + Dz[o[3]] * w[3];
      }
      Tz[3] *= m3;
#pragma unroll
      for (int an = 0; an < T::NEN; ++an) {
        const double g0 = S.G[gq][an][0], g1 = S.G[gq][an][1], g2 = S.G[gq][an][2], nn = S.N[gq][an];
        Kacc[2 * an] += g0 * Tz[0] + g1 * Tz[1] + g2 * Tz[2];
        Kacc[2 * an + 1] += nn * Tz[3] + g0 * Tz[4] + g1 * Tz[5] + g2 * Tz[6];
      }
    }
    // stage K_e in LDS (the D buffer is free now), then write the segments
    double* Ke = &S.D[0][0][0];
    wave_lds_sync();
#pragma unroll
    for (int an = 0; an < T::NEN; ++an) {
      Ke[(an * 4 + 2 * h) * T::NDOFE + col] = Kacc[2 * an];
      Ke[(an * 4 + 2 * h + 1) * T::NDOFE + col] = Kacc[2 * an + 1];
    }
    wave_lds_sync();
#pragma unroll
    for (int t = 0; t < SPL; ++t) {
      const int sg = lane + 64 * t;
      const int r = sg / T::NEN, bn = sg % T::NEN;
      const d2_t* s2 = reinterpret_cast<const d2_t*>(Ke + r * T::NDOFE + bn * T::ND);
      d2_t* k2 = reinterpret_cast<d2_t*>(a.K + soff[t]);
      k2[0] = s2[0] + old0[t];
      k2[1] = s2[1] + old1[t];
    }
  } else {
    // Q4 (two elements per wavefront): lane owns one column and a block of rows
    constexpr int RPL = 6;   // rows per lane
    const int eslot = lane >> 5;
    const int li = lane & 31;
    const int col = li % T::NDOFE;
    const int rb = (li / T::NDOFE) * RPL;
    const bool own = li < 2 * T::NDOFE && (slot_base + eslot < a.e_end);
    const int bnode = col / T::ND, kc = col % T::ND;
    double Kacc[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) Kacc[t] = 0.0;
#pragma unroll 1
    for (int qq = 0; qq < (own ? T::NQP : 0); ++qq) {
      const int gq = eslot * 4 + qq;
      // B[:, col] nonzeros -> T = D B[:, col]
      double Tz[T::NZ];
#pragma unroll
      for (int z = 0; z < T::NZ; ++z) {
        double t;
        if (kc < DIM) {
          t = 0.0;
#pragma unroll
          for (int L = 0; L < DIM; ++L) t += S.D[gq][z][kc * DIM + L] * S.G[gq][bnode][L];
        } else {
          const int zp = DIM * DIM;
          t = S.D[gq][z][zp] * S.N[gq][bnode];
#pragma unroll
          for (int L = 0; L < DIM; ++L) t += S.D[gq][z][zp + 1 + L] * S.G[gq][bnode][L];
        }
        Tz[z] = t;
      }
      const double jw = S.Jw[gq];
#pragma unroll
      for (int t = 0; t < RPL; ++t) {
        const int r = rb + t;
        const int an = r / T::ND, cr = r % T::ND;
        double v;
        if (cr < DIM) {
          v = 0.0;
#pragma unroll
          for (int J = 0; J < DIM; ++J) v += S.G[gq][an][J] * Tz[cr * DIM + J];
        } else {
          const int zp = DIM * DIM;
          v = S.N[gq][an] * Tz[zp];
#pragma unroll
          for (int J = 0; J < DIM; ++J) v += S.G[gq][an][J] * Tz[zp + 1 + J];
        }
        Kacc[t] += jw * v;
      }
    }
    // stage K_e in LDS (the D buffer is free now), then write it one CSR
    // block-row segment (the ND columns of one element node) per lane; the
    // first colour that touches a block stores it, later colours add to it
    double* Ke = &S.D[0][0][0] + eslot * T::NDOFE * T::NDOFE;
    wave_lds_sync();
    if (own) {
#pragma unroll
      for (int t = 0; t < RPL; ++t) Ke[(rb + t) * T::NDOFE + col] = Kacc[t];
    }
    wave_lds_sync();
    constexpr int NSEG = T::EPW * T::NDOFE * T::NEN;  // segments per wavefront
#pragma unroll 1
    for (int sg = lane; sg < NSEG; sg += 64) {
      const int es = sg / (T::NDOFE * T::NEN);
      const int rem = sg - es * (T::NDOFE * T::NEN);
      const int r = rem / T::NEN, bn = rem % T::NEN;
      if (slot_base + es >= a.e_end) continue;
      const uint32_t sv = (uint32_t)a.seg[(long)(slot_base + es) * (T::NDOFE * T::NEN) + rem];
      const long off = (long)(sv & 0x7fffffffu);
      const double* src = &S.D[0][0][0] + es * T::NDOFE * T::NDOFE + r * T::NDOFE + bn * T::ND;
      const bool first = (sv >> 31) != 0u;
      double v[T::ND];
#pragma unroll
      for (int k = 0; k < T::ND; ++k) v[k] = src[k];
      if (!first) {
#pragma unroll
        for (int k = 0; k < T::ND; ++k) v[k] += a.K[off + k];
      }
#pragma unroll
      for (int k = 0; k < T::ND; ++k) a.K[off + k] = v[k];
    }
  }
}

hipError_t launch_qp_inputs(int dim, const KinArgs& a, hipStream_t s) {
  const int nqp = dim == 3 ? 8 : 4;
  const long n = (long)a.n_elems * nqp;
  const int blocks = (int)((n + 255) / 256);
  if (blocks == 0) return hipSuccess;
  if (dim == 3)
    hipLaunchKernelGGL(qp_inputs_kernel<3>, dim3(blocks), dim3(256), 0, s, a);
  else
    hipLaunchKernelGGL(qp_inputs_kernel<2>, dim3(blocks), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_element(int dim, bool tangent, const ElemArgs& a, hipStream_t s) {
  const int epw = dim == 3 ? 1 : 2;
  const int n = a.e_end - a.e_begin;
  const int blocks = (n + epw - 1) / epw;
  if (blocks == 0) return hipSuccess;
  if (dim == 3) {
    if (tangent) hipLaunchKernelGGL((element_kernel<3, true>), dim3(blocks), dim3(64), 0, s, a);
    else hipLaunchKernelGGL((element_kernel<3, false>), dim3(blocks), dim3(64), 0, s, a);
  } else {
    if (tangent) hipLaunchKernelGGL((element_kernel<2, true>), dim3(blocks), dim3(64), 0, s, a);
    else hipLaunchKernelGGL((element_kernel<2, false>), dim3(blocks), dim3(64), 0, s, a);
  }
  return hipGetLastError();
}

}  // namespace gedmg
