// Quadrature-point update, element residual / consistent tangent and the
// atomic-free coloured scatter into CSR (Sec. 3.1 residual, Sec. 3.2 history
// treatment of the monolithic scheme, Sec. 4.2 constitutive model).
//
// One wavefront owns 8 quadrature points: one Hex8 element, or two Q4
// elements.  Each quadrature point is served by a group of 8 lanes: the lanes
// reduce the element gather, evaluate the yield network neuron-parallel and
// split the consistent tangent's entries; the whole wavefront then integrates
// K_e = sum_q Jw B^T D B column-parallel and writes its rows into CSR with
// plain read-modify-write stores (elements of one colour share no node).
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
#pragma unroll
  for (int n = 0; n < T::NEN; ++n) {
    nodes[n] = a.conn[(long)e * T::NEN + n];
    double Nv;
    shape_at<DIM>(n, q, Nv, dNs[n]);
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
}

// ------------------------------------------------------------------ yield network
// N^_kappa(q) and its derivative, neurons split over the 8 lanes of a group.
// `sc` is this group's LDS scratch of 2*H doubles.
template <int H>
__device__ double yield_eval_h(const double* __restrict__ net, int L, double yN0, int sub, double q,
                               double* sc, double& dN) {
  const NetLayout lay = make_layout_hd(1, H, L, 1);
  double pN = 0.0, pD = 0.0;
  constexpr int per = H / 8;
  double z[per], zt[per];
#pragma unroll
  for (int j = 0; j < per; ++j) {
    const int n = sub + 8 * j;
    const double w = net[lay.W0 + n];
    double s;
    z[j] = softplus_d(w * q + net[lay.b0 + n], s);
    zt[j] = s * w;
  }
  for (int k = 1; k < L; ++k) {
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < per; ++j) {
      sc[sub + 8 * j] = z[j];
      sc[H + sub + 8 * j] = zt[j];
    }
    wave_lds_sync();
#pragma unroll
    for (int j = 0; j < per; ++j) {
      const int n = sub + 8 * j;
      const double* Wz = net + lay.Wz[k] + n * H;
      double acc = net[lay.Wx[k] + n] * q + net[lay.b[k] + n];
      double acct = net[lay.Wx[k] + n];
      for (int m = 0; m < H; ++m) {
        acc = fma(Wz[m], sc[m], acc);
        acct = fma(Wz[m], sc[H + m], acct);
      }
      double s;
      z[j] = softplus_d(acc, s);
      zt[j] = s * acct;
    }
  }
#pragma unroll
  for (int j = 0; j < per; ++j) {
    const double w = net[lay.wz + sub + 8 * j];
    pN = fma(w, z[j], pN);
    pD = fma(w, zt[j], pD);
  }
  pN = group8_sum(pN);
  pD = group8_sum(pD);
  const double wx = net[lay.wx];
  dN = pD + wx;
  return pN + wx * q + net[lay.bout] - yN0;
}



// ------------------------------------------------------------------ per-qp state
// Per-quadrature-point quantities the consistent tangent is built from.  The
// 8 lanes of a group compute them redundantly; one copy per group lives in
// LDS for the entry-parallel tangent (runtime-indexed, so not in registers).
struct Qp {
  double F[9], A[9], Fi[9], Ci[9], C[9], b[9], Q[9];
  double x1F[9], x2F[9], psiF[9];
  double Hx[9][3];   // sum_p d2N/dx_p dx_t * dx_p/dF_r
  double v[3], w[3];
  double J, I1, I2, Jm23, Jm53, Jm83, Jm4, Jm5, Jm6;
  double m[3];
  double pv1, pv2;
  double f, fp, rhoF, kphi;
};

// Entry (r, c) of the consistent tangent D = dPz/dz in 3-D z indices.
__device__ double d_entry(const Qp& __restrict__ s, const Material& M, int r, int c) {
  if (r < 9 && c < 9) {
    const int i = r / 3, J = r % 3, k = c / 3, L = c % 3;
    const double dik = (i == k) ? 1.0 : 0.0, dJL = (J == L) ? 1.0 : 0.0;
    const double JFF = (s.A[r] * s.A[c] - s.A[i * 3 + L] * s.A[k * 3 + J]) / s.J;
    const double x1FF = 2.0 * s.Jm23 * dik * dJL -
                        (4.0 / 3.0) * s.Jm53 * (s.F[r] * s.A[c] + s.A[r] * s.F[c]) +
                        (10.0 / 9.0) * s.I1 * s.Jm83 * s.A[r] * s.A[c] -
                        (2.0 / 3.0) * s.I1 * s.Jm53 * JFF;
    const double I2FF = 2.0 * (2.0 * s.F[r] * s.F[c] + s.I1 * dik * dJL - dik * s.C[J * 3 + L] -
                               s.F[i * 3 + L] * s.F[k * 3 + J] - s.b[i * 3 + k] * dJL);
    const double I22 = s.I2 * s.I2, I23 = I22 * s.I2;
    const double x2FF = (2.0 / 3.0) * s.I2 * s.Jm4 * s.Q[r] * s.Q[c] -
                        (4.0 / 3.0) * I22 * s.Jm5 * (s.Q[r] * s.A[c] + s.A[r] * s.Q[c]) +
                        (1.0 / 3.0) * I22 * s.Jm4 * I2FF + (20.0 / 9.0) * I23 * s.Jm6 * s.A[r] * s.A[c] -
                        (4.0 / 9.0) * I23 * s.Jm5 * JFF;
    const double hterm = s.Hx[r][0] * s.x1F[c] + s.Hx[r][1] * s.x2F[c] + s.Hx[r][2] * s.A[c];
    const double psiFF = M.mu * (hterm + s.m[0] * x1FF + s.m[1] * x2FF + s.m[2] * JFF) +
                         M.lam * (s.pv2 * s.A[r] * s.A[c] + s.pv1 * JFF);
    const double grad = M.c * (s.Fi[L * 3 + i] * s.w[k] * s.v[J] + s.w[i] * s.w[k] * s.Ci[J * 3 + L] +
                               s.w[i] * s.v[L] * s.Fi[J * 3 + k]);
    return s.f * psiFF + grad + s.fp * s.psiF[r] * s.rhoF * s.psiF[c];
  }
  if (r < 9 && c == 9) return s.fp * s.psiF[r] * s.kphi;
  if (r < 9) {
    const int i = r / 3, J = r % 3, L = c - 10;
    return -M.c * (s.Fi[L * 3 + i] * s.v[J] + s.w[i] * s.Ci[J * 3 + L]);
  }
  if (r == 9) {
    if (c < 9) return -M.beta * s.rhoF * s.psiF[c];
    if (c == 9) return M.beta * (1.0 - s.kphi);
    return 0.0;
  }
  const int Jp = r - 10;
  if (c < 9) {
    const int k = c / 3, L = c % 3;
    return -M.c * (s.Fi[Jp * 3 + k] * s.v[L] + s.w[k] * s.Ci[L * 3 + Jp]);
  }
  if (c == 9) return 0.0;
  return M.c * s.Ci[Jp * 3 + (c - 10)];
}

// ------------------------------------------------------------------ element kernel
template <int DIM, int YH>
struct ElemLds {
  using T = Tr<DIM>;
  double G[8][T::NEN][3];  // grad N per qp
  double N[8][T::NEN];
  double Jw[8];
  double Pz[8][T::NZ];
  double D[8][T::NZ][T::NZ];
  double ysc[8][2 * YH];   // yield-network scratch per group
  Qp qs[8];                // per-group state for the tangent entries
};

template <int DIM, bool TANGENT, int YH>
__global__ __launch_bounds__(64) void element_kernel(ElemArgs a) {
  using T = Tr<DIM>;
  __shared__ ElemLds<DIM, YH> S;
  const int lane = threadIdx.x;
  const int g = lane >> 3, sub = lane & 7;
  const int es = (DIM == 3) ? 0 : (g >> 2);        // element slot of this group
  const int q = (DIM == 3) ? g : (g & 3);           // qp within the element
  const int slot_base = a.e_begin + blockIdx.x * T::EPW;
  const int pe = slot_base + es;
  const bool valid = pe < a.e_end;
  const int e = valid ? a.perm[pe] : 0;
  const Material M = a.m;

  // ---------------- gather and kinematics (lane sub serves node sub)
  const bool has_node = valid && sub < T::NEN;
  int node = 0;
  double Xn[DIM] = {}, un[DIM] = {}, phin = 0.0, Nv = 0.0, dN[DIM] = {};
  if (has_node) {
    node = a.conn[(long)e * T::NEN + sub];
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
      Xn[d] = a.X[(long)d * a.n_nodes + node];
      un[d] = a.u[(long)d * a.n_nodes + node];
    }
    phin = a.phi[node];
    shape_at<DIM>(sub, q, Nv, dN);
  }
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
  const double* F = s.F;
  s.A[0] = F[4] * F[8] - F[5] * F[7];
  s.A[1] = F[5] * F[6] - F[3] * F[8];
  s.A[2] = F[3] * F[7] - F[4] * F[6];
  s.A[3] = F[2] * F[7] - F[1] * F[8];
  s.A[4] = F[0] * F[8] - F[2] * F[6];
  s.A[5] = F[1] * F[6] - F[0] * F[7];
  s.A[6] = F[1] * F[5] - F[2] * F[4];
  s.A[7] = F[2] * F[3] - F[0] * F[5];
  s.A[8] = F[0] * F[4] - F[1] * F[3];
  s.J = F[0] * s.A[0] + F[1] * s.A[1] + F[2] * s.A[2];
  if (valid && !(s.J > 0.0)) a.status[0] = GEDMG_E_JNONPOS;
  const double iJ = 1.0 / s.J;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) s.Fi[i * 3 + j] = s.A[j * 3 + i] * iJ;
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      s.C[i * 3 + j] = F[i] * F[j] + F[3 + i] * F[3 + j] + F[6 + i] * F[6 + j];
      s.b[i * 3 + j] = F[i * 3] * F[j * 3] + F[i * 3 + 1] * F[j * 3 + 1] + F[i * 3 + 2] * F[j * 3 + 2];
      s.Ci[i * 3 + j] = s.Fi[i * 3] * s.Fi[j * 3] + s.Fi[i * 3 + 1] * s.Fi[j * 3 + 1] +
                        s.Fi[i * 3 + 2] * s.Fi[j * 3 + 2];
    }
  s.I1 = s.C[0] + s.C[4] + s.C[8];
  double CC = 0.0;
#pragma unroll
  for (int i = 0; i < 9; ++i) CC += s.C[i] * s.C[i];
  s.I2 = 0.5 * (s.I1 * s.I1 - CC);
  // Q = dI2/dF = 2 (I1 F - F C)
#pragma unroll
  for (int i = 0; i < 3; ++i)
#pragma unroll
    for (int j = 0; j < 3; ++j) {
      const double FC = F[i * 3] * s.C[j] + F[i * 3 + 1] * s.C[3 + j] + F[i * 3 + 2] * s.C[6 + j];
      s.Q[i * 3 + j] = 2.0 * (s.I1 * F[i * 3 + j] - FC);
    }
  const double cj = cbrt(s.J);
  s.Jm23 = 1.0 / (cj * cj);
  s.Jm53 = s.Jm23 * iJ;
  s.Jm83 = s.Jm53 * iJ;
  s.Jm4 = iJ * iJ * iJ * iJ;
  s.Jm5 = s.Jm4 * iJ;
  s.Jm6 = s.Jm5 * iJ;
  const double x3 = s.J - 1.0;
  const double I22 = s.I2 * s.I2;
#pragma unroll
  for (int r = 0; r < 9; ++r) {
    s.x1F[r] = 2.0 * s.Jm23 * F[r] - (2.0 / 3.0) * s.I1 * s.Jm53 * s.A[r];
    s.x2F[r] = (1.0 / 3.0) * I22 * s.Jm4 * s.Q[r] - (4.0 / 9.0) * I22 * s.I2 * s.Jm5 * s.A[r];
  }
  // v = C^-1 grad phi, w = F v
#pragma unroll
  for (int i = 0; i < 3; ++i) s.v[i] = s.Ci[i * 3] * gphi[0] + s.Ci[i * 3 + 1] * gphi[1] + s.Ci[i * 3 + 2] * gphi[2];
#pragma unroll
  for (int i = 0; i < 3; ++i) s.w[i] = F[i * 3] * s.v[0] + F[i * 3 + 1] * s.v[1] + F[i * 3 + 2] * s.v[2];

  // ---------------- energy from the network jet
  const long qg = (long)e * T::NQP + q;
  const double* jt = a.jet + qg * 10;
  const double dNx = jt[0];
  s.m[0] = jt[1];
  s.m[1] = jt[2];
  s.m[2] = jt[3] - a.n0;
  if (TANGENT) {
    const double h6[6] = {jt[4], jt[5], jt[6], jt[7], jt[8], jt[9]};
    const double Hm[3][3] = {{h6[0], h6[3], h6[4]}, {h6[3], h6[1], h6[5]}, {h6[4], h6[5], h6[2]}};
#pragma unroll
    for (int r = 0; r < 9; ++r)
#pragma unroll
      for (int t = 0; t < 3; ++t)
        s.Hx[r][t] = Hm[0][t] * s.x1F[r] + Hm[1][t] * s.x2F[r] + Hm[2][t] * s.A[r];
  }
  const double vol = s.J + iJ - 2.0;
  s.pv1 = 2.0 * vol * (1.0 - iJ * iJ);
  s.pv2 = 2.0 * (1.0 - iJ * iJ) * (1.0 - iJ * iJ) + 4.0 * vol * iJ * iJ * iJ;
  const double psi_e = M.mu * (dNx - a.n0 * x3) + M.lam * vol * vol;
#pragma unroll
  for (int r = 0; r < 9; ++r)
    s.psiF[r] = M.mu * (s.m[0] * s.x1F[r] + s.m[1] * s.x2F[r] + s.m[2] * s.A[r]) + M.lam * s.pv1 * s.A[r];

  // ---------------- local history update (Eq. dd_7), safeguarded Newton
  const double kn = valid ? a.kappa_n[qg] : 0.0;
  double* sc = S.ysc[g];
  const double gb = M.gamma * M.beta;
  double kap = kn, dNy = 0.0;
  bool yielded = false;
  {
    const double f0 = exp(-M.eta * fmax(kn - M.kd, 0.0));
    const double q0 = psi_e + gb * (phi - kn) / (M.eta * f0);
    double d0;
    const double h0 = yield_eval_h<YH>(a.ynet, a.yL, a.yN0, sub, q0, sc, d0) - kn;
    dNy = d0;
    yielded = valid && (h0 > 0.0);
    if (yielded) {
      double dtmp;
      const double top = yield_eval_h<YH>(a.ynet, a.yL, a.yN0, sub, psi_e, sc, dtmp);
      double lo = kn, hi = fmax(fmax(kn, phi), top);
      double k = kn, h = h0;
      bool conv = false;
      for (int it = 0; it < a.max_local; ++it) {
        // Newton correction from the current iterate; the convergence test comes
        // before the bracket safeguard so that a root reached on the bracket's
        // end is accepted rather than bisected away from.
        const double fk = exp(-M.eta * fmax(k - M.kd, 0.0));
        const double dq = gb / (M.eta * fk) * (-1.0 + ((k > M.kd) ? M.eta * (phi - k) : 0.0));
        const double dk = -h / (dNy * dq - 1.0);
        if (fabs(dk) <= 1e-15 * fmax(1.0, fabs(k))) {
          k = fmin(fmax(k + dk, lo), hi);
          conv = true;
          break;
        }
        double kn1 = k + dk;
        if (!(kn1 > lo && kn1 < hi)) kn1 = 0.5 * (lo + hi);
        k = kn1;
        const double fk1 = exp(-M.eta * fmax(k - M.kd, 0.0));
        const double qk = psi_e + gb * (phi - k) / (M.eta * fk1);
        h = yield_eval_h<YH>(a.ynet, a.yL, a.yN0, sub, qk, sc, dNy) - k;
        if (h > 0.0) lo = k; else hi = k;
        if (h == 0.0 || !(hi > lo)) { conv = true; break; }
      }
      if (!conv) a.status[0] = GEDMG_E_LOCAL_NOCONV;
      kap = k;
    }
  }
  s.f = exp(-M.eta * fmax(kap - M.kd, 0.0));
  s.fp = (kap > M.kd) ? -M.eta * s.f : 0.0;
  if (yielded) {
    const double dq = gb / (M.eta * s.f) * (-1.0 + ((kap > M.kd) ? M.eta * (phi - kap) : 0.0));
    const double hk = dNy * dq - 1.0;
    s.rhoF = -dNy / hk;
    s.kphi = -dNy * gb / (M.eta * s.f) / hk;
  } else {
    s.rhoF = 0.0;
    s.kphi = 0.0;
  }

  // ---------------- conjugates Pz = (P, dPsi/dphi, Y_vec) and the tangent
  if (sub == 0) {
#pragma unroll
    for (int i = 0; i < DIM; ++i)
#pragma unroll
      for (int j = 0; j < DIM; ++j) S.Pz[g][i * DIM + j] = s.f * s.psiF[i * 3 + j] - M.c * s.w[i] * s.v[j];
    S.Pz[g][DIM * DIM] = M.beta * (phi - kap);
#pragma unroll
    for (int j = 0; j < DIM; ++j) S.Pz[g][DIM * DIM + 1 + j] = M.c * s.v[j];
    if (valid) a.kappa_out[qg] = kap;
  }
  if (TANGENT) {
    wave_lds_sync();
    for (int idx = sub; idx < T::NZ * T::NZ; idx += 8) {
      const int r = idx / T::NZ, c = idx % T::NZ;
      S.D[g][r][c] = d_entry(S.qs[g], M, z3<DIM>(r), z3<DIM>(c));
    }
  }
  __syncthreads();

  // ---------------- element residual: lanes own element dofs
  {
    const int eslot = (DIM == 3) ? 0 : (lane >> 5);
    const int dl = (DIM == 3) ? lane : (lane & 31);
    const bool own = (DIM == 3 ? lane < T::NDOFE : dl < T::NDOFE) &&
                     (slot_base + eslot < a.e_end);
    if (own) {
      const int ae = a.perm[slot_base + eslot];
      const int an = dl / T::ND, cc = dl % T::ND;
      double acc = 0.0;
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
      const int nodea = a.conn[(long)ae * T::NEN + an];
      a.R[(long)nodea * T::ND + cc] += acc;
    }
  }
  if (!TANGENT) return;

  // ---------------- element tangent: lane owns one column and a block of rows
  {
    constexpr int RPL = (DIM == 3) ? 16 : 6;   // rows per lane
    const int eslot = (DIM == 3) ? 0 : (lane >> 5);
    const int li = (DIM == 3) ? lane : (lane & 31);
    const int col = li % T::NDOFE;
    const int rb = (li / T::NDOFE) * RPL;
    const bool own = (DIM == 3 ? true : li < 2 * T::NDOFE) && (slot_base + eslot < a.e_end);
    if (!own) return;
    const int bnode = col / T::ND, kc = col % T::ND;
    double Kacc[RPL];
#pragma unroll
    for (int t = 0; t < RPL; ++t) Kacc[t] = 0.0;
    for (int qq = 0; qq < T::NQP; ++qq) {
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
    const int ae = a.perm[slot_base + eslot];
    const int32_t* blk = a.blk + (long)ae * T::NEN * T::NEN;
#pragma unroll
    for (int t = 0; t < RPL; ++t) {
      const int r = rb + t;
      const int an = r / T::ND, cr = r % T::ND;
      const int nodea = a.conn[(long)ae * T::NEN + an];
      const long off = (long)blk[an * T::NEN + bnode] + (long)cr * a.rowstride[nodea] + kc;
      a.K[off] += Kacc[t];
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

template <int DIM, bool TAN>
static void launch_elem_t(const ElemArgs& a, int blocks, hipStream_t s) {
  if (a.yH == 16)
    hipLaunchKernelGGL((element_kernel<DIM, TAN, 16>), dim3(blocks), dim3(64), 0, s, a);
  else
    hipLaunchKernelGGL((element_kernel<DIM, TAN, 32>), dim3(blocks), dim3(64), 0, s, a);
}

hipError_t launch_element(int dim, bool tangent, const ElemArgs& a, int, hipStream_t s, int) {
  if (a.yH != 16 && a.yH != 32) return hipErrorInvalidValue;
  const int epw = dim == 3 ? 1 : 2;
  const int n = a.e_end - a.e_begin;
  const int blocks = (n + epw - 1) / epw;
  if (blocks == 0) return hipSuccess;
  if (dim == 3) {
    if (tangent) launch_elem_t<3, true>(a, blocks, s);
    else launch_elem_t<3, false>(a, blocks, s);
  } else {
    if (tangent) launch_elem_t<2, true>(a, blocks, s);
    else launch_elem_t<2, false>(a, blocks, s);
  }
  return hipGetLastError();
}

}  // namespace gedmg
