// Global Newton step of the monolithic scheme (Sec. 3.2: history updated in
// every global iteration, tangent contributions of kappa included; each step
// starts from the caller's predictor built on the last converged solution)
// with a preconditioned Krylov solve per iteration.  The CG preconditioner is
// two-level: Jacobi plus a coarse correction on node aggregates (piecewise
// constant per aggregate and dof component), whose span holds the uniform
// damage field: once the points yield, the damage block's only stiffness
// against a uniform phi is beta_d (1 - d kappa / d phi), orders of magnitude
// below the rest of the spectrum, and this mode and the aggregates' smooth
// modes would otherwise set the CG iteration count.
//
// Sparse kernels are deterministic: fixed grids, per-block partial sums in a
// fixed order, one-block final reductions; Krylov scalars stay on the device
// and the host polls the residual norm only every few iterations.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "gedmg_internal.h"

namespace gedmg {

constexpr int kRedBlocks = 512;  // blocks of every reduction kernel
// Krylov solves multiply an ELL copy of the masked matrix: kEllSlots slots per
// lane, 1 to kEllMaxLanes lanes per row, enough for the longest row.
constexpr int kEllSlots = 27;
constexpr int kEllMaxLanes = 64;
constexpr int kEllMaxBlocks = 8192;  // grid cap of the ELL products (partials)
// Two-level preconditioner: at most kCoarseMax coarse dofs (the dense inverse
// is formed in LDS), and the aggregate-aligned update kernel's grid.
constexpr int kCoarseMax = 128;
constexpr int kUpdMaxBlocks = 1024;
constexpr int kMaxBacktracks = 12;  // halvings of one Newton correction
constexpr int kThreads = 256;

gedmg_solver_opts default_solver_opts() {
  gedmg_solver_opts o{};
  o.max_newton = 25;
  o.max_krylov = 20000;
  o.max_local = 100;
  o.newton_rtol = 1e-10;
  o.newton_atol = 0.0;
  o.krylov_rtol = 1e-12;
  o.krylov_forcing = 1;
  o.refine_max = 10;
  o.refine_rtol = 1e-8;
  o.scheme = GEDMG_MONOLITHIC;
  o.newton_rscale = 1.0;
  o.krylov_method = 0;
  return o;
}

// Device scalar slots (doubles).
// S_FLAG + 1 holds sums read back by the host; S_RDR = r.D^-1.r and S_RZC =
// r_c . A_c^-1 r_c of the current CG residual (r.z = S_RDR + S_RZC).
enum Slot { S_RZ = 0, S_PAP, S_ALPHA, S_BETA, S_RR, S_BB, S_RHO, S_OMEGA, S_TT, S_TS, S_VR, S_RZNEW,
            S_FLAG, S_RDR = 15, S_RZC = 16, S_NSLOTS = 17 };


__device__ __forceinline__ double block_sum(double v, double* sh) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  __syncthreads();
  if (l == 0) sh[w] = v;
  __syncthreads();
  double t = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += sh[i];
  return t;  // valid in thread 0
}

// ------------------------------------------------------------------ field kernels
__global__ void set_dirichlet_kernel(double* u, double* phi, const int32_t* dof, const double* val,
                                     int n, int dim, int n_nodes, uint8_t* mask, double* scal) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = dof[i];
  if (d < 0 || d >= n_nodes * (dim + 1)) {  // caller index out of range: flag, write nothing
    scal[S_FLAG] = 3.0;
    return;
  }
  const int node = d / (dim + 1), c = d % (dim + 1);
  if (c < dim)
    u[(long)c * n_nodes + node] = val[i];
  else
    phi[node] = val[i];
  mask[d] = 1;
}

// Prescribed dofs at lambda times their unit values (arc-length continuation).
__global__ void set_dirichlet_scaled_kernel(double* u, double* phi, const int32_t* dof, const double* val,
                                            double lambda, int n, int dim, int n_nodes) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = dof[i];  // range checked by set_mask_kernel before the first use
  const int node = d / (dim + 1), c = d % (dim + 1);
  if (c < dim)
    u[(long)c * n_nodes + node] = lambda * val[i];
  else
    phi[node] = lambda * val[i];
}

__global__ void scatter_kernel(double* y, const int32_t* idx, const double* val, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[idx[i]] = val[i];
}

// b = -y with Dirichlet rows zeroed.
__global__ void masked_neg_kernel(const double* y, const uint8_t* mask, double* b, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = mask[i] ? 0.0 : -y[i];
}

__global__ void axpy_scalar_kernel(double* y, double alpha, const double* x, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = fma(alpha, x[i], y[i]);
}

__global__ void scale_copy_kernel(double* y, double alpha, const double* x, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = alpha * x[i];
}

// inc = (u, phi) - (ub, phib) in the node-major dof layout, zero on Dirichlet rows.
__global__ void field_increment_kernel(const double* u, const double* phi, const double* ub, const double* phib,
                                       const uint8_t* mask, double* inc, int dim, int n_nodes) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_nodes * (dim + 1)) return;
  const int node = (int)(i / (dim + 1)), c = (int)(i % (dim + 1));
  const double v = (c < dim) ? u[(long)c * n_nodes + node] - ub[(long)c * n_nodes + node] : phi[node] - phib[node];
  inc[i] = mask[i] ? 0.0 : v;
}

__global__ void update_fields_kernel(double* u, double* phi, const double* delta, int dim, int n_nodes) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_nodes * (dim + 1)) return;
  const int node = (int)(i / (dim + 1)), c = (int)(i % (dim + 1));
  if (c < dim)
    u[(long)c * n_nodes + node] += delta[i];
  else
    phi[node] += delta[i];
}

// Halve the last Newton correction: x holds it on entry and half of it on
// exit, and the fields lose that half.
__global__ void backtrack_kernel(double* u, double* phi, double* x, int dim, int n_nodes) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (long)n_nodes * (dim + 1)) return;
  const double d = 0.5 * x[i];
  x[i] = d;
  const int node = (int)(i / (dim + 1)), c = (int)(i % (dim + 1));
  if (c < dim)
    u[(long)c * n_nodes + node] -= d;
  else
    phi[node] -= d;
}

__global__ void set_mask_kernel(const int32_t* dof, int n, long ndof, uint8_t* mask, double* scal) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const int d = dof[i];
  if (d < 0 || d >= ndof) {
    scal[S_FLAG] = 3.0;
    return;
  }
  mask[d] = 1;
}

// b = rhs with Dirichlet rows zeroed.
__global__ void masked_copy_kernel(const double* rhs, const uint8_t* mask, double* b, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = mask[i] ? 0.0 : rhs[i];
}

// b = rhs - Ax with Dirichlet rows zeroed (Ax given).
__global__ void masked_residual_kernel(const double* rhs, const double* Ax, const uint8_t* mask, double* b,
                                       long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = mask[i] ? 0.0 : rhs[i] - Ax[i];
}

__global__ void add_kernel(double* x, const double* d, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] += d[i];
}

// b = -R with Dirichlet rows zeroed; partial sums of |b|^2 and non-finite flag.
__global__ void rhs_kernel(const double* R, const uint8_t* mask, double* b, long n, double* part) {
  __shared__ double sh[8];
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    const double v = mask[i] ? 0.0 : -R[i];
    b[i] = v;
    s += v * v;
  }
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// Dirichlet rows / columns of K become identity rows / zero columns; the
// inverse diagonal is stored for the Jacobi preconditioner.
__global__ void mask_matrix_kernel(double* K, const int32_t* rowptr, const int32_t* col,
                                   const uint8_t* mask, double* dinv, long nrows) {
  const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nrows) return;
  const bool mr = mask[r];
  double diag = 1.0;
  for (int j = rowptr[r]; j < rowptr[r + 1]; ++j) {
    const int c = col[j];
    if (mr || mask[c]) K[j] = (c == r) ? 1.0 : 0.0;
    if (c == r) diag = K[j];
  }
  dinv[r] = (diag != 0.0) ? 1.0 / diag : 1.0;
}

// y = K x (rows served by groups of G lanes) and partial sums of w . y.
template <int G>
__global__ void spmv_dot_kernel(const double* K, const int32_t* rowptr, const int32_t* col,
                                const double* x, double* y, const double* w, long nrows, double* part) {
  __shared__ double sh[8];
  const int lane = threadIdx.x % G;
  const long groups = (long)gridDim.x * (blockDim.x / G);
  double acc_dot = 0.0;
  for (long r = (long)blockIdx.x * (blockDim.x / G) + threadIdx.x / G; r < nrows; r += groups) {
    double s = 0.0;
    for (int j = rowptr[r] + lane; j < rowptr[r + 1]; j += G) s += K[j] * x[col[j]];
#pragma unroll
    for (int o = G / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, G);
    if (lane == 0) {
      y[r] = s;
      if (w) acc_dot += w[r] * s;
    }
  }
  const double t = block_sum(acc_dot, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void dot2_kernel(const double* a, const double* b, const double* c, const double* d, long n,
                            double* part) {
  __shared__ double sh[8];
  double s1 = 0.0, s2 = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    s1 += a[i] * b[i];
    if (c) s2 += c[i] * d[i];
  }
  const double t1 = block_sum(s1, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t1;
  const double t2 = block_sum(s2, sh);
  if (threadIdx.x == 0) part[kRedBlocks + blockIdx.x] = t2;
}

// Partials of a . b with the nonlocal damage dofs (every nd-th, last of a
// node) weighted by w2 and the others by 1: the arc-length norm.
__global__ void wdot_kernel(const double* a, const double* b, long n, int nd, double w2, double* part) {
  __shared__ double sh[8];
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    s += ((i % nd) == nd - 1 ? w2 : 1.0) * a[i] * b[i];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// One-block reduction of np partials into scal[slot] (fixed order); a second
// array of np partials at part + kRedBlocks goes to scal[slot2].
__global__ void reduce_kernel(const double* part, double* scal, int slot, int slot2, int np) {
  __shared__ double sh[8];
  double s = 0.0, s2 = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) {
    s += part[i];
    if (slot2 >= 0) s2 += part[kRedBlocks + i];
  }
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) scal[slot] = t;
  if (slot2 >= 0) {
    const double t2 = block_sum(s2, sh);
    if (threadIdx.x == 0) scal[slot2] = t2;
  }
}

// ---- CG pieces.  The preconditioner is two-level (additive):
//   M^-1 r = D^-1 r + P A_c^-1 P^T r,   A_c = P^T K P,
// P the piecewise-constant prolongation from node aggregates (boxes of the
// mesh's bounding box), one coarse dof per aggregate and dof component, zero on
// Dirichlet dofs.  The coarse space holds the uniform damage field over the
// free damage dofs, the soft mode of a yielding tangent (stiffness beta_d
// (1 - d kappa / d phi), orders of magnitude below the rest of the spectrum),
// and the aggregates' smooth modes that set Jacobi-CG's iteration count.  A_c
// (at most kCoarseMax dofs) is assembled and inverted densely at the start of
// a solve (a solve with the previous one's matrix keeps it); BiCGStab applies
// the same M.  In CG z = M^-1 r is never stored: the update kernel leaves D^-1 r
// and partials, a one-block kernel the coarse correction y_c = A_c^-1 P^T r
// with the scalars r.D^-1.r, r_c.y_c and r.r, and the direction kernel forms z
// on the fly.  r.z of the current and of the previous direction alternate
// between two slots.

// A_c from the masked matrix: one block per coarse nonzero sums, in a fixed
// order, the entries of K whose row and column are free and map to it (seg_e
// lists them by coarse nonzero, seg_row their rows).
__global__ __launch_bounds__(256) void coarse_matrix_kernel(const double* K, const int32_t* col,
                                                            const int32_t* seg_ptr, const int32_t* seg_key,
                                                            const int32_t* seg_e, const int32_t* seg_row,
                                                            const uint8_t* mask, double* Ac) {
  __shared__ double sh[8];
  const int seg = blockIdx.x;
  double v = 0.0;
  for (int k = seg_ptr[seg] + threadIdx.x; k < seg_ptr[seg + 1]; k += blockDim.x) {
    const int e = seg_e[k];
    if (!mask[seg_row[k]] && !mask[col[e]]) v += K[e];
  }
  const double t = block_sum(v, sh);
  if (threadIdx.x == 0) Ac[seg_key[seg]] = t;
}

// Gauss-Jordan inverse of A_c (nc <= kCoarseMax) in one block of 1024
// threads: thread t owns row t / 8, columns t % 8 + 8 m, in registers.  No
// pivoting (A_c is symmetric positive definite for a symmetric positive
// definite tangent, and Gauss-Jordan without interchanges is stable there); a
// pivot not above 1e-13 of the largest diagonal entry of A_c leaves the coarse
// correction out of this solve (zero inverse: plain Jacobi).  A
// coarse dof without free dofs has a zero row and column and gets a unit
// diagonal.  Writes the transpose of the inverse (for coalesced products).
__global__ __launch_bounds__(1024) void coarse_invert_kernel(const double* Ac, int nc, double* AinvT) {
  constexpr int M = kCoarseMax / 8;
  __shared__ double prow[2][kCoarseMax];
  __shared__ double colk[2][kCoarseMax];
  __shared__ double dmax_w[16];
  __shared__ int singular;
  const int t = threadIdx.x;
  const int ti = t >> 3, tj = t & 7;
  const bool own = ti < nc;
  double a[M];
#pragma unroll
  for (int m = 0; m < M; ++m) {
    const int j = tj + 8 * m;
    a[m] = (own && j < nc) ? Ac[ti * nc + j] : 0.0;
  }
  double dmax = 0.0;
#pragma unroll
  for (int m = 0; m < M; ++m)
    if (own && tj + 8 * m == ti) {
      if (a[m] == 0.0) a[m] = 1.0;  // a coarse dof without free dofs
      dmax = fabs(a[m]);
    }
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) dmax = fmax(dmax, __shfl_xor(dmax, o, 64));
  if ((t & 63) == 0) dmax_w[t >> 6] = dmax;
  if (t == 0) singular = 0;
  __syncthreads();
  double dm = 0.0;
  for (int w = 0; w < (int)(blockDim.x >> 6); ++w) dm = fmax(dm, dmax_w[w]);
  const double tiny = 1e-13 * dm;
  for (int k = 0; k < nc; ++k) {
    double* pr = prow[k & 1];
    double* ck = colk[k & 1];
    // column k of every row, and row k scaled by its pivot (in-place: the
    // pivot's own entry becomes 1 / pivot)
    if (own && tj == (k & 7)) {
      double v = 0.0;
#pragma unroll
      for (int m = 0; m < M; ++m)
        if (m == (k >> 3)) v = a[m];
      ck[ti] = v;
    }
    __syncthreads();
    const double piv = ck[k];
    if (!(fabs(piv) > tiny)) {
      if (t == 0) singular = 1;
      break;
    }
    const double pivinv = 1.0 / piv;
    if (ti == k) {
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int j = tj + 8 * m;
        const double v = (j == k ? 1.0 : a[m]) * pivinv;
        a[m] = v;
        if (j < nc) pr[j] = v;
      }
    }
    __syncthreads();
    if (own && ti != k) {
      const double f = ck[ti];
#pragma unroll
      for (int m = 0; m < M; ++m) {
        const int j = tj + 8 * m;
        if (j < nc) a[m] = (j == k ? 0.0 : a[m]) - f * pr[j];
      }
    }
  }
  __syncthreads();
  if (singular) {
    for (int i = t; i < nc * nc; i += blockDim.x) AinvT[i] = 0.0;
    return;
  }
  if (own) {
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int j = tj + 8 * m;
      if (j < nc) AinvT[j * nc + ti] = a[m];
    }
  }
}

// Every block sums the np partials of p.Ap of the sparse product itself (same
// order in every block, so all blocks get the same alpha); block 0 publishes it.
__device__ __forceinline__ double block_total(const double* part, int np, double* sh, double* bc) {
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += blockDim.x) s += part[i];
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) *bc = t;
  __syncthreads();
  return *bc;
}

// x += alpha p, r -= alpha q, zd = D^-1 r, over the dofs of node aggregates:
// block b serves aggregate b / sub (its dofs agg_dofs[agg_ptr[a] ..
// agg_ptr[a + 1]), one sub-block of sub), and leaves partials of r.D^-1.r,
// r.r and, per component, of r over its dofs (the restriction P^T r).
// init = 1 leaves x and r as they are (the first residual).  The vector
// operands of a block's first dof are loaded before its sum of the p.q
// partials.
__global__ __launch_bounds__(256) void cg_update_kernel(double* x, double* r, const double* p, const double* q,
                                                        const double* dinv, double* zd, const int32_t* agg_ptr,
                                                        const int32_t* agg_dofs, int sub, int nd,
                                                        const double* part_pap, int npap, double* scal, int cur,
                                                        int init, double* part, double* partc) {
  __shared__ double sh[8];
  __shared__ double bc;
  const int a = blockIdx.x / sub, s = blockIdx.x % sub;
  const int k_end = agg_ptr[a + 1];
  const int stride = sub * blockDim.x;
  int k = agg_ptr[a] + s * blockDim.x + threadIdx.x;
  int i = k < k_end ? agg_dofs[k] : 0;
  double xi = 0.0, ri = 0.0, pi = 0.0, qi = 0.0, di = 0.0;
  if (k < k_end) {
    ri = r[i];
    di = dinv[i];
    if (!init) {
      xi = x[i];
      pi = p[i];
      qi = q[i];
    }
  }
  double alpha = 0.0;
  if (!init) {
    const double pap = block_total(part_pap, npap, sh, &bc);
    alpha = (pap > 0.0) ? scal[cur] / pap : 0.0;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
      scal[S_PAP] = pap;
      if (!(pap > 0.0)) scal[S_FLAG] = 1.0;  // non-positive curvature
    }
  }
  double s1 = 0.0, s2 = 0.0, c0 = 0.0, c1 = 0.0, c2 = 0.0, c3 = 0.0;
  while (k < k_end) {
    double rn = ri;
    if (!init) {
      x[i] = xi + alpha * pi;
      rn = ri - alpha * qi;
      r[i] = rn;
    }
    const double zi = di * rn;
    zd[i] = zi;
    s1 += rn * zi;
    s2 += rn * rn;
    const int comp = i % nd;
    c0 += comp == 0 ? rn : 0.0;
    c1 += comp == 1 ? rn : 0.0;
    c2 += comp == 2 ? rn : 0.0;
    c3 += comp == 3 ? rn : 0.0;
    k += stride;
    if (k < k_end) {
      i = agg_dofs[k];
      ri = r[i];
      di = dinv[i];
      if (!init) {
        xi = x[i];
        pi = p[i];
        qi = q[i];
      }
    }
  }
  // the six sums: wavefront shuffles, then the block's wavefronts in order
  __shared__ double shv[6][4];
  double v[6] = {s1, s2, c0, c1, c2, c3};
#pragma unroll
  for (int qq = 0; qq < 6; ++qq) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[qq] += __shfl_xor(v[qq], o, 64);
    if ((threadIdx.x & 63) == 0) shv[qq][threadIdx.x >> 6] = v[qq];
  }
  __syncthreads();
  if (threadIdx.x < 6) {
    const int qq = threadIdx.x;
    double tsum = 0.0;
    for (int w = 0; w < (int)(blockDim.x >> 6); ++w) tsum += shv[qq][w];
    if (qq == 0) part[blockIdx.x] = tsum;
    else if (qq == 1) part[kUpdMaxBlocks + blockIdx.x] = tsum;
    else partc[blockIdx.x * 4 + (qq - 2)] = tsum;
  }
}

// One block of 1024 threads: the update kernel's nb partials summed in a fixed
// order into r.D^-1.r (scal[S_RDR]) and r.r (scal[S_RR]), the restriction r_c
// = P^T r, the coarse correction y_c = A_c^-1 r_c (yc) and r_c.y_c
// (scal[S_RZC]).  Thread t serves coarse dof t % 128 and an eighth (t / 128)
// of each sum; the eighths are added in order.
__global__ __launch_bounds__(1024) void coarse_tail_kernel(const double* part, const double* partc, int nb, int sub,
                                                           int nd, int nc, const double* AinvT, double* scal,
                                                           double* yc) {
  __shared__ double ph[8][kCoarseMax];
  __shared__ double rcs[kCoarseMax];
  __shared__ double sh[3][16];
  const int t = threadIdx.x;
  const int c = t & (kCoarseMax - 1), q = t >> 7;
  // this thread's entries of A_c^-1 first (they do not depend on the sums):
  // rows j = q + 8 m of column c, addresses clamped into the matrix
  constexpr int M = kCoarseMax / 8;
  double ai[M];
  {
    const int cc = c < nc ? c : nc - 1;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int j = q + 8 * m;
      ai[m] = AinvT[(j < nc ? j : nc - 1) * nc + cc];
    }
  }
  double S1 = 0.0, S2 = 0.0;
  for (int b = t; b < nb; b += blockDim.x) {
    S1 += part[b];
    S2 += part[kUpdMaxBlocks + b];
  }
  if (c < nc) {
    const int ag = c / nd, comp = c - ag * nd;
    double v = 0.0;
    for (int j = q; j < sub; j += 8) v += partc[(ag * sub + j) * 4 + comp];
    ph[q][c] = v;
  }
  __syncthreads();
  if (t < nc) {
    double v = 0.0;
    for (int qq = 0; qq < 8; ++qq) v += ph[qq][t];
    rcs[t] = v;
  }
  __syncthreads();
  if (c < nc) {
    double y = 0.0;
#pragma unroll
    for (int m = 0; m < M; ++m) {
      const int j = q + 8 * m;
      if (j < nc) y += ai[m] * rcs[j];
    }
    ph[q][c] = y;
  }
  __syncthreads();
  double rzc = 0.0;
  if (t < nc) {
    double y = 0.0;
    for (int qq = 0; qq < 8; ++qq) y += ph[qq][t];
    yc[t] = y;
    rzc = rcs[t] * y;
  }
  // the three sums: wavefront shuffles, then the 16 wavefronts in order
  double v[3] = {S1, S2, rzc};
#pragma unroll
  for (int k = 0; k < 3; ++k) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v[k] += __shfl_xor(v[k], o, 64);
    if ((t & 63) == 0) sh[k][t >> 6] = v[k];
  }
  __syncthreads();
  if (t == 0) {
    double T[3] = {0.0, 0.0, 0.0};
    for (int k = 0; k < 3; ++k)
      for (int w = 0; w < (int)(blockDim.x >> 6); ++w) T[k] += sh[k][w];
    scal[S_RDR] = T[0];
    scal[S_RR] = T[1];
    scal[S_RZC] = T[2];
  }
}

// ---- ELL copy of the masked matrix for the Krylov iterations.  Slot s of a
// row (its s-th CSR entry, or a zero past its length) is stored at
// ((s / L) * nrows + row) * L + s % L: the L lanes of a row and consecutive
// rows read consecutive words, and no row length is loaded.  The columns are
// not stored per entry: the pattern is made of nd x nd node blocks, every row
// of node a has the columns (b, 0..nd-1) of its neighbour nodes b in order, so
// slot s lies in column nbr(a, s / nd) * nd + s mod nd.  ncol holds nbr(a, t)
// at t * n_nodes + a, and a itself past the neighbour count (the padding
// slots then fall on the row's own node block, with value zero).
__global__ void ell_ncols_kernel(const int32_t* rowptr, const int32_t* col, long nn, int nd, int nbmax,
                                 int32_t* ncol) {
  const long a = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (a >= nn) return;
  const int j0 = rowptr[a * nd], deg = (rowptr[a * nd + 1] - j0) / nd;
  for (int t = 0; t < nbmax; ++t) ncol[(long)t * nn + a] = t < deg ? col[j0 + t * nd] / nd : (int32_t)a;
}

// Blocks are dealt to the 8 XCDs round-robin (block b to XCD b mod 8).  The
// ELL kernels use logical block xcd_block(b) instead, which gives every XCD a
// contiguous range of row groups, so that the neighbouring rows a row's
// columns gather are mostly in the same XCD's L2.  A bijection of [0, nb).
__device__ __forceinline__ int xcd_block(int b, int nb) {
  const int q = nb >> 3, r = nb & 7, x = b & 7;
  return x * q + min(x, r) + (b >> 3);
}

// column of slot k of lane `lane` in row group of node a (see ell_ncols_kernel)
template <int L, int ND>
__device__ __forceinline__ int32_t ell_col(const int32_t* ncol, long nn, long a, int k, int lane) {
  const int s = k * L + lane;
  return ncol[(long)(s / ND) * nn + a] * ND + s % ND;
}

// ELL values of K, and the coarse dof of every free dof (-1 on Dirichlet dofs)
// for this solve's mask
__global__ void ell_pack_kernel(const double* K, const int32_t* rowptr, const uint8_t* mask, const int32_t* cmap0,
                                long nrows, int L, double* eval, int32_t* cmap) {
  const long row = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (row >= nrows) return;
  const int j0 = rowptr[row], len = rowptr[row + 1] - j0;
  for (int s = 0; s < L * kEllSlots; ++s)
    eval[((long)(s / L) * nrows + row) * L + s % L] = s < len ? K[j0 + s] : 0.0;
  cmap[row] = mask[row] ? -1 : cmap0[row];
}

// y = K x from the ELL copy (L lanes per row, ND dofs per node) and partials of w . y
template <int L, int ND>
__global__ __launch_bounds__(256) void ell_spmv_kernel(const double* eval, const int32_t* ncol, const double* x,
                                                       double* y, const double* w, long nrows, double* part) {
  const long nn = nrows / ND;
  __shared__ double sh[8];
  const int lane = threadIdx.x % L;
  const long groups = (long)gridDim.x * (blockDim.x / L);
  double acc = 0.0;
  const int lb = xcd_block(blockIdx.x, gridDim.x);
  for (long row = (long)lb * (blockDim.x / L) + threadIdx.x / L; row < nrows; row += groups) {
    double s = 0.0;
    const long a = row / ND;
#pragma unroll
    for (int k = 0; k < kEllSlots; ++k)
      s += eval[((long)k * nrows + row) * L + lane] * x[ell_col<L, ND>(ncol, nn, a, k, lane)];
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, L);
    if (lane == 0) {
      y[row] = s;
      if (w) acc += w[row] * s;
    }
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

// The slots of one row of the ELL copy with every operand of its product that
// does not depend on this iteration's scalars: column values, and D^-1 r, the
// previous direction and the coarse dof at each column and at the row itself.
struct EllRow {
  double val[kEllSlots], zd[kEllSlots], po[kEllSlots];
  int32_t cm[kEllSlots];
  double zd_own, po_own;
  int32_t cm_own;
};

template <int L, int ND>
__device__ __forceinline__ void ell_row_load(EllRow& e, long row, int lane, long nrows, const double* eval,
                                             const int32_t* ncol, const double* zd, const int32_t* cmap,
                                             const double* p_old) {
  if (row >= nrows) return;
  const long nn = nrows / ND, a = row / ND;
  int col[kEllSlots];
#pragma unroll
  for (int k = 0; k < kEllSlots; ++k) {
    col[k] = ell_col<L, ND>(ncol, nn, a, k, lane);
    e.val[k] = eval[((long)k * nrows + row) * L + lane];
  }
#pragma unroll
  for (int k = 0; k < kEllSlots; ++k) {
    e.zd[k] = zd[col[k]];
    e.po[k] = p_old[col[k]];
    e.cm[k] = cmap[col[k]];
  }
  e.zd_own = zd[row];
  e.po_own = p_old[row];
  e.cm_own = cmap[row];
}

// Entry of the new search direction p = z + beta p_old, z = D^-1 r + P y_c,
// from the loaded operands (ys: y_c in LDS).  The first direction is z: beta
// = 0 and p_old is zeroed at the start of the solve.
__device__ __forceinline__ double cg_dir(double zd, double po, int32_t cm, const double* ys, double beta) {
  return fma(beta, po, zd + (cm >= 0 ? ys[cm] : 0.0));
}

// The new search direction and its product in one launch: (r.z)_new =
// r.D^-1.r + r_c.y_c from the one-block sums, beta = (r.z)_new /
// scal[prv]; block 0 publishes (r.z)_new in scal[cur].  The operands of a row's
// product do not depend on these scalars, so the first row's loads are issued
// before them.  A row group forms the direction of every column it touches
// with the same operations as the column's own row, which alone stores it
// (p_old and p_new are two buffers); q = K p_new and partials of p_new . q.
template <int L, int ND, bool LOOP>
__global__ __launch_bounds__(256) void cg_dir_spmv_kernel(const double* eval, const int32_t* ncol, const double* zd,
                                                          const int32_t* cmap, const double* yc, int nc,
                                                          const double* p_old, double* p_new, double* q,
                                                          double* scal, int cur, int prv, int first, long nrows,
                                                          double* part_pap) {
  __shared__ double sh[8];
  __shared__ double ys[kCoarseMax];
  const int lane = threadIdx.x % L;
  const long groups = (long)gridDim.x * (blockDim.x / L);
  long row = (long)xcd_block(blockIdx.x, gridDim.x) * (blockDim.x / L) + threadIdx.x / L;
  EllRow e;
  ell_row_load<L, ND>(e, row, lane, nrows, eval, ncol, zd, cmap, p_old);
  for (int c = threadIdx.x; c < nc; c += blockDim.x) ys[c] = yc[c];
  const double rz_new = scal[S_RDR] + scal[S_RZC];
  const double rz = first ? 0.0 : scal[prv];
  const double beta = (!first && rz != 0.0) ? rz_new / rz : 0.0;
  if (blockIdx.x == 0 && threadIdx.x == 0) scal[cur] = rz_new;
  __syncthreads();
  double acc = 0.0;
  // LOOP = false: the grid has a row group for every row (fewer live registers
  // than the loop's prefetch of the next row, two waves per SIMD instead of one)
  for (; row < nrows; row += groups) {
    double s = 0.0;
#pragma unroll
    for (int k = 0; k < kEllSlots; ++k) s += e.val[k] * cg_dir(e.zd[k], e.po[k], e.cm[k], ys, beta);
#pragma unroll
    for (int o = L / 2; o > 0; o >>= 1) s += __shfl_xor(s, o, L);
    if (lane == 0) {
      const double pi = cg_dir(e.zd_own, e.po_own, e.cm_own, ys, beta);
      p_new[row] = pi;
      q[row] = s;
      acc += pi * s;
    }
    if (!LOOP) break;
    ell_row_load<L, ND>(e, row + groups, lane, nrows, eval, ncol, zd, cmap, p_old);
  }
  const double t = block_sum(acc, sh);
  if (threadIdx.x == 0) part_pap[blockIdx.x] = t;
}

// z += P y_c (the coarse correction's prolongation; -1 marks a Dirichlet dof)
__global__ void coarse_prolong_kernel(double* z, const int32_t* cmap, const double* yc, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && cmap[i] >= 0) z[i] += yc[cmap[i]];
}

// ---- BiCGStab pieces (right preconditioning with the two-level M)
// p = r + beta (p - omega v), beta = (rho_new/rho) (alpha/omega)
__global__ void bicg_p_kernel(double* p, const double* r, const double* v, const double* scal, long n) {
  const double beta = scal[S_BETA], omega = scal[S_OMEGA];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    p[i] = r[i] + beta * (p[i] - omega * v[i]);
}

__global__ void bicg_scalars_kernel(double* scal, int stage) {
  if (stage == 0) {  // after rho_new = r0 . r: beta
    const double rho = scal[S_RHO], rn = scal[S_RZNEW];
    const double om = scal[S_OMEGA], al = scal[S_ALPHA];
    if (rho == 0.0 || om == 0.0) scal[S_FLAG] = 2.0;
    scal[S_BETA] = (rho != 0.0 && om != 0.0) ? (rn / rho) * (al / om) : 0.0;
    scal[S_RHO] = rn;
  } else if (stage == 1) {  // after vr = r0 . v: alpha
    const double vr = scal[S_VR];
    if (vr == 0.0) scal[S_FLAG] = 2.0;
    scal[S_ALPHA] = (vr != 0.0) ? scal[S_RHO] / vr : 0.0;
  } else {  // after tt = t.t, ts = t.s: omega
    const double tt = scal[S_TT];
    scal[S_OMEGA] = (tt > 0.0) ? scal[S_TS] / tt : 0.0;
    if (!(tt > 0.0)) scal[S_FLAG] = 2.0;
  }
}

// s = r - alpha v (stored in r)
__global__ void bicg_s_kernel(double* r, const double* v, const double* scal, long n) {
  const double alpha = scal[S_ALPHA];
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    r[i] -= alpha * v[i];
}

// x += alpha phat + omega shat; r = s - omega t; partial |r|^2
__global__ void bicg_update_kernel(double* x, double* r, const double* ph, const double* sh_, const double* t,
                                   const double* scal, long n, double* part) {
  __shared__ double sh[8];
  const double alpha = scal[S_ALPHA], omega = scal[S_OMEGA];
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) {
    x[i] += alpha * ph[i] + omega * sh_[i];
    const double ri = r[i] - omega * t[i];
    r[i] = ri;
    s += ri * ri;
  }
  const double tt = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = tt;
}

__global__ void count_growth_kernel(const double* k1, const double* k0, long n, double* part) {
  __shared__ double sh[8];
  double s = 0.0;
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x)
    s += (k1[i] > k0[i]) ? 1.0 : 0.0;
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

__global__ void gather_sum_kernel(const double* R, const int32_t* idx, int n, long ndof, double* part) {
  __shared__ double sh[8];
  double s = 0.0;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const int j = idx[i];
    if (j >= 0 && j < ndof) s += R[j];
  }
  const double t = block_sum(s, sh);
  if (threadIdx.x == 0) part[blockIdx.x] = t;
}

}  // namespace gedmg

using namespace gedmg;

namespace {

#define GH(expr)                                                              \
  do {                                                                        \
    hipError_t e_ = (expr);                                                   \
    if (e_ != hipSuccess) {                                                   \
      c->err = std::string(#expr) + ": " + hipGetErrorString(e_);             \
      return GEDMG_E_HIP;                                                     \
    }                                                                         \
  } while (0)

struct Work {
  long ndof = 0, nnz = 0, nq = 0;
  double *K = nullptr, *Kmp = nullptr, *R = nullptr, *Rmp = nullptr, *kt = nullptr, *ktmp = nullptr;
  double *b = nullptr, *x = nullptr, *r = nullptr, *z = nullptr, *p = nullptr, *q = nullptr;
  double *v = nullptr, *t = nullptr, *r0 = nullptr, *dinv = nullptr;
  // Krylov iterations (allocated on the first solve): the ELL copy of the
  // masked matrix (ell_lanes lanes per row), the second direction buffer and
  // D^-1 r
  int ell_lanes = 0;
  int32_t* ell_col = nullptr;
  double *ell_val = nullptr, *p2 = nullptr, *zd = nullptr;
  // two-level preconditioner: n_agg node aggregates, n_coarse = n_agg * nd
  // coarse dofs; cmap0 the coarse dof of every dof, cmap the same with -1 on
  // the solve's Dirichlet dofs; agg_ptr / agg_dofs the dofs of each aggregate;
  // the n_seg coarse nonzeros (seg_key = row * n_coarse + column) with the
  // matrix entries that sum to each (seg_ptr, seg_e, and their rows seg_row);
  // A_c, the transpose of its inverse, y_c and the update kernel's partials
  // of the restriction
  bool krylov_ready = false;
  int n_agg = 0, n_coarse = 0, upd_sub = 1, n_seg = 0;
  int32_t *cmap0 = nullptr, *cmap = nullptr, *agg_ptr = nullptr, *agg_dofs = nullptr;
  int32_t *seg_ptr = nullptr, *seg_key = nullptr, *seg_e = nullptr, *seg_row = nullptr;
  double *Ac = nullptr, *AinvT = nullptr, *yc = nullptr, *partc = nullptr;
  double *ub = nullptr, *phib = nullptr;
  double *part = nullptr, *scal = nullptr, *hscal = nullptr;
  uint8_t* mask = nullptr;
  // arc-length continuation (allocated on its first use): the unit loading
  // pattern, the predictor, the two corrector solutions and K times the pattern
  double *al_uh = nullptr, *al_dp = nullptr, *al_a = nullptr, *al_y = nullptr;
};


}  // namespace

// The context keeps its Newton workspace behind an opaque pointer.
namespace {
struct WorkHolder {
  gedmg_ctx* ctx;
  Work w;
};
std::vector<WorkHolder*>& holders() {
  static std::vector<WorkHolder*> h;
  return h;
}
}  // namespace

namespace gedmg {
void release_newton_work(gedmg_ctx* c) {
  auto& h = holders();
  for (size_t i = 0; i < h.size(); ++i)
    if (h[i]->ctx == c) {
      Work& w = h[i]->w;
      void* ptrs[] = {w.K, w.Kmp, w.R, w.Rmp, w.kt, w.ktmp, w.b, w.x, w.r, w.z, w.p, w.q,
                      w.v, w.t, w.r0, w.dinv, w.ub, w.phib, w.part, w.scal, w.mask,
                      w.al_uh, w.al_dp, w.al_a, w.al_y, w.ell_col, w.ell_val, w.p2, w.zd,
                      w.cmap0, w.cmap, w.agg_ptr, w.agg_dofs, w.seg_ptr, w.seg_key, w.seg_e, w.seg_row,
                      w.Ac, w.AinvT, w.yc, w.partc};
      for (void* p : ptrs)
        if (p) (void)hipFree(p);
      if (w.hscal) (void)hipHostFree(w.hscal);
      delete h[i];
      h.erase(h.begin() + i);
      return;
    }
}
}  // namespace gedmg

namespace {

int ensure_work(gedmg_ctx* c, Work** out) {
  for (auto* h : holders())
    if (h->ctx == c) {
      *out = &h->w;
      return GEDMG_OK;
    }
  auto* h = new WorkHolder{c, Work{}};
  holders().push_back(h);
  Work& w = h->w;
  w.ndof = c->ndof;
  w.nnz = c->nnz;
  w.nq = (long)c->n_elems * c->nqp;
  auto al = [&](double** p, long n) { return hipMalloc((void**)p, sizeof(double) * std::max(n, 1L)); };
  if (al(&w.K, w.nnz) || al(&w.R, w.ndof) || al(&w.Rmp, w.ndof) || al(&w.kt, w.nq) ||
      al(&w.ktmp, w.nq) || al(&w.b, w.ndof) || al(&w.x, w.ndof) || al(&w.r, w.ndof) ||
      al(&w.z, w.ndof) || al(&w.p, w.ndof) || al(&w.q, w.ndof) || al(&w.v, w.ndof) ||
      al(&w.t, w.ndof) || al(&w.r0, w.ndof) || al(&w.dinv, w.ndof) ||
      al(&w.ub, (long)c->dim * c->n_nodes) || al(&w.phib, c->n_nodes) ||
      al(&w.part, std::max(3 * kRedBlocks, 2 * kUpdMaxBlocks) + kEllMaxBlocks) || al(&w.scal, S_NSLOTS) ||
      hipMalloc((void**)&w.mask, std::max(w.ndof, 1L)) ||
      hipHostMalloc((void**)&w.hscal, sizeof(double) * S_NSLOTS, 0)) {
    c->err = "device allocation for the Newton workspace failed";
    gedmg::release_newton_work(c);
    return GEDMG_E_NOMEM;
  }
  *out = &w;
  return GEDMG_OK;
}

// The ELL column layout of the CSR pattern, built on the first Krylov solve:
// the lane count is the smallest power of two whose kEllSlots slots per lane
// hold the longest row.
// The Krylov layouts, built on the first solve: the ELL column layout of the
// CSR pattern (the lane count is the smallest power of two whose kEllSlots
// slots per lane hold the longest row) and the two-level preconditioner's
// aggregates: the mesh's bounding box cut into k^dim boxes, k the largest
// with k^dim * nd <= kCoarseMax, one aggregate per box that holds a node.
int ensure_ell(gedmg_ctx* c, Work& w) {
  if (w.krylov_ready) return GEDMG_OK;
  const long n = w.ndof;
  const int nd = c->dim + 1, nn = c->n_nodes, dim = c->dim;
  std::vector<int32_t> rp(n + 1);
  GH(hipMemcpy(rp.data(), c->drowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost));
  int longest = 1;
  for (long i = 0; i < n; ++i) longest = std::max(longest, rp[i + 1] - rp[i]);
  int L = 1;
  while (L * kEllSlots < longest && L < kEllMaxLanes) L *= 2;
  if (L * kEllSlots < longest) {
    c->err = "a row of the sparse pattern is longer than the Krylov solver's limit of " +
             std::to_string(kEllMaxLanes * kEllSlots) + " entries";
    return GEDMG_E_ARG;
  }
  // aggregates
  std::vector<double> X((size_t)dim * nn);
  GH(hipMemcpy(X.data(), c->dX, sizeof(double) * X.size(), hipMemcpyDeviceToHost));
  int k = 1;
  while (true) {
    long cells = 1;
    for (int d = 0; d < dim; ++d) cells *= (k + 1);
    if (cells * nd > kCoarseMax) break;
    ++k;
  }
  double lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
  for (int d = 0; d < dim; ++d) {
    lo[d] = hi[d] = nn ? X[(size_t)d * nn] : 0.0;
    for (int i = 0; i < nn; ++i) {
      lo[d] = std::min(lo[d], X[(size_t)d * nn + i]);
      hi[d] = std::max(hi[d], X[(size_t)d * nn + i]);
    }
  }
  std::vector<int> box(nn);
  for (int i = 0; i < nn; ++i) {
    int b = 0;
    for (int d = dim - 1; d >= 0; --d) {
      const double ext = hi[d] - lo[d];
      int q = ext > 0.0 ? (int)((X[(size_t)d * nn + i] - lo[d]) / ext * k) : 0;
      q = std::min(std::max(q, 0), k - 1);
      b = b * k + q;
    }
    box[i] = b;
  }
  long ncell = 1;
  for (int d = 0; d < dim; ++d) ncell *= k;
  std::vector<int> agg_of_box(ncell, -1);
  int n_agg = 0;
  for (int i = 0; i < nn; ++i)
    if (agg_of_box[box[i]] < 0) agg_of_box[box[i]] = n_agg++;  // numbered by first node
  const int nc = n_agg * nd;
  std::vector<int32_t> cmap0(n), agg_ptr(n_agg + 1, 0), agg_dofs(n);
  for (long i = 0; i < n; ++i) {
    const int a = agg_of_box[box[i / nd]];
    cmap0[i] = a * nd + (int)(i % nd);
    agg_ptr[a + 1]++;
  }
  for (int a = 0; a < n_agg; ++a) agg_ptr[a + 1] += agg_ptr[a];
  {
    std::vector<int32_t> fill(agg_ptr.begin(), agg_ptr.end() - 1);
    for (long i = 0; i < n; ++i) agg_dofs[fill[cmap0[i] / nd]++] = (int32_t)i;
  }
  // coarse nonzeros: the CSR entries counting-sorted by (coarse row, coarse column)
  const long nnz = rp[n];
  std::vector<int32_t> col(nnz);
  GH(hipMemcpy(col.data(), c->dcol, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost));
  std::vector<int32_t> cnt((size_t)nc * nc + 1, 0);
  for (long i = 0; i < n; ++i)
    for (long e = rp[i]; e < rp[i + 1]; ++e) cnt[(size_t)cmap0[i] * nc + cmap0[col[e]] + 1]++;
  for (size_t q = 0; q < (size_t)nc * nc; ++q) cnt[q + 1] += cnt[q];
  std::vector<int32_t> seg_e(nnz), seg_row(nnz);
  {
    std::vector<int32_t> fill(cnt.begin(), cnt.end() - 1);
    for (long i = 0; i < n; ++i)
      for (long e = rp[i]; e < rp[i + 1]; ++e) {
        const int32_t pos = fill[(size_t)cmap0[i] * nc + cmap0[col[e]]]++;
        seg_e[pos] = (int32_t)e;
        seg_row[pos] = (int32_t)i;
      }
  }
  std::vector<int32_t> seg_ptr(1, 0), seg_key;
  for (size_t q = 0; q < (size_t)nc * nc; ++q)
    if (cnt[q + 1] > cnt[q]) {
      seg_key.push_back((int32_t)q);
      seg_ptr.push_back(cnt[q + 1]);
    }
  const int n_seg = (int)seg_key.size();
  const int sub = std::max(1, std::min(kUpdMaxBlocks / std::max(n_agg, 1), (512 + n_agg - 1) / std::max(n_agg, 1)));

  const long slots = (long)L * kEllSlots * std::max(n, 1L);
  const long nbmax = ((long)L * kEllSlots - 1) / nd + 1;
  const long n1 = std::max(n, 1L), nnz1 = std::max(nnz, 1L);
  auto ai = [&](int32_t** p, long m) { return hipMalloc((void**)p, sizeof(int32_t) * std::max(m, 1L)); };
  auto ad = [&](double** p, long m) { return hipMalloc((void**)p, sizeof(double) * std::max(m, 1L)); };
  if (ai(&w.ell_col, nbmax * std::max(nn, 1)) || ad(&w.ell_val, slots) || ad(&w.p2, n1) || ad(&w.zd, n1) || ai(&w.cmap0, n1) ||
      ai(&w.cmap, n1) || ai(&w.agg_ptr, n_agg + 1) || ai(&w.agg_dofs, n1) || ai(&w.seg_ptr, n_seg + 1) ||
      ai(&w.seg_key, n_seg) || ai(&w.seg_e, nnz1) || ai(&w.seg_row, nnz1) ||
      ad(&w.Ac, (long)nc * nc) || ad(&w.AinvT, (long)nc * nc) || ad(&w.yc, kCoarseMax) ||
      ad(&w.partc, 4L * kUpdMaxBlocks)) {
    c->err = "device allocation for the Krylov workspace failed";
    int32_t** ip[] = {&w.ell_col, &w.cmap0, &w.cmap, &w.agg_ptr, &w.agg_dofs, &w.seg_ptr, &w.seg_key, &w.seg_e,
                      &w.seg_row};
    double** dp[] = {&w.ell_val, &w.p2, &w.zd, &w.Ac, &w.AinvT, &w.yc, &w.partc};
    for (auto q : ip) { if (*q) (void)hipFree(*q); *q = nullptr; }
    for (auto q : dp) { if (*q) (void)hipFree(*q); *q = nullptr; }
    return GEDMG_E_NOMEM;
  }
  GH(hipMemcpy(w.cmap0, cmap0.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  GH(hipMemcpy(w.agg_ptr, agg_ptr.data(), sizeof(int32_t) * (n_agg + 1), hipMemcpyHostToDevice));
  GH(hipMemcpy(w.agg_dofs, agg_dofs.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice));
  GH(hipMemcpy(w.seg_ptr, seg_ptr.data(), sizeof(int32_t) * (n_seg + 1), hipMemcpyHostToDevice));
  GH(hipMemcpy(w.seg_key, seg_key.data(), sizeof(int32_t) * n_seg, hipMemcpyHostToDevice));
  GH(hipMemcpy(w.seg_e, seg_e.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
  GH(hipMemcpy(w.seg_row, seg_row.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
  w.n_agg = n_agg;
  w.n_coarse = nc;
  w.n_seg = n_seg;
  w.upd_sub = sub;
  w.ell_lanes = L;
  if (nn > 0)
    hipLaunchKernelGGL(ell_ncols_kernel, dim3((nn + 255) / 256), dim3(256), 0, c->stream, c->drowptr, c->dcol, nn,
                       nd, (int)nbmax, w.ell_col);
  GH(hipGetLastError());
  w.krylov_ready = true;
  return GEDMG_OK;
}

// grid of the ELL kernels: one row group per row, at most kEllMaxBlocks blocks
// (beyond that the row groups loop over rows)
int ell_grid(const Work& w) {
  const long groups_per_block = kThreads / w.ell_lanes;
  return (int)std::max(1L, std::min<long>(kEllMaxBlocks, (w.ndof + groups_per_block - 1) / groups_per_block));
}

// launch KERNEL<L, ND(, T)> for the row lanes L of the ELL copy and the dofs per
// node of the mesh (3 for Q4, 4 for Hex8)
#define ELL_CASES(KERNEL, ND, T, GRID, ...)                                                                \
  switch (L_) {                                                                                            \
    case 1: hipLaunchKernelGGL((KERNEL<1, ND T>), dim3(GRID), dim3(kThreads), 0, c->stream, __VA_ARGS__); break;   \
    case 2: hipLaunchKernelGGL((KERNEL<2, ND T>), dim3(GRID), dim3(kThreads), 0, c->stream, __VA_ARGS__); break;   \
    case 4: hipLaunchKernelGGL((KERNEL<4, ND T>), dim3(GRID), dim3(kThreads), 0, c->stream, __VA_ARGS__); break;   \
    case 8: hipLaunchKernelGGL((KERNEL<8, ND T>), dim3(GRID), dim3(kThreads), 0, c->stream, __VA_ARGS__); break;   \
    case 16: hipLaunchKernelGGL((KERNEL<16, ND T>), dim3(GRID), dim3(kThreads), 0, c->stream, __VA_ARGS__); break; \
    case 32: hipLaunchKernelGGL((KERNEL<32, ND T>), dim3(GRID), dim3(kThreads), 0, c->stream, __VA_ARGS__); break; \
    default: hipLaunchKernelGGL((KERNEL<64, ND T>), dim3(GRID), dim3(kThreads), 0, c->stream, __VA_ARGS__); break; \
  }
#define ELL_LAUNCH(KERNEL, L, GRID, ...)                 \
  do {                                                   \
    const int L_ = (L);                                  \
    if (c->dim == 2) {                                   \
      ELL_CASES(KERNEL, 3, , GRID, __VA_ARGS__)          \
    } else {                                             \
      ELL_CASES(KERNEL, 4, , GRID, __VA_ARGS__)          \
    }                                                    \
  } while (0)
#define ELL_LAUNCH_T(KERNEL, L, T, GRID, ...)            \
  do {                                                   \
    const int L_ = (L);                                  \
    if (c->dim == 2) {                                   \
      ELL_CASES(KERNEL, 3, ELL_COMMA T, GRID, __VA_ARGS__) \
    } else {                                             \
      ELL_CASES(KERNEL, 4, ELL_COMMA T, GRID, __VA_ARGS__) \
    }                                                    \
  } while (0)
#define ELL_COMMA ,

// The ELL values of the masked matrix K and the coarse map of w.mask (at the
// start of every Krylov solve).
int ell_pack(gedmg_ctx* c, Work& w, const double* K) {
  int rc = ensure_ell(c, w);
  if (rc) return rc;
  if (w.ndof > 0)
    hipLaunchKernelGGL(ell_pack_kernel, dim3((w.ndof + 255) / 256), dim3(256), 0, c->stream, K, c->drowptr, w.mask,
                       w.cmap0, w.ndof, w.ell_lanes, w.ell_val, w.cmap);
  GH(hipGetLastError());
  return GEDMG_OK;
}

// y = K x with the ELL copy of the last ell_pack, scal[slot] = w . y
int ell_spmv(gedmg_ctx* c, Work& w, const double* x, double* y, const double* wv, int slot) {
  const int gs = ell_grid(w);
  double* part = w.part + std::max(3 * kRedBlocks, 2 * kUpdMaxBlocks);
  ELL_LAUNCH(ell_spmv_kernel, w.ell_lanes, gs, w.ell_val, w.ell_col, x, y, wv, w.ndof, part);
  GH(hipGetLastError());
  if (slot >= 0) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, c->stream, part, w.scal, slot, -1, gs);
    GH(hipGetLastError());
  }
  return GEDMG_OK;
}

// y = K x, scal[slot] = w . y
int spmv(gedmg_ctx* c, Work& w, const double* K, const double* x, double* y, const double* wv, int slot) {
  const int G = c->dim == 3 ? 32 : 16;
  if (G == 32)
    hipLaunchKernelGGL((spmv_dot_kernel<32>), dim3(kRedBlocks), dim3(kThreads), 0, c->stream, K, c->drowptr,
                       c->dcol, x, y, wv, w.ndof, w.part);
  else
    hipLaunchKernelGGL((spmv_dot_kernel<16>), dim3(kRedBlocks), dim3(kThreads), 0, c->stream, K, c->drowptr,
                       c->dcol, x, y, wv, w.ndof, w.part);
  GH(hipGetLastError());
  if (slot >= 0) {
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, c->stream, w.part, w.scal, slot, -1, kRedBlocks);
    GH(hipGetLastError());
  }
  return GEDMG_OK;
}

int dot2(gedmg_ctx* c, Work& w, const double* a, const double* b, const double* cc, const double* d,
         int s1, int s2) {
  hipLaunchKernelGGL(dot2_kernel, dim3(kRedBlocks), dim3(kThreads), 0, c->stream, a, b, cc, d, w.ndof, w.part);
  GH(hipGetLastError());
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, c->stream, w.part, w.scal, s1, s2, kRedBlocks);
  GH(hipGetLastError());
  return GEDMG_OK;
}

int read_scalars(gedmg_ctx* c, Work& w);

// a .W b for the arc-length norm, read back to the host.
int wdot(gedmg_ctx* c, Work& w, const double* a, const double* b, double w2, double* out) {
  hipLaunchKernelGGL(wdot_kernel, dim3(kRedBlocks), dim3(kThreads), 0, c->stream, a, b, w.ndof, c->dim + 1, w2,
                     w.part);
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, c->stream, w.part, w.scal, S_TT, -1, kRedBlocks);
  GH(hipGetLastError());
  const int rc = read_scalars(c, w);
  if (rc) return rc;
  *out = w.hscal[S_TT];
  return GEDMG_OK;
}

int read_scalars(gedmg_ctx* c, Work& w) {
  GH(hipMemcpyAsync(w.hscal, w.scal, sizeof(double) * S_NSLOTS, hipMemcpyDeviceToHost, c->stream));
  GH(hipStreamSynchronize(c->stream));
  return GEDMG_OK;
}

// Solve K x = b (CG with the Jacobi + coarse preconditioner; BiCGStab with
// Jacobi on non-positive curvature).  K is the masked matrix and w.mask the
// Dirichlet mask of this solve.  Returns iterations in *its.
// A_c = P^T K P from the masked matrix and its dense inverse (once per Krylov
// solve, after the ELL copy and the coarse map of the solve's mask).
int coarse_setup(gedmg_ctx* c, Work& w, const double* K) {
  const int nc = w.n_coarse;
  GH(hipMemsetAsync(w.Ac, 0, sizeof(double) * nc * nc, c->stream));
  if (w.n_seg > 0)
    hipLaunchKernelGGL(coarse_matrix_kernel, dim3(w.n_seg), dim3(256), 0, c->stream, K, c->dcol, w.seg_ptr,
                       w.seg_key, w.seg_e, w.seg_row, w.mask, w.Ac);
  hipLaunchKernelGGL(coarse_invert_kernel, dim3(1), dim3(1024), 0, c->stream, w.Ac, nc, w.AinvT);
  GH(hipGetLastError());
  return GEDMG_OK;
}

// z = M^-1 x with the two-level preconditioner: D^-1 x and the restriction
// P^T x over the aggregates (the update kernel in its first-residual mode, x
// in the place of r), y_c = A_c^-1 P^T x, then z += P y_c.  Overwrites the
// update kernel's partials and the scalars S_RDR, S_RR and S_RZC.
int apply_two_level(gedmg_ctx* c, Work& w, const double* x, double* z) {
  const long n = w.ndof;
  const int nd = c->dim + 1, nc = w.n_coarse, gu = w.n_agg * w.upd_sub;
  hipLaunchKernelGGL(cg_update_kernel, dim3(gu), dim3(kThreads), 0, c->stream, nullptr, const_cast<double*>(x),
                     nullptr, nullptr, w.dinv, z, w.agg_ptr, w.agg_dofs, w.upd_sub, nd, nullptr, 0, w.scal, S_RZ, 1,
                     w.part, w.partc);
  hipLaunchKernelGGL(coarse_tail_kernel, dim3(1), dim3(1024), 0, c->stream, w.part, w.partc, gu, w.upd_sub, nd, nc,
                     w.AinvT, w.scal, w.yc);
  hipLaunchKernelGGL(coarse_prolong_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, z, w.cmap, w.yc, n);
  GH(hipGetLastError());
  return GEDMG_OK;
}

// CG with the two-level preconditioner (A_c^-1 formed by the caller).  Per
// iteration three launches: the new search
// direction with its product from the ELL copy (and partials of p.q), the
// update over the aggregates, and the one-block sums that form the scalars
// and the coarse correction for the next direction.  The host polls the residual adaptively
// (each poll stalls the stream, so the next one is placed at 70 % of the
// iterations that the observed decay rate still needs, 8 to 128 ahead).  The
// ELL copy of K and the coarse map are packed by the caller.
// Sets *curvature on non-positive curvature; *bb_out receives b.b.
int cg_multi(gedmg_ctx* c, Work& w, const double* K, int max_it, double rtol, int* its, bool* curvature,
             double* bb_out) {
  const long n = w.ndof;
  const int gs = ell_grid(w);
  const bool loop = (long)gs * (kThreads / w.ell_lanes) < n;
  const int nd = c->dim + 1, nc = w.n_coarse;
  const int gu = w.n_agg * w.upd_sub;
  double* part_pap = w.part + std::max(3 * kRedBlocks, 2 * kUpdMaxBlocks);
  double* pbuf[2] = {w.p, w.p2};
  int rc;
  *its = 0;
  *curvature = false;
  GH(hipMemsetAsync(w.x, 0, sizeof(double) * n, c->stream));
  GH(hipMemsetAsync(w.p, 0, sizeof(double) * n, c->stream));  // p_old of the first iteration
  GH(hipMemsetAsync(w.scal, 0, sizeof(double) * S_NSLOTS, c->stream));
  GH(hipMemcpyAsync(w.r, w.b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  // the first residual's scalars and coarse correction (x and r unchanged)
  hipLaunchKernelGGL(cg_update_kernel, dim3(gu), dim3(kThreads), 0, c->stream, w.x, w.r, w.p, w.q, w.dinv, w.zd,
                     w.agg_ptr, w.agg_dofs, w.upd_sub, nd, part_pap, 0, w.scal, S_RZ, 1, w.part, w.partc);
  hipLaunchKernelGGL(coarse_tail_kernel, dim3(1), dim3(1024), 0, c->stream, w.part, w.partc, gu, w.upd_sub, nd,
                     nc, w.AinvT, w.scal, w.yc);
  GH(hipGetLastError());
  if ((rc = read_scalars(c, w))) return rc;
  const double bb = w.hscal[S_RR];
  *bb_out = bb;
  if (bb == 0.0) return GEDMG_OK;
  if (!std::isfinite(bb)) { c->err = "non-finite right-hand side"; return GEDMG_E_NONFINITE; }
  const double tol2 = rtol * rtol * bb;
  const int check = 8;
  int next_poll = check, prev_it = 0;
  double prev_rr = bb;
  for (int it = 1; it <= max_it; ++it) {
    // (r.z) of this iteration's direction goes to slot cur; the previous one is in prv
    const int cur = (it & 1) ? S_RZ : S_RZNEW, prv = (it & 1) ? S_RZNEW : S_RZ;
    double* p_old = pbuf[(it - 1) & 1];
    double* p_new = pbuf[it & 1];
    if (loop) {
      ELL_LAUNCH_T(cg_dir_spmv_kernel, w.ell_lanes, true, gs, w.ell_val, w.ell_col, w.zd, w.cmap, w.yc, nc, p_old,
                   p_new, w.q, w.scal, cur, prv, (int)(it == 1), n, part_pap);
    } else {
      ELL_LAUNCH_T(cg_dir_spmv_kernel, w.ell_lanes, false, gs, w.ell_val, w.ell_col, w.zd, w.cmap, w.yc, nc, p_old,
                   p_new, w.q, w.scal, cur, prv, (int)(it == 1), n, part_pap);
    }
    hipLaunchKernelGGL(cg_update_kernel, dim3(gu), dim3(kThreads), 0, c->stream, w.x, w.r, p_new, w.q, w.dinv,
                       w.zd, w.agg_ptr, w.agg_dofs, w.upd_sub, nd, part_pap, gs, w.scal, cur, 0, w.part, w.partc);
    hipLaunchKernelGGL(coarse_tail_kernel, dim3(1), dim3(1024), 0, c->stream, w.part, w.partc, gu, w.upd_sub,
                       nd, nc, w.AinvT, w.scal, w.yc);
    GH(hipGetLastError());
    *its = it;
    if (it == next_poll || it == max_it) {
      if ((rc = read_scalars(c, w))) return rc;
      if (w.hscal[S_FLAG] != 0.0) { *curvature = true; return GEDMG_OK; }
      const double rr = w.hscal[S_RR];
      if (!std::isfinite(rr)) { c->err = "non-finite Krylov residual"; return GEDMG_E_NONFINITE; }
      if (rr <= tol2) return GEDMG_OK;
      int ahead = check;
      if (rr > 0.0 && rr < prev_rr) {
        const double rate = std::log(rr / prev_rr) / (it - prev_it);  // per iteration, < 0
        const double need = std::log(tol2 / rr) / rate;
        ahead = (int)std::min(128.0, std::max((double)check, 0.7 * need));
      }
      prev_rr = rr;
      prev_it = it;
      next_poll = it + ahead;
    }
  }
  c->err = "CG reached the iteration limit";
  return GEDMG_E_LINSOLVE;
}

// reuse = true: K, the mask and D^-1 are those of the previous call, whose
// ELL copy and coarse inverse are kept.
int krylov(gedmg_ctx* c, Work& w, const double* K, int max_it, double rtol, int* its, int method = 0,
           int* fallbacks = nullptr, bool reuse = false) {
  const long n = w.ndof;
  const int gr = kRedBlocks;
  *its = 0;
  double bb = 0.0;
  if (!reuse) {
    int rcp = ell_pack(c, w, K);
    if (!rcp) rcp = coarse_setup(c, w, K);
    if (rcp) return rcp;
  }
  if (method == 1) {  // BiCGStab requested (non-symmetric tangents)
    hipLaunchKernelGGL(dot2_kernel, dim3(kRedBlocks), dim3(kThreads), 0, c->stream, w.b, w.b, nullptr, nullptr,
                       n, w.part);
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, c->stream, w.part, w.scal, S_BB, -1, kRedBlocks);
    GH(hipGetLastError());
    int rc0 = read_scalars(c, w);
    if (rc0) return rc0;
    bb = w.hscal[S_BB];
    if (bb == 0.0) {
      GH(hipMemsetAsync(w.x, 0, sizeof(double) * n, c->stream));
      return GEDMG_OK;
    }
    if (!std::isfinite(bb)) { c->err = "non-finite right-hand side"; return GEDMG_E_NONFINITE; }
  } else {
    bool curvature = false;
    const int rc1 = cg_multi(c, w, K, max_it, rtol, its, &curvature, &bb);
    // CG is left for BiCGStab on non-positive curvature (the tangent is not
    // positive definite here) and when it does not converge: while points
    // yield with kappa below kappa_d the history enters the damage rows but,
    // with f_d' = 0, not the displacement rows, so the tangent is not
    // symmetric there
    if (!(rc1 == GEDMG_E_LINSOLVE && *its >= max_it) && (rc1 || !curvature)) return rc1;
    if (fallbacks) ++*fallbacks;
  }
  // BiCGStab from x = 0, right-preconditioned with the two-level M.
  int rc;
  const int check = 8;
  const double tol2 = rtol * rtol * bb;
  const int cg_its = *its;
  GH(hipMemsetAsync(w.x, 0, sizeof(double) * n, c->stream));
  GH(hipMemsetAsync(w.scal, 0, sizeof(double) * S_NSLOTS, c->stream));
  GH(hipMemcpyAsync(w.r, w.b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  GH(hipMemcpyAsync(w.r0, w.b, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  GH(hipMemsetAsync(w.p, 0, sizeof(double) * n, c->stream));
  GH(hipMemsetAsync(w.v, 0, sizeof(double) * n, c->stream));
  {
    // rho = alpha = omega = 1
    std::vector<double> init(S_NSLOTS, 0.0);
    init[S_RHO] = init[S_ALPHA] = init[S_OMEGA] = 1.0;
    std::copy(init.begin(), init.end(), w.hscal);
    GH(hipMemcpyAsync(w.scal, w.hscal, sizeof(double) * S_NSLOTS, hipMemcpyHostToDevice, c->stream));
    GH(hipStreamSynchronize(c->stream));
  }
  for (int it = 1; it <= max_it; ++it) {
    if ((rc = dot2(c, w, w.r0, w.r, nullptr, nullptr, S_RZNEW, -1))) return rc;
    hipLaunchKernelGGL(bicg_scalars_kernel, dim3(1), dim3(1), 0, c->stream, w.scal, 0);
    hipLaunchKernelGGL(bicg_p_kernel, dim3(gr), dim3(kThreads), 0, c->stream, w.p, w.r, w.v, w.scal, n);
    if ((rc = apply_two_level(c, w, w.p, w.z))) return rc;  // phat
    if ((rc = ell_spmv(c, w, w.z, w.v, w.r0, S_VR))) return rc;                                            // v = K phat
    hipLaunchKernelGGL(bicg_scalars_kernel, dim3(1), dim3(1), 0, c->stream, w.scal, 1);
    hipLaunchKernelGGL(bicg_s_kernel, dim3(gr), dim3(kThreads), 0, c->stream, w.r, w.v, w.scal, n);     // s in r
    if ((rc = apply_two_level(c, w, w.r, w.q))) return rc;  // shat
    if ((rc = ell_spmv(c, w, w.q, w.t, nullptr, -1))) return rc;                                         // t = K shat
    if ((rc = dot2(c, w, w.t, w.t, w.t, w.r, S_TT, S_TS))) return rc;
    hipLaunchKernelGGL(bicg_scalars_kernel, dim3(1), dim3(1), 0, c->stream, w.scal, 2);
    hipLaunchKernelGGL(bicg_update_kernel, dim3(gr), dim3(kThreads), 0, c->stream, w.x, w.r, w.z, w.q, w.t,
                       w.scal, n, w.part);
    hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, c->stream, w.part, w.scal, S_RR, -1, kRedBlocks);
    GH(hipGetLastError());
    *its = cg_its + it;
    if (it % check == 0 || it == max_it) {
      if ((rc = read_scalars(c, w))) return rc;
      if (!std::isfinite(w.hscal[S_RR])) { c->err = "non-finite Krylov residual"; return GEDMG_E_NONFINITE; }
      if (w.hscal[S_RR] <= tol2) return GEDMG_OK;
      if (w.hscal[S_FLAG] == 2.0) { c->err = "BiCGStab breakdown"; return GEDMG_E_LINSOLVE; }
    }
  }
  c->err = "BiCGStab reached the iteration limit";
  return GEDMG_E_LINSOLVE;
}

double sum_partials_host(gedmg_ctx* c, Work& w, int* rc) {
  hipLaunchKernelGGL(reduce_kernel, dim3(1), dim3(kThreads), 0, c->stream, w.part, w.scal, S_FLAG + 1, -1, kRedBlocks);
  *rc = read_scalars(c, w);
  return w.hscal[S_FLAG + 1];
}

}  // namespace

namespace gedmg {

int solver_spmv(gedmg_ctx* c, const double* K, const double* x, double* y) {
  Work* wp = nullptr;
  int rc = ensure_work(c, &wp);
  if (rc) return rc;
  return spmv(c, *wp, K, x, y, nullptr, -1);
}

int solver_solve_free(gedmg_ctx* c, double* A, const gedmg_dirichlet* bc, const double* rhs, double* x,
                      int max_it, double rtol, int refine, int* its) {
  Work* wp = nullptr;
  int rc = ensure_work(c, &wp);
  if (rc) return rc;
  Work& w = *wp;
  const long n = w.ndof;
  *its = 0;
  GH(hipMemsetAsync(w.mask, 0, n, c->stream));
  GH(hipMemsetAsync(w.scal, 0, sizeof(double) * S_NSLOTS, c->stream));
  if (bc && bc->n > 0) {
    hipLaunchKernelGGL(set_mask_kernel, dim3((bc->n + 255) / 256), dim3(256), 0, c->stream, bc->dof, bc->n, n,
                       w.mask, w.scal);
    GH(hipGetLastError());
    if ((rc = read_scalars(c, w))) return rc;
    if (w.hscal[S_FLAG] != 0.0) {
      c->err = "Dirichlet dof index out of range";
      return GEDMG_E_ARG;
    }
  }
  hipLaunchKernelGGL(masked_copy_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, rhs, w.mask, w.b, n);
  hipLaunchKernelGGL(mask_matrix_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, A, c->drowptr, c->dcol,
                     w.mask, w.dinv, n);
  GH(hipGetLastError());
  if ((rc = krylov(c, w, A, max_it, rtol, its))) return rc;
  GH(hipMemcpyAsync(x, w.x, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
  // iterative refinement on the true FP64 residual: the Krylov recurrence
  // residual drifts from b - Ax, and without an outer Newton loop the
  // solution keeps the error cond(A) * rtol.  A correction only has to remove
  // that drift, so each pass solves to max(rtol, 1e-3) of its own residual
  // (three orders per pass).
  const double rtol_pass = std::max(rtol, 1e-3);
  for (int pass = 0; pass < refine; ++pass) {
    if ((rc = spmv(c, w, A, x, w.q, nullptr, -1))) return rc;
    hipLaunchKernelGGL(masked_residual_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, rhs, w.q, w.mask,
                       w.b, n);
    GH(hipGetLastError());
    int more = 0;  // same matrix and mask: the ELL copy and the coarse inverse are kept
    if ((rc = krylov(c, w, A, max_it, rtol_pass, &more, 0, nullptr, true))) return rc;
    *its += more;
    hipLaunchKernelGGL(add_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, x, w.x, n);
    GH(hipGetLastError());
  }
  return GEDMG_OK;
}

}  // namespace gedmg

extern "C" int gedmg_newton_step(gedmg_ctx* c, const gedmg_dirichlet* bc, const gedmg_solver_opts* opts_in,
                                 int precision, const double* predictor_du, double* u, double* phi,
                                 double* kappa, const int32_t* reaction_dofs, int32_t n_reaction,
                                 gedmg_newton_report* rep) {
  if (!c) return GEDMG_E_ARG;
  if (!bc || !u || !phi || !kappa || (bc->n > 0 && (!bc->dof || !bc->value)) || bc->n < 0 ||
      (n_reaction > 0 && !reaction_dofs)) {
    c->err = "null or inconsistent argument";
    return GEDMG_E_ARG;
  }
  if (precision != GEDMG_FP64 && precision != GEDMG_BF16 && precision != GEDMG_FP16) {
    c->err = "unknown precision";
    return GEDMG_E_ARG;
  }
  gedmg_solver_opts o = default_solver_opts();
  if (opts_in) o = *opts_in;
  if (o.max_local <= 0 || o.max_newton < 0 || o.max_krylov <= 0 || o.refine_max < 0) {
    c->err = "solver limits must be positive";
    return GEDMG_E_ARG;
  }
  if (o.krylov_method != 0 && o.krylov_method != 1) {
    c->err = "unknown Krylov method";
    return GEDMG_E_ARG;
  }
  if (!(o.newton_rscale >= 0.0)) {
    c->err = "newton_rscale must be non-negative";
    return GEDMG_E_ARG;
  }
  if (o.scheme != GEDMG_MONOLITHIC && o.scheme != GEDMG_STAGGERED) {
    c->err = "unknown solution scheme";
    return GEDMG_E_ARG;
  }
  if (n_reaction < 0) {
    c->err = "negative reaction dof count";
    return GEDMG_E_ARG;
  }
  // reaction dofs must be in range (checked on the host, before any work)
  if (n_reaction > 0) {
    std::vector<int32_t> rd(n_reaction);
    GH(hipMemcpyAsync(rd.data(), reaction_dofs, sizeof(int32_t) * n_reaction, hipMemcpyDeviceToHost, c->stream));
    GH(hipStreamSynchronize(c->stream));
    for (int32_t d : rd)
      if (d < 0 || d >= c->ndof) {
        c->err = "reaction dof index out of range";
        return GEDMG_E_ARG;
      }
  }
  c->max_local = o.max_local;
  gedmg_newton_report local{};
  gedmg_newton_report& r = rep ? *rep : local;
  r = gedmg_newton_report{};
  Work* wp = nullptr;
  int rc = ensure_work(c, &wp);
  if (rc) return rc;
  Work& w = *wp;
  const long n = w.ndof;
  const int gr = kRedBlocks;
  // backups for rollback
  GH(hipMemcpyAsync(w.ub, u, sizeof(double) * c->dim * c->n_nodes, hipMemcpyDeviceToDevice, c->stream));
  GH(hipMemcpyAsync(w.phib, phi, sizeof(double) * c->n_nodes, hipMemcpyDeviceToDevice, c->stream));
  if (predictor_du) {
    const long nu = (long)c->dim * c->n_nodes;
    hipLaunchKernelGGL(add_kernel, dim3((nu + 255) / 256), dim3(256), 0, c->stream, u, predictor_du, nu);
    GH(hipGetLastError());
  }
  GH(hipMemsetAsync(w.mask, 0, n, c->stream));
  GH(hipMemsetAsync(w.scal, 0, sizeof(double) * S_NSLOTS, c->stream));
  if (bc->n > 0) {
    hipLaunchKernelGGL(set_dirichlet_kernel, dim3((bc->n + 255) / 256), dim3(256), 0, c->stream, u, phi,
                       bc->dof, bc->value, bc->n, c->dim, c->n_nodes, w.mask, w.scal);
    GH(hipGetLastError());
    if ((rc = read_scalars(c, w))) return rc;
    if (w.hscal[S_FLAG] != 0.0) {
      c->err = "Dirichlet dof index out of range";
      (void)hipMemcpyAsync(u, w.ub, sizeof(double) * c->dim * c->n_nodes, hipMemcpyDeviceToDevice, c->stream);
      (void)hipMemcpyAsync(phi, w.phib, sizeof(double) * c->n_nodes, hipMemcpyDeviceToDevice, c->stream);
      (void)hipStreamSynchronize(c->stream);
      return GEDMG_E_ARG;
    }
  }
  auto rollback = [&](int code) {
    (void)hipMemcpyAsync(u, w.ub, sizeof(double) * c->dim * c->n_nodes, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(phi, w.phib, sizeof(double) * c->n_nodes, hipMemcpyDeviceToDevice, c->stream);
    (void)hipStreamSynchronize(c->stream);
    r.status = code;
    return code;
  };
  const bool mixed = precision != GEDMG_FP64;
  const int max_it = o.max_newton + (mixed ? o.refine_max : 0);
  // staggered scheme: every assembly of the global solve holds kappa_n
  struct FrozenGuard {
    gedmg_ctx* c;
    ~FrozenGuard() { c->frozen_history = 0; }
  } guard{c};
  c->frozen_history = o.scheme == GEDMG_STAGGERED ? 1 : 0;
  double res0 = -1.0;
  for (int it = 0; it <= max_it; ++it) {
    // residual (FP64) and tangent (FP64 or mixed)
    if (mixed) {
      // one pass: low-precision Hessian in the tangent, FP64 value and gradient
      // for the residual and the history
      const AssembleScratch sc{c->dx, c->djet, c->dphiq, c->dsens};
      if ((rc = assemble_impl(c, u, phi, kappa, precision, w.R, w.K, w.kt, sc, false, true))) return rollback(rc);
    } else {
      if ((rc = gedmg_assemble(c, u, phi, kappa, GEDMG_FP64, w.R, w.K, w.kt))) return rollback(rc);
    }
    hipLaunchKernelGGL(rhs_kernel, dim3(gr), dim3(kThreads), 0, c->stream, w.R, w.mask, w.b, n, w.part);
    GH(hipGetLastError());
    const double res2 = sum_partials_host(c, w, &rc);
    if (rc) return rollback(rc);
    const int st = gedmg_status(c);
    const double res = std::sqrt(res2);
    // A correction that inverts an element or makes the residual non-finite is
    // halved (up to kMaxBacktracks times) before the step gives up: far from the
    // solution the full Newton correction of a softening state can overshoot.
    if ((st == GEDMG_E_JNONPOS || (st == GEDMG_OK && !std::isfinite(res))) && it > 0 &&
        r.backtracks < kMaxBacktracks) {
      hipLaunchKernelGGL(backtrack_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, u, phi, w.x, c->dim,
                         c->n_nodes);
      GH(hipGetLastError());
      r.backtracks++;
      --it;
      continue;
    }
    if (st) return rollback(st);
    if (it < 32) r.res_norm[it] = res;
    r.newton_iters = it;
    if (!std::isfinite(res)) { c->err = "non-finite residual"; return rollback(GEDMG_E_NONFINITE); }
    if (res0 < 0.0) res0 = res;
    if (res <= std::max(o.newton_rtol * std::max(o.newton_rscale, res0), o.newton_atol)) {
      // converged: commit the history and report
      if (o.scheme == GEDMG_STAGGERED) {
        // the local update at the converged fields (residual of this pass unused)
        c->frozen_history = 0;
        if ((rc = gedmg_assemble(c, u, phi, kappa, GEDMG_FP64, w.Rmp, nullptr, w.kt))) return rollback(rc);
        if ((rc = gedmg_status(c))) return rollback(rc);
      }
      GH(hipMemcpyAsync(w.ktmp, kappa, sizeof(double) * w.nq, hipMemcpyDeviceToDevice, c->stream));
      GH(hipMemcpyAsync(kappa, w.kt, sizeof(double) * w.nq, hipMemcpyDeviceToDevice, c->stream));
      hipLaunchKernelGGL(count_growth_kernel, dim3(gr), dim3(kThreads), 0, c->stream, kappa, w.ktmp, w.nq,
                         w.part);
      GH(hipGetLastError());
      r.n_yielded_qp = (int)sum_partials_host(c, w, &rc);
      if (rc) return rc;
      if (n_reaction > 0) {
        hipLaunchKernelGGL(gather_sum_kernel, dim3(gr), dim3(kThreads), 0, c->stream, w.R, reaction_dofs,
                           n_reaction, n, w.part);
        GH(hipGetLastError());
        r.reaction = sum_partials_host(c, w, &rc);
        if (rc) return rc;
      }
      r.status = GEDMG_OK;
      return GEDMG_OK;
    }
    if (it == max_it) break;
    hipLaunchKernelGGL(mask_matrix_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, w.K, c->drowptr,
                       c->dcol, w.mask, w.dinv, n);
    GH(hipGetLastError());
    int its = 0;
    double eta =
        o.krylov_forcing ? std::max(o.krylov_rtol, std::min(1e-3, res / std::max(res0, 1e-300))) : o.krylov_rtol;
    if (mixed) eta = std::max(eta, o.refine_rtol);
    rc = krylov(c, w, w.K, o.max_krylov, eta, &its, o.krylov_method, &r.krylov_fallbacks);
    r.krylov_iters_total += its;
    if (rc) return rollback(rc);
    hipLaunchKernelGGL(update_fields_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, u, phi, w.x,
                       c->dim, c->n_nodes);
    GH(hipGetLastError());
  }
  c->err = "Newton did not converge";
  return rollback(GEDMG_E_NEWTON_NOCONV);
}

// Arc-length continuation of displacement-controlled loading (Riks; see the
// declaration in gedmg.h): the prescribed dofs carry lambda times their unit
// values, lambda is solved for with the fields under the constraint
// ||Delta d||^2 + psi^2 Delta lambda^2 = ds^2, the corrector iterating in the
// plane normal to the predictor.  Per corrector iteration: one FP64 assembly
// (monolithic history), y = K uhat with the unmasked tangent, the masked
// tangent, two Krylov solves a = -K_ff^-1 R_f, b = -K_ff^-1 y_f, and
// dlambda = -(Dd . a) / (Dd . b + psi^2 Dlambda), dd = a + dlambda b.
extern "C" int gedmg_arclength_step(gedmg_ctx* c, const gedmg_dirichlet* pattern, const gedmg_solver_opts* opts_in,
                                    double ds, double psi, double phi_weight, double* lambda, double* increment,
                                    double* u, double* phi, double* kappa, const int32_t* reaction_dofs,
                                    int32_t n_reaction, gedmg_newton_report* rep) {
  if (!c) return GEDMG_E_ARG;
  if (!pattern || pattern->n <= 0 || !pattern->dof || !pattern->value || !lambda || !increment || !u || !phi ||
      !kappa || (n_reaction > 0 && !reaction_dofs) || n_reaction < 0 || !(ds > 0.0) || !(psi >= 0.0) ||
      !(phi_weight >= 0.0) || !std::isfinite(phi_weight) || !std::isfinite(*lambda)) {
    c->err = "null or inconsistent arc-length argument";
    return GEDMG_E_ARG;
  }
  gedmg_solver_opts o = default_solver_opts();
  if (opts_in) o = *opts_in;
  if (o.max_local <= 0 || o.max_newton < 0 || o.max_krylov <= 0 || !(o.newton_rscale >= 0.0) ||
      (o.krylov_method != 0 && o.krylov_method != 1)) {
    c->err = "invalid solver options";
    return GEDMG_E_ARG;
  }
  c->max_local = o.max_local;
  gedmg_newton_report local{};
  gedmg_newton_report& r = rep ? *rep : local;
  r = gedmg_newton_report{};
  Work* wp = nullptr;
  int rc = ensure_work(c, &wp);
  if (rc) return rc;
  Work& w = *wp;
  const long n = w.ndof, nu = (long)c->dim * c->n_nodes;
  const int gr = kRedBlocks;
  if (!w.al_uh) {
    auto al = [&](double** p) { return hipMalloc((void**)p, sizeof(double) * std::max(n, 1L)); };
    if (al(&w.al_uh) || al(&w.al_dp) || al(&w.al_a) || al(&w.al_y)) {
      c->err = "device allocation for the arc-length workspace failed";
      return GEDMG_E_NOMEM;
    }
  }
  if (n_reaction > 0) {
    std::vector<int32_t> rd(n_reaction);
    GH(hipMemcpyAsync(rd.data(), reaction_dofs, sizeof(int32_t) * n_reaction, hipMemcpyDeviceToHost, c->stream));
    GH(hipStreamSynchronize(c->stream));
    for (int32_t d : rd)
      if (d < 0 || d >= n) {
        c->err = "reaction dof index out of range";
        return GEDMG_E_ARG;
      }
  }
  // Dirichlet mask (with the range check of the pattern) and the unit pattern
  GH(hipMemsetAsync(w.mask, 0, n, c->stream));
  GH(hipMemsetAsync(w.scal, 0, sizeof(double) * S_NSLOTS, c->stream));
  hipLaunchKernelGGL(set_mask_kernel, dim3((pattern->n + 255) / 256), dim3(256), 0, c->stream, pattern->dof,
                     pattern->n, n, w.mask, w.scal);
  GH(hipGetLastError());
  if ((rc = read_scalars(c, w))) return rc;
  if (w.hscal[S_FLAG] != 0.0) {
    c->err = "Dirichlet dof index out of range";
    return GEDMG_E_ARG;
  }
  GH(hipMemsetAsync(w.al_uh, 0, sizeof(double) * n, c->stream));
  hipLaunchKernelGGL(scatter_kernel, dim3((pattern->n + 255) / 256), dim3(256), 0, c->stream, w.al_uh, pattern->dof,
                     pattern->value, pattern->n);
  // previous increment's load-factor part (host) for the orientation of the predictor
  double prev_dlam = 0.0;
  GH(hipMemcpyAsync(&prev_dlam, increment + n, sizeof(double), hipMemcpyDeviceToHost, c->stream));
  GH(hipMemcpyAsync(w.ub, u, sizeof(double) * nu, hipMemcpyDeviceToDevice, c->stream));
  GH(hipMemcpyAsync(w.phib, phi, sizeof(double) * c->n_nodes, hipMemcpyDeviceToDevice, c->stream));
  GH(hipStreamSynchronize(c->stream));
  const double lam0 = *lambda;
  auto rollback = [&](int code) {
    (void)hipMemcpyAsync(u, w.ub, sizeof(double) * nu, hipMemcpyDeviceToDevice, c->stream);
    (void)hipMemcpyAsync(phi, w.phib, sizeof(double) * c->n_nodes, hipMemcpyDeviceToDevice, c->stream);
    (void)hipStreamSynchronize(c->stream);
    *lambda = lam0;
    r.status = code;
    return code;
  };
  auto set_prescribed = [&](double lam) -> int {
    hipLaunchKernelGGL(set_dirichlet_scaled_kernel, dim3((pattern->n + 255) / 256), dim3(256), 0, c->stream, u, phi,
                       pattern->dof, pattern->value, lam, pattern->n, c->dim, c->n_nodes);
    GH(hipGetLastError());
    return GEDMG_OK;
  };
  // assembly with the masked tangent, b = -R_f (res^2 returned) and y = K uhat
  auto assemble_step = [&](double* res2) -> int {
    int e;
    if ((e = gedmg_assemble(c, u, phi, kappa, GEDMG_FP64, w.R, w.K, w.kt))) return e;
    if ((e = spmv(c, w, w.K, w.al_uh, w.al_y, nullptr, -1))) return e;
    hipLaunchKernelGGL(rhs_kernel, dim3(gr), dim3(kThreads), 0, c->stream, w.R, w.mask, w.b, n, w.part);
    GH(hipGetLastError());
    *res2 = sum_partials_host(c, w, &e);
    if (e) return e;
    if ((e = gedmg_status(c))) return e;
    hipLaunchKernelGGL(mask_matrix_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, w.K, c->drowptr, c->dcol,
                       w.mask, w.dinv, n);
    GH(hipGetLastError());
    return GEDMG_OK;
  };
  auto solve_into = [&](double* dst, double eta) -> int {
    int its = 0;
    const int e = krylov(c, w, w.K, o.max_krylov, eta, &its, o.krylov_method, &r.krylov_fallbacks);
    r.krylov_iters_total += its;
    if (e) return e;
    GH(hipMemcpyAsync(dst, w.x, sizeof(double) * n, hipMemcpyDeviceToDevice, c->stream));
    return GEDMG_OK;
  };

  // ---- predictor.  After a first increment: the previous increment scaled to
  // ds (secant).  First increment (zero previous increment): the path tangent
  // t = -K_ff^-1 K_fp uhat with the history held at kappa_n, scaled to ds,
  // forward.  At a converged state the yielded points lie on the yield surface
  // to rounding, so a loading / elastic tangent there would be chosen by
  // rounding; neither predictor depends on that choice.
  if ((rc = set_prescribed(lam0))) return rollback(rc);
  double res2 = 0.0;
  const double w2 = phi_weight * phi_weight;
  double pp = 0.0;
  if ((rc = wdot(c, w, increment, increment, w2, &pp))) return rollback(rc);
  const double prev_len2 = pp + psi * psi * prev_dlam * prev_dlam;
  double dlam_p = 0.0;
  if (prev_len2 > 0.0 && std::isfinite(prev_len2)) {
    const double scale = ds / std::sqrt(prev_len2);
    // al_dp = scale * previous increment (zero on the Dirichlet rows it was taken on)
    hipLaunchKernelGGL(scale_copy_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, w.al_dp, scale, increment,
                       n);
    GH(hipGetLastError());
    dlam_p = scale * prev_dlam;
  } else {
    {
      struct Hold {
        gedmg_ctx* c;
        ~Hold() { c->frozen_history = 0; }
      } hold{c};
      c->frozen_history = 1;
      if ((rc = assemble_step(&res2))) return rollback(rc);
    }
    hipLaunchKernelGGL(masked_neg_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, w.al_y, w.mask, w.b, n);
    GH(hipGetLastError());
    if ((rc = solve_into(w.al_dp, o.krylov_rtol))) return rollback(rc);
    double tt = 0.0;
    if ((rc = wdot(c, w, w.al_dp, w.al_dp, w2, &tt))) return rollback(rc);
    dlam_p = ds / std::sqrt(tt + psi * psi);
    hipLaunchKernelGGL(axpy_scalar_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, w.al_dp, dlam_p - 1.0,
                       w.al_dp, n);  // al_dp = dlam_p * t
    GH(hipGetLastError());
  }
  hipLaunchKernelGGL(update_fields_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, u, phi, w.al_dp, c->dim,
                     c->n_nodes);
  GH(hipGetLastError());
  double lam = lam0 + dlam_p;
  if ((rc = set_prescribed(lam))) return rollback(rc);

  // ---- corrector in the normal plane
  double res0 = -1.0;
  for (int it = 0; it <= o.max_newton; ++it) {
    if ((rc = assemble_step(&res2))) return rollback(rc);
    const double res = std::sqrt(res2);
    if (it < 32) r.res_norm[it] = res;
    r.newton_iters = it;
    if (!std::isfinite(res)) { c->err = "non-finite residual"; return rollback(GEDMG_E_NONFINITE); }
    if (res0 < 0.0) res0 = res;
    if (res <= std::max(o.newton_rtol * std::max(o.newton_rscale, res0), o.newton_atol)) {
      GH(hipMemcpyAsync(w.ktmp, kappa, sizeof(double) * w.nq, hipMemcpyDeviceToDevice, c->stream));
      GH(hipMemcpyAsync(kappa, w.kt, sizeof(double) * w.nq, hipMemcpyDeviceToDevice, c->stream));
      hipLaunchKernelGGL(count_growth_kernel, dim3(gr), dim3(kThreads), 0, c->stream, kappa, w.ktmp, w.nq, w.part);
      GH(hipGetLastError());
      r.n_yielded_qp = (int)sum_partials_host(c, w, &rc);
      if (rc) return rc;
      if (n_reaction > 0) {
        hipLaunchKernelGGL(gather_sum_kernel, dim3(gr), dim3(kThreads), 0, c->stream, w.R, reaction_dofs, n_reaction,
                           n, w.part);
        GH(hipGetLastError());
        r.reaction = sum_partials_host(c, w, &rc);
        if (rc) return rc;
      }
      hipLaunchKernelGGL(field_increment_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, u, phi, w.ub,
                         w.phib, w.mask, increment, c->dim, c->n_nodes);
      const double dlam = lam - lam0;
      GH(hipMemcpyAsync(increment + n, &dlam, sizeof(double), hipMemcpyHostToDevice, c->stream));
      GH(hipStreamSynchronize(c->stream));
      *lambda = lam;
      r.status = GEDMG_OK;
      return GEDMG_OK;
    }
    if (it == o.max_newton) break;
    const double eta =
        o.krylov_forcing ? std::max(o.krylov_rtol, std::min(1e-3, res / std::max(res0, 1e-300))) : o.krylov_rtol;
    if ((rc = solve_into(w.al_a, eta))) return rollback(rc);  // a = -K_ff^-1 R_f (w.b holds -R_f)
    hipLaunchKernelGGL(masked_neg_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, w.al_y, w.mask, w.b, n);
    GH(hipGetLastError());
    int its = 0;
    // b in w.x; same matrix and mask as the solve for a: the ELL copy and the coarse inverse are kept
    rc = krylov(c, w, w.K, o.max_krylov, eta, &its, o.krylov_method, &r.krylov_fallbacks, true);
    r.krylov_iters_total += its;
    if (rc) return rollback(rc);
    double da = 0.0, db = 0.0;
    if ((rc = wdot(c, w, w.al_dp, w.al_a, w2, &da)) || (rc = wdot(c, w, w.al_dp, w.x, w2, &db)))
      return rollback(rc);
    const double den = db + psi * psi * dlam_p;
    if (!(std::fabs(den) > 0.0)) { c->err = "arc-length corrector breakdown"; return rollback(GEDMG_E_LINSOLVE); }
    const double dl = -da / den;
    hipLaunchKernelGGL(axpy_scalar_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, w.al_a, dl, w.x, n);
    hipLaunchKernelGGL(update_fields_kernel, dim3((n + 255) / 256), dim3(256), 0, c->stream, u, phi, w.al_a, c->dim,
                       c->n_nodes);
    GH(hipGetLastError());
    lam += dl;
    if ((rc = set_prescribed(lam))) return rollback(rc);
  }
  c->err = "arc-length corrector did not converge";
  return rollback(GEDMG_E_NEWTON_NOCONV);
}
