// Internal declarations shared by the gedmg runtime and its kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "gedmg.h"

namespace gedmg {

constexpr int kMaxHidden = 3;

// Offsets of one network's arrays inside a packed double buffer.  The packed
// buffer holds the *effective* weights (softplus applied where the ICNN
// constraints require it), followed by reference-state constants.
struct NetLayout {
  int n_in = 0, H = 0, L = 0, mask = 0;
  int W0 = 0, b0 = 0;                              // [H][n_in], [H]
  int Wz[kMaxHidden] = {0}, Wx[kMaxHidden] = {0}, b[kMaxHidden] = {0};  // hidden k=1..L-1 at [k]
  int wz = 0, wx = 0, bout = 0;
  int a0 = 0, s0 = 0, sb0 = 0;                     // [L][H]: pre-activation at x = 0 and its logistic pair
  int total = 0;
  int n_raw = 0;
};

// Packed order: W0[H][n_in], b0[H]; per hidden->hidden layer k = 1..L-1:
// Wz[H][H], Wx[H][n_in], b[H]; then wz[H], wx[n_in], b_out; then the
// reference-state constants a0, s0 = logistic(a0), sb0 = logistic(-a0), each
// [L][H] (pre-activations of every layer at x = 0).
__host__ __device__ inline NetLayout make_layout_hd(int n_in, int H, int L, int mask) {
  NetLayout l;
  l.n_in = n_in; l.H = H; l.L = L; l.mask = mask;
  int o = 0;
  l.W0 = o; o += H * n_in;
  l.b0 = o; o += H;
  for (int k = 1; k < L; ++k) {
    l.Wz[k] = o; o += H * H;
    l.Wx[k] = o; o += H * n_in;
    l.b[k] = o; o += H;
  }
  l.wz = o; o += H;
  l.wx = o; o += n_in;
  l.bout = o; o += 1;
  l.n_raw = o;
  l.a0 = o; o += L * H;
  l.s0 = o; o += L * H;
  l.sb0 = o; o += L * H;
  l.total = o;
  return l;
}

// Host-side reference-state quantities of a network.
struct NetRef {
  double N0 = 0.0;   // N(0)
  double n0 = 0.0;   // dN/dx_{n_in-1} at 0 (energy: derivative w.r.t. J - 1)
};

// Fill `packed` (size layout.total) from raw parameters; returns N(0), n0.
NetRef pack_network(const NetLayout& lay, const double* raw, std::vector<double>& packed);

struct Material {
  double mu, lam, eta, kd, c, beta, gamma;
};

// Arguments of the quadrature-input kernel and the energy-network jet kernel.
struct JetArgs {
  const double* x;       // [nq][3] network inputs (I1G-3, I2G-3, J-1)
  double* jet;           // [nq][10]: N(x)-N(0), dN/dx (3), d2N/dx2 (xx,yy,zz,xy,xz,yz)
  const double* net;     // packed effective network (double)
  const uint16_t* w16;   // [L-1][H][H+8] low-precision copies of Wz (bf16 or fp16 bits)
  const double* wop;     // [L-1][2][H/16][H/4][64] FP64 hidden weights in matrix-core operand
                         // order: [..][0] forward W[16t + l%16][4s + l/16], [..][1] backward
                         // W[4s + l/16][16t + l%16] (lane l of output tile t, step s)
  int nq;
  int L;
  int with_hessian;
  const double* mtab;    // [kMathTabDoubles] exp / log tables (FP64 kernel)
  double cf_mu, cf_lam;  // closed-form model (L == 0): Neo-Hooke moduli
};

struct KinArgs {
  const double* X;       // [dim][n_nodes]
  const int32_t* conn;   // [n_elems][nen]
  const double* u;       // [dim][n_nodes]
  const double* phi;     // [n_nodes]
  int n_nodes, n_elems;
  double* x;             // [n_elems*nqp][3]
  double* phiq;          // [n_elems*nqp] phi interpolated at the point
  int* status;
};

// Arguments of the local damage update (one lane per quadrature point).
struct HistArgs {
  const double* x;       // [nq][3] network inputs; x[2] = J - 1
  const double* jet;     // [nq][10]; jet[0] = N(x) - N(0)
  const double* phiq;    // [nq]
  const double* kappa_n; // [nq]
  const double* ynet;    // packed yield network
  double* kappa_out;     // [nq]
  double* sens;          // [nq][2]: d kappa / d psi_e, d kappa / d phi
  int* status;
  long nq;
  Material m;
  double n0;             // energy network dN/dx3 at 0
  double yN0;            // yield network N(0)
  int yL;                // hidden layers of the yield network; 0: G = identity (closed-form model)
  int max_local;
  int frozen;            // 1: keep kappa_n and report zero sensitivities (staggered scheme)
  const double* mtab;    // exp / log tables of the table-driven FP64 functions (kMathTabDoubles)
};

// Mesh data of the element kernel are stored by colour slot (the position of
// the element in perm), so a wavefront reaches its element's nodes and CSR
// segments without first loading the element number.
struct ElemArgs {
  const double* Xs;          // [n_elems][dim][nen] node coordinates, by slot
  const int32_t* conn_s;     // [n_elems][nen] connectivity, by slot
  const int32_t* perm;       // slot -> element (elements sorted by colour)
  const int32_t* seg;        // [n_elems][nen * nd][nen], by slot: CSR offset of the nd values of element row
                             // (a, c) in node block (a, b); bit 31 set: this element is the first (lowest
                             // colour) to write block (a, b)
  const double* u;
  const double* phi;
  const double* jet;         // [n_elems*nqp][10]
  const double* kappa;       // [n_elems*nqp] updated history (local update output)
  const double* sens;        // [n_elems*nqp][2] its sensitivities to psi_e and phi
  double* R;
  double* K;                 // may be null (residual only)
  int* status;
  int n_nodes, n_elems;
  int e_begin, e_end;        // range in perm of the colour being assembled
  Material m;
  double n0;                 // energy network dN/dx3 at 0
};

// Host: the exp / log tables of the table-driven FP64 functions.
constexpr int kMathTabDoubles = 64 * 2 + 64 * 4;
void build_math_tables(std::vector<double>& t);

// Kernel launchers (defined in the .hip translation units).
hipError_t launch_qp_inputs(int dim, const KinArgs& a, hipStream_t s);
hipError_t launch_energy_jet(int precision, int H, const JetArgs& a, hipStream_t s, int num_cu);
hipError_t launch_closed_form_jet(const JetArgs& a, hipStream_t s);
hipError_t launch_history(const HistArgs& a, int yH, hipStream_t s);
hipError_t launch_element(int dim, bool tangent, const ElemArgs& a, hipStream_t s);
void release_newton_work(gedmg_ctx* c);

// Per-point scratch of one assembly: network inputs x [nq][3], jets [nq][10],
// phi at the points [nq] and the history sensitivities [nq][2].
struct AssembleScratch {
  double* x;
  double* jet;
  double* phiq;
  double* sens;
};

// Material seen by the history and element kernels (unit energy scale and no
// volumetric term for the closed-form energy, whose jet is the whole psi_e).
Material element_material(const gedmg_ctx* c);

// One assembly (gedmg_assemble) with the given scratch.  fill_kernel: clear R
// with a kernel instead of hipMemsetAsync and record no profiling events (the
// form that a caller may capture in a graph).  refine64 (low precision only):
// the network value and gradient are recomputed in FP64, so R and the history
// are those of the FP64 path and only the tangent carries the low-precision
// Hessian (one pass per iteration of the mixed-precision Newton step).
int assemble_impl(gedmg_ctx* c, const double* u, const double* phi, const double* kappa_n, int precision,
                  double* R, double* K_vals, double* kappa_trial, const AssembleScratch& sc, bool fill_kernel,
                  bool refine64);

// Device address of the static scratch array on `device` (set up by gedmg_create).
int static_scratch_init(int device, std::string& err);
double* static_scratch_ptr(int device);

// Defaults of gedmg_solver_opts (used when a caller passes NULL).
gedmg_solver_opts default_solver_opts();

// Sparse helpers of the Newton driver, reused by the adjoint.
// y = K x over the context's CSR pattern.
int solver_spmv(gedmg_ctx* c, const double* K, const double* x, double* y);
// Solve A x = rhs on the free dofs: A (CSR values) is masked in place (rows and
// columns of bc->dof become identity rows / zero columns), prescribed entries of
// rhs are ignored and x is zero there.  `refine` passes of iterative refinement
// on the true residual follow the first Krylov solve.
int solver_solve_free(gedmg_ctx* c, double* A, const gedmg_dirichlet* bc, const double* rhs, double* x,
                      int max_it, double rtol, int refine, int* its);

}  // namespace gedmg

// The opaque context.
struct gedmg_ctx {
  std::string err;
  hipStream_t stream = nullptr;
  int device = 0, num_cu = 256;
  int dim = 0, nen = 0, nqp = 0, nd = 0, n_nodes = 0, n_elems = 0;
  int64_t ndof = 0, nnz = 0;
  gedmg::Material mat{};
  gedmg::NetLayout elay, ylay;
  gedmg::NetRef eref, yref;
  std::vector<double> eraw, yraw;      // host copies of the raw parameters
  std::vector<int> color_begin;        // n_colors + 1 offsets into perm
  // device buffers owned by the context
  double* dX = nullptr;
  int32_t* dconn = nullptr;
  int32_t* dperm = nullptr;
  double* dXs = nullptr;               // element-kernel mesh data by colour slot (see ElemArgs)
  int32_t* dconn_s = nullptr;
  int32_t* dseg = nullptr;
  int32_t* drowptr = nullptr;
  int32_t* dcol = nullptr;
  double* denet = nullptr;             // packed energy network
  double* dynet = nullptr;             // packed yield network
  uint16_t* dw_bf16 = nullptr;         // low-precision hidden weights
  uint16_t* dw_f16 = nullptr;
  double* dwop = nullptr;              // FP64 hidden weights in operand order (JetArgs::wop)
  double* dmtab = nullptr;             // exp / log tables of the FP64 jets (JetArgs::mtab)
  double* dx = nullptr;                // [nq][3]
  double* djet = nullptr;              // [nq][10]
  double* dphiq = nullptr;             // [nq]
  double* dsens = nullptr;             // [nq][2]
  int* dstatus = nullptr;
  int max_local = 100;                 // history-update iteration limit
  int frozen_history = 0;              // staggered scheme: assemblies keep kappa_n (set by newton_step)
  bool closed_energy = false;          // energy: compressible Neo-Hooke (Sec. 4.1) instead of a network
  bool closed_yield = false;           // yield: G = identity (Eq. ostwald_potential) instead of a network
  // per-phase event profiling of gedmg_assemble
  bool prof = false;
  std::vector<hipEvent_t> prof_ev;     // 5 events per timed assembly
  int prof_calls = 0;
};
