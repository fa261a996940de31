/*
 * gedmg -- gradient-enhanced damage with input-convex-network constitutive
 * laws: quadrature-point update, element residual/tangent and CSR assembly on
 * AMD Instinct MI355X (gfx950).
 *
 * The model (paper: "A Differentiable Framework for Gradient Enhanced Damage
 * with Physics-Augmented Neural Networks in JAX-FEM"):
 *   Psi(F, phi, grad phi, kappa) = f_d(kappa) psi_e(C) + c_d/2 grad phi.C^-1.grad phi
 *                                  + beta_d/2 (phi - kappa)^2            (Eq. dd_3)
 *   psi_e = mu_e [N(x) - N(0) - n0 (J-1)] + lambda_e (J + 1/J - 2)^2     (Eq. dd_0)
 *   x = (J^-2/3 I1 - 3, I2^3/(9 J^4) - 3, J - 1),  n0 = dN/dx_3 at x = 0
 *   f_d = exp(-eta_d <kappa - kappa_d>_+)                  (Eq. degradation_function)
 *   q = psi_e + gamma_d beta_d (phi - kappa)/(eta_d f_d)   (Eqs. q_q_loc_q_nloc, ostwald_potential)
 *   yield: N^_kappa(q) - kappa <= 0, N^_kappa(q) = N_kappa(q) - N_kappa(0)  (Eqs. Gq_NN, dd_7)
 * residual (Sec. 3.1): r_u,a = sum_q P grad N_a Jw, R_phi,a = sum_q (Y.grad N_a - Y N_a) Jw;
 * monolithic tangent (Sec. 3.2): history update inside every Newton iteration,
 * its sensitivities part of the consistent tangent.
 *
 * Conventions
 *   - 2-D: Q4 plane strain (unit thickness, F33 = 1); 3-D: Hex8.  Node order
 *     counter-clockwise (Q4) / standard (Hex8).  Quadrature: 2x2 / 2x2x2 Gauss,
 *     qp q at the natural coordinates of node q divided by sqrt(3), weight 1.
 *   - dofs interleaved node-major: dof(node, c) = node*(dim+1) + c, c < dim the
 *     displacement, c == dim the nonlocal damage phi.
 *   - nodal fields structure-of-arrays: u[dim][n_nodes], phi[n_nodes];
 *     history kappa[n_elems][nqp] (nqp = 4 or 8).
 *   - ICNN raw parameters (Sec. 4.2.1, Amos-type input-convex network):
 *       z1 = s(W0 x + b0); z_{k+1} = s(Wz_k z_k + Wx_k x + b_k); N = wz.z_L + wx.x + b
 *     with s = softplus; Wz_k, wz are softplus(raw); the weights multiplying
 *     input i (column i of W0 and Wx_k, wx[i]) are softplus(raw) when bit i of
 *     monotone_mask is set, raw otherwise.  Flat order: W0 (width x n_in,
 *     row-major), b0, then per hidden->hidden layer Wz (width x width), Wx
 *     (width x n_in), b, then wz (width), wx (n_in), b_out.
 *
 * Memory and streams
 *   - Setup data passed to gedmg_create / gedmg_set_params are HOST pointers;
 *     the library copies them.  Every per-call array of gedmg_assemble,
 *     gedmg_newton_step and gedmg_adjoint is a DEVICE pointer on the context's
 *     device, owned by the caller, FP64 unless stated, contiguous.
 *   - Work is ordered on the HIP stream given to gedmg_create.  A call returns
 *     after enqueueing, except when it must hand a host report back
 *     (newton_step, adjoint), which synchronise the stream.
 *
 * Errors: every call returns 0 on success or a negative GEDMG_E_* code;
 * gedmg_last_error() gives a message.  On error the outputs are unspecified,
 * except that gedmg_newton_step leaves u, phi and kappa at their input values.
 */
#ifndef GEDMG_H
#define GEDMG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct gedmg_ctx gedmg_ctx;

enum {
  GEDMG_OK = 0,
  GEDMG_E_ARG = -1,            /* invalid argument (null pointer, bad size, bad enum) */
  GEDMG_E_SHAPE = -2,          /* mesh / network shape not supported */
  GEDMG_E_NONFINITE = -3,      /* NaN or Inf in a residual or solution */
  GEDMG_E_LOCAL_NOCONV = -4,   /* history update did not converge in max_local iterations */
  GEDMG_E_NEWTON_NOCONV = -5,  /* global Newton did not converge in max_newton iterations */
  GEDMG_E_LINSOLVE = -6,       /* Krylov solver failed (breakdown or max iterations) */
  GEDMG_E_HIP = -7,            /* HIP runtime error */
  GEDMG_E_NOMEM = -8,          /* device allocation failed */
  GEDMG_E_JNONPOS = -9         /* det F <= 0 at a quadrature point */
};

enum { GEDMG_FP64 = 0, GEDMG_BF16 = 1, GEDMG_FP16 = 2 };

typedef struct {
  int32_t dim;          /* 2 (Q4 plane strain) or 3 (Hex8) */
  int32_t n_nodes, n_elems;
  const double* X;      /* host, [dim][n_nodes] reference coordinates */
  const int32_t* conn;  /* host, [n_elems][nen], nen = 4 or 8 */
} gedmg_mesh;

typedef struct {
  double mu_e, lambda_e;  /* energy scale and volumetric modulus (Eq. dd_0) */
  double eta_d, kappa_d;  /* degradation rate and threshold (Eq. degradation_function) */
  double c_d, beta_d;     /* gradient and penalty parameters (Sec. 4.1) */
  double gamma_d;         /* factor of q_nloc (Eq. ostwald_potential), 1 in the paper's chain rule */
} gedmg_material;

typedef struct {
  int32_t n_in;           /* 3 for the energy network, 1 for the yield network */
  int32_t width;          /* hidden width: energy 16, 32 or 64; yield 16 or 32 */
  int32_t n_hidden;       /* number of hidden layers (1..3), or 0 for the closed-form model of
                             Sec. 4.1: energy psi_e = compressible Neo-Hooke
                             mu_e/2 (I1 - 3) - mu_e ln J + lambda_e/2 (ln J)^2 (width, mask and
                             theta ignored); yield G(q) = q, which makes the yield condition the
                             loading function of Eq. ostwald_potential.  Either network may be
                             closed-form independently. */
  int32_t monotone_mask;  /* energy: 3 (I1G, I2G); yield: 1 */
  const double* theta;    /* host, raw parameters in the order described above (NULL allowed
                             when n_hidden == 0) */
} gedmg_icnn;

typedef struct {
  int32_t n;              /* number of prescribed dofs */
  const int32_t* dof;     /* device, [n] dof indices (no duplicates) */
  const double* value;    /* device, [n] prescribed values */
} gedmg_dirichlet;

typedef struct {
  int32_t max_newton;     /* global Newton iterations (default 25) */
  int32_t max_krylov;     /* Krylov iterations per linear solve (default 20000) */
  int32_t max_local;      /* history-update iterations (default 100, as in the paper's notched plate) */
  double newton_rtol;     /* ||R_f|| <= max(newton_rtol * max(newton_rscale, ||R_f^0||), newton_atol) */
  double newton_atol;
  double krylov_rtol;     /* relative residual of each linear solve (default 1e-12) */
  int32_t krylov_forcing; /* 1 (default): inexact Newton, iteration k solves to the relative residual
                             max(krylov_rtol, min(1e-3, ||R_f^k|| / ||R_f^0||)), so early iterations do
                             not pay for accuracy the Newton residual cannot use; 0: every solve to
                             krylov_rtol.  The Newton test on the FP64 residual decides convergence
                             either way. */
  /* Mixed precision (precision != GEDMG_FP64): each iteration solves with the
   * low-precision tangent against the FP64 residual, i.e. one pass of iterative
   * refinement.  refine_max extra iterations are allowed on top of max_newton
   * (default 10), and each solve stops at the relative residual
   * max(refine_rtol, the FP64 rule above): the tangent itself carries relative
   * errors of about 1e-5 (FP16) to 1e-4 (BF16), so accuracy below that is not
   * used by the refinement (default 1e-8; 0 keeps the FP64 rule). */
  int32_t refine_max;
  double refine_rtol;
  /* Solution scheme of the history variable (Sec. 3.2): GEDMG_MONOLITHIC (default)
   * updates kappa inside every global Newton iteration with its sensitivities in
   * the tangent; GEDMG_STAGGERED solves the global problem with kappa held at
   * kappa_n (no history sensitivities) and updates kappa once at the converged
   * fields, so the history lags the fields by one load step. */
  int32_t scheme;
  /* Residual scale of the relative Newton test (default 1, so residuals below 1
   * are tested absolutely); 0 makes the test purely relative to ||R_f^0||, for
   * states whose whole residual is scaled by a tiny degradation f_d. */
  double newton_rscale;
  /* Krylov method of the Newton solves: 0 (default) CG with the two-level
   * preconditioner (Jacobi plus a coarse correction on node aggregates of the
   * mesh's bounding box), switching to BiCGStab when it meets non-positive curvature
   * or reaches max_krylov without converging (each switch counts in
   * krylov_fallbacks); 1 BiCGStab (same preconditioner) from the start, for tangents that
   * are not symmetric (gamma_d != 1, or points yielding with kappa below
   * kappa_d, where the history enters the damage rows but not the displacement
   * rows). */
  int32_t krylov_method;
} gedmg_solver_opts;

enum { GEDMG_MONOLITHIC = 0, GEDMG_STAGGERED = 1 };

typedef struct {
  int32_t newton_iters;       /* assemblies - 1 */
  int32_t krylov_iters_total;
  int32_t n_yielded_qp;       /* quadrature points whose history grew in the accepted state */
  int32_t status;             /* same code as the return value */
  double res_norm[32];        /* ||R_f|| per Newton iteration (first 32) */
  double reaction;            /* sum of R over the reaction dofs given to newton_step, 0 if none */
  int32_t backtracks;         /* halvings of Newton corrections that inverted an element or gave a
                                 non-finite residual (at most 12 per load step) */
  int32_t krylov_fallbacks;   /* linear solves in which CG met non-positive curvature and BiCGStab
                                 took over */
} gedmg_newton_report;

typedef struct {
  int32_t n_checkpoints;       /* states stored (one per segment) */
  int32_t recomputed_steps;    /* load steps solved again from a checkpoint in the reverse sweep */
  int32_t newton_iters_total;  /* forward and recomputed steps */
  int32_t krylov_iters_total;  /* Newton solves and transposed adjoint solves */
  double t_forward_s, t_recompute_s, t_reverse_s;  /* wall time of the three phases */
} gedmg_adjoint_report;

/* Message for the last failure on this context (never NULL). */
const char* gedmg_last_error(const gedmg_ctx* ctx);

/* Build a context for one mesh, material and pair of networks: the element
 * data the residual kernel consumes (Table 1: nodal coordinates from which the
 * shape-function gradients and quadrature measures follow, connectivity for
 * the nodal u and phi values) and the ICNN parameters of Eqs. dd_0 and Gq_NN.
 * Copies the mesh, builds the CSR pattern of the (dim+1)^2 node-pair blocks,
 * the element colouring and the element -> CSR offset map, and uploads the
 * effective network weights.  All pointers in the descriptors are HOST
 * pointers, read during the call only.  hip_stream may be NULL (the null
 * stream).  On failure *ctx still receives a context (when it could be
 * allocated) whose gedmg_last_error() explains the failure; destroy it.
 * Returns GEDMG_E_ARG for null or empty meshes and connectivity indices out of
 * range, GEDMG_E_SHAPE for widths other than 16/32/64, energy n_in != 3, yield
 * n_in != 1, n_hidden outside 0..3 or more than 2^31 CSR entries,
 * GEDMG_E_NOMEM / GEDMG_E_HIP for device failures. */
int gedmg_create(gedmg_ctx** ctx, const gedmg_mesh* mesh, const gedmg_material* mat,
                 const gedmg_icnn* energy, const gedmg_icnn* yield, void* hip_stream);
int gedmg_destroy(gedmg_ctx* ctx);

/* Replace the raw network parameters (same architecture; host pointers; either
 * may be NULL to keep it).  Stream-ordered. */
int gedmg_set_params(gedmg_ctx* ctx, const double* theta_energy, const double* theta_yield);

/* The library-owned CSR pattern (device pointers, valid until destroy):
 * rowptr[n_rows+1], col[nnz], columns sorted in each row. */
int gedmg_csr(gedmg_ctx* ctx, int64_t* n_rows, int64_t* nnz, const int32_t** rowptr,
              const int32_t** col);

/* One assembly at the state (u, phi) with history kappa_n (Sec. 3.1-3.2):
 * R[ndof] = global residual (internal forces; every row, Dirichlet rows
 * included), K_vals[nnz] = consistent tangent in the CSR pattern (NULL:
 * residual only, skips the tangent; otherwise 16-byte aligned, and every entry
 * is overwritten, so it needs no clearing), kappa_trial[n_elems][nqp] = history after
 * the local update (it may be the kappa_n array itself: every point reads its
 * kappa_n before writing).  precision selects the arithmetic of the energy-network
 * layer products: GEDMG_FP64, or GEDMG_BF16 / GEDMG_FP16 matrix-core products
 * with FP32 accumulation (everything else stays FP64).
 * GEDMG_E_LOCAL_NOCONV / GEDMG_E_JNONPOS are reported by a later synchronising
 * call (gedmg_status) because assembly does not synchronise. */
int gedmg_assemble(gedmg_ctx* ctx, const double* u, const double* phi, const double* kappa_n,
                   int precision, double* R, double* K_vals, double* kappa_trial);

/* For callers that cannot allocate device memory while they run (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * gedmg_assemble with the per-point scratch of the assembly (network inputs,
 * jets, phi at the points, history sensitivities) in a static device array of
 * the library instead of buffers of the context.  Arguments, outputs and
 * errors are those of gedmg_assemble; the results are bitwise identical to it.
 * The call allocates nothing (no hipMalloc / hipFree, no events), clears R
 * with a kernel rather than a memset node, and rejects meshes with more than
 * GEDMG_STATIC_MAX_QP quadrature points (n_elems * nqp) with GEDMG_E_ARG.  The
 * array (GEDMG_STATIC_MAX_QP x 16 doubles = 32 MiB) exists once per GPU and
 * lives until the process ends; it is shared by every context on that GPU and
 * keeps the last call's contents, so calls that overlap on one GPU (two
 * streams, two host threads) race and must be serialised by the caller. */
#define GEDMG_STATIC_MAX_QP 262144
int gedmg_assemble_static(gedmg_ctx* ctx, const double* u, const double* phi, const double* kappa_n,
                          int precision, double* R, double* K_vals, double* kappa_trial);

/* Diagnostic: the energy-network jet at given inputs, in the arithmetic
 * selected by precision (used by the tests and by the mixed-precision error
 * report).  x: device [n][3] inputs (I1G - 3, I2G - 3, J - 1); jet: device
 * [n][10] = N(x) - N(0), dN/dx (3), d2N/dx2 (xx, yy, zz, xy, xz, yz).
 * n = 0 is a no-op (x and jet may then be NULL); n above 2^31 - 1 is
 * GEDMG_E_ARG. */
int gedmg_energy_jet(gedmg_ctx* ctx, const double* x, int64_t n, int precision, double* jet);

/* Per-phase timing of gedmg_assemble with HIP events recorded on the
 * context's stream (for benchmarks).  enable != 0 starts recording and clears
 * the totals.  gedmg_profile_read synchronises and returns, in ms summed over
 * the assemblies since enabling: out[0] quadrature inputs, out[1] energy-
 * network jets, out[2] local damage update, out[3] element kernels (all
 * colours), out[4] zero fills; *n_calls = assemblies timed.  out must hold 5
 * doubles (host). */
int gedmg_profile(gedmg_ctx* ctx, int enable);
int gedmg_profile_read(gedmg_ctx* ctx, double* out_ms, int32_t* n_calls);

/* Counter calibration (for profiling only): launches `blocks` workgroups of
 * 256 threads (4 waves) on hip_stream, each wave issuing 4 x iters FP64
 * 16x16x4 matrix products (2048 flop each) and nothing else, so an MFMA-busy
 * counter reading can be related to a known number of products.  sink: device
 * [blocks * 256] doubles that receive the sums (keeps the products live).
 * Returns GEDMG_E_ARG for null sink or non-positive sizes. */
int gedmg_probe_mfma(double* sink, int32_t blocks, int32_t iters, void* hip_stream);

/* Synchronise the stream and return the sticky device status of the last
 * assemblies (GEDMG_OK, GEDMG_E_LOCAL_NOCONV or GEDMG_E_JNONPOS), then clear it. */
int gedmg_status(gedmg_ctx* ctx);

/* One load step of incremental quasi-static loading (Sec. 3.2; the step starts
 * from the last converged solution), with the monolithic scheme by default (the
 * history update of Eq. dd_7 runs inside every global Newton iteration and its
 * sensitivities enter the tangent) or the staggered one (opts->scheme).  The call
 *   1. adds the predictor increment predictor_du (device [dim][n_nodes], may be
 *      NULL for none) to u: the caller's extrapolation of the last converged
 *      displacement, e.g. the boundary increment spread over the body;
 *   2. sets the prescribed dofs bc (device dof / value arrays);
 *   3. runs Newton on the free dofs, with a preconditioned Krylov solve of
 *      K_ff d = -R_f per iteration (CG with Jacobi plus a coarse correction on
 *      node aggregates, whose span holds the uniform damage field; BiCGStab
 *      with the same preconditioner when CG meets
 *      non-positive curvature on a non-symmetric or indefinite tangent), a
 *      correction that inverts an element being halved (up to 12 times), until
 *      ||R_f|| <= max(newton_rtol max(newton_rscale, ||R_f^0||), newton_atol);
 *   4. commits kappa_{n+1} (staggered: the local update of Eq. dd_7 at the
 *      converged fields, computed once after the global solve with kappa_n).
 * precision != GEDMG_FP64 uses the mixed-precision tangent with the FP64
 * residual (iterative refinement, see refine_max / refine_rtol).  u, phi:
 * device [dim][n_nodes], [n_nodes], in: the last converged state, out: the
 * converged state; kappa: device [n_elems][nqp], in kappa_n, out kappa_{n+1}.
 * On failure all three are restored to their input values (before the
 * predictor).  opts may be NULL (defaults).  reaction_dofs (device, distinct,
 * in range; may be NULL when n_reaction == 0) selects the rows of the converged
 * residual summed into report->reaction (staggered: the residual of the global
 * solve, with the history at kappa_n).  report is a host struct, may be NULL.
 * Synchronises the stream.  Allocates its Krylov workspace on the first call
 * for a context (freed by gedmg_destroy).  Errors: GEDMG_E_ARG (null or
 * inconsistent arguments, dofs out of range), GEDMG_E_NONFINITE,
 * GEDMG_E_LOCAL_NOCONV, GEDMG_E_JNONPOS, GEDMG_E_LINSOLVE,
 * GEDMG_E_NEWTON_NOCONV, GEDMG_E_NOMEM, GEDMG_E_HIP. */
int gedmg_newton_step(gedmg_ctx* ctx, const gedmg_dirichlet* bc, const gedmg_solver_opts* opts,
                      int precision, const double* predictor_du, double* u, double* phi, double* kappa,
                      const int32_t* reaction_dofs, int32_t n_reaction,
                      gedmg_newton_report* report);

/* One increment of arc-length continuation for displacement-controlled loading
 * (the paper solves its strongly softening single-element study with an
 * arc-length continuation, Sec. 5.1; Sec. 3.2 names the approach): the
 * prescribed dofs carry lambda times their unit values pattern->value, and the
 * load factor lambda is solved for together with the free dofs under
 * ||Delta d_f||_W^2 + psi^2 Delta lambda^2 = ds^2, so the path is followed
 * through limit points of the load factor (snap-back), where displacement
 * control has no solution nearby.  Riks' scheme: the predictor is the previous
 * increment scaled to length ds (secant); for a first increment (increment all
 * zero) it is the path tangent t = -K_ff^-1 K_fp uhat with the history held at
 * kappa, scaled to ds, with Delta lambda > 0.  (The yielded points of a
 * converged state sit on the yield surface to rounding; neither predictor asks
 * whether they load.)  The corrector iterates in the plane normal to the predictor with
 * two Krylov solves per iteration, a = -K_ff^-1 R_f and b = -K_ff^-1 K_fp uhat,
 * dlambda = -(Dd . a) / (Dd . b + psi^2 Dlambda), dd = a + dlambda b, until the
 * Newton test of gedmg_newton_step holds.  FP64, monolithic history (opts->
 * scheme and refine_* are ignored).
 *   pattern     Dirichlet set: device dof indices and their unit values uhat
 *   ds, psi     arc length (> 0) and load-factor scale (>= 0; 0: cylindrical)
 *   phi_weight  weight (>= 0, finite) of the nonlocal damage dofs in ||.||_W, the
 *               displacement dofs having weight 1: 1 gives the plain norm of
 *               all free dofs; phi is an energy-like field, and where its
 *               increments outgrow the displacements' (a notched plate), 0
 *               measures the arc length in displacements only
 *   lambda      host, in: the load factor of the state passed in; out: the
 *               converged one
 *   increment   device [ndof + 1], in: the previous increment (free dofs in the
 *               node-major dof layout, zero on Dirichlet rows, Delta lambda
 *               last; all zeros for a first increment); out: this increment
 *   u, phi, kappa, reaction_dofs, n_reaction, report: as for gedmg_newton_step
 *               (u, phi, kappa and lambda restored on failure)
 * Synchronises the stream; allocates four vectors of workspace on its first
 * call for a context.  Errors: those of gedmg_newton_step, GEDMG_E_LINSOLVE
 * when the constraint cannot be solved (Dd . b + psi^2 Dlambda = 0). */
int gedmg_arclength_step(gedmg_ctx* ctx, const gedmg_dirichlet* pattern, const gedmg_solver_opts* opts,
                         double ds, double psi, double phi_weight, double* lambda, double* increment, double* u,
                         double* phi, double* kappa, const int32_t* reaction_dofs, int32_t n_reaction,
                         gedmg_newton_report* report);

/* Gradient of the load-path loss L = sum_n (r_n - t_n)^2, r_n the reaction of
 * step n, with respect to the raw parameters of both networks (the paper
 * motivates differentiating through the solver for design and inverse
 * problems, Sec. 5; the residual and history update are those of Secs. 3.1-3.2).
 *
 * Runs the n_steps load steps of gedmg_newton_step (FP64) from the state
 * (u, phi, kappa) passed in, then the discrete adjoint backwards over the
 * steps: per step a transposed Krylov solve K_T^T lambda = d(ell_n + abar .
 * kappa_n)/dU on the free dofs, the vector-Jacobian products of the residual
 * and of the history update with respect to the parameters, and the history
 * adjoint abar_{n-1}.  States are stored only at the start of every segment of
 * checkpoint_every steps and recomputed segment by segment (checkpoint_every
 * <= 0 or >= n_steps: one segment, nothing recomputed).  The recompute is
 * bitwise identical to the forward pass, so the gradient does not depend on
 * checkpoint_every.
 *
 *   bc_per_step   host array [n_steps] of Dirichlet sets (device dof/value)
 *   predictor_du  device [n_steps][dim][n_nodes] displacement increments added
 *                 to u before each step (the predictor), or NULL
 *   reaction_dofs device [n_reaction], distinct, prescribed in every step
 *   targets       device [n_steps]
 *   opts          Newton / Krylov options of every solve (NULL: defaults)
 *   u, phi, kappa device state: in, the start of the path; out, its end
 *   loss          host scalar
 *   grad_energy   host [n_params(energy)], raw order
 *   grad_yield    host [n_params(yield)], raw order
 *   report        host, may be NULL
 * The output biases cancel in N - N(0): their gradients are exactly zero.
 * Synchronises the stream.  Device memory: about (n_steps / checkpoint_every
 * + checkpoint_every) states, two CSR value arrays and per-point network
 * activations, allocated per call.  Errors: those of gedmg_newton_step
 * (then the state is unspecified), GEDMG_E_ARG for bad reaction dofs,
 * GEDMG_E_SHAPE for yield widths above 32. */
int gedmg_adjoint(gedmg_ctx* ctx, int32_t n_steps, const gedmg_dirichlet* bc_per_step,
                  const double* predictor_du, const int32_t* reaction_dofs, int32_t n_reaction,
                  const double* targets, int32_t checkpoint_every, const gedmg_solver_opts* opts,
                  double* u, double* phi, double* kappa, double* loss, double* grad_energy,
                  double* grad_yield, gedmg_adjoint_report* report);

#ifdef __cplusplus
}
#endif
#endif /* GEDMG_H */
