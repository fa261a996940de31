"""Load-path Newton solves and the load-path-loss adjoint (oracle; test
infrastructure only).

Monolithic scheme (Sec. 3.2): the history update runs inside every global
Newton iteration and its sensitivities are part of the tangent; each load
step starts from a predictor built from the last converged solution
(Sec. 3.2, last paragraph).  The linear systems are solved directly (sparse
LU, as the paper does with PETSc).

The adjoint differentiates L = sum_n (reaction_n - target_n)^2 with respect to
the raw network parameters through the converged load path: for steps
n = N..1, with abar_n the sensitivity of the later losses to kappa_n,
    K_T^T lambda_n = d/dU [ell_n + abar_n . kappa_n],
    dL/dtheta     += d/dtheta [ell_n + abar_n . kappa_n - lambda_n . R_f],
    abar_{n-1}     = d/dkappa_{n-1} [ell_n + abar_n . kappa_n - lambda_n . R_f],
where every partial derivative is an autograd vector-Jacobian product of the
residual written as a function of (U, kappa_{n-1}, theta).  The paper only
motivates differentiating through the solver (Sec. 5); the loss is the
reaction-force misfit of the benchmark.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla
import torch

from . import fem

DT = torch.float64


def default_atol(mesh):
    """Absolute floor of the Newton test: the penalty term beta_d (phi - kappa)
    leaves a rounding floor that grows like the square root of the number of
    equations."""
    return 1e-9 * float(np.sqrt(mesh.ndof))


def newton(model, mesh, d0, kappa_n, bc_dofs, bc_vals, rtol=1e-10, atol=None, max_iter=25,
           scheme="monolithic", rscale=1.0):
    """Solve R_f(d) = 0 for one load step.  Converged when
    ||R_f|| <= max(rtol * max(rscale, ||R_f^0||), atol).  Returns (d, kappa_{n+1},
    history, converged).

    scheme (Sec. 3.2): "monolithic" updates the history inside every global
    iteration (its sensitivities are part of the tangent); "staggered" solves
    the global problem with the history held at kappa_n and updates the
    history once, at the converged fields."""
    if scheme not in ("monolithic", "staggered"):
        raise ValueError(scheme)
    upd = scheme == "monolithic"
    atol = default_atol(mesh) if atol is None else atol
    d = np.array(d0, dtype=np.float64, copy=True)
    d[bc_dofs] = bc_vals
    free = np.ones(mesh.ndof, bool)
    free[bc_dofs] = False
    hist = []
    res0 = None
    for it in range(max_iter + 1):
        R, K, kt = fem.assemble(model, mesh, d, kappa_n, update_history=upd)
        Rf = R[free]
        res = float(np.linalg.norm(Rf))
        res0 = res if res0 is None else res0
        hist.append(res)
        if res <= max(rtol * max(rscale, res0), atol):
            if not upd:
                _, _, kt = fem.assemble(model, mesh, d, kappa_n, tangent=False)
            return d, kt, hist, True
        if it == max_iter or not np.isfinite(res):
            break
        Kff = K[free][:, free].tocsc()
        d[free] += spla.spsolve(Kff, -Rf)
    return d, kt, hist, False


def reaction(R, react_dofs):
    return float(np.sum(R[react_dofs]))


def load_path(case, model, steps=None, bc_fn=None, predictor_fn=None, react_dofs=None,
              rtol=1e-10, atol=None, scheme="monolithic", rscale=1.0):
    """Run the incremental quasi-static load path.  Returns a list of per-step
    records with the converged dofs, the history before/after and the
    reaction force (at the converged fields and the history the global solve
    used: kappa_{n+1} for the monolithic scheme, kappa_n for the staggered one)."""
    import workloads as W

    mesh = case.mesh
    steps = case.n_steps if steps is None else steps
    bc_fn = bc_fn or W.uniaxial_bc
    predictor_fn = predictor_fn or W.uniaxial_predictor
    react_dofs = W.reaction_dofs(case) if react_dofs is None else react_dofs
    u, phi = case.u.copy(), case.phi.copy()
    kappa = case.kappa.copy()
    out = []
    for n in range(1, steps + 1):
        u0 = predictor_fn(case, u, n)
        d0 = fem.dof_vector(u0, phi)
        bd, bv = bc_fn(case, n)
        d, kt, hist, ok = newton(model, mesh, d0, kappa, bd, bv, rtol=rtol, atol=atol, scheme=scheme,
                                 rscale=rscale)
        if not ok:
            raise RuntimeError(f"oracle Newton did not converge at step {n}: {hist}")
        R, _, _ = fem.assemble(model, mesh, d, kappa, tangent=False,
                               update_history=scheme == "monolithic")
        out.append(dict(step=n, d=d.copy(), kappa_prev=kappa.copy(), kappa=kt.copy(),
                        reaction=reaction(R, react_dofs), hist=hist, bc=(bd, bv)))
        u, phi = fem.split_dofs(d, mesh.dim)
        kappa = kt
    return out


def loss_and_gradient(case, records, targets, theta_e=None, theta_y=None, react_dofs=None):
    """Loss sum_n (r_n - t_n)^2 over a converged load path and its gradient
    with respect to the raw energy and yield parameters (discrete adjoint)."""
    import workloads as W

    mesh = case.mesh
    te0 = torch.as_tensor(case.theta_e if theta_e is None else theta_e, dtype=DT)
    ty0 = torch.as_tensor(case.theta_y if theta_y is None else theta_y, dtype=DT)
    react = torch.as_tensor(W.reaction_dofs(case) if react_dofs is None else react_dofs)
    loss = sum((r["reaction"] - t) ** 2 for r, t in zip(records, targets))
    g_e = torch.zeros_like(te0)
    g_y = torch.zeros_like(ty0)
    abar = torch.zeros(mesh.n_elems * mesh.nqp, dtype=DT)
    for rec, t in zip(reversed(records), reversed(list(targets))):
        te = te0.clone().requires_grad_(True)
        ty = ty0.clone().requires_grad_(True)
        model = fem.Model(case, te, ty)
        bd = rec["bc"][0]
        free = np.ones(mesh.ndof, bool)
        free[bd] = False
        U = torch.tensor(rec["d"], dtype=DT, requires_grad=True)
        kp = torch.tensor(rec["kappa_prev"].reshape(-1), dtype=DT, requires_grad=True)
        R, kap = fem.residual_torch(model, mesh, U, kp)
        ell = (R[react].sum() - t) ** 2
        Phi = ell + (abar * kap).sum()
        (dPhi_dU,) = torch.autograd.grad(Phi, U, retain_graph=True)
        _, K, _ = fem.assemble(fem.Model(case, te0, ty0), mesh, rec["d"], rec["kappa_prev"])
        Kff = K[free][:, free].tocsc()
        lam = np.zeros(mesh.ndof)
        lam[free] = spla.spsolve(Kff.T.tocsc(), dPhi_dU.numpy()[free])
        lam_t = torch.tensor(lam, dtype=DT)
        G = Phi - (lam_t * R).sum()
        ge, gy, gk = torch.autograd.grad(G, (te, ty, kp))
        g_e += ge
        g_y += gy
        abar = gk.detach()
    return loss, g_e.numpy(), g_y.numpy()


def arclength_step(model, mesh, d, lam, kappa_n, bc_dofs, bc_unit, ds, psi=1.0, prev=None, rtol=1e-10,
                   atol=None, max_iter=25, rscale=1.0, phi_weight=1.0):
    """One increment of arc-length continuation for displacement-controlled
    loading (the paper's arc-length remark in Sec. 3.2 and its use in Sec. 5.1):
    the prescribed dofs carry lam * bc_unit, and the load factor lam is an
    unknown next to the free dofs, tied by the constraint
    ||Delta d_f||_W^2 + psi^2 Delta lam^2 = ds^2 (Riks: the corrector iterates in
    the plane normal to the predictor).  ||.||_W weights the nonlocal damage
    dofs by phi_weight (1: the plain norm of all free dofs; 0: the displacement
    dofs only, for problems where phi, an energy-like field, would dominate
    the length of an increment).

    Predictor: the previous increment `prev` = (Delta d_f, Delta lam) scaled to
    length ds (secant); for the first increment (prev None) the tangent
    t = -K_ff^-1 K_fp bc_unit of the equilibrium path with the history held at
    kappa_n, scaled to ds, forward.  (At a converged state the yielded points sit
    on the yield surface to rounding, so whether a loading or an elastic
    tangent is taken there would be decided by rounding; the secant and the
    held-history tangent are defined without that decision.)  Corrector:
    a = -K_ff^-1 R_f, b = -K_ff^-1 K_fp bc_unit,
    dlam = -(Dd . a) / (Dd . b + psi^2 Dlam), dd = a + dlam b, with (Dd, Dlam)
    the predictor.  The history is updated inside every iteration (monolithic).
    Converged when ||R_f|| <= max(rtol * max(rscale, ||R_f^0||), atol), R_f^0
    the residual at the predictor.

    Returns (d, lam, kappa_{n+1}, (Delta d_f, Delta lam), residual history,
    converged)."""
    atol = default_atol(mesh) if atol is None else atol
    free = np.ones(mesh.ndof, bool)
    free[bc_dofs] = False
    nd = mesh.dim + 1
    wt = np.where(np.arange(mesh.ndof) % nd == nd - 1, phi_weight * phi_weight, 1.0)[free]

    def wdot(a, b):
        return float(np.sum(wt * a * b))

    uhat = np.zeros(mesh.ndof)
    uhat[bc_dofs] = bc_unit
    d = np.array(d, dtype=np.float64, copy=True)
    d[bc_dofs] = lam * np.asarray(bc_unit)
    d0f = d[free].copy()
    lam0 = lam
    if prev is not None:
        scale = ds / np.sqrt(wdot(prev[0], prev[0]) + psi * psi * prev[1] ** 2)
        dd_p = scale * np.asarray(prev[0])
        dlam_p = scale * prev[1]
    else:
        R, K, _ = fem.assemble(model, mesh, d, kappa_n, update_history=False)
        Kff = K[free][:, free].tocsc()
        t = spla.spsolve(Kff, -(K @ uhat)[free])
        dlam_p = ds / np.sqrt(wdot(t, t) + psi * psi)
        dd_p = dlam_p * t
    lam = lam0 + dlam_p
    d[free] = d0f + dd_p
    d[bc_dofs] = lam * np.asarray(bc_unit)
    hist = []
    res0 = None
    for it in range(max_iter + 1):
        R, K, kt = fem.assemble(model, mesh, d, kappa_n)
        Rf = R[free]
        res = float(np.linalg.norm(Rf))
        res0 = res if res0 is None else res0
        hist.append(res)
        if res <= max(rtol * max(rscale, res0), atol):
            return d, lam, kt, (d[free] - d0f, lam - lam0), hist, True
        if it == max_iter or not np.isfinite(res):
            break
        Kff = K[free][:, free].tocsc()
        lu = spla.splu(Kff)
        a = lu.solve(-Rf)
        b = lu.solve(-(K @ uhat)[free])
        dl = -wdot(dd_p, a) / (wdot(dd_p, b) + psi * psi * dlam_p)
        d[free] += a + dl * b
        lam += dl
        d[bc_dofs] = lam * np.asarray(bc_unit)
    return d, lam, kt, (d[free] - d0f, lam - lam0), hist, False
