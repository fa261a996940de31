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
