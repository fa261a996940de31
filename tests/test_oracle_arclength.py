"""Pins of the oracle's arc-length continuation (Riks' scheme for the load
factor of displacement-controlled loading): its converged states are
equilibrium states of the same discrete problem as displacement control, so
on the monotonic part of the path a displacement-controlled Newton step to the
same load factor lands on the same state; and the increments satisfy the
normal-plane constraint's consequence ||Delta d||^2 + psi^2 Delta lambda^2 >= ds^2
(the corrector leaves the predictor's sphere outwards).

The single-element path of Sec. 5.1 (local closed-form model, strong
softening) has a closed form at every load factor: the deformation is the
homogeneous uniaxial one F = diag(s, t, t) whose lateral Neo-Hooke stress
vanishes, kappa = psi_NH(F) and the axial force is f_d(kappa) P11_NH(F) on the
unit face.  Every converged arc-length increment must lie on it."""
import math

import numpy as np
import pytest

import workloads as W
from oracle import fem, solve


@pytest.mark.parametrize("psi,wphi", [(1.0, 1.0), (0.0, 1.0), (1.0, 0.0)])
def test_arclength_states_are_displacement_controlled_equilibria(psi, wphi):
    """psi = 0 is the cylindrical form: the arc length counts the free dofs
    only; wphi = 0 leaves the nonlocal damage dofs out of it."""
    case = W.strip_case(nx=20)
    m = fem.Model(case)
    bd, bu = W.arclength_pattern(case)
    d = fem.dof_vector(case.u, case.phi)
    kap = case.kappa.copy()
    lam, prev, ds = 0.0, None, 0.1
    for n in range(8):
        d_prev, k_prev, lam_prev = d.copy(), kap.copy(), lam
        d, lam, kt, inc, hist, ok = solve.arclength_step(m, case.mesh, d, lam, kap, bd, bu, ds, psi=psi, prev=prev,
                                                         atol=1e-11, phi_weight=wphi)
        assert ok
        assert lam > lam_prev  # rising part of the path
        free = np.ones(case.mesh.ndof, bool)
        free[bd] = False
        wt = np.where(np.arange(case.mesh.ndof) % 3 == 2, wphi * wphi, 1.0)[free]
        L2 = float(np.sum(wt * inc[0] * inc[0]) + psi * psi * inc[1] ** 2)
        assert L2 >= ds * ds * (1.0 - 1e-12)
        # displacement control to the same load factor from the same start
        dc, kc, h2, ok2 = solve.newton(m, case.mesh, d_prev, k_prev, bd, lam * bu, rtol=0.0, atol=1e-11)
        assert ok2
        assert np.abs(dc - d).max() <= 1e-8 * np.abs(d).max()
        assert np.abs(kc - kt).max() <= 1e-8 * max(1e-3, np.abs(kt).max())
        kap, prev = kt, inc


def _uniaxial_neo_hooke(s, mu, lam):
    """Lateral stretch t of the uniaxial Neo-Hooke state at axial stretch s
    (P22 = mu (t - 1/t) + lam ln(s t^2) / t = 0, by bisection on (0, 1]),
    with the energy and the axial first Piola-Kirchhoff stress."""
    g = lambda t: mu * (t - 1.0 / t) + lam * math.log(s * t * t) / t
    lo, hi = 1e-3, 1.0
    for _ in range(200):
        mid = 0.5 * (lo + hi)
        if g(mid) > 0.0:
            hi = mid
        else:
            lo = mid
    t = 0.5 * (lo + hi)
    lnJ = math.log(s * t * t)
    psi = 0.5 * mu * (s * s + 2.0 * t * t - 3.0) - mu * lnJ + 0.5 * lam * lnJ * lnJ
    p11 = mu * (s - 1.0 / s) + lam * lnJ / s
    return t, psi, p11


def test_single_element_arclength_follows_the_closed_form_softening_path():
    eta, kd = 10.0, 1.0
    case = W.single_element_case(eta_d=eta, kappa_d=kd)
    mu, lam_l = W.lame(42.0, 0.45)
    m = fem.Model(case)
    bd, bu = W.arclength_pattern(case, W.symmetric_tension_bc)
    rd = W.reaction_dofs(case)
    X = case.mesh.X
    top_y = np.nonzero(np.abs(X[1] - 1.0) < 1e-12)[0]
    top_z = np.nonzero(np.abs(X[2] - 1.0) < 1e-12)[0]
    d = fem.dof_vector(case.u, case.phi)
    kap = case.kappa.copy()
    lam, prev, ds = 0.0, None, 0.02
    forces = []
    while lam < 0.5:
        lam_prev = lam
        d, lam, kt, inc, hist, ok = solve.arclength_step(m, case.mesh, d, lam, kap, bd, bu, ds, prev=prev,
                                                         rtol=1e-9, atol=0.0, rscale=0.0)
        assert ok and lam > lam_prev
        u, _ = fem.split_dofs(d, 3)
        s = 1.0 + lam
        t, psi, p11 = _uniaxial_neo_hooke(s, mu, lam_l)
        # homogeneous lateral contraction of the Neo-Hooke uniaxial state
        assert np.allclose(1.0 + u[1, top_y], t, rtol=0.0, atol=1e-10)
        assert np.allclose(1.0 + u[2, top_z], t, rtol=0.0, atol=1e-10)
        # kappa = psi_NH at every point; d = 1 - f_d(kappa)
        assert np.allclose(kt, psi, rtol=1e-10, atol=0.0)
        R, _, _ = fem.assemble(m, case.mesh, d, kap, tangent=False)
        f = solve.reaction(R, rd)
        f_ref = math.exp(-eta * max(psi - kd, 0.0)) * p11
        assert abs(f - f_ref) <= 1e-9 * abs(f_ref)
        forces.append(f)
        kap, prev = kt, inc
    forces = np.array(forces)
    k = int(forces.argmax())
    # the path passes the peak and follows the softening branch to a small force
    assert 0 < k < len(forces) - 1 and forces[-1] < 1e-3 * forces[k]
