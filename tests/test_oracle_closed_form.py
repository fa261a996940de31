"""Pins of the oracle's closed-form model (Sec. 4.1: compressible Neo-Hooke
energy, Ostwald loading function with G = identity), the local model and the
staggered scheme (Sec. 3.2), against closed forms and the single-element
result of Sec. 5.1."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import constitutive as cm
from oracle import fem, solve

DT = torch.float64


def nh_mat():
    mu, lam = W.lame(42.0, 0.45)
    return dict(mu_e=mu, lambda_e=lam, eta_d=10.0, kappa_d=1.0, c_d=0.0, beta_d=0.0, gamma_d=1.0)


def test_neo_hooke_energy_hand_value():
    """F = diag(2, 1, 1): I1 = 6, J = 2; psi = mu/2 * 3 - mu ln 2 + lam/2 (ln 2)^2."""
    mat = nh_mat()
    E = cm.NeoHooke(mat)
    F = torch.diag(torch.tensor([2.0, 1.0, 1.0], dtype=DT))[None]
    mu, lam = mat["mu_e"], mat["lambda_e"]
    ref = 1.5 * mu - mu * math.log(2.0) + 0.5 * lam * math.log(2.0) ** 2
    assert abs(float(E(F)) - ref) < 1e-12 * ref


def test_neo_hooke_stress_is_the_textbook_closed_form():
    """P = mu (F - F^-T) + lambda ln J F^-T, and P(I) = 0."""
    mat = nh_mat()
    E = cm.NeoHooke(mat)
    rng = np.random.default_rng(4)
    Fn = np.eye(3)[None] + 0.2 * rng.standard_normal((6, 3, 3))
    Fn[np.linalg.det(Fn) < 0] *= -1.0
    F = torch.tensor(Fn, dtype=DT, requires_grad=True)
    (P,) = torch.autograd.grad(E(F).sum(), F)
    for k in range(6):
        FiT = np.linalg.inv(Fn[k]).T
        ref = mat["mu_e"] * (Fn[k] - FiT) + mat["lambda_e"] * math.log(np.linalg.det(Fn[k])) * FiT
        assert np.allclose(P[k].numpy(), ref, rtol=1e-12, atol=1e-12)
    F0 = torch.eye(3, dtype=DT)[None].requires_grad_(True)
    (P0,) = torch.autograd.grad(E(F0).sum(), F0)
    assert float(P0.abs().max()) == 0.0 and float(E(F0.detach())) == 0.0


def test_ostwald_root_with_identity_yield():
    """With G = identity the local update solves Eq. ostwald_potential:
    psi_NH + gamma beta (phi - kappa) / (eta f_d(kappa)) - kappa = 0, evaluated
    here in plain floating point at the oracle's root."""
    mat = dict(nh_mat(), beta_d=50.0, c_d=1.0, eta_d=2.0, kappa_d=0.5)
    E = cm.NeoHooke(mat)
    Y = cm.IdentityYield()
    F = torch.diag(torch.tensor([1.35, 0.9, 0.92], dtype=DT))[None].expand(4, 3, 3)
    psi = E(F)
    phi = torch.tensor([0.2, 0.9, 1.4, 2.5], dtype=DT)
    kn = torch.tensor([0.1, 0.3, 0.4, 5.0], dtype=DT)
    k, yielded, _ = cm.local_update(psi, phi, kn, Y, mat)
    for i in range(4):
        p, ph, kk = float(psi[i]), float(phi[i]), float(k[i])
        fd = math.exp(-mat["eta_d"] * max(kk - mat["kappa_d"], 0.0))
        h = p + mat["gamma_d"] * mat["beta_d"] * (ph - kk) / (mat["eta_d"] * fd) - kk
        if bool(yielded[i]):
            assert kk > float(kn[i]) and abs(h) < 1e-9 * max(1.0, p + abs(mat["beta_d"] * (ph - kk) / (mat["eta_d"] * fd)))
        else:
            assert kk == float(kn[i]) and h <= 0.0
    assert bool(yielded[:3].all()) and not bool(yielded[3])


def single_element_path(eta, kd, steps=12):
    """The local model of the single-element study, with the history updated
    after each converged step (staggered scheme).  The monolithic local
    iteration does not converge here once the element softens: its tangent
    f_d (psi_FF - eta_d psi_F (x) psi_F) is indefinite and Newton runs towards
    the trivial branch f_d -> 0, where the residual vanishes with f_d (the
    failure of the local monolithic strategy that Sec. 5.2 reports).  The
    relative Newton test (rscale = 0) keeps the lateral equilibrium accurate
    however small f_d becomes."""
    case = W.single_element_case(eta_d=eta, kappa_d=kd, n_steps=steps)
    du = W.uniaxial_increment(case)
    recs = solve.load_path(case, fem.Model(case), bc_fn=W.symmetric_tension_bc,
                           predictor_fn=lambda c, u, n: u + du, rtol=1e-12, atol=0.0, rscale=0.0,
                           scheme="staggered")
    return case, recs


def test_single_element_kappa_does_not_depend_on_damage_parameters():
    """Sec. 5.1: with the nonlocal regularisation disabled (local model), the
    history kappa(stretch) of the uniaxially stretched element does not change
    with eta_d and kappa_d: f_d(kappa) scales the whole stress, so the lateral
    equilibrium is the damage-free one, and with G = identity kappa is the
    running maximum of psi_NH along it.  Each point's kappa must equal
    psi_NH(F_n) of the converged deformation."""
    runs = [single_element_path(eta, kd) for eta, kd in ((1.0, 0.0), (10.0, 1.0), (100.0, 2.0))]
    k_ref = np.array([r["kappa"] for r in runs[0][1]])
    for case, recs in runs:
        ks = np.array([r["kappa"] for r in recs])
        assert np.allclose(ks, k_ref, rtol=1e-9, atol=1e-12), case.name
        # every point carries the same value, growing with the stretch
        assert np.ptp(ks, axis=(1, 2)).max() <= 1e-10 * ks.max()
        assert np.all(np.diff(ks[:, 0, 0]) > 0.0)
    # kappa = psi_NH of the converged deformation gradient (uniform F)
    case, recs = runs[1]
    m = fem.Model(case)
    for r in recs[::4]:
        u, _ = fem.split_dofs(r["d"], 3)
        L = 1.0 + u[:, 7]  # node 7 sits at (1, 1, 1): F = diag(1 + u7)
        F = torch.diag(torch.tensor(L, dtype=DT))[None]
        assert abs(float(m.energy(F)) - r["kappa"][0, 0]) < 1e-9 * r["kappa"][0, 0]


def test_single_element_damage_follows_degradation_function():
    """d = 1 - exp(-eta_d <kappa - kappa_d>_+) (Eq. degradation_function) and
    the axial force falls with eta_d at the same stretch."""
    (c1, r1), (c2, r2) = single_element_path(1.0, 1.0), single_element_path(5.0, 1.0)
    k = r1[-1]["kappa"][0, 0]
    d1, d2 = 1.0 - math.exp(-1.0 * max(k - 1.0, 0.0)), 1.0 - math.exp(-5.0 * max(k - 1.0, 0.0))
    assert d2 > d1 > 0.0
    assert abs(r2[-1]["reaction"]) < abs(r1[-1]["reaction"])


def test_staggered_scheme_lags_the_history_by_one_step():
    """Staggered scheme on the uniform-stretch box: the global solve holds
    kappa_n, so the uniform nonlocal field converges to phi_n = kappa_{n-1}
    (R_phi = beta_d (phi - kappa_{n-1}) at a uniform state), and the history
    then solves the local problem at phi_n: N^(psi_e + gamma beta (phi_n -
    kappa) / (eta f_d(kappa))) = kappa, found here by bisection on the scalar."""
    case = W.make_case(2, n=2, nz=1)
    m = fem.Model(case)
    mat = case.material
    lam = case.extra["stretch"]
    kap, phi = case.kappa.copy(), case.phi.copy()
    k_prev = 0.0
    for n in range(1, 4):
        bd, bv = W.affine_stretch_bc(case, n)
        s = n / case.n_steps
        u0 = s * (lam[:, None] - 1.0) * case.mesh.X
        d, kt, hist, ok = solve.newton(m, case.mesh, fem.dof_vector(u0, phi), kap, bd, bv, rtol=0.0, atol=1e-11,
                                       scheme="staggered")
        assert ok
        u, phi = fem.split_dofs(d, 3)
        assert np.abs(phi - k_prev).max() < 1e-9 * max(1.0, k_prev)
        F = torch.diag(torch.tensor(1.0 + s * (lam - 1.0), dtype=DT))[None]
        pe = float(m.energy(F))
        gbe = mat["gamma_d"] * mat["beta_d"] / mat["eta_d"]

        def h(k):
            fd = math.exp(-mat["eta_d"] * max(k - mat["kappa_d"], 0.0))
            q = pe + gbe * (k_prev - k) / fd
            return float(m.yld(torch.tensor([q], dtype=DT))[0]) - k

        lo, hi = k_prev, max(k_prev, float(m.yld(torch.tensor([pe], dtype=DT))[0]))
        if h(lo) > 0.0:
            for _ in range(200):
                mid = 0.5 * (lo + hi)
                lo, hi = (mid, hi) if h(mid) > 0.0 else (lo, mid)
            k_new = 0.5 * (lo + hi)
        else:
            k_new = k_prev
        assert np.abs(kt - k_new).max() < 1e-9 * max(1.0, k_new)
        # the lag: the staggered history stays far below the monolithic one
        assert k_new < float(m.yld(torch.tensor([pe], dtype=DT))[0])
        kap, k_prev = kt, k_new
