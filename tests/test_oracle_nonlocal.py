"""Pins of the oracle's nonlocal energy terms (Sec. 4.1, the gradient and
penalty contributions reused unchanged by the data-driven model of Eq. dd_3):

    psi_grad = c_d / 2  grad phi . C^-1 . grad phi,
    psi_plty = beta_d / 2 (phi - kappa)^2,

their conjugates Y_vec = d Psi / d grad phi = c_d C^-1 grad phi and
Y = -d Psi / d phi = -beta_d (phi - kappa) (Eqs. nonlocal_conjugate_calc), and
the stress part of the gradient term, d psi_grad / dF = -c_d (F C^-1 g) (x) (C^-1 g).

Every expected value is written out by hand (diagonal stretches, where
C^-1 = diag(1 / lambda_i^2)) or computed from an explicitly inverted C with
numpy, never from the oracle's own formulas.  Replacing C^-1 by C, or dropping
the factor 1/2 of either term, fails a test below.
"""
import numpy as np
import torch

import workloads as W
from oracle import constitutive as cm

DT = torch.float64

# Diagonal stretch and gradient used by the hand-value tests.
LAM = (2.0, 0.5, 1.25)
G = (0.3, -0.7, 1.1)
C_D = 2.5
BETA = 1000.0


def _mat(**kw):
    # A small elastic scale keeps f_d psi_e (about 1e8 mu_e at these stretches with
    # the seeded network) from swamping the nonlocal terms in the differences below.
    m = dict(W.MATERIAL)
    m.update(c_d=C_D, beta_d=BETA, mu_e=1e-9, lambda_e=1e-9)
    m.update(kw)
    return m


def _energy(mat):
    c = W.make_case(4, n=2)
    return cm.Energy(torch.tensor(c.theta_e), c.energy, mat), c


def _diag_state():
    F = torch.diag(torch.tensor(LAM, dtype=DT))[None]
    g = torch.tensor(G, dtype=DT)[None]
    return F, g


def test_gradient_energy_hand_value_diagonal_stretch():
    """psi_grad = c_d/2 sum_i g_i^2 / lambda_i^2:
    0.09/4 + 0.49/0.25 + 1.21/1.5625 = 0.0225 + 1.96 + 0.7744 = 2.7569, times
    2.5/2 = 3.446125.  (C in place of C^-1 gives 2.96640625; a dropped 1/2 gives
    6.89225.)"""
    mat = _mat()
    E, _ = _energy(mat)
    F, g = _diag_state()
    k = torch.tensor([0.25], dtype=DT)
    phi = k.clone()                     # penalty term zero
    with_g = cm.free_energy(F, phi, g, k, E, mat)
    no_g = cm.free_energy(F, phi, torch.zeros_like(g), k, E, mat)
    assert abs(float(with_g - no_g) - 3.446125) < 1e-12


def test_penalty_energy_and_damage_conjugate_hand_values():
    """psi_plty = beta_d/2 (phi - kappa)^2 = 500 * 0.2^2 = 20 and
    d Psi / d phi = beta_d (phi - kappa) = 200 at phi = 0.3, kappa = 0.1
    (-200 at phi = 0.1, kappa = 0.3)."""
    mat = _mat()
    E, _ = _energy(mat)
    F, g = _diag_state()
    k = torch.tensor([0.1], dtype=DT)
    for phi_v, dpsi in ((0.3, 200.0), (-0.1, -200.0)):
        phi = torch.tensor([phi_v], dtype=DT, requires_grad=True)
        psi = cm.free_energy(F, phi, g, k, E, mat)
        ref = cm.free_energy(F, k.clone(), g, k, E, mat)
        assert abs(float(psi - ref) - 20.0) < 1e-10
        (d,) = torch.autograd.grad(psi.sum(), phi)
        assert abs(float(d) - dpsi) < 1e-10


def test_nonlocal_flux_hand_value_diagonal_stretch():
    """Y_vec = c_d C^-1 g = 2.5 (0.3/4, -0.7/0.25, 1.1/1.5625) = (0.1875, -7.0, 1.76)."""
    mat = _mat()
    E, _ = _energy(mat)
    F, g = _diag_state()
    g = g.clone().requires_grad_(True)
    k = torch.tensor([0.25], dtype=DT)
    psi = cm.free_energy(F, k.clone(), g, k, E, mat)
    (Y,) = torch.autograd.grad(psi.sum(), g)
    assert np.allclose(Y[0].numpy(), [0.1875, -7.0, 1.76], rtol=0, atol=1e-13)


def test_gradient_term_stress_hand_values_diagonal_stretch():
    """d psi_grad / dF = -c_d (F C^-1 g) (x) (C^-1 g); for diagonal F,
    F C^-1 g = (g_i / lambda_i) = (0.15, -1.4, 0.88) and C^-1 g = (g_i / lambda_i^2)
    = (0.075, -2.8, 0.704), so e.g. P_11 = -2.5 * 0.15 * 0.075 = -0.028125,
    P_12 = -2.5 * 0.15 * (-2.8) = 1.05, P_32 = -2.5 * 0.88 * (-2.8) = 6.16."""
    mat = _mat()
    E, _ = _energy(mat)
    F, g = _diag_state()
    F = F.clone().requires_grad_(True)
    k = torch.tensor([0.25], dtype=DT)
    (P1,) = torch.autograd.grad(cm.free_energy(F, k.clone(), g, k, E, mat).sum(), F)
    (P0,) = torch.autograd.grad(cm.free_energy(F, k.clone(), torch.zeros_like(g), k, E, mat).sum(), F)
    Pg = (P1 - P0)[0].numpy()
    a = np.array([0.15, -1.4, 0.88])
    b = np.array([0.075, -2.8, 0.704])
    assert np.allclose(Pg, -C_D * np.outer(a, b), rtol=0, atol=1e-12)
    assert abs(Pg[0, 0] + 0.028125) < 1e-13 and abs(Pg[0, 1] - 1.05) < 1e-12 and abs(Pg[2, 1] - 6.16) < 1e-12


def test_gradient_term_with_sheared_deformation_against_explicit_inverse():
    """A general (sheared, rotated) F: psi_grad, Y_vec and the stress part against
    c_d/2 g.inv(C).g, c_d inv(C) g and -c_d (F inv(C) g) (x) (inv(C) g) with
    C inverted by numpy."""
    mat = _mat()
    E, _ = _energy(mat)
    rng = np.random.default_rng(11)
    for _ in range(4):
        Fn = np.eye(3) + np.array([[0.0, 0.4, 0.0], [0.0, 0.0, -0.3], [0.2, 0.0, 0.1]]) \
            + 0.1 * rng.standard_normal((3, 3))
        gn = rng.standard_normal(3)
        Ci = np.linalg.inv(Fn.T @ Fn)
        F = torch.tensor(Fn, dtype=DT)[None].requires_grad_(True)
        g = torch.tensor(gn, dtype=DT)[None].requires_grad_(True)
        k = torch.tensor([0.25], dtype=DT)
        psi1 = cm.free_energy(F, k.clone(), g, k, E, mat)
        psi0 = cm.free_energy(F, k.clone(), torch.zeros_like(g), k, E, mat)
        assert abs(float(psi1 - psi0) - 0.5 * C_D * gn @ Ci @ gn) < 1e-11 * max(1.0, abs(float(psi1)))
        P1, Y = torch.autograd.grad(psi1.sum(), (F, g))
        (P0,) = torch.autograd.grad(psi0.sum(), F)
        assert np.allclose(Y[0].numpy(), C_D * Ci @ gn, rtol=1e-12, atol=1e-12)
        assert np.allclose((P1 - P0)[0].numpy(), -C_D * np.outer(Fn @ Ci @ gn, Ci @ gn), rtol=1e-11,
                           atol=1e-11)


def test_qp_response_conjugates_at_an_elastic_point():
    """The per-point conjugates that the residual integrates (Pz = (P, dPsi/dphi,
    Y_vec) of qp_response) at an elastic point (phi < kappa_n makes the driving
    force negative, so kappa stays): dPsi/dphi = beta_d (phi - kappa_n) =
    1000 * (0.1 - 0.3) = -200 exactly, and Y_vec = (0.1875, -7.0, 1.76)."""
    mat = _mat()
    E, c = _energy(mat)
    Y = cm.Yield(torch.tensor(c.theta_y), c.yield_)
    z = torch.zeros(1, 13, dtype=DT)
    z[0, :9] = torch.diag(torch.tensor(LAM, dtype=DT)).reshape(9)
    z[0, 9] = 0.1
    z[0, 10:13] = torch.tensor(G, dtype=DT)
    kn = torch.tensor([0.3], dtype=DT)
    Pz, D, kap, yielded = cm.qp_response(z, kn, E, Y, mat, 3, tangent=True)
    assert not bool(yielded[0]) and float(kap[0]) == 0.3
    assert abs(float(Pz[0, 9]) + 200.0) < 1e-10
    assert np.allclose(Pz[0, 10:13].numpy(), [0.1875, -7.0, 1.76], rtol=0, atol=1e-12)
    # elastic point: D's damage block is beta_d on the phi diagonal and c_d C^-1 on
    # the gradient block (diag(2.5/4, 2.5/0.25, 2.5/1.5625) = diag(0.625, 10, 1.6))
    assert abs(float(D[0, 9, 9]) - BETA) < 1e-9
    assert np.allclose(D[0, 10:13, 10:13].numpy(), np.diag([0.625, 10.0, 1.6]), rtol=0, atol=1e-12)
    assert np.allclose(D[0, 9, 10:13].numpy(), 0.0, atol=1e-14)


def test_plane_strain_gradient_term_hand_value():
    """2-D plane strain: F = diag(l1, l2, 1), g = (g1, g2, 0); psi_grad =
    c_d/2 (g1^2/l1^2 + g2^2/l2^2) = 1.25 (0.0225 + 1.96) = 2.478125 for
    l = (2, 0.5), g = (0.3, -0.7)."""
    mat = _mat()
    E, c = _energy(mat)
    z = torch.tensor([[2.0, 0.0, 0.0, 0.5, 0.25, 0.3, -0.7]], dtype=DT)
    F, phi, g = cm.fields_from_z(z, 2)
    k = torch.tensor([0.25], dtype=DT)
    psi1 = cm.free_energy(F, phi, g, k, E, mat)
    psi0 = cm.free_energy(F, phi, torch.zeros_like(g), k, E, mat)
    assert abs(float(psi1 - psi0) - 2.478125) < 1e-12
