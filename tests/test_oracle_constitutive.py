"""Pins of the oracle's constitutive layer against facts the paper and the
mathematics fix (not against the oracle's own formulas)."""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import constitutive as cm
from oracle import fem
from oracle.icnn import ICNN, n_params, softplus

DT = torch.float64


def rand_F(rng, B, scale=0.15):
    return torch.tensor(np.eye(3) + scale * rng.standard_normal((B, 3, 3)), dtype=DT)


def rotation(rng):
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return torch.tensor(q, dtype=DT)


# ------------------------------------------------------------------ invariants
def test_invariants_of_diagonal_stretch_match_hand_values():
    # F = diag(2, 1, 1): C = diag(4, 1, 1), I1 = 6, I2 = 4 + 4 + 1 = 9, J = 2
    F = torch.diag(torch.tensor([2.0, 1.0, 1.0], dtype=DT))[None]
    _, I1, I2, I3, J = cm.invariants(F)
    assert float(I1) == 6.0 and float(I2) == 9.0 and float(I3) == 4.0 and float(J) == 2.0
    x = cm.icnn_inputs(F)[0]
    assert abs(float(x[0]) - (6.0 * 2.0 ** (-2.0 / 3.0) - 3.0)) < 1e-15
    assert abs(float(x[1]) - (729.0 / 144.0 - 3.0)) < 1e-14
    assert float(x[2]) == 1.0


def test_isochoric_inputs_vanish_under_dilation_and_rotation():
    rng = np.random.default_rng(0)
    Q = rotation(rng)
    for lam in (0.7, 1.0, 1.3):
        x = cm.icnn_inputs((lam * Q)[None])[0]
        assert abs(float(x[0])) < 1e-14 and abs(float(x[1])) < 1e-13
        assert abs(float(x[2]) - (lam ** 3 - 1.0)) < 1e-14


def test_invariant_derivatives_match_eq_dd1():
    """dI1G/dC and dI2G/dC of Eq. dd_1 (4th and 5th rows), via dx/dF = 2 F dx/dC."""
    rng = np.random.default_rng(1)
    F = rand_F(rng, 6).requires_grad_(True)
    x = cm.icnn_inputs(F)
    C = F.transpose(1, 2) @ F
    Ci = torch.linalg.inv(C).detach()
    _, I1, I2, I3, _ = [t.detach() if torch.is_tensor(t) else t for t in cm.invariants(F)]
    I = torch.eye(3, dtype=DT)
    dI1G_dC = I3[:, None, None] ** (-1.0 / 3.0) * (I - I1[:, None, None] / 3.0 * Ci)
    dI2G_dC = (I2 ** 2 / (9.0 * I3 ** 2))[:, None, None] * (
        3.0 * I1[:, None, None] * I - 3.0 * C.detach() - 2.0 * I2[:, None, None] * Ci)
    for k, ref in ((0, dI1G_dC), (1, dI2G_dC)):
        (g,) = torch.autograd.grad(x[:, k].sum(), F, retain_graph=True)
        assert torch.allclose(g, 2.0 * F.detach() @ ref, rtol=1e-12, atol=1e-12)


# ------------------------------------------------------------------ networks
@pytest.mark.parametrize("cfg", [1, 2, 3, 4, 5])
def test_icnn_convex_and_yield_increasing(cfg):
    c = W.make_case(cfg, n=2, nz=1)
    net = ICNN(torch.tensor(c.theta_e), 3, c.energy.width, c.energy.n_hidden, c.energy.monotone_mask)
    for Wz, _, _ in net.hidden:
        assert bool((Wz >= 0).all())
    assert bool((net.wz >= 0).all())
    rng = np.random.default_rng(cfg)
    x = torch.tensor(rng.uniform(-0.3, 0.6, (16, 3)), dtype=DT, requires_grad=True)
    (g,) = torch.autograd.grad(net(x).sum(), x, create_graph=True)
    H = torch.stack([torch.autograd.grad(g[:, i].sum(), x, retain_graph=True)[0] for i in range(3)], 1)
    ev = torch.linalg.eigvalsh(H.detach())
    assert float(ev.min()) >= -1e-12 * float(ev.abs().max())
    # non-decreasing in the polyconvex invariants
    assert bool((g[:, :2] >= 0).all())
    y = cm.Yield(torch.tensor(c.theta_y), c.yield_)
    q = torch.linspace(-50, 50, 101, dtype=DT, requires_grad=True)
    Nq = y(q)
    (dq,) = torch.autograd.grad(Nq.sum(), q)
    assert bool((dq >= 0).all())
    assert float(y(torch.zeros(1, dtype=DT))[0]) == 0.0


def test_icnn_reduces_to_linear_map_when_convex_weights_vanish():
    """softplus(-800) is exactly 0 in FP64: the network collapses to wx.x + b."""
    spec = W.NetSpec(3, 8, 3, 3)
    theta = torch.full((n_params(3, 8, 3),), -800.0, dtype=DT)
    net0 = ICNN(theta, 3, 8, 3, 3)
    off = n_params(3, 8, 3) - 4
    theta[off:off + 3] = torch.tensor([0.3, 0.2, -0.7], dtype=DT)  # wx (x1, x2 softplus'd)
    theta[off + 3] = 1.25
    net = ICNN(theta, 3, 8, 3, 3)
    assert float(softplus(torch.tensor(-800.0, dtype=DT))) == 0.0
    x = torch.tensor(np.random.default_rng(2).standard_normal((5, 3)), dtype=DT)
    wx = torch.tensor([math.log1p(math.exp(0.3)), math.log1p(math.exp(0.2)), -0.7], dtype=DT)
    assert torch.allclose(net(x), x @ wx + 1.25, rtol=0, atol=1e-14)
    assert spec.n_params == n_params(3, 8, 3) and net0.b_out.numel() == 1


# ------------------------------------------------------------------ energy
def _mat():
    return dict(W.MATERIAL)


@pytest.mark.parametrize("cfg", [1, 3, 4])
def test_reference_state_stress_and_energy_vanish(cfg):
    """Energy and stress normality at C = I (Sec. 4.2.1, sentence after Eq. dd_1)."""
    c = W.make_case(cfg, n=2)
    E = cm.Energy(torch.tensor(c.theta_e), c.energy, c.material)
    F = torch.eye(3, dtype=DT)[None].clone().requires_grad_(True)
    psi = E(F)
    (P,) = torch.autograd.grad(psi.sum(), F)
    assert abs(float(psi)) < 1e-13 * max(1.0, float(E.N0.abs()) * c.material["mu_e"])
    assert float(P.abs().max()) < 1e-12 * max(1.0, float(E.N0.abs()) * c.material["mu_e"])


def test_linear_network_gives_textbook_isochoric_neo_hooke_stress():
    """With the network collapsed to N = x1/2 + a3 x3 (+b), psi_e is the decoupled
    compressible Neo-Hooke energy mu/2 (I1G - 3) + lambda (J + 1/J - 2)^2, whose
    first Piola stress is mu J^(-2/3) (F - I1/3 F^-T) + lambda psi_vol'(J) J F^-T."""
    n_in, H, L = 3, 4, 2
    theta = torch.full((n_params(n_in, H, L),), -800.0, dtype=DT)
    off = n_params(n_in, H, L) - 4
    theta[off] = math.log(math.expm1(0.5))       # softplus -> 0.5 exactly (to rounding)
    theta[off + 2] = 0.37                        # raw J-1 pass-through weight
    spec = W.NetSpec(n_in, H, L, 3)
    mat = _mat()
    E = cm.Energy(theta, spec, mat)
    rng = np.random.default_rng(3)
    F = rand_F(rng, 8).requires_grad_(True)
    (P,) = torch.autograd.grad(E(F).sum(), F)
    Fd = F.detach()
    J = cm.det3(Fd)
    Fit = torch.linalg.inv(Fd).transpose(1, 2)
    I1 = (Fd * Fd).sum((1, 2))
    half = float(softplus(theta[off:off + 1]))
    dvol = 2.0 * (J + 1.0 / J - 2.0) * (1.0 - J ** -2)
    Pref = (mat["mu_e"] * 2.0 * half * J[:, None, None] ** (-2.0 / 3.0) * (Fd - I1[:, None, None] / 3.0 * Fit)
            + mat["lambda_e"] * (dvol * J)[:, None, None] * Fit)
    assert torch.allclose(P, Pref, rtol=1e-12, atol=1e-12)


def test_energy_objective_and_stress_rotates():
    rng = np.random.default_rng(4)
    c = W.make_case(5, n=2)
    E = cm.Energy(torch.tensor(c.theta_e), c.energy, c.material)
    F = rand_F(rng, 5).requires_grad_(True)
    Q = rotation(rng)
    QF = (Q[None] @ F.detach()).requires_grad_(True)
    psi, psiq = E(F), E(QF)
    assert torch.allclose(psi, psiq, rtol=1e-12, atol=1e-12)
    (P,) = torch.autograd.grad(psi.sum(), F)
    (PQ,) = torch.autograd.grad(psiq.sum(), QF)
    assert torch.allclose(PQ, Q[None] @ P, rtol=1e-11, atol=1e-11)


# ------------------------------------------------------------------ local update
def _ostwald_yield(spec_width=4):
    """Yield network with N^ = identity: convex weights vanish, wx = 1."""
    spec = W.NetSpec(1, spec_width, 1, 1)
    th = torch.full((spec.n_params,), -800.0, dtype=DT)
    th[-2] = math.log(math.e - 1.0)   # softplus -> 1
    th[-1] = 0.3                      # bias, removed by N^
    return cm.Yield(th, spec)


def test_local_model_history_independent_of_eta_and_kappa_d():
    """beta_d = 0 (no nonlocal coupling): kappa_{n+1} = max(kappa_n, N^(psi_e)) for any
    eta_d, kappa_d -- the single-element observation of Sec. 5.1."""
    c = W.make_case(1, n=2)
    yld = cm.Yield(torch.tensor(c.theta_y), c.yield_)
    rng = np.random.default_rng(5)
    pe = torch.tensor(rng.uniform(0, 3, 50), dtype=DT)
    phi = torch.tensor(rng.uniform(0, 1, 50), dtype=DT)
    kn = torch.tensor(rng.uniform(0, 6, 50), dtype=DT)
    ref = torch.maximum(kn, yld(pe))
    for eta, kd in ((1.0, 0.0), (10.0, 1.0), (100.0, 2.0)):
        mat = dict(_mat(), beta_d=0.0, eta_d=eta, kappa_d=kd)
        k, y, _ = cm.local_update(pe, phi, kn, yld, mat)
        assert torch.allclose(k, ref, rtol=1e-15, atol=1e-15)


def test_ostwald_loading_function_root():
    """With N^ = id the yield condition is Eq. ostwald_potential:
    psi + gamma beta (phi - kappa)/(eta f_d) - kappa = 0 at yielding points."""
    yld = _ostwald_yield()
    rng = np.random.default_rng(6)
    mat = dict(_mat(), eta_d=0.5, beta_d=3.0)
    pe = torch.tensor(rng.uniform(0, 2, 64), dtype=DT)
    phi = torch.tensor(rng.uniform(0, 1, 64), dtype=DT)
    kn = torch.tensor(rng.uniform(0, 0.5, 64), dtype=DT)
    k, y, _ = cm.local_update(pe, phi, kn, yld, mat)
    fd = torch.exp(-mat["eta_d"] * torch.clamp(k - mat["kappa_d"], min=0))
    phi_d = pe + mat["beta_d"] * (phi - k) / (mat["eta_d"] * fd) - k
    assert bool(y.any()) and bool((~y).any())
    assert float(phi_d[y].abs().max()) < 1e-12
    assert bool((k >= kn).all()) and bool((k[~y] == kn[~y]).all())
    # elastic points are inside the yield surface
    fdn = torch.exp(-mat["eta_d"] * torch.clamp(kn - mat["kappa_d"], min=0))
    assert bool((pe + mat["beta_d"] * (phi - kn) / (mat["eta_d"] * fdn) - kn)[~y].le(0).all())


def test_seeded_local_update_kkt():
    """KKT of Eq. dd_7: h(kappa_{n+1}) = 0 and Delta lambda >= 0 where yielding."""
    c = W.make_case(3, n=2)
    yld = cm.Yield(torch.tensor(c.theta_y), c.yield_)
    rng = np.random.default_rng(7)
    mat = c.material
    pe = torch.tensor(rng.uniform(0, 5, 200), dtype=DT)
    phi = torch.tensor(rng.uniform(0, 0.3, 200), dtype=DT)
    kn = torch.tensor(rng.uniform(0, 0.2, 200), dtype=DT)
    k, y, _ = cm.local_update(pe, phi, kn, yld, mat)
    h = cm.h_yield(k, pe, phi, yld, mat)
    q = cm.drive_q(pe, phi, k, mat).clone().requires_grad_(True)
    (dN,) = torch.autograd.grad(yld(q).sum(), q)
    dlam = (k - kn) / dN
    # |h| is at the rounding level of its slope times one ulp of kappa
    slope = mat["beta_d"] / (mat["eta_d"]) * dN * 2.0
    assert bool((h[y].abs() <= slope[y] * 4e-16 * k[y].abs().clamp(min=1)).all())
    assert bool((dlam[y] >= 0).all()) and bool(y.any())


# ------------------------------------------------------------------ conjugates / tangent
def _qp_batch(cfg, B, seed):
    c = W.make_case(cfg, n=2)
    m = fem.Model(c)
    rng = np.random.default_rng(seed)
    dim = c.mesh.dim
    nz = cm.nz_of(dim)
    z = np.zeros((B, nz))
    if dim == 3:
        z[:, :9] = (np.eye(3) + 0.08 * rng.standard_normal((B, 3, 3))).reshape(B, 9)
        z[:, 9] = rng.uniform(0, 0.2, B)
        z[:, 10:] = 0.3 * rng.standard_normal((B, 3))
    else:
        F2 = np.eye(2) + 0.08 * rng.standard_normal((B, 2, 2))
        z[:, :4] = F2.reshape(B, 4)
        z[:, 4] = rng.uniform(0, 0.2, B)
        z[:, 5:] = 0.3 * rng.standard_normal((B, 2))
    kn = rng.uniform(0, 0.1, B)
    return c, m, torch.tensor(z, dtype=DT), torch.tensor(kn, dtype=DT)


@pytest.mark.parametrize("cfg", [1, 2])
def test_conjugates_are_fd_derivatives_of_free_energy(cfg):
    """(P, -Y, Y_vec) = central differences of Psi at frozen kappa (Eqs. PK1_stress_calc,
    nonlocal_conjugate_calc)."""
    c, m, z, kn = _qp_batch(cfg, 12, 10 + cfg)
    dim = c.mesh.dim
    Pz, _, kap, _ = cm.qp_response(z, kn, m.energy, m.yld, m.mat, dim, tangent=False)

    def psi(zz):
        F, phi, g = cm.fields_from_z(zz, dim)
        return cm.free_energy(F, phi, g, kap, m.energy, m.mat)

    h = 1e-6
    for j in range(z.shape[1]):
        e = torch.zeros_like(z)
        e[:, j] = h
        fd = (psi(z + e) - psi(z - e)) / (2 * h)
        scale = float(Pz.abs().max())
        assert float((fd - Pz[:, j]).abs().max()) < 1e-7 * scale


@pytest.mark.parametrize("cfg", [1, 2])
def test_tangent_is_fd_derivative_with_history_update(cfg):
    """D = dPz/dz with kappa_{n+1}(z) re-solved at every perturbed point (monolithic
    tangent, Sec. 3.2).  Points within 10 FD steps of the f_d kink are skipped."""
    c, m, z, kn = _qp_batch(cfg, 12, 20 + cfg)
    dim = c.mesh.dim
    Pz, D, kap, y = cm.qp_response(z, kn, m.energy, m.yld, m.mat, dim, tangent=True)
    h = 1e-6
    keep = (kap - m.mat["kappa_d"]).abs() > 1e-4
    assert bool(y.any())
    for j in range(z.shape[1]):
        e = torch.zeros_like(z)
        e[:, j] = h
        Pp = cm.qp_response(z + e, kn, m.energy, m.yld, m.mat, dim, tangent=False)[0]
        Pm = cm.qp_response(z - e, kn, m.energy, m.yld, m.mat, dim, tangent=False)[0]
        fd = (Pp - Pm) / (2 * h)
        scale = float(D.abs().max())
        assert float((fd - D[:, :, j])[keep].abs().max()) < 2e-6 * scale


def test_tangent_symmetric_above_threshold():
    """With gamma_d = 1 and kappa > kappa_d the rank-one history term is symmetric."""
    c, m, z, kn = _qp_batch(2, 16, 31)
    Pz, D, kap, y = cm.qp_response(z, kn + 0.2, m.energy, m.yld, m.mat, 3, tangent=True)
    sel = kap > m.mat["kappa_d"]
    assert bool(sel.all())
    asym = (D - D.transpose(1, 2)).abs().amax((1, 2))
    assert float(asym.max()) < 1e-10 * float(D.abs().max())
