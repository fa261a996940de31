"""Per-quadrature-point constitutive response (oracle; test infrastructure only).

Free energy of the nonlocal data-driven model (Sec. 4.2.2, Eq. dd_3):

    Psi(F, phi, grad phi, kappa) = f_d(kappa) psi_e(C)
                                   + c_d/2 grad phi . C^-1 . grad phi
                                   + beta_d/2 (phi - kappa)^2

with the PANN elastic energy (Sec. 4.2.1, Eq. dd_0)

    psi_e = mu_e [N(x) - N(0) - n0 (J - 1)] + lambda_e (J + 1/J - 2)^2,
    x = (I1G - 3, I2G - 3, J - 1),  I1G = J^(-2/3) I1,  I2G = I2^3 / (9 J^4),

the degradation f_d = exp(-eta_d <kappa - kappa_d>_+) (Eq. degradation_function),
the driving force q = psi_e + gamma_d beta_d (phi - kappa) / (eta_d f_d)
(Eqs. q_q_loc_q_nloc and ostwald_potential) and the yield condition
N^_kappa(q) - kappa <= 0 with N^_kappa(q) = N_kappa(q) - N_kappa(0)
(Eqs. potential_function, Gq_NN, dd_7).

Readings (where the paper is silent or garbled):
* ICNN inputs are the paper's isochoric invariants shifted to vanish at
  C = I plus J - 1; the term -n0 (J - 1), n0 = dN/dx3 at x = 0, restores the
  stress normality S(C = I) = 0 that the paper states (Eq. dd_1 and the
  sentence after it) once J - 1 is an input.
* The stray lambda_e in the volumetric stress derivative of Eq. dd_1 is a
  typo; the energy above is differentiated as written in Eq. dd_0.
* The garbled yield argument of Eq. Gq_NN is read as G(q) = N^_kappa(q), so
  yielding implies q > 0 (non-negative dissipation).
* gamma_d = 1 (the value that the chain rule d kappa / d d = 1/(eta_d f_d)
  gives for q_nloc); eta_d f_d is used as the divisor also below kappa_d.
* The local problem (Eq. dd_7) is solved for kappa_{n+1} on the bracket
  [kappa_n, max(kappa_n, phi, N^_kappa(psi_e))], on which the residual
  h(kappa) = N^_kappa(q(kappa)) - kappa is strictly decreasing; h(kappa_n) <= 0
  is the elastic case.  Delta lambda follows from the first row of Eq. dd_7.
  The oracle solves it by bisection (exact to the last bit); the
  consistent sensitivities come from the implicit function theorem.
"""
from __future__ import annotations

import torch

from .icnn import ICNN

DT = torch.float64


# ---------------------------------------------------------------- kinematics
def det3(F):
    return (F[..., 0, 0] * (F[..., 1, 1] * F[..., 2, 2] - F[..., 1, 2] * F[..., 2, 1])
            - F[..., 0, 1] * (F[..., 1, 0] * F[..., 2, 2] - F[..., 1, 2] * F[..., 2, 0])
            + F[..., 0, 2] * (F[..., 1, 0] * F[..., 2, 1] - F[..., 1, 1] * F[..., 2, 0]))


def inv3(A):
    """Inverse of a batch of 3x3 matrices through the adjugate."""
    c = torch.stack([
        torch.stack([A[..., 1, 1] * A[..., 2, 2] - A[..., 1, 2] * A[..., 2, 1],
                     A[..., 0, 2] * A[..., 2, 1] - A[..., 0, 1] * A[..., 2, 2],
                     A[..., 0, 1] * A[..., 1, 2] - A[..., 0, 2] * A[..., 1, 1]], -1),
        torch.stack([A[..., 1, 2] * A[..., 2, 0] - A[..., 1, 0] * A[..., 2, 2],
                     A[..., 0, 0] * A[..., 2, 2] - A[..., 0, 2] * A[..., 2, 0],
                     A[..., 0, 2] * A[..., 1, 0] - A[..., 0, 0] * A[..., 1, 2]], -1),
        torch.stack([A[..., 1, 0] * A[..., 2, 1] - A[..., 1, 1] * A[..., 2, 0],
                     A[..., 0, 1] * A[..., 2, 0] - A[..., 0, 0] * A[..., 2, 1],
                     A[..., 0, 0] * A[..., 1, 1] - A[..., 0, 1] * A[..., 1, 0]], -1),
    ], -2)
    return c / det3(A)[..., None, None]


def invariants(F):
    """C = F^T F, I1 = tr C, I2 = tr cof C = (I1^2 - tr C^2)/2, I3 = det C, J = det F
    (Sec. 4.2.1, Eq. dd_0)."""
    C = F.transpose(-1, -2) @ F
    I1 = C.diagonal(dim1=-2, dim2=-1).sum(-1)
    I2 = 0.5 * (I1 * I1 - (C * C).sum((-1, -2)))
    I3 = det3(C)
    J = det3(F)
    return C, I1, I2, I3, J


def icnn_inputs(F):
    """x = (I1G - 3, I2G - 3, J - 1), I1G = J^(-2/3) I1, I2G = I2^3/(9 J^4) (Eq. dd_0)."""
    _, I1, I2, _, J = invariants(F)
    return torch.stack([J ** (-2.0 / 3.0) * I1 - 3.0, I2 ** 3 / (9.0 * J ** 4) - 3.0, J - 1.0], -1)


def fields_from_z(z, dim):
    """Unpack the per-qp state vector.

    3-D: z = (F row-major 9, phi, grad phi 3).  2-D plane strain:
    z = (F11, F12, F21, F22, phi, phi_,1, phi_,2) with F33 = 1 and no
    out-of-plane gradient.
    """
    B = z.shape[0]
    if dim == 3:
        return z[:, :9].reshape(B, 3, 3), z[:, 9], z[:, 10:13]
    zero, one = torch.zeros(B, dtype=z.dtype), torch.ones(B, dtype=z.dtype)
    F = torch.stack([torch.stack([z[:, 0], z[:, 1], zero], -1),
                     torch.stack([z[:, 2], z[:, 3], zero], -1),
                     torch.stack([zero, zero, one], -1)], -2)
    g = torch.stack([z[:, 5], z[:, 6], zero], -1)
    return F, z[:, 4], g


def nz_of(dim):
    return 13 if dim == 3 else 7


# ---------------------------------------------------------------- energies
class Energy:
    """psi_e(C) of Eq. dd_0 with an ICNN isochoric part (see module doc)."""

    def __init__(self, theta, spec, mat):
        self.net = ICNN(theta, spec.n_in, spec.width, spec.n_hidden, spec.monotone_mask)
        self.mu, self.lam = mat["mu_e"], mat["lambda_e"]
        with torch.enable_grad():
            x0 = torch.zeros(1, 3, dtype=DT, requires_grad=True)
            N0 = self.net(x0)
            (gx,) = torch.autograd.grad(N0.sum(), x0, create_graph=True)
        self.N0 = N0[0]
        self.n0 = gx[0, 2]

    def __call__(self, F):
        x = icnn_inputs(F)
        J = det3(F)
        vol = J + 1.0 / J - 2.0
        return self.mu * (self.net(x) - self.N0 - self.n0 * x[:, 2]) + self.lam * vol * vol


class Yield:
    """N^_kappa(q) = N_kappa(q) - N_kappa(0), an increasing function (Sec. 4.2.1)."""

    def __init__(self, theta, spec):
        self.net = ICNN(theta, spec.n_in, spec.width, spec.n_hidden, spec.monotone_mask)
        self.N0 = self.net(torch.zeros(1, 1, dtype=DT))[0]

    def __call__(self, q):
        return self.net(q[:, None]) - self.N0


class NeoHooke:
    """Closed-form compressible Neo-Hooke energy of Sec. 4.1:
    psi_NH = mu_e/2 (I1 - 3) - mu_e ln J + lambda_e/2 (ln J)^2 (mu_e, lambda_e the
    shear and bulk moduli of the undamaged material)."""

    def __init__(self, mat):
        self.mu, self.lam = mat["mu_e"], mat["lambda_e"]
        self.N0 = torch.zeros((), dtype=DT)
        self.n0 = torch.zeros((), dtype=DT)

    def __call__(self, F):
        _, I1, _, _, J = invariants(F)
        lnJ = torch.log(J)
        return 0.5 * self.mu * (I1 - 3.0) - self.mu * lnJ + 0.5 * self.lam * lnJ * lnJ


class IdentityYield:
    """G(q) = q: the yield function under which Eq. potential_function becomes the
    Ostwald loading function of Eq. ostwald_potential."""

    def __call__(self, q):
        return q * 1.0


def f_d(kappa, mat):
    """Degradation exp(-eta_d <kappa - kappa_d>_+) (Eq. degradation_function)."""
    return torch.exp(-mat["eta_d"] * torch.clamp(kappa - mat["kappa_d"], min=0.0))


def free_energy(F, phi, g, kappa, energy, mat):
    """Psi of Eq. dd_3 (gradient and penalty terms of the closed-form model,
    Sec. 4.1, reused unchanged by the data-driven model)."""
    C = F.transpose(-1, -2) @ F
    Ci = inv3(C)
    grad_term = 0.5 * mat["c_d"] * torch.einsum("bi,bij,bj->b", g, Ci, g)
    pen = 0.5 * mat["beta_d"] * (phi - kappa) ** 2
    return f_d(kappa, mat) * energy(F) + grad_term + pen


def drive_q(psi_e, phi, kappa, mat):
    """q = q_loc + q_nloc = psi_e + gamma_d beta_d (phi - kappa)/(eta_d f_d(kappa))
    (Eqs. q_q_loc_q_nloc, ostwald_potential)."""
    return psi_e + mat["gamma_d"] * mat["beta_d"] * (phi - kappa) / (mat["eta_d"] * f_d(kappa, mat))


def h_yield(kappa, psi_e, phi, yld, mat):
    """Yield residual N^_kappa(q(kappa)) - kappa (Eq. dd_7, second row)."""
    return yld(drive_q(psi_e, phi, kappa, mat)) - kappa


@torch.no_grad()
def local_update(psi_e, phi, kappa_n, yld, mat, max_iter=400):
    """kappa_{n+1} from the KKT system of Eq. dd_7 (see module doc for the
    bracket).  Returns (kappa_{n+1}, yielded mask, iterations used)."""
    yielded = h_yield(kappa_n, psi_e, phi, yld, mat) > 0
    lo = kappa_n.clone()
    hi = torch.maximum(torch.maximum(kappa_n, phi), yld(psi_e))
    done = ~yielded
    it = 0
    while not bool(done.all()) and it < max_iter:
        mid = 0.5 * (lo + hi)
        stuck = (mid <= lo) | (mid >= hi)
        done = done | stuck
        hm = h_yield(mid, psi_e, phi, yld, mat)
        up = (~done) & (hm > 0)
        dn = (~done) & (hm <= 0)
        lo = torch.where(up, mid, lo)
        hi = torch.where(dn, mid, hi)
        it += 1
    hl = h_yield(lo, psi_e, phi, yld, mat).abs()
    hh = h_yield(hi, psi_e, phi, yld, mat).abs()
    root = torch.where(hl <= hh, lo, hi)
    return torch.where(yielded, root, kappa_n), yielded, it


def kappa_of_z(z, kappa_star, yielded, kappa_n, energy, yld, mat, dim):
    """kappa_{n+1} as a differentiable function of (z, kappa_n, parameters).

    At yielding points it is kappa* - h(kappa*)/h_kappa(kappa*) with kappa*
    the converged root held constant, whose first derivatives are exactly the
    implicit-function sensitivities -h_(.)/h_kappa; at elastic points it is
    kappa_n.
    """
    F, phi, _ = fields_from_z(z, dim)
    pe = energy(F)
    k = kappa_star.detach().clone().requires_grad_(True)
    h = h_yield(k, pe, phi, yld, mat)
    (hk,) = torch.autograd.grad(h.sum(), k, create_graph=True)
    k_new = k.detach() - h / hk
    return torch.where(yielded, k_new, kappa_n)


def qp_response(z, kappa_n, energy, yld, mat, dim, tangent=True, create_graph=False, update_history=True):
    """Per-qp conjugates and consistent tangent.

    Returns (Pz, D, kappa_{n+1}, yielded):
      Pz = dPsi/dz at fixed kappa, evaluated at kappa_{n+1}: (P, -Y, Y_vec)
           = first Piola-Kirchhoff stress, d Psi / d phi, nonlocal flux
           (Eqs. PK1_stress_calc, nonlocal_conjugate_calc);
      D  = dPz/dz including the history update (monolithic scheme, Sec. 3.2),
           D[b, i, j] = d Pz_i / d z_j;  None when tangent is False.
    update_history=False holds kappa at kappa_n (the global solve of the
    staggered scheme, Sec. 3.2): no local update, no history sensitivities.
    """
    nz = nz_of(dim)
    with torch.no_grad():
        F0, phi0, _ = fields_from_z(z.detach(), dim)
        pe0 = energy(F0)
        if update_history:
            kstar, yielded, _ = local_update(pe0, phi0, kappa_n.detach(), yld, mat)
        else:
            kstar, yielded = kappa_n.detach().clone(), torch.zeros_like(kappa_n, dtype=torch.bool)
    with torch.enable_grad():
        zz = z if z.requires_grad else z.detach().clone().requires_grad_(True)
        ze = zz * 1.0
        kap = kappa_of_z(zz, kstar, yielded, kappa_n, energy, yld, mat, dim)
        F, phi, g = fields_from_z(ze, dim)
        psi = free_energy(F, phi, g, kap, energy, mat)
        (Pz,) = torch.autograd.grad(psi.sum(), ze, create_graph=tangent or create_graph)
        D = None
        if tangent:
            rows = []
            for j in range(nz):
                (r,) = torch.autograd.grad(Pz[:, j].sum(), zz, retain_graph=True,
                                           create_graph=create_graph)
                rows.append(r)
            D = torch.stack(rows, 1)
    if not create_graph:
        Pz = Pz.detach()
        kap = kap.detach()
    return Pz, D, kap, yielded
