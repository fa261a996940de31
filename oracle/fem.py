"""Element residual, consistent tangent and global assembly (oracle; test
infrastructure only).

Follows Sec. 3.1 (Table 1 and the residual equations):
  F_q = I + sum_a u_a (x) grad N_a(X_q),  phi_q = sum_a N_a phi_a,
  grad phi_q = sum_a phi_a grad N_a,
  r_u,a   = sum_q P_q grad N_a J_q w_q,
  R_phi,a = sum_q (Y_q . grad N_a - Y_q N_a) J_q w_q,
and the monolithic tangent (Sec. 3.2): K_e = sum_q J_q w_q B^T D B where B
maps element dofs to z = (F, phi, grad phi) and D = dPz/dz includes the
history update.  Quadrature is 2x2 / 2x2x2 Gauss at +-1/sqrt(3), weight 1;
Q4 elements are plane strain with unit thickness.

The global matrix is a scipy CSR matrix whose pattern the oracle builds by
summing a COO list (every (dim+1)^2 block of every node pair that shares an
element), independently of the GPU library's pattern builder.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp
import torch

from . import constitutive as cm

DT = torch.float64
GP = 1.0 / math.sqrt(3.0)
_Q4 = np.array([[-1, -1], [1, -1], [1, 1], [-1, 1]], np.float64)
_H8 = np.array([[-1, -1, -1], [1, -1, -1], [1, 1, -1], [-1, 1, -1],
                [-1, -1, 1], [1, -1, 1], [1, 1, 1], [-1, 1, 1]], np.float64)


def reference_nodes(dim):
    return _Q4 if dim == 2 else _H8


def shape_at(dim, xi):
    """Multilinear shape functions and natural derivatives at points xi [Q, dim].
    N_a = prod_d (1 + xi_a,d xi_d)/2."""
    nodes = reference_nodes(dim)
    Q, nen = xi.shape[0], nodes.shape[0]
    N = np.ones((Q, nen))
    dN = np.ones((Q, nen, dim))
    for d in range(dim):
        f = 0.5 * (1.0 + nodes[None, :, d] * xi[:, None, d])
        N *= f
        for k in range(dim):
            dN[:, :, k] *= (0.5 * nodes[None, :, d]) if k == d else f
    return N, dN


def gauss_points(dim):
    """Quadrature point q sits at the natural coordinates of node q / sqrt(3)."""
    return reference_nodes(dim) * GP


class Geometry:
    """Per-element, per-qp shape data: N [Q, nen], G = grad_X N [E, Q, nen, dim],
    Jw = det(dX/dxi) * w [E, Q]."""

    def __init__(self, mesh, elems=None):
        dim = mesh.dim
        self.dim = dim
        self.elems = np.arange(mesh.n_elems) if elems is None else np.asarray(elems)
        conn = mesh.conn[self.elems]
        N, dN = shape_at(dim, gauss_points(dim))
        Xe = np.transpose(mesh.X[:, conn], (1, 2, 0))                 # [E, nen, dim]
        Jx = np.einsum("ead,qak->eqdk", Xe, dN)                       # dX_d/dxi_k
        Jinv = np.linalg.inv(Jx)
        G = np.einsum("eqkd,qak->eqad", Jinv, dN)                     # dN_a/dX_d
        self.N = torch.tensor(N, dtype=DT)
        self.G = torch.tensor(G, dtype=DT)
        self.Jw = torch.tensor(np.linalg.det(Jx), dtype=DT)
        self.conn = conn
        nd = dim + 1
        self.edofs = (conn[:, :, None].astype(np.int64) * nd + np.arange(nd)).reshape(len(conn), -1)


def b_matrix(geo):
    """B[e, q, z, k]: derivative of the qp state z w.r.t. element dof k
    (dofs ordered node-major, components u_1..u_dim then phi)."""
    dim = geo.dim
    E, Q, nen, _ = geo.G.shape
    nd = dim + 1
    nz = cm.nz_of(dim)
    B = torch.zeros(E, Q, nz, nen, nd, dtype=DT)
    for i in range(dim):
        for Jd in range(dim):
            zi = i * 3 + Jd if dim == 3 else i * 2 + Jd
            B[:, :, zi, :, i] = geo.G[:, :, :, Jd]
    iphi = 9 if dim == 3 else 4
    B[:, :, iphi, :, dim] = geo.N[None, :, :].expand(E, Q, nen)
    for Jd in range(dim):
        B[:, :, iphi + 1 + Jd, :, dim] = geo.G[:, :, :, Jd]
    return B.reshape(E, Q, nz, nen * nd)


def z_reference(dim, E, Q):
    nz = cm.nz_of(dim)
    z0 = torch.zeros(E, Q, nz, dtype=DT)
    if dim == 3:
        for i in range(3):
            z0[:, :, 4 * i] = 1.0
    else:
        z0[:, :, 0] = 1.0
        z0[:, :, 3] = 1.0
    return z0


def dof_vector(u, phi):
    """Interleave SoA nodal fields into the node-major dof vector."""
    u = np.asarray(u)
    return np.concatenate([u.T, np.asarray(phi)[:, None]], 1).ravel()


def split_dofs(d, dim):
    d = np.asarray(d).reshape(-1, dim + 1)
    return d[:, :dim].T.copy(), d[:, dim].copy()


class Model:
    """Material + networks built from raw parameter tensors.  A network spec with
    no hidden layer selects the closed-form model of Sec. 4.1 instead: the
    compressible Neo-Hooke energy, and G = identity for the yield function."""

    def __init__(self, case, theta_e=None, theta_y=None):
        self.mat = case.material
        te = torch.as_tensor(case.theta_e if theta_e is None else theta_e, dtype=DT)
        ty = torch.as_tensor(case.theta_y if theta_y is None else theta_y, dtype=DT)
        self.theta_e, self.theta_y = te, ty
        if case.energy.n_hidden == 0:
            self.energy = cm.NeoHooke(self.mat)
        else:
            self.energy = cm.Energy(te, case.energy, self.mat)
        if case.yield_.n_hidden == 0:
            self.yld = cm.IdentityYield()
        else:
            self.yld = cm.Yield(ty, case.yield_)


def element_response(model, mesh, d, kappa_n, elems=None, tangent=True,
                     d_torch=None, kappa_torch=None, create_graph=False, update_history=True):
    """Element residuals R_e [E, nd*nen], tangents K_e [E, nd*nen, nd*nen]
    (None if not requested) and kappa_{n+1} [E, Q] for the listed elements."""
    geo = Geometry(mesh, elems)
    E, Q = geo.Jw.shape
    B = b_matrix(geo)
    if d_torch is None:
        de = torch.tensor(np.asarray(d)[geo.edofs], dtype=DT)
    else:
        de = d_torch[torch.as_tensor(geo.edofs)]
    if kappa_torch is None:
        kn = torch.tensor(np.asarray(kappa_n)[geo.elems], dtype=DT).reshape(-1)
    else:
        kn = kappa_torch.reshape(-1, Q)[torch.as_tensor(geo.elems)].reshape(-1)
    z = z_reference(mesh.dim, E, Q) + torch.einsum("eqzk,ek->eqz", B, de)
    Pz, D, kap, yielded = cm.qp_response(z.reshape(E * Q, -1), kn, model.energy, model.yld,
                                         model.mat, mesh.dim, tangent=tangent,
                                         create_graph=create_graph, update_history=update_history)
    nz = Pz.shape[1]
    Pz = Pz.reshape(E, Q, nz)
    Re = torch.einsum("eq,eqzk,eqz->ek", geo.Jw, B, Pz)
    Ke = None
    if tangent:
        D = D.reshape(E, Q, nz, nz)
        Ke = torch.einsum("eq,eqzk,eqzy,eqyl->ekl", geo.Jw, B, D, B)
    return geo, Re, Ke, kap.reshape(E, Q), yielded.reshape(E, Q)


def assemble(model, mesh, d, kappa_n, tangent=True, chunk=4096, update_history=True):
    """Global residual R [ndof], tangent K (scipy CSR, or None) and
    kappa_trial [n_elems, nqp] for dof vector d and history kappa_n
    (update_history=False: kappa held at kappa_n, see qp_response)."""
    ndof = mesh.ndof
    R = np.zeros(ndof)
    kt = np.zeros((mesh.n_elems, mesh.nqp))
    rows, cols, vals = [], [], []
    for s in range(0, mesh.n_elems, chunk):
        el = np.arange(s, min(mesh.n_elems, s + chunk))
        geo, Re, Ke, kap, _ = element_response(model, mesh, d, kappa_n, el, tangent,
                                               update_history=update_history)
        np.add.at(R, geo.edofs.ravel(), Re.numpy().ravel())
        kt[el] = kap.numpy()
        if tangent:
            nde = geo.edofs.shape[1]
            rows.append(np.repeat(geo.edofs, nde, axis=1).ravel())
            cols.append(np.tile(geo.edofs, (1, nde)).ravel())
            vals.append(Ke.numpy().ravel())
    K = None
    if tangent:
        K = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(ndof, ndof)).tocsr()
        K.sum_duplicates()
        K.sort_indices()
    return R, K, kt


def residual_torch(model, mesh, d_t, kappa_t):
    """Differentiable global residual and kappa_{n+1} as torch tensors of the
    dof vector d_t, the history kappa_t [n_elems*nqp] and the parameters held
    by `model` (used by the adjoint)."""
    geo, Re, _, kap, _ = element_response(model, mesh, None, None, None, tangent=False,
                                          d_torch=d_t, kappa_torch=kappa_t, create_graph=True)
    R = torch.zeros(mesh.ndof, dtype=DT).index_add(0, torch.as_tensor(geo.edofs.ravel()),
                                                  Re.reshape(-1))
    return R, kap.reshape(-1)


def energy_total(model, mesh, d, kappa):
    """Discrete potential Pi_h = sum_e sum_q Psi J w at fixed history (Eq.
    total_potential_energy without external loads); used by the tests."""
    geo = Geometry(mesh)
    E, Q = geo.Jw.shape
    B = b_matrix(geo)
    de = torch.tensor(np.asarray(d)[geo.edofs], dtype=DT)
    z = z_reference(mesh.dim, E, Q) + torch.einsum("eqzk,ek->eqz", B, de)
    F, phi, g = cm.fields_from_z(z.reshape(E * Q, -1), mesh.dim)
    k = torch.tensor(np.asarray(kappa), dtype=DT).reshape(-1)
    psi = cm.free_energy(F, phi, g, k, model.energy, model.mat)
    return float((psi.reshape(E, Q) * geo.Jw).sum())
