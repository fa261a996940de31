"""Pins of the oracle's element / assembly / solver layers."""
import numpy as np
import pytest
import scipy.sparse as sp
import torch

import workloads as W
from oracle import constitutive as cm
from oracle import fem, solve

DT = torch.float64


@pytest.mark.parametrize("dim", [2, 3])
def test_shape_functions_partition_of_unity_and_reproduce_affine_fields(dim):
    mesh = W.q4_grid(3, 2, 1.5, 1.0) if dim == 2 else W.hex8_grid(2, 2, 1, 1.0, 1.2, 0.5)
    geo = fem.Geometry(mesh)
    assert torch.allclose(geo.N.sum(1), torch.ones(mesh.nqp, dtype=DT))
    assert float(geo.G.sum(2).abs().max()) < 1e-13
    rng = np.random.default_rng(0)
    A = rng.standard_normal((dim, dim))
    vals = A @ mesh.X                                  # affine field u = A X
    grad = torch.einsum("dea,eqak->eqdk", torch.tensor(vals[:, geo.conn]), geo.G)
    assert torch.allclose(grad, torch.tensor(A)[None, None].expand_as(grad), atol=1e-12)
    # quadrature integrates the volume exactly
    vol = 1.5 if dim == 2 else 1.0 * 1.2 * 0.5
    assert abs(float(geo.Jw.sum()) - vol) < 1e-13


def _elastic_state(cfg, n, seed, big_kappa=True):
    c = W.make_case(cfg, n=n, nz=1) if cfg in (2, 4) else W.make_case(cfg, n=n)
    rng = np.random.default_rng(seed)
    m = fem.Model(c)
    u = 0.05 * rng.standard_normal(c.mesh.X.shape)
    phi = rng.uniform(0.0, 0.2, c.mesh.n_nodes)
    kap = np.full((c.mesh.n_elems, c.mesh.nqp), 1.0 if big_kappa else 0.0)
    return c, m, fem.dof_vector(u, phi), kap


@pytest.mark.parametrize("cfg", [1, 2])
def test_residual_is_gradient_of_discrete_energy(cfg):
    """Elastic state (history above the yield surface): R = dPi_h/dd, Pi_h = sum Psi J w."""
    c, m, d, kap = _elastic_state(cfg, 2, 1)
    R, _, kt = fem.assemble(m, c.mesh, d, kap, tangent=False)
    assert np.array_equal(kt, kap)
    rng = np.random.default_rng(2)
    for j in rng.choice(c.mesh.ndof, 12, replace=False):
        h = 1e-6
        dp, dm = d.copy(), d.copy()
        dp[j] += h
        dm[j] -= h
        fd = (fem.energy_total(m, c.mesh, dp, kap) - fem.energy_total(m, c.mesh, dm, kap)) / (2 * h)
        assert abs(fd - R[j]) < 1e-7 * max(1.0, np.abs(R).max())


@pytest.mark.parametrize("cfg", [1, 2])
def test_tangent_is_fd_of_residual_including_history(cfg):
    c = W.make_case(cfg, n=2, nz=1) if cfg == 2 else W.make_case(cfg, n=2)
    rng = np.random.default_rng(3)
    m = fem.Model(c)
    u = 0.08 * rng.standard_normal(c.mesh.X.shape)
    phi = rng.uniform(0.0, 0.2, c.mesh.n_nodes)
    kap = rng.uniform(0.0, 0.1, (c.mesh.n_elems, c.mesh.nqp))
    d = fem.dof_vector(u, phi)
    R, K, kt = fem.assemble(m, c.mesh, d, kap)
    assert (kt > kap).any()
    near = np.abs(kt - c.material["kappa_d"]) < 1e-4
    assert not near.any()
    Kd = K.toarray()
    for j in rng.choice(c.mesh.ndof, 10, replace=False):
        h = 1e-6
        dp, dm = d.copy(), d.copy()
        dp[j] += h
        dm[j] -= h
        fd = (fem.assemble(m, c.mesh, dp, kap, tangent=False)[0]
              - fem.assemble(m, c.mesh, dm, kap, tangent=False)[0]) / (2 * h)
        assert np.abs(fd - Kd[:, j]).max() < 1e-6 * np.abs(Kd).max()


def test_csr_pattern_counts_match_mesh_adjacency():
    """nnz = (dim+1)^2 * number of node pairs sharing an element (21 609 for 16x16 Q4)."""
    c = W.make_case(1)
    _, K, _ = fem.assemble(fem.Model(c), c.mesh, fem.dof_vector(c.u, c.phi), c.kappa)
    assert K.nnz == 21609
    c3 = W.make_case(2, n=4, nz=2)
    pairs = set()
    for e in c3.mesh.conn:
        for a in e:
            for b in e:
                pairs.add((a, b))
    _, K3, _ = fem.assemble(fem.Model(c3), c3.mesh, fem.dof_vector(c3.u, c3.phi), c3.kappa)
    assert K3.nnz == 16 * len(pairs)


@pytest.mark.parametrize("cfg", [1, 2])
def test_patch_test_affine_field_uniform_damage(cfg):
    """Affine u, uniform phi = kappa (elastic): interior rows of R vanish and every qp
    sees the same stress."""
    c = W.make_case(cfg, n=3) if cfg == 1 else W.make_case(cfg, n=3, nz=3)
    m = fem.Model(c)
    dim = c.mesh.dim
    rng = np.random.default_rng(4)
    A = 0.1 * rng.standard_normal((dim, dim))
    u = A @ c.mesh.X
    phi = np.full(c.mesh.n_nodes, 0.05)
    kap = np.full((c.mesh.n_elems, c.mesh.nqp), 0.05)
    d = fem.dof_vector(u, phi)
    # make the point elastic: a history far above the yield surface keeps phi = kappa
    R, _, kt = fem.assemble(m, c.mesh, d, kap + 0.0, tangent=False)
    interior = np.setdiff1d(np.arange(c.mesh.n_nodes), W.boundary_nodes(c.mesh))
    rows = (interior[:, None] * (dim + 1) + np.arange(dim)).ravel()
    scale = np.abs(R).max()
    if (kt == kap).all():
        assert np.abs(R[rows]).max() < 1e-11 * max(1.0, scale)
    geo, Re, _, _, _ = fem.element_response(m, c.mesh, d, kap, tangent=False)
    assert scale > 0


def test_rotation_of_displacement_rotates_residual():
    c = W.make_case(2, n=2, nz=1)
    m = fem.Model(c)
    rng = np.random.default_rng(5)
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    Q = q * np.sign(np.diag(r))
    if np.linalg.det(Q) < 0:
        Q[:, 0] *= -1
    u = 0.05 * rng.standard_normal(c.mesh.X.shape)
    phi = rng.uniform(0, 0.2, c.mesh.n_nodes)
    kap = rng.uniform(0, 0.1, (c.mesh.n_elems, 8))
    R1, _, k1 = fem.assemble(m, c.mesh, fem.dof_vector(u, phi), kap, tangent=False)
    x = c.mesh.X + u
    u2 = Q @ x - c.mesh.X
    R2, _, k2 = fem.assemble(m, c.mesh, fem.dof_vector(u2, phi), kap, tangent=False)
    R1n, R2n = R1.reshape(-1, 4), R2.reshape(-1, 4)
    assert np.allclose(R2n[:, :3], R1n[:, :3] @ Q.T, atol=1e-10 * np.abs(R1).max())
    assert np.allclose(R2n[:, 3], R1n[:, 3], atol=1e-10 * np.abs(R1).max())
    assert np.allclose(k1, k2, rtol=1e-11, atol=1e-13)


def test_newton_matches_dense_brute_force_on_one_element():
    """One Hex8 element, 3 load steps: Newton with scipy's sparse LU and with
    numpy's dense solve reach the same converged state."""
    c = W.make_case(2, n=1, nz=1)
    m = fem.Model(c)
    u, phi, kap = c.u, c.phi, c.kappa
    for step in (1, 2, 3):
        u0 = W.affine_stretch_guess(c, step)
        bd, bv = W.affine_stretch_bc(c, step)
        d, kt, hist, ok = solve.newton(m, c.mesh, fem.dof_vector(u0, phi), kap, bd, bv,
                                       rtol=0.0, atol=1e-12)
        assert ok
        # brute force: dense Newton from the same guess
        dd = fem.dof_vector(u0, phi)
        dd[bd] = bv
        free = np.setdiff1d(np.arange(c.mesh.ndof), bd)
        for _ in range(30):
            R, K, _ = fem.assemble(m, c.mesh, dd, kap)
            if np.linalg.norm(R[free]) < 1e-12:
                break
            dd[free] += np.linalg.solve(K.toarray()[np.ix_(free, free)], -R[free])
        assert np.abs(dd - d).max() < 1e-10 * max(1.0, np.abs(d).max())
        u, phi = fem.split_dofs(d, 3)
        kap = kt


def test_uniform_stretch_load_path_has_closed_form_solution():
    """All boundary nodes on the affine field: the converged state is uniform,
    u = s (F_t - I) X and phi = kappa = max(kappa_prev, N^(psi_e(F_n))), which satisfies
    every equation (q = psi_e when phi = kappa; grad phi = 0)."""
    c = W.make_case(2, n=3, nz=2)
    m = fem.Model(c)
    u, phi, kap = c.u, c.phi, c.kappa
    lam = c.extra["stretch"]
    kprev = 0.0
    for step in (1, 2, 3):
        u0 = W.affine_stretch_guess(c, step)
        bd, bv = W.affine_stretch_bc(c, step)
        d, kt, hist, ok = solve.newton(m, c.mesh, fem.dof_vector(u0, phi), kap, bd, bv,
                                       rtol=0.0, atol=1e-12)
        assert ok
        s = step / c.n_steps
        Fn = torch.diag(torch.tensor(1.0 + s * (lam - 1.0), dtype=DT))[None]
        kref = max(kprev, float(m.yld(m.energy(Fn))[0]))
        uu, pp = fem.split_dofs(d, 3)
        assert np.abs(uu - s * (lam[:, None] - 1.0) * c.mesh.X).max() < 1e-10
        # the uniform phi mode is soft (stiffness ~ eta_d f_d / N^'), so the converged
        # damage fields carry the residual tolerance amplified by that compliance
        assert np.abs(pp - kref).max() < 1e-7 * max(1.0, kref)
        assert np.abs(kt - kref).max() < 1e-7 * max(1.0, kref)
        u, phi, kap, kprev = uu, pp, kt, kref


def test_dissipation_nonnegative_along_notched_path():
    """kappa never decreases and D = q (d_{n+1} - d_n) >= 0 at every qp and step."""
    c = W.make_case(3, n=8)
    c.n_steps = 40
    m = fem.Model(c)
    recs = solve.load_path(c, m, steps=12)
    mat = c.material
    for r in recs:
        k0, k1 = r["kappa_prev"].ravel(), r["kappa"].ravel()
        assert (k1 >= k0).all()
        d0 = 1 - np.exp(-mat["eta_d"] * np.clip(k0 - mat["kappa_d"], 0, None))
        d1 = 1 - np.exp(-mat["eta_d"] * np.clip(k1 - mat["kappa_d"], 0, None))
        geo, _, _, _, _ = fem.element_response(m, c.mesh, r["d"], r["kappa_prev"], tangent=False)
        de = torch.tensor(r["d"][geo.edofs], dtype=DT)
        z = fem.z_reference(2, *geo.Jw.shape) + torch.einsum("eqzk,ek->eqz", fem.b_matrix(geo), de)
        F, phi, _ = cm.fields_from_z(z.reshape(-1, 7), 2)
        q = cm.drive_q(m.energy(F), phi, torch.tensor(k1), mat).detach().numpy()
        moved = k1 > k0
        assert (q[moved] * (d1 - d0)[moved] >= -1e-12).all()
