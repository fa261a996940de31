"""Seeded synthetic inputs shaped like the paper's finite-element studies.

This module only *generates* inputs: structured meshes (2-D Q4 plane strain,
3-D Hex8), the raw ICNN parameter vectors, nodal displacement / nonlocal-damage
fields, quadrature-point history values and Dirichlet data for displacement-
controlled load paths.  It contains none of the method's arithmetic (no
invariants, networks, energies, local updates, element integrals or solvers),
so the oracle and the GPU path can both consume it without sharing any code
of the method.

Conventions shared by every consumer (they define the array layouts of the
C ABI as well):

* node numbering is lexicographic (x fastest, then y, then z);
* Q4 connectivity is counter-clockwise; Hex8 is the standard ordering (bottom
  face counter-clockwise, then the top face in the same order);
* the quadrature point with local index q is the 2x2 / 2x2x2 Gauss point that
  lies on the ray from the element centre to local node q (natural coordinates
  of node q divided by sqrt(3)), weight 1;
* degrees of freedom are interleaved node-major: dof(node, c) = node*(dim+1)+c,
  with c < dim the displacement components and c == dim the nonlocal damage
  phi;
* nodal fields are structure-of-arrays: u[dim][n_nodes], phi[n_nodes],
  X[dim][n_nodes]; history kappa[n_elems][nqp].

Material constants follow the uniform-plate study of the paper (E = 210 MPa,
nu = 0.3, eta_d = 0.002 MPa^-1, kappa_d = 0.1 MPa, c_d = 1 MPa^-1 mm^2,
beta_d = 1000 MPa^-1; eta_d = 0.001 for the notched plate), with gamma_d = 1.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# --------------------------------------------------------------------------
# material constants (Section "Uniform Deformation and Mesh Independence")
# --------------------------------------------------------------------------
_E, _NU = 210.0, 0.3
MATERIAL = dict(
    mu_e=_E / (2.0 * (1.0 + _NU)),
    lambda_e=_E * _NU / ((1.0 + _NU) * (1.0 - 2.0 * _NU)),
    eta_d=0.002,
    kappa_d=0.1,
    c_d=1.0,
    beta_d=1000.0,
    gamma_d=1.0,
)


# Energy scale per workload.  The network energy is dimensionless and mu_e is
# the stress factor in front of it (Sec. 4.2.1); these values make the initial
# shear modulus of each seeded network equal E / (2 (1 + nu)) = 80.77 MPa.
# Written by `python -m oracle.calibrate` (shear slope 2 (N_1 + 3 N_2) at x = 0).
MU_E = {
    1: 0.20226426887624965,
    2: 0.053942359359390527,
    3: 0.052817139041526226,
    4: 0.00030980000503664254,
    5: 0.05437242663969557,
}


# --------------------------------------------------------------------------
# ICNN descriptors (only shapes and raw parameter draws live here)
# --------------------------------------------------------------------------
@dataclass
class NetSpec:
    """Architecture of an input-convex network: n_in -> width x n_hidden -> 1.

    monotone_mask: bit i set means every weight that multiplies input i is
    passed through softplus (non-negative).  The yield network uses 1 (its
    single input q, so that it is increasing); the energy network uses 3
    (inputs I1G - 3 and I2G - 3, so that the energy is non-decreasing in the
    polyconvex invariants), leaving the J - 1 pass-through weights raw.
    """

    n_in: int
    width: int
    n_hidden: int
    monotone_mask: int = 0

    @property
    def n_params(self) -> int:
        if self.n_hidden == 0:  # closed-form model (no network)
            return 0
        h, n = self.width, self.n_in
        return h * n + h + (self.n_hidden - 1) * (h * h + h * n + h) + h + n + 1


def draw_theta(rng: np.random.Generator, spec: NetSpec, std: float = 0.1) -> np.ndarray:
    """Raw parameters, i.i.d. N(0, std^2), in the flat layer order."""
    return rng.normal(0.0, std, size=spec.n_params)


# --------------------------------------------------------------------------
# meshes
# --------------------------------------------------------------------------
@dataclass
class Mesh:
    dim: int
    X: np.ndarray            # [dim][n_nodes] float64
    conn: np.ndarray         # [n_elems][nen] int32
    grid: tuple = ()         # structured element counts (before removals)

    @property
    def n_nodes(self) -> int:
        return self.X.shape[1]

    @property
    def n_elems(self) -> int:
        return self.conn.shape[0]

    @property
    def nen(self) -> int:
        return self.conn.shape[1]

    @property
    def nqp(self) -> int:
        return 4 if self.dim == 2 else 8

    @property
    def ndof(self) -> int:
        return self.n_nodes * (self.dim + 1)


def q4_grid(nx: int, ny: int, lx: float = 1.0, ly: float = 1.0) -> Mesh:
    i = np.arange(nx + 1)
    j = np.arange(ny + 1)
    ii, jj = np.meshgrid(i, j, indexing="xy")
    X = np.stack([ii.ravel() * (lx / nx), jj.ravel() * (ly / ny)]).astype(np.float64)
    nid = lambda a, b: b * (nx + 1) + a  # noqa: E731
    ei, ej = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    ei, ej = ei.ravel(), ej.ravel()
    conn = np.stack([nid(ei, ej), nid(ei + 1, ej), nid(ei + 1, ej + 1), nid(ei, ej + 1)], 1)
    return Mesh(2, X, conn.astype(np.int32), (nx, ny))


def hex8_grid(nx: int, ny: int, nz: int, lx=1.0, ly=1.0, lz=1.0) -> Mesh:
    i, j, k = np.arange(nx + 1), np.arange(ny + 1), np.arange(nz + 1)
    kk, jj, ii = np.meshgrid(k, j, i, indexing="ij")
    X = np.stack([ii.ravel() * (lx / nx), jj.ravel() * (ly / ny), kk.ravel() * (lz / nz)])
    nid = lambda a, b, c: (c * (ny + 1) + b) * (nx + 1) + a  # noqa: E731
    ek, ej, ei = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ei, ej, ek = ei.ravel(), ej.ravel(), ek.ravel()
    conn = np.stack([
        nid(ei, ej, ek), nid(ei + 1, ej, ek), nid(ei + 1, ej + 1, ek), nid(ei, ej + 1, ek),
        nid(ei, ej, ek + 1), nid(ei + 1, ej, ek + 1), nid(ei + 1, ej + 1, ek + 1), nid(ei, ej + 1, ek + 1),
    ], 1)
    return Mesh(3, X.astype(np.float64), conn.astype(np.int32), (nx, ny, nz))


def remove_elements_near(mesh: Mesh, centre, radius: float) -> Mesh:
    """Drop elements whose centroid lies closer than `radius` to `centre`,
    then drop nodes no element uses and renumber (order preserved)."""
    cen = mesh.X[:, mesh.conn].mean(axis=2)  # [dim][n_elems]
    d = np.sqrt(((cen - np.asarray(centre, dtype=np.float64)[:, None]) ** 2).sum(0))
    keep = d >= radius
    conn = mesh.conn[keep]
    used = np.zeros(mesh.n_nodes, bool)
    used[conn.ravel()] = True
    new_id = -np.ones(mesh.n_nodes, np.int64)
    new_id[used] = np.arange(used.sum())
    return Mesh(mesh.dim, mesh.X[:, used].copy(), new_id[conn].astype(np.int32), mesh.grid)


# --------------------------------------------------------------------------
# load cases
# --------------------------------------------------------------------------
@dataclass
class Case:
    name: str
    mesh: Mesh
    material: dict
    energy: NetSpec
    yield_: NetSpec
    theta_e: np.ndarray
    theta_y: np.ndarray
    u: np.ndarray            # [dim][n_nodes]
    phi: np.ndarray          # [n_nodes]
    kappa: np.ndarray        # [n_elems][nqp]
    n_steps: int = 0
    extra: dict = field(default_factory=dict)


def _dof(node, comp, dim):
    return np.asarray(node, np.int64) * (dim + 1) + comp


def boundary_nodes(mesh: Mesh, tol: float = 1e-12) -> np.ndarray:
    X = mesh.X
    lo, hi = X.min(axis=1, keepdims=True), X.max(axis=1, keepdims=True)
    on = ((np.abs(X - lo) < tol) | (np.abs(X - hi) < tol)).any(axis=0)
    return np.nonzero(on)[0]


def affine_stretch_bc(case: Case, step: int):
    """Every boundary node gets u = s_n (F_t - I) X, s_n = step / n_steps."""
    m = case.mesh
    s = step / case.n_steps
    lam = case.extra["stretch"]
    nodes = boundary_nodes(m)
    dofs, vals = [], []
    for c in range(m.dim):
        dofs.append(_dof(nodes, c, m.dim))
        vals.append(s * (lam[c] - 1.0) * m.X[c, nodes])
    return np.concatenate(dofs).astype(np.int32), np.concatenate(vals)


def boundary_field_bc(case: Case):
    """Every dof (displacement and phi) of every boundary node prescribed to the
    case's own nodal field: the heterogeneous-stretch cube then has a unique
    converged interior state to compare precisions on."""
    m = case.mesh
    nodes = boundary_nodes(m)
    dofs, vals = [], []
    for c in range(m.dim):
        dofs.append(_dof(nodes, c, m.dim))
        vals.append(case.u[c, nodes])
    dofs.append(_dof(nodes, m.dim, m.dim))
    vals.append(case.phi[nodes])
    return np.concatenate(dofs).astype(np.int32), np.concatenate(vals)


def affine_stretch_guess(case: Case, step: int):
    """Initial guess for load step `step`: the affine field plus seeded noise."""
    m = case.mesh
    s = step / case.n_steps
    lam = case.extra["stretch"]
    rng = np.random.default_rng([case.extra["seed"], step])
    u = np.stack([s * (lam[c] - 1.0) * m.X[c] for c in range(m.dim)])
    u = u + rng.normal(0.0, 1e-3, size=u.shape)
    return u


def uniaxial_bc(case: Case, step: int):
    """Left edge u_x = 0, node at the origin u_y = 0, right edge
    u_x = total * step / n_steps (displacement control)."""
    m = case.mesh
    x = m.X[0]
    total = case.extra["total_disp"]
    left = np.nonzero(np.abs(x - x.min()) < 1e-12)[0]
    right = np.nonzero(np.abs(x - x.max()) < 1e-12)[0]
    origin = np.nonzero((np.abs(m.X) < 1e-12).all(axis=0))[0]
    dofs = np.concatenate([_dof(left, 0, m.dim), _dof(origin, 1, m.dim), _dof(right, 0, m.dim)])
    vals = np.concatenate([np.zeros(left.size), np.zeros(origin.size),
                           np.full(right.size, total * step / case.n_steps)])
    return dofs.astype(np.int32), vals


def uniaxial_increment(case: Case) -> np.ndarray:
    """Predictor increment of one uniaxial load step, [dim][n_nodes]: the
    boundary displacement increment spread linearly in x (zero on the left
    edge, the full increment on the right edge), other components zero."""
    m = case.mesh
    x = m.X[0]
    span = x.max() - x.min()
    du = np.zeros((m.dim, m.n_nodes))
    du[0] = case.extra["total_disp"] / case.n_steps * (x - x.min()) / span
    return du


def uniaxial_predictor(case: Case, u_prev: np.ndarray, step: int):
    """Previous converged u plus the boundary increment spread linearly in x."""
    return u_prev + uniaxial_increment(case)


def reaction_dofs(case: Case) -> np.ndarray:
    """x-displacement dofs of the right edge (where the load is applied)."""
    m = case.mesh
    x = m.X[0]
    right = np.nonzero(np.abs(x - x.max()) < 1e-12)[0]
    return _dof(right, 0, m.dim).astype(np.int32)


def _uniaxial_fields(mesh):
    return (np.zeros((mesh.dim, mesh.n_nodes)), np.zeros(mesh.n_nodes),
            np.zeros((mesh.n_elems, mesh.nqp)))


def make_case(cfg: int, n: int | None = None, nz: int | None = None) -> Case:
    """Build the seeded input of one of the five workloads.

    cfg 1: Q4 16x16 unit square, single assembly.
    cfg 2: Hex8 32x32x8 box 1 x 1 x 0.25, 10 affine-stretch load steps.
    cfg 3: Q4 256x256 notched plate, 40 uniaxial load steps.
    cfg 4: Hex8 64^3 unit cube, heterogeneous stretch, single assembly.
    cfg 5: Q4 128x128, 20 uniaxial load steps (adjoint).

    `n` (and `nz` for cfg 2) shrink the mesh for small parity cases while
    keeping every other ingredient (networks, distributions, load path).
    """
    seed = cfg
    rng = np.random.default_rng(seed)
    mat = dict(MATERIAL)
    mat["mu_e"] = MU_E[cfg]
    if cfg == 1:
        nx = n or 16
        mesh = q4_grid(nx, nx)
        es, ys = NetSpec(3, 16, 2, 3), NetSpec(1, 16, 1, 1)
        te, ty = draw_theta(rng, es), draw_theta(rng, ys)
        Ft = np.array([1.3, 1.0])
        u = (Ft[:, None] - 1.0) * mesh.X + rng.normal(0.0, 1e-3, size=mesh.X.shape)
        phi = rng.uniform(0.0, 0.2, size=mesh.n_nodes)
        kap = rng.uniform(0.0, 0.1, size=(mesh.n_elems, mesh.nqp))
        return Case("q4_16x16_single_assembly", mesh, mat, es, ys, te, ty, u, phi, kap)
    if cfg == 2:
        nx = n or 32
        nzz = nz or max(1, nx // 4)
        mesh = hex8_grid(nx, nx, nzz, 1.0, 1.0, nzz / nx)
        es, ys = NetSpec(3, 32, 2, 3), NetSpec(1, 16, 1, 1)
        te, ty = draw_theta(rng, es), draw_theta(rng, ys)
        lam = rng.uniform(1.0, 1.5, size=3)
        u, phi, kap = _uniaxial_fields(mesh)
        return Case("hex8_32x32x8_newton_10_steps", mesh, mat, es, ys, te, ty, u, phi, kap, 10,
                    dict(stretch=lam, seed=seed))
    if cfg == 3:
        nx = n or 256
        mesh = remove_elements_near(q4_grid(nx, nx), (0.0, 0.5), 0.05)
        mat["eta_d"] = 0.001
        es, ys = NetSpec(3, 32, 2, 3), NetSpec(1, 32, 2, 1)
        te, ty = draw_theta(rng, es), draw_theta(rng, ys)
        u, phi, kap = _uniaxial_fields(mesh)
        return Case("q4_256x256_notched_40_steps", mesh, mat, es, ys, te, ty, u, phi, kap, 40,
                    dict(total_disp=0.25, seed=seed))
    if cfg == 4:
        nx = n or 64
        mesh = hex8_grid(nx, nx, nx)
        es, ys = NetSpec(3, 64, 3, 3), NetSpec(1, 16, 1, 1)
        te, ty = draw_theta(rng, es), draw_theta(rng, ys)
        m = rng.integers(1, 4, size=3)
        ph = rng.uniform(0.0, 2.0 * math.pi, size=3)
        X = mesh.X
        u = np.stack([0.25 * X[i] - 0.25 / (2 * math.pi * m[i])
                      * (np.cos(2 * math.pi * m[i] * X[i] + ph[i]) - np.cos(ph[i]))
                      for i in range(3)])
        u = u + rng.normal(0.0, 1e-3, size=u.shape)
        phi = rng.uniform(0.0, 0.2, size=mesh.n_nodes)
        kap = rng.uniform(0.0, 0.1, size=(mesh.n_elems, mesh.nqp))
        return Case("hex8_64x64x64_assembly", mesh, mat, es, ys, te, ty, u, phi, kap, 0,
                    dict(modes=m, phases=ph))
    if cfg == 5:
        nx = n or 128
        mesh = q4_grid(nx, nx)
        es, ys = NetSpec(3, 32, 2, 3), NetSpec(1, 32, 2, 1)
        te, ty = draw_theta(rng, es), draw_theta(rng, ys)
        u, phi, kap = _uniaxial_fields(mesh)
        trng = np.random.default_rng(55)
        pe = te + trng.normal(0.0, 0.01, size=te.shape)
        py = ty + trng.normal(0.0, 0.01, size=ty.shape)
        # The homogeneous bar reaches its limit point near 16 % strain; the
        # loss path stops at 12.5 % so that every converged state is unique.
        return Case("q4_128x128_adjoint_20_steps", mesh, mat, es, ys, te, ty, u, phi, kap, 20,
                    dict(total_disp=0.125, seed=seed, theta_e_star=pe, theta_y_star=py))
    raise ValueError(f"unknown workload {cfg}")


# --------------------------------------------------------------------------
# closed-form model studies (Neo-Hooke energy, G = identity yield)
# --------------------------------------------------------------------------
CLOSED_FORM = NetSpec(3, 0, 0, 0)     # energy: compressible Neo-Hooke (no network)
IDENTITY_YIELD = NetSpec(1, 0, 0, 0)  # yield: G(q) = q


def lame(E: float, nu: float):
    """Shear and bulk-type Lame moduli (mu, lambda) of Young's modulus E and
    Poisson ratio nu."""
    return E / (2.0 * (1.0 + nu)), E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))


def _closed_material(E, nu, eta_d, kappa_d, c_d, beta_d):
    mu, lam = lame(E, nu)
    return dict(mu_e=mu, lambda_e=lam, eta_d=eta_d, kappa_d=kappa_d, c_d=c_d, beta_d=beta_d, gamma_d=1.0)


def single_element_case(eta_d: float = 10.0, kappa_d: float = 1.0, n_steps: int = 50,
                        total_disp: float = 0.5) -> Case:
    """One 1 x 1 x 1 mm Hex8 element of the closed-form model under uniaxial
    tension to total_disp mm (E = 42 MPa, nu = 0.45), local model: no
    gradient or penalty term (c_d = beta_d = 0), so q = psi_e and the nonlocal
    field is unused (every phi dof is prescribed to 0)."""
    mesh = hex8_grid(1, 1, 1)
    mat = _closed_material(42.0, 0.45, eta_d, kappa_d, 0.0, 0.0)
    u, phi, kap = _uniaxial_fields(mesh)
    return Case(f"hex8_single_element_eta{eta_d:g}_kd{kappa_d:g}", mesh, mat, CLOSED_FORM, IDENTITY_YIELD,
                np.zeros(0), np.zeros(0), u, phi, kap, n_steps, dict(total_disp=total_disp, local=True))


def uniform_plate_case(mesh_kind: str = "coarse", nonlocal_: bool = True, n_steps: int = 1000,
                       total_disp: float = 1.0, seed: int = 7) -> Case:
    """The 10 x 10 x 1 mm plate of the uniform-deformation study with the
    closed-form model (E = 210 MPa, nu = 0.3, eta_d = 0.002, kappa_d = 0.1,
    c_d = 1, beta_d = 1000), one Hex8 element through the thickness.
    mesh_kind: "coarse" (10 x 10), "refined" (20 x 20) or "nonuniform" (10 x 10
    with the interior node columns and rows moved by a seeded +-30 % of the
    spacing).  nonlocal_=False gives the local model (c_d = beta_d = 0, every
    phi dof prescribed to 0)."""
    n = {"coarse": 10, "refined": 20, "nonuniform": 10}[mesh_kind]
    mesh = hex8_grid(n, n, 1, 10.0, 10.0, 1.0)
    if mesh_kind == "nonuniform":
        rng = np.random.default_rng(seed)
        h = 10.0 / n
        sx = np.concatenate([[0.0], np.arange(1, n) * h + rng.uniform(-0.3, 0.3, n - 1) * h, [10.0]])
        sy = np.concatenate([[0.0], np.arange(1, n) * h + rng.uniform(-0.3, 0.3, n - 1) * h, [10.0]])
        i = np.rint(mesh.X[0] / h).astype(int)
        j = np.rint(mesh.X[1] / h).astype(int)
        mesh.X[0] = sx[i]
        mesh.X[1] = sy[j]
    cd, bd = (1.0, 1000.0) if nonlocal_ else (0.0, 0.0)
    mat = _closed_material(210.0, 0.3, 0.002, 0.1, cd, bd)
    u, phi, kap = _uniaxial_fields(mesh)
    return Case(f"hex8_plate_{mesh_kind}_{'nonlocal' if nonlocal_ else 'local'}", mesh, mat, CLOSED_FORM,
                IDENTITY_YIELD, np.zeros(0), np.zeros(0), u, phi, kap, n_steps,
                dict(total_disp=total_disp, local=not nonlocal_))


def symmetric_tension_bc(case: Case, step: int):
    """Uniaxial tension of a box: u_x = 0 on the face x = min, u_y = 0 on
    y = min, u_z = 0 on z = min (symmetry planes), u_x = total * step / n_steps
    on x = max; with case.extra["local"] every phi dof is prescribed to 0."""
    m = case.mesh
    X = m.X
    lo = X.min(axis=1)
    hi_x = X[0].max()
    dofs, vals = [], []
    for c in range(m.dim):
        on = np.nonzero(np.abs(X[c] - lo[c]) < 1e-12)[0]
        dofs.append(_dof(on, c, m.dim))
        vals.append(np.zeros(on.size))
    right = np.nonzero(np.abs(X[0] - hi_x) < 1e-12)[0]
    dofs.append(_dof(right, 0, m.dim))
    vals.append(np.full(right.size, case.extra["total_disp"] * step / case.n_steps))
    if case.extra.get("local"):
        allnodes = np.arange(m.n_nodes)
        dofs.append(_dof(allnodes, m.dim, m.dim))
        vals.append(np.zeros(m.n_nodes))
    return np.concatenate(dofs).astype(np.int32), np.concatenate(vals)


def training_case(n: int = 4, seed: int = 5, teacher_std: float = 0.02, beta_d: float = 10.0) -> Case:
    """Synthetic stress-stretch data for fitting the two networks through the
    load-path adjoint: an n x n Q4 bar (unit square) pulled uniaxially along a
    cyclic path with unloading and reloading (loading to 5 %, back to 2 %, to
    9 %, back to 4 %, to 12 %), the networks of the 128 x 128 adjoint workload
    (3-32-32-1 energy, 1-32-32-1 yield) as the starting point and a teacher
    with the raw parameters perturbed by N(0, teacher_std^2) (seed 77) whose
    reactions are the targets.  The homogeneous states have phi = kappa, so
    the response does not depend on beta_d; beta_d = 10 (instead of 1000)
    keeps the uniform-damage mode of the tangent, and with it the gradient,
    well conditioned."""
    base = make_case(5, n=n)
    base.material = dict(base.material, beta_d=beta_d)
    levels = np.concatenate([np.linspace(0.01, 0.05, 5), [0.035, 0.02], np.linspace(0.034, 0.09, 5),
                             [0.065, 0.04], np.linspace(0.06, 0.12, 4)])
    trng = np.random.default_rng(77)
    te_star = base.theta_e + trng.normal(0.0, teacher_std, size=base.theta_e.shape)
    ty_star = base.theta_y + trng.normal(0.0, teacher_std, size=base.theta_y.shape)
    return Case(f"q4_{n}x{n}_cyclic_training", base.mesh, base.material, base.energy, base.yield_,
                base.theta_e, base.theta_y, base.u, base.phi, base.kappa, len(levels),
                dict(levels=levels, theta_e_star=te_star, theta_y_star=ty_star, seed=seed, total_disp=1.0))


def cyclic_bc(case: Case, step: int):
    """uniaxial_bc with the right-edge displacement of the cyclic path."""
    dofs, vals = uniaxial_bc(case, step)
    lvl = case.extra["levels"][step - 1]
    return dofs, np.where(vals != 0.0, lvl, vals)


def cyclic_increment(case: Case, step: int) -> np.ndarray:
    """Predictor increment of step `step` of the cyclic path (the change of the
    boundary displacement spread linearly in x)."""
    lv = case.extra["levels"]
    prev = lv[step - 2] if step > 1 else 0.0
    return uniaxial_increment(case) * case.n_steps * (lv[step - 1] - prev)


def strip_case(nx: int = 20, eta_d: float = 2.0, kappa_d: float = 0.1, c_d: float = 1.0,
               beta_d: float = 1000.0, neck: float = 0.1, E: float = 210.0, nu: float = 0.3) -> Case:
    """A Q4 strip of nx unit elements (length nx, height 1) of the closed-form
    model, necked at mid-length (the two top nodes there lowered by `neck`):
    under tension the damage starts and localises in the neck while the rest
    of the strip unloads; with nx = 20 and eta_d = 2 the end displacement falls
    with the force past the force maximum (snap-back), which only arc-length
    continuation follows.
    Loading: u_x = 0 on the left edge, u_y = 0 at the origin, u_x = lambda on
    the right edge (unit pattern, see arclength_pattern)."""
    mesh = q4_grid(nx, 1, float(nx), 1.0)
    mid = nx // 2
    top = np.nonzero((np.abs(mesh.X[1] - 1.0) < 1e-12) & ((np.abs(mesh.X[0] - mid) < 1e-12)
                                                          | (np.abs(mesh.X[0] - mid - 1) < 1e-12)))[0]
    mesh.X[1, top] -= neck
    mat = _closed_material(E, nu, eta_d, kappa_d, c_d, beta_d)
    u, phi, kap = _uniaxial_fields(mesh)
    return Case(f"q4_strip_{nx}x1", mesh, mat, CLOSED_FORM, IDENTITY_YIELD, np.zeros(0), np.zeros(0), u, phi, kap,
                0, dict(total_disp=1.0))


def arclength_pattern(case: Case, bc_fn=None):
    """Prescribed dofs of a displacement-controlled loading with their values
    per unit load factor: 1 where bc_fn (default uniaxial_bc) moves a dof, 0
    where it holds one."""
    dofs, vals = (bc_fn or uniaxial_bc)(dataclass_replace_steps(case), 1)
    return dofs, np.where(vals != 0.0, 1.0, 0.0)


def dataclass_replace_steps(case: Case) -> Case:
    """A shallow copy of case with one load step of unit total displacement."""
    import dataclasses
    return dataclasses.replace(case, n_steps=1, extra=dict(case.extra, total_disp=1.0))
