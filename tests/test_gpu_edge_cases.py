"""Edge and degenerate cases through the C ABI: an empty batch, single-element
meshes, inverted elements, the local-update iteration limit forced from the
host, and rejected arguments.  None of them can fault the device (table
indices are masked, every loop is bounded, arguments are checked before any
launch); the conditions surface as status or error codes."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fem

from gpu_common import rel_err, state, sync, to_scipy

pytestmark = pytest.mark.gpu
E_ARG, E_SHAPE, E_LOCAL_NOCONV, E_JNONPOS = -1, -2, -4, -9
E_NEWTON_NOCONV = -5


@pytest.fixture(scope="module")
def G():
    from paper_2604_03411_amd import gedmg
    return gedmg


def test_empty_jet_batch(G):
    case = W.make_case(1, n=2)
    ctx = G.Context.from_case(case)
    jet = ctx.energy_jet(torch.zeros(0, 3, dtype=torch.float64, device=ctx.dev))
    sync()
    assert tuple(jet.shape) == (0, 10)
    ctx.close()


@pytest.mark.parametrize("cfg,kw", [(1, dict(n=1)), (2, dict(n=1, nz=1))])
def test_single_element_mesh_matches_oracle(G, cfg, kw):
    """One element: one colour, one (partly idle) wavefront.

    Every point of this state yields, and a single element's K has no
    unyielded entries to dilute the norm: a one-ulp change of the local
    solution κ moves the oracle's own K by 7e-12 (Q4) and 4.4e-12 (Hex8).
    The local solve fixes κ to about one ulp on either side, so K is held to
    3 ulps of κ (2e-11).  The same perturbation leaves R unchanged (the
    implicit-function step on κ corrects its value to first order), so R
    stays at 1e-12."""
    case = W.make_case(cfg, **kw)
    assert case.mesh.n_elems == 1
    print(f"[edge] single element, dim {case.mesh.dim}", flush=True)
    u, phi, kap = state(case, 31 + cfg)
    R0, K0, k0 = fem.assemble(fem.Model(case), case.mesh, fem.dof_vector(u, phi), kap)
    ctx = G.Context.from_case(case)
    R, K, kt = ctx.assemble(*ctx.fields(u, phi, kap), "fp64")
    sync()
    assert ctx.status() == 0
    Kg = to_scipy(ctx, K)
    assert np.array_equal(Kg.indptr, K0.indptr) and np.array_equal(Kg.indices, K0.indices)
    assert rel_err(R.cpu().numpy(), R0) <= 1e-12
    assert rel_err(Kg.data, K0.data) <= 2e-11
    assert rel_err(kt.cpu().numpy(), k0) <= 1e-12
    ctx.close()


def test_inverted_elements_report_status(G):
    """u = -2 X1 e1 gives F11 = -1, J = -1 at every point: the assembly
    completes, the status reports det F <= 0, and reading it clears it."""
    case = W.make_case(1, n=4)
    _, phi, kap = state(case, 5)
    u = np.zeros_like(case.mesh.X)
    u[0] = -2.0 * case.mesh.X[0]
    ctx = G.Context.from_case(case)
    ctx.assemble(*ctx.fields(u, phi, kap), "fp64")
    sync()
    assert ctx.status() == E_JNONPOS
    assert ctx.status() == 0
    ctx.close()


def test_local_update_iteration_limit_is_reported(G):
    """With max_local = 1 the FP64 local Newton cannot reach its acceptance test
    (a correction below 1e-13 max(1, |kappa|), or a bracket narrower than 1e-15
    max(1, |kappa|)) at damaging points: the load step returns the local
    non-convergence code and leaves the fields at their input values."""
    case = W.make_case(2, n=4, nz=2)
    ctx = G.Context.from_case(case)
    u, phi, kap = ctx.fields(case.u, case.phi, case.kappa)
    u.copy_(torch.as_tensor(W.affine_stretch_guess(case, case.n_steps), device=ctx.dev))
    u0, p0, k0 = u.clone(), phi.clone(), kap.clone()
    bd, bv = W.affine_stretch_bc(case, case.n_steps)
    rep = ctx.newton_step(u, phi, kap, bd, bv, max_local=1, raise_on_error=False)
    sync()
    print(f"[edge] max_local = 1: status {rep['status']}", flush=True)
    assert rep["status"] == E_LOCAL_NOCONV
    assert torch.equal(u, u0) and torch.equal(phi, p0) and torch.equal(kap, k0)
    ctx.close()


def test_invalid_arguments_are_rejected(G):
    case = W.make_case(1, n=2)
    ctx = G.Context.from_case(case)
    f = ctx.fields(case.u, case.phi, case.kappa)
    with pytest.raises(G.GedmgError) as e:
        ctx.assemble(*f, 7)
    assert e.value.code == E_ARG
    with pytest.raises(G.GedmgError) as e:
        ctx.newton_step(*f, [0], [0.0], max_local=0)
    assert e.value.code == E_ARG
    ctx.close()
    bad = W.Mesh(case.mesh.dim, case.mesh.X, case.mesh.conn.copy())
    bad.conn[0, 0] = case.mesh.n_nodes
    with pytest.raises(G.GedmgError) as e:
        G.Context(bad, case.material, case.energy, case.theta_e, case.yield_, case.theta_y)
    assert e.value.code == E_ARG
    wide = W.NetSpec(3, 48, 2, 3)
    with pytest.raises(G.GedmgError) as e:
        G.Context(case.mesh, case.material, wide, np.zeros(wide.n_params), case.yield_, case.theta_y)
    assert e.value.code == E_SHAPE


def test_library_rejects_out_of_range_reaction_dofs(G):
    """The C entry point checks reaction dofs itself (a caller of the C ABI has
    no binding in front of it): GEDMG_E_ARG, fields untouched."""
    import ctypes as C
    case = W.make_case(1, n=2)
    ctx = G.Context.from_case(case)
    u, phi, kap = ctx.fields(case.u, case.phi, case.kappa)
    u0 = u.clone()
    dofs = torch.tensor([0], dtype=torch.int32, device=ctx.dev)
    vals = torch.zeros(1, dtype=torch.float64, device=ctx.dev)
    rd = torch.tensor([ctx.ndof], dtype=torch.int32, device=ctx.dev)
    bc = G.Dirichlet(1, C.c_void_p(dofs.data_ptr()), C.c_void_p(vals.data_ptr()))
    opts = G.solver_opts()
    rep = G.NewtonReport()
    rc = G.lib().gedmg_newton_step(ctx._h, C.byref(bc), C.byref(opts), 0, None, C.c_void_p(u.data_ptr()),
                                   C.c_void_p(phi.data_ptr()), C.c_void_p(kap.data_ptr()),
                                   C.c_void_p(rd.data_ptr()), 1, C.byref(rep))
    sync()
    assert rc == E_ARG
    assert torch.equal(u, u0)
    ctx.close()


def _homogeneous_state(case, stretch):
    """u of the homogeneous deformation diag(s, 0.99 / sqrt(s), 1.01 / sqrt(s))
    on the unit cube (nearly isochoric), phi = 0."""
    X = case.mesh.X
    t = 1.0 / np.sqrt(stretch)
    u = np.stack([(stretch - 1.0) * X[0], (0.99 * t - 1.0) * X[1], (1.01 * t - 1.0) * X[2]])
    return u, np.zeros(case.mesh.n_nodes)


def test_history_tie_on_the_yield_surface(G):
    """kappa_n equal to the driving force (h(kappa_n) = 0 up to rounding) at
    every point of one homogeneously stretched element of the closed-form
    local model, above kappa_d.  Whether such a point counts as loading is
    decided by rounding, so R and kappa_trial must match the oracle while K
    must equal either the oracle's loading tangent or its elastic one (taken
    with kappa_n moved by 1e-13 relative to either side), which differ here."""
    case = W.single_element_case(eta_d=10.0, kappa_d=0.1)
    u, phi = _homogeneous_state(case, 1.2)
    m = fem.Model(case)
    d = fem.dof_vector(u, phi)
    _, _, psi = fem.assemble(m, case.mesh, d, np.zeros_like(case.kappa), tangent=False)
    kap = psi.copy()  # local model: the updated history is psi_NH itself
    assert kap.min() > 0.1 and np.ptp(kap) <= 1e-14 * kap.max()
    print(f"[edge] history tie at kappa_n = psi_NH = {kap.max():.6f}", flush=True)
    R0, _, k0 = fem.assemble(m, case.mesh, d, kap)
    _, K_load, _ = fem.assemble(m, case.mesh, d, kap * (1.0 - 1e-13))
    _, K_el, _ = fem.assemble(m, case.mesh, d, kap * (1.0 + 1e-13))
    assert rel_err(K_load.data, K_el.data) > 1e-3
    ctx = G.Context.from_case(case)
    R, K, kt = ctx.assemble(*ctx.fields(u, phi, kap), "fp64")
    sync()
    assert ctx.status() == 0
    Kg = to_scipy(ctx, K).data
    assert rel_err(R.cpu().numpy(), R0) <= 1e-12
    assert rel_err(kt.cpu().numpy(), k0) <= 1e-12
    e_load, e_el = rel_err(Kg, K_load.data), rel_err(Kg, K_el.data)
    print(f"  K against the loading tangent {e_load:.2e}, against the elastic one {e_el:.2e}", flush=True)
    assert min(e_load, e_el) <= 1e-11
    ctx.close()


def test_history_at_kappa_d(G):
    """kappa_n exactly kappa_d at every point: elastic points (psi_NH below
    kappa_d) keep f_d = 1, so R is the undamaged response; points stretched
    past kappa_d yield from the kink of the degradation function.  Both
    against the oracle at 1e-12."""
    for stretch, yields in ((1.05, False), (1.2, True)):
        case = W.single_element_case(eta_d=10.0, kappa_d=0.3)
        u, phi = _homogeneous_state(case, stretch)
        kap = np.full_like(case.kappa, 0.3)
        m = fem.Model(case)
        d = fem.dof_vector(u, phi)
        R0, K0, k0 = fem.assemble(m, case.mesh, d, kap)
        assert bool((k0 > 0.3).all()) == yields and bool((k0 == 0.3).all()) != yields
        print(f"[edge] kappa_n = kappa_d, stretch {stretch}: yields {yields}", flush=True)
        ctx = G.Context.from_case(case)
        R, K, kt = ctx.assemble(*ctx.fields(u, phi, kap), "fp64")
        sync()
        assert ctx.status() == 0
        assert rel_err(R.cpu().numpy(), R0) <= 1e-12
        assert rel_err(to_scipy(ctx, K).data, K0.data) <= 1e-12
        assert rel_err(kt.cpu().numpy(), k0) <= 1e-12
        if not yields:
            assert np.array_equal(kt.cpu().numpy(), kap)
        ctx.close()


def test_arclength_rejects_invalid_arguments(G):
    """gedmg_arclength_step's own checks (a C caller has no binding in front):
    non-positive arc length, negative load-factor scale or damage weight, a
    non-finite load factor, pattern dofs out of range; each GEDMG_E_ARG with
    u, phi and lambda untouched."""
    case = W.strip_case(nx=4)
    ctx = G.Context.from_case(case)
    u, phi, kap = ctx.fields(case.u, case.phi, case.kappa)
    u0 = u.clone()
    inc = torch.zeros(ctx.ndof + 1, dtype=torch.float64, device=ctx.dev)
    bd, bu = W.arclength_pattern(case)
    print("[edge] arc-length argument checks", flush=True)
    for kw in (dict(ds=0.0, psi=1.0, lam=0.0), dict(ds=-0.1, psi=1.0, lam=0.0), dict(ds=0.1, psi=-1.0, lam=0.0),
               dict(ds=0.1, psi=1.0, lam=float("nan")), dict(ds=0.1, psi=1.0, lam=0.0, wphi=-1.0)):
        lam, rep = ctx.arclength_step(u, phi, kap, bd, bu, kw["lam"], inc, kw["ds"], kw["psi"], raise_on_error=False,
                                      phi_weight=kw.get("wphi", 1.0))
        sync()
        assert rep["status"] == E_ARG, kw
    import ctypes as C
    dofs = torch.tensor([ctx.ndof], dtype=torch.int32, device=ctx.dev)
    vals = torch.ones(1, dtype=torch.float64, device=ctx.dev)
    pat = G.Dirichlet(1, C.c_void_p(dofs.data_ptr()), C.c_void_p(vals.data_ptr()))
    lamc = C.c_double(0.25)
    rep = G.NewtonReport()
    opts = G.solver_opts()
    rc = G.lib().gedmg_arclength_step(ctx._h, C.byref(pat), C.byref(opts), 0.1, 1.0, 1.0, C.byref(lamc),
                                      C.c_void_p(inc.data_ptr()), C.c_void_p(u.data_ptr()),
                                      C.c_void_p(phi.data_ptr()), C.c_void_p(kap.data_ptr()), None, 0, C.byref(rep))
    sync()
    assert rc == E_ARG and lamc.value == 0.25
    assert torch.equal(u, u0)
    ctx.close()


def test_diverging_newton_step_backtracks(G):
    """A load step whose Newton corrections invert elements.  The 20^3
    heterogeneous cube with every boundary node on its seeded field (random phi
    against beta_d = 1000 drives the interior into damage at once) sends the
    Newton iteration far from the start: corrections that leave a point with
    det F <= 0 are halved, up to 12 times in the step.  Whether the iteration
    then recovers and converges or runs out of halvings depends on the rounding
    of every Krylov solve on the way, so both outcomes are accepted: a
    converged step meets the residual test, and a failed one reports
    GEDMG_E_JNONPOS after all 12 halvings (or the Newton iteration limit) with
    u, phi and kappa exactly as they were passed in."""
    case = W.make_case(4, n=20)
    bd, bv = W.boundary_field_bc(case)
    ctx = G.Context.from_case(case)
    u, phi, kap = ctx.fields(case.u, case.phi, case.kappa)
    u0, p0, k0 = u.clone(), phi.clone(), kap.clone()
    print("[edge] diverging Newton step on the 20^3 heterogeneous cube", flush=True)
    atol = 1e-9 * np.sqrt(case.mesh.ndof)
    rep = ctx.newton_step(u, phi, kap, bd, bv, raise_on_error=False, max_newton=40, newton_rtol=1e-10,
                          newton_atol=atol)
    sync()
    print(f"  status {rep['status']}, iterations {rep['newton_iters']}, backtracks {rep['backtracks']}", flush=True)
    assert rep["backtracks"] >= 1
    if rep["status"] == 0:
        if rep["newton_iters"] < 32:  # the report keeps the first 32 residual norms
            assert rep["res_norm"][-1] <= max(atol, 1e-10 * max(1.0, rep["res_norm"][0]))
    else:
        assert rep["status"] in (E_JNONPOS, E_NEWTON_NOCONV)
        if rep["status"] == E_JNONPOS:
            assert rep["backtracks"] == 12
        assert torch.equal(u, u0) and torch.equal(phi, p0) and torch.equal(kap, k0)
    ctx.close()


def test_newton_step_from_an_inverted_state_fails_and_restores_fields(G):
    """Boundary values that invert the elements at the boundary (u_x = -2 X_1 on
    every boundary node: F_11 = -1 there) leave the step nothing to halve: the
    first assembly reports det F <= 0, and the step returns GEDMG_E_JNONPOS
    without a correction, with u, phi and kappa exactly as they were passed in
    (the boundary values it wrote are taken back)."""
    case = W.make_case(4, n=6)
    m = case.mesh
    nodes = W.boundary_nodes(m)
    bd = (nodes * (m.dim + 1)).astype(np.int32)  # u_x of every boundary node
    bv = -2.0 * m.X[0, nodes]
    ctx = G.Context.from_case(case)
    u, phi, kap = ctx.fields(case.u, case.phi, case.kappa)
    u0, p0, k0 = u.clone(), phi.clone(), kap.clone()
    print("[edge] Newton step from an inverted boundary state, 6^3 cube", flush=True)
    rep = ctx.newton_step(u, phi, kap, bd, bv, raise_on_error=False)
    sync()
    print(f"  status {rep['status']}, iterations {rep['newton_iters']}, backtracks {rep['backtracks']}", flush=True)
    assert rep["status"] == E_JNONPOS and rep["backtracks"] == 0
    assert torch.equal(u, u0) and torch.equal(phi, p0) and torch.equal(kap, k0)
    ctx.close()
