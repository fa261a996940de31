"""Mixed-precision (BF16 / FP16 matrix-core) energy-network jets, assembly and
converged states, against the FP64 oracle and the FP64 GPU path.  The paper
fixes no precision: the low-precision products carry the operand rounding of
the format (2^-9 for BF16, 2^-12 for FP16), so jets, stresses and tangents are
checked at a few times that unit, while converged states (the FP64 residual
decides convergence) must match the oracle to the Newton tolerance: u and
reactions to 1e-8, phi and kappa to 1e-6 (the soft uniform-damage mode
amplifies the residual floor there)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fem, solve
from oracle.icnn import ICNN

from gpu_common import rel_err, small_case, state, sync, to_scipy
from test_gpu_jet import oracle_jet

pytestmark = pytest.mark.gpu
JET_TOL = {"bf16": 3e-2, "fp16": 4e-3}
ATOL = 1e-11


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("cfg", [1, 3, 4])
def test_mixed_jet_error_vs_fp64(precision, cfg):
    from paper_2604_03411_amd import gedmg as G
    case = small_case(cfg)
    ctx = G.Context.from_case(case)
    rng = np.random.default_rng(cfg)
    x = torch.tensor(rng.uniform(-0.05, 0.3, (777, 3)), device=ctx.dev)
    ref = ctx.energy_jet(x, "fp64").cpu().numpy()
    got = ctx.energy_jet(x, precision).cpu().numpy()
    sync()
    errs = {k: rel_err(got[:, sl], ref[:, sl]) for k, sl in
            (("value", [0]), ("grad", [1, 2, 3]), ("hessian", list(range(4, 10))))}
    print(f"[mixed jet] cfg {cfg} {precision}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()), flush=True)
    for v in errs.values():
        assert v < JET_TOL[precision]
    ctx.close()


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
@pytest.mark.parametrize("cfg", [1, 3, 4])
def test_mixed_jet_error_vs_oracle(precision, cfg):
    """The low-precision jets against the oracle network's autograd jets (FP64):
    the error is the operand rounding of the format, at the same bound as
    against the FP64 GPU path."""
    from paper_2604_03411_amd import gedmg as G
    case = small_case(cfg)
    ctx = G.Context.from_case(case)
    rng = np.random.default_rng(50 + cfg)
    x = rng.uniform(-0.05, 0.3, (513, 3))
    got = ctx.energy_jet(torch.tensor(x, device=ctx.dev), precision).cpu().numpy()
    sync()
    ref = oracle_jet(case.theta_e, case.energy, x)
    errs = {k: rel_err(got[:, sl], ref[:, sl]) for k, sl in
            (("value", [0]), ("grad", [1, 2, 3]), ("hessian", list(range(4, 10))))}
    print(f"[mixed jet vs oracle] cfg {cfg} {precision}: " + " ".join(f"{k} {v:.2e}" for k, v in errs.items()),
          flush=True)
    for v in errs.values():
        assert v < JET_TOL[precision]
    ctx.close()


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_mixed_assembly_error_vs_oracle(precision):
    """Mixed-precision residual and tangent against the oracle's FP64 assembly
    (the stress and tangent errors of the low-precision network products)."""
    from paper_2604_03411_amd import gedmg as G
    case = small_case(4)
    u, phi, kap = state(case, 45)
    R0, K0, k0 = fem.assemble(fem.Model(case), case.mesh, fem.dof_vector(u, phi), kap)
    ctx = G.Context.from_case(case)
    R, K, kt = ctx.assemble(*ctx.fields(u, phi, kap), precision)
    sync()
    assert ctx.status() == 0
    Kg = to_scipy(ctx, K)
    eR, eK = rel_err(R.cpu().numpy(), R0), rel_err(Kg.data, K0.data)
    ek = rel_err(kt.cpu().numpy(), k0)
    print(f"[mixed assembly vs oracle] {precision}: R {eR:.2e} K {eK:.2e} kappa {ek:.2e}", flush=True)
    assert eR < 10 * JET_TOL[precision] and eK < 10 * JET_TOL[precision] and ek < 10 * JET_TOL[precision]
    ctx.close()


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_mixed_assembly_error_report(precision):
    from paper_2604_03411_amd import gedmg as G
    case = small_case(4)
    u, phi, kap = state(case, 44)
    ctx = G.Context.from_case(case)
    f = ctx.fields(u, phi, kap)
    R0, K0, k0 = [t.clone() for t in ctx.assemble(*f, "fp64")]
    R1, K1, k1 = ctx.assemble(*f, precision)
    sync()
    assert ctx.status() == 0
    eR = rel_err(R1.cpu().numpy(), R0.cpu().numpy())
    eK = rel_err(K1.cpu().numpy(), K0.cpu().numpy())
    ek = rel_err(k1.cpu().numpy(), k0.cpu().numpy())
    print(f"[mixed assembly] {precision}: R {eR:.2e} K {eK:.2e} kappa {ek:.2e}", flush=True)
    assert eR < 10 * JET_TOL[precision] and eK < 10 * JET_TOL[precision]


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_mixed_newton_converges_to_fp64_solution(precision):
    """Mixed-precision tangent with the FP64 residual (iterative refinement):
    the converged load path equals the FP64 path to the Newton tolerance
    (displacement error <= 1e-8), at the price of more Newton iterations."""
    from paper_2604_03411_amd import gedmg as G
    from test_gpu_newton import run_gpu_path
    case = W.make_case(3, n=16)
    case.n_steps = 8

    du = W.uniaxial_increment(case)
    print(f"[mixed newton] notched plate q4 16x16, 4 steps, fp64 vs {precision} vs oracle", flush=True)
    ref = run_gpu_path(G, case, 4, W.uniaxial_bc, precision="fp64", predictor_du=du)
    got = run_gpu_path(G, case, 4, W.uniaxial_bc, precision=precision, predictor_du=du)
    recs = solve.load_path(case, fem.Model(case), steps=4, rtol=0.0, atol=ATOL)
    for (u1, p1, k1, r1), rec in zip(got, recs):
        uo, po = fem.split_dofs(rec["d"], 2)
        eu, ep, ek = rel_err(u1, uo), rel_err(p1, po), rel_err(k1, rec["kappa"])
        er = abs(r1["reaction"] - rec["reaction"]) / abs(rec["reaction"])
        print(f"  vs oracle: u {eu:.2e} phi {ep:.2e} kappa {ek:.2e} reaction {er:.2e}", flush=True)
        assert eu <= 1e-8 and er <= 1e-8 and ep <= 1e-6 and ek <= 1e-6
    for (u0, p0, k0, r0), (u1, p1, k1, r1) in zip(ref, got):
        eu, ep, ek = rel_err(u1, u0), rel_err(p1, p0), rel_err(k1, k0)
        er = abs(r1["reaction"] - r0["reaction"]) / abs(r0["reaction"])
        print(f"  iters fp64 {r0['newton_iters']} {precision} {r1['newton_iters']}: u {eu:.2e} phi {ep:.2e} "
              f"kappa {ek:.2e} reaction {er:.2e}", flush=True)
        assert r1["res_norm"][-1] <= ATOL
        assert eu <= 1e-8 and er <= 1e-8
        # phi and kappa carry the soft uniform-damage mode's amplification
        assert ep <= 1e-6 and ek <= 1e-6


@pytest.mark.parametrize("precision", ["bf16", "fp16"])
def test_mixed_staggered_steps_match_oracle(precision):
    """The staggered scheme (history held in the global solve) with the
    low-precision tangent: the converged states and reactions equal the
    oracle's staggered path; and the closed-form model, whose jet is FP64 in
    every precision, gives the FP64 path's states."""
    from paper_2604_03411_amd import gedmg as G
    from test_gpu_newton import run_gpu_path
    case = W.make_case(3, n=16)
    case.n_steps = 8
    du = W.uniaxial_increment(case)
    print(f"[mixed staggered] notched plate q4 16x16, 4 steps, {precision} vs oracle", flush=True)
    got = run_gpu_path(G, case, 4, W.uniaxial_bc, precision=precision, predictor_du=du, scheme="staggered")
    recs = solve.load_path(case, fem.Model(case), steps=4, rtol=0.0, atol=ATOL, scheme="staggered")
    for (u1, p1, k1, r1), rec in zip(got, recs):
        uo, po = fem.split_dofs(rec["d"], 2)
        eu, ep, ek = rel_err(u1, uo), rel_err(p1, po), rel_err(k1, rec["kappa"])
        er = abs(r1["reaction"] - rec["reaction"]) / abs(rec["reaction"])
        print(f"  vs oracle: u {eu:.2e} phi {ep:.2e} kappa {ek:.2e} reaction {er:.2e}", flush=True)
        assert eu <= 1e-8 and er <= 1e-8 and ep <= 1e-6 and ek <= 1e-6
    plate = W.uniform_plate_case("coarse", n_steps=40, total_disp=40.0)
    ref = run_gpu_path(G, plate, 4, W.symmetric_tension_bc, precision="fp64",
                       predictor_du=W.uniaxial_increment(plate), newton_rscale=0.0)
    low = run_gpu_path(G, plate, 4, W.symmetric_tension_bc, precision=precision,
                       predictor_du=W.uniaxial_increment(plate), newton_rscale=0.0)
    for (u0, p0, k0, r0), (u1, p1, k1, r1) in zip(ref, low):
        print(f"  closed form, {precision} vs fp64: u {rel_err(u1, u0):.2e} kappa {rel_err(k1, k0):.2e} "
              f"(max kappa {k0.max():.4g})", flush=True)
        assert rel_err(u1, u0) <= 1e-9 and rel_err(k1, k0) <= 1e-9


@pytest.mark.parametrize("precision", ["fp64", "bf16", "fp16"])
def test_converged_displacement_heterogeneous_cube_vs_oracle(precision):
    """The converged-displacement error of the 3-D heterogeneous-stretch
    workload on a 6^3 sub-cube: every boundary node (u and phi) prescribed to
    the seeded field, the interior solved by Newton with the FP64 residual and
    the FP64 / BF16 / FP16 tangent, against the oracle's Newton with a direct
    sparse solve.  Both converge to ||R_f|| <= 1e-11."""
    from paper_2604_03411_amd import gedmg as G
    case = W.make_case(4, n=6)
    bd, bv = W.boundary_field_bc(case)
    d, kt, hist, ok = solve.newton(fem.Model(case), case.mesh, fem.dof_vector(case.u, case.phi), case.kappa,
                                   bd, bv, rtol=0.0, atol=ATOL)
    assert ok
    uo, po = fem.split_dofs(d, 3)
    ctx = G.Context.from_case(case)
    u, phi, kap = ctx.fields(case.u, case.phi, case.kappa)
    rep = ctx.newton_step(u, phi, kap, bd, bv, precision, newton_rtol=0.0, newton_atol=ATOL, krylov_rtol=1e-13)
    sync()
    eu, ep = rel_err(u.cpu().numpy(), uo), rel_err(phi.cpu().numpy(), po)
    ek = rel_err(kap.cpu().numpy(), kt)
    print(f"[cube converged u] {precision}: iters {rep['newton_iters']} (oracle {len(hist) - 1}) u {eu:.2e} "
          f"phi {ep:.2e} kappa {ek:.2e}", flush=True)
    assert eu <= 1e-8 and ep <= 1e-6 and ek <= 1e-6
    ctx.close()
