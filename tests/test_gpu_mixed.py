"""Mixed-precision (BF16 / FP16 matrix-core) energy-network jets and assembly
vs FP64.  Parity for mixed precision is not fixed by the paper; it is pinned
to the FP64 path: the low-precision products carry the operand rounding of
the format (2^-9 for BF16, 2^-12 for FP16), so the jets are checked at a few
times that unit, and the assembled residual / tangent errors are reported."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.icnn import ICNN

from gpu_common import rel_err, small_case, state, sync, to_scipy

pytestmark = pytest.mark.gpu
JET_TOL = {"bf16": 3e-2, "fp16": 4e-3}


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
    from test_gpu_newton import ATOL, run_gpu_path
    case = W.make_case(3, n=16)
    case.n_steps = 8

    def guess(n, u_prev):
        return W.uniaxial_predictor(case, u_prev, n)

    print(f"[mixed newton] notched plate q4 16x16, 4 steps, fp64 vs {precision}", flush=True)
    ref = run_gpu_path(G, case, 4, W.uniaxial_bc, guess, "fp64")
    got = run_gpu_path(G, case, 4, W.uniaxial_bc, guess, precision)
    for (u0, p0, k0, r0), (u1, p1, k1, r1) in zip(ref, got):
        eu, ep, ek = rel_err(u1, u0), rel_err(p1, p0), rel_err(k1, k0)
        er = abs(r1["reaction"] - r0["reaction"]) / abs(r0["reaction"])
        print(f"  iters fp64 {r0['newton_iters']} {precision} {r1['newton_iters']}: u {eu:.2e} phi {ep:.2e} "
              f"kappa {ek:.2e} reaction {er:.2e}", flush=True)
        assert r1["res_norm"][-1] <= ATOL
        assert eu <= 1e-8 and er <= 1e-8
        # phi and kappa carry the soft uniform-damage mode's amplification
        assert ep <= 1e-6 and ek <= 1e-6
