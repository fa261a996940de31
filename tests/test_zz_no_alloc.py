"""gedmg_assemble_static (the entry point that allocates nothing) against
gedmg_assemble: two calls in a row through the C ABI, the second on a smaller
mesh (the static scratch keeps the first call's contents, so stale data would
show), both bitwise equal to the allocating entry point; meshes above the
static limit are rejected with GEDMG_E_ARG."""
import numpy as np
import pytest
import torch

import workloads as W

from gpu_common import small_case, state, sync

pytestmark = pytest.mark.gpu
E_ARG = -1


def _both(G, case, seed, precision):
    ctx = G.Context.from_case(case)
    u, phi, kap = state(case, seed)
    f = ctx.fields(u, phi, kap)
    ref = [t.clone() for t in ctx.assemble(*f, precision)]
    sync()
    assert ctx.status() == 0
    out = (torch.full((ctx.ndof,), np.nan, dtype=torch.float64, device=ctx.dev),
           torch.full((ctx.nnz,), np.nan, dtype=torch.float64, device=ctx.dev),
           torch.full((ctx.n_elems, ctx.nqp), np.nan, dtype=torch.float64, device=ctx.dev))
    got = ctx.assemble(*f, precision, out=out, static_scratch=True)
    sync()
    assert ctx.status() == 0
    ctx.close()
    return ref, got


@pytest.mark.parametrize("precision", ["fp64", "bf16"])
def test_static_assembly_matches_allocating_assembly_twice(precision):
    from paper_2604_03411_amd import gedmg as G
    big = W.make_case(3, n=48)      # 2296 elements, 9184 points
    small = small_case(4)           # 125 Hex8 elements, 1000 points
    assert big.mesh.n_elems * big.mesh.nqp > small.mesh.n_elems * small.mesh.nqp
    for case, seed in ((big, 71), (small, 72)):
        print(f"[no-alloc] {case.name} reduced: {case.mesh.n_elems} elements, {precision}", flush=True)
        ref, got = _both(G, case, seed, precision)
        for a, b, name in zip(got, ref, ("R", "K", "kappa_trial")):
            assert torch.equal(a, b), name


def test_static_assembly_rejects_meshes_above_the_limit():
    from paper_2604_03411_amd import gedmg as G
    case = W.make_case(2, n=32, nz=9)   # 9216 Hex8 elements = 73 728 points: fits
    ok = W.make_case(1, n=256)          # 65 536 Q4 elements = 262 144 points: exactly the limit
    over = W.make_case(1, n=257)        # 66 049 elements = 264 196 points: above
    assert ok.mesh.n_elems * 4 == G.STATIC_MAX_QP and over.mesh.n_elems * 4 > G.STATIC_MAX_QP
    for c, fits in ((case, True), (ok, True), (over, False)):
        ctx = G.Context.from_case(c)
        # the reference configuration (the seeded noise of the single-assembly
        # workload would invert elements of a 256 x 256 mesh)
        f = ctx.fields(np.zeros_like(c.u), np.zeros_like(c.phi), np.zeros_like(c.kappa))
        print(f"[no-alloc] limit check: {c.mesh.n_elems * c.mesh.nqp} points", flush=True)
        if fits:
            R, K, kt = ctx.assemble(*f, "fp64", tangent=False, static_scratch=True)
            sync()
            assert ctx.status() == 0 and bool(torch.isfinite(R).all())
        else:
            with pytest.raises(G.GedmgError) as e:
                ctx.assemble(*f, "fp64", static_scratch=True)
            assert e.value.code == E_ARG
        ctx.close()
