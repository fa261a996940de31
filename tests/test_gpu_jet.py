"""Energy-network jet kernel vs autograd of the oracle network.

Raw parameters are drawn with std 1.5 so that the softplus'd weights vary
widely (a permuted lane layout or a wrong neuron index changes the result at
O(1)); widths 16/32/64 and depths 1..3; a ragged number of points.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle.icnn import ICNN

from gpu_common import rel_err, sync

pytestmark = pytest.mark.gpu


def oracle_jet(theta, spec, x):
    net = ICNN(torch.tensor(theta), 3, spec.width, spec.n_hidden, spec.monotone_mask)
    xt = torch.tensor(x, requires_grad=True)
    N = net(xt)
    N0 = net(torch.zeros(1, 3, dtype=torch.float64))[0]
    (g,) = torch.autograd.grad(N.sum(), xt, create_graph=True)
    H = torch.stack([torch.autograd.grad(g[:, i].sum(), xt, retain_graph=True)[0] for i in range(3)], 1)
    out = np.zeros((x.shape[0], 10))
    out[:, 0] = (N - N0).detach().numpy()
    out[:, 1:4] = g.detach().numpy()
    Hn = H.detach().numpy()
    out[:, 4], out[:, 5], out[:, 6] = Hn[:, 0, 0], Hn[:, 1, 1], Hn[:, 2, 2]
    out[:, 7], out[:, 8], out[:, 9] = Hn[:, 0, 1], Hn[:, 0, 2], Hn[:, 1, 2]
    return out


@pytest.mark.parametrize("width,depth", [(16, 1), (16, 2), (32, 2), (32, 3), (64, 2), (64, 3)])
def test_fp64_jet_matches_autograd(width, depth):
    from paper_2604_03411_amd import gedmg as G
    print(f"[jet] width {width} depth {depth}", flush=True)
    case = W.make_case(1, n=2)
    spec = W.NetSpec(3, width, depth, 3)
    rng = np.random.default_rng(width * 10 + depth)
    theta = rng.normal(0.0, 1.5, spec.n_params)
    ctx = G.Context(case.mesh, case.material, spec, theta, case.yield_, case.theta_y)
    x = rng.uniform(-0.3, 0.6, (1000 + width - 7, 3))
    jet = ctx.energy_jet(torch.tensor(x, device=ctx.dev)).cpu().numpy()
    sync()
    ref = oracle_jet(theta, spec, x)
    for name, sl in (("value", [0]), ("grad", [1, 2, 3]), ("hessian", list(range(4, 10)))):
        e = rel_err(jet[:, sl], ref[:, sl])
        print(f"  {name}: rel err {e:.2e}", flush=True)
        assert e <= 1e-12, (name, e)
    ctx.close()


@pytest.mark.parametrize("width,depth", [(16, 1), (64, 3)])
def test_fp64_jet_increment_keeps_relative_precision(width, depth):
    """At |x| = 1e-8 the jet value N(x) - N(0) must carry relative precision:
    it is compared with the second-order Taylor expansion at 0 built from the
    oracle's autograd gradient and Hessian there (the third-order remainder is
    about 1e-16 of the first-order term).  A value formed by subtracting N(0)
    from N(x) would be off by about 1e-16 |N(0)| / (|grad N(0)| |x|) ~ 1e-8."""
    from paper_2604_03411_amd import gedmg as G
    print(f"[jet increment] width {width} depth {depth}", flush=True)
    case = W.make_case(1, n=2)
    spec = W.NetSpec(3, width, depth, 3)
    rng = np.random.default_rng(100 + width + depth)
    theta = rng.normal(0.0, 1.5, spec.n_params)
    ctx = G.Context(case.mesh, case.material, spec, theta, case.yield_, case.theta_y)
    dirs = rng.normal(size=(517, 3))
    x = 1e-8 * dirs / np.linalg.norm(dirs, axis=1, keepdims=True)
    jet = ctx.energy_jet(torch.tensor(x, device=ctx.dev)).cpu().numpy()
    sync()
    ref0 = oracle_jet(theta, spec, np.zeros((1, 3)))[0]
    g0 = ref0[1:4]
    H0 = np.array([[ref0[4], ref0[7], ref0[8]], [ref0[7], ref0[5], ref0[9]], [ref0[8], ref0[9], ref0[6]]])
    taylor = x @ g0 + 0.5 * np.einsum("ni,ij,nj->n", x, H0, x)
    scale = np.linalg.norm(g0) * np.linalg.norm(x, axis=1)
    e = float(np.max(np.abs(jet[:, 0] - taylor) / scale))
    print(f"  max |N(x) - N(0) - taylor| / (|g0| |x|) = {e:.2e}", flush=True)
    assert e <= 1e-11, e
    ctx.close()
