"""GPU load-path adjoint (gedmg_adjoint) against the oracle's discrete
adjoint, against central differences of the GPU loss, and for the
checkpointing invariants, on a reduced adjoint workload (notched Q4 8x8
plate, widths 32, three loading steps and one unloading step).

Conditioning sets the attainable agreement with the oracle.  The gradient is
a sensitive function of the converged nonlocal damage field: a change of the
converged state moves the oracle's own gradient by about 2e4 times as much
(relative to its largest entry).  Both sides converge every step to an
absolute residual of 1e-12, and the soft uniform-damage mode turns that
into a state difference of 6e-12 (beta_d = 10) or 6e-10 (the workload's
penalty beta_d = 1000) in phi, so the gradients are compared at 1e-6 and
1e-3 respectively.

The GPU loss carries about 1e-9 relative noise from the converged states, so
central differences use a step of 1e-3 max(1, |theta|) (at 1e-5 the noise
dominates the quotient).
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fem, solve

from gpu_common import rel_err, sync

pytestmark = pytest.mark.gpu
ATOL = 1e-12
OPTS = dict(newton_rtol=0.0, newton_atol=ATOL, krylov_rtol=1e-13)


@pytest.fixture(scope="module")
def G():
    from paper_2604_03411_amd import gedmg
    return gedmg


# Load levels (multiples of the per-step increment): three loading steps, then
# partial unloading, so that the adjoint passes both the yielding branch and
# the elastic branch that carries the history adjoint backwards.
LEVELS = (1.0, 2.0, 3.0, 2.5)


def small_adjoint_case(n=8, beta_d=None):
    """Adjoint workload on a Q4 n x n plate with a notch at the left-edge
    midpoint (radius 0.2), widths 32, per-step increment of the 20-step path
    times 5."""
    c = W.make_case(5, n=n)
    c.mesh = W.remove_elements_near(W.q4_grid(n, n), (0.0, 0.5), 0.2)
    c.u = np.zeros((2, c.mesh.n_nodes))
    c.phi = np.zeros(c.mesh.n_nodes)
    c.kappa = np.zeros((c.mesh.n_elems, c.mesh.nqp))
    c.n_steps = len(LEVELS)
    if beta_d is not None:
        c.material = dict(c.material, beta_d=beta_d)
    return c


def path_bc(case, n):
    d, v = W.uniaxial_bc(case, n)
    return d, np.where(v != 0.0, v / n * LEVELS[n - 1], v)


def path_increment(case, n):
    prev = LEVELS[n - 2] if n > 1 else 0.0
    return W.uniaxial_increment(case) * (LEVELS[n - 1] - prev)


def oracle_path(case, theta_e=None, theta_y=None):
    m = fem.Model(case, theta_e, theta_y) if theta_e is not None else fem.Model(case)
    return solve.load_path(case, m, steps=case.n_steps, bc_fn=path_bc,
                           predictor_fn=lambda c, u, n: u + path_increment(c, n), rtol=0.0, atol=ATOL)


def oracle_targets(case):
    """Reactions of the perturbed-weight forward run (the oracle's)."""
    recs = oracle_path(case, case.extra["theta_e_star"], case.extra["theta_y_star"])
    return np.array([r["reaction"] for r in recs])


def make_path(G, case, targets):
    steps = case.n_steps
    du = np.stack([path_increment(case, n) for n in range(1, steps + 1)])
    bcs = [path_bc(case, n) for n in range(1, steps + 1)]
    return G.LoadPath(case.u, case.phi, case.kappa, bcs, W.reaction_dofs(case), targets,
                      predictor_du=du, **OPTS)


def _setup(G, beta_d):
    case = small_adjoint_case(beta_d=beta_d)
    targets = oracle_targets(case)
    recs = oracle_path(case)
    assert [bool((r["kappa"] > r["kappa_prev"]).any()) for r in recs] == [True, True, True, False]
    loss_o, ge_o, gy_o = solve.loss_and_gradient(case, recs, targets)
    ctx = G.Context.from_case(case)
    path = make_path(G, case, targets)
    return case, ctx, path, (loss_o, ge_o, gy_o, recs)


@pytest.fixture(scope="module")
def setup(G):
    s = _setup(G, None)
    yield s
    s[1].close()


@pytest.fixture(scope="module")
def setup_wc(G):
    s = _setup(G, 10.0)
    yield s
    s[1].close()


def _compare(setup, tol_grad, tol_loss):
    case, ctx, path, (loss_o, ge_o, gy_o, recs) = setup
    print(f"[adjoint parity] q4 {case.mesh.n_elems} elems, {path.n_steps} steps, beta_d "
          f"{case.material['beta_d']}, checkpoint 2", flush=True)
    loss, ge, gy, rep = ctx.adjoint(path, checkpoint_every=2)
    sync()
    scale = max(np.abs(ge_o).max(), np.abs(gy_o).max())
    e_l = abs(loss - loss_o) / loss_o
    e_e = np.abs(ge - ge_o).max() / scale
    e_y = np.abs(gy - gy_o).max() / scale
    print(f"  loss {loss:.10e} oracle {loss_o:.10e} rel {e_l:.2e}; grad err energy {e_e:.2e} yield {e_y:.2e}; "
          f"recomputed {rep['recomputed_steps']} krylov {rep['krylov_iters_total']}", flush=True)
    assert loss_o > 0
    assert e_l <= tol_loss and e_e <= tol_grad and e_y <= tol_grad
    # the end state is the forward path's end state
    u, phi, kap = rep["state"]
    uo, po = fem.split_dofs(recs[-1]["d"], 2)
    assert rel_err(u.cpu().numpy(), uo) < 1e-7
    assert rel_err(kap.cpu().numpy(), recs[-1]["kappa"]) < 1e-6


def test_adjoint_matches_oracle_well_conditioned(G, setup_wc):
    _compare(setup_wc, 1e-6, 1e-8)


def test_adjoint_matches_oracle_workload_penalty(G, setup):
    _compare(setup, 1e-3, 1e-6)


def test_output_bias_gradients_are_zero(G, setup):
    case, ctx, path, _ = setup
    _, ge, gy, _ = ctx.adjoint(path, checkpoint_every=2)
    assert ge[-1] == 0.0 and gy[-1] == 0.0


def test_checkpointing_is_bitwise_store_all(G, setup):
    case, ctx, path, _ = setup
    ref = ctx.adjoint(path, checkpoint_every=path.n_steps)
    assert ref[3]["recomputed_steps"] == 0 and ref[3]["n_checkpoints"] == 1
    for ce, n_re in ((1, path.n_steps - 1), (3, 3), (2, 2)):
        out = ctx.adjoint(path, checkpoint_every=ce)
        print(f"  checkpoint_every {ce}: recomputed {out[3]['recomputed_steps']}", flush=True)
        assert out[3]["recomputed_steps"] == n_re
        assert out[0] == ref[0]
        assert np.array_equal(out[1], ref[1]) and np.array_equal(out[2], ref[2])
        for a, b in zip(out[3]["state"], ref[3]["state"]):
            assert torch.equal(a, b)


def test_adjoint_matches_central_differences(G, setup_wc):
    """20 random raw parameters (none of the cancelling output biases)."""
    case, ctx, path, _ = setup_wc
    loss, ge, gy, _ = ctx.adjoint(path, checkpoint_every=2)
    rng = np.random.default_rng(21)
    picks = [("e", j) for j in rng.choice(case.energy.n_params - 1, 10, replace=False)]
    picks += [("y", j) for j in rng.choice(case.yield_.n_params - 1, 10, replace=False)]
    scale = max(np.abs(ge).max(), np.abs(gy).max())
    worst = 0.0
    for which, j in picks:
        th = case.theta_e if which == "e" else case.theta_y
        h = 1e-3 * max(1.0, abs(th[j]))
        vals = []
        for sgn in (1, -1):
            te, ty = case.theta_e.copy(), case.theta_y.copy()
            (te if which == "e" else ty)[j] += sgn * h
            ctx.set_params(te, ty)
            vals.append(ctx.adjoint(path, checkpoint_every=path.n_steps)[0])
        fd = (vals[0] - vals[1]) / (2 * h)
        g = (ge if which == "e" else gy)[j]
        worst = max(worst, abs(fd - g) / scale)
        assert abs(fd - g) <= 1e-6 * scale + 1e-5 * abs(g), (which, j, fd, g)
    ctx.set_params(case.theta_e, case.theta_y)
    print(f"  central differences: worst |fd - g| / max|g| = {worst:.2e}", flush=True)


def test_load_path_loss_autograd(G, setup):
    case, ctx, path, _ = setup
    te = torch.tensor(case.theta_e, dtype=torch.float64, requires_grad=True)
    ty = torch.tensor(case.theta_y, dtype=torch.float64, requires_grad=True)
    loss = G.load_path_loss(ctx, te, ty, path, checkpoint_every=2)
    (2.0 * loss).backward()
    l2, ge, gy, _ = ctx.adjoint(path, checkpoint_every=2)
    assert float(loss) == l2
    assert np.array_equal(te.grad.numpy(), 2.0 * ge) and np.array_equal(ty.grad.numpy(), 2.0 * gy)
