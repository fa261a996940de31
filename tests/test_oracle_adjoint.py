"""Pin of the oracle's discrete adjoint against central finite differences of
the load-path loss (the loss is re-evaluated by full Newton solves)."""
import numpy as np

import workloads as W
from oracle import fem, solve


def _path(case, te, ty, steps):
    m = fem.Model(case, te, ty)
    return solve.load_path(case, m, steps=steps, rtol=0.0, atol=1e-13)


def test_adjoint_matches_central_differences():
    c = W.make_case(5, n=3)
    c.n_steps = 4
    steps = 3
    recs = _path(c, c.theta_e, c.theta_y, steps)
    targets = [0.9 * r["reaction"] for r in recs]
    loss, ge, gy = solve.loss_and_gradient(c, recs, targets)
    assert loss > 0
    # the output biases cancel in N(x) - N(0) and N^(q): exactly zero gradient
    assert ge[-1] == 0.0 and gy[-1] == 0.0
    rng = np.random.default_rng(9)
    picks = [("e", j) for j in rng.choice(c.energy.n_params - 1, 4, replace=False)]
    picks += [("y", j) for j in rng.choice(c.yield_.n_params - 1, 4, replace=False)]
    for which, j in picks:
        th = c.theta_e if which == "e" else c.theta_y
        # the soft uniform-phi mode leaves ~1e-9 relative noise in converged
        # states, so the step must be large enough to dominate it
        h = 1e-3 * max(1.0, abs(th[j]))
        vals = []
        for sgn in (1, -1):
            te, ty = c.theta_e.copy(), c.theta_y.copy()
            (te if which == "e" else ty)[j] += sgn * h
            rr = _path(c, te, ty, steps)
            vals.append(sum((r["reaction"] - t) ** 2 for r, t in zip(rr, targets)))
        fd = (vals[0] - vals[1]) / (2 * h)
        g = (ge if which == "e" else gy)[j]
        scale = max(np.abs(ge).max(), np.abs(gy).max())
        assert abs(fd - g) <= 1e-4 * scale + 1e-3 * abs(g), (which, j, fd, g)
