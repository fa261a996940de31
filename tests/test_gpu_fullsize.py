"""Full-size parity: the 64^3 Hex8 assembly (262144 elements, 2097152 qp, the
workload and launch configuration that bench.py times) against the oracle on
sampled outputs.

The oracle cannot assemble the whole cube in seconds, so nodes are sampled
(interior, face, edge and corner nodes) and the oracle evaluates every element
that touches a sampled node; the rows of the sampled nodes are then complete
and are compared with the same rows of the GPU's global R and CSR K, and the
updated history of those elements with the GPU's kappa_trial.  Tolerance as in
the small-mesh parity tests: 1e-12 norm-wise per output.
"""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fem

from gpu_common import rel_err, sync

pytestmark = pytest.mark.gpu
TOL = 1e-12


def test_full_size_cube_sampled_rows_match_oracle():
    from paper_2604_03411_amd import gedmg as G
    case = W.make_case(4)
    m = case.mesh
    print(f"[full-size parity] hex8 64^3: {m.n_elems} elements, {m.n_nodes} nodes", flush=True)
    ctx = G.Context.from_case(case)
    R, K, kt = ctx.assemble(*ctx.fields(case.u, case.phi, case.kappa), "fp64")
    sync()
    assert ctx.status() == 0
    rng = np.random.default_rng(2024)
    n1 = 65  # nodes per edge
    corner = [0, n1 - 1, n1 * n1 - 1, m.n_nodes - 1]
    edge = [n1 // 2, n1 * (n1 // 2), n1 * n1 * (n1 // 2)]
    face = [n1 * n1 * (n1 // 2) + n1 // 2, n1 * (n1 // 3) + n1 // 3]
    nodes = np.unique(np.concatenate([corner, edge, face, rng.integers(0, m.n_nodes, 24)]))
    conn = np.asarray(m.conn)
    elems = np.nonzero(np.isin(conn, nodes).any(axis=1))[0]
    print(f"  {nodes.size} sampled nodes, {elems.size} elements evaluated by the oracle", flush=True)
    d = fem.dof_vector(case.u, case.phi)
    geo, Re, Ke, kap, _ = fem.element_response(fem.Model(case), m, d, case.kappa, elems, True)
    nd = m.dim + 1
    rows = (nodes[:, None] * nd + np.arange(nd)[None, :]).ravel()
    R_ref = np.zeros(m.ndof)
    np.add.at(R_ref, geo.edofs.ravel(), Re.numpy().ravel())
    # oracle rows of K restricted to the sampled rows, as {row: {col: value}}
    Kd = {}
    row_set = set(rows.tolist())
    Ke_n = Ke.numpy()
    for e in range(geo.edofs.shape[0]):
        ed = geo.edofs[e]
        for i, r in enumerate(ed):
            if r in row_set:
                dr = Kd.setdefault(int(r), {})
                for j, cdof in enumerate(ed):
                    dr[int(cdof)] = dr.get(int(cdof), 0.0) + Ke_n[e, i, j]
    rp, cl = ctx.csr()
    rp_h = rp.cpu().numpy()
    idx = np.concatenate([np.arange(rp_h[r], rp_h[r + 1]) for r in rows])
    idx_t = torch.as_tensor(idx, device=K.device)
    K_rows = K[idx_t].cpu().numpy()
    C_rows = cl[idx_t].cpu().numpy()
    K_ref = []
    pos = 0
    for r in rows:
        n = rp_h[r + 1] - rp_h[r]
        cols = C_rows[pos:pos + n]
        assert set(cols.tolist()) == set(Kd[int(r)].keys()), f"pattern of row {r}"
        K_ref.append([Kd[int(r)][int(c)] for c in cols])
        pos += n
    K_ref = np.concatenate(K_ref)
    R_g = R[torch.as_tensor(rows, device=R.device)].cpu().numpy()
    kt_g = kt[torch.as_tensor(elems, device=kt.device)].cpu().numpy()
    eR = rel_err(R_g, R_ref[rows])
    eK = rel_err(K_rows, K_ref)
    ek = rel_err(kt_g, kap.numpy())
    print(f"  rel err R {eR:.2e} K {eK:.2e} kappa {ek:.2e} over {rows.size} rows / {K_rows.size} entries",
          flush=True)
    assert eR <= TOL and eK <= TOL and ek <= TOL
    ctx.close()
