"""Helpers for GPU parity tests: seeded states and conversions (no method arithmetic)."""
import numpy as np
import scipy.sparse as sp
import torch

import workloads as W


def state(case, seed, amp=0.06):
    """A seeded non-trivial state: an affine stretch plus noise, phi ~ U(0, 0.2),
    kappa ~ U(0, 0.1) (the distributions of the single-assembly workloads)."""
    rng = np.random.default_rng(seed)
    m = case.mesh
    A = np.eye(m.dim) * amp + 0.02 * rng.standard_normal((m.dim, m.dim))
    u = A @ m.X + 1e-3 * rng.standard_normal(m.X.shape)
    phi = rng.uniform(0.0, 0.2, m.n_nodes)
    kap = rng.uniform(0.0, 0.1, (m.n_elems, m.nqp))
    return u, phi, kap


def small_case(cfg):
    sizes = {1: dict(), 2: dict(n=6, nz=3), 3: dict(n=24), 4: dict(n=5), 5: dict(n=12)}
    return W.make_case(cfg, **sizes[cfg])


def to_scipy(ctx, K):
    rp, cl = ctx.csr()
    return sp.csr_matrix((K.cpu().numpy(), cl.cpu().numpy(), rp.cpu().numpy()),
                         shape=(ctx.ndof, ctx.ndof))


def rel_err(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def sync():
    torch.cuda.synchronize()
