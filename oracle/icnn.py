"""Input-convex neural networks (oracle; test infrastructure only).

The paper parameterises the isochoric energy psi_iso(I1G, I2G) and the
damage yield function N_kappa(q) with ICNNs (Sec. 4.2.1, citing Amos et al.).
The architecture is not printed; the reading used here (also by the GPU
path) is the standard ICNN with input pass-through:

    z_1     = s(W0 x + b0)
    z_{k+1} = s(Wz_k z_k + Wx_k x + b_k),        k = 1 .. L-1
    N(x)    = wz . z_L + wx . x + b_out

with s = softplus.  Convexity in x needs Wz_k >= 0 and wz >= 0; they are the
softplus of raw parameters.  Weights multiplying input i (the i-th column of
W0 and Wx_k, and wx[i]) are raw unless bit i of `monotone_mask` is set, in
which case they are softplus'd too; the yield network sets it for its single
input q so that N_kappa is increasing (Sec. 4.2.1, "increasing function").

Raw parameter order: W0 (row-major, width x n_in), b0; then for every
hidden->hidden layer Wz (width x width), Wx (width x n_in), b; then wz,
wx, b_out.
"""
from __future__ import annotations

import torch


class _Logistic(torch.autograd.Function):
    """logistic(t) = 1/(1+exp(-t)); derivative logistic(t) logistic(-t).

    Written as a Function so that every derivative order is exact at t = 0
    (a piecewise formula through |t| would lose the kink's derivative).
    """

    @staticmethod
    def forward(ctx, t):
        e = torch.exp(-t.abs())
        s = torch.where(t >= 0, 1.0 / (1.0 + e), e / (1.0 + e))
        ctx.save_for_backward(t)
        return s

    @staticmethod
    def backward(ctx, g):
        (t,) = ctx.saved_tensors
        return g * logistic(t) * logistic(-t)


class _Softplus(torch.autograd.Function):
    """softplus(t) = log(1 + exp(t)) = max(t, 0) + log1p(exp(-|t|))."""

    @staticmethod
    def forward(ctx, t):
        ctx.save_for_backward(t)
        return torch.clamp(t, min=0.0) + torch.log1p(torch.exp(-t.abs()))

    @staticmethod
    def backward(ctx, g):
        (t,) = ctx.saved_tensors
        return g * logistic(t)


def logistic(t):
    return _Logistic.apply(t)


def softplus(t):
    return _Softplus.apply(t)


def n_params(n_in: int, width: int, n_hidden: int) -> int:
    h = width
    return h * n_in + h + (n_hidden - 1) * (h * h + h * n_in + h) + h + n_in + 1


class ICNN:
    """Callable ICNN built from a raw parameter tensor (kept in the autograd
    graph, so derivatives with respect to the raw parameters are available)."""

    def __init__(self, theta: torch.Tensor, n_in: int, width: int, n_hidden: int,
                 monotone_mask: int = 0):
        assert theta.numel() == n_params(n_in, width, n_hidden)
        self.theta = theta
        self.n_in, self.width, self.n_hidden = n_in, width, n_hidden
        self.mask = torch.tensor([(monotone_mask >> i) & 1 == 1 for i in range(n_in)])
        h, n = width, n_in
        off = 0

        def take(cnt, shape):
            nonlocal off
            t = theta[off:off + cnt].reshape(shape)
            off += cnt
            return t

        def passthrough(w):  # columns of monotone inputs become non-negative
            return torch.where(self.mask, softplus(w), w)

        self.W0 = passthrough(take(h * n, (h, n)))
        self.b0 = take(h, (h,))
        self.hidden = []
        for _ in range(n_hidden - 1):
            Wz = softplus(take(h * h, (h, h)))
            Wx = passthrough(take(h * n, (h, n)))
            b = take(h, (h,))
            self.hidden.append((Wz, Wx, b))
        self.wz = softplus(take(h, (h,)))
        self.wx = passthrough(take(n, (n,)))
        self.b_out = take(1, ())
        assert off == theta.numel()

    def __call__(self, x: torch.Tensor) -> torch.Tensor:
        """x: [B, n_in] -> N(x): [B]."""
        z = softplus(x @ self.W0.T + self.b0)
        for Wz, Wx, b in self.hidden:
            z = softplus(z @ Wz.T + x @ Wx.T + b)
        return z @ self.wz + x @ self.wx + self.b_out
