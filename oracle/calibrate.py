"""Calibration of the energy scale mu_e for the seeded networks (oracle; test
infrastructure only).

The paper treats mu_e as a factor with units of stress that scales a
non-dimensional network energy (Sec. 4.2.1, after Eq. dd_0).  With the
seeded raw parameters the network's reference-state slopes are large and
seed-dependent, so each workload fixes mu_e such that the initial shear
modulus of psi_e equals the Neo-Hookean value E / (2 (1 + nu)) of the plate
study (E = 210 MPa, nu = 0.3).  For a simple shear of amount g at J = 1,
I1G - 3 = g^2 and I2G - 3 = 3 g^2 + O(g^4), so psi_e = mu_e (N_1 + 3 N_2) g^2
+ O(g^4) and the shear modulus is 2 mu_e (N_1 + 3 N_2), N_i = dN/dx_i at 0.

Running this module prints the literals stored in `workloads.MU_E`.
"""
from __future__ import annotations

import torch

from .icnn import ICNN


def shear_slope(theta, spec) -> float:
    net = ICNN(torch.as_tensor(theta, dtype=torch.float64), spec.n_in, spec.width,
               spec.n_hidden, spec.monotone_mask)
    x0 = torch.zeros(1, 3, dtype=torch.float64, requires_grad=True)
    (g,) = torch.autograd.grad(net(x0).sum(), x0)
    return float(2.0 * (g[0, 0] + 3.0 * g[0, 1]))


def calibrated_mu(theta, spec, shear_modulus) -> float:
    return shear_modulus / shear_slope(theta, spec)


if __name__ == "__main__":  # pragma: no cover
    import workloads as W

    G = W._E / (2.0 * (1.0 + W._NU))
    for cfg in (1, 2, 3, 4, 5):
        c = W.make_case(cfg, n=2, nz=1)
        print(cfg, repr(calibrated_mu(c.theta_e, c.energy, G)))
