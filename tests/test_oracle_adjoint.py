"""Pin of the oracle's reverse mode against central finite differences (FP64):
dL/dM, dL/dsigma, dL/dxi (the interface width, through the counter-term and
the chemical potential) and dL/dphi0 along random directions."""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as AD
from oracle import pflbm as P


def _case(collision):
    wl = W.capillary_wave(8, 12, 3, depth=6.0, amplitude=0.8, xi=3.0, noise=1e-6,
                          params=W.Params(tau_H=0.6, tau_L=0.7, mobility=0.05, sigma=2e-3,
                                          rho_L=0.05, g=(0.0, -1e-5, 0.0)))
    grid = P.Grid(wl.nx, wl.ny, wl.nz, wl.periodic, wl.solid)
    prm = P.OracleParams.from_workload(wl.params, collision)
    return wl, grid, prm


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_autograd_gradients_match_central_differences(collision):
    wl, grid, prm = _case(collision)
    n, K = 12, 3
    rng = np.random.default_rng(2)
    target = rng.normal(0, 0.05, n // K)
    args = (wl.u0, wl.pstar0, n, K, 6.0, target)
    r = AD.gradients(grid, prm, wl.phi0, *args)
    dphi, dM, ds, dxi = r["dphi0"], r["dM"], r["dsigma"], r["dxi"]
    for name, val, grad in (("mobility", prm.mobility, dM), ("sigma", prm.sigma, ds),
                            ("xi", prm.xi, dxi)):
        hstep = 1e-4 * val
        lp = AD.loss_only(grid, dataclasses.replace(prm, **{name: val + hstep}), wl.phi0, *args)
        lm = AD.loss_only(grid, dataclasses.replace(prm, **{name: val - hstep}), wl.phi0, *args)
        fd = (lp - lm) / (2 * hstep)
        assert abs(fd - grad) <= 1e-6 * abs(grad) + 1e-14, (name, fd, grad)
    # directional derivative along random directions of phi0
    for k in range(2):
        d = rng.standard_normal(wl.phi0.shape)
        eps = 1e-6
        lp = AD.loss_only(grid, prm, wl.phi0 + eps * d, *args)
        lm = AD.loss_only(grid, prm, wl.phi0 - eps * d, *args)
        fd = (lp - lm) / (2 * eps)
        ad = float((dphi.numpy() * d.reshape(-1)).sum())
        assert abs(fd - ad) <= 1e-6 * abs(ad) + 1e-14, (fd, ad)
