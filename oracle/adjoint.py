"""Reverse-mode gradients of the oracle rollout, by torch autograd.

Test infrastructure only (see oracle/__init__.py).

The loss follows the wave-amplitude reading of the paper's elevation probe
(sec. gravity-wave setup: the column sum of the fill level at x = 0):
    a(n)  = < sum_y phi^n(x0, y, z) >_z - depth
    L     = sum_{s=1..S} (a(s K) - target_s)^2 ,   N = S K steps.
Gradients are taken with respect to the mobility M, the surface tension
sigma, the interface width xi (through the counter-term 4 phi (1 - phi)/xi
and the chemical potential's beta = 12 sigma/xi and kappa = 3 sigma xi/2;
phi0 itself is an input, so a phi0 built from xi adds its own term) and the
initial phase field phi0 (cell by cell), with u0 and p*0 held fixed.  Autograd differentiates the oracle's own forward step, so this
adjoint is exact for the oracle up to rounding.
"""
from __future__ import annotations

import dataclasses

import torch

from . import pflbm as P


def rollout_trace(grid: P.Grid, prm: P.OracleParams, phi0: torch.Tensor, u0, pstar0,
                  nsteps: int, sample_every: int, depth: float, x0: int = 0):
    """Amplitude samples a(sample_every), a(2 sample_every), ..., a(nsteps)."""
    h, g = P.init_equilibrium(grid, phi0, u0, pstar0, prm.phase_lattice)
    out = []
    for n in range(1, nsteps + 1):
        h, g = P.step(grid, prm, h, g)
        if n % sample_every == 0:
            out.append(P.amplitude(grid, h, depth, x0))
    return torch.stack(out)


def gradients(grid: P.Grid, prm: P.OracleParams, phi0, u0, pstar0, nsteps: int,
              sample_every: int, depth: float, target, x0: int = 0) -> dict:
    """L, dL/dphi0 [N], dL/dM, dL/dsigma, dL/dxi and the trace, in float64."""
    M = torch.tensor(float(prm.mobility), dtype=torch.float64, requires_grad=True)
    s = torch.tensor(float(prm.sigma), dtype=torch.float64, requires_grad=True)
    xi = torch.tensor(float(prm.xi), dtype=torch.float64, requires_grad=True)
    phi = torch.as_tensor(phi0, dtype=torch.float64).reshape(-1).clone().requires_grad_(True)
    p = dataclasses.replace(prm, mobility=M, sigma=s, xi=xi)
    trace = rollout_trace(grid, p, phi, u0, pstar0, nsteps, sample_every, depth, x0)
    target = torch.as_tensor(target, dtype=torch.float64)
    L = ((trace - target) ** 2).sum()
    dphi, dM, ds, dxi = torch.autograd.grad(L, (phi, M, s, xi), allow_unused=True)
    zero = torch.zeros((), dtype=torch.float64)
    return dict(L=L.detach(), dphi0=dphi, dM=dM.item(), dsigma=ds.item(),
                dxi=(dxi if dxi is not None else zero).item(), trace=trace.detach())


def loss_and_gradients(grid: P.Grid, prm: P.OracleParams, phi0, u0, pstar0, nsteps: int,
                       sample_every: int, depth: float, target, x0: int = 0):
    """Returns (L, dL/dphi0 [N], dL/dM, dL/dsigma, trace) in float64."""
    r = gradients(grid, prm, phi0, u0, pstar0, nsteps, sample_every, depth, target, x0)
    return r["L"], r["dphi0"], r["dM"], r["dsigma"], r["trace"]


def loss_only(grid, prm, phi0, u0, pstar0, nsteps, sample_every, depth, target, x0=0):
    with torch.no_grad():
        trace = rollout_trace(grid, prm, torch.as_tensor(phi0, dtype=torch.float64).reshape(-1),
                              u0, pstar0, nsteps, sample_every, depth, x0)
        return ((trace - torch.as_tensor(target, dtype=torch.float64)) ** 2).sum().item()
