"""Invariants of the HIP path (through the C ABI) that the method fixes
without any reference solution: a fluid at rest stays at rest, and without
forcing the total momentum and the pressure sum are conserved."""
import dataclasses
import math

import numpy as np
import pytest
import torch

import workloads as W

from gpu_util import say

pytestmark = pytest.mark.gpu


def _uniform(phi, xi=4.0, periodic=(True, False, True), solid=True):
    p = W.Params(tau_H=0.6, tau_L=0.8, mobility=0.05, xi=xi, sigma=1e-3, rho_L=0.01)
    wl = W.random_state(40, 21, 9, periodic=periodic, params=p, solid_fraction=0.08 if solid else 0.0,
                        seed=3)
    phi0 = np.where(wl.solid, 0.0, phi) if solid else np.full_like(wl.phi0, phi)
    return dataclasses.replace(wl, phi0=phi0, u0=np.zeros_like(wl.u0), pstar0=np.zeros_like(wl.pstar0))


@pytest.mark.parametrize("streaming", ["ab", "aa"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
@pytest.mark.parametrize("phi,xi", [(0.0, 4.0), (1.0, 4.0), (0.3, math.inf)])
def test_fluid_at_rest_stays_at_rest(phi, xi, precision, streaming):
    """Uniform phi at rest with walls and solids (the counter-term off for the
    intermediate value, where the Allen-Cahn flux would otherwise separate the
    phases from rounding): populations unchanged after 9 steps.  Bitwise for
    the shifted forms (their deviations are exactly zero) and for phi = 0;
    FP64 otherwise to rounding (sum_i w_i of the FP64 weights is 1 only to
    rounding, so phi = sum h is not exactly 1 or 0.3)."""
    from paper_2206_11637_amd.sim import from_workload
    wl = _uniform(phi, xi)
    say(f"case: rest phi={phi} xi={xi} {precision} {streaming}")
    sim = from_workload(wl, precision=precision, streaming=streaming)
    h0, g0 = sim.populations()
    sim.step(9)
    h1, g1 = sim.populations()
    if precision == "fp64" and phi != 0.0:
        assert (h1 - h0).abs().max().item() <= 1e-15 and (g1 - g0).abs().max().item() <= 1e-15
    else:
        assert torch.equal(h0, h1) and torch.equal(g0, g1)
    _, u, _ = sim.moments()
    assert u.abs().max().item() <= (1e-15 if precision == "fp64" else 0.0)


@pytest.mark.parametrize("streaming", ["ab", "aa"])
def test_momentum_and_pressure_sums_conserved_without_forcing(streaming):
    """sigma = 0, g = 0, rho_H = rho_L (so F_s = F_b = F_p = F_mu = 0), fully
    periodic, random phase field and velocities: sum p* and sum j = sum c g
    are conserved (FP64), and the phase mass too."""
    from paper_2206_11637_amd.sim import from_workload
    p = W.Params(tau_H=0.6, tau_L=0.9, mobility=0.05, xi=4.0, sigma=0.0, rho_H=1.0, rho_L=1.0,
                 g=(0.0, 0.0, 0.0))
    wl = W.random_state(37, 20, 11, periodic=(True, True, True), params=p, u_amp=0.02, seed=17)
    say(f"case: momentum {streaming}")
    sim = from_workload(wl, precision="fp64", streaming=streaming)
    r0 = sim.reduce()
    _, u, _ = sim.moments()
    scale = u.abs().sum().item()          # sum |j| (no force: u = j)
    sim.step(50)
    r1 = sim.reduce()
    say(f"  sum phi {r0[0]:.6e} -> {r1[0]:.6e}; sum p* {r0[1]:.3e} -> {r1[1]:.3e}; "
        f"sum j {r0[2:]} -> {r1[2:]} (sum |j| {scale:.3e})")
    assert abs(r1[0] - r0[0]) <= 1e-13 * abs(r0[0])
    assert abs(r1[1] - r0[1]) <= 1e-13 * max(1.0, abs(r0[1]))
    assert np.abs(r1[2:] - r0[2:]).max() <= 1e-13 * scale
    assert scale > 10.0   # the test has momentum to conserve
