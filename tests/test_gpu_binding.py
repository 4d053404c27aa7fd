"""The Python binding's stream ordering: a Simulation created on one torch
stream and then driven while another stream is current gives bitwise the
results of one driven on its creation stream (inputs produced on the other
stream are read after they are written, outputs are read after the library
wrote them)."""
import numpy as np
import pytest
import torch

import workloads as W

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_calls_from_another_stream_match_the_creation_stream(precision):
    from paper_2206_11637_amd.sim import Simulation
    wl = W.random_state(40, 19, 9, periodic=(True, False, False), solid_fraction=0.05, seed=11)
    say(f"case: binding, second stream, {precision}")

    def make():
        return Simulation(wl.nx, wl.ny, wl.nz, wl.periodic, precision, "mrt", wl.solid, wl.params)

    ref = make()
    ref.init_equilibrium(wl.phi0, wl.u0, wl.pstar0)
    ref.step(6)
    phi_r, u_r, p_r = ref.moments()
    torch.cuda.synchronize()

    sim = make()
    other = torch.cuda.Stream()
    with torch.cuda.stream(other):
        # inputs produced on the other stream, dropped right after the call
        phi0 = torch.as_tensor(wl.phi0, device=sim.device).mul(1.0)
        u0 = torch.as_tensor(wl.u0, device=sim.device).mul(1.0)
        p0 = torch.as_tensor(wl.pstar0, device=sim.device).mul(1.0)
        sim.init_equilibrium(phi0, u0, p0)
        del phi0, u0, p0
        sim.step(6)
        phi, u, p = sim.moments()
        # consumers on the other stream
        phi2, u2, p2 = phi * 1.0, u * 1.0, p * 1.0
    torch.cuda.synchronize()
    # (the moments are zero in solid cells on both sides)
    same = [torch.equal(a, b) for a, b in ((phi2, phi_r), (u2, u_r), (p2, p_r))]
    say(f"  phi, u, p* bitwise equal: {same}")
    assert all(same)
    assert np.isfinite(sim.reduce()).all()
