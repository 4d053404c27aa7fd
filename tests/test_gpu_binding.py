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


def test_fp16_scale_is_fixed_once_the_state_exists():
    """With FP16 storage the populations are stored scaled by 2^k: after
    initialisation a different k is refused (state error, nothing changed),
    the same k is accepted, and a new initialisation may use a new k."""
    from paper_2206_11637_amd import _lib
    from paper_2206_11637_amd.sim import from_workload
    wl = W.random_state(24, 12, 6, periodic=(True, False, True), seed=4)
    say("case: binding, fp16 scale after init")
    sim = from_workload(wl, precision="fp16s")
    sim.step(2)
    before = sim.reduce()
    with pytest.raises(_lib.PFLBMError) as e:
        sim.set_params(wl.params.copy(fp16_scale_log2=(10.0, 12.0)))
    assert e.value.status == _lib.PFLBM_ERR_STATE and "fp16_scale_log2" in str(e.value)
    assert np.array_equal(sim.reduce(), before)
    sim.set_params(wl.params)                       # same scale: fine
    sim2 = from_workload(wl, precision="fp16s", params=wl.params.copy(fp16_scale_log2=(10.0, 12.0)))
    sim2.step(2)
    assert np.isfinite(sim2.reduce()).all()


def test_binding_refuses_short_or_mistyped_buffers():
    """Buffers of the wrong length, dtype or size are refused by the binding
    with ValueError before the library sees them (no kernel reads them)."""
    from paper_2206_11637_amd.sim import from_workload
    wl = W.random_state(16, 8, 4, periodic=(True, False, True), seed=6)
    say("case: binding, buffer refusals")
    sim = from_workload(wl, precision="fp32")
    dev = sim.device
    with pytest.raises(ValueError):
        sim.init_equilibrium(np.zeros(sim.N - 1))
    with pytest.raises(ValueError):
        sim.init_equilibrium(wl.phi0, np.zeros(sim.N))          # u0 needs 3 N values
    with pytest.raises(ValueError):
        sim.phi(out=torch.empty(sim.N, dtype=torch.float32, device=dev))
    with pytest.raises(ValueError):
        sim.save_state(torch.empty(sim.state_bytes() - 1, dtype=torch.uint8, device=dev))
    with pytest.raises(ValueError):
        sim.load_state(torch.empty(16, dtype=torch.uint8, device=dev), 0)
    buf = sim.save_state()
    with pytest.raises(ValueError):
        sim.step_states(buf, torch.empty(8, dtype=torch.uint8, device=dev), 0)
    sim.step(1)
    assert np.isfinite(sim.reduce()).all()
