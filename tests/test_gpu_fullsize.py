"""Full-size workloads in the launch configuration the benchmark times:
one-step parity with the oracle on sampled windows, plus invariants."""
import numpy as np
import pytest
import torch

import workloads as W

from gpu_util import perm_to_oracle, say, window_check

pytestmark = pytest.mark.gpu


def _sampled_check(wl, precision, warm, centres, tol_h, tol_g, collision="mrt", streaming="ab",
                   phase="d3q15"):
    from paper_2206_11637_amd.sim import from_workload
    say(f"case: {wl.name} {precision} {streaming} {phase} warm {warm}")
    sim = from_workload(wl, precision=precision, collision=collision, streaming=streaming,
                        phase_lattice=phase)
    r0 = sim.reduce()
    sim.step(warm)
    h_n, g_n = sim.populations()
    sim.step(1)
    h_n1, g_n1 = sim.populations()
    r1 = sim.reduce()
    perms = (torch.as_tensor(perm_to_oracle(sim.q_h, phase)), torch.as_tensor(perm_to_oracle(27, phase)))
    eh, eg, n = window_check(sim, wl, collision, h_n, g_n, h_n1, g_n1, centres, perms=perms)
    say(f"  {precision}: window errors h={eh:.2e} g={eg:.2e} over {n} cells; "
        f"mass drift {(r1[0] - r0[0]) / r0[0]:.2e}")
    assert n > 0
    assert eh <= tol_h and eg <= tol_g
    return sim


def test_rising_bubble_fp32_full_size_windows():
    wl = W.config1()
    centres = [(64, 64, 64), (64 + 16, 64, 64), (3, 2, 100), (127, 511, 0), (40, 300, 90)]
    _sampled_check(wl, "fp32", 40, centres, 2e-5, 2e-5)


def test_rising_bubble_fp32_in_place_full_size_windows():
    wl = W.config1()
    centres = [(64, 64, 64), (127, 0, 127), (20, 400, 30)]
    _sampled_check(wl, "fp32", 41, centres, 2e-5, 2e-5, streaming="aa")


def test_rising_bubble_fp64_full_size_windows():
    wl = W.config1()
    centres = [(64, 64 + 16, 64), (0, 0, 0), (100, 500, 127)]
    _sampled_check(wl, "fp64", 21, centres, 1e-12, 1e-12)


def test_rising_bubble_fp16_storage_full_size_windows():
    wl = W.config1()
    centres = [(64, 64 + 16, 64), (127, 0, 0), (30, 450, 100)]
    _sampled_check(wl, "fp16s", 20, centres, 2e-3, 2e-3)


def test_drop_impact_fp16_storage_full_size_windows():
    wl = W.config2()
    centres = [(192, 100, 192), (192 + 30, 136, 192), (10, 0, 380), (200, 383, 5)]
    # FP16 storage rounds every stored population (relative 2^-11 of the
    # shifted value); the bound below is a few units of that on h ~ 0.2
    _sampled_check(wl, "fp16s", 20, centres, 2e-3, 2e-3)


def test_rising_bubble_d3q27_phase_fp32_full_size_windows():
    """The D3Q27-phase build (the bench's FP32 D3Q27 form, k_step with 27 h)."""
    wl = W.config1()
    centres = [(64, 64, 64), (0, 511, 127), (90, 250, 40)]
    _sampled_check(wl, "fp32", 20, centres, 2e-5, 2e-5, phase="d3q27")


def test_drop_impact_fp32_full_size_windows():
    """The pipelined FP32 step on the 384^3 drop (the bench's FP32 drop form)."""
    wl = W.config2()
    centres = [(192, 100, 192), (192 + 30, 136, 192), (10, 0, 380), (383, 383, 0)]
    _sampled_check(wl, "fp32", 20, centres, 2e-5, 2e-5)


def test_drop_impact_slab_fp32_windows_across_the_periodic_z_faces():
    """One GPU's z-slab of the drop, 384 x 384 x 48 (the bench's shard form,
    z periodic where the slab exchange would be): windows on both z faces,
    which wrap, and inside the slab."""
    wl2 = W.config2()
    z0 = 192 - 24
    shard = W.Workload("drop_impact_shard_384x384x48", 384, 384, 48, (True, False, True), wl2.params,
                       wl2.phi0[z0:z0 + 48].copy(), wl2.u0[:, z0:z0 + 48].copy(),
                       wl2.pstar0[z0:z0 + 48].copy(), None, wl2.steps)
    del wl2
    centres = [(192, 100, 0), (192 + 20, 136, 47), (5, 200, 24)]
    _sampled_check(shard, "fp32", 10, centres, 2e-5, 2e-5)


def test_taylor_bubble_tube_mask_full_size_windows():
    wl = W.config4()
    centres = [(64, 120, 64), (64 + 42, 320, 64), (64, 1023, 5 + 4), (64 + 59, 500, 64)]
    _sampled_check(wl, "fp32", 11, centres, 2e-5, 2e-5)
