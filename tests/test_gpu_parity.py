"""Parity of the HIP path (through the C ABI) with the FP64 oracle."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import pflbm as OP

from gpu_util import gpu_pops_oracle_order, normwise, oracle_setup, say

pytestmark = pytest.mark.gpu

TOL64 = 1e-12   # normwise per field after N steps (FP64 path vs FP64 oracle)


def _sim(wl, precision="fp64", collision="mrt"):
    from paper_2206_11637_amd.sim import from_workload
    return from_workload(wl, precision=precision, collision=collision)


def _compare_fields(sim, grid, prm, h, g, tol, label):
    hg, gg = gpu_pops_oracle_order(sim)
    phi_o, u_o, p_o = OP.moments(grid, prm, h, g)
    phi, u, p = sim.moments()
    errs = dict(h=normwise(hg, h), g=normwise(gg, g), phi=normwise(phi.reshape(-1), phi_o),
                u=normwise(u.reshape(3, -1), u_o), pstar=normwise(p.reshape(-1), p_o))
    say(f"{label}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= tol, (label, k, v)
    return errs


@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_capillary_wave_32cube_fp64_matches_oracle_after_200_steps(collision):
    wl = W.config0()
    say(f"case: capillary wave 32^3 fp64 {collision} 200 steps")
    grid, prm, h, g = oracle_setup(wl, collision)
    h, g = OP.run(grid, prm, h, g, wl.steps)
    sim = _sim(wl, "fp64", collision)
    sim.step(wl.steps)
    _compare_fields(sim, grid, prm, h, g, TOL64, f"config0 {collision}")
    r = sim.reduce()
    ro = OP.reductions(grid, h, g).numpy()
    assert abs(r[0] - ro[0]) <= 1e-12 * abs(ro[0])
    assert np.abs(r[1:] - ro[1:]).max() <= 1e-12 * max(1.0, np.abs(ro[1:]).max())


RAGGED = [
    # (nx, ny, nz, periodic, solid_fraction, steps)
    (70, 21, 13, (True, False, True), 0.05, 7),
    (70, 21, 13, (True, False, True), 0.05, 8),
    (37, 9, 6, (False, False, False), 0.1, 5),
    (17, 33, 5, (True, True, True), 0.0, 6),
    (1, 24, 1, (True, False, True), 0.0, 9),
    (40, 3, 1, (True, True, True), 0.0, 4),
]


@pytest.mark.parametrize("case", RAGGED, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}-p{''.join(str(int(v)) for v in c[3])}-s{c[4]}-n{c[5]}")
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_ragged_grids_walls_and_solids_match_oracle(case, collision):
    nx, ny, nz, per, frac, steps = case
    wl = W.random_state(nx, ny, nz, periodic=per, solid_fraction=frac, seed=nx * 7 + ny,
                        steps=steps)
    say(f"case: ragged {case} {collision}")
    grid, prm, h, g = oracle_setup(wl, collision)
    sim = _sim(wl, "fp64", collision)
    _compare_fields(sim, grid, prm, h, g, TOL64, "init")
    h, g = OP.run(grid, prm, h, g, steps)
    sim.step(steps)
    assert sim.step_count == steps
    _compare_fields(sim, grid, prm, h, g, TOL64, f"after {steps}")


def test_zero_steps_and_resume_are_bitwise():
    wl = W.random_state(70, 21, 13, periodic=(True, False, True), solid_fraction=0.05, seed=4)
    say("case: resume 70x21x13")
    a = _sim(wl, "fp64")
    h0, g0 = a.populations()
    a.step(0)
    h1, g1 = a.populations()
    assert torch.equal(h0, h1) and torch.equal(g0, g1)
    a.step(5)
    buf = a.save_state()
    a.step(6)
    ha, ga = a.populations()
    b = _sim(wl, "fp64")
    b.load_state(buf, 5)
    b.step(6)
    hb, gb = b.populations()
    assert torch.equal(ha, hb) and torch.equal(ga, gb)
    # FP16 storage resumes bitwise too
    c = _sim(wl, "fp16s")
    c.step(3)
    buf = c.save_state()
    c.step(4)
    hc, _ = c.populations()
    d = _sim(wl, "fp16s")
    d.load_state(buf, 3)
    d.step(4)
    hd, _ = d.populations()
    assert torch.equal(hc, hd)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_translation_invariance_is_bitwise(precision):
    wl = W.random_state(70, 12, 9, periodic=(True, True, True), seed=8)
    say(f"case: translation {precision}")
    sx, sy, sz = 5, 3, 2
    rolled = W.Workload(wl.name, wl.nx, wl.ny, wl.nz, wl.periodic, wl.params,
                        np.roll(wl.phi0, (sz, sy, sx), (0, 1, 2)),
                        np.roll(wl.u0, (sz, sy, sx), (1, 2, 3)),
                        np.roll(wl.pstar0, (sz, sy, sx), (0, 1, 2)), None, wl.steps)
    a, b = _sim(wl, precision), _sim(rolled, precision)
    a.step(7)
    b.step(7)
    pa, _, _ = a.moments()
    pb, _, _ = b.moments()
    assert torch.equal(torch.roll(pa, (sz, sy, sx), (0, 1, 2)), pb)


def test_mass_conserved_on_gpu_all_precisions():
    wl = W.config4(scale=8)   # tube mask, walls
    say("case: mass conservation taylor tube /8")
    for precision, tol in (("fp64", 1e-13), ("fp32", 2e-6), ("fp16s", 1e-3)):
        sim = _sim(wl, precision)
        r0 = sim.reduce()
        sim.step(100)
        r1 = sim.reduce()
        drift = abs(r1[0] - r0[0]) / abs(r0[0])
        say(f"  {precision}: relative mass drift over 100 steps {drift:.2e}")
        assert drift <= tol


@pytest.mark.parametrize("precision,tol_phi", [("fp32", 1e-4), ("fp16s", 5e-2)])
def test_reduced_precision_forms_track_fp64(precision, tol_phi):
    """FP32 and FP16-storage forms against the FP64 path on the capillary
    wave (errors reported; bounds set from the rounding units)."""
    wl = W.config0()
    say(f"case: config0 {precision} vs fp64")
    ref = _sim(wl, "fp64")
    ref.step(wl.steps)
    sim = _sim(wl, precision)
    sim.step(wl.steps)
    pr, ur, _ = ref.moments()
    p, u, _ = sim.moments()
    dphi = (p - pr).abs().max().item()
    du = (u - ur).abs().max().item() / max(ur.abs().max().item(), 1e-30)
    say(f"  {precision}: max|dphi|={dphi:.2e} max|du|/max|u|={du:.2e}")
    assert dphi <= tol_phi
