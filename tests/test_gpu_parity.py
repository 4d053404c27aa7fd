"""Parity of the HIP path (through the C ABI) with the FP64 oracle."""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as W
from oracle import pflbm as OP

from gpu_util import gpu_pops_oracle_order, normwise, oracle_setup, say

pytestmark = pytest.mark.gpu

TOL64 = 1e-12   # normwise per field after N steps (FP64 path vs FP64 oracle)


STREAMING = ["ab", "aa"]


def _sim(wl, precision="fp64", collision="mrt", streaming="ab"):
    from paper_2206_11637_amd.sim import from_workload
    return from_workload(wl, precision=precision, collision=collision, streaming=streaming)


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


@pytest.mark.parametrize("streaming", STREAMING)
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_capillary_wave_32cube_fp64_matches_oracle_after_200_steps(collision, streaming):
    wl = W.config0()
    say(f"case: capillary wave 32^3 fp64 {collision} {streaming} 200 steps")
    grid, prm, h, g = oracle_setup(wl, collision)
    h, g = OP.run(grid, prm, h, g, wl.steps)
    sim = _sim(wl, "fp64", collision, streaming)
    sim.step(wl.steps)
    _compare_fields(sim, grid, prm, h, g, TOL64, f"config0 {collision} {streaming}")
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
    # several tiles in x and y, interior ones included
    (200, 20, 12, (True, False, True), 0.0, 5),
    (200, 20, 12, (False, False, False), 0.0, 5),
    # walls in x only: every wave takes the FP64 kernel's x-wall fast path,
    # the ragged last tile (130 = 2 x 64 + 2) included
    (130, 12, 10, (False, True, True), 0.0, 6),
]


@pytest.mark.parametrize("streaming", STREAMING)
@pytest.mark.parametrize("case", RAGGED, ids=lambda c: f"{c[0]}x{c[1]}x{c[2]}-p{''.join(str(int(v)) for v in c[3])}-s{c[4]}-n{c[5]}")
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_ragged_grids_walls_and_solids_match_oracle(case, collision, streaming):
    nx, ny, nz, per, frac, steps = case
    wl = W.random_state(nx, ny, nz, periodic=per, solid_fraction=frac, seed=nx * 7 + ny,
                        steps=steps)
    say(f"case: ragged {case} {collision} {streaming}")
    grid, prm, h, g = oracle_setup(wl, collision)
    sim = _sim(wl, "fp64", collision, streaming)
    _compare_fields(sim, grid, prm, h, g, TOL64, "init")
    h, g = OP.run(grid, prm, h, g, steps)
    sim.step(steps)
    assert sim.step_count == steps
    _compare_fields(sim, grid, prm, h, g, TOL64, f"after {steps}")


@pytest.mark.parametrize("streaming", STREAMING)
@pytest.mark.parametrize("s_bulk,tau_L,rho_L", [(1.0, 0.512, 1.0 / 744.0), (1.6, 0.6, 0.05)])
def test_bulk_mode_rate_matches_oracle(s_bulk, tau_L, rho_L, streaming):
    """MRT with the bulk mode of g relaxed at its own rate: FP64 parity on a
    walled ragged grid with solids, at the Taylor-bubble density ratio 744 and
    gas relaxation time (bulk rate 1) and on a milder case (bulk rate 1.6; at
    the Taylor values that rate lets the random start diverge), and BGK
    ignoring the rate (identical to s_bulk = 0)."""
    p = W.Params(tau_H=0.568, tau_L=tau_L, mobility=0.08, xi=3.0, sigma=6.6e-4,
                 rho_L=rho_L, g=(0.0, -1.6e-5, 0.0), s_bulk=s_bulk)
    wl = W.random_state(37, 19, 6, periodic=(False, False, False), params=p,
                        solid_fraction=0.1, seed=41, steps=9)
    say(f"case: bulk rate {s_bulk} {streaming}")
    grid, prm, h, g = oracle_setup(wl, "mrt")
    assert prm.s_bulk == s_bulk
    sim = _sim(wl, "fp64", "mrt", streaming)
    h, g = OP.run(grid, prm, h, g, wl.steps)
    sim.step(wl.steps)
    _compare_fields(sim, grid, prm, h, g, TOL64, f"bulk {s_bulk} after {wl.steps}")
    # the rate changes the result ... (fluid cells: solid slots are never written)
    fl = torch.as_tensor(~wl.solid.reshape(-1), device=sim.device)
    wl0 = dataclasses.replace(wl, params=p.copy(s_bulk=0.0))
    sim0 = _sim(wl0, "fp64", "mrt", streaming)
    sim0.step(wl.steps)
    d = (sim0.populations()[1][:, fl] - sim.populations()[1][:, fl]).abs().max().item()
    assert d > 1e-9, d
    # ... except under BGK, where every moment shares omega(phi) (milder
    # parameters: BGK itself diverges at these within a few steps)
    mild = p.copy(tau_L=0.7, rho_L=0.05)
    a = _sim(dataclasses.replace(wl, params=mild), "fp64", "bgk", streaming)
    b = _sim(dataclasses.replace(wl, params=mild.copy(s_bulk=0.0)), "fp64", "bgk", streaming)
    a.step(wl.steps)
    b.step(wl.steps)
    ga, gb = a.populations()[1][:, fl], b.populations()[1][:, fl]
    assert bool(torch.isfinite(ga).all()) and torch.equal(ga, gb)


@pytest.mark.parametrize("precision,tol_phi", [("fp32", 1e-6), ("fp16s", 2e-4)])
def test_bulk_mode_rate_in_reduced_precision(precision, tol_phi):
    """The bulk rate in the FP32 forms against the FP64 path (capillary wave,
    200 steps, s_bulk = 1)."""
    wl = W.config0()
    wl = dataclasses.replace(wl, params=wl.params.copy(s_bulk=1.0))
    say(f"case: config0 s_bulk=1 {precision} vs fp64")
    ref = _sim(wl, "fp64")
    ref.step(wl.steps)
    sim = _sim(wl, precision)
    sim.step(wl.steps)
    dphi = (sim.phi() - ref.phi()).abs().max().item()
    say(f"  {precision}: max|dphi|={dphi:.2e}")
    assert dphi <= tol_phi


@pytest.mark.parametrize("streaming", STREAMING)
@pytest.mark.parametrize("collision,precision", [("mrt", "fp64"), ("bgk", "fp64"), ("mrt", "fp32")])
def test_buoyant_body_force_matches_oracle(collision, precision, streaming):
    """Gravity on rho - rho_g_ref (rho_g_ref = rho_H: buoyancy only): parity
    with the oracle on a walled ragged grid with solids (FP64 to 1e-12, FP32
    to 1e-5), and the reference changes the result against rho_g_ref = 0."""
    p = W.Params(tau_H=0.6, tau_L=0.7, mobility=0.05, xi=4.0, sigma=5e-4, rho_L=0.05,
                 g=(1e-5, -3e-5, 0.0), rho_g_ref=1.0)
    wl = W.random_state(37, 19, 6, periodic=(False, False, True), params=p,
                        solid_fraction=0.1, seed=53, steps=8, u_amp=0.02)
    say(f"case: buoyant body force {collision} {precision} {streaming}")
    grid = OP.Grid(wl.nx, wl.ny, wl.nz, wl.periodic, wl.solid)
    prm = OP.OracleParams.from_workload(wl.params, collision)
    assert prm.rho_g_ref == 1.0
    h, g = OP.init_equilibrium(grid, wl.phi0, wl.u0, wl.pstar0)
    h, g = OP.run(grid, prm, h, g, wl.steps)
    sim = _sim(wl, precision, collision, streaming)
    sim.step(wl.steps)
    _compare_fields(sim, grid, prm, h, g, TOL64 if precision == "fp64" else 1e-5,
                    f"rho_g_ref {collision} {precision} after {wl.steps}")
    plain = _sim(dataclasses.replace(wl, params=p.copy(rho_g_ref=0.0)), precision, collision,
                 streaming)
    plain.step(wl.steps)
    assert (plain.phi() - sim.phi()).abs().max().item() > 0 or \
        (plain.moments()[1] - sim.moments()[1]).abs().max().item() > 1e-9


@pytest.mark.parametrize("streaming", STREAMING)
@pytest.mark.parametrize("collision,s_bulk", [("mrt", 0.0), ("bgk", 0.0), ("mrt", 1.2)])
def test_full_guo_source_matches_oracle(collision, s_bulk, streaming):
    """Guo's full source for g (forcing="guo"): FP64 parity on a walled ragged
    grid with solids and gravity, with and without a bulk rate."""
    p = W.Params(tau_H=0.6, tau_L=0.7, mobility=0.05, xi=4.0, sigma=5e-4, rho_L=0.05,
                 g=(1e-5, -2e-5, 0.0), s_bulk=s_bulk)
    wl = W.random_state(37, 19, 6, periodic=(False, False, True), params=p,
                        solid_fraction=0.1, seed=43, steps=8, u_amp=0.02)
    say(f"case: guo forcing {collision} s_bulk={s_bulk} {streaming}")
    grid = OP.Grid(wl.nx, wl.ny, wl.nz, wl.periodic, wl.solid)
    prm = OP.OracleParams.from_workload(wl.params, collision, "guo")
    h, g = OP.init_equilibrium(grid, wl.phi0, wl.u0, wl.pstar0)
    from paper_2206_11637_amd.sim import from_workload
    sim = from_workload(wl, precision="fp64", collision=collision, streaming=streaming,
                        forcing="guo")
    h, g = OP.run(grid, prm, h, g, wl.steps)
    sim.step(wl.steps)
    _compare_fields(sim, grid, prm, h, g, TOL64, f"guo {collision} after {wl.steps}")
    # and the source makes a difference against the first-order one
    first = from_workload(wl, precision="fp64", collision=collision, streaming=streaming)
    first.step(wl.steps)
    fl = torch.as_tensor(~wl.solid.reshape(-1), device=sim.device)
    d = (first.populations()[1][:, fl] - sim.populations()[1][:, fl]).abs().max().item()
    assert d > 1e-9, d


@pytest.mark.parametrize("precision,tol_phi", [("fp32", 1e-6), ("fp16s", 2e-4)])
def test_full_guo_source_in_reduced_precision(precision, tol_phi):
    """Guo's full source in the FP32 forms against the FP64 path (capillary
    wave, 200 steps)."""
    from paper_2206_11637_amd.sim import from_workload
    wl = W.config0()
    say(f"case: config0 guo {precision} vs fp64")
    ref = from_workload(wl, precision="fp64", forcing="guo")
    ref.step(wl.steps)
    sim = from_workload(wl, precision=precision, forcing="guo")
    sim.step(wl.steps)
    dphi = (sim.phi() - ref.phi()).abs().max().item()
    say(f"  {precision}: max|dphi|={dphi:.2e}")
    assert dphi <= tol_phi


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
@pytest.mark.parametrize("periodic", [(True, False, True), (False, False, False)])
def test_an_all_fluid_mask_changes_nothing_bitwise(precision, periodic):
    """The masked kernel variants (solid neighbour bits read per cell) with a
    mask that marks no solid give bit for bit the results of the unmasked
    variants, on a lattice of several tiles in x and y."""
    wl = W.random_state(264, 28, 13, periodic=periodic, solid_fraction=0.0, seed=8, steps=7)
    say(f"case: all-fluid mask vs no mask {precision} periodic={periodic}")
    a = _sim(wl, precision)
    b = _sim(dataclasses.replace(wl, solid=np.zeros((wl.nz, wl.ny, wl.nx), dtype=bool)),
             precision)
    a.step(wl.steps)
    b.step(wl.steps)
    ha, ga = a.populations()
    hb, gb = b.populations()
    assert torch.equal(ha, hb) and torch.equal(ga, gb)
    assert torch.equal(a.phi(), b.phi())


@pytest.mark.parametrize("streaming", STREAMING)
def test_zero_steps_and_resume_are_bitwise(streaming):
    wl = W.random_state(70, 21, 13, periodic=(True, False, True), solid_fraction=0.05, seed=4)
    say(f"case: resume 70x21x13 {streaming}")
    a = _sim(wl, "fp64", streaming=streaming)
    h0, g0 = a.populations()
    a.step(0)
    h1, g1 = a.populations()
    assert torch.equal(h0, h1) and torch.equal(g0, g1)
    a.step(5)
    buf = a.save_state()
    a.step(6)
    ha, ga = a.populations()
    b = _sim(wl, "fp64", streaming=streaming)
    b.load_state(buf, 5)
    b.step(6)
    hb, gb = b.populations()
    assert torch.equal(ha, hb) and torch.equal(ga, gb)
    # FP16 storage resumes bitwise too
    c = _sim(wl, "fp16s", streaming=streaming)
    c.step(3)
    buf = c.save_state()
    c.step(4)
    hc, _ = c.populations()
    d = _sim(wl, "fp16s", streaming=streaming)
    d.load_state(buf, 3)
    d.step(4)
    hd, _ = d.populations()
    assert torch.equal(hc, hd)


@pytest.mark.parametrize("streaming", STREAMING)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_translation_invariance_is_bitwise(precision, streaming):
    wl = W.random_state(70, 12, 9, periodic=(True, True, True), seed=8)
    say(f"case: translation {precision} {streaming}")
    sx, sy, sz = 5, 3, 2
    rolled = W.Workload(wl.name, wl.nx, wl.ny, wl.nz, wl.periodic, wl.params,
                        np.roll(wl.phi0, (sz, sy, sx), (0, 1, 2)),
                        np.roll(wl.u0, (sz, sy, sx), (1, 2, 3)),
                        np.roll(wl.pstar0, (sz, sy, sx), (0, 1, 2)), None, wl.steps)
    a, b = _sim(wl, precision, streaming=streaming), _sim(rolled, precision, streaming=streaming)
    a.step(7)
    b.step(7)
    pa, _, _ = a.moments()
    pb, _, _ = b.moments()
    assert torch.equal(torch.roll(pa, (sz, sy, sx), (0, 1, 2)), pb)


@pytest.mark.parametrize("streaming", STREAMING)
def test_mass_conserved_on_gpu_all_precisions(streaming):
    wl = W.config4(scale=8)   # tube mask, walls
    say(f"case: mass conservation taylor tube /8 {streaming}")
    # FP32 and FP16 storage keep h shifted (w_i phi of the reader), so the
    # rounding acts on the deviations: measured 9e-11 and 4e-7 over 100 steps
    for precision, tol in (("fp64", 1e-13), ("fp32", 1e-9), ("fp16s", 1e-5)):
        sim = _sim(wl, precision, streaming=streaming)
        r0 = sim.reduce()
        sim.step(100)
        r1 = sim.reduce()
        drift = abs(r1[0] - r0[0]) / abs(r0[0])
        say(f"  {precision}: relative mass drift over 100 steps {drift:.2e}")
        assert drift <= tol


@pytest.mark.parametrize("streaming", STREAMING)
@pytest.mark.parametrize("precision,tol_phi", [("fp32", 1e-6), ("fp16s", 2e-4)])
def test_reduced_precision_forms_track_fp64(precision, tol_phi, streaming):
    """FP32 and FP16-storage forms against the FP64 path on the capillary
    wave after 200 steps (measured max|dphi| 7.6e-8 FP32, 4.2e-5 FP16
    storage; the bounds leave a margin of ~5-10x)."""
    wl = W.config0()
    say(f"case: config0 {precision} {streaming} vs fp64")
    ref = _sim(wl, "fp64")
    ref.step(wl.steps)
    sim = _sim(wl, precision, streaming=streaming)
    sim.step(wl.steps)
    pr, ur, _ = ref.moments()
    p, u, _ = sim.moments()
    dphi = (p - pr).abs().max().item()
    du = (u - ur).abs().max().item() / max(ur.abs().max().item(), 1e-30)
    say(f"  {precision}: max|dphi|={dphi:.2e} max|du|/max|u|={du:.2e}")
    assert dphi <= tol_phi


def _unstable_case():
    p = W.Params(tau_H=0.5001, tau_L=0.5001, mobility=0.02, xi=4.0, sigma=1e-3, rho_L=1e-3)
    return W.random_state(40, 24, 8, periodic=(True, True, True), params=p, u_amp=0.3, seed=77)


def test_unstable_run_is_reported_not_silent():
    """tau -> 1/2 with large velocities and density ratio 1000 blows up (the
    oracle does too, see test_oracle_invariants); with a check interval the
    step call stops with PFLBM_ERR_UNSTABLE and names the step."""
    from paper_2206_11637_amd._lib import PFLBM_ERR_UNSTABLE, PFLBMError
    say("case: unstable run")
    sim = _sim(_unstable_case(), "fp32")
    sim.set_check_interval(5)
    with pytest.raises(PFLBMError) as e:
        sim.step(400)
    assert e.value.status == PFLBM_ERR_UNSTABLE
    assert "after step" in str(e.value)
    assert 0 < sim.step_count <= 400 and sim.step_count % 5 == 0
    # a stable run with the same check interval goes through
    ok = _sim(W.random_state(40, 24, 8, seed=5), "fp32")
    ok.set_check_interval(5)
    ok.step(50)
    assert ok.step_count == 50


def _split_state(buf, N, precision):
    """Saved-state bytes -> (h, g, phi[, phi_prev]) as integer views (bitwise
    comparison); layout h[15][N], g[27][N], phi^n[N] and, for the shifted
    forms (FP32, FP16 storage), phi^{n-1}[N]."""
    ss, rs = {"fp64": (8, 8), "fp32": (4, 4), "fp16s": (2, 4)}[precision]
    it = {2: torch.int16, 4: torch.int32, 8: torch.int64}
    o1, o2, o3 = 15 * N * ss, 42 * N * ss, 42 * N * ss + N * rs
    parts = [buf[:o1].view(it[ss]).reshape(15, N), buf[o1:o2].view(it[ss]).reshape(27, N),
             buf[o2:o3].view(it[rs])]
    if precision != "fp64":
        parts.append(buf[o3:o3 + N * rs].view(it[rs]))
    assert buf.numel() == o3 + (N * rs if precision != "fp64" else 0)
    return parts


@pytest.mark.parametrize("streaming", STREAMING)
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
def test_out_of_place_step_between_saved_states_is_bitwise(precision, streaming):
    """pflbm_step_states (used by checkpoint recompute) equals the in-place
    step over several steps, with walls and solids.  Solid cells' population
    slots and shift references are never written by a step (nor read),
    so only fluid cells are compared there."""
    wl = W.random_state(70, 21, 13, periodic=(True, False, True), solid_fraction=0.05, seed=9)
    say(f"case: step_states {precision} {streaming}")
    sim = _sim(wl, precision, streaming=streaming)
    N = wl.nx * wl.ny * wl.nz
    fluid = torch.from_numpy(~np.asarray(wl.solid, dtype=bool).reshape(-1)).to(sim.device)
    assert 0 < int(fluid.sum()) < N
    sim.step(3)
    bufs = [sim.save_state()]
    for n in range(3, 7):
        nxt = torch.full_like(bufs[-1], 0xFF)
        sim.step_states(bufs[-1], nxt, n)
        bufs.append(nxt)
        sim.step(1)
        ref = sim.save_state()
        a, b = _split_state(nxt, N, precision), _split_state(ref, N, precision)
        assert torch.equal(a[0][:, fluid], b[0][:, fluid]), ("h", n)
        assert torch.equal(a[1][:, fluid], b[1][:, fluid]), ("g", n)
        assert torch.equal(a[2], b[2]), ("phi", n)
        if precision != "fp64":   # the shift reference is defined on fluid cells
            assert torch.equal(a[3][fluid], b[3][fluid]), ("phi_prev", n)


@pytest.mark.parametrize("precision", ["fp32", "fp16s"])
def test_waves_without_own_cells_read_their_ring_after_the_pulls_land(precision):
    """Regression test for the pipelined FP32 step's direct-to-LDS pulls: in a
    lattice with ny = 4k + 1 the last row of tiles has three waves whose own
    cells all lie outside the lattice but which still form ring cells, and
    with 40 planes in chunks of 4 every chunk starts with such a read.  The
    step must wait for the pulls in those waves too; then the two-buffer step
    equals the in-place step (which pulls into registers) bitwise."""
    wl = W.random_state(70, 21, 40, periodic=(True, False, True), solid_fraction=0.02, seed=31)
    say(f"case: outside rows, AB vs AA {precision}")
    a, b = _sim(wl, precision, streaming="ab"), _sim(wl, precision, streaming="aa")
    for n in (3, 4):
        a.step(n)
        b.step(n)
        for x, y in zip(a.moments(), b.moments()):
            assert torch.equal(x, y)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
def test_both_streaming_schemes_give_identical_results(precision):
    """The two-buffer fused step and the in-place AA step do the same
    arithmetic on the same values (phi summed in the same order, the same
    reader-referenced shifts), so their moments and populations agree
    bitwise, for both parities, with walls and solids."""
    wl = W.random_state(70, 21, 13, periodic=(True, False, True), solid_fraction=0.05, seed=21)
    say(f"case: AB vs AA {precision}")
    a, b = _sim(wl, precision, streaming="ab"), _sim(wl, precision, streaming="aa")
    for n in (5, 2):
        a.step(n)
        b.step(n)
        for x, y in zip(a.moments(), b.moments()):
            assert torch.equal(x, y)
        for x, y in zip(a.populations(), b.populations()):
            assert torch.equal(x, y)


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
def test_chained_state_steps_fill_every_phase_field(precision):
    """The checkpoint recompute's chain (each step writes the phi it forms into
    the state it read and skips the next state's gather; the last one gathers)
    leaves every state identical to one saved from the running context."""
    from paper_2206_11637_amd._lib import (PFLBMError, STATES_SKIP_DST_PHI,
                                           STATES_WRITE_SRC_PHI)
    wl = W.random_state(70, 21, 13, periodic=(True, False, True), solid_fraction=0.05, seed=10)
    say(f"case: chained step_states {precision}")
    sim = _sim(wl, precision)
    N = wl.nx * wl.ny * wl.nz
    fluid = torch.from_numpy(~np.asarray(wl.solid, dtype=bool).reshape(-1)).to(sim.device)
    sim.step(2)
    states = [sim.save_state()]
    refs = [states[0].clone()]
    for n in range(2, 6):
        states.append(torch.full_like(states[0], 0xFF))
        flags = STATES_WRITE_SRC_PHI | (STATES_SKIP_DST_PHI if n < 5 else 0)
        sim.step_states(states[-2], states[-1], n, flags)
        sim.step(1)
        refs.append(sim.save_state())
    for k, (a, b) in enumerate(zip(states, refs)):
        a, b = _split_state(a, N, precision), _split_state(b, N, precision)
        assert torch.equal(a[0][:, fluid], b[0][:, fluid]), ("h", k)
        assert torch.equal(a[1][:, fluid], b[1][:, fluid]), ("g", k)
        assert torch.equal(a[2][fluid], b[2][fluid]), ("phi", k)
        if precision != "fp64":
            assert torch.equal(a[3][fluid], b[3][fluid]), ("phi_prev", k)
    aa = _sim(wl, precision, streaming="aa")
    buf = aa.save_state()
    with pytest.raises(PFLBMError):
        aa.step_states(buf, torch.empty_like(buf), 0, STATES_WRITE_SRC_PHI)
