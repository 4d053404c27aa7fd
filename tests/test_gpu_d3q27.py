"""The D3Q27-phase build (libpflbm_d3q27.so: the velocity set the paper uses for
both lattices in 3D) through the C ABI: FP64 parity with the oracle run with
the same phase lattice, both streaming schemes, the FP32 forms against FP64,
phase mass, and the reverse mode against the oracle's autograd."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import adjoint as AD
from oracle import pflbm as OP

from gpu_util import gpu_pops_oracle_order, normwise, say

pytestmark = pytest.mark.gpu

TOL64 = 1e-12
PHASE = "d3q27"


def _sim(wl, precision="fp64", collision="mrt", streaming="ab"):
    from paper_2206_11637_amd.sim import from_workload
    sim = from_workload(wl, precision=precision, collision=collision, streaming=streaming,
                        phase_lattice=PHASE)
    assert sim.q_h == 27
    return sim


def _oracle(wl, collision):
    grid = OP.Grid(wl.nx, wl.ny, wl.nz, wl.periodic, wl.solid)
    prm = OP.OracleParams.from_workload(wl.params, collision, phase_lattice=PHASE)
    h, g = OP.init_equilibrium(grid, wl.phi0, wl.u0, wl.pstar0, PHASE)
    return grid, prm, h, g


def _compare(sim, grid, prm, h, g, label):
    hg, gg = gpu_pops_oracle_order(sim)
    phi_o, u_o, p_o = OP.moments(grid, prm, h, g)
    phi, u, p = sim.moments()
    errs = dict(h=normwise(hg, h), g=normwise(gg, g), phi=normwise(phi.reshape(-1), phi_o),
                u=normwise(u.reshape(3, -1), u_o), pstar=normwise(p.reshape(-1), p_o))
    say(f"{label}: " + " ".join(f"{k}={v:.2e}" for k, v in errs.items()))
    for k, v in errs.items():
        assert v <= TOL64, (label, k, v)


@pytest.mark.parametrize("streaming", ["ab", "aa"])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_capillary_wave_fp64_matches_oracle(collision, streaming):
    wl = W.config0()
    say(f"case: d3q27 capillary wave 32^3 fp64 {collision} {streaming} 200 steps")
    grid, prm, h, g = _oracle(wl, collision)
    h, g = OP.run(grid, prm, h, g, wl.steps)
    sim = _sim(wl, "fp64", collision, streaming)
    sim.step(wl.steps)
    _compare(sim, grid, prm, h, g, f"d3q27 config0 {collision} {streaming}")


@pytest.mark.parametrize("streaming", ["ab", "aa"])
@pytest.mark.parametrize("case", [(37, 9, 6, (False, False, False), 0.1, 5),
                                  (70, 21, 13, (True, False, True), 0.05, 7)],
                         ids=["walls-solids", "ragged-tiles"])
def test_ragged_grids_walls_and_solids_match_oracle(case, streaming):
    nx, ny, nz, per, frac, steps = case
    wl = W.random_state(nx, ny, nz, periodic=per, solid_fraction=frac, seed=nx * 7 + ny,
                        steps=steps)
    say(f"case: d3q27 ragged {case} {streaming}")
    grid, prm, h, g = _oracle(wl, "mrt")
    sim = _sim(wl, "fp64", "mrt", streaming)
    _compare(sim, grid, prm, h, g, "init")
    h, g = OP.run(grid, prm, h, g, steps)
    sim.step(steps)
    _compare(sim, grid, prm, h, g, f"after {steps}")


@pytest.mark.parametrize("precision,tol_phi,tol_mass", [("fp32", 1e-6, 1e-9),
                                                        ("fp16s", 2e-4, 1e-5)])
def test_reduced_precision_forms_track_fp64(precision, tol_phi, tol_mass):
    """Capillary wave 32^3, 200 steps: FP32 and FP16 storage against FP64 and
    their phase mass (the shifted storage carries over to 27 h)."""
    wl = W.config0()
    say(f"case: d3q27 config0 {precision} vs fp64")
    ref = _sim(wl, "fp64")
    ref.step(wl.steps)
    sim = _sim(wl, precision)
    m0 = sim.reduce()[0]
    sim.step(wl.steps)
    dphi = (sim.phi() - ref.phi()).abs().max().item()
    drift = abs(sim.reduce()[0] - m0) / abs(m0)
    say(f"  {precision}: max|dphi|={dphi:.2e} mass drift {drift:.1e}")
    assert dphi <= tol_phi
    assert drift <= tol_mass


@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
def test_both_streaming_schemes_give_identical_results(precision):
    wl = W.random_state(40, 19, 9, periodic=(True, False, False), solid_fraction=0.05, seed=9)
    say(f"case: d3q27 ab vs aa {precision}")
    a, b = _sim(wl, precision, streaming="ab"), _sim(wl, precision, streaming="aa")
    a.step(7)
    b.step(7)
    fl = torch.as_tensor(~wl.solid.reshape(-1), device=a.device)
    ha, ga = a.populations()
    hb, gb = b.populations()
    assert torch.equal(ha[:, fl], hb[:, fl]) and torch.equal(ga[:, fl], gb[:, fl])


def test_fp64_adjoint_matches_oracle_autograd():
    from paper_2206_11637_amd.rollout import amplitude_rollout
    from paper_2206_11637_amd.sim import Simulation
    wl = W.capillary_wave(16, 24, 6, depth=12.0, amplitude=1.5, xi=4.0, noise=1e-6,
                          params=W.Params(tau_H=0.6, tau_L=0.7, mobility=0.05, sigma=2e-3,
                                          rho_L=0.05, g=(0.0, -1e-5, 0.0)))
    nsteps, K = 18, 3
    target = np.random.default_rng(5).normal(0, 0.05, nsteps // K)
    say("case: d3q27 adjoint fp64 mrt N=18 ckpt=4")
    grid, prm, _, _ = _oracle(wl, "mrt")
    Lo, dphio, dMo, dso, _ = AD.loss_and_gradients(grid, prm, wl.phi0, wl.u0, wl.pstar0, nsteps,
                                                   K, 12.0, target)
    sim = Simulation(wl.nx, wl.ny, wl.nz, wl.periodic, "fp64", "mrt", wl.solid, wl.params,
                     phase_lattice=PHASE)
    dev = sim.device
    phi0 = torch.tensor(wl.phi0, dtype=torch.float64, device=dev, requires_grad=True)
    Mt = torch.tensor(wl.params.mobility, dtype=torch.float64, device=dev, requires_grad=True)
    st = torch.tensor(wl.params.sigma, dtype=torch.float64, device=dev, requires_grad=True)
    trace = amplitude_rollout(sim, phi0, Mt, st, params=wl.params, nsteps=nsteps, sample_every=K,
                              depth=12.0, u0=wl.u0, pstar0=wl.pstar0, checkpoint_every=4)
    L = ((trace - torch.as_tensor(target, device=dev)) ** 2).sum()
    L.backward()

    def rel(a, b):
        return abs(a - b) / max(abs(b), 1e-300)
    e_phi = (phi0.grad.reshape(-1).cpu() - dphio).abs().max().item() / dphio.abs().max().item()
    say(f"  L {L.item():.6e} vs {Lo:.6e}; dM {rel(Mt.grad.item(), dMo):.1e}; "
        f"dsigma {rel(st.grad.item(), dso):.1e}; dphi0 {e_phi:.1e}")
    assert rel(L.item(), float(Lo)) <= 1e-10
    assert rel(Mt.grad.item(), dMo) <= 1e-10
    assert rel(st.grad.item(), dso) <= 1e-10
    assert e_phi <= 1e-9


@pytest.mark.parametrize("streaming", ["ab", "aa"])
@pytest.mark.parametrize("forcing,s_bulk", [("guo", 0.0), ("guo", 1.2), ("first", 1.2)])
def test_forcing_and_bulk_rate_variants_match_oracle(forcing, s_bulk, streaming):
    """Guo's full source and the bulk rate of g in this build: FP64 parity on a
    walled ragged grid with solids and gravity."""
    from paper_2206_11637_amd.sim import from_workload
    p = W.Params(tau_H=0.6, tau_L=0.7, mobility=0.05, xi=4.0, sigma=5e-4, rho_L=0.05,
                 g=(1e-5, -2e-5, 0.0), s_bulk=s_bulk)
    wl = W.random_state(37, 19, 6, periodic=(False, False, True), params=p,
                        solid_fraction=0.1, seed=47, steps=8, u_amp=0.02)
    say(f"case: d3q27 {forcing} s_bulk={s_bulk} {streaming}")
    grid = OP.Grid(wl.nx, wl.ny, wl.nz, wl.periodic, wl.solid)
    prm = OP.OracleParams.from_workload(wl.params, "mrt", forcing, phase_lattice=PHASE)
    h, g = OP.init_equilibrium(grid, wl.phi0, wl.u0, wl.pstar0, PHASE)
    h, g = OP.run(grid, prm, h, g, wl.steps)
    sim = from_workload(wl, precision="fp64", collision="mrt", streaming=streaming,
                        forcing=forcing, phase_lattice=PHASE)
    assert sim.q_h == 27
    sim.step(wl.steps)
    _compare(sim, grid, prm, h, g, f"d3q27 {forcing} s_bulk={s_bulk} after {wl.steps}")
