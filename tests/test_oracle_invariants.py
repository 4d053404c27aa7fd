"""Invariants and symmetries of the oracle step (conservation, rest state, translation)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import lattice as L
from oracle import pflbm as P


def _setup(wl, collision="mrt", phase="d3q15"):
    grid = P.Grid(wl.nx, wl.ny, wl.nz, wl.periodic, wl.solid)
    prm = P.OracleParams.from_workload(wl.params, collision, phase_lattice=phase)
    h, g = P.init_equilibrium(grid, wl.phi0, wl.u0, wl.pstar0, phase)
    return grid, prm, h, g


@pytest.mark.parametrize("phase", ["d3q15", "d3q27"])
@pytest.mark.parametrize("collision", ["bgk", "mrt"])
def test_phase_mass_and_pressure_sum_conserved_with_walls_and_solids(collision, phase):
    """Sum of phi and sum of p* over fluid cells are invariants of the step
    (paper: the model is mass conserving); walls and solids included; both
    phase lattices."""
    wl = W.random_state(11, 9, 7, periodic=(True, False, True), solid_fraction=0.1, seed=3)
    grid, prm, h, g = _setup(wl, collision, phase)
    r0 = P.reductions(grid, h, g)
    h, g = P.run(grid, prm, h, g, 60)
    r1 = P.reductions(grid, h, g)
    assert abs(r1[0] - r0[0]) / abs(r0[0]) < 1e-13
    scale = torch.abs(g.sum(0)).sum()
    assert abs(r1[1] - r0[1]) / scale < 1e-13


def test_momentum_conserved_without_forces():
    """sigma = 0, g = 0 and rho_H = rho_L make every force vanish; then the
    lattice momentum sum_x sum_i c_i g_i is invariant on a periodic box."""
    p = W.Params(tau_H=0.7, tau_L=0.6, mobility=0.05, xi=4.0, sigma=0.0, rho_H=1.0, rho_L=1.0,
                 g=(0.0, 0.0, 0.0))
    wl = W.random_state(8, 7, 6, periodic=(True, True, True), params=p, seed=9)
    grid, prm, h, g = _setup(wl)
    r0 = P.reductions(grid, h, g)
    h, g = P.run(grid, prm, h, g, 40)
    r1 = P.reductions(grid, h, g)
    jscale = torch.abs(L.D3Q27.c.t() @ g).sum()
    assert torch.abs(r1[2:] - r0[2:]).max() / jscale < 1e-13


@pytest.mark.parametrize("phi_value,xi", [(0.0, 4.0), (1.0, 4.0), (0.3, float("inf"))])
def test_rest_state_is_a_fixed_point(phi_value, xi):
    """Uniform phi, u = 0, uniform p* (and any sigma): nothing changes.  A
    uniform intermediate phi is only a fixed point with the counter-term off:
    with it on, the conservative Allen-Cahn flux separates the phases from any
    rounding-level perturbation."""
    n = (6, 5, 4)
    p = W.Params(tau_H=0.55, tau_L=0.9, mobility=0.03, xi=xi, sigma=3e-4)
    grid = P.Grid(*n, (True, False, True))
    prm = P.OracleParams.from_workload(p)
    phi0 = np.full(n[::-1], phi_value)
    h0, g0 = P.init_equilibrium(grid, phi0, np.zeros((3,) + n[::-1]), np.full(n[::-1], 2e-3))
    h, g = P.run(grid, prm, h0, g0, 20)
    # fixed to rounding: the dense M^-1 S M product is not an exact identity
    assert torch.abs(h - h0).max() < 1e-14
    assert torch.abs(g - g0).max() < 1e-14
    _, u, _ = P.moments(grid, prm, h, g)
    assert torch.abs(u).max() < 1e-15


def test_translation_invariance_on_periodic_axes():
    wl = W.random_state(8, 6, 5, periodic=(True, True, True), seed=21)
    grid, prm, h, g = _setup(wl)
    shift = (3, 2, 1)  # (x, y, z)

    def roll(f):
        q = f.shape[0]
        return torch.roll(f.reshape(q, wl.nz, wl.ny, wl.nx), shifts=(shift[2], shift[1], shift[0]),
                          dims=(1, 2, 3)).reshape(q, -1)

    ha, ga = P.run(grid, prm, h, g, 5)
    hb, gb = P.run(grid, prm, roll(h), roll(g), 5)
    assert torch.abs(roll(ha) - hb).max() < 1e-15
    assert torch.abs(roll(ga) - gb).max() < 1e-15


def test_streaming_is_a_permutation_with_bounce_back():
    """Pure streaming (no collision) moves each population exactly once:
    every post-collision value lands in exactly one slot."""
    rng = np.random.default_rng(1)
    solid = rng.uniform(size=(4, 5, 6)) < 0.15
    grid = P.Grid(6, 5, 4, (False, True, False), solid)
    for lat in (L.D3Q15, L.D3Q27):
        fstar = torch.tensor(rng.uniform(1, 2, size=(lat.q, grid.N)))
        fstar = torch.where(grid.fluid[None], fstar, torch.zeros_like(fstar))
        out = P.stream(grid, lat, fstar)
        a = np.sort(fstar[:, grid.fluid].reshape(-1).numpy())
        b = np.sort(out[:, grid.fluid].reshape(-1).numpy())
        assert np.array_equal(a, b)


def test_unstable_parameters_blow_up_in_the_oracle():
    """The case the GPU stability check is tested on is genuinely unstable:
    tau -> 1/2 with velocities of 0.3 at density ratio 1000."""
    p = W.Params(tau_H=0.5001, tau_L=0.5001, mobility=0.02, xi=4.0, sigma=1e-3, rho_L=1e-3)
    wl = W.random_state(40, 24, 8, periodic=(True, True, True), params=p, u_amp=0.3, seed=77)
    grid, prm, h, g = _setup(wl)
    finite = True
    for _ in range(40):
        h, g = P.step(grid, prm, h, g)
        if not (torch.isfinite(h).all() and torch.isfinite(g).all()):
            finite = False
            break
    assert not finite
