"""Pins of the oracle's two-dimensional D2Q9 pair, the velocity set of the
paper's two-dimensional runs (sec. "Numerical experiments", standing waves):
lattice isotropy, the weighted-orthogonal moment basis and its per-degree
operator, the exact projection of the 3D pair onto it on z-invariant lattices,
conservation with walls and solids, and the two-dimensional Laplace law
p_in - p_out = sigma / R."""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as W
from oracle import lattice as OL
from oracle import pflbm as P


def test_d2q9_weights_and_isotropy():
    L = OL.D2Q9
    assert L.q == 9 and (L.c_np[:, 2] == 0).all()
    c, w = L.c_np[:, :2].astype(float), L.w_np
    assert abs(w.sum() - 1) < 1e-15
    assert np.abs((w[:, None] * c).sum(0)).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib->ab", w, c, c) - np.eye(2) / 3).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, c, c, c)).max() < 1e-15
    d = np.eye(2)
    iso = (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d) +
           np.einsum("ad,bc->abcd", d, d)) / 9.0
    assert np.abs(np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c) - iso).max() < 1e-15
    assert (L.c_np[L.opp] == -L.c_np).all()


def test_d2q9_mrt_operator_is_the_per_degree_projection():
    """M^-1 diag(s) M with one rate per degree (s_lo up to degree 2, s_hi
    above) equals s_hi I + (s_lo - s_hi) P, P the weighted least-squares
    projection onto polynomials of degree <= 2 (built here from the normal
    equations); all rates equal gives BGK."""
    L = OL.D2Q9
    c, w = L.c_np[:, :2].astype(float), L.w_np
    V = np.stack([np.ones(9), c[:, 0], c[:, 1], c[:, 0] ** 2, c[:, 1] ** 2, c[:, 0] * c[:, 1]], 1)
    # P f = w * (V a), a = argmin sum_i w_i (f_i / w_i - (V a)_i)^2 (normal equations)
    Wd = np.diag(w)
    Pm = Wd @ V @ np.linalg.solve(V.T @ Wd @ V, V.T)
    s_lo, s_hi = 1.3, 0.9
    rates = torch.where(L.degree >= 3, torch.tensor(s_hi, dtype=torch.float64),
                        torch.tensor(s_lo, dtype=torch.float64))[:, None]
    op = (L.Minv @ (rates * L.M)).numpy()
    assert np.abs(op - (s_hi * np.eye(9) + (s_lo - s_hi) * Pm)).max() < 1e-13
    eq = (L.Minv @ (torch.full((9, 1), 1.7, dtype=torch.float64) * L.M)).numpy()
    assert np.abs(eq - 1.7 * np.eye(9)).max() < 1e-14
    assert np.linalg.matrix_rank(L.M.numpy()) == 9


def _project(f, lat):
    """Sum a 3D lattice's populations over c_z into the D2Q9 order."""
    out = torch.zeros(9, f.shape[1], dtype=torch.float64)
    pos = {tuple(v[:2]): i for i, v in enumerate(OL.D2Q9.c_np)}
    for i, v in enumerate(lat.c_np):
        out[pos[(int(v[0]), int(v[1]))]] += f[i]
    return out


def _planar_case():
    wl = W.random_state(17, 13, 1, periodic=(True, False, True), solid_fraction=0.05, seed=3)
    wl = dataclasses.replace(wl, params=wl.params.copy(g=(1e-6, -2e-6, 0.0)))
    wl.u0[2] = 0.0
    return wl


@pytest.mark.parametrize("collision,phase3,exact", [("bgk", "d3q27", True), ("mrt", "d3q27", True),
                                                    ("bgk", "d3q15", True), ("mrt", "d3q15", False)])
def test_3d_pair_on_a_z_invariant_lattice_projects_onto_the_d2q9_pair(collision, phase3, exact):
    """On nx x ny x 1 lattices (z periodic, in-plane velocity and gravity) the
    3D model's populations summed over c_z evolve as the D2Q9 pair: the D3Q27
    weights factor as D2Q9 x (2/3, 1/6, 1/6) along z, so equilibria, forcing,
    the grad/lap stencils and the per-degree MRT projection (its zz Hermite
    term sums to zero over c_z) all project exactly.  D3Q15 projects onto the
    D2Q9 weights too, exactly under BGK; with MRT its zz second moment does not
    vanish under the projection and the two models differ at O(1e-3) here."""
    wl = _planar_case()
    grid = P.Grid(wl.nx, wl.ny, 1, wl.periodic, wl.solid)
    p3 = P.OracleParams.from_workload(wl.params, collision, phase_lattice=phase3)
    p2 = P.OracleParams.from_workload(wl.params, collision, phase_lattice="d2q9")
    h3, g3 = P.init_equilibrium(grid, wl.phi0, wl.u0, wl.pstar0, phase3)
    h2, g2 = P.init_equilibrium(grid, wl.phi0, wl.u0, wl.pstar0, "d2q9")
    h3, g3 = P.run(grid, p3, h3, g3, 20)
    h2, g2 = P.run(grid, p2, h2, g2, 20)
    lat_h = OL.D3Q27 if phase3 == "d3q27" else OL.D3Q15
    eh = float((_project(h3, lat_h) - h2).abs().max() / h2.abs().max())
    eg = float((_project(g3, OL.D3Q27) - g2).abs().max() / g2.abs().max())
    if exact:
        assert eh < 1e-13 and eg < 1e-13, (eh, eg)
    else:
        assert eh > 1e-6


def test_d2q9_conserves_phase_mass_and_pressure_sum_with_walls_and_solids():
    wl = _planar_case()
    grid = P.Grid(wl.nx, wl.ny, 1, wl.periodic, wl.solid)
    prm = P.OracleParams.from_workload(wl.params, "mrt", phase_lattice="d2q9")
    h, g = P.init_equilibrium(grid, wl.phi0, wl.u0, wl.pstar0, "d2q9")
    r0 = P.reductions(grid, h, g, "d2q9")
    h, g = P.run(grid, prm, h, g, 50)
    r1 = P.reductions(grid, h, g, "d2q9")
    assert abs(float(r1[0] - r0[0])) / float(r0[0]) < 1e-13
    assert abs(float(r1[1] - r0[1])) <= 1e-13 * float(g.abs().sum())


def test_d2q9_pair_rejects_3d_lattices():
    grid = P.Grid(6, 6, 2, (True, True, True))
    prm = P.OracleParams(0.8, 0.8, 0.05, 4.0, 1e-3, 1.0, 1e-3, (0, 0, 0), phase_lattice="d2q9")
    h, g = P.init_equilibrium(grid, np.full(72, 0.5), np.zeros((3, 72)), np.zeros(72), "d2q9")
    with pytest.raises(ValueError):
        P.step(grid, prm, h, g)


def test_d2q9_laplace_pressure_of_a_static_disk():
    """A heavy disk (R = 8) in a light phase (density ratio 1000) on the D2Q9
    pair: the pressure p = p* rho c_s^2 jumps by sigma / R, the
    two-dimensional Young-Laplace law (one curvature instead of two)."""
    n, R, xi, sigma, rL = 32, 8.0, 4.0, 1e-3, 1e-3
    grid = P.Grid(n, n, 1, (True, True, True))
    y, x = np.meshgrid(np.arange(n) + 0.5, np.arange(n) + 0.5, indexing="ij")
    r = np.sqrt((x - n / 2) ** 2 + (y - n / 2) ** 2)
    prm = P.OracleParams(0.8, 0.8, 0.05, xi, sigma, 1.0, rL, (0, 0, 0), phase_lattice="d2q9")
    h, g = P.init_equilibrium(grid, 0.5 + 0.5 * np.tanh(2 * (R - r) / xi), np.zeros((3, n * n)),
                              np.zeros(n * n), "d2q9")
    h, g = P.run(grid, prm, h, g, 1500)
    phi, u, ps = P.moments(grid, prm, h, g)
    p = (ps * (rL + phi * (1 - rL)) / 3).numpy().reshape(n, n)
    dp = p[r < R - 4].mean() - p[r > R + 5].mean()
    assert abs(dp / (sigma / R) - 1) < 0.05, dp / (sigma / R)
