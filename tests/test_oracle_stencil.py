"""Pins of the oracle's finite-difference stencils and chemical potential."""
import math

import numpy as np
import torch

from oracle import lattice as L
from oracle import pflbm as P


def _aux_for_phi(grid, phi, prm=None):
    prm = prm or P.OracleParams(0.6, 0.6, 0.05, 4.0, 1e-3, 1.0, 1.0, (0, 0, 0))
    phi = torch.as_tensor(phi, dtype=torch.float64).reshape(-1)
    h = P.equilibrium(L.D3Q15, phi, torch.zeros(3, grid.N, dtype=torch.float64), True)
    g = torch.zeros(27, grid.N, dtype=torch.float64)
    return P.collide(grid, prm, h, g)[2]


def _coords(grid):
    z, y, x = np.meshgrid(np.arange(grid.nz), np.arange(grid.ny), np.arange(grid.nx),
                          indexing="ij")
    return x.reshape(-1).astype(float), y.reshape(-1).astype(float), z.reshape(-1).astype(float)


def test_gradient_exact_on_affine_and_laplacian_on_quadratic():
    grid = P.Grid(9, 8, 7, (False, False, False))
    x, y, z = _coords(grid)
    interior = (x > 0) & (x < 8) & (y > 0) & (y < 7) & (z > 0) & (z < 6)
    a = np.array([0.013, -0.021, 0.007])
    phi = 0.3 + a[0] * x + a[1] * y + a[2] * z
    aux = _aux_for_phi(grid, phi)
    grad = aux["grad"].numpy()
    assert np.abs(grad[:, interior] - a[:, None]).max() < 1e-14
    assert np.abs(aux["lap"].numpy()[interior]).max() < 1e-14
    # quadratic: lap = 2(qa+qb+qc), grad exact at the cell
    q = np.array([1e-3, -2e-3, 1.5e-3])
    phi2 = 0.4 + q[0] * x * x + q[1] * y * y + q[2] * z * z + 1e-3 * x * y - 2e-3 * y * z
    aux = _aux_for_phi(grid, phi2)
    lap = aux["lap"].numpy()
    assert np.abs(lap[interior] - 2 * q.sum()).max() < 1e-14
    gx = 2 * q[0] * x + 1e-3 * y
    gy = 2 * q[1] * y + 1e-3 * x - 2e-3 * z
    gz = 2 * q[2] * z - 2e-3 * y
    g = aux["grad"].numpy()
    assert np.abs(g[0, interior] - gx[interior]).max() < 1e-14
    assert np.abs(g[1, interior] - gy[interior]).max() < 1e-14
    assert np.abs(g[2, interior] - gz[interior]).max() < 1e-14


def test_wall_and_solid_neighbours_take_own_value_bruteforce():
    """Brute force over a tiny box with walls in y and solid cells: every
    missing neighbour (outside a wall or solid) repeats the cell's own phi."""
    rng = np.random.default_rng(5)
    nx, ny, nz = 5, 4, 3
    solid = rng.uniform(size=(nz, ny, nx)) < 0.2
    grid = P.Grid(nx, ny, nz, (True, False, True), solid)
    phi = rng.uniform(0, 1, size=(nz, ny, nx))
    aux = _aux_for_phi(grid, phi)
    grad = aux["grad"].numpy().reshape(3, nz, ny, nx)
    lap = aux["lap"].numpy().reshape(nz, ny, nx)
    wts = {0: 8 / 27, 1: 2 / 27, 2: 1 / 54, 3: 1 / 216}
    for z in range(nz):
        for y in range(ny):
            for x in range(nx):
                if solid[z, y, x]:
                    continue
                gref = np.zeros(3)
                lref = 0.0
                for cx in (-1, 0, 1):
                    for cy in (-1, 0, 1):
                        for cz in (-1, 0, 1):
                            w = wts[cx * cx + cy * cy + cz * cz]
                            X, Y, Z = (x + cx) % nx, y + cy, (z + cz) % nz
                            if 0 <= Y < ny and not solid[Z, Y, X]:
                                v = phi[Z, Y, X]
                            else:
                                v = phi[z, y, x]
                            gref += 3 * w * np.array([cx, cy, cz]) * v
                            lref += 6 * w * (v - phi[z, y, x])
                assert np.abs(grad[:, z, y, x] - gref).max() < 1e-14
                assert abs(lap[z, y, x] - lref) < 1e-14


def test_chemical_potential_vanishes_on_tanh_profile():
    """mu_phi = 4 beta phi(phi-1)(phi-1/2) - kappa lap phi is zero on the
    equilibrium profile phi = 1/2 + 1/2 tanh(2x/xi) in the continuum; on the
    lattice the residual is O(dx^2) relative to the bulk term."""
    xi, sigma = 4.0, 1e-3
    grid = P.Grid(64, 1, 1, (True, True, True))
    x = np.arange(64) + 0.5
    d = np.minimum(x - 16.0, 48.0 - x)       # two interfaces, periodic
    phi = 0.5 + 0.5 * np.tanh(2 * d / xi)
    aux = _aux_for_phi(grid, phi, P.OracleParams(0.6, 0.6, 0.05, xi, sigma, 1.0, 1.0, (0, 0, 0)))
    mu = aux["mu"].numpy()
    beta = 12 * sigma / xi
    bulk = 4 * beta * np.abs(phi * (phi - 1) * (phi - 0.5)).max()
    assert np.abs(mu).max() < 0.1 * bulk
    # halving the grid spacing (xi -> 2 xi in lattice units) cuts the residual ~4x
    xi2 = 8.0
    grid2 = P.Grid(128, 1, 1, (True, True, True))
    x2 = np.arange(128) + 0.5
    d2 = np.minimum(x2 - 32.0, 96.0 - x2)
    phi2 = 0.5 + 0.5 * np.tanh(2 * d2 / xi2)
    # sigma scales with dx in lattice units to keep the same physical surface tension
    aux2 = _aux_for_phi(grid2, phi2, P.OracleParams(0.6, 0.6, 0.05, xi2, sigma, 1.0, 1.0, (0, 0, 0)))
    mu2 = aux2["mu"].numpy()
    bulk2 = 4 * (12 * sigma / xi2) * np.abs(phi2 * (phi2 - 1) * (phi2 - 0.5)).max()
    r1 = np.abs(mu).max() / bulk
    r2 = np.abs(mu2).max() / bulk2
    assert 3.0 < r1 / r2 < 5.0


def test_surface_tension_identity_of_the_constants():
    """With beta = 12 sigma/xi and kappa = 3 sigma xi/2, the excess free energy
    of the tanh profile, int kappa (dphi/dx)^2 dx, equals sigma."""
    sigma, xi = 1e-4, 4.0
    x = np.linspace(-40, 40, 200001)
    dphi = (1.0 / xi) / np.cosh(2 * x / xi) ** 2
    val = np.trapezoid(1.5 * sigma * xi * dphi * dphi, x)
    assert abs(val - sigma) < 1e-9 * sigma + 1e-12
