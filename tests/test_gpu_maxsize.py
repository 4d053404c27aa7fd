"""Lattices at the library's size limit (population offsets within one
opposite pair must stay below 2^32 bytes: N < 2^29 cells with 4-byte
storage or adjoint arrays, N < 2^28 in FP64), in the benchmark's launch
configuration.

The full state of such a lattice is too large to read back next to the
workspace, so the check uses a property that holds at any size: a random
state that is periodic with a small tile, on a fully periodic lattice, evolves
exactly like the tile on its own.  Every tile of phi after a few steps must
equal the tile's own run bitwise (the per-cell arithmetic does not depend on
position), including the tiles at the largest offsets; the tile's run is
checked against the oracle."""
import gc

import numpy as np
import pytest
import torch

import workloads as W
from oracle import pflbm as OP

from gpu_util import normwise, say

pytestmark = pytest.mark.gpu

STEPS = 3


def _tile_state(tile):
    p = W.Params(tau_H=0.6, tau_L=0.8, mobility=0.05, xi=4.0, sigma=2e-4, rho_L=0.1,
                 g=(0.0, -1e-5, 0.0))
    return W.random_state(*tile, periodic=(True, True, True), params=p, seed=29, steps=STEPS)


def _tiled(wl, reps):
    rz, ry, rx = reps
    phi0 = np.tile(wl.phi0, (rz, ry, rx))
    u0 = np.tile(wl.u0, (1, rz, ry, rx))
    p0 = np.tile(wl.pstar0, (rz, ry, rx))
    nz, ny, nx = phi0.shape
    return W.Workload(f"tiled_{nx}x{ny}x{nz}", nx, ny, nz, (True, True, True), wl.params, phi0,
                      u0, p0, None, wl.steps)


# (precision, lattice, tile (tx, ty, tz) dividing it)
@pytest.mark.parametrize("precision,dims,TILE", [("fp32", (1024, 512, 1023), (32, 16, 31)),
                                                 ("fp64", (1024, 512, 511), (32, 16, 7)),
                                                 ("fp16s", (1024, 512, 1023), (32, 16, 31))])
def test_lattice_at_the_offset_limit_evolves_like_its_tile(precision, dims, TILE):
    from paper_2206_11637_amd.sim import from_workload
    gc.collect()
    torch.cuda.empty_cache()          # earlier tests' cached blocks: room for ~190 GiB
    nx, ny, nz = dims
    N = nx * ny * nz
    per_cell = 8 if precision == "fp64" else 4
    # the largest lattice of this cross-section: one more plane reaches the limit
    assert 2 * N * per_cell < 2 ** 32 <= 2 * (N + nx * ny) * per_cell
    small = _tile_state(TILE)
    reps = (nz // TILE[2], ny // TILE[1], nx // TILE[0])
    assert (reps[2] * TILE[0], reps[1] * TILE[1], reps[0] * TILE[2]) == dims
    say(f"case: max size {precision} {nx}x{ny}x{nz} ({N:,} cells), {STEPS} steps")

    ref = from_workload(small, precision=precision)
    ref.step(STEPS)
    phi_tile = ref.phi()
    del ref
    # the tile against the oracle
    grid = OP.Grid(*TILE, (True, True, True))
    prm = OP.OracleParams.from_workload(small.params)
    h, g = OP.init_equilibrium(grid, small.phi0, small.u0, small.pstar0)
    h, g = OP.run(grid, prm, h, g, STEPS)
    e_or = normwise(phi_tile.reshape(-1).cpu(), h.sum(0))
    tol = {"fp64": 1e-12, "fp32": 1e-5, "fp16s": 2e-3}[precision]
    say(f"  tile vs oracle: phi normwise {e_or:.2e}")
    assert e_or <= tol

    big_wl = _tiled(small, reps)
    sim = from_workload(big_wl, precision=precision)
    del big_wl
    gc.collect()
    say(f"  workspace {sim.workspace.numel() / 2**30:.1f} GiB")
    sim.step(STEPS)
    phi = sim.phi()
    del sim
    gc.collect()
    torch.cuda.empty_cache()
    tiles = phi.reshape(reps[0], TILE[2], reps[1], TILE[1], reps[2], TILE[0])
    tiles = tiles.permute(0, 2, 4, 1, 3, 5)            # [rz, ry, rx, tz, ty, tx]
    same = (tiles == phi_tile.view(1, 1, 1, *phi_tile.shape)).flatten(3).all(-1)
    bad = int((~same).sum())
    say(f"  tiles equal to the tile's own run: {int(same.sum())} of {same.numel()} "
        f"(last tile max|d| {(tiles[-1, -1, -1] - phi_tile).abs().max().item():.1e})")
    del phi, tiles
    torch.cuda.empty_cache()
    assert bad == 0
