"""The D2Q9 pair of the paper's two-dimensional runs (sec. "Numerical
experiments", velocity sets of the standing waves) on the GPU.  On nx x ny x 1
lattices with z periodic and in-plane velocity and gravity, the library's
D3Q27-phase build (BGK and MRT) and its default D3Q15 build (BGK) evolve, once
their populations are summed over c_z, exactly as the D2Q9 pair: compared here
with the oracle's D2Q9 pair (FP64, walls and solids) after N steps, normwise
per lattice."""
import dataclasses

import numpy as np
import pytest
import torch

import workloads as W
from oracle import lattice as OL
from oracle import pflbm as OP

from gpu_util import normwise, say

pytestmark = pytest.mark.gpu


def _project(f, c_lib):
    """Library-order populations [q, N] summed over c_z, in the oracle's D2Q9 order."""
    out = torch.zeros(9, f.shape[1], dtype=torch.float64)
    pos = {tuple(v[:2]): i for i, v in enumerate(OL.D2Q9.c_np)}
    for i, v in enumerate(c_lib):
        out[pos[(int(v[0]), int(v[1]))]] += f[i]
    return out


@pytest.mark.parametrize("phase,collision", [("d3q27", "bgk"), ("d3q27", "mrt"), ("d3q15", "bgk")])
@pytest.mark.parametrize("shape,periodic,solids", [((37, 29), (True, False, True), 0.05),
                                                   ((64, 48), (True, True, True), 0.0)])
def test_planar_lattices_evolve_as_the_d2q9_pair(phase, collision, shape, periodic, solids):
    from paper_2206_11637_amd.sim import from_workload, lattice
    nx, ny = shape
    wl = W.random_state(nx, ny, 1, periodic=periodic, solid_fraction=solids, seed=9)
    wl = dataclasses.replace(wl, params=wl.params.copy(g=(1e-6, -2e-6, 0.0)))
    wl.u0[2] = 0.0
    nsteps = 40
    say(f"case: d2q9 pair via {phase} build, {collision}, {nx}x{ny}x1 periodic={periodic} "
        f"solids={solids}, {nsteps} steps")
    sim = from_workload(wl, precision="fp64", collision=collision, phase_lattice=phase)
    sim.step(nsteps)
    h, g = sim.populations()
    ch, _ = lattice(sim.q_h, phase)
    cg, _ = lattice(27, phase)
    hp, gp = _project(h.cpu(), ch), _project(g.cpu(), cg)
    grid = OP.Grid(nx, ny, 1, wl.periodic, wl.solid)
    prm = OP.OracleParams.from_workload(wl.params, collision, phase_lattice="d2q9")
    ho, go = OP.init_equilibrium(grid, wl.phi0, wl.u0, wl.pstar0, "d2q9")
    ho, go = OP.run(grid, prm, ho, go, nsteps)
    eh, eg = normwise(hp, ho), normwise(gp, go)
    say(f"  projected h vs D2Q9 oracle {eh:.2e}, g {eg:.2e}")
    assert eh <= 1e-12 and eg <= 1e-12
    assert np.isfinite(sim.reduce()).all()
