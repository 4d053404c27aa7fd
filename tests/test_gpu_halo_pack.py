"""The halo pack of a z-slab decomposition (pflbm_pack_faces): the packed rows
are bitwise the rows of the state that stream across the two z faces (c_z = -1
at plane 0, c_z = +1 at plane nz - 1), read from a saved state, in every
storage form and on both phase lattices."""
import pytest
import torch

import workloads as W

from gpu_util import say

pytestmark = pytest.mark.gpu

DT = {"fp64": torch.float64, "fp32": torch.float32, "fp16s": torch.float16}
# integer views for a bitwise comparison (the slots of solid cells are never
# written and may hold NaN patterns, which compare unequal as floats)
BITS = {torch.float64: torch.int64, torch.float32: torch.int32, torch.float16: torch.int16}


def saved_rows(sim, precision):
    """h [q_h, nz, ny, nx] and g [27, nz, ny, nx] in the storage dtype, from a
    saved state (h rows, then g rows, then the phase fields)."""
    nz, ny, nx = sim.shape
    st = sim.save_state()
    dt = DT[precision]
    es = torch.empty((), dtype=dt).element_size()
    nh, ng = sim.q_h * sim.N, 27 * sim.N
    pops = st[:(nh + ng) * es].view(dt)
    return pops[:nh].reshape(sim.q_h, nz, ny, nx), pops[nh:].reshape(27, nz, ny, nx)


@pytest.mark.parametrize("phase", ["d3q15", "d3q27"])
@pytest.mark.parametrize("precision", ["fp64", "fp32", "fp16s"])
def test_face_pack_holds_the_crossing_rows_of_the_state(precision, phase):
    from paper_2206_11637_amd.sim import from_workload, lattice
    wl = W.random_state(37, 11, 6, periodic=(True, False, True), seed=5, solid_fraction=0.05)
    say(f"case: halo pack, 37x11x6, {precision}, {phase}")
    sim = from_workload(wl, precision=precision, phase_lattice=phase)
    sim.step(3)
    pack = sim.pack_faces()
    h, g = saved_rows(sim, precision)
    torch.cuda.synchronize()
    c_h = torch.as_tensor(lattice(sim.q_h, phase)[0])
    c_g = torch.as_tensor(lattice(27, phase)[0])
    for face, (plane, dz) in enumerate(((0, -1), (sim.shape[0] - 1, 1))):
        ih = [int(i) for i in torch.nonzero(c_h[:, 2] == dz).flatten()]
        ig = [int(i) for i in torch.nonzero(c_g[:, 2] == dz).flatten()]
        want = torch.cat([h[ih, plane], g[ig, plane]])
        assert pack.shape[1] == len(ih) + len(ig) == (9 if sim.q_h == 27 else 5) + 9
        bits = BITS[want.dtype]
        assert torch.equal(pack[face].view(bits), want.contiguous().view(bits)), (face, precision, phase)

