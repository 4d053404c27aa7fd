"""Shared helpers of the GPU tests (host-side glue only, no method arithmetic)."""
import math
import sys

import numpy as np
import torch

from oracle import lattice as OL
from oracle import pflbm as OP


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def perm_to_oracle(q, phase="d3q15"):
    """perm[j] = library index of oracle direction j (q = 15 or 27, in the
    build of the given phase lattice)."""
    from paper_2206_11637_amd.sim import lattice
    c_lib, _ = lattice(q, phase)
    lat = OL.D3Q15 if q == 15 else OL.D3Q27
    pos = {tuple(v): i for i, v in enumerate(c_lib)}
    return np.array([pos[tuple(v)] for v in lat.c_np])


def gpu_pops_oracle_order(sim, to_cpu=True):
    h, g = sim.populations()
    ph, pg = perm_to_oracle(sim.q_h, sim.phase_lattice), perm_to_oracle(27, sim.phase_lattice)
    h = h[torch.as_tensor(ph, device=h.device)]
    g = g[torch.as_tensor(pg, device=g.device)]
    return (h.cpu(), g.cpu()) if to_cpu else (h, g)


def normwise(a, ref):
    a = torch.as_tensor(a, dtype=torch.float64).cpu()
    ref = torch.as_tensor(ref, dtype=torch.float64).cpu()
    den = ref.abs().max().item()
    v = (a - ref).abs().max().item() / (den if den > 0 else 1.0)
    # a NaN on either side counts as the worst error (max() would skip it)
    return v if math.isfinite(v) else math.inf


def oracle_setup(wl, collision):
    grid = OP.Grid(wl.nx, wl.ny, wl.nz, wl.periodic, wl.solid)
    prm = OP.OracleParams.from_workload(wl.params, collision)
    h, g = OP.init_equilibrium(grid, wl.phi0, wl.u0, wl.pstar0)
    return grid, prm, h, g


def window_check(sim, wl, collision, h_n, g_n, h_n1, g_n1, centres, half=6, perms=None):
    """One-step oracle check on windows of a large GPU state.

    h_n, g_n: GPU state at step n ([q, N] float64, any device), in oracle
    order, or in library order with perms = (perm_h, perm_g) given;
    h_n1, g_n1: GPU state at step n + 1.  For each centre a window of
    (2 half + 1)^3 cells (clipped at walls) is cut, advanced one step by the
    oracle with the window faces as walls, and compared on the cells at least
    two cells away from every artificial face.  Returns the worst normwise
    errors (h, g) and the number of compared cells.
    """
    nz, ny, nx = wl.nz, wl.ny, wl.nx
    dims = (nx, ny, nz)
    per = wl.periodic
    qh = h_n.shape[0]      # 15, or 27 for the D3Q27 phase lattice
    prm = OP.OracleParams.from_workload(wl.params, collision,
                                        phase_lattice="d3q27" if qh == 27 else "d3q15")
    worst_h = worst_g = 0.0
    ncmp = 0
    H4 = h_n.reshape(qh, nz, ny, nx)
    G4 = g_n.reshape(27, nz, ny, nx)
    H41 = h_n1.reshape(qh, nz, ny, nx)
    G41 = g_n1.reshape(27, nz, ny, nx)
    for cen in centres:
        idx, keep = [], []
        for ax in range(3):
            n = dims[ax]
            lo, hi = cen[ax] - half, cen[ax] + half + 1
            if not per[ax]:
                lo, hi = max(lo, 0), min(hi, n)
            ids = np.arange(lo, hi) % n
            k = np.ones(len(ids), dtype=bool)
            # artificial faces: the window edge unless it is a real wall
            if per[ax] or lo > 0:
                k[:2] = False
            if per[ax] or hi < n:
                k[-2:] = False
            if per[ax] and len(ids) >= n:
                raise ValueError("window wraps the whole periodic axis")
            idx.append(ids)
            keep.append(k)
        ix, iy, iz = idx
        sel = np.ix_(iz, iy, ix)
        tsel = tuple(torch.as_tensor(a, device=H4.device) for a in sel)
        hw = H4[(slice(None),) + tsel].reshape(qh, -1).double().cpu()
        gw = G4[(slice(None),) + tsel].reshape(27, -1).double().cpu()
        if perms is not None:
            hw, gw = hw[perms[0]], gw[perms[1]]
        solid = None if wl.solid is None else wl.solid[sel]
        grid = OP.Grid(len(ix), len(iy), len(iz), (False, False, False), solid)
        ho, go = OP.step(grid, prm, hw, gw)
        kz, ky, kx = np.meshgrid(keep[2], keep[1], keep[0], indexing="ij")
        m = torch.as_tensor((kz & ky & kx).reshape(-1))
        if solid is not None:
            m &= ~torch.as_tensor(solid.reshape(-1))
        hg = H41[(slice(None),) + tsel].reshape(qh, -1).double().cpu()
        gg = G41[(slice(None),) + tsel].reshape(27, -1).double().cpu()
        if perms is not None:
            hg, gg = hg[perms[0]], gg[perms[1]]
        worst_h = max(worst_h, normwise(hg[:, m], ho[:, m]))
        worst_g = max(worst_g, normwise(gg[:, m], go[:, m]))
        ncmp += int(m.sum())
    return worst_h, worst_g, ncmp
