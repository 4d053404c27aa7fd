"""Pins of the oracle's lattices and MRT matrices (closed forms, identities)."""
import dataclasses
import itertools
import math

import numpy as np
import pytest
import torch

from oracle import lattice as L
from oracle import pflbm as P

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("lat", [L.D3Q15, L.D3Q27], ids=lambda l: l.name)
def test_isotropy(lat):
    c = lat.c_np.astype(float)
    w = lat.w_np
    d = np.eye(3)
    assert abs(w.sum() - 1.0) < 1e-15
    assert np.abs(np.einsum("i,ia->a", w, c)).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib->ab", w, c, c) - CS2 * d).max() < 1e-15
    assert np.abs(np.einsum("i,ia,ib,ic->abc", w, c, c, c)).max() < 1e-15
    t4 = np.einsum("i,ia,ib,ic,id->abcd", w, c, c, c, c)
    iso = CS2 ** 2 * (np.einsum("ab,cd->abcd", d, d) + np.einsum("ac,bd->abcd", d, d)
                      + np.einsum("ad,bc->abcd", d, d))
    assert np.abs(t4 - iso).max() < 1e-15
    # opposite directions
    assert (c[lat.opp] == -c).all()
    assert lat.q == {"D3Q15": 15, "D3Q27": 27}[lat.name]


@pytest.mark.parametrize("lat", [L.D3Q15, L.D3Q27], ids=lambda l: l.name)
def test_moment_rows_weighted_orthogonal(lat):
    M = lat.M.numpy()
    G = M @ np.diag(lat.w_np) @ M.T
    off = G - np.diag(np.diag(G))
    assert np.abs(off).max() < 1e-13
    deg = lat.degree.numpy()
    assert (np.diff(deg) >= 0).all() and deg[0] == 0 and (deg[1:4] == 1).all()
    assert (deg[4:10] == 2).all()


def _operator(lat, monomials, rates_by_degree):
    M, deg = L.gram_schmidt_moments(lat.c_np, lat.w_np, monomials)
    S = np.diag([rates_by_degree(d) for d in deg])
    return np.linalg.inv(M) @ S @ M


@pytest.mark.parametrize("lat", [L.D3Q15, L.D3Q27], ids=lambda l: l.name)
def test_operator_independent_of_ordering_within_degree(lat):
    rng = np.random.default_rng(0)
    rate = lambda d: 1.3 if d <= 2 else 0.7
    ref = _operator(lat, lat.monomials, rate)
    for _ in range(5):
        by_deg = {}
        for m in lat.monomials:
            by_deg.setdefault(sum(m), []).append(m)
        order = []
        for d in sorted(by_deg):
            grp = list(by_deg[d])
            rng.shuffle(grp)
            order += grp
        alt = _operator(lat, order, rate)
        assert np.abs(alt - ref).max() < 1e-13


@pytest.mark.parametrize("lat", [L.D3Q15, L.D3Q27], ids=lambda l: l.name)
def test_mrt_equals_projection_form(lat):
    """M^-1 S M with rate s_lo on degree <= 2 and s_hi above equals
    s_hi I + (s_lo - s_hi) P, where P is the weighted least-squares projection
    of Delta_i / w_i onto quadratic polynomials of c (built here by lstsq)."""
    s_lo, s_hi = 1.7, 0.9
    op = _operator(lat, lat.monomials, lambda d: s_lo if d <= 2 else s_hi)
    c = lat.c_np.astype(float)
    w = lat.w_np
    cols = [np.ones(lat.q)] + [c[:, a] for a in range(3)] + \
        [c[:, a] * c[:, b] for a in range(3) for b in range(a, 3)]
    V = np.stack(cols, 1)                                      # [q, 10]
    # fit coefficients a minimising sum_i w_i (Delta_i/w_i - V a)^2
    W = np.diag(w)
    P = W @ V @ np.linalg.solve(V.T @ W @ V, V.T)              # maps Delta -> w (V a)
    ref = s_hi * np.eye(lat.q) + (s_lo - s_hi) * P
    assert np.abs(op - ref).max() < 1e-13
    # all rates equal: BGK
    op_bgk = _operator(lat, lat.monomials, lambda d: 1.2)
    assert np.abs(op_bgk - 1.2 * np.eye(lat.q)).max() < 1e-13


def test_hydro_first_moment_with_guo_forcing():
    """After the g collision, j* = j + F / rho whatever omega is (degree-1
    moments of g^eq - g equal F/(2 rho) and the forcing adds (1 - omega/2) F/rho)."""
    rng = np.random.default_rng(3)
    grid = P.Grid(4, 3, 5, (True, True, True))
    N = grid.N
    for omega_tau in (0.55, 0.9, 1.4):
        prm = P.OracleParams(omega_tau, omega_tau, 0.05, 4.0, 3e-4, 1.0, 0.2, (1e-4, -2e-4, 3e-4))
        phi = torch.tensor(rng.uniform(0.1, 0.9, N))
        u = torch.tensor(rng.uniform(-0.01, 0.01, (3, N)))
        h = P.equilibrium(L.D3Q15, phi, u, True)
        g = P.equilibrium(L.D3Q27, torch.tensor(rng.uniform(-1e-3, 1e-3, N)), u, False)
        g = g + 1e-4 * torch.tensor(rng.standard_normal((27, N)))
        gs, hs = None, None
        hs, gs, aux = P.collide(grid, prm, h, g)
        j = L.D3Q27.c.t() @ g
        js = L.D3Q27.c.t() @ gs
        want = j + aux["F"] / aux["rho"][None]
        assert torch.abs(js - want).max() < 1e-15
        # zeroth moments conserved by both collisions
        assert torch.abs(gs.sum(0) - g.sum(0)).max() < 1e-15
        assert torch.abs(hs.sum(0) - h.sum(0)).max() < 1e-15


def test_hydro_second_moment_relaxes_at_omega():
    """BGK and MRT both relax the hydrodynamic stress Pi = sum c c g at the
    local omega towards Pi^eq = p* c_s^2 I + u u^T; the forcing adds its own
    second moment (1 - omega/2) sum c c F^g = 0 here (F^g has no second moment)."""
    rng = np.random.default_rng(4)
    grid = P.Grid(3, 4, 2, (True, True, True))
    N = grid.N
    for coll in ("bgk", "mrt"):
        prm = P.OracleParams(0.7, 0.55, 0.05, 4.0, 3e-4, 1.0, 0.3, (0, 0, 0), s_high=1.1,
                             collision=coll)
        phi = torch.tensor(rng.uniform(0.1, 0.9, N))
        u = torch.tensor(rng.uniform(-0.01, 0.01, (3, N)))
        h = P.equilibrium(L.D3Q15, phi, u, True)
        g = P.equilibrium(L.D3Q27, torch.zeros(N), u, False) + \
            1e-4 * torch.tensor(rng.standard_normal((27, N)))
        _, gs, aux = P.collide(grid, prm, h, g)
        c = L.D3Q27.c
        Pi = torch.einsum("ia,ib,in->abn", c, c, g)
        Pis = torch.einsum("ia,ib,in->abn", c, c, gs)
        ueq = aux["u"]
        Pieq = aux["pstar"][None, None] * CS2 * torch.eye(3, dtype=torch.float64)[:, :, None] + \
            torch.einsum("an,bn->abn", ueq, ueq)
        tau = prm.tau_L + aux["phi"] * (prm.tau_H - prm.tau_L)
        om = 1.0 / tau
        want = Pi + om[None, None] * (Pieq - Pi)
        assert torch.abs(Pis - want).max() < 1e-15


def _bulk_case(seed, s_bulk, N_shape=(3, 4, 2)):
    rng = np.random.default_rng(seed)
    grid = P.Grid(*N_shape, (True, True, True))
    N = grid.N
    prm = P.OracleParams(0.7, 0.55, 0.05, 4.0, 3e-4, 1.0, 0.3, (0, 0, 0), s_high=1.1,
                         s_bulk=s_bulk)
    phi = torch.tensor(rng.uniform(0.1, 0.9, N))
    u = torch.tensor(rng.uniform(-0.01, 0.01, (3, N)))
    h = P.equilibrium(L.D3Q15, phi, u, True)
    g = P.equilibrium(L.D3Q27, torch.zeros(N), u, False) + \
        1e-4 * torch.tensor(rng.standard_normal((27, N)))
    return grid, prm, h, g


def test_hydro_bulk_rate_relaxes_the_trace_of_the_stress():
    """With a separate bulk rate s_b (MRT), the traceless part of Pi = sum c c g
    relaxes at omega and its trace at s_b; mass and the forced first moment
    are as without it; no moment of degree >= 3 changes."""
    for sb in (1.0, 1.7):
        grid, prm, h, g = _bulk_case(5, sb)
        _, gs, aux = P.collide(grid, prm, h, g)
        prm0 = dataclasses.replace(prm, s_bulk=0.0)
        _, gs0, aux0 = P.collide(grid, prm0, h, g)
        c = L.D3Q27.c
        eye = torch.eye(3, dtype=torch.float64)[:, :, None]
        Pi = torch.einsum("ia,ib,in->abn", c, c, g)
        Pis = torch.einsum("ia,ib,in->abn", c, c, gs)
        ueq = aux["u"]
        X = aux["pstar"][None, None] * CS2 * eye + torch.einsum("an,bn->abn", ueq, ueq) - Pi
        tr = (X[0, 0] + X[1, 1] + X[2, 2])[None, None] / 3.0 * eye
        om = 1.0 / (prm.tau_L + aux["phi"] * (prm.tau_H - prm.tau_L))
        want = Pi + om[None, None] * (X - tr) + sb * tr
        assert torch.abs(Pis - want).max() < 1e-15
        assert torch.abs(gs.sum(0) - g.sum(0)).max() < 1e-15
        js = c.t() @ gs
        assert torch.abs(js - (c.t() @ g + aux["F"] / aux["rho"][None])).max() < 1e-15
        # moments of degree >= 3 of the two results agree (rows of the
        # weighted-orthogonal moment matrix)
        hi = L.D3Q27.degree >= 3
        diff = L.D3Q27.M[hi] @ (gs - gs0)
        assert torch.abs(diff).max() < 1e-15
        assert torch.abs(L.D3Q27.M[hi] @ gs0).max() > 1e-6   # the check has content


def test_viscous_force_reads_the_bulk_strain_with_its_own_rate():
    """F_mu recovers (grad u + grad u^T) from Pi_neq mode by mode: a bulk
    (trace) non-equilibrium is read with the bulk rate, so its force scales by
    s_b / omega against s_b = 0; a traceless (shear) non-equilibrium gives the
    same force whatever s_b is."""
    grid = P.Grid(6, 5, 4, (True, True, True))
    N = grid.N
    x = torch.tensor(np.tile(np.arange(6), 20), dtype=torch.float64)
    phi = 0.5 + 0.3 * torch.sin(2 * math.pi * x / 6)           # interface-like gradient
    u = torch.zeros(3, N, dtype=torch.float64)
    h = P.equilibrium(L.D3Q15, phi, u, True)
    g0 = P.equilibrium(L.D3Q27, torch.zeros(N), u, False)
    c, w = L.D3Q27.c, L.D3Q27.w
    bulk = (w * ((c * c).sum(1) - 1.0))[:, None] * torch.ones(1, N, dtype=torch.float64)
    shear = (w * c[:, 0] * c[:, 1])[:, None] * torch.ones(1, N, dtype=torch.float64)
    sb = 1.3
    base = P.OracleParams(0.7, 0.55, 0.05, 4.0, 0.0, 1.0, 0.3, (0, 0, 0))

    def force(pert, s_bulk):
        prm = dataclasses.replace(base, s_bulk=s_bulk)
        return P.collide(grid, prm, h, g0 + 1e-3 * pert)[2]

    ref = P.collide(grid, base, h, g0)[2]["F"]
    a0, ab = force(bulk, 0.0), force(bulk, sb)
    tau = base.tau_L + a0["phi"] * (base.tau_H - base.tau_L)
    fmu0 = a0["F"] - ref
    assert torch.abs(fmu0).max() > 1e-6
    assert torch.abs((ab["F"] - ref) - (sb * tau)[None] * fmu0).max() < 1e-15
    s0, ss = force(shear, 0.0), force(shear, sb)
    assert torch.abs(s0["F"] - ref).max() > 1e-6
    assert torch.abs(ss["F"] - s0["F"]).max() == 0.0


@pytest.mark.parametrize("coll,sb", [("mrt", 0.0), ("bgk", 0.0), ("mrt", 1.3)])
def test_full_guo_source_adds_its_second_moment_to_the_stress(coll, sb):
    """Guo's full source w_i [3 (c - u) + 9 (c.u) c].F / rho has zeroth moment
    0, first F/rho and second (u F^T + F u^T)/rho.  Against the first-order
    source, the collision then changes nothing but the stress, by
    (1 - omega/2)(u F^T + F u^T)/rho in its traceless part and (1 - s_b/2)
    in its trace (s_b = omega without a bulk rate); no moment of degree >= 3
    moves."""
    grid, prm, h, g = _bulk_case(9, sb)
    prm = dataclasses.replace(prm, collision=coll)
    _, g1, a1 = P.collide(grid, dataclasses.replace(prm, forcing="first"), h, g)
    _, g2, a2 = P.collide(grid, dataclasses.replace(prm, forcing="guo"), h, g)
    for k in ("F", "u", "rho"):
        assert torch.equal(a1[k], a2[k])
    c = L.D3Q27.c
    u, F, rho = a1["u"], a1["F"], a1["rho"]
    assert torch.abs(g2.sum(0) - g1.sum(0)).max() < 1e-16
    assert torch.abs(c.t() @ (g2 - g1)).max() < 1e-16
    S = (torch.einsum("an,bn->abn", u, F) + torch.einsum("an,bn->abn", F, u)) / rho[None, None]
    eye = torch.eye(3, dtype=torch.float64)[:, :, None]
    trS = (S[0, 0] + S[1, 1] + S[2, 2])[None, None] / 3.0 * eye
    om = 1.0 / (prm.tau_L + a1["phi"] * (prm.tau_H - prm.tau_L))
    s_tr = om if (sb == 0.0 or coll == "bgk") else torch.full_like(om, sb)
    want = (1 - 0.5 * om)[None, None] * (S - trS) + (1 - 0.5 * s_tr)[None, None] * trS
    dPi = torch.einsum("ia,ib,in->abn", c, c, g2 - g1)
    assert torch.abs(S).max() > 1e-9
    assert torch.abs(dPi - want).max() < 1e-17
    if coll == "mrt":
        hi = L.D3Q27.degree >= 3
        assert torch.abs(L.D3Q27.M[hi] @ (g2 - g1)).max() < 1e-17
