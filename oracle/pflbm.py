"""FP64 CPU oracle of one coupled phase-field LBM time step.

Test infrastructure only (see oracle/__init__.py).  Plain PyTorch CPU ops in
float64, vectorised over cells but otherwise taking the steps of the method
in the order below, with two-buffer (A -> B) streaming and dense
M^-1 S M collision matrices.  Nothing here is shared with the HIP library.

State: h [15, N] (phase field, D3Q15; [27, N] with the D3Q27 phase lattice the
paper uses in 3D, phase_lattice="d3q27") and g [27, N] (hydrodynamics, D3Q27);
with phase_lattice="d2q9" both are D2Q9 [9, N] on an nz = 1 grid (the pair of
the paper's two-dimensional runs, stencils over D2Q9 as well),
post-streaming, with N = nx*ny*nz cells and cell index x + nx*(y + ny*z).
Solid cells hold zeros and are never updated.

One step n -> n+1 (paper sec. "Conservative Allen-Cahn model"):
  S1  phi_c = sum_i h_i                               (eq. zeroth_moment_phase)
  S2  neighbour phi over D3Q27, periodic wrap; a solid or out-of-box
      neighbour takes the cell's own phi (no-flux wall, 90 degree contact)
  S3  grad phi = 3 sum_k w_k c_k (phi_k - phi) ; lap phi = 6 sum_k w_k (phi_k - phi)
      (the gradient is written with the cell's own value subtracted, which is
      the same stencil since sum_k w_k c_k = 0, and is exactly zero on a
      uniform field, so rounding cannot feed the normalised n below)
  S4  n = grad phi / sqrt(|grad phi|^2 + eps^2) ; theta = 4 phi (1-phi) / xi
      (the paper's n = grad phi / |grad phi| regularised where |grad phi| is
      below eps, default 1e-4: far outside the interface, where theta is also
      negligible; a much smaller eps makes the derivative of the step blow up on
      rounding noise in the bulk over long rollouts)
  S5  rho(phi), tau(phi) by linear interpolation, omega = 1/tau
  S6  mu_phi = 4 beta phi (phi-1)(phi-1/2) - kappa lap phi,
      beta = 12 sigma/xi, kappa = 3 sigma xi / 2
  S7  p* = sum_i g_i (eq. zeroth_moment_hydro), j = sum_i c_i g_i
  S8  F_s = mu_phi grad phi, F_b = (rho - rho_g_ref) g (rho_g_ref = 0 as the
      paper writes it; rho_H applies the buoyant part only, a reading that
      moves the heavy phase's hydrostatic pressure into p),
      F_p = -p* c_s^2 (rho_H - rho_L) grad phi
  S9  u' = j + (F_s + F_b + F_p) / (2 rho)
  S10 Pi_neq = sum_i c_i c_i^T (g_i - g_i^eq(p*, u')),
      F_mu = -(1 - omega/2)(rho_H - rho_L) Pi_neq grad phi
      (with a separate bulk rate s_b, MRT only: the trace part of Pi_neq is
      scaled by s_b/omega, so that the force still equals
      nu (rho_H - rho_L)(grad u + grad u^T) grad phi when the trace of the
      strain rate is read from a mode relaxed at s_b)
      (the viscous force from non-equilibrium moments instead of finite
      differences of u, as the paper remarks at the end of the LBE section)
  S11 F = F_s + F_b + F_p + F_mu ; u = j + F / (2 rho)
  S12 g^eq_i = w_i [p* + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u]  (eq. feq, rho_0 = 1)
      F^g_i = 3 w_i c_i.F / rho (first-order source, the default), or Guo's
      full source w_i [3 (c_i - u) + 9 (c_i.u) c_i].F / rho (forcing="guo":
      the paper names Guo's scheme; its second-order part adds
      (u F^T + F u^T)/rho to the second moment of the source)
  S13 g*_i = g_i + [M^-1 S M (g^eq - g)]_i + [M^-1 (I - S/2) M F^g]_i
  S14 h^eq_i = phi w_i [1 + 3 c_i.u + 9/2 (c_i.u)^2 - 3/2 u.u] ; F^h_i = w_i theta c_i.n
  S15 h*_i = h_i + [M^-1 S M (h^eq - h)]_i + [M^-1 (I - S/2) M F^h]_i
  S16 streaming (eq. streaming): f_i(x + c_i) = f*_i(x); if x + c_i is solid
      or outside a wall, f_opp(i)(x) = f*_i(x) (halfway bounce-back)
  S17 phi^{n+1} = sum_i h_i^{n+1}

Relaxation rates (one rate per polynomial degree of the moment basis):
  h: degrees 1 and 2 relax with omega_phi = 1/(3M + 1/2) (tau_phi = M/c_s^2 is
     the relaxation time measured from the half-step, eq. pflbm-tau), degrees
     >= 3 with s_high.
  g: degrees <= 2 relax with omega(phi), degrees >= 3 with s_high; optionally
     (s_bulk > 0) the bulk mode w_i (|c_i|^2 - 1), the trace of the degree-2
     moments, relaxes with s_bulk instead (a reading: the paper relaxes the
     moments after a reference it does not restate; see bulk_part).
  BGK: every degree relaxes with omega_phi (h) or omega(phi) (g) (eq. BGK).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional, Union

import numpy as np
import torch

from .lattice import CS2, D2Q9, D3Q15, D3Q27, Lattice

Num = Union[float, torch.Tensor]
F64 = torch.float64


@dataclasses.dataclass
class OracleParams:
    tau_H: float
    tau_L: float
    mobility: Num
    xi: Num
    sigma: Num
    rho_H: float
    rho_L: float
    g: tuple
    s_high: float = 1.0
    collision: str = "mrt"  # "mrt" or "bgk"
    eps_normal: float = 1e-4
    s_bulk: float = 0.0     # 0: the bulk mode of g relaxes with omega(phi)
    forcing: str = "first"  # "first" or "guo" (source of the g collision, S12)
    phase_lattice: str = "d3q15"  # or "d3q27" (the paper's own 3D phase lattice), or
                                  # "d2q9": the D2Q9 pair of the paper's 2D runs (nz = 1)
    rho_g_ref: float = 0.0  # F_b = (rho - rho_g_ref) g

    @classmethod
    def from_workload(cls, p, collision="mrt", forcing="first",
                      phase_lattice="d3q15") -> "OracleParams":
        return cls(p.tau_H, p.tau_L, p.mobility, p.xi, p.sigma, p.rho_H, p.rho_L,
                   tuple(p.g), p.s_high, collision, p.normal_eps,
                   float(getattr(p, "s_bulk", 0.0)), forcing, phase_lattice,
                   float(getattr(p, "rho_g_ref", 0.0)))


def phase_lattice(name: str) -> Lattice:
    """Velocity set of the phase field: D3Q15 (default), D3Q27, or D2Q9 (the
    two-dimensional pair)."""
    if name == "d3q15":
        return D3Q15
    if name == "d3q27":
        return D3Q27
    if name == "d2q9":
        return D2Q9
    raise ValueError(name)


def hydro_lattice(name: str) -> Lattice:
    """Velocity set of the hydrodynamics (and of the grad/lap stencils): D3Q27
    with either 3D phase lattice, D2Q9 in the two-dimensional pair."""
    return D2Q9 if name == "d2q9" else D3Q27


class Grid:
    """Box of nx*ny*nz cells with per-axis periodicity and an optional solid mask."""

    def __init__(self, nx: int, ny: int, nz: int, periodic=(True, True, True),
                 solid: Optional[np.ndarray] = None):
        self.nx, self.ny, self.nz = nx, ny, nz
        self.N = nx * ny * nz
        self.periodic = tuple(bool(p) for p in periodic)
        if solid is None:
            self.solid = torch.zeros(self.N, dtype=torch.bool)
        else:
            self.solid = torch.as_tensor(np.asarray(solid, dtype=bool).reshape(-1))
        self.fluid = ~self.solid
        z, y, x = torch.meshgrid(torch.arange(nz), torch.arange(ny), torch.arange(nx),
                                 indexing="ij")
        self._xyz = (x.reshape(-1), y.reshape(-1), z.reshape(-1))
        self._cache = {}

    def neighbour(self, c):
        """(index of x + c, valid) for every cell x; valid = inside the box and fluid."""
        key = tuple(int(v) for v in c)
        if key not in self._cache:
            inside = torch.ones(self.N, dtype=torch.bool)
            coords = []
            for ax, (v, n) in enumerate(zip(self._xyz, (self.nx, self.ny, self.nz))):
                t = v + key[ax]
                if self.periodic[ax]:
                    t = torch.remainder(t, n)
                else:
                    inside &= (t >= 0) & (t < n)
                    t = t.clamp(0, n - 1)
                coords.append(t)
            idx = coords[0] + self.nx * (coords[1] + self.ny * coords[2])
            valid = inside & self.fluid[idx]
            self._cache[key] = (idx, valid)
        return self._cache[key]


def _as_t(v) -> torch.Tensor:
    return v if isinstance(v, torch.Tensor) else torch.tensor(float(v), dtype=F64)


def equilibrium(lat: Lattice, zeroth: torch.Tensor, u: torch.Tensor, scale_by_zeroth: bool):
    """Paper eq. feq with rho_0 = 1 (incompressible form).

    g form (scale_by_zeroth=False): w_i [p* + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u]
    h form (scale_by_zeroth=True):  phi w_i [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u]
    """
    cu = lat.c @ u                       # [q, N]
    uu = (u * u).sum(0)                  # [N]
    poly = 3.0 * cu + 4.5 * cu * cu - 1.5 * uu
    w = lat.w[:, None]
    if scale_by_zeroth:
        return w * zeroth * (1.0 + poly)
    return w * (zeroth + poly)


def mrt_apply(lat: Lattice, rates: torch.Tensor, vec: torch.Tensor) -> torch.Tensor:
    """M^-1 diag(rates) M vec, per cell (rates [q, N] or [q, 1])."""
    return lat.Minv @ (rates * (lat.M @ vec))


def bulk_part(lat: Lattice, vec: torch.Tensor) -> torch.Tensor:
    """Component of vec [q, N] along the bulk mode.

    The polynomial b(c) = |c|^2 - 1 = 3 (|c|^2 - c_s^2) lies in the degree-2
    space of the weighted-orthogonal basis (it is orthogonal to 1 and to c
    under <p, q> = sum_i w_i p(c_i) q(c_i)) and is orthogonal to its traceless
    members, so a distribution splits into w_i b(c_i) m_b / <b, b> plus parts
    the other rates act on, with m_b = sum_i b(c_i) vec_i."""
    b = (lat.c * lat.c).sum(1) - 1.0
    norm = (lat.w * b * b).sum()
    return (lat.w * b)[:, None] * ((b[:, None] * vec).sum(0) / norm)[None, :]


def _rates(lat: Lattice, low: torch.Tensor, s_high, bgk: bool, n: int) -> torch.Tensor:
    """Per-moment, per-cell rate: degree <= 2 -> low, degree >= 3 -> s_high (or low if BGK)."""
    low = low.reshape(1, -1).expand(lat.q, n) if low.dim() > 0 else low.reshape(1, 1).expand(lat.q, n)
    hi = low if bgk else torch.full_like(low, float(s_high))
    return torch.where((lat.degree >= 3)[:, None], hi, low)


def collide(grid: Grid, prm: OracleParams, h: torch.Tensor, g: torch.Tensor):
    """S1-S15.  Returns (h*, g*, aux) where aux holds the cell moments and forces."""
    LH, LG = phase_lattice(prm.phase_lattice), hydro_lattice(prm.phase_lattice)
    if LG is D2Q9 and (grid.nz != 1 or prm.s_bulk > 0):
        raise ValueError("the D2Q9 pair needs nz = 1 and no separate bulk rate")
    N = grid.N
    bgk = prm.collision == "bgk"
    drho = prm.rho_H - prm.rho_L
    # S1 (the phi field of S2 is the same quantity, phi^n = sum_i h_i^n)
    phi = h.sum(0)
    # S2, S3
    grad = torch.zeros(3, N, dtype=F64)
    lap = torch.zeros(N, dtype=F64)
    for k in range(LG.q):
        ck = LG.c_np[k]
        idx, valid = grid.neighbour(ck)
        phik = torch.where(valid, phi[idx], phi)
        grad = grad + 3.0 * LG.w[k] * LG.c[k][:, None] * (phik - phi)[None, :]
        lap = lap + 6.0 * LG.w[k] * (phik - phi)
    # S4
    normal = grad / torch.sqrt((grad * grad).sum(0) + prm.eps_normal ** 2)
    xi_inf = math.isinf(float(prm.xi.detach()) if isinstance(prm.xi, torch.Tensor) else float(prm.xi))
    if xi_inf:
        theta = torch.zeros(N, dtype=F64)
    else:
        theta = 4.0 * phi * (1.0 - phi) / _as_t(prm.xi)
    # S5
    rho = prm.rho_L + phi * drho
    tau = prm.tau_L + phi * (prm.tau_H - prm.tau_L)
    omega = 1.0 / tau
    # S6
    sigma = _as_t(prm.sigma)
    if xi_inf:
        mu = torch.zeros(N, dtype=F64)
    else:
        xi = _as_t(prm.xi)
        beta = 12.0 * sigma / xi
        kappa = 1.5 * sigma * xi
        mu = 4.0 * beta * phi * (phi - 1.0) * (phi - 0.5) - kappa * lap
    # S7
    pstar = g.sum(0)
    j = LG.c.t() @ g                      # [3, N]
    # S8
    Fs = mu[None, :] * grad
    gvec = torch.tensor(prm.g, dtype=F64)[:, None]
    Fb = (rho - prm.rho_g_ref)[None, :] * gvec
    Fp = -(pstar * CS2 * drho)[None, :] * grad
    # S9
    u1 = j + (Fs + Fb + Fp) / (2.0 * rho[None, :])
    # S10
    geq1 = equilibrium(LG, pstar, u1, False)
    neq = g - geq1
    Pi = torch.einsum("ia,ib,in->abn", LG.c, LG.c, neq)
    bulk = (not bgk) and prm.s_bulk > 0
    if bulk:
        tr = (Pi[0, 0] + Pi[1, 1] + Pi[2, 2]) / 3.0
        Pi = Pi + (prm.s_bulk * tau - 1.0)[None, None, :] * tr[None, None, :] \
            * torch.eye(3, dtype=F64)[:, :, None]
    Fmu = -((1.0 - 0.5 * omega) * drho)[None, :] * torch.einsum("abn,bn->an", Pi, grad)
    # S11
    F = Fs + Fb + Fp + Fmu
    u = j + F / (2.0 * rho[None, :])
    # S12, S13
    geq = equilibrium(LG, pstar, u, False)
    cF = LG.c @ F                        # [q, N]
    if prm.forcing == "guo":
        cu = LG.c @ u
        uF = (u * F).sum(0)
        Fg = LG.w[:, None] * (3.0 * cF + 9.0 * cu * cF - 3.0 * uF[None, :]) / rho[None, :]
    elif prm.forcing == "first":
        Fg = 3.0 * LG.w[:, None] * cF / rho[None, :]
    else:
        raise ValueError(prm.forcing)
    sg = _rates(LG, omega, prm.s_high, bgk, N)
    gstar = g + mrt_apply(LG, sg, geq - g) + mrt_apply(LG, 1.0 - 0.5 * sg, Fg)
    if bulk:   # the bulk mode at s_b: relaxation s_b, source factor 1 - s_b/2
        sb = (prm.s_bulk - omega)[None, :]
        gstar = gstar + sb * bulk_part(LG, geq - g) - 0.5 * sb * bulk_part(LG, Fg)
    # S14, S15
    heq = equilibrium(LH, phi, u, True)
    Fh = LH.w[:, None] * theta[None, :] * (LH.c @ normal)
    omega_phi = 1.0 / (3.0 * _as_t(prm.mobility) + 0.5)
    sh = _rates(LH, omega_phi, prm.s_high, bgk, N)
    hstar = h + mrt_apply(LH, sh, heq - h) + mrt_apply(LH, 1.0 - 0.5 * sh, Fh)
    fl = grid.fluid[None, :]
    hstar = torch.where(fl, hstar, torch.zeros_like(hstar))
    gstar = torch.where(fl, gstar, torch.zeros_like(gstar))
    aux = dict(phi=phi, u=u, pstar=pstar, rho=rho, F=F, grad=grad, lap=lap, mu=mu)
    return hstar, gstar, aux


def stream(grid: Grid, lat: Lattice, fstar: torch.Tensor) -> torch.Tensor:
    """S16 in pull form: f_i(x) = f*_i(x - c_i), or f*_opp(i)(x) if x - c_i is a wall/solid."""
    rows = []
    for i in range(lat.q):
        idx, valid = grid.neighbour(-lat.c_np[i])
        rows.append(torch.where(valid, fstar[i][idx], fstar[lat.opp[i]]))
    out = torch.stack(rows)
    return torch.where(grid.fluid[None, :], out, torch.zeros_like(out))


def step(grid: Grid, prm: OracleParams, h: torch.Tensor, g: torch.Tensor):
    hs, gs, _ = collide(grid, prm, h, g)
    return (stream(grid, phase_lattice(prm.phase_lattice), hs),
            stream(grid, hydro_lattice(prm.phase_lattice), gs))


def run(grid: Grid, prm: OracleParams, h, g, nsteps: int):
    for _ in range(nsteps):
        h, g = step(grid, prm, h, g)
    return h, g


def init_equilibrium(grid: Grid, phi0, u0, pstar0, phase: str = "d3q15"):
    """h = phi0 w_i [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u], g = g^eq(p*0, u0); zero in solids.

    phi0 [N] or [nz,ny,nx]; u0 [3, ...]; pstar0 like phi0 (numpy or torch);
    phase: the phase field's velocity set ("d3q15", "d3q27" or "d2q9", the
    last with the D2Q9 hydrodynamics).
    """
    phi0 = torch.as_tensor(phi0, dtype=F64).reshape(-1)
    u0 = torch.as_tensor(u0, dtype=F64).reshape(3, -1)
    pstar0 = torch.as_tensor(pstar0, dtype=F64).reshape(-1)
    h = equilibrium(phase_lattice(phase), phi0, u0, True)
    g = equilibrium(hydro_lattice(phase), pstar0, u0, False)
    fl = grid.fluid[None, :]
    return torch.where(fl, h, torch.zeros_like(h)), torch.where(fl, g, torch.zeros_like(g))


def moments(grid: Grid, prm: OracleParams, h, g):
    """(phi, u [3,N], p*) of the current state, with the force-corrected velocity."""
    _, _, aux = collide(grid, prm, h, g)
    fl = grid.fluid
    z = torch.zeros((), dtype=F64)
    return (torch.where(fl, aux["phi"], z), torch.where(fl[None], aux["u"], z),
            torch.where(fl, aux["pstar"], z))


def reductions(grid: Grid, h, g, phase: str = "d3q15"):
    """[sum phi, sum p*, sum j_x, sum j_y, sum j_z] over fluid cells (fp64)."""
    fl = grid.fluid
    phi = h.sum(0)[fl].sum()
    ps = g.sum(0)[fl].sum()
    j = (hydro_lattice(phase).c.t() @ g)[:, fl].sum(1)
    return torch.stack([phi, ps, j[0], j[1], j[2]])


def amplitude(grid: Grid, h, depth: float, x0: int = 0):
    """Interface elevation a = <sum_y phi(x0, y, z)>_z - depth (column sum of phi)."""
    phi = h.sum(0).reshape(grid.nz, grid.ny, grid.nx)
    return phi[:, :, x0].sum(1).mean() - depth


def interface_crossing(phi_col: np.ndarray, near: float) -> float:
    """Position y where phi = 1/2 by linear interpolation between cell centres,
    choosing the crossing nearest to `near` (paper: elevation of the phi = 0.5
    level, sec. gravity-wave setup)."""
    phi_col = np.asarray(phi_col, dtype=np.float64)
    best = None
    for j in range(len(phi_col) - 1):
        a, b = phi_col[j] - 0.5, phi_col[j + 1] - 0.5
        if a == 0.0 or a * b < 0:
            y = (j + 0.5) + a / (a - b)
            if best is None or abs(y - near) < abs(best - near):
                best = y
    return float("nan") if best is None else best
