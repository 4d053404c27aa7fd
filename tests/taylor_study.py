"""Taylor bubble rising in a vertical tube, run through the library and
compared with the Reynolds numbers the paper reports for its PFLBM (sec.
"Taylor bubble", table of Re: 26.83 at D = 64, 27.12 at D = 128; D <= 32
reported unstable).

Setup (paper): a D x D x 10D box holding a no-slip cylindrical tube of
diameter D along the long axis, with no-slip walls at both ends; a gas
cylinder of diameter 0.75 D and length 3 D, coaxial with the tube, its bottom
at height D; the rest liquid at rest.  Bo = 100 and Mo = 0.015 on the tube
diameter and the heavy phase (eq. Mo, eq. Bo), density ratio 744, dynamic
viscosity ratio 4236, M = 0.08, xi = 3, heavy-phase relaxation rate 1.76.
The liquid starts in hydrostatic balance with the reference pressure
p0 = rho_0 c_s^2 = 1/3 at height 5D.  The rise velocity U comes from the
bubble's centre of mass at t* = 10 and t* = 15, with t* = t sqrt(g / D), and
Re = rho_H D U / mu_H (eq. Re).

Readings (where the setup leaves a choice):
  * The long axis is y, gravity along -y; x and z carry box walls, so the
    tube's wall is the bounce-back boundary of the cells outside radius D/2
    (cell centres) together with the box faces.
  * g and sigma follow from Bo and Mo with mu_H = rho_H (1/1.76 - 1/2) / 3;
    the light phase's relaxation time from mu_L = mu_H / 4236 and
    rho_L = rho_H / 744.
  * The gas cylinder's phase field is the tanh profile of the signed
    distance to the capped cylinder (flat ends).
  * Pressure: the library carries p* = p / (rho c_s^2).  The liquid starts at
    p = p0 + rho_H g (5D - y), the gas at the uniform pressure of the liquid
    at the bubble's mid-height, p is blended by phi across the interface and
    p* = 3 p / rho(phi).  In the continuum a constant added to p changes
    nothing; the discrete model sees it through F_p = -p* c_s^2 (rho_H -
    rho_L) grad phi, whose balance against rho c_s^2 grad p* across the
    interface is only approximate, with an error that grows with |p*| in the
    gas.  With the paper's p0 = 1/3 the gas starts at p* ~ 750 and every run
    diverges within the first unit of t* (gauge="paper"); the study therefore
    starts from p = 0 at the bubble's mid-height (gauge="mid", the default),
    where the gas starts at p* = 0.
  * Centre of mass: sum (1 - phi) y / sum (1 - phi) over the gas region
    (fluid cells with phi < 1/2); the same over all fluid cells, which also
    collects the liquid's small overshoot of phi above 1, is reported beside
    it.
  * Collision: MRT with the bulk mode of g (the trace of its second-order
    moments) relaxed at rate 1 (s_bulk = 1).  The paper relaxes the moments
    after a reference it does not restate; with the bulk mode at omega(phi)
    instead, the gas (tau_L = 0.512 at these ratios) has almost no bulk
    viscosity and every run here diverges within ~200 steps, with or without
    gravity or surface tension (s_bulk = 0 reproduces that).

Host-side glue only: the time stepping runs in the library.  Run as a
script for the study:
    python tests/taylor_study.py [--D 64 128] [--precision fp64 fp32]
                                 [--gauge mid paper buoyant] [--s-bulk 1] [--every 0.5]
                                 [--tmax 15] [--out FILE]
    python tests/taylor_study.py --diagnose --D 64 --precision fp32 --every 0.5
"""
from __future__ import annotations

import argparse
import dataclasses
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "taylor_bubble.txt")


def golden(path: str = GOLDEN) -> dict:
    """The paper's printed setup and Re values (tests/golden/taylor_bubble.txt)."""
    out = {}
    for line in open(path):
        line = line.split("#", 1)[0].strip()
        if not line:
            continue
        k, v = (s.strip() for s in line.split("=", 1))
        vals = [float(t) for t in v.split()]
        out[k] = vals[0] if len(vals) == 1 else vals
    return out


_G = golden()
BO, MO, RHO_RATIO, MU_RATIO = _G["Bo"], _G["Mo"], _G["density_ratio"], _G["viscosity_ratio"]
OMEGA_H, MOBILITY, XI = _G["omega_H"], _G["mobility"], _G["xi"]
RE_PAPER = {64: _G["Re_PFLBM_D64"], 128: _G["Re_PFLBM_D128"]}
UNSTABLE_PAPER = {int(d) for d in (_G["PFLBM_unstable_D"] if isinstance(_G["PFLBM_unstable_D"], (list, tuple))
                                   else [_G["PFLBM_unstable_D"]])}


@dataclasses.dataclass(frozen=True)
class Constants:
    D: int
    g: float
    sigma: float
    tau_H: float
    tau_L: float
    mu_H: float
    rho_L: float
    t_ref: float          # steps per unit of t* = sqrt(D / g)


def constants(D: int) -> Constants:
    """Lattice g, sigma and relaxation times from Bo, Mo and the ratios.

    With rho_H = 1: Bo = g D^2 / sigma and Mo = g mu^4 / sigma^3 give
    g = mu^2 sqrt(Bo^3 / Mo) / D^3 and sigma = g D^2 / Bo."""
    tau_H = 1.0 / OMEGA_H
    mu_H = (tau_H - 0.5) / 3.0
    g = mu_H ** 2 * math.sqrt(BO ** 3 / MO) / D ** 3
    sigma = g * D * D / BO
    rho_L = 1.0 / RHO_RATIO
    nu_L = (mu_H / MU_RATIO) / rho_L
    return Constants(D, g, sigma, tau_H, 3.0 * nu_L + 0.5, mu_H, rho_L, math.sqrt(D / g))


def setup(D: int, gauge: str = "mid", s_bulk: float = 1.0):
    """Workload of one Taylor-bubble run and its constants."""
    c = constants(D)
    lx, ly, lz = (int(round(v * D)) for v in _G["domain"])     # the paper's x, y, z
    nx, ny, nz = lx, lz, ly                                    # its tube axis z is our y
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij")
    rr = np.sqrt((x - 0.5 * D) ** 2 + (z - 0.5 * D) ** 2)
    solid = rr > 0.5 * D
    R = 0.5 * _G["bubble_diameter"] * D
    y0 = _G["bubble_bottom"] * D
    y1 = y0 + _G["bubble_length"] * D
    dist = np.maximum(np.maximum(rr - R, y0 - y), y - y1)      # > 0 outside the gas
    phi0 = W.tanh_profile(dist, XI)
    del rr, x, z
    ymid = 0.5 * (y0 + y1)
    if gauge == "paper":
        yref = _G["reference_pressure_height"] * D
        p_liq = 1.0 / 3.0 + c.g * (yref - y)
        p_gas = 1.0 / 3.0 + c.g * (yref - ymid)
    elif gauge == "mid":
        p_liq = c.g * (ymid - y)
        p_gas = 0.0
    elif gauge == "buoyant":
        # gravity on rho - rho_H (rho_g_ref = rho_H): the liquid carries no
        # hydrostatic pressure, the gas the one of its net upward force
        p_liq = np.zeros_like(y)
        p_gas = (c.rho_L - 1.0) * c.g * (ymid - y)
    else:
        raise ValueError(gauge)
    rho = c.rho_L + phi0 * (1.0 - c.rho_L)
    pstar = 3.0 * (phi0 * p_liq + (1.0 - phi0) * p_gas) / rho
    pstar[solid] = 0.0
    phi0[solid] = 0.0
    p = W.Params(tau_H=c.tau_H, tau_L=c.tau_L, mobility=MOBILITY, xi=XI, sigma=c.sigma,
                 rho_H=1.0, rho_L=c.rho_L, g=(0.0, -c.g, 0.0), s_bulk=s_bulk,
                 rho_g_ref=1.0 if gauge == "buoyant" else 0.0)
    steps = int(math.ceil(15.0 * c.t_ref))
    wl = W.Workload(f"taylor_bubble_D{D}_{nx}x{ny}x{nz}", nx, ny, nz, (False, False, False), p,
                    phi0, np.zeros((3, nz, ny, nx)), pstar, solid, steps)
    return wl, c


def reynolds(c: Constants, y10: float, y15: float) -> float:
    """Re = rho_H D U / mu_H with U from the centre of mass at t* = 10 and 15."""
    U = (y15 - y10) / (5.0 * c.t_ref)
    return float(c.D) * U / c.mu_H


def run(D: int, precision: str = "fp64", gauge: str = "mid", streaming: str = "ab",
        tmax: float = 15.0, s_bulk: float = 1.0, every: float = 0.5, log=None,
        phase_lattice: str = "d3q15"):
    """Simulate to t* = tmax, sampling the centre of mass every `every` of t*.

    Re is the paper's (t* = 10 to 15) when the run reaches t* = 15; a run that
    diverges earlier reports Re over t* = 10 to its last finite sample as
    "Re_last" with that window."""
    import torch

    from paper_2206_11637_amd.sim import from_workload
    wl, c = setup(D, gauge, s_bulk)
    fluid = torch.as_tensor(~wl.solid, device="cuda:0")
    yy = (torch.arange(wl.ny, dtype=torch.float64, device="cuda:0") + 0.5).view(1, wl.ny, 1)
    sim = from_workload(wl, precision=precision, collision="mrt", streaming=streaming,
                        phase_lattice=phase_lattice)
    del wl.phi0, wl.pstar0, wl.u0

    def centre(phi):
        light = torch.where(fluid, 1.0 - phi, torch.zeros_like(phi))
        vol = float(light.sum())
        gas = torch.where(phi < 0.5, light, torch.zeros_like(light))
        return float((gas * yy).sum() / gas.sum()), vol, float((light * yy).sum()) / vol

    m0 = sim.reduce()[0]
    t0 = time.time()
    ts, ys, ys_all, vols, done = [], [], [], [], 0
    nsamp = int(round(tmax / every))
    finite = True
    for i in range(nsamp + 1):
        s = int(round(i * every * c.t_ref))
        if s > done:
            sim.step(s - done)
        done = s
        phi = sim.phi()
        if not bool(torch.isfinite(phi).all()):
            finite = False
            if log:
                log(f"  D={D} {precision} {gauge}: non-finite phi at t*={i * every:g} (step {s})")
            break
        yc, vol, yc_all = centre(phi)
        ts.append(i * every)
        ys.append(yc)
        ys_all.append(yc_all)
        vols.append(vol)
        del phi
        if log:
            log(f"  D={D} {precision} {gauge}: t*={i * every:5.2f} step {s:6d} centre {yc:8.3f} "
                f"gas volume {vol:10.1f} ({time.time() - t0:.0f} s)")
    torch.cuda.synchronize()
    out = dict(D=D, precision=precision, gauge=gauge, streaming=streaming, s_bulk=s_bulk,
               phase_lattice=phase_lattice,
               g=c.g, sigma=c.sigma,
               tau_H=c.tau_H, tau_L=c.tau_L, t_ref=c.t_ref, steps=done, finite=finite,
               tstar=ts, centre=ys, centre_all_cells=ys_all, gas_volume=vols,
               seconds=time.time() - t0,
               mass_drift=float((sim.reduce()[0] - m0) / m0) if finite else None,
               re_paper=RE_PAPER.get(D))
    tv = {round(t, 6): y for t, y in zip(ts, ys)}
    if 15.0 in tv and 10.0 in tv:
        out["Re"] = reynolds(c, tv[10.0], tv[15.0])
        ta = {round(t, 6): y for t, y in zip(ts, ys_all)}
        out["Re_all_cells"] = reynolds(c, ta[10.0], ta[15.0])
    elif ts and ts[-1] > 10.0 and 10.0 in tv:
        U = (ys[-1] - tv[10.0]) / ((ts[-1] - 10.0) * c.t_ref)
        out["Re_last"] = float(c.D) * U / c.mu_H
        ta = {round(t, 6): y for t, y in zip(ts, ys_all)}
        U_all = (ys_all[-1] - ta[10.0]) / ((ts[-1] - 10.0) * c.t_ref)
        out["Re_last_all_cells"] = float(c.D) * U_all / c.mu_H
        out["Re_last_window"] = (10.0, ts[-1])
    del sim
    torch.cuda.empty_cache()
    return out


def field_stats(sim, fluid):
    """Diagnostics of one state: the phase field's range over fluid cells, and
    max |u| with its cell and the p* range in the gas (phi < 1/2) and in the
    liquid."""
    import torch
    phi, u, ps = sim.moments()
    umag = torch.sqrt((u * u).sum(0))
    gas = fluid & (phi < 0.5)
    liq = fluid & (phi >= 0.5)
    out = dict(phi_min=float(phi[fluid].min()), phi_max=float(phi[fluid].max()))
    for name, m in (("gas", gas), ("liquid", liq)):
        um = torch.where(m, umag, torch.zeros_like(umag))
        k = int(torch.argmax(um))
        nz, ny, nx = phi.shape
        out[f"umax_{name}"] = float(um.reshape(-1)[k])
        out[f"umax_{name}_cell"] = (k % nx, (k // nx) % ny, k // (nx * ny))
        out[f"pstar_{name}"] = (float(ps[m].min()), float(ps[m].max()))
    del phi, u, ps, umag
    return out


def force_terms(sim, wl, cell, half=3):
    """The four force terms of the cells around `cell` (x, y, z): the state's
    populations are read back and the oracle's collision is evaluated on a
    (2 half + 1)^3 window (walls at its faces, so only the inner cells are
    exact).  Returns the largest |F_s|, |F_b|, |F_p|, |F_mu| and |u| over the
    window's inner cube, and phi, p* at the cell itself."""
    import torch

    from gpu_util import gpu_pops_oracle_order
    from oracle import pflbm as OP
    h, g = gpu_pops_oracle_order(sim)
    nz, ny, nx = wl.nz, wl.ny, wl.nx
    x, y, z = cell
    xs = slice(max(x - half, 0), min(x + half + 1, nx))
    ys = slice(max(y - half, 0), min(y + half + 1, ny))
    zs = slice(max(z - half, 0), min(z + half + 1, nz))
    hw = h.reshape(h.shape[0], nz, ny, nx)[:, zs, ys, xs].reshape(h.shape[0], -1).clone()
    gw = g.reshape(27, nz, ny, nx)[:, zs, ys, xs].reshape(27, -1).clone()
    del h, g
    sol = wl.solid[zs, ys, xs]
    grid = OP.Grid(sol.shape[2], sol.shape[1], sol.shape[0], (False, False, False), sol)
    prm = OP.OracleParams.from_workload(wl.params, "mrt")
    _, _, aux = OP.collide(grid, prm, hw, gw)
    drho = prm.rho_H - prm.rho_L
    Fs = aux["mu"][None] * aux["grad"]
    Fb = (aux["rho"] - prm.rho_g_ref)[None] * torch.tensor(prm.g, dtype=torch.float64)[:, None]
    Fp = -(aux["pstar"] * drho / 3.0)[None] * aux["grad"]
    Fmu = aux["F"] - Fs - Fb - Fp
    shp = sol.shape
    inner = torch.zeros(shp, dtype=torch.bool)
    inner[1:-1, 1:-1, 1:-1] = True
    inner &= ~torch.as_tensor(sol)
    inner = inner.reshape(-1)

    def mx(v):
        return float(torch.sqrt((v * v).sum(0))[inner].max())
    c = ((z - zs.start) * shp[1] + (y - ys.start)) * shp[2] + (x - xs.start)
    return dict(F_s=mx(Fs), F_b=mx(Fb), F_p=mx(Fp), F_mu=mx(Fmu), u=mx(aux["u"]),
                phi=float(aux["phi"][c]), pstar=float(aux["pstar"][c]))


def diagnose(D: int, precision: str = "fp32", tmax: float = 15.0, every: float = 0.5, log=print):
    """Run to t* = tmax recording field_stats every `every`; if the run turns
    non-finite, step again one step at a time from the last finite sample to
    the first step with a non-finite phase field, and report the statistics of
    the steps before it and the force terms around the cell where the
    velocity peaks."""
    import torch

    from paper_2206_11637_amd.sim import from_workload
    wl, c = setup(D)
    fluid = torch.as_tensor(~wl.solid, device="cuda:0")
    sim = from_workload(wl, precision=precision, collision="mrt")
    samples, done, last_ok = [], 0, None
    nsamp = int(round(tmax / every))
    bad_at = None
    for i in range(nsamp + 1):
        s = int(round(i * every * c.t_ref))
        if s > done:
            sim.step(s - done)
        done = s
        if not bool(torch.isfinite(sim.phi()).all()):
            bad_at = s
            break
        st = field_stats(sim, fluid)
        st.update(tstar=i * every, step=s)
        samples.append(st)
        last_ok = (s, sim.save_state())
        log(f"  t*={i * every:5.2f} step {s:6d} phi [{st['phi_min']:+.3f}, {st['phi_max']:.3f}] "
            f"|u|max gas {st['umax_gas']:.3e} at {st['umax_gas_cell']} liquid {st['umax_liquid']:.3e} "
            f"p* gas [{st['pstar_gas'][0]:+.3f}, {st['pstar_gas'][1]:+.3f}] "
            f"liquid [{st['pstar_liquid'][0]:+.3f}, {st['pstar_liquid'][1]:+.3f}]")
    out = dict(D=D, precision=precision, samples=samples, first_nonfinite_step=None)
    if bad_at is None:
        return out
    s0, buf = last_ok
    sim.load_state(buf, s0)
    steps = []
    n = s0
    while n < bad_at:
        st = field_stats(sim, fluid)
        st.update(step=n, tstar=n / c.t_ref)
        steps.append(st)
        sim.step(1)
        n += 1
        if not bool(torch.isfinite(sim.phi()).all()):
            break
    out["first_nonfinite_step"] = n
    out["first_nonfinite_tstar"] = n / c.t_ref
    out["last_steps"] = steps[-20:]
    log(f"  first non-finite phase field after step {n} (t* = {n / c.t_ref:.3f})")
    for st in steps[-8:]:
        log(f"    step {st['step']}: |u|max gas {st['umax_gas']:.3e} at {st['umax_gas_cell']} "
            f"liquid {st['umax_liquid']:.3e} at {st['umax_liquid_cell']} "
            f"p* gas [{st['pstar_gas'][0]:+.3f}, {st['pstar_gas'][1]:+.3f}]")
    # force terms around the peak velocity a few steps before the fault
    back = max(s0, n - 6)
    sim.load_state(buf, s0)
    if back > s0:
        sim.step(back - s0)
    st = field_stats(sim, fluid)
    for name in ("gas", "liquid"):
        cell = st[f"umax_{name}_cell"]
        f = force_terms(sim, wl, cell)
        out[f"forces_step{back}_{name}_peak"] = dict(cell=cell, **f)
        log(f"  step {back}, peak |u| in the {name} at {cell}: " +
            " ".join(f"{k} {v:.3e}" if isinstance(v, float) else f"{k} {v}" for k, v in f.items()))
    return out


def write_table(res, path, argv):
    """Results table (markdown) of the runs in res."""
    rows = ["| D | lattice | precision | phase lattice | steps | Re, gas region | Re, all cells | "
            "window t* | paper PFLBM | phase-mass drift | GPU s |",
            "|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in res:
        D = r["D"]
        lat = f"{D}x{10 * D}x{D}"
        if "Re" in r:
            re_gas, re_all, win = f"{r['Re']:.3f}", f"{r['Re_all_cells']:.3f}", "10-15"
        elif "Re_last" in r:
            re_gas, re_all = f"{r['Re_last']:.3f}", f"{r.get('Re_last_all_cells', float('nan')):.3f}"
            win = f"10-{r['Re_last_window'][1]:g} (non-finite before 15)"
        else:
            re_gas, re_all, win = "diverges", "", ""
        paper = r["re_paper"] or ("unstable" if D in UNSTABLE_PAPER else "-")
        drift = r.get("mass_drift")
        drift = f"{drift:.1e}" if isinstance(drift, float) else "-"
        rows.append(f"| {D} | {lat} | {r['precision']} | {r.get('phase_lattice', 'd3q15')} | {r['steps']} | "
                    f"{re_gas} | {re_all} | {win} | {paper} | {drift} | {r['seconds']:.0f} |")
    head = ("# The paper's Taylor bubble on the GPU: Reynolds number of the rise\n\n"
            "Written by `python tests/taylor_study.py " + argv + "` on one MI355X (MRT with the bulk\n"
            "rate s_bulk = 1, two buffers; Re = rho_H D U / mu_H with U the rise velocity of the centre of\n"
            "mass over the window; gas region: weights 1 - phi over cells with phi < 1/2; all cells: over\n"
            "every fluid cell).\n\n")
    with open(path, "w") as f:
        f.write(head + "\n".join(rows) + "\n")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--D", type=int, nargs="+", default=[64, 128])
    ap.add_argument("--precision", nargs="+", default=["fp64"])
    ap.add_argument("--gauge", nargs="+", default=["mid"])
    ap.add_argument("--s-bulk", type=float, default=1.0)
    ap.add_argument("--tmax", type=float, default=15.0)
    ap.add_argument("--every", type=float, default=0.5)
    ap.add_argument("--phase-lattice", default="d3q15", choices=["d3q15", "d3q27"])
    ap.add_argument("--out", default=None)
    ap.add_argument("--table", default=None, help="write a markdown table of the runs here")
    ap.add_argument("--diagnose", action="store_true",
                    help="per-sample diagnostics and the first non-finite step (first --D, --precision)")
    args = ap.parse_args()

    def log(m):
        print(m, flush=True)

    if args.diagnose:
        r = diagnose(args.D[0], args.precision[0], args.tmax, args.every, log)
        if args.out:
            with open(args.out, "w") as f:
                json.dump(r, f)
        return

    res = []
    for D in args.D:
        for prec in args.precision:
            for gauge in args.gauge:
                log(f"Taylor bubble D={D} {prec} gauge={gauge} s_bulk={args.s_bulk} "
                    f"phase lattice {args.phase_lattice}")
                r = run(D, prec, gauge, tmax=args.tmax, s_bulk=args.s_bulk, every=args.every,
                        log=log, phase_lattice=args.phase_lattice)
                if "Re" in r:
                    what = (f"Re(t* 10-15) = {r['Re']:.3f} (all-cell weights "
                            f"{r['Re_all_cells']:.3f})")
                elif "Re_last" in r:
                    what = f"Re(t* 10-{r['Re_last_window'][1]:g}) = {r['Re_last']:.3f}"
                else:
                    what = "Re not available"
                log(f"  {what} (paper PFLBM {r['re_paper']}) mass drift {r['mass_drift']} "
                    f"[{r['steps']} steps, {r['seconds']:.0f} s]")
                res.append(r)
                if args.out:
                    with open(args.out, "w") as f:
                        json.dump(res, f)
                if args.table:
                    write_table(res, args.table, " ".join(sys.argv[1:]))


if __name__ == "__main__":
    main()
