"""Rising gas bubbles in an 8D x 8D x 20D box, run through the library and
compared with the Reynolds numbers the paper reports for its PFLBM (sec.
"Rising bubble": four cases of Bo, Mo and heavy-phase rate; PFLBM Re at
D = 32 and 64, unstable at D = 8 and 16), from tests/golden/rising_bubbles.txt.

Setup (paper): a spherical gas bubble of diameter D centred at (4D, 4D, 1D)
in an 8D x 8D x 20D box, periodic on the sides and no-slip at the top and
bottom; Bo and Mo on D and the heavy phase (eq. Bo, eq. Mo), density ratio
1000, dynamic viscosity ratio 100, M = 0.02, xi = 5; Re = rho_H D U / mu_H
(eq. Re) with U from the centre of mass at t* = 5 and 10, t* = t sqrt(g/D).

Readings (as for the Taylor bubble, tests/taylor_study.py): the vertical axis
is y (gravity along -y); g and sigma follow from Bo and Mo with
mu_H = (1/omega_H - 1/2)/3 and the light phase's relaxation time from the
viscosity ratio; the liquid starts hydrostatic with p = 0 at the bubble's
centre height and the gas at p = 0 (the paper's reference pressure puts the
gas at p* ~ 3000, where the discrete F_p balance fails); MRT with s_bulk = 1;
the bubble's centre of mass weights the gas region (phi < 1/2) with 1 - phi
(summed over the whole box, 1 - phi would also collect the liquid's small
overshoot of phi above 1, which over a liquid volume ~2000 times the
bubble's outweighs the bubble; that sum is reported beside it).

Also recorded: the bubble's volume (cells with phi < 1/2) against the
initial sphere at each sample.

Host-side glue only.  Run as a script:
    python tests/rising_bubble_study.py [--cases 1 2 3 4] [--D 32] [--precision fp32]
"""
from __future__ import annotations

import argparse
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

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rising_bubbles.txt")


def golden(path: str = GOLDEN) -> dict:
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


def constants(case: int, D: int) -> dict:
    """Lattice g, sigma and relaxation times of one case at bubble diameter D."""
    Bo, Mo, omega_H = _G[f"case{case}"]
    tau_H = 1.0 / omega_H
    mu_H = (tau_H - 0.5) / 3.0
    g = mu_H ** 2 * math.sqrt(Bo ** 3 / Mo) / D ** 3
    sigma = g * D * D / Bo
    rho_L = 1.0 / _G["density_ratio"]
    nu_L = (mu_H / _G["dynamic_viscosity_ratio"]) / rho_L
    return dict(case=case, D=D, Bo=Bo, Mo=Mo, g=g, sigma=sigma, tau_H=tau_H,
                tau_L=3.0 * nu_L + 0.5, mu_H=mu_H, rho_L=rho_L, t_ref=math.sqrt(D / g))


def setup(case: int, D: int, s_bulk: float = 1.0, buoyant: bool = False):
    """buoyant: gravity acts on rho - rho_H (rho_g_ref = rho_H); the liquid
    then starts at p = 0 and the gas with the hydrostatic pressure of its net
    upward force.  Otherwise gravity acts on rho, with the liquid's
    hydrostatic start."""
    c = constants(case, D)
    lx, ly, lz = (int(round(v * D)) for v in _G["domain"])        # the paper's x, y, z
    nx, ny, nz = lx, lz, ly                                        # its vertical z is our y
    cx, cy, cz = (v * D for v in _G["bubble_centre"])
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij")
    r = np.sqrt((x - cx) ** 2 + (y - cz) ** 2 + (z - cy) ** 2)
    del x, z
    phi0 = W.tanh_profile(r - 0.5 * D, _G["xi"])
    del r
    rho = c["rho_L"] + phi0 * (1.0 - c["rho_L"])
    if buoyant:
        pstar = 3.0 * (1.0 - phi0) * (c["rho_L"] - 1.0) * c["g"] * (cz - y) / rho
    else:
        pstar = 3.0 * phi0 * c["g"] * (cz - y) / rho
    p = W.Params(tau_H=c["tau_H"], tau_L=c["tau_L"], mobility=_G["mobility"], xi=_G["xi"],
                 sigma=c["sigma"], rho_H=1.0, rho_L=c["rho_L"], g=(0.0, -c["g"], 0.0),
                 s_bulk=s_bulk, rho_g_ref=1.0 if buoyant else 0.0)
    wl = W.Workload(f"rising_bubble_case{case}_D{D}_{nx}x{ny}x{nz}", nx, ny, nz,
                    (True, False, True), p, phi0, np.zeros((3, nz, ny, nx)), pstar, None,
                    int(math.ceil(10.0 * c["t_ref"])))
    return wl, c


def run(case: int, D: int, precision: str = "fp32", tmax: float = 10.0, every: float = 1.0,
        s_bulk: float = 1.0, log=None, buoyant: bool = False):
    import torch

    from paper_2206_11637_amd.sim import from_workload
    wl, c = setup(case, D, s_bulk, buoyant)
    yy = (torch.arange(wl.ny, dtype=torch.float64, device="cuda:0") + 0.5).view(1, wl.ny, 1)
    sim = from_workload(wl, precision=precision, collision="mrt")
    del wl.phi0, wl.pstar0, wl.u0
    m0 = sim.reduce()[0]
    t0 = time.time()
    ts, ys, ys_all, vol, done, finite = [], [], [], [], 0, True
    v_sphere = math.pi / 6.0 * D ** 3
    for i in range(int(round(tmax / every)) + 1):
        s = int(round(i * every * c["t_ref"]))
        if s > done:
            sim.step(s - done)
        done = s
        phi = sim.phi()
        if not bool(torch.isfinite(phi).all()):
            finite = False
            if log:
                log(f"  case {case} D={D} {precision}: non-finite phi at t*={i * every:g}")
            break
        light = 1.0 - phi
        ys_all.append(float((light * yy).sum() / light.sum()))
        gas = torch.where(phi < 0.5, light, torch.zeros_like(light))
        ys.append(float((gas * yy).sum() / gas.sum()))
        # the bubble's volume (cells with phi < 1/2) against the initial sphere
        vol.append(float((phi < 0.5).sum()) / v_sphere)
        ts.append(i * every)
        del phi, light, gas
        if log:
            log(f"  case {case} D={D} {precision}: t*={i * every:5.2f} step {s:6d} "
                f"centre {ys[-1]:9.3f} volume {vol[-1]:.3f} ({time.time() - t0:.0f} s)")
    out = dict(c, precision=precision, s_bulk=s_bulk, buoyant=buoyant, steps=done, finite=finite,
               tstar=ts,
               centre=ys, centre_all_cells=ys_all, bubble_volume=vol, seconds=time.time() - t0,
               mass_drift=float((sim.reduce()[0] - m0) / m0) if finite else None,
               re_paper=_G[f"Re_PFLBM_case{case}"])
    tv = {round(t, 6): y for t, y in zip(ts, ys)}
    if 5.0 in tv and 10.0 in tv:
        out["Re"] = D * (tv[10.0] - tv[5.0]) / (5.0 * c["t_ref"]) / c["mu_H"]
        ta = {round(t, 6): y for t, y in zip(ts, ys_all)}
        out["Re_all_cells"] = D * (ta[10.0] - ta[5.0]) / (5.0 * c["t_ref"]) / c["mu_H"]
    del sim
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--cases", type=int, nargs="+", default=[1, 2, 3, 4])
    ap.add_argument("--D", type=int, nargs="+", default=[32])
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--s-bulk", type=float, default=1.0)
    ap.add_argument("--buoyant", action="store_true",
                    help="gravity on rho - rho_H (rho_g_ref = rho_H)")
    ap.add_argument("--out", default=None)
    args = ap.parse_args()

    def log(m):
        print(m, flush=True)

    res = []
    for D in args.D:
        for case in args.cases:
            log(f"rising bubble case {case} D={D} {args.precision} s_bulk={args.s_bulk}"
                f"{' buoyant' if args.buoyant else ''}")
            r = run(case, D, args.precision, s_bulk=args.s_bulk, log=log, buoyant=args.buoyant)
            k = {32: 0, 64: 1}.get(D)
            ref = r["re_paper"][k] if k is not None else None
            log(f"  Re(t* 5-10) = {r.get('Re')} (all-cell weights {r.get('Re_all_cells')}; "
                f"paper PFLBM {ref}) mass drift {r['mass_drift']} "
                f"[{r['steps']} steps, {r['seconds']:.0f} s]")
            res.append(r)
            if args.out:
                with open(args.out, "w") as f:
                    json.dump(res, f)


if __name__ == "__main__":
    main()
