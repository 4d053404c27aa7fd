"""Standing gravity and capillary waves on the GPU path against their closed
forms, at the paper's parameters (sec. "Standing waves": quasi-2D L x L x 1
box, x periodic, no-slip walls in y, liquid depth d = L/2, initial profile
y(x) = d + a0 cos(kx) with a0 = 0.01 L, Re = a0 omega0 L / nu = 10, density
ratio 1000, equal kinematic viscosities, heavy-phase relaxation rate 1.99,
M = 0.02, xi = 5; the amplitude at x = 0 sampled every t* = omega0 t = 0.1).

References: the linear gravity wave with viscous decay a0 exp(-2 nu k^2 t)
cos(omega0 t), omega0^2 = g k tanh(k d) (sec. gravity-wave analytical model),
and Prosperetti's small-amplitude capillary wave with omega0^2 = sigma k^3 /
(rho_H + rho_L) (sec. capillary-wave analytical model), both from
oracle/analytic.py.

Readings (where the setup leaves a choice): the gravity wave runs with
sigma = 0 (the paper calls surface tension negligible there); its heavy and
light phases start in hydrostatic balance about the flat level d, which in the
velocity-based formulation (p = p* rho c_s^2, F_p cancelling the density
gradient) is p*(y) = 3 g (d - y) in both phases; the capillary wave starts at
p* = 0.  The profile uses the integer column index, so column 0 is the crest.
The elevation is read both as the phi = 1/2 crossing at column 0 (linear
interpolation, the paper's PFLBM probe) and as the column sum of phi.

Velocity sets: the paper runs its two-dimensional waves on the D2Q9 pair.  On
these L x L x 1 lattices (z periodic, in-plane flow) the library's D3Q27-phase
build evolves exactly as the D2Q9 pair once its populations are summed over
c_z (tests/test_gpu_d2q9.py), so --phase d3q27 runs the paper's lattices;
the default D3Q15 phase lattice differs from it only in the MRT relaxation of
the phase field's zz moment.

Host-side glue only: the time stepping runs in the library; the closed forms
are the oracle's.  Run as a script for the full study:
    python tests/wave_study.py [--L 50 100 200 400] [--tmax 80] [--phase d3q27]
                               [--out FILE.json] [--table FILE.md]
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
from oracle import analytic as A  # noqa: E402
from oracle.pflbm import interface_crossing  # noqa: E402

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "standing_waves.txt")


def golden(path: str = GOLDEN) -> dict:
    """The paper's printed wave setup (tests/golden/standing_waves.txt)."""
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
RE, OMEGA_H, MOBILITY, XI = _G["Re"], _G["omega_H"], _G["mobility"], _G["xi"]
RHO_H = 1.0
RHO_L = RHO_H / _G["density_ratio"]
DT_STAR = _G["sample_every_t_star"]
assert _G["kinematic_viscosity_ratio"] == 1.0    # one tau for both phases below


def setup(kind: str, L: int):
    """Workload and constants of one standing-wave run."""
    tau = 1.0 / OMEGA_H
    nu = (tau - 0.5) / 3.0
    a0, d, k = _G["amplitude"] * L, _G["depth"] * L, 2.0 * math.pi / L
    w0 = RE * nu / (a0 * L)
    if kind == "capillary":
        sigma, g = w0 ** 2 * (RHO_H + RHO_L) / k ** 3, 0.0
    elif kind == "gravity":
        sigma, g = 0.0, w0 ** 2 / (k * math.tanh(k * d))
    else:
        raise ValueError(kind)
    p = W.Params(tau_H=tau, tau_L=tau, mobility=MOBILITY, xi=XI, sigma=sigma, rho_H=RHO_H,
                 rho_L=RHO_L, g=(0.0, -g, 0.0))
    wl = W.capillary_wave(L, L, 1, depth=d, amplitude=a0, xi=XI, params=p, noise=0.0,
                          name=f"{kind}_wave_{L}")
    if g > 0:
        y = np.arange(L, dtype=np.float64) + 0.5
        pstar = np.broadcast_to((3.0 * g * (d - y))[None, :, None], (1, L, L)).copy()
        wl = W.Workload(wl.name, wl.nx, wl.ny, wl.nz, wl.periodic, p, wl.phi0, wl.u0, pstar,
                        None, wl.steps)
    return wl, dict(kind=kind, L=L, nu=nu, a0=a0, d=d, k=k, w0=w0, sigma=sigma, g=g)


def reference(c, t):
    """Analytic amplitude a(0, t) / a0."""
    if c["kind"] == "gravity":
        return A.gravity_wave(t, 1.0, c["nu"], c["k"], c["g"], c["d"])
    return A.prosperetti_amplitude(t, 1.0, c["nu"], c["k"], c["w0"], RHO_H, RHO_L)


def run(kind: str, L: int, tmax: float, precision: str = "fp32", streaming: str = "ab",
        log=None, phase: str = "d3q15"):
    """Simulate to t* = tmax; returns times t*, a*(crossing), a*(column sum),
    the analytic a*, and summary errors."""
    import torch

    from paper_2206_11637_amd.sim import from_workload
    wl, c = setup(kind, L)
    sim = from_workload(wl, precision=precision, collision="mrt", streaming=streaming,
                        phase_lattice=phase)
    m0 = sim.reduce()[0]
    every = DT_STAR / c["w0"]
    nsamp = int(round(tmax / DT_STAR))
    steps = [int(round(i * every)) for i in range(nsamp + 1)]
    ac, asum, done, t0 = [], [], 0, time.time()
    for i, s in enumerate(steps):
        sim.step(s - done)
        done = s
        col = sim.phi()[0, :, 0].double().cpu().numpy()
        ac.append((interface_crossing(col, c["d"]) - c["d"]) / c["a0"])
        asum.append((col.sum() - c["d"]) / c["a0"])
        if log and (i % 100 == 0 or i == nsamp):
            log(f"  {kind} L={L}: t*={i * DT_STAR:5.1f} step {s} a*={ac[-1]:+.4f} "
                f"({time.time() - t0:.0f} s)")
    mass_drift = float((sim.reduce()[0] - m0) / m0)
    torch.cuda.synchronize()
    ts = np.array(steps, dtype=np.float64)
    tstar = ts * c["w0"]
    ref = reference(c, ts)
    ac, asum = np.array(ac), np.array(asum)
    return dict(c, tstar=tstar.tolist(), a_cross=ac.tolist(), a_sum=asum.tolist(),
                a_ref=ref.tolist(), steps=steps[-1], seconds=time.time() - t0,
                mass_drift=mass_drift, precision=precision, streaming=streaming, phase=phase,
                **summary(tstar, ac, ref))


def _first_min(t, a):
    i = int(np.argmin(a[: max(3, int(len(a) * 0.75))]))
    if 0 < i < len(a) - 1:          # parabolic refinement
        y0, y1, y2 = a[i - 1], a[i], a[i + 1]
        den = y0 - 2 * y1 + y2
        if den != 0:
            dt = t[1] - t[0]
            off = 0.5 * (y0 - y2) / den
            return t[i] + off * dt, y1 - 0.25 * (y0 - y2) * off
    return t[i], a[i]


def summary(tstar, a, ref):
    """Phase and damping errors of a simulated trace against the reference:
    first-minimum time and depth, RMS difference, and the envelope ratio over
    the last quarter of the run (max |a| / max |a_ref| there)."""
    tm, am = _first_min(tstar, a)
    tr, ar = _first_min(tstar, ref)
    q = len(a) * 3 // 4
    env = float(np.max(np.abs(a[q:])) / max(np.max(np.abs(ref[q:])), 1e-300))
    return dict(t_min=float(tm), t_min_ref=float(tr), a_min=float(am), a_min_ref=float(ar),
                rms=float(np.sqrt(np.mean((a - ref) ** 2))), envelope_ratio_last_quarter=env)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--L", type=int, nargs="+", default=[int(v) for v in _G["L"]])
    ap.add_argument("--tmax", type=float, default=_G["t_star_max"])
    ap.add_argument("--tmax-large", type=float, default=None,
                    help="t* limit for L >= 400 (default: --tmax)")
    ap.add_argument("--kinds", nargs="+", default=["gravity", "capillary"])
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--phase", default="d3q15", choices=["d3q15", "d3q27"],
                    help="phase lattice build (d3q27 on these planar lattices = the D2Q9 pair)")
    ap.add_argument("--out", default=None, help="JSON with the full traces")
    ap.add_argument("--table", default=None, help="Markdown table of the summaries")
    args = ap.parse_args()

    def log(m):
        print(m, flush=True)

    res = []
    for kind in args.kinds:
        for L in args.L:
            tmax = args.tmax_large if (args.tmax_large and L >= 400) else args.tmax
            log(f"{kind} wave L={L} to t*={tmax}")
            r = run(kind, L, tmax, args.precision, log=log, phase=args.phase)
            log(f"  first minimum t*={r['t_min']:.3f} (ref {r['t_min_ref']:.3f}) "
                f"a*={r['a_min']:.4f} (ref {r['a_min_ref']:.4f}) rms={r['rms']:.4f} "
                f"envelope(last quarter)={r['envelope_ratio_last_quarter']:.3f} "
                f"mass drift {r['mass_drift']:.2e} "
                f"[{r['steps']} steps, {r['seconds']:.0f} s]")
            res.append(r)
            if args.out:
                with open(args.out, "w") as f:
                    json.dump(res, f)
            if args.table:
                write_table(res, args.table, " ".join(sys.argv[1:]))


def write_table(res, path, argv):
    """Markdown table of the runs' summaries (the numbers the study reports)."""
    lat = {"d3q15": "D3Q15 + D3Q27", "d3q27": "D2Q9 pair (D3Q27 build, planar)"}
    rows = ["| wave | L | lattices | precision | t* run | steps | first min t* (ref) | "
            "first min a* (ref) | rms a* | envelope, last quarter | mass drift | GPU s |",
            "|---|---|---|---|---|---|---|---|---|---|---|---|"]
    for r in res:
        rows.append(f"| {r['kind']} | {r['L']} | {lat[r['phase']]} | {r['precision']} | "
                    f"{r['tstar'][-1]:.0f} | {r['steps']} | {r['t_min']:.3f} ({r['t_min_ref']:.3f}) | "
                    f"{r['a_min']:.3f} ({r['a_min_ref']:.3f}) | {r['rms']:.3f} | "
                    f"{r['envelope_ratio_last_quarter']:.2f} | {r['mass_drift']:.0e} | "
                    f"{r['seconds']:.0f} |")
    head = ("# Standing waves on the GPU against their closed forms\n\n"
            "Written by `python tests/wave_study.py " + argv + "` (elevation at x = 0 from the\n"
            "phi = 1/2 crossing, a* = a / a0, t* = omega0 t; references: gravity wave with viscous\n"
            "decay, Prosperetti's capillary wave; envelope = max|a*| over the last quarter of the\n"
            "run relative to the reference's).\n\n")
    with open(path, "w") as f:
        f.write(head + "\n".join(rows) + "\n")


if __name__ == "__main__":
    main()
