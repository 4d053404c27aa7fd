"""Benchmark of the coupled phase-field LBM step on one MI355X.

A "step" is one time step of the whole hot path over the lattice: the fused
collide-and-stream kernel of both populations (D3Q15 phase field + D3Q27
hydrodynamics, forces, stencils, bounce-back) followed by the phase-field
update.  The headline workload is the rising-bubble lattice 128 x 512 x 128
(8.4 M cells, six bounce-back faces) in FP32; the line also carries the FP64
and FP16-storage forms and the reverse-mode cost.

  python bench.py [--steps K] [--warmup W] [--no-cpu-baseline] [--no-forms]

Prints one JSON line.  Inputs are resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "coupled PFLBM MLUPS & %HBM roofline; FP32 vs FP16-store; adjoint/fwd cost"
HBM_PEAK_GBPS = 8000.0
# Algorithmic bytes per cell and step (what the method must move): read and
# write the 15 + 27 populations once each, read and write phi once.  The step
# is one kernel (k_step), so this is also that kernel's figure.
STEP_BYTES = {"fp64": 688, "fp32": 344, "fp16s": 176}
CELL_KERNEL_BYTES = STEP_BYTES
# the in-place AA scheme's collide-and-stream kernel alone: populations once
# each way and phi read once (its separate phi pass writes phi)
AA_CELL_KERNEL_BYTES = {"fp64": 680, "fp32": 340, "fp16s": 172}
# the D3Q27-phase build: 27 + 27 populations
STEP_BYTES_D3Q27 = {"fp64": 880, "fp32": 440, "fp16s": 224}
# HBM bytes per launch of k_step on the rising-bubble lattice from rocprofv3
# FETCH_SIZE / WRITE_SIZE, scaled by the factors a plain 2 GiB device copy
# gives on the same box (2.0 for FETCH_SIZE, 1.0 for WRITE_SIZE); taken for
# the current kernel (profiles/k_step_rising_bubble_128x512x128_hbm_traffic.txt)
# and to be re-measured whenever it changes
TRAFFIC = {"fp32": 3.405e9, "fp16s": 1.558e9, "fp64": 6.038e9}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def time_form(wl, precision, steps, warmup, collision="mrt", streaming="ab", phase="d3q15"):
    import torch

    from paper_2206_11637_amd.sim import from_workload
    sim = from_workload(wl, precision=precision, collision=collision, streaming=streaming,
                        phase_lattice=phase)
    sim.step(warmup)
    torch.cuda.synchronize()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    t0.record()
    cell_ms, phi_ms, total_ms = sim.profile_step(steps)
    t1.record()
    torch.cuda.synchronize()
    wall_ms = t0.elapsed_time(t1)
    r = sim.reduce()
    cells = wl.cells
    mlups = cells * steps / (wall_ms * 1e-3) / 1e6
    cell_avg = cell_ms / steps
    if phase == "d3q27":
        kb = sb = STEP_BYTES_D3Q27[precision]
    else:
        kb = (AA_CELL_KERNEL_BYTES if streaming == "aa" else CELL_KERNEL_BYTES)[precision]
        sb = STEP_BYTES[precision]
    achieved = kb * cells / (cell_avg * 1e-3) / 1e9
    out = dict(mlups=mlups, ms_per_step=wall_ms / steps, cell_kernel_ms=cell_avg,
               phi_kernel_ms=phi_ms / steps, cell_kernel_GBps=achieved,
               cell_kernel_frac=achieved / HBM_PEAK_GBPS,
               effective_GBps=mlups * sb / 1e3,
               effective_frac=mlups * sb / 1e3 / HBM_PEAK_GBPS,
               mass=r[0])
    del sim
    torch.cuda.empty_cache()
    return out


def adjoint_form(wl, precision, nsteps, sample_every, x0, depth, ckpt=None):
    """Forward (with checkpoints) and backward (with segment recompute) of the
    differentiable amplitude rollout; wall times of the second of two identical
    runs, their ratio and peak HBM."""
    import time as _t

    import torch

    from paper_2206_11637_amd.rollout import amplitude_rollout
    from paper_2206_11637_amd.sim import Simulation
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    sim = Simulation(wl.nx, wl.ny, wl.nz, wl.periodic, precision, "mrt", wl.solid, wl.params)
    dev = sim.device
    phi0 = torch.tensor(wl.phi0, dtype=torch.float64, device=dev, requires_grad=True)
    M = torch.tensor(wl.params.mobility, dtype=torch.float64, requires_grad=True)
    sg = torch.tensor(wl.params.sigma, dtype=torch.float64, requires_grad=True)
    u0 = torch.as_tensor(wl.u0, dtype=torch.float64).to(dev)
    p0 = torch.as_tensor(wl.pstar0, dtype=torch.float64).to(dev)
    stats = {}
    # two identical runs, the second timed: the first warms the code objects
    # and the allocator's pools for the checkpoint and adjoint buffers
    for _ in range(2):
        for t in (phi0, M, sg):
            t.grad = None
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        trace = amplitude_rollout(sim, phi0, M, sg, params=wl.params, nsteps=nsteps,
                                  sample_every=sample_every, depth=depth, x0=x0, u0=u0, pstar0=p0,
                                  checkpoint_every=ckpt, stats=stats)
        loss = (trace ** 2).sum()
        torch.cuda.synchronize()
        t1 = _t.perf_counter()
        loss.backward()
        torch.cuda.synchronize()
        t2 = _t.perf_counter()
        del trace, loss          # frees this run's checkpoints before the next one
    fwd, bwd = t1 - t0, t2 - t1
    cells = wl.cells
    out = dict(steps=nsteps, forward_s=fwd, backward_s=bwd, backward_over_forward=bwd / fwd,
               forward_mlups=cells * nsteps / fwd / 1e6,
               backward_mlups=cells * nsteps / bwd / 1e6,
               checkpoints=stats.get("checkpoints"), checkpoint_every=stats.get("checkpoint_every"),
               peak_hbm_GB=torch.cuda.max_memory_allocated() / 1e9,
               dL_dM=float(M.grad), dL_dsigma=float(sg.grad))
    del sim, phi0
    torch.cuda.empty_cache()
    return out


def precision_errors(wl, checkpoints=(100, 500, 1000)):
    """FP32 and FP16-storage forms against the FP64 path (which matches the FP64
    oracle to ~1e-14): max|dphi|, max|du| / max|u|, mass drift at each checkpoint."""
    import torch

    from paper_2206_11637_amd.sim import from_workload
    ref = {}
    sim = from_workload(wl, precision="fp64")
    m0 = sim.reduce()[0]
    n = 0
    for k in checkpoints:
        sim.step(k - n)
        n = k
        phi, u, _ = sim.moments()
        ref[k] = (phi, u, (sim.reduce()[0] - m0) / m0)
    del sim
    out = {}
    for prec in ("fp32", "fp16s"):
        sim = from_workload(wl, precision=prec)
        m0 = sim.reduce()[0]
        n = 0
        for k in checkpoints:
            sim.step(k - n)
            n = k
            phi, u, _ = sim.moments()
            pr, ur, dr = ref[k]
            out[f"{prec}_step{k}"] = {
                "max_abs_dphi": (phi - pr).abs().max().item(),
                "max_abs_du_over_max_u": ((u - ur).abs().max() / ur.abs().max()).item(),
                "mass_drift": (sim.reduce()[0] - m0) / m0,
                "fp64_mass_drift": dr}
            del phi, u
        del sim
        torch.cuda.empty_cache()
    del ref
    torch.cuda.empty_cache()
    return out


def long_run(wl, steps=20000, every=5000):
    """The workload's full run in FP32 against FP64: max|dphi|, mass drift and
    the rise of the light phase's centroid (sum (1 - phi) y / sum (1 - phi))."""
    import torch

    from paper_2206_11637_amd.sim import from_workload
    y = torch.arange(wl.ny, dtype=torch.float64, device="cuda").view(1, wl.ny, 1) + 0.5

    def centroid(phi):
        light = 1.0 - phi
        return float((light * y).sum() / light.sum())

    out, ref = {}, {}
    for prec in ("fp64", "fp32"):
        sim = from_workload(wl, precision=prec)
        m0 = sim.reduce()[0]
        c0 = centroid(sim.phi())
        n = 0
        for k in range(every, steps + 1, every):
            sim.step(k - n)
            n = k
            phi = sim.phi()
            rec = {"light_centroid_rise": centroid(phi) - c0,
                   "mass_drift": (sim.reduce()[0] - m0) / m0}
            if prec == "fp64":
                ref[k] = phi
            else:
                rec["max_abs_dphi_vs_fp64"] = (phi - ref[k]).abs().max().item()
            out[f"{prec}_step{k}"] = rec
            del phi
        del sim
        torch.cuda.empty_cache()
    del ref
    torch.cuda.empty_cache()
    return out


def cpu_baseline():
    """The FP64 oracle on a bounded sample of the same workload (a z-slab of
    the rising-bubble lattice with its walls), timed on the host cores."""
    import numpy as np
    import torch

    import workloads as W
    from oracle import pflbm as OP
    threads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or os.cpu_count() or 1
    threads = min(threads, 16)
    torch.set_num_threads(threads)
    wl = W.config1()
    z0, z1 = 56, 72
    grid = OP.Grid(wl.nx, wl.ny, z1 - z0, (False, False, False))
    prm = OP.OracleParams.from_workload(wl.params, "mrt")
    h, g = OP.init_equilibrium(grid, wl.phi0[z0:z1], wl.u0[:, z0:z1], wl.pstar0[z0:z1])
    h, g = OP.step(grid, prm, h, g)   # first step builds the neighbour tables
    # timed steps until about 15 s of host time (at least 4)
    nsteps = 0
    t = time.perf_counter()
    while True:
        h, g = OP.step(grid, prm, h, g)
        nsteps += 1
        dt = time.perf_counter() - t
        if nsteps >= 4 and dt >= 15.0:
            break
    cells = grid.N
    return {"value": cells * nsteps / dt / 1e6, "unit": "MLUPS", "cores": torch.get_num_threads(),
            "kind": "oracle",
            "sample": f"rising-bubble lattice cut to z in [{z0},{z1}) ({wl.nx}x{wl.ny}x{z1 - z0} "
                      f"cells, walls on all faces), FP64 MRT, {nsteps} timed steps, {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--precision", default="fp32", choices=["fp32", "fp16s", "fp64"],
                    help="storage/arithmetic form of the headline run (default fp32)")
    ap.add_argument("--adj-steps", type=int, default=4000,
                    help="steps of the Taylor-tube reverse-mode leg (sqrt(N) checkpoints)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only run a plain device copy of 2 GiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU (the multi-GPU slab "
              "decomposition is designed, not implemented); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import torch

    import workloads as W
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        n = 1 << 29   # 2 GiB of float32 read and 2 GiB written per copy
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes_read": 4 * n, "copy_probe_bytes_written": 4 * n}))
        return
    prec = args.precision
    log(f"bench: rising bubble 128x512x128 {prec} mrt")
    wl1 = W.config1()
    main_form = time_form(wl1, prec, args.steps, args.warmup)
    log(f"  {prec}: {main_form['mlups']:.0f} MLUPS")
    forms = {}

    def form(name, fn, *a):
        log(f"bench: {name}")
        try:
            forms[name] = fn(*a)
        except Exception as e:          # report, keep the headline line
            forms[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()

    if not args.no_forms:
        half = max(args.steps // 2, 10)
        form("fp64_rising_bubble_128x512x128", time_form, wl1, "fp64", half, args.warmup)
        form("rising_bubble_20k_steps_fp32_vs_fp64", long_run, wl1)
        # the in-place AA scheme: half the population memory, a separate phi pass
        form("fp32_in_place_aa_rising_bubble_128x512x128", time_form, wl1, "fp32", half, args.warmup,
             "mrt", "aa")
        # the D3Q27 phase lattice (the paper's 3D choice; a separate build)
        form("fp32_d3q27_phase_rising_bubble_128x512x128", time_form, wl1, "fp32", half,
             args.warmup, "mrt", "ab", "d3q27")
        del wl1
        wl2 = W.config2()
        form("fp32_drop_impact_384^3", time_form, wl2, "fp32", half, args.warmup)
        form("fp16s_drop_impact_384^3", time_form, wl2, "fp16s", half, args.warmup)
        form("precision_errors_drop_impact_384^3", precision_errors, wl2)
        # one GPU's share of the 384^3 drop on 8 GPUs (z-slabs of 48 planes
        # through the drop; z wraps where the slab exchange would be)
        z0 = 192 - 24
        shard = W.Workload("drop_impact_shard_384x384x48", 384, 384, 48, (True, False, True),
                           wl2.params, wl2.phi0[z0:z0 + 48].copy(), wl2.u0[:, z0:z0 + 48].copy(),
                           wl2.pstar0[z0:z0 + 48].copy(), None, wl2.steps)
        form("fp32_shard_384x384x48_of_drop_impact", time_form, shard, "fp32", half, args.warmup)
        del shard
        del wl2
        # the benchmark's M = 0.01 impact goes unstable after ~1.1k steps in
        # every precision; the 5000-step growth of the errors runs at M = 0.03
        wl2s = W.config2(mobility=0.03)
        form("precision_errors_drop_impact_384^3_M0.03", precision_errors, wl2s,
             (100, 500, 1000, 5000))
        del wl2s
        wl3 = W.config3()
        form("adjoint_capillary_64x128x64_fp32", adjoint_form, wl3, "fp32", wl3.steps, 10, 0, 64.0)
        del wl3
        wl4 = W.config4()
        form("adjoint_taylor_bubble_128x1024x128_fp16s", adjoint_form, wl4, "fp16s",
             args.adj_steps, 10, 64, 0.0)
        del wl4
    cpu = None
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline()
    line = {
        "metric": METRIC,
        "value": round(main_form["mlups"], 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(main_form["ms_per_step"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32", "fp16s": "f32 (f16 storage)", "fp64": "f64"}[prec],
        "data": "synthetic",
        "config": {"workload": "rising_bubble_128x512x128", "cells": 128 * 512 * 128,
                   "lattices": "D3Q15+D3Q27", "collision": "mrt", "storage": prec,
                   "streaming": "two buffers, pull, phase field fused into the step",
                   "boundaries": "bounce-back on all faces"},
        "roofline": {"bound": "hbm", "achieved": round(main_form["cell_kernel_GBps"], 1),
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": round(main_form["cell_kernel_frac"], 4), "traffic": TRAFFIC.get(prec),
                     "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)",
                     "algorithmic_bytes_per_launch": CELL_KERNEL_BYTES[prec] * 128 * 512 * 128,
                     "kernel": "k_step (fused pull, phase field, collide, store)",
                     "bytes_per_cell": CELL_KERNEL_BYTES[prec]},
        "step_effective": {"bytes_per_cell": STEP_BYTES[prec],
                           "GBps": round(main_form["effective_GBps"], 1),
                           "frac": round(main_form["effective_frac"], 4),
                           "phi_kernel_ms": round(main_form["phi_kernel_ms"], 4),
                           "cell_kernel_ms": round(main_form["cell_kernel_ms"], 4)},
        "cpu_baseline": cpu,
        "forms": forms,
    }
    def _round(v):
        if isinstance(v, float):
            return float(f"{v:.5g}")
        if isinstance(v, dict):
            return {k: _round(x) for k, x in v.items()}
        return v

    line["forms"] = _round(line["forms"])
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
