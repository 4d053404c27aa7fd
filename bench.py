"""Benchmark of the coupled phase-field LBM step on one MI355X.

A "step" is one time step of the whole hot path over the lattice: the fused
collide-and-stream kernel of both populations (D3Q15 phase field + D3Q27
hydrodynamics, forces, stencils, bounce-back) followed by the phase-field
update.  The headline workload is the rising-bubble lattice 128 x 512 x 128
(8.4 M cells, six bounce-back faces) in FP64, the arithmetic of the paper's
runs; the line also carries the FP32 and FP16-storage forms (each with its
own roofline block), a hand-written streaming-copy ceiling, one GPU's z-slab
of the 384^3 drop with the pack of its faces for the slab exchange, the
reverse-mode cost and the gradient error of the reduced-precision forms
against FP64.

  python bench.py [--steps K] [--warmup W] [--runs R] [--no-cpu-baseline]
                  [--no-forms] [--only NAME,NAME] [--precision P]

Timing: W untimed warm-up steps, then R runs of K steps each (HIP events on
the library's stream, synchronised on both sides); the reported figures are
those of the median run.  Kernel durations come from a second set of R runs
with an event between consecutive launches.  Prints one JSON line.  Inputs
are resident in HBM before the timed region.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import statistics
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
# HBM bytes per launch of the step kernel from rocprofv3 FETCH_SIZE /
# WRITE_SIZE, scaled by the factors a plain 2 GiB device copy gives on the
# same box (2.0 for FETCH_SIZE, 1.0 for WRITE_SIZE), keyed by form; taken for
# the current kernel (profiles/k_step_hbm_traffic.txt) and re-measured
# whenever it changes.  Forms without an entry report null.
TRAFFIC = {"fp64_rising_bubble_128x512x128": 6.0920e9,
           "fp32_rising_bubble_128x512x128": 3.2388e9,
           "fp16s_rising_bubble_128x512x128": 1.5514e9,
           "fp32_d3q27_phase_rising_bubble_128x512x128": 4.2801e9,
           "fp32_drop_impact_384^3": 2.3102e10,
           "fp16s_drop_impact_384^3": 1.1193e10,
           "fp32_in_place_aa_rising_bubble_128x512x128": 3.0657e9}
TRAFFIC_UNIT = "HBM bytes per launch (rocprofv3 FETCH_SIZE x2.0 + WRITE_SIZE x1.0)"
# Vector ALU instructions per wave and z plane of the step kernel (= per cell
# for one lane), rocprofv3 SQ_INSTS_VALU over SQ_WAVES and the planes each wave
# marches (profiles/k_step_instruction_counts.txt), for the FP32-arithmetic
# forms.  Their issue ceiling: a wave64 FP32 VALU instruction occupies a SIMD
# for 4 cycles (16 lanes), so 256 CUs x 4 SIMDs x 2.4 GHz / 4 = 614.4 G wave
# instructions per second (= 157.3 TFLOP/s FP32 vector / 64 lanes / 2 flops
# per FMA / 2 for the packed forms, which these kernels do not use).
VALU_PER_CELL = {"fp32_rising_bubble_128x512x128": 1265.9,
                 "fp16s_rising_bubble_128x512x128": 1353.9,
                 "fp16s_drop_impact_384^3": 1312.9}
VALU_PEAK_G = 256 * 4 * 2.4 / 4
DTYPE = {"fp32": "f32", "fp16s": "f32 (f16 storage)", "fp64": "f64"}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def roofline(name, bytes_per_cell, cells, kernel_ms, kernel):
    """Roofline block of one kernel: algorithmic bytes per launch over its
    average launch duration against the 8 TB/s datasheet peak, with the
    counter-measured traffic where the committed counters cover this form."""
    alg = bytes_per_cell * cells
    achieved = alg / (kernel_ms * 1e-3) / 1e9
    tr = TRAFFIC.get(name)
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBPS, 4), "traffic": tr, "traffic_unit": TRAFFIC_UNIT,
            "traffic_over_algorithmic": None if tr is None else round(tr / alg, 4),
            "algorithmic_bytes_per_launch": alg, "bytes_per_cell": bytes_per_cell,
            "kernel": kernel, "kernel_ms": round(kernel_ms, 5)}


def roofline_alu(name, cells, kernel_ms):
    """Issue roofline of the step kernel for the forms whose instruction count
    is committed: VALU wave instructions per launch over the kernel's average
    duration against the FP32 VALU issue ceiling."""
    n = VALU_PER_CELL.get(name)
    if n is None:
        return None
    per_launch = n * cells / 64.0
    achieved = per_launch / (kernel_ms * 1e-3) / 1e9
    return {"bound": "alu", "achieved": round(achieved, 1), "peak": VALU_PEAK_G,
            "unit": "G VALU wave-instructions/s", "frac": round(achieved / VALU_PEAK_G, 4),
            "valu_per_cell": n, "valu_per_launch": per_launch, "kernel_ms": round(kernel_ms, 5)}


def time_form(name, wl, precision, steps, warmup, runs, collision="mrt", streaming="ab",
              phase="d3q15"):
    """Median of `runs` timed runs of `steps` steps (plain stepping), and the
    kernels' average durations from as many profiled runs."""
    import torch

    from paper_2206_11637_amd.sim import from_workload
    sim = from_workload(wl, precision=precision, collision=collision, streaming=streaming,
                        phase_lattice=phase)
    sim.step(warmup)
    torch.cuda.synchronize()
    walls, cells_ms, phis_ms = [], [], []
    for _ in range(runs):
        t0 = torch.cuda.Event(enable_timing=True)
        t1 = torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        t0.record(sim.stream)
        sim.step(steps)
        t1.record(sim.stream)
        torch.cuda.synchronize()
        walls.append(t0.elapsed_time(t1))
    for _ in range(runs):
        cell_ms, phi_ms, _ = sim.profile_step(steps)
        cells_ms.append(cell_ms / steps)
        phis_ms.append(phi_ms / steps)
    r = sim.reduce()
    wall = statistics.median(walls)
    cell_avg = statistics.median(cells_ms)
    phi_avg = statistics.median(phis_ms)
    cells = wl.cells
    mlups = cells * steps / (wall * 1e-3) / 1e6
    if phase == "d3q27":
        kb = sb = STEP_BYTES_D3Q27[precision]
        kernel = "k_step (D3Q27 phase lattice build)"
    elif streaming == "aa":
        kb, sb = AA_CELL_KERNEL_BYTES[precision], STEP_BYTES[precision]
        kernel = "k_cell_aa (in-place collide and stream; + k_light phi gather)"
    else:
        kb = sb = STEP_BYTES[precision]
        kernel = "k_step (fused pull, phase field, collide, store)"
    out = dict(mlups=round(mlups, 1), ms_per_step=round(wall / steps, 5),
               runs=runs, steps_per_run=steps,
               ms_per_step_range=[round(min(walls) / steps, 5), round(max(walls) / steps, 5)],
               phi_kernel_ms=round(phi_avg, 5),
               effective_frac=round(mlups * sb / 1e3 / HBM_PEAK_GBPS, 4),
               roofline=roofline(name, kb, cells, cell_avg, kernel),
               roofline_alu=roofline_alu(name, cells, cell_avg),
               mass=float(r[0]))
    del sim
    torch.cuda.empty_cache()
    return out


def halo_pack(wl, steps, warmup, runs, launches=100):
    """The z-slab shard's step (FP32) and the pack of its two faces for the
    slab exchange (pflbm_pack_faces: the populations with c_z = -1 at plane 0
    and c_z = +1 at plane nz - 1 into one staging buffer).  The packs are
    queued behind a run of steps so that they execute back to back; their
    HIP-event time over `launches` packs, median of `runs`."""
    import ctypes as C

    import torch

    from paper_2206_11637_amd.sim import from_workload
    sim = from_workload(wl, precision="fp32")
    sim.step(warmup)
    buf = sim.pack_faces()
    nbytes = buf.numel() * buf.element_size()
    need = C.c_size_t()
    args = (sim.ctx, C.c_void_p(buf.data_ptr()), C.c_size_t(nbytes), C.byref(need))
    steps_ms, pack_ms = [], []
    for _ in range(runs):
        e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
        torch.cuda.synchronize()
        e[0].record(sim.stream)
        sim.step(steps)
        e[1].record(sim.stream)
        for _ in range(launches):
            st = sim.lib.pflbm_pack_faces(*args)
            if st:
                raise RuntimeError(f"pflbm_pack_faces failed with status {st}")
        e[2].record(sim.stream)
        torch.cuda.synchronize()
        steps_ms.append(e[0].elapsed_time(e[1]) / steps)
        pack_ms.append(e[1].elapsed_time(e[2]) / launches)
    step = statistics.median(steps_ms)
    pack = statistics.median(pack_ms)
    gbps = 2 * nbytes / (pack * 1e-3) / 1e9
    out = dict(ms_per_step=round(step, 5), mlups=round(wl.cells / (step * 1e-3) / 1e6, 1),
               pack_ms=round(pack, 6), pack_rows_per_face=int(buf.shape[1]),
               face_cells=int(buf.shape[2] * buf.shape[3]), pack_bytes_read=nbytes,
               pack_bytes_written=nbytes, pack_GBps=round(gbps, 1),
               pack_frac_of_8TBps=round(gbps / HBM_PEAK_GBPS, 4),
               pack_over_step=round(pack / step, 5), launches=launches, runs=runs)
    del sim, buf
    torch.cuda.empty_cache()
    return out


def attach_copy_ceiling(forms, extra=None):
    """Each two-buffer FP32 and FP64 form's achieved bandwidth over the faster
    of the two step-pattern copies of its element size (cached or
    non-temporal loads) measured on the same lattice in the same run:
    roofline.vs_copy_ceiling.  extra: more forms by name (the headline)."""
    cc = forms.get("hbm_copy_ceiling")
    if not isinstance(cc, dict) or "error" in cc:
        return
    every = dict(forms)
    every.update(extra or {})
    targets = {"fp32_rising_bubble_128x512x128": "fp32_step_pattern_128x512x128",
               "fp32_drop_impact_384^3": "fp32_step_pattern_384x384x384",
               "fp64_rising_bubble_128x512x128": "fp64_step_pattern_128x512x128"}
    for name, pattern in targets.items():
        f = every.get(name)
        rates = [v["GBps"] for k, v in cc.items() if k.endswith(pattern)]
        if not f or "roofline" not in f or not rates:
            continue
        ceiling = max(rates)
        f["roofline"]["copy_ceiling_GBps"] = ceiling
        f["roofline"]["vs_copy_ceiling"] = round(f["roofline"]["achieved"] / ceiling, 4)


def copy_ceiling(steps, runs):
    """Hand-written streaming kernels with no arithmetic (pflbm_hbm_copy):
    2 GiB plain copies with 4- and 16-byte accesses, and the FP32 step's own
    access pattern (43 rows of N floats read and written, cached or
    non-temporal loads, N = the rising-bubble lattice and the 384^3 drop) and
    the FP64 step's (43 rows of N doubles, the rising-bubble lattice).  GB/s
    counts bytes read plus bytes written."""
    import ctypes as C

    import torch

    from paper_2206_11637_amd import _lib
    lib = _lib.load()
    stream = torch.cuda.current_stream()
    out = {}
    cases = [("w4_2GiB", "w4", 1 << 31), ("w16_2GiB", "w16", 1 << 31),
             ("w16_cached_2GiB", "w16_cached", 1 << 31),
             ("soa43_fp32_step_pattern_128x512x128", "soa43", 43 * 4 * 128 * 512 * 128),
             ("soa43_nt_fp32_step_pattern_128x512x128", "soa43_nt", 43 * 4 * 128 * 512 * 128),
             ("soa43_fp32_step_pattern_384x384x384", "soa43", 43 * 4 * 384 ** 3),
             ("soa43_nt_fp32_step_pattern_384x384x384", "soa43_nt", 43 * 4 * 384 ** 3),
             ("soa43_f64_fp64_step_pattern_128x512x128", "soa43_f64", 43 * 8 * 128 * 512 * 128),
             ("soa43_f64_nt_fp64_step_pattern_128x512x128", "soa43_f64_nt", 43 * 8 * 128 * 512 * 128)]
    for name, form, nbytes in cases:
        a = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)

        def launch():
            _lib.check(lib.pflbm_hbm_copy(C.c_void_p(a.data_ptr()), C.c_void_p(b.data_ptr()),
                                          nbytes, _lib.COPY_FORMS[form],
                                          C.c_void_p(stream.cuda_stream)), None, "pflbm_hbm_copy")
        for _ in range(3):
            launch()
        ts = []
        for _ in range(runs):
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(steps):
                launch()
            e1.record(stream)
            torch.cuda.synchronize()
            ts.append(e0.elapsed_time(e1) / steps)
        ms = statistics.median(ts)
        gbps = 2 * nbytes / (ms * 1e-3) / 1e9
        assert torch.equal(a[:1024], b[:1024]) and torch.equal(a[-1024:], b[-1024:])
        out[name] = {"ms": round(ms, 5), "GBps": round(gbps, 1), "frac": round(gbps / HBM_PEAK_GBPS, 4),
                     "bytes_moved": 2 * nbytes}
        del a, b
        torch.cuda.empty_cache()
    return out


def adjoint_run(wl, precision, nsteps, sample_every, x0, depth, ckpt=None, timed=True):
    """Forward (with checkpoints) and backward (with segment recompute) of the
    differentiable amplitude rollout, loss = sum of squared samples; wall
    times of the second of two identical runs (timed) and the gradients."""
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
    xi = torch.tensor(wl.params.xi, dtype=torch.float64, requires_grad=True)
    u0 = torch.as_tensor(wl.u0, dtype=torch.float64).to(dev)
    p0 = torch.as_tensor(wl.pstar0, dtype=torch.float64).to(dev)
    stats = {}
    # two identical runs when timed, the second timed: the first warms the code
    # objects and the allocator's pools for the checkpoint and adjoint buffers
    for _ in range(2 if timed else 1):
        for t in (phi0, M, sg, xi):
            t.grad = None
        torch.cuda.synchronize()
        t0 = _t.perf_counter()
        trace = amplitude_rollout(sim, phi0, M, sg, xi=xi, params=wl.params, nsteps=nsteps,
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
               peak_hbm_GB=torch.cuda.max_memory_allocated() / 1e9)
    grads = dict(dM=float(M.grad), dsigma=float(sg.grad), dxi=float(xi.grad),
                 dphi0=phi0.grad.detach().clone())
    del sim, phi0
    torch.cuda.empty_cache()
    return out, grads


def grad_errors(g, ref):
    """Relative errors of a reduced-precision form's gradients against FP64
    (parameters: |d - d_64| / |d_64|; the field dL/dphi0: max norm over max norm)."""
    e = {k: abs(g[k] - ref[k]) / abs(ref[k]) for k in ("dM", "dsigma", "dxi")}
    d = (g["dphi0"] - ref["dphi0"]).abs().max() / ref["dphi0"].abs().max()
    e["dphi0_normwise"] = float(d)
    return e


def column_level(wl, x0):
    """Initial column sum of phi at x = x0, averaged over z (the probe's value at
    t = 0): as the probe's depth it makes the samples measure the change."""
    import numpy as np
    return float(np.asarray(wl.phi0)[:, :, x0].sum(axis=1).mean())


def adjoint_form(wl, precision, nsteps, sample_every, x0, depth, ref_wl=None, ckpt=None,
                 conditioning=False):
    """Reverse-mode cost of a form, plus its gradients' relative error against
    the FP64 form of the same rollout (on ref_wl, probed on its axis column
    x = nx/2 with its own initial level as depth, when the full lattice's FP64
    checkpoints would not fit in HBM)."""
    out, grads = adjoint_run(wl, precision, nsteps, sample_every, x0, depth, ckpt)
    out.update({k: v for k, v in grads.items() if k != "dphi0"})
    rw = ref_wl or wl
    if ref_wl is not None:
        x0 = rw.nx // 2
        depth = column_level(rw, x0)
        _, grads = adjoint_run(rw, precision, nsteps, sample_every, x0, depth, ckpt, timed=False)
    _, ref = adjoint_run(rw, "fp64", nsteps, sample_every, x0, depth, ckpt, timed=False)
    out["grad_rel_err_vs_fp64"] = grad_errors(grads, ref)
    out["grad_rel_err_lattice"] = rw.name
    if conditioning:
        # the FP64 gradients' own change when phi0 moves by 1e-7 relative (an
        # FP32 rounding): where it is of the order of the error above, that
        # gradient is ill-conditioned on this rollout, not lost by the form
        import dataclasses

        import numpy as np

        import workloads as W
        rng = np.random.default_rng(W.SEED + 2)
        fluid = np.ones(rw.phi0.shape, bool) if rw.solid is None else ~rw.solid
        pert = dataclasses.replace(rw, phi0=np.where(
            fluid, rw.phi0 * (1 + 1e-7 * rng.standard_normal(rw.phi0.shape)), 0.0))
        _, g_p = adjoint_run(pert, "fp64", nsteps, sample_every, x0, depth, ckpt, timed=False)
        out["fp64_grad_change_under_1e-7_phi0_perturbation"] = grad_errors(g_p, ref)
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


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _oracle_steps(wl, z0, z1, threads, min_s, min_steps):
    import torch

    from oracle import pflbm as OP
    torch.set_num_threads(threads)
    grid = OP.Grid(wl.nx, wl.ny, z1 - z0, (False, False, False))
    prm = OP.OracleParams.from_workload(wl.params, "mrt")
    h, g = OP.init_equilibrium(grid, wl.phi0[z0:z1], wl.u0[:, z0:z1], wl.pstar0[z0:z1])
    h, g = OP.step(grid, prm, h, g)   # first step builds the neighbour tables
    nsteps = 0
    t = time.perf_counter()
    while True:
        h, g = OP.step(grid, prm, h, g)
        nsteps += 1
        dt = time.perf_counter() - t
        if nsteps >= min_steps and dt >= min_s:
            break
    return grid.N * nsteps / dt / 1e6, nsteps, dt, torch.get_num_threads()


def cpu_baseline():
    """The FP64 oracle as it stands, timed on the host: the whole rising-bubble
    lattice at reduced steps on every thread the process is given (the
    benchmark workload itself), and a z-slab of it on one thread."""
    import torch

    import workloads as W
    wl = W.config1()
    threads = torch.get_num_threads()   # follows OMP_NUM_THREADS (the host share of one GPU)
    v, n, dt, used = _oracle_steps(wl, 0, wl.nz, threads, 5.0, 2)
    v1, n1, dt1, _ = _oracle_steps(wl, 60, 68, 1, 8.0, 1)
    torch.set_num_threads(threads)
    return {"value": v, "unit": "MLUPS", "cores": used, "kind": "oracle",
            "sample": f"the whole rising-bubble lattice {wl.nx}x{wl.ny}x{wl.nz} (six walls), FP64 MRT, "
                      f"{n} timed steps after one untimed, {dt:.1f} s on {used} threads",
            "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "single_thread": {"value": v1, "unit": "MLUPS", "cores": 1,
                              "sample": f"z-slab {wl.nx}x{wl.ny}x8 of the same lattice (walls on all "
                                        f"faces), {n1} timed steps, {dt1:.1f} s"}}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--runs", type=int, default=5, help="timed runs; the median run is reported")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true")
    ap.add_argument("--only", default="",
                    help="comma-separated form names (of the slow legs only the adjoint_ ones)")
    ap.add_argument("--precision", default="fp64", choices=["fp32", "fp16s", "fp64"],
                    help="storage/arithmetic form of the headline run (default fp64, the paper's)")
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
    only = [s for s in args.only.split(",") if s]
    prec = args.precision
    K, Wm, R = args.steps, args.warmup, args.runs
    wl1 = W.config1()
    head_name = f"{prec}_rising_bubble_128x512x128"
    main_form = None
    if not only or head_name in only:
        log(f"bench: {head_name}")
        main_form = time_form(head_name, wl1, prec, K, Wm, R)
        log(f"  {main_form['mlups']:.0f} MLUPS")
    forms = {}

    def form(name, fn, *a, **kw):
        if only and name not in only:
            return
        log(f"bench: {name}")
        t = time.perf_counter()
        try:
            forms[name] = fn(*a, **kw)
        except Exception as e:          # report, keep the headline line
            forms[name] = {"error": f"{type(e).__name__}: {e}"}
            torch.cuda.empty_cache()
        log(f"  done in {time.perf_counter() - t:.1f} s")

    slow = not only
    if not args.no_forms:
        form("hbm_copy_ceiling", copy_ceiling, max(K // 5, 10), R)
        for p in ("fp64", "fp32", "fp16s"):
            if p != prec:
                n = f"{p}_rising_bubble_128x512x128"
                form(n, time_form, n, wl1, p, K, Wm, R)
        if slow:
            form("rising_bubble_20k_steps_fp32_vs_fp64", long_run, wl1)
        # the in-place AA scheme: half the population memory, a separate phi pass
        n = "fp32_in_place_aa_rising_bubble_128x512x128"
        form(n, time_form, n, wl1, "fp32", K, Wm, R, "mrt", "aa")
        # the D3Q27 phase lattice (the paper's 3D choice; a separate build)
        n = "fp32_d3q27_phase_rising_bubble_128x512x128"
        form(n, time_form, n, wl1, "fp32", K, Wm, R, "mrt", "ab", "d3q27")
        del wl1
        half = max(K // 4, 10)
        wl2 = W.config2()
        for p in ("fp32", "fp16s"):
            n = f"{p}_drop_impact_384^3"
            form(n, time_form, n, wl2, p, half, Wm, R)
        if slow:
            form("precision_errors_drop_impact_384^3", precision_errors, wl2)
        # one GPU's share of the 384^3 drop on 8 GPUs (z-slabs of 48 planes
        # through the drop; z wraps where the slab exchange would be)
        z0 = 192 - 24
        shard = W.Workload("drop_impact_shard_384x384x48", 384, 384, 48, (True, False, True),
                           wl2.params, wl2.phi0[z0:z0 + 48].copy(), wl2.u0[:, z0:z0 + 48].copy(),
                           wl2.pstar0[z0:z0 + 48].copy(), None, wl2.steps)
        n = "fp32_shard_384x384x48_of_drop_impact"
        # as many steps as the full drop: the cut drop, wrapped in z, turns
        # non-finite after ~1k steps at M = 0.01
        form(n, time_form, n, shard, "fp32", half, Wm, R)
        # the same shard with the pack of its two faces for the slab exchange
        n = "fp32_halo_pack_of_shard_384x384x48"
        form(n, halo_pack, shard, half, Wm, R)
        del shard
        del wl2
        if slow:
            # the benchmark's M = 0.01 impact goes unstable after ~1.1k steps in
            # every precision; the 5000-step growth of the errors runs at M = 0.03
            wl2s = W.config2(mobility=0.03)
            form("precision_errors_drop_impact_384^3_M0.03", precision_errors, wl2s,
                 (100, 500, 1000, 5000))
            del wl2s
        # the reverse-mode legs also run when --only names them
        if slow or any(n.startswith("adjoint_") for n in only):
            wl3 = W.config3()
            form("adjoint_capillary_64x128x64_fp32", adjoint_form, wl3, "fp32", wl3.steps, 10, 0,
                 64.0)
            del wl3
            wl4 = W.config4()
            # the FP64 reference of the gradients runs on the tube at half the
            # resolution (64x512x64), where its checkpoints fit in HBM
            form("adjoint_taylor_bubble_128x1024x128_fp16s", adjoint_form, wl4, "fp16s",
                 args.adj_steps, 10, 64, column_level(wl4, 64), W.config4(scale=2),
                 conditioning=True)
            del wl4
    attach_copy_ceiling(forms, {head_name: main_form} if main_form else None)
    cpu = None
    if not args.no_cpu_baseline and not only:
        log("bench: cpu baseline (oracle)")
        cpu = cpu_baseline()

    def _round(v):
        if isinstance(v, float):
            return float(f"{v:.5g}")
        if isinstance(v, dict):
            return {k: _round(x) for k, x in v.items()}
        return v

    if main_form is None:
        print(json.dumps({"forms": _round(forms)}), flush=True)
        return
    line = {
        "metric": METRIC,
        "value": main_form["mlups"],
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": K,
        "warmup": Wm,
        "ms_per_step": main_form["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": DTYPE[prec],
        "data": "synthetic",
        "config": {"workload": "rising_bubble_128x512x128", "cells": 128 * 512 * 128,
                   "lattices": "D3Q15+D3Q27", "collision": "mrt", "storage": prec,
                   "streaming": "two buffers, pull, phase field fused into the step",
                   "boundaries": "bounce-back on all faces",
                   "timing": f"median of {R} runs of {K} steps"},
        "roofline": main_form["roofline"],
        "step_effective_frac": main_form["effective_frac"],
        "ms_per_step_range": main_form["ms_per_step_range"],
        "cpu_baseline": cpu,
        "forms": _round(forms),
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
