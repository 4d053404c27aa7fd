"""The benchmark's command line on the CPU: more than one GPU is refused with a
message and a non-zero status before anything touches a GPU; the algorithmic
byte counts it prices the roofline with follow from the population counts."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=120,
                       env=dict(os.environ, CUDA_VISIBLE_DEVICES=""))
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr) or "--gpus 1" in (r.stdout + r.stderr)


def test_algorithmic_bytes_per_cell():
    sys.path.insert(0, ROOT)
    import bench as B
    for prec, s in (("fp64", 8), ("fp32", 4), ("fp16s", 2)):
        phi = 4 if prec != "fp64" else 8
        # populations read and written once, phi read (shift reference) and written once
        assert B.STEP_BYTES[prec] == 2 * (15 + 27) * s + 2 * phi
        assert B.STEP_BYTES_D3Q27[prec] == 2 * (27 + 27) * s + 2 * phi
        assert B.AA_CELL_KERNEL_BYTES[prec] == 2 * (15 + 27) * s + phi


def test_reported_traffic_matches_the_committed_counter_summary():
    """The benchmark's roofline.traffic figures are those of the committed
    rocprofv3 summary (FETCH_SIZE x 2 + WRITE_SIZE x 1 per launch, one line per
    form); forms without committed counters report null."""
    sys.path.insert(0, ROOT)
    import bench as B
    path = os.path.join(ROOT, "profiles", "k_step_hbm_traffic.txt")
    rows = {}
    if os.path.exists(path):
        for line in open(path):
            f = line.split()
            if f and f[0].endswith(("128x512x128", "384^3")) and len(f) >= 8:
                fetch, write = (float(v.replace(",", "")) for v in f[1:3])
                rows[f[0]] = (2.0 * fetch + 1.0 * write) * 1024
    assert set(rows) == set(B.TRAFFIC)
    for name, total in rows.items():
        assert abs(B.TRAFFIC[name] - total) / total < 2e-3, (name, B.TRAFFIC[name], total)


def test_reported_instruction_counts_match_the_committed_counter_summary():
    """The issue roofline's VALU instructions per cell are those of the committed
    rocprofv3 SQ counter summary (the current-kernel block), and its ceiling
    follows from the unit counts: 256 CUs x 4 SIMDs x 2.4 GHz / 4 cycles."""
    sys.path.insert(0, ROOT)
    import bench as B
    path = os.path.join(ROOT, "profiles", "k_step_instruction_counts.txt")
    rows = {}
    cur = False
    for line in open(path):
        if line.startswith("kernel: "):
            cur = True
            continue
        f = line.split()
        if cur and len(f) > 3 and f[2] == "VALU":
            rows[f"{f[0]}_{f[1]}"] = float(f[3])
    for name, n in B.VALU_PER_CELL.items():
        assert rows[name] == n, (name, rows.get(name), n)
    assert abs(B.VALU_PEAK_G - 614.4) < 1e-9
    r = B.roofline_alu("fp16s_drop_impact_384^3", 56623104, 3.0)
    assert r["bound"] == "alu" and abs(r["achieved"] - 1312.9 * 56623104 / 64 / 3e-3 / 1e9) < 0.1
    assert B.roofline_alu("fp64_rising_bubble_128x512x128", 8388608, 1.0) is None


def test_fp32_forms_are_set_against_the_faster_step_pattern_copy():
    """attach_copy_ceiling divides each FP32 two-buffer form's achieved rate by
    the faster step-pattern copy of its own lattice, and leaves the line alone
    when the copy leg is missing or failed."""
    sys.path.insert(0, ROOT)
    import bench as B
    forms = {"hbm_copy_ceiling": {
        "soa43_fp32_step_pattern_128x512x128": {"GBps": 5600.0},
        "soa43_nt_fp32_step_pattern_128x512x128": {"GBps": 6000.0},
        "soa43_fp32_step_pattern_384x384x384": {"GBps": 5200.0},
        "soa43_nt_fp32_step_pattern_384x384x384": {"GBps": 5250.0},
        "w4_2GiB": {"GBps": 6300.0},
        "soa43_f64_fp64_step_pattern_128x512x128": {"GBps": 5500.0},
        "soa43_f64_nt_fp64_step_pattern_128x512x128": {"GBps": 6400.0}},
        "fp32_rising_bubble_128x512x128": {"roofline": {"achieved": 4500.0}},
        "fp32_drop_impact_384^3": {"roofline": {"achieved": 4462.5}}}
    head = {"roofline": {"achieved": 4800.0}}
    B.attach_copy_ceiling(forms, {"fp64_rising_bubble_128x512x128": head})
    assert head["roofline"]["vs_copy_ceiling"] == 0.75
    assert forms["fp32_rising_bubble_128x512x128"]["roofline"]["vs_copy_ceiling"] == 0.75
    assert forms["fp32_rising_bubble_128x512x128"]["roofline"]["copy_ceiling_GBps"] == 6000.0
    assert forms["fp32_drop_impact_384^3"]["roofline"]["vs_copy_ceiling"] == 0.85
    bad = {"hbm_copy_ceiling": {"error": "x"}, "fp32_drop_impact_384^3": {"roofline": {"achieved": 1.0}}}
    B.attach_copy_ceiling(bad)
    assert "vs_copy_ceiling" not in bad["fp32_drop_impact_384^3"]["roofline"]
