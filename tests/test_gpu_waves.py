"""Standing gravity and capillary waves through the library against their
closed forms (paper sec. "Standing waves"; setup and readings in
tests/wave_study.py), short version: L = 50 and 100 up to t* = 20 on the
default build, and L = 100 and 200 up to t* = 40 on the paper's D2Q9 pair
(planar lattices of the D3Q27-phase build).

What is pinned: the wave converges towards the analytic amplitude as L grows
(RMS error of a*(t*) and first-minimum time), the phase mass is conserved to
rounding over ~10^5 FP32 steps (shifted storage), and FP32 and FP64 traces
agree.  The paper reports that the PFLBM underestimates the damping of the
gravity wave; that is measured, not asserted, here (the full study in
tests/wave_study.py covers L up to 400 and t* = 80)."""
import numpy as np
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["gravity", "capillary"])
def test_standing_wave_converges_towards_the_closed_form(kind):
    import wave_study as S
    runs = {}
    for L in (50, 100):
        r = S.run(kind, L, 20.0, "fp32")
        runs[L] = r
        say(f"  {kind} L={L}: rms {r['rms']:.4f} first minimum t* {r['t_min']:.3f} "
            f"(ref {r['t_min_ref']:.3f}) a* {r['a_min']:.4f} (ref {r['a_min_ref']:.4f}) "
            f"mass drift {r['mass_drift']:.1e} [{r['steps']} steps]")
        assert abs(r["mass_drift"]) < 1e-7
    e50 = abs(runs[50]["t_min"] / runs[50]["t_min_ref"] - 1)
    e100 = abs(runs[100]["t_min"] / runs[100]["t_min_ref"] - 1)
    assert runs[100]["rms"] < runs[50]["rms"]
    assert e100 < e50 and e100 < 0.08
    assert abs(runs[100]["a_min"] / runs[100]["a_min_ref"] - 1) < 0.05
    # the crossing and the column-sum probes see the same wave
    a = np.array(runs[100]["a_cross"])
    b = np.array(runs[100]["a_sum"])
    assert np.abs(a - b).max() < 0.05


def test_fp32_and_fp64_waves_agree():
    import wave_study as S
    r32 = S.run("gravity", 50, 20.0, "fp32")
    r64 = S.run("gravity", 50, 20.0, "fp64")
    d = np.abs(np.array(r32["a_cross"]) - np.array(r64["a_cross"])).max()
    say(f"  gravity L=50 to t*=20: max |a*(fp32) - a*(fp64)| = {d:.2e}; "
        f"mass drift fp32 {r32['mass_drift']:.1e} fp64 {r64['mass_drift']:.1e}")
    assert d < 2e-3


@pytest.mark.parametrize("kind", ["gravity", "capillary"])
def test_d2q9_pair_converges_from_l100_to_l200(kind):
    """The paper's D2Q9 pair (planar lattices of the D3Q27-phase build) from
    L = 100 to L = 200 over t* = 40: the first minimum moves towards the
    closed form's and the rms error of a*(t*) falls (the full study to t* = 80
    at L = 50 to 400: tests/results/standing_waves_d2q9.md, first-minimum time
    errors 5.3 % -> 4.7 % (gravity) and 3.4 % -> 2.6 % (capillary) from L = 100
    to 200); phase mass to rounding over ~2 x 10^6 FP32 steps."""
    import wave_study as S
    runs = {}
    for L in (100, 200):
        r = S.run(kind, L, 40.0, "fp32", phase="d3q27")
        runs[L] = r
        say(f"  {kind} D2Q9 L={L}: rms {r['rms']:.4f} first minimum t* {r['t_min']:.3f} "
            f"(ref {r['t_min_ref']:.3f}) a* {r['a_min']:.4f} (ref {r['a_min_ref']:.4f}) "
            f"mass drift {r['mass_drift']:.1e} [{r['steps']} steps]")
        assert abs(r["mass_drift"]) < 1e-7
    e100 = abs(runs[100]["t_min"] / runs[100]["t_min_ref"] - 1)
    e200 = abs(runs[200]["t_min"] / runs[200]["t_min_ref"] - 1)
    assert e200 < e100 and e200 < 0.06
    assert runs[200]["rms"] < runs[100]["rms"]
    assert abs(runs[200]["a_min"] / runs[200]["a_min_ref"] - 1) < 0.05
