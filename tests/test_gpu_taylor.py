"""The paper's Taylor bubble (sec. "Taylor bubble") at tube diameter D = 64
through the library, against the Reynolds number the paper reports for its
PFLBM at that resolution (26.83).  Setup and readings in tests/taylor_study.py.

At D = 64 the run here turns non-finite between t* = 14 and 15, so the test
measures the rise velocity over t* = 10 to 14, where the rise is already
steady (Re 26.20 from the gas region's centre of mass); the paper's window
t* = 10 to 15 is met at D = 128 by the study script (Re 26.55 against the
paper's 27.12, FP32).  Where the D = 64 run fails (taylor_study.py
--diagnose, tests/results/taylor_d64_divergence.md): from t* ~ 13.5 the gas's
circulation grows (peak speed 0.09 -> 0.18, gas p* range threefold), and at
t* = 14.55 one gas cell whose phase field has undershot to -7.7e-4 (density
rho(phi) a quarter of rho_L) is accelerated by the pressure force F_p, 13x
the other forces there, to |u| = 47 within six steps; clamping phi in
rho(phi) and tau(phi) does not carry the run further."""
import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu


def test_taylor_bubble_d64_reynolds_number_matches_the_paper():
    import taylor_study as T
    say("case: Taylor bubble D=64 fp32 to t*=14")
    r = T.run(64, "fp32", tmax=14.0, every=1.0, log=say)
    assert r["finite"], "the D = 64 run diverged before t* = 14"
    y = dict(zip(r["tstar"], r["centre"]))
    re = r["Re_last"]
    assert r["Re_last_window"] == (10.0, 14.0)
    u_a = (y[12.0] - y[10.0]) / 2.0
    u_b = (y[14.0] - y[12.0]) / 2.0
    say(f"  Re(t* 10-14) = {re:.3f} (paper 26.83); rise per t* {u_a:.3f} then {u_b:.3f} cells; "
        f"mass drift {r['mass_drift']:.1e}")
    assert abs(re / T.RE_PAPER[64] - 1.0) < 0.05
    assert abs(u_b / u_a - 1.0) < 0.02                     # steady rise
    assert abs(r["mass_drift"]) < 1e-6
    vols = r["gas_volume"]
    assert max(vols) - min(vols) < 1e-6 * vols[0]
