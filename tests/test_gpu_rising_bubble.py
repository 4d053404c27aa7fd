"""The paper's free rising bubble, case 3, at D = 16 (128 x 320 x 128, to
t* = 10, FP32; setup and readings in tests/rising_bubble_study.py): with
gravity on rho - rho_H (rho_g_ref = rho_H) the bubble keeps at least 90 % of
its volume (cells with phi < 1/2), clearly more than with gravity on rho,
where the gas pressure follows the liquid's hydrostatic pressure down as the
bubble rises; the phase mass holds in both, and both rise."""
import os
import sys

import pytest

from gpu_util import say

pytestmark = pytest.mark.gpu

sys.path.insert(0, os.path.dirname(os.path.abspath(__file__)))


def test_buoyant_body_force_keeps_the_free_bubble_whole():
    import rising_bubble_study as RB
    out = {}
    for buoyant in (False, True):
        say(f"case: rising bubble case 3 D=16 fp32 buoyant={buoyant}")
        r = RB.run(3, 16, "fp32", every=5.0, buoyant=buoyant)
        assert r["finite"]
        say(f"  Re {r['Re']:.2f}, volume {r['bubble_volume']}, mass drift {r['mass_drift']:.1e}")
        assert abs(r["mass_drift"]) < 1e-8
        assert r["Re"] > 3.0
        out[buoyant] = r["bubble_volume"][-1]
    assert out[True] >= 0.9
    assert out[True] > out[False] + 0.03
