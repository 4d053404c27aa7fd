"""Host-side checks of the standing-wave setup (tests/wave_study.py) against
the numbers the paper prints (tests/golden/standing_waves.txt, sec.
"Standing waves"): Re = a0 omega0 L / nu, the dispersion relations that fix g
(gravity wave) and sigma (capillary wave), the density and viscosity ratios,
the heavy-phase rate, and the initial profile.  No GPU."""
import math

import numpy as np
import pytest

import wave_study as S


@pytest.mark.parametrize("kind", ["gravity", "capillary"])
@pytest.mark.parametrize("L", [50, 100, 200, 400])
def test_wave_constants_reproduce_the_printed_numbers(kind, L):
    G = S.golden()
    wl, c = S.setup(kind, L)
    p = wl.params
    nu_H, nu_L = (p.tau_H - 0.5) / 3.0, (p.tau_L - 0.5) / 3.0
    assert abs(c["a0"] * c["w0"] * L / nu_H / G["Re"] - 1) < 1e-12
    assert abs(1.0 / p.tau_H - G["omega_H"]) < 1e-12
    assert abs(nu_H / nu_L - G["kinematic_viscosity_ratio"]) < 1e-12
    assert abs(p.rho_H / p.rho_L / G["density_ratio"] - 1) < 1e-12
    assert (p.mobility, p.xi) == (G["mobility"], G["xi"])
    k, d = 2 * math.pi / L, G["depth"] * L
    if kind == "gravity":
        assert abs(c["g"] * k * math.tanh(k * d) / c["w0"] ** 2 - 1) < 1e-12
        assert p.sigma == 0.0 and abs(p.g[1] + c["g"]) == 0.0
    else:
        assert abs(c["sigma"] * k ** 3 / (p.rho_H + p.rho_L) / c["w0"] ** 2 - 1) < 1e-12
        assert p.g == (0.0, 0.0, 0.0)


def test_initial_profile_is_the_printed_cosine():
    G = S.golden()
    L = 100
    wl, c = S.setup("capillary", L)
    from oracle.pflbm import interface_crossing
    for i in (0, 13, 25, 50):
        col = wl.phi0[0, :, i]
        want = G["depth"] * L + G["amplitude"] * L * math.cos(2 * math.pi * i / L)
        assert abs(interface_crossing(col, G["depth"] * L) - want) < 0.02
