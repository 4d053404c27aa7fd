"""Host-side checks of the rising-bubble setup (tests/rising_bubble_study.py)
against the numbers the paper prints (tests/golden/rising_bubbles.txt, sec.
"Rising bubble"): each case's lattice constants reproduce its Bo, Mo and
heavy-phase rate and the density and viscosity ratios; the geometry is the
8D x 8D x 20D box with the bubble at (4D, 4D, 1D); the liquid starts
hydrostatic.  No GPU."""
import math

import numpy as np
import pytest

import rising_bubble_study as R


@pytest.mark.parametrize("case", [1, 2, 3, 4])
def test_case_constants_reproduce_the_printed_numbers(case):
    G = R.golden()
    Bo, Mo, omega_H = G[f"case{case}"]
    D = 32
    c = R.constants(case, D)
    mu_H = (c["tau_H"] - 0.5) / 3.0
    mu_L = c["rho_L"] * (c["tau_L"] - 0.5) / 3.0
    assert abs(c["g"] * D * D / c["sigma"] / Bo - 1) < 1e-12                   # eq. Bo
    assert abs(c["g"] * mu_H ** 4 / c["sigma"] ** 3 / Mo - 1) < 1e-12           # eq. Mo
    assert abs(1.0 / c["tau_H"] - omega_H) < 1e-12
    assert abs(1.0 / c["rho_L"] / G["density_ratio"] - 1) < 1e-12
    assert abs(mu_H / mu_L / G["dynamic_viscosity_ratio"] - 1) < 1e-12
    assert len(G[f"Re_PFLBM_case{case}"]) == 2


def test_geometry_and_hydrostatic_start():
    G = R.golden()
    D = 16
    wl, c = R.setup(2, D)
    assert (wl.nx, wl.ny, wl.nz) == (8 * D, 20 * D, 8 * D)
    assert wl.periodic == (True, False, True)
    # the bubble: the phi = 1/2 surface is the sphere of diameter D at (4D, 1D, 4D)
    cx, cy, cz = (v * D for v in G["bubble_centre"])
    col = wl.phi0[int(cy), :, int(cx)]               # along the vertical through the centre
    gas = np.nonzero(col < 0.5)[0]
    assert abs((gas.min() + gas.max() + 1) / 2 - cz) <= 0.5
    assert abs(gas.max() + 1 - gas.min() - D) <= 1
    # hydrostatic liquid: p* falls by 3 g per cell above the bubble
    liq = wl.pstar0[int(cy), int(3 * D):int(3 * D) + 40, int(cx)]
    assert np.allclose(np.diff(liq), -3.0 * c["g"], rtol=1e-6, atol=0)
