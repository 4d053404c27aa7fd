"""Host-side checks of the Taylor-bubble setup (tests/taylor_study.py) against
the numbers the paper prints (tests/golden/taylor_bubble.txt, sec. "Taylor
bubble"): the lattice constants reproduce Bo, Mo, the density and viscosity
ratios and the heavy-phase rate; the geometry is the tube and gas cylinder of
the setup; the liquid starts hydrostatic; Re follows eq. Re.  No GPU."""
import math

import numpy as np
import pytest

import taylor_study as T


@pytest.mark.parametrize("D", [32, 64, 128])
def test_lattice_constants_reproduce_the_printed_numbers(D):
    G = T.golden()
    c = T.constants(D)
    mu_H = 1.0 * (c.tau_H - 0.5) / 3.0                # rho_H = 1, nu = (tau - 1/2)/3
    mu_L = c.rho_L * (c.tau_L - 0.5) / 3.0
    assert abs(c.g * D * D / c.sigma / G["Bo"] - 1) < 1e-12                    # eq. Bo
    assert abs(c.g * mu_H ** 4 / c.sigma ** 3 / G["Mo"] - 1) < 1e-12            # eq. Mo
    assert abs(1.0 / c.rho_L / G["density_ratio"] - 1) < 1e-12
    assert abs(mu_H / mu_L / G["viscosity_ratio"] - 1) < 1e-12
    assert abs(1.0 / c.tau_H - G["omega_H"]) < 1e-12
    assert abs(c.t_ref - math.sqrt(D / c.g)) < 1e-9                          # t* = t sqrt(g/D)


def test_geometry_and_hydrostatic_start():
    G = T.golden()
    D = 32
    wl, c = T.setup(D)
    assert (wl.nx, wl.ny, wl.nz) == (D, int(G["domain"][2]) * D, D)
    fluid = ~wl.solid
    # the tube: cells within D/2 of the axis, about pi/4 of the cross-section
    assert abs(fluid[:, 0, :].mean() - math.pi / 4) < 0.02
    # the gas cylinder's volume (diffuse interface: within a few per cent)
    gas = float(((1.0 - wl.phi0) * fluid).sum())
    want = math.pi * (0.5 * G["bubble_diameter"] * D) ** 2 * G["bubble_length"] * D
    assert abs(gas / want - 1) < 0.05
    # its axial extent
    col = wl.phi0[D // 2, :, D // 2]
    inside = np.nonzero(col < 0.5)[0]
    assert abs(inside.min() - G["bubble_bottom"] * D) <= 1
    assert abs(inside.max() + 1 - (G["bubble_bottom"] + G["bubble_length"]) * D) <= 1
    # liquid hydrostatic: p*(y) falls by 3 g per cell (p = p* rho c_s^2, rho_H = 1)
    liq = wl.pstar0[D // 2, :, 1 + D // 2]
    y_top = (G["bubble_bottom"] + G["bubble_length"]) * D
    seg = liq[int(y_top) + 20:int(y_top) + 70]          # away from the interface's tail
    assert np.allclose(np.diff(seg), -3.0 * c.g, rtol=1e-6, atol=0)
    assert float(np.abs(wl.u0).max()) == 0.0


def test_reynolds_number_follows_its_definition():
    c = T.constants(64)
    U = 0.01
    y10 = 300.0
    y15 = y10 + U * 5.0 * c.t_ref
    assert abs(T.reynolds(c, y10, y15) - 64 * U / c.mu_H) < 1e-9
    assert T.RE_PAPER == {64: 26.83, 128: 27.12}


def test_results_table_marks_windows_and_the_papers_unstable_resolutions(tmp_path):
    """The study's markdown table: the paper's window where a run reached
    t* = 15, the shortened window of a run that turned non-finite earlier,
    and "unstable" for the resolutions the paper reports unstable."""
    assert T.UNSTABLE_PAPER == {16, 32}
    res = [dict(D=16, precision="fp32", phase_lattice="d3q15", steps=62, re_paper=None,
                mass_drift=None, seconds=0.0),
           dict(D=64, precision="fp32", phase_lattice="d3q15", steps=28920, Re_last=26.21,
                Re_last_all_cells=27.71, Re_last_window=(10.0, 14.0), re_paper=26.83,
                mass_drift=None, seconds=10.0),
           dict(D=128, precision="fp64", phase_lattice="d3q15", steps=119670, Re=26.545,
                Re_all_cells=26.958, re_paper=27.12, mass_drift=-6.6e-12, seconds=400.0)]
    path = tmp_path / "t.md"
    T.write_table(res, str(path), "--D 16 64 128")
    rows = {int(l.split("|")[1]): [c.strip() for c in l.split("|")[1:-1]]
            for l in path.read_text().splitlines() if l.startswith("| ") and l.split("|")[1].strip().isdigit()}
    assert rows[16][5] == "diverges" and rows[16][8] == "unstable"
    assert rows[64][5] == "26.210" and rows[64][7].startswith("10-14") and rows[64][8] == "26.83"
    assert rows[128][5:9] == ["26.545", "26.958", "10-15", "27.12"] and rows[128][9] == "-6.6e-12"
