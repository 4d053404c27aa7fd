"""Seeded synthetic inputs for the coupled phase-field LBM step.

This module is the one place that both the CPU oracle (through the tests)
and the HIP path (through the tests and the benchmark) take their inputs
from.  It holds no arithmetic of the method itself: it only produces initial
fields (phase field phi0, velocity u0, normalised pressure p*0), solid masks,
grid descriptions and parameter sets.  The equilibrium initialisation, the
collision, the streaming and everything else happen separately on each side.

Initial phase fields use the diffuse-interface profile of the paper's
experimental section (sec. "Numerical experiments", the tanh initialisation):
phi = 1/2 +- 1/2 tanh((d)/(xi/2)) across an interface at signed distance d.

Velocity noise is drawn from SplitMix64 (Steele, Lea, Flood 2014; finaliser
constants as published by Vigna), keyed by (seed, cell index, component), so
any implementation can reproduce it bit for bit.

All arrays are float64 numpy arrays in [z][y][x] order (x fastest); vector
fields are [3][z][y][x] with components (x, y, z).  Cell centres sit at
(i + 1/2, j + 1/2, k + 1/2); walls lie on the box faces.
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np

SEED = 11637

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(counter: np.ndarray) -> np.ndarray:
    """SplitMix64 output for 64-bit counters (vectorised, wraps mod 2^64)."""
    with np.errstate(over="ignore"):
        z = counter.astype(np.uint64) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_noise(seed: int, n: int, comp: int, amplitude: float) -> np.ndarray:
    """U(-amplitude, amplitude) for cells 0..n-1 and one vector component.

    Counter = seed * 2^32 + 3 * idx + comp + 1; the top 53 bits of the
    SplitMix64 output give a double in [0, 1).
    """
    idx = np.arange(n, dtype=np.uint64)
    with np.errstate(over="ignore"):
        ctr = (np.uint64(seed) << np.uint64(32)) + idx * np.uint64(3) + np.uint64(comp + 1)
    bits = splitmix64(ctr) >> np.uint64(11)
    unit = bits.astype(np.float64) * (1.0 / 9007199254740992.0)
    return (2.0 * unit - 1.0) * amplitude


def tanh_profile(dist: np.ndarray, xi: float) -> np.ndarray:
    """phi = 1/2 + 1/2 tanh(dist / (xi/2)); dist > 0 on the heavy side."""
    return 0.5 + 0.5 * np.tanh(2.0 * dist / xi)


@dataclasses.dataclass
class Params:
    """Physical parameters in lattice units (dx = dt = 1, c_s^2 = 1/3)."""
    tau_H: float = 0.53
    tau_L: float = 0.53
    mobility: float = 0.02
    xi: float = 4.0
    sigma: float = 1e-4
    rho_H: float = 1.0
    rho_L: float = 1e-3
    g: tuple = (0.0, 0.0, 0.0)
    s_high: float = 1.0
    fp16_scale_log2: tuple = (12.0, 12.0)
    normal_eps: float = 1e-4
    s_bulk: float = 0.0        # MRT rate of g's bulk mode; 0 = the second-order rate
    rho_g_ref: float = 0.0     # body force (rho - rho_g_ref) g; rho_H: buoyancy only

    def copy(self, **kw) -> "Params":
        return dataclasses.replace(self, **kw)


@dataclasses.dataclass
class Workload:
    name: str
    nx: int
    ny: int
    nz: int
    periodic: tuple            # (px, py, pz) booleans; non-periodic axes carry walls
    params: Params
    phi0: np.ndarray           # [nz, ny, nx]
    u0: np.ndarray             # [3, nz, ny, nx]
    pstar0: np.ndarray         # [nz, ny, nx]
    solid: Optional[np.ndarray]  # [nz, ny, nx] bool or None (box walls only)
    steps: int

    @property
    def cells(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def periodic_bits(self) -> int:
        return int(self.periodic[0]) | (int(self.periodic[1]) << 1) | (int(self.periodic[2]) << 2)


def _centres(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz) + 0.5, np.arange(ny) + 0.5, np.arange(nx) + 0.5,
                          indexing="ij")
    return x, y, z


def capillary_wave(nx: int, ny: int, nz: int, *, depth: float, amplitude: float,
                   xi: float = 4.0, params: Optional[Params] = None, noise: float = 1e-8,
                   seed: int = SEED, steps: int = 200, periodic=(True, False, True),
                   name: str = "capillary_wave") -> Workload:
    """Standing capillary wave: heavy phase below y0(i) = depth + a0 cos(2 pi i / nx).

    The integer column index i is used so that column 0 holds the crest.
    """
    i = np.arange(nx, dtype=np.float64)
    y0 = depth + amplitude * np.cos(2.0 * math.pi * i / nx)
    _, y, _ = _centres(nx, ny, nz)
    phi0 = tanh_profile(y0[None, None, :] - y, xi)
    n = nx * ny * nz
    u0 = np.stack([uniform_noise(seed, n, c, noise).reshape(nz, ny, nx) for c in range(3)])
    p = (params or Params()).copy(xi=xi)
    return Workload(name, nx, ny, nz, tuple(bool(v) for v in periodic), p, phi0, u0,
                    np.zeros((nz, ny, nx)), None, steps)


def config0() -> Workload:
    """32x32x32 standing capillary wave, FP64 parity case (200 steps)."""
    return capillary_wave(32, 32, 32, depth=16.0, amplitude=0.05 * 32, xi=4.0,
                          params=Params(tau_H=0.53, tau_L=0.53, mobility=0.02, sigma=1e-4),
                          steps=200, name="capillary_wave_32^3")


def config1(scale: int = 1) -> Workload:
    """Rising gas bubble, 128x512x128 with six bounce-back faces (scale divides sizes)."""
    nx, ny, nz = 128 // scale, 512 // scale, 128 // scale
    D = 32.0 / scale
    x, y, z = _centres(nx, ny, nz)
    c = 64.0 / scale
    r = np.sqrt((x - c) ** 2 + (y - c) ** 2 + (z - c) ** 2)
    phi0 = tanh_profile(r - D / 2, 5.0)
    p = Params(tau_H=0.52, tau_L=0.70, mobility=0.02, xi=5.0, sigma=1e-4,
               g=(0.0, -1e-6, 0.0))
    return Workload(f"rising_bubble_{nx}x{ny}x{nz}", nx, ny, nz, (False, False, False), p,
                    phi0, np.zeros((3, nz, ny, nx)), np.zeros((nz, ny, nx)), None, 20000)


def config2(scale: int = 1, mobility: float = 0.01) -> Workload:
    """Drop impact into a pool, 384^3, x/z periodic, y walls, drop falling at 0.05.

    With the benchmark's mobility M = 0.01 the impact becomes unstable after
    ~1.1k steps in every precision; M = 0.03 (the lowest mobility the paper
    found stable for its drop impacts) runs the full 5000 steps."""
    n = 384 // scale
    x, y, z = _centres(n, n, n)
    pool = tanh_profile(96.0 / scale - y, 5.0)
    c = np.array([192.0, 136.0, 192.0]) / scale
    r = np.sqrt((x - c[0]) ** 2 + (y - c[1]) ** 2 + (z - c[2]) ** 2)
    drop = tanh_profile(32.0 / scale - r, 5.0)
    phi0 = np.maximum(pool, drop)
    u0 = np.zeros((3, n, n, n))
    u0[1][drop > 0.5] = -0.05
    p = Params(tau_H=0.52, tau_L=0.70, mobility=mobility, xi=5.0, sigma=5e-5,
               g=(0.0, -1e-6, 0.0))
    name = f"drop_impact_{n}^3" + ("" if mobility == 0.01 else f"_M{mobility:g}")
    return Workload(name, n, n, n, (True, False, True), p, phi0, u0,
                    np.zeros((n, n, n)), None, 5000)


def config3() -> Workload:
    """64x128x64 capillary wave for the parameter-gradient form (2000 steps)."""
    return capillary_wave(64, 128, 64, depth=64.0, amplitude=0.05 * 64, xi=4.0,
                          params=Params(tau_H=0.53, tau_L=0.53, mobility=0.02, sigma=1e-4),
                          steps=2000, name="capillary_wave_64x128x64")


def config4(scale: int = 1) -> Workload:
    """Taylor bubble in a cylindrical tube (diameter 120) of a 128x1024x128 box."""
    nx, ny, nz = 128 // scale, 1024 // scale, 128 // scale
    x, y, z = _centres(nx, ny, nz)
    cx = 64.0 / scale
    rr = np.sqrt((x - cx) ** 2 + (z - cx) ** 2)
    solid = rr > 60.0 / scale
    # signed distance to a capped cylinder of radius 42 spanning y in [120, 320]
    R, y0, y1 = 42.0 / scale, 120.0 / scale, 320.0 / scale
    d = np.maximum(np.maximum(rr - R, y0 - y), y - y1)
    phi0 = tanh_profile(d, 5.0)
    p = Params(tau_H=0.52, tau_L=0.70, mobility=0.02, xi=5.0, sigma=1e-4,
               g=(0.0, -2e-6, 0.0))
    return Workload(f"taylor_bubble_{nx}x{ny}x{nz}", nx, ny, nz, (True, False, True), p,
                    phi0, np.zeros((3, nz, ny, nx)), np.zeros((nz, ny, nx)), solid, 4000)


def random_state(nx: int, ny: int, nz: int, *, periodic=(True, False, True), seed: int = 7,
                 params: Optional[Params] = None, solid_fraction: float = 0.0,
                 u_amp: float = 0.005, p_amp: float = 1e-4, steps: int = 10,
                 name: str = "random") -> Workload:
    """Smooth random phase field plus random velocity/pressure, optional random solids.

    Used for parity cases on ragged grids: phi is a sum of a few low Fourier
    modes passed through the tanh profile, so interfaces of width ~xi appear.
    """
    rng = np.random.default_rng(seed)
    p = params or Params(tau_H=0.6, tau_L=0.8, mobility=0.05, xi=4.0, sigma=2e-4,
                         rho_L=0.1, g=(1e-6, -2e-6, 5e-7))
    x, y, z = _centres(nx, ny, nz)
    field = np.zeros((nz, ny, nx))
    for _ in range(4):
        k = rng.integers(1, 3, size=3)
        ph = rng.uniform(0, 2 * math.pi, size=3)
        field += np.cos(2 * math.pi * k[0] * x / nx + ph[0]) * \
            np.cos(2 * math.pi * k[1] * y / ny + ph[1]) * np.cos(2 * math.pi * k[2] * z / nz + ph[2])
    phi0 = tanh_profile(3.0 * field, p.xi)
    u0 = rng.uniform(-u_amp, u_amp, size=(3, nz, ny, nx))
    pstar0 = rng.uniform(-p_amp, p_amp, size=(nz, ny, nx))
    solid = None
    if solid_fraction > 0:
        solid = rng.uniform(size=(nz, ny, nx)) < solid_fraction
        phi0 = np.where(solid, 0.0, phi0)
        u0 = np.where(solid[None], 0.0, u0)
        pstar0 = np.where(solid, 0.0, pstar0)
    return Workload(name, nx, ny, nz, tuple(bool(v) for v in periodic), p, phi0, u0, pstar0,
                    solid, steps)


CONFIGS = {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}
