"""Closed-form references used to pin the oracle.

Test infrastructure only (see oracle/__init__.py).
"""
from __future__ import annotations

import math

import numpy as np
from scipy.special import erfc as _erfc_real
from scipy.special import wofz


def erfc_complex(z: complex) -> complex:
    """erfc(z) = exp(-z^2) w(i z) with the Faddeeva function w."""
    return complex(np.exp(-z * z) * wofz(1j * z))


def capillary_omega0(sigma: float, k: float, rho_H: float, rho_L: float) -> float:
    """Inviscid capillary-wave angular frequency (paper, capillary-wave setup)."""
    return math.sqrt(sigma * k ** 3 / (rho_H + rho_L))


def prosperetti_amplitude(t, a0: float, nu: float, k: float, omega0: float,
                          rho_H: float, rho_L: float) -> np.ndarray:
    """Prosperetti's small-amplitude capillary-wave amplitude a(t) (paper eq.
    prosperetti-amplitude with the quartic for z_i and beta = rho_L rho_H /
    (rho_L + rho_H)^2); equal kinematic viscosities, no gravity, at rest at t=0."""
    beta = rho_L * rho_H / (rho_L + rho_H) ** 2
    nk2 = nu * k * k
    coeffs = [1.0, -4.0 * beta * math.sqrt(nk2), 2.0 * (1.0 - 6.0 * beta) * nk2,
              4.0 * (1.0 - 3.0 * beta) * nk2 ** 1.5, (1.0 - 4.0 * beta) * nk2 ** 2 + omega0 ** 2]
    z = np.roots(coeffs)
    Z = [np.prod([z[m] - z[i] for m in range(4) if m != i]) for i in range(4)]
    t = np.atleast_1d(np.asarray(t, dtype=np.float64))
    out = np.empty_like(t)
    pre = 4.0 * (1.0 - 4.0 * beta) * nk2 ** 2 / (8.0 * (1.0 - 4.0 * beta) * nk2 ** 2 + omega0 ** 2)
    for n, tt in enumerate(t):
        s = pre * a0 * _erfc_real(math.sqrt(nk2 * tt))
        acc = 0j
        for i in range(4):
            acc += (z[i] / Z[i]) * (omega0 ** 2 * a0 / (z[i] ** 2 - nk2)) * \
                np.exp((z[i] ** 2 - nk2) * tt) * erfc_complex(z[i] * math.sqrt(tt))
        out[n] = s + acc.real
    return out


def gravity_wave(t, a0: float, nu: float, k: float, g: float, d: float) -> np.ndarray:
    """Linear standing gravity wave amplitude at x = 0 with viscous decay
    (paper, gravity-wave analytical model): a0 exp(-2 nu k^2 t) cos(omega0 t)."""
    w0 = math.sqrt(g * k * math.tanh(k * d))
    t = np.asarray(t, dtype=np.float64)
    return a0 * np.exp(-2.0 * nu * k * k * t) * np.cos(w0 * t)


def poiseuille(y, H: float, accel: float, nu: float) -> np.ndarray:
    """Body-force driven channel flow between walls at y = 0 and y = H."""
    y = np.asarray(y, dtype=np.float64)
    return accel * y * (H - y) / (2.0 * nu)


def laplace_jump(sigma: float, R: float) -> float:
    """Young-Laplace pressure jump of a spherical drop: 2 sigma / R."""
    return 2.0 * sigma / R
