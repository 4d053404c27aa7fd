"""Velocity sets and weighted-orthogonal moment matrices for the oracle.

Test infrastructure only (see oracle/__init__.py).

Velocity sets (paper sec. "The lattice Boltzmann method", eq. LBE: c_i in
{-1,0,1}^d, c_s^2 = 1/3).  The phase field uses D3Q15 and the hydrodynamics
D3Q27 here; the weights are the textbook ones, selected by |c|^2:
  D3Q15: 2/9 (rest), 1/9 (|c|^2 = 1), 1/72 (|c|^2 = 3)
  D3Q27: 8/27, 2/27 (|c|^2 = 1), 1/54 (|c|^2 = 2), 1/216 (|c|^2 = 3)
  D2Q9:  4/9, 1/9 (|c|^2 = 1), 1/36 (|c|^2 = 2), in the x-y plane (c_z = 0);
         the velocity set of the paper's two-dimensional runs (sec. "Numerical
         experiments", standing waves), used for both lattices there

MRT (paper eq. mrt, and the remark in sec. "Numerical experiments" that a
weighted orthogonal MRT was used): the moment matrix M has one row per
polynomial of c, obtained by Gram-Schmidt orthogonalisation of monomials
c_x^a c_y^b c_z^c under the weighted inner product <p, q> = sum_i w_i p(c_i)
q(c_i), taken in order of increasing total degree.  Each row remembers the
degree of the monomial it came from; relaxation rates are assigned per
degree.
"""
from __future__ import annotations

import itertools

import numpy as np
import torch

CS2 = 1.0 / 3.0


class Lattice:
    def __init__(self, name: str, c: np.ndarray, w: np.ndarray, monomials):
        self.name = name
        self.q = c.shape[0]
        self.c_np = c.astype(np.int64)
        self.w_np = w.astype(np.float64)
        self.c = torch.tensor(c, dtype=torch.float64)
        self.w = torch.tensor(w, dtype=torch.float64)
        # opposite direction index: c_opp = -c
        lookup = {tuple(v): i for i, v in enumerate(self.c_np)}
        self.opp = np.array([lookup[tuple(-v)] for v in self.c_np], dtype=np.int64)
        self.monomials = list(monomials)
        M, deg = gram_schmidt_moments(self.c_np, self.w_np, self.monomials)
        self.M = torch.tensor(M, dtype=torch.float64)
        self.Minv = torch.linalg.inv(self.M)
        self.degree = torch.tensor(deg, dtype=torch.int64)


def _velocities(max_norm2_allowed):
    out = []
    for c in itertools.product((-1, 0, 1), repeat=3):
        n2 = sum(v * v for v in c)
        if n2 in max_norm2_allowed:
            out.append(c)
    # stable order: by |c|^2, then lexicographic
    out.sort(key=lambda v: (sum(x * x for x in v), v))
    return np.array(out, dtype=np.int64)


def gram_schmidt_moments(c: np.ndarray, w: np.ndarray, monomials):
    """Rows of M: w-orthogonalised monomials evaluated at the lattice velocities.

    monomials: list of (a, b, c) exponents, already ordered by total degree.
    Returns (M [q, q], degree [q]).
    """
    rows = []
    degs = []
    for (a, b, e) in monomials:
        v = (c[:, 0].astype(np.float64) ** a) * (c[:, 1].astype(np.float64) ** b) * \
            (c[:, 2].astype(np.float64) ** e)
        for r in rows:
            v = v - (np.sum(w * v * r) / np.sum(w * r * r)) * r
        if np.sqrt(np.sum(w * v * v)) < 1e-12:
            raise ValueError(f"monomial {(a, b, e)} is linearly dependent on this lattice")
        rows.append(v)
        degs.append(a + b + e)
    return np.array(rows), np.array(degs, dtype=np.int64)


def d3q15() -> Lattice:
    c = _velocities({0, 1, 3})
    n2 = (c * c).sum(1)
    w = np.where(n2 == 0, 2.0 / 9.0, np.where(n2 == 1, 1.0 / 9.0, 1.0 / 72.0))
    mon = [(0, 0, 0),
           (1, 0, 0), (0, 1, 0), (0, 0, 1),
           (2, 0, 0), (0, 2, 0), (0, 0, 2), (1, 1, 0), (0, 1, 1), (1, 0, 1),
           (1, 1, 1), (1, 2, 0), (0, 1, 2), (2, 0, 1),
           (2, 2, 0)]
    return Lattice("D3Q15", c, w, mon)


def d3q27() -> Lattice:
    c = _velocities({0, 1, 2, 3})
    n2 = (c * c).sum(1)
    w = np.select([n2 == 0, n2 == 1, n2 == 2, n2 == 3],
                  [8.0 / 27.0, 2.0 / 27.0, 1.0 / 54.0, 1.0 / 216.0])
    mon = sorted(itertools.product((0, 1, 2), repeat=3), key=lambda m: (sum(m), m))
    return Lattice("D3Q27", c, w, mon)


def d2q9() -> Lattice:
    c = np.array([v for v in _velocities({0, 1, 2}) if v[2] == 0], dtype=np.int64)
    n2 = (c * c).sum(1)
    w = np.select([n2 == 0, n2 == 1, n2 == 2], [4.0 / 9.0, 1.0 / 9.0, 1.0 / 36.0])
    mon = sorted(((a, b, 0) for a in (0, 1, 2) for b in (0, 1, 2)), key=lambda m: (sum(m), m))
    return Lattice("D2Q9", c, w, mon)


D3Q15 = d3q15()
D3Q27 = d3q27()
D2Q9 = d2q9()
