"""Oracle (test infrastructure only): k-point sets of the two-step scheme.

* Monkhorst-Pack grid, Eq. (8), Sec. II.A.
* Shifted Monkhorst-Pack grid, Eq. (10), Sec. II.B, with shift (q, p, r).
* Uniform shift grids: with M shifts per axis q_j = ((2j + M - 1) / (2M)) mod 1
  makes the union of the M^3 shifted N^3 grids exactly the (NM)^3 MP grid.
* Halton sequence in bases 2, 3, 5 (Sec. II.B) for quasi-random shifts.

All k are fractional coordinates in units of the reciprocal vectors b_d and are
wrapped into (-1/2, 1/2]: the finite-difference Hamiltonian is not invariant
under k -> k + G, so the two-step sub-grids must use exactly the dense grid's
representatives.
"""
from __future__ import annotations

from fractions import Fraction
import itertools

import numpy as np


def wrap_half(x):
    """Map fractional coordinates into (-1/2, 1/2]."""
    x = np.asarray(x, dtype=float)
    return x - np.ceil(x - 0.5)


def monkhorst_pack(n, shift=(0.0, 0.0, 0.0)):
    """k_{n1 n2 n3} = sum_j (2 n_j - N_j - 1 + 2 q_j) / (2 N_j) b_j, n_j = 1..N_j
    (Eq. (8) for q = 0, Eq. (10) otherwise), ordered with n1 fastest."""
    n = tuple(int(v) for v in n)
    pts = []
    for n3 in range(1, n[2] + 1):
        for n2 in range(1, n[1] + 1):
            for n1 in range(1, n[0] + 1):
                idx = (n1, n2, n3)
                pts.append([(2 * idx[j] - n[j] - 1 + 2 * shift[j]) / (2 * n[j]) for j in range(3)])
    return wrap_half(np.array(pts, dtype=float))


def uniform_shift(m: int, j: int) -> float:
    """j-th of m uniform shifts per axis, q_j = ((2j + m - 1) / (2m)) mod 1."""
    return ((2 * j + m - 1) / (2 * m)) % 1.0


def uniform_shift_fraction(m: int, j: int) -> Fraction:
    return Fraction(2 * j + m - 1, 2 * m) % 1


def kset(kspec):
    """Fractional k-points of one instance from its KSpec: Eq. (10) with the shift
    (q, p, r) taken from a uniform shift grid, a Halton point (Sec. II.B) or given."""
    if getattr(kspec, "halton_index", None) is not None:
        m = int(kspec.halton_index)
        q = [radical_inverse(m, b) for b in (2, 3, 5)]
        return monkhorst_pack(kspec.coarse, q)
    if getattr(kspec, "shift_q", None) is not None:
        return monkhorst_pack(kspec.coarse, list(kspec.shift_q))
    if kspec.shifts is None:
        return monkhorst_pack(kspec.coarse)
    q = [uniform_shift(kspec.shifts[d], kspec.shift_index[d]) for d in range(3)]
    return monkhorst_pack(kspec.coarse, q)


def mp_fractions(n, shift=(Fraction(0),) * 3):
    """Exact rational version of the shifted MP grid, for tests."""
    out = []
    for idx in itertools.product(*[range(1, v + 1) for v in n]):
        p = []
        for j in range(3):
            x = Fraction(2 * idx[j] - n[j] - 1, 2 * n[j]) + Fraction(shift[j]) / n[j]
            x = x - ((x - Fraction(1, 2)).__ceil__())  # wrap into (-1/2, 1/2]
            p.append(x)
        out.append(tuple(p))
    return out


def radical_inverse(i: int, base: int) -> float:
    """van der Corput radical inverse of the integer i in the given base."""
    f, r = 1.0, 0.0
    while i > 0:
        f /= base
        r += f * (i % base)
        i //= base
    return r


def halton(n_points: int, bases=(2, 3, 5), start: int = 1):
    """Halton points m = start..start+n-1 in (0,1)^3 (m = 0 would give 0)."""
    return np.array([[radical_inverse(m, b) for b in bases]
                     for m in range(start, start + n_points)])
