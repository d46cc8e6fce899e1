"""k-point sets of the two-step scheme (library side).

Monkhorst-Pack grid (Eq. (8)) and its shifted version (Eq. (10)):
k = sum_j (2 n_j - N_j - 1 + 2 q_j) / (2 N_j) b_j, n_j = 1..N_j, in fractional
coordinates, ordered with n_1 fastest and wrapped into (-1/2, 1/2] so that the
sub-grids use exactly the representatives of the dense grid (the
finite-difference Hamiltonian is not periodic in k).  Uniform shift grids use
q = (2 j + M - 1) / (2 M) mod 1, j = 0..M-1; their union over j is the (N M)-point
MP grid.  Quasi-random shifts use the Halton sequence in bases 2, 3, 5
(Sec. II.B).
"""
from __future__ import annotations

import numpy as np


def _wrap(x):
    return x - np.ceil(x - 0.5)


def mp_grid(n, shift=(0.0, 0.0, 0.0)) -> np.ndarray:
    n = [int(v) for v in n]
    i3, i2, i1 = np.meshgrid(np.arange(1, n[2] + 1), np.arange(1, n[1] + 1), np.arange(1, n[0] + 1),
                             indexing="ij")
    idx = np.stack([i1.ravel(), i2.ravel(), i3.ravel()], axis=1).astype(float)
    N = np.asarray(n, float)
    q = np.asarray(shift, float)
    return _wrap((2.0 * idx - N - 1.0 + 2.0 * q) / (2.0 * N))


def uniform_shifts(m):
    """(2j + M - 1) / (2M) mod 1 for j = 0..M-1 along each axis."""
    return [((2.0 * j + m - 1) / (2.0 * m)) % 1.0 for j in range(int(m))]


def shifted_grid(coarse, shifts, index) -> np.ndarray:
    q = [uniform_shifts(shifts[d])[index[d]] for d in range(3)]
    return mp_grid(coarse, q)


def from_spec(kspec) -> np.ndarray:
    """k-points of one sub-simulation: the coarse MP grid shifted by a uniform-grid shift,
    a Halton point or an explicit shift (Eq. (10))."""
    given = [kspec.shifts is not None, getattr(kspec, "halton_index", None) is not None,
             getattr(kspec, "shift_q", None) is not None]
    if sum(given) > 1:
        raise ValueError("give at most one of shifts, halton_index, shift_q")
    if given[1]:
        if int(kspec.halton_index) < 1:
            raise ValueError("halton_index counts from 1")
        return mp_grid(kspec.coarse, halton_shifts(1, start=int(kspec.halton_index))[0])
    if given[2]:
        q = np.asarray(kspec.shift_q, float)
        if q.shape != (3,) or np.any(q < 0.0) or np.any(q >= 1.0):
            raise ValueError("shift_q must be three numbers in [0, 1)")
        return mp_grid(kspec.coarse, q)
    if not given[0]:
        return mp_grid(kspec.coarse)
    return shifted_grid(kspec.coarse, kspec.shifts, kspec.shift_index)


def halton_shifts(n, bases=(2, 3, 5), start=1) -> np.ndarray:
    out = np.zeros((n, len(bases)))
    for r, m in enumerate(range(start, start + n)):
        for c, b in enumerate(bases):
            f, x, i = 1.0, 0.0, m
            while i > 0:
                f /= b
                x += f * (i % b)
                i //= b
            out[r, c] = x
    return out
