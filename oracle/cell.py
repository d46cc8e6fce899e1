"""Oracle (test infrastructure only): cell geometry, real-space grid and the
4th-order finite-difference representation of the kinetic operator
[p + kappa]^2 / 2 of Eq. (2), Sec. II.A.

Grid arrays are indexed [i3, i2, i1] (i1 fastest), so the last array axis is
lattice direction a_1 and axis ``-1 - d`` is direction a_{d+1}.
"""
from __future__ import annotations

import numpy as np

# 4th-order accurate central differences with +-2 neighbours.
D1_COEF = {1: 2.0 / 3.0, 2: -1.0 / 12.0}  # odd: f(s+j) - f(s-j)
D2_COEF = {0: -5.0 / 2.0, 1: 4.0 / 3.0, 2: -1.0 / 12.0}  # even


class Cell:
    """Periodic cell with lattice rows a_d, a real-space grid N_d along a_d,
    and atoms at fractional positions."""

    def __init__(self, lattice, grid, atom_frac=None, atom_species=None, species=None):
        self.A = np.asarray(lattice, dtype=float).reshape(3, 3)
        self.N = tuple(int(n) for n in grid)
        self.omega = abs(float(np.linalg.det(self.A)))
        self.B = 2.0 * np.pi * np.linalg.inv(self.A).T  # rows b_d, a_d . b_e = 2 pi delta
        self.ng = self.N[0] * self.N[1] * self.N[2]
        self.dV = self.omega / self.ng
        # grad = sum_d c_d d/ds_d with s_d the grid index along a_d
        self.c = np.array([self.N[d] * self.B[d] / (2.0 * np.pi) for d in range(3)])
        self.g = self.c @ self.c.T  # metric g_de = c_d . c_e
        self.atom_frac = np.zeros((0, 3)) if atom_frac is None else np.asarray(atom_frac, float)
        self.atom_species = (np.zeros(len(self.atom_frac), int) if atom_species is None
                             else np.asarray(atom_species, int))
        self.species = [] if species is None else list(species)
        self.tau = self.atom_frac @ self.A  # Cartesian atom positions

    @property
    def shape(self):
        """Array shape of one grid function, (N3, N2, N1)."""
        return (self.N[2], self.N[1], self.N[0])

    def positions(self):
        """Cartesian grid points r(i) = sum_d (i_d / N_d) a_d, shape (N3,N2,N1,3)."""
        i3, i2, i1 = np.meshgrid(np.arange(self.N[2]), np.arange(self.N[1]),
                                 np.arange(self.N[0]), indexing="ij")
        s = np.stack([i1 / self.N[0], i2 / self.N[1], i3 / self.N[2]], axis=-1)
        return s @ self.A

    def k_cart(self, k_frac):
        """Cartesian k = sum_d k_frac_d b_d."""
        return np.asarray(k_frac, float) @ self.B


def _ax(d):
    return -1 - d


def D1(f, d):
    """First derivative along grid index s_d (4th order, periodic)."""
    ax = _ax(d)
    out = D1_COEF[1] * (np.roll(f, -1, ax) - np.roll(f, 1, ax))
    out += D1_COEF[2] * (np.roll(f, -2, ax) - np.roll(f, 2, ax))
    return out


def D2(f, d):
    """Second derivative along grid index s_d (4th order, periodic)."""
    ax = _ax(d)
    out = D2_COEF[0] * f
    out = out + D2_COEF[1] * (np.roll(f, -1, ax) + np.roll(f, 1, ax))
    out += D2_COEF[2] * (np.roll(f, -2, ax) + np.roll(f, 2, ax))
    return out


def laplacian(cell: Cell, f):
    """L f = sum_d g_dd D2_d f + sum_{d != e} g_de D1_d D1_e f."""
    out = np.zeros_like(f)
    for d in range(3):
        if cell.g[d, d] != 0.0:
            out = out + cell.g[d, d] * D2(f, d)
    for d in range(3):
        for e in range(3):
            if d != e and cell.g[d, e] != 0.0:
                out = out + cell.g[d, e] * D1(D1(f, e), d)
    return out


def gradient(cell: Cell, f):
    """grad_FD f = sum_d c_d D1_d f; returns the 3 Cartesian components."""
    d1 = [D1(f, d) for d in range(3)]
    return [sum(cell.c[d, j] * d1[d] for d in range(3)) for j in range(3)]


def kinetic(cell: Cell, kappa, f):
    """T_kappa f = [-1/2 L - i kappa . grad_FD + |kappa|^2 / 2] f, i.e. the grid
    form of [p + kappa]^2 / 2 with p = -i grad acting on the periodic part
    (Eq. (2) with kappa = k + A(t))."""
    kappa = np.asarray(kappa, float)
    out = -0.5 * laplacian(cell, f)
    kc = cell.c @ kappa  # kappa . c_d
    for d in range(3):
        if kc[d] != 0.0:
            out = out - 1j * kc[d] * D1(f, d)
    out = out + 0.5 * float(kappa @ kappa) * f
    return out
