"""Oracle (test infrastructure only): the time-dependent Kohn-Sham Hamiltonian
h_k(t) = [p + k + A(t)]^2 / 2 + v_ion + v_Hxc[rho]   (Eq. (2), Sec. II.A)
on the real-space grid, for the periodic part u_bk of the Bloch orbitals.
"""
from __future__ import annotations

import numpy as np

from . import kpoints
from .cell import Cell, kinetic
from .pseudo import Projectors, local_potential


class System:
    """One independent TDDFT simulation: a cell, its grid, potentials, k-set
    and occupations.  Orbitals are arrays u[k][b][N3][N2][N1]."""

    def __init__(self, inst, k_frac=None):
        self.inst = inst
        self.cell = Cell(inst.lattice, inst.grid, inst.atom_frac, inst.atom_species, inst.species)
        self.k_frac = kpoints.kset(inst.kspec) if k_frac is None else np.asarray(k_frac, float)
        self.k_cart = self.cell.k_cart(self.k_frac)
        self.nk = len(self.k_frac)
        self.nb = inst.n_bands
        self.wk = np.full(self.nk, 1.0 / self.nk)  # Eq. (7): uniform weights
        self.occ = np.full(self.nb, 2.0)  # spin-unpolarised occupation
        self.v_loc = local_potential(self.cell)
        self.proj = Projectors(self.cell)

    def apply_h(self, kappa, v_hxc, w):
        """h_kappa w with kappa = k + A: kinetic + (v_loc + v_Hxc) + V_NL."""
        out = kinetic(self.cell, kappa, w)
        out = out + (self.v_loc + v_hxc) * w
        out = out + self.proj.apply(kappa, w)
        return out

    def dense_h(self, kappa, v_hxc):
        """Dense N_g x N_g matrix of h_kappa (columns = h applied to unit vectors)."""
        ng = self.cell.ng
        eye = np.eye(ng, dtype=complex).reshape((ng,) + self.cell.shape)
        cols = self.apply_h(kappa, v_hxc, eye)
        return cols.reshape(ng, ng).T
