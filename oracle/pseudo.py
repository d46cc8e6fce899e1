"""Oracle (test infrastructure only): electron-ion potential v_ion of Eq. (2),
Sec. II.A -- a local part plus norm-conserving-style non-local
Kleinman-Bylander projectors ("may consist of non-local operators").

Model (the paper's HGH tables are not available):
* local: v_loc(r) = sum_a sum_L D_s exp(-|r - tau_a - L|^2 / (2 w_s^2)), with
  every lattice image within 15 w_s of the point;
* non-local: V^kappa = sum_{a,lm} E_l |P^kappa_{a,lm}> <P^kappa_{a,lm}|, with
  P^kappa_{a,lm}(r) = exp(-i kappa . d_a(r)) f_lm(d_a(r)), d_a(r) the
  minimum-image displacement r - tau_a - L, and
  f_s = N_s g, f_{p,i} = N_p d_i g, g(d) = max(0, exp(-|d|^2/2rc^2) - exp(-Rc^2/2rc^2)),
  N_s = (pi^{3/2} rc^3)^{-1/2}, N_p = (pi^{3/2} rc^5 / 2)^{-1/2};
  <P|v> = sum_r conj(P) v dV.  The exp(-i kappa . d) factor is the
  e^{-i kappa r} V e^{i kappa r} form of the operator for the periodic part.
"""
from __future__ import annotations

import itertools

import numpy as np

from .cell import Cell


def local_potential(cell: Cell, cutoff_widths: float = 15.0):
    r = cell.positions()
    v = np.zeros(cell.shape)
    nmax = []
    for a in range(len(cell.tau)):
        sp = cell.species[cell.atom_species[a]]
        rcut = cutoff_widths * sp.w
        # plane spacing along b_d is 2 pi / |b_d|; enough images to cover rcut
        nmax = [int(np.ceil(rcut * np.linalg.norm(cell.B[d]) / (2 * np.pi))) + 1 for d in range(3)]
        for n in itertools.product(*[range(-m, m + 1) for m in nmax]):
            L = np.asarray(n, float) @ cell.A
            dd = r - cell.tau[a] - L
            d2 = np.einsum("...i,...i->...", dd, dd)
            mask = d2 < rcut * rcut
            if mask.any():
                v = v + np.where(mask, sp.D * np.exp(-d2 / (2.0 * sp.w * sp.w)), 0.0)
    return v


class Projectors:
    """Support points and radial data of the s + p KB projectors of each atom."""

    def __init__(self, cell: Cell):
        self.cell = cell
        r = cell.positions().reshape(-1, 3)
        self.atoms = []
        covered = np.zeros(cell.ng, dtype=int)
        for a in range(len(cell.tau)):
            sp = cell.species[cell.atom_species[a]]
            gcut = np.exp(-sp.Rc ** 2 / (2.0 * sp.rc ** 2))
            ns = (np.pi ** 1.5 * sp.rc ** 3) ** -0.5
            npn = (np.pi ** 1.5 * sp.rc ** 5 / 2.0) ** -0.5
            idx_all, d_all = [], []
            hits = np.zeros(cell.ng, dtype=int)
            for n in itertools.product(range(-2, 3), repeat=3):
                L = np.asarray(n, float) @ cell.A
                dd = r - cell.tau[a] - L
                d2 = np.einsum("ij,ij->i", dd, dd)
                sel = np.nonzero(d2 < sp.Rc ** 2)[0]
                if len(sel):
                    idx_all.append(sel)
                    d_all.append(dd[sel])
                    hits[sel] += 1
            if (hits > 1).any():
                raise ValueError("projector radius exceeds half the minimum image distance")
            idx = np.concatenate(idx_all)
            d = np.concatenate(d_all)
            order = np.argsort(idx)
            idx, d = idx[order], d[order]
            g = np.maximum(0.0, np.exp(-np.einsum("ij,ij->i", d, d) / (2.0 * sp.rc ** 2)) - gcut)
            f = np.stack([ns * g, npn * d[:, 0] * g, npn * d[:, 1] * g, npn * d[:, 2] * g])
            E = np.array([sp.Es, sp.Ep, sp.Ep, sp.Ep])
            self.atoms.append({"idx": idx, "d": d, "f": f, "E": E})
            covered[idx] += 1
        self.covered = covered

    def phased(self, a, kappa):
        """P^kappa_{a,lm} on the support points, shape (4, n_sup)."""
        at = self.atoms[a]
        ph = np.exp(-1j * (at["d"] @ np.asarray(kappa, float)))
        return at["f"] * ph[None, :]

    def project(self, kappa, w):
        """c[a][..., lm] = <P^kappa_{a,lm} | w> for w of shape (..., N3, N2, N1)."""
        flat = w.reshape(w.shape[:-3] + (-1,))
        out = []
        for a, at in enumerate(self.atoms):
            P = self.phased(a, kappa)
            out.append(self.cell.dV * flat[..., at["idx"]] @ np.conj(P).T)
        return out

    def apply(self, kappa, w):
        """V^kappa_NL w."""
        flat = w.reshape(w.shape[:-3] + (-1,))
        res = np.zeros_like(flat)
        for a, at in enumerate(self.atoms):
            P = self.phased(a, kappa)
            c = self.cell.dV * flat[..., at["idx"]] @ np.conj(P).T
            res[..., at["idx"]] += (c * at["E"]) @ P
        return res.reshape(w.shape)
