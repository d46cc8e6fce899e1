"""Oracle (test infrastructure only): Kohn-Sham ground state by self-consistent
dense diagonalisation.  The runs of Sec. III start from the ground state, and
the induced current delta J(t) = J(t) - J(t < 0) is measured against it
(Sec. III.A).  Pulay (DIIS) mixing of the density."""
from __future__ import annotations

import numpy as np
import scipy.linalg

from .hamiltonian import System
from .hxc import v_hxc as hxc_potential
from .propagate import density


def diagonalise(sys: System, v_hxc):
    """Lowest n_bands eigenpairs of h_k (A = 0) for every k; orbitals are
    normalised to sum_r |u|^2 dV = 1."""
    u = np.empty((sys.nk, sys.nb) + sys.cell.shape, dtype=complex)
    eps = np.empty((sys.nk, sys.nb))
    for k in range(sys.nk):
        H = sys.dense_h(sys.k_cart[k], v_hxc)
        H = 0.5 * (H + H.conj().T)
        e, vec = scipy.linalg.eigh(H, subset_by_index=[0, sys.nb - 1], driver="evr")
        eps[k] = e
        u[k] = (vec.T / np.sqrt(sys.cell.dV)).reshape((sys.nb,) + sys.cell.shape)
    return u, eps


def scf(sys: System, tol=1e-10, max_iter=200, alpha=0.4, history=6, verbose=False):
    """Returns (u, eps, v_hxc, residual).  Converged when sum|rho_out - rho_in| dV < tol."""
    rho_in = np.full(sys.cell.shape, np.sum(sys.occ) / sys.cell.omega)
    hist_in, hist_res = [], []
    res_norm = np.inf
    for it in range(max_iter):
        v = hxc_potential(sys.cell, rho_in)
        u, eps = diagonalise(sys, v)
        rho_out = density(sys, u)
        res = rho_out - rho_in
        res_norm = float(np.sum(np.abs(res)) * sys.cell.dV)
        if verbose:
            print(f"scf {it}: residual {res_norm:.3e}")
        if res_norm < tol:
            return u, eps, v, res_norm
        hist_in.append(rho_in.ravel().copy())
        hist_res.append(res.ravel().copy())
        hist_in, hist_res = hist_in[-history:], hist_res[-history:]
        m = len(hist_res)
        R = np.array(hist_res)
        Bm = np.zeros((m + 1, m + 1))
        Bm[:m, :m] = R @ R.T
        Bm[m, :m] = Bm[:m, m] = -1.0
        rhs = np.zeros(m + 1)
        rhs[m] = -1.0
        try:
            coef = np.linalg.solve(Bm, rhs)[:m]
        except np.linalg.LinAlgError:
            coef = np.zeros(m)
            coef[-1] = 1.0
        rho_opt = coef @ np.array(hist_in)
        res_opt = coef @ R
        rho_in = np.maximum((rho_opt + alpha * res_opt).reshape(sys.cell.shape), 0.0)
    return u, eps, v, res_norm
