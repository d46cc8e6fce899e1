"""Oracle (test infrastructure only): Kohn-Sham ground state.  The runs of
Sec. III start from the ground state, and the induced current
delta J(t) = J(t) - J(t < 0) is measured against it (Sec. III.A).

Two routes:
* scf: self-consistent dense diagonalisation with Pulay (DIIS) mixing of the
  density (the reference route, small grids only);
* imaginary_time_scf: the route the GPU library takes, written out step by
  step.  The propagator of Eq. (1) taken at imaginary time, exp(-tau h), with
  the same 4th-order Taylor expansion as the real-time step (w_0 = u,
  w_m = (-tau/m) h w_{m-1}, sum over m <= 4), filters every band towards the
  lowest eigenvectors of h_k; after each step the bands of each k are
  orthonormalised (Cholesky: S = U^H U dV = L L^H, U <- U L^{-H}), the density
  is formed (Eq. (3)) and mixed linearly into the input density,
  rho_in <- (1 - alpha) rho_in + alpha rho_out, from which v_Hxc is rebuilt.
  With every band occupied the density, the current and the total energy depend
  only on the span of the bands, so no subspace rotation is needed.
"""
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


def imaginary_time_step(sys: System, kappa, v_hxc, u, tau, order=4):
    """exp(-tau h_kappa) u by its Taylor expansion to the given order."""
    w = u
    acc = u.copy()
    for m in range(1, order + 1):
        w = (-tau / m) * sys.apply_h(kappa, v_hxc, w)
        acc = acc + w
    return acc


def orthonormalise(u, dV):
    """Cholesky orthonormalisation of the bands u[b] of one k: with the bands as columns
    of U and S = U^H U dV = L L^H (L lower triangular), return U L^{-H}, whose first
    band is the first input band normalised (Gram-Schmidt order)."""
    nb = u.shape[0]
    U = u.reshape(nb, -1).T
    S = (U.conj().T @ U) * dV
    L = np.linalg.cholesky(S)
    # U_new L^H = U  <=>  conj(L) U_new^T = U^T
    Y = scipy.linalg.solve_triangular(L.conj(), U.T, lower=True)
    return Y.reshape(u.shape)


def imaginary_time_scf(sys: System, u0, tau, alpha, n_iter, hxc_mode="scf", v_hxc_frozen=None):
    """n_iter iterations of: imaginary-time Taylor step of every k with v_Hxc[rho_in],
    orthonormalisation, rho_out, residual sum |rho_out - rho_in| dV, linear mixing
    (scf) or rho_in <- rho_out (frozen / none).  rho_in starts as the density of u0.
    Returns (u, rho(u), v_Hxc[rho(u)] (the frozen or zero potential otherwise),
    residuals per iteration)."""
    u = np.array(u0, dtype=complex)
    rho_in = density(sys, u)
    if hxc_mode == "scf":
        v = hxc_potential(sys.cell, rho_in)
    elif hxc_mode == "frozen":
        v = np.asarray(v_hxc_frozen, float)
    else:
        v = np.zeros(sys.cell.shape)
    res = []
    for it in range(n_iter):
        for k in range(sys.nk):
            u[k] = orthonormalise(imaginary_time_step(sys, sys.k_cart[k], v, u[k], tau), sys.cell.dV)
        rho_out = density(sys, u)
        res.append(float(np.sum(np.abs(rho_out - rho_in)) * sys.cell.dV))
        if hxc_mode == "scf":
            rho_in = (1.0 - alpha) * rho_in + alpha * rho_out
            v = hxc_potential(sys.cell, rho_in)
        else:
            rho_in = rho_out
    rho = density(sys, u)
    v_final = hxc_potential(sys.cell, rho) if hxc_mode == "scf" else v
    return u, rho, v_final, res


def subspace_energy(sys: System, v_hxc, u):
    """sum_k w_k sum_b <u_bk| h_k |u_bk> dV (the band-energy sum of the occupied span)."""
    e = 0.0
    for k in range(sys.nk):
        hu = sys.apply_h(sys.k_cart[k], v_hxc, u[k])
        e += sys.wk[k] * float(np.real(np.sum(np.conj(u[k]) * hu)) * sys.cell.dV)
    return e
