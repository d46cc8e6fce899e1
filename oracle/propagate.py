"""Oracle (test infrastructure only): real-time propagation of the TDKS
equation (Eq. (1)) with density (Eq. (3)), current (Eqs. (5)-(6)) and the
two-step average (Eq. (9), Sec. II.B procedure steps 1-4).

Step n -> n+1 (explicit 4th-order Taylor expansion of exp(-i h dt)):
  kappa = k + A(t_n + dt/2), v_Hxc from rho(t_n);
  w_0 = u, w_m = (-i dt / m) h_kappa w_{m-1}, u(t_{n+1}) = sum_{m=0..4} w_m;
  rho^{n+1} = rho(u^{n+1}); v_Hxc^{n+1} recomputed ('scf'), kept ('frozen'),
  or zero ('none');  J^{n+1} = J(u^{n+1}, kappa = k + A(t_{n+1})).

Predictor-corrector variant ('pc', SCF only; the paper's Octopus runs leave the
propagator to that code): the Hxc potential of the step is taken at the mid-step,
  predictor  u~ = T4(h[v_n]) u^n, v~ = v_Hxc[rho(u~)],
  corrector  u^{n+1} = T4(h[(v_n + v~) / 2]) u^n,
which makes the coupling through v_Hxc second order in dt (the explicit step holds
v_Hxc[rho(t_n)] over the whole step: first order).  With a frozen or zero
potential both variants are the same step.

Current (Eq. (5)) with the kinetic momentum pi = (1/i)[r, h] (Eq. (6)):
  J = -(1/Omega) sum_k w_k sum_b f_b [ sum_r u* (-i grad_FD + kappa) u dV
                                       + sum_{a,lm} 2 E_l Im(conj(c_d) c) ],
  c = <P_{a,lm}|u>, c_d = <d P_{a,lm}|u>; the second term is the commutator of
  the non-local projectors with r, i.e. d V^kappa / d kappa.
"""
from __future__ import annotations

import numpy as np

from .cell import gradient
from .hamiltonian import System
from .hxc import v_hxc as hxc_potential

TAYLOR_ORDER = 4


def taylor_step(sys: System, kappa, v_hxc, u, dt, order=TAYLOR_ORDER):
    """One Taylor step for the orbitals u[b] of a single k."""
    w = u
    acc = u.copy()
    for m in range(1, order + 1):
        w = (-1j * dt / m) * sys.apply_h(kappa, v_hxc, w)
        acc = acc + w
    return acc


def density(sys: System, u):
    """rho(r) = sum_k w_k sum_b f_b |u_bk(r)|^2 (Eq. (3) with Eq. (7))."""
    return np.einsum("k,b,kbijl->ijl", sys.wk, sys.occ, np.abs(u) ** 2)


def current_k(sys: System, kappa, u):
    """Per-k band sum  sum_b f_b <u_b| pi_kappa |u_b>, a Cartesian 3-vector."""
    cell = sys.cell
    kappa = np.asarray(kappa, float)
    out = np.zeros(3)
    grad = gradient(cell, u)
    nrm = np.sum(np.abs(u) ** 2, axis=(-3, -2, -1)) * cell.dV
    for j in range(3):
        kin = np.real(np.sum(np.conj(u) * (-1j) * grad[j], axis=(-3, -2, -1))) * cell.dV
        out[j] += np.sum(sys.occ * (kin + kappa[j] * nrm))
    flat = u.reshape(u.shape[0], -1)
    for a, at in enumerate(sys.proj.atoms):
        P = sys.proj.phased(a, kappa)  # (4, nsup)
        us = flat[:, at["idx"]]
        c = cell.dV * us @ np.conj(P).T  # (nb, 4)
        for j in range(3):
            cd = cell.dV * us @ (np.conj(P) * at["d"][:, j][None, :]).T
            out[j] += np.sum(sys.occ[:, None] * 2.0 * at["E"][None, :] * np.imag(np.conj(cd) * c))
    return out


def current(sys: System, A, u):
    """J = -(1/Omega) sum_k w_k J_k (Eq. (5)) at vector potential A."""
    J = np.zeros(3)
    for k in range(sys.nk):
        J += sys.wk[k] * current_k(sys, sys.k_cart[k] + np.asarray(A, float), u[k])
    return -J / sys.cell.omega


def norms(sys: System, u):
    return np.sum(np.abs(u) ** 2, axis=(-3, -2, -1)) * sys.cell.dV


class Run:
    """A single TDDFT simulation driven step by step."""

    def __init__(self, sys: System, u0, dt, hxc_mode="scf", v_hxc_frozen=None, propagator="taylor"):
        if propagator not in ("taylor", "pc"):
            raise ValueError(propagator)
        self.propagator = propagator
        self.sys = sys
        self.u = np.array(u0, dtype=complex)
        self.dt = float(dt)
        self.mode = hxc_mode
        if hxc_mode == "frozen":
            self.v_hxc = np.asarray(v_hxc_frozen, float).reshape(sys.cell.shape)
        elif hxc_mode == "none":
            self.v_hxc = np.zeros(sys.cell.shape)
        elif hxc_mode == "scf":
            self.v_hxc = hxc_potential(sys.cell, density(sys, self.u))
        else:
            raise ValueError(hxc_mode)
        self.J_pre = current(sys, np.zeros(3), self.u)

    def step(self, A_mid, A_end):
        sys = self.sys
        v = self.v_hxc
        if self.propagator == "pc" and self.mode == "scf":
            u_pred = np.empty_like(self.u)
            for k in range(sys.nk):
                kappa = sys.k_cart[k] + np.asarray(A_mid, float)
                u_pred[k] = taylor_step(sys, kappa, self.v_hxc, self.u[k], self.dt)
            v_pred = hxc_potential(sys.cell, density(sys, u_pred))
            v = 0.5 * (self.v_hxc + v_pred)
        for k in range(sys.nk):
            kappa = sys.k_cart[k] + np.asarray(A_mid, float)
            self.u[k] = taylor_step(sys, kappa, v, self.u[k], self.dt)
        if self.mode == "scf":
            self.v_hxc = hxc_potential(sys.cell, density(sys, self.u))
        return current(sys, A_end, self.u)

    def run(self, A_tab):
        """Advance len(A_tab) steps; returns J^{n+1} for each step, shape (n, 3)."""
        out = np.empty((len(A_tab), 3))
        for n in range(len(A_tab)):
            out[n] = self.step(A_tab[n, 0], A_tab[n, 1])
        return out


def two_step_average(delta_j_per_instance):
    """O(t) = (1/N_H) sum_m O_m(t) (Eq. (9), procedure step 4)."""
    return np.mean(np.asarray(delta_j_per_instance), axis=0)
