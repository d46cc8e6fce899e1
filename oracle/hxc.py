"""Oracle (test infrastructure only): the Hartree-exchange-correlation
potential v_Hxc[rho] of Eq. (2), Sec. II.A.

* Hartree: v_H(G) = 4 pi rho(G) / |G|^2 by FFT; G = 0 and the Nyquist planes
  (m_d = -N_d/2 for even N_d) are set to zero.  The G = 0 choice fixes the
  energy reference; the Nyquist choice keeps v_H real.
* Exchange (Slater, spin-unpolarised): v_x = -(3 rho / pi)^{1/3}.
* Correlation: Perdew-Zunger 1981 parametrisation of the unpolarised
  Ceperley-Alder gas, with r_s = (3 / (4 pi rho))^{1/3}.
* rho < 1e-30 gives v_xc = 0.
"""
from __future__ import annotations

import numpy as np

from .cell import Cell

PZ_GAMMA, PZ_BETA1, PZ_BETA2 = -0.1423, 1.0529, 0.3334
PZ_A, PZ_B, PZ_C, PZ_D = 0.0311, -0.048, 0.0020, -0.0116
RHO_MIN = 1e-30


def g_squared(cell: Cell):
    """|G|^2 on the FFT grid (array order [m3, m2, m1]) and the Nyquist mask."""
    m = [np.fft.fftfreq(cell.N[d]) * cell.N[d] for d in range(3)]
    m3, m2, m1 = np.meshgrid(m[2], m[1], m[0], indexing="ij")
    G = (m1[..., None] * cell.B[0] + m2[..., None] * cell.B[1] + m3[..., None] * cell.B[2])
    g2 = np.einsum("...i,...i->...", G, G)
    nyq = np.zeros(cell.shape, dtype=bool)
    for d, md in zip(range(3), (m1, m2, m3)):
        if cell.N[d] % 2 == 0:
            nyq |= md == -cell.N[d] // 2
    return g2, nyq


def hartree(cell: Cell, rho):
    g2, nyq = g_squared(cell)
    rg = np.fft.fftn(rho)
    with np.errstate(divide="ignore", invalid="ignore"):
        vg = 4.0 * np.pi * rg / g2
    vg[0, 0, 0] = 0.0
    vg[nyq] = 0.0
    return np.real(np.fft.ifftn(vg))


def slater_exchange(rho):
    rho = np.asarray(rho, float)
    safe = np.where(rho > RHO_MIN, rho, 1.0)
    return np.where(rho > RHO_MIN, -np.cbrt(3.0 * safe / np.pi), 0.0)


def pz81_eps(rs):
    """Correlation energy per electron eps_c(r_s)."""
    rs = np.asarray(rs, float)
    hi = PZ_GAMMA / (1.0 + PZ_BETA1 * np.sqrt(rs) + PZ_BETA2 * rs)
    lrs = np.log(rs)
    lo = PZ_A * lrs + PZ_B + PZ_C * rs * lrs + PZ_D * rs
    return np.where(rs >= 1.0, hi, lo)


def pz81_v(rs):
    """Correlation potential v_c = d(rho eps_c)/d rho = eps_c - (r_s/3) d eps_c / d r_s."""
    rs = np.asarray(rs, float)
    sq = np.sqrt(rs)
    den = 1.0 + PZ_BETA1 * sq + PZ_BETA2 * rs
    hi = PZ_GAMMA / den * (1.0 + 7.0 / 6.0 * PZ_BETA1 * sq + 4.0 / 3.0 * PZ_BETA2 * rs) / den
    lrs = np.log(rs)
    lo = (PZ_A * lrs + (PZ_B - PZ_A / 3.0) + 2.0 / 3.0 * PZ_C * rs * lrs
          + (2.0 * PZ_D - PZ_C) / 3.0 * rs)
    return np.where(rs >= 1.0, hi, lo)


def correlation(rho):
    rho = np.asarray(rho, float)
    safe = np.where(rho > RHO_MIN, rho, 1.0)
    rs = np.cbrt(3.0 / (4.0 * np.pi * safe))
    return np.where(rho > RHO_MIN, pz81_v(rs), 0.0)


def v_hxc(cell: Cell, rho):
    return hartree(cell, rho) + slater_exchange(rho) + correlation(rho)
