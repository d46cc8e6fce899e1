"""Host-side observables from the recorded current (library side).

* delta J of the two-step scheme: per-shift delta J_m averaged over the N_H
  shifts (Eq. (9), procedure step 4; Sec. III.A).
* Linear response to the impulsive field: J~(omega) = int_0 dt e^{i omega t}
  e^{-gamma t} delta J(t) (Eq. (13) with a damping window), sigma = J~ / k0
  (Eq. (12)), epsilon = 1 + 4 pi i sigma / omega (Eq. (14)).
* High-harmonic power spectrum: omega^2 |int dt e^{i omega t} W(t) J(t)|^2 with
  W = cos^4(pi (t - T/2) / T) on (0, T) (Eqs. (16)-(17)).
Integrals use the trapezoid rule on the step grid.
"""
from __future__ import annotations

import numpy as np


def _ft(t, f, omega):
    t = np.asarray(t, float)
    w = np.full(len(t), t[1] - t[0])
    w[0] *= 0.5
    w[-1] *= 0.5
    ph = np.exp(1j * np.outer(np.asarray(omega, float), t))
    return ph @ (w * np.asarray(f))


def dielectric_function(t, dj, k0, omega, gamma=0.005):
    sigma = _ft(t, np.exp(-gamma * np.asarray(t)) * np.asarray(dj), omega) / k0
    return sigma, 1.0 + 4j * np.pi * sigma / np.asarray(omega)


def hhg_spectrum(t, j, T, omega):
    t = np.asarray(t, float)
    win = np.where((t > 0) & (t < T), np.cos(np.pi * (t - T / 2) / T) ** 4, 0.0)
    return np.asarray(omega) ** 2 * np.abs(_ft(t, win * np.asarray(j), omega)) ** 2


def group_mean_and_sem(dj_per_instance):
    """Mean over the N_H sub-simulations and its standard error (Sec. III.A)."""
    x = np.asarray(dj_per_instance)
    m = x.mean(axis=0)
    sem = x.std(axis=0, ddof=1) / np.sqrt(x.shape[0]) if x.shape[0] > 1 else np.zeros_like(m)
    return m, sem
