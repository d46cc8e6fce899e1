"""Oracle (test infrastructure only): observables derived from the current.

* Linear response to the impulsive field (Sec. III.A): J~(omega) is the
  Fourier transform of delta J(t) (Eq. (13)) with a damping exp(-gamma t) or the
  window W_L(x) = 1 - 3x^2 + 2x^3 of the paper; sigma = J~ / k0 (Eq. (12));
  epsilon = 1 + 4 pi i sigma / omega (Eq. (14)).
* High-harmonic spectrum (Sec. III.B): I(omega) = omega^2 |FT[W(t) J(t)]|^2
  (Eq. (16)) with W(t) = cos^4(pi (t - T/2) / T) on (0, T) (Eq. (17), with the
  duration T restored in the argument).
Time integrals use the trapezoid rule on t_n = n dt.
"""
from __future__ import annotations

import numpy as np


def _trapezoid_weights(n):
    w = np.ones(n)
    w[0] = w[-1] = 0.5
    return w


def fourier(t, f, omega):
    """int dt e^{i omega t} f(t) by the trapezoid rule."""
    t = np.asarray(t, float)
    dt = t[1] - t[0]
    w = _trapezoid_weights(len(t)) * dt
    return np.exp(1j * np.outer(omega, t)) @ (w * np.asarray(f))


def conductivity(t, dj, k0, omega, gamma=0.005, window_T=None):
    t = np.asarray(t, float)
    if window_T is None:
        env = np.exp(-gamma * t)
    else:
        x = t / window_T
        env = np.where((x > 0) & (x < 1), 1 - 3 * x ** 2 + 2 * x ** 3, 0.0)
        env[0] = 1.0
    return fourier(t, env * np.asarray(dj), omega) / k0


def dielectric(sigma, omega):
    return 1.0 + 4j * np.pi * sigma / np.asarray(omega)


def hhg_window(t, T):
    t = np.asarray(t, float)
    inside = (t > 0) & (t < T)
    return np.where(inside, np.cos(np.pi * (t - T / 2) / T) ** 4, 0.0)


def hhg_spectrum(t, j, T, omega):
    return np.asarray(omega) ** 2 * np.abs(fourier(t, hhg_window(t, T) * np.asarray(j), omega)) ** 2


def standard_error(samples):
    """Standard error of the mean over the N_H sub-simulations (Sec. III.A)."""
    s = np.asarray(samples)
    n = s.shape[0]
    return np.std(s, axis=0, ddof=1) / np.sqrt(n)


def nh_convergence(t, samples, k0, omega, n_values, gamma=0.005):
    """Two-step average over the first N_H shifts for each N_H in n_values (Sec. III.A):
    per N_H the dielectric function of the mean delta J (Eqs. (12)-(14)), and the standard
    error of its real and imaginary parts over the N_H per-shift results.  samples is
    [N_H, n_t] (one field direction)."""
    out = []
    for n in n_values:
        dj_mean = np.zeros(len(t))
        for m in range(n):
            dj_mean = dj_mean + np.asarray(samples[m], float)
        dj_mean = dj_mean / n
        eps = dielectric(conductivity(t, dj_mean, k0, omega, gamma), omega)
        per = np.array([dielectric(conductivity(t, samples[m], k0, omega, gamma), omega) for m in range(n)])
        if n > 1:
            sem = standard_error(per.real) + 1j * standard_error(per.imag)
        else:
            sem = np.zeros(len(omega), dtype=complex)
        out.append((n, eps, sem))
    return out
