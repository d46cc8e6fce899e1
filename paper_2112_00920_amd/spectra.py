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


def nh_convergence(t, dj_per_instance, k0, omega, n_list=None, gamma=0.005, axis=0):
    """Convergence of the two-step average in the number of shifts N_H (Sec. III.A).

    dj_per_instance: [N_H, n_t] or [N_H, n_t, 3] delta J_m(t) of the sub-simulations, in
    the order their shifts were drawn; `axis` picks the field direction of a 3-vector.
    For every N_H in n_list (default 1, 2, 4, ... and N_H itself) the first N_H
    sub-simulations give: the mean delta J, the dielectric function eps from it, and the
    standard error of that eps from the N_H per-shift eps_m (eps is affine in delta J,
    so the mean of the eps_m is eps), real and imaginary parts separately; `dev` is
    max over omega of |eps - eps(largest N_H)|.
    """
    x = np.asarray(dj_per_instance, float)
    if x.ndim == 3:
        x = x[:, :, axis]
    n_tot = x.shape[0]
    if n_list is None:
        n_list = sorted({min(2 ** i, n_tot) for i in range(int(np.ceil(np.log2(max(n_tot, 1)))) + 1)} | {n_tot})
    n_list = [int(n) for n in n_list]
    if any(n < 1 or n > n_tot for n in n_list):
        raise ValueError("every N_H must lie in 1..number of sub-simulations")
    eps_m = np.stack([dielectric_function(t, x[m], k0, omega, gamma)[1] for m in range(n_tot)])
    rows = []
    for n in n_list:
        e = eps_m[:n].mean(axis=0)
        if n > 1:
            sem = (eps_m[:n].real.std(axis=0, ddof=1) + 1j * eps_m[:n].imag.std(axis=0, ddof=1)) / np.sqrt(n)
        else:
            sem = np.zeros_like(e)
        rows.append({"n_h": n, "eps": e, "eps_sem": sem, "dj_mean": x[:n].mean(axis=0)})
    ref = rows[int(np.argmax(n_list))]["eps"]
    for r in rows:
        r["dev"] = float(np.max(np.abs(r["eps"] - ref)))
    return rows


def group_mean_and_sem(dj_per_instance):
    """Mean over the N_H sub-simulations and its standard error (Sec. III.A)."""
    x = np.asarray(dj_per_instance)
    m = x.mean(axis=0)
    sem = x.std(axis=0, ddof=1) / np.sqrt(x.shape[0]) if x.shape[0] > 1 else np.zeros_like(m)
    return m, sem
