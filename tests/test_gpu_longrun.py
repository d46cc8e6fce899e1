"""Accuracy of the FP32 propagation over the workloads' full length.

The FP64 GPU path matches the oracle to 1e-10 over short runs (test_gpu_parity);
here it is the reference for 4000-step FP32 runs, where the oracle would take
days:

* linear response (delta kick 1e-3, Sec. III.A): two sub-simulations of the
  two-step workload (8^3 coarse k x one 4^3 shift each, 16 bands, 16^3, SCF),
  started from their Kohn-Sham ground state (prepared on the GPU by imaginary-time
  iterations, as the runs of Sec. III start from the ground state), their mean
  delta J(t) and the dielectric function derived from it (Eqs. 12-14, damping
  0.005 Ha); the same with the predictor-corrector propagator;
* nonlinear response (Sec. III.B): the sin^2 pulse of the HHG workload taken at
  its peak, one of its sub-simulations on its own 20^3 grid (64 k, 16 bands), J(t)
  and the harmonic spectrum of the segment.

The bar is 1e-4 of the peak of the compared current.
"""
import sys

import numpy as np
import pytest

import workloads as W
from paper_2112_00920_amd import spectra

pytestmark = pytest.mark.gpu

N_STEPS = 4000


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(insts, u0s, A, precision, dt, propagator="taylor"):
    import paper_2112_00920_amd as tdks

    with tdks.Propagator(insts, precision=precision, dt=dt, norm_stride=100, propagator=propagator) as prop:
        for i, u in enumerate(u0s):
            prop.load_orbitals(i, u)
        prop.step(A)
        prop.check()  # the numeric health check over the whole run
        return prop.current(per="instance"), prop.current_pre()


GS_ITER, GS_TAU, GS_MIX = 1500, 0.1, 0.5


@pytest.fixture(scope="module")
def ground_pair():
    """Two sub-simulations of the two-step workload relaxed to their Kohn-Sham ground state in
    FP64 (imaginary-time Taylor-4 filter, orthonormalisation, density mixing), returned as
    host orbitals so that the FP32 and FP64 runs start from the same state."""
    import paper_2112_00920_amd as tdks

    wl = W.config("twostep_g16_mp8_s4")
    insts = [wl.instances[0], wl.instances[21]]
    _say(f"ground state: {GS_ITER} imaginary-time iterations (tau {GS_TAU}) of {len(insts)} sub-simulations, FP64")
    with tdks.Propagator(insts, precision="fp64", dt=wl.dt) as prop:
        for i, inst in enumerate(insts):
            prop.load_orbitals(i, W.random_orbitals_torch(500 + i, inst.n_k, inst.n_bands, inst.grid, inst.omega))
        res = prop.ground_state(GS_ITER, GS_TAU, GS_MIX)
        us = [prop.get_orbitals(i) for i in range(len(insts))]
        jpre = prop.current_pre()
    _say(f"  density residual per sub-simulation {res}; J_pre {jpre.tolist()}")
    assert np.all(res < 1e-4), res
    return wl, insts, us


def test_kick_linear_response_4000_steps(ground_pair):
    wl, insts, u0s = ground_pair
    A = wl.field.table(N_STEPS, wl.dt)
    _say(f"kick from the ground state: {len(insts)} sub-simulations, {N_STEPS} steps, FP32 then FP64")
    dj32, _ = _run(insts, u0s, A, "fp32", wl.dt)
    dj64, _ = _run(insts, u0s, A, "fp64", wl.dt)
    m32, m64 = dj32.mean(axis=0), dj64.mean(axis=0)
    peak = np.max(np.abs(m64))
    n_e = 2 * insts[0].n_bands / insts[0].omega
    err_t = np.max(np.abs(m32 - m64), axis=0) / peak
    err_step = np.max(np.abs(m32 - m64), axis=1) / peak
    _say(f"  peak |dJ| {peak:.3e} (n k0 = {n_e * wl.field.k0:.3e}); max |dJ32 - dJ64| / peak per axis {err_t}")
    for n in (100, 500, 1000, 2000, 4000):
        _say(f"    by step {n}: {np.max(err_step[:n]):.2e}")
    assert np.max(err_t) < 1e-4
    # dielectric function along the kick (x), 0.02..1.0 Ha
    t = wl.dt * np.arange(1, N_STEPS + 1)
    om = np.linspace(0.02, 1.0, 200)
    _, e32 = spectra.dielectric_function(t, m32[:, 0], wl.field.k0, om)
    _, e64 = spectra.dielectric_function(t, m64[:, 0], wl.field.k0, om)
    de = np.max(np.abs(e32 - e64)) / np.max(np.abs(e64 - 1.0))
    _say(f"  eps(omega): max |eps32 - eps64| / max |eps64 - 1| = {de:.2e}")
    assert de < 1e-4


def test_pulse_nonlinear_4000_steps():
    wl = W.config("hhg_twostep_g20_mp4_s4")
    insts = [wl.instances[27]]  # shift (3, 2, 1) of the 4^3, on 20^3
    u0s = [W.random_orbitals_torch(600, insts[0].n_k, insts[0].n_bands, insts[0].grid, insts[0].omega)]
    start = int(round(0.5 * wl.field.T / wl.dt))
    A = wl.field.table(N_STEPS, wl.dt, start)
    _say(f"pulse: peak A {np.max(np.abs(A)):.3f}, {N_STEPS} steps from step {start}, FP32 then FP64")
    dj32, pre32 = _run(insts, u0s, A, "fp32", wl.dt)
    dj64, pre64 = _run(insts, u0s, A, "fp64", wl.dt)
    j32, j64 = dj32[0] + pre32[0], dj64[0] + pre64[0]  # the pulse test starts from random orbitals
    peak = np.max(np.abs(j64))
    err = np.max(np.abs(j32 - j64)) / peak
    _say(f"  peak |J| {peak:.3e}; max |J32 - J64| / peak = {err:.2e}")
    assert err < 1e-4
    t = wl.dt * np.arange(1, N_STEPS + 1)
    T = t[-1]
    om = wl.field.omega * np.arange(1, 16)
    h32 = spectra.hhg_spectrum(t, j32[:, 0], T, om)
    h64 = spectra.hhg_spectrum(t, j64[:, 0], T, om)
    rel = np.abs(h32 - h64) / np.max(h64)
    _say(f"  harmonic power, |H32 - H64| / max H64 at orders 1..15: max {np.max(rel):.2e}")
    assert np.max(rel) < 1e-4


def test_predictor_corrector_kick_4000_steps(ground_pair):
    """The predictor-corrector propagator over the kick workload's length from the same
    ground state: FP32 against FP64 (both predictor-corrector), and the dielectric function."""
    wl, insts, u0s = ground_pair
    A = wl.field.table(N_STEPS, wl.dt)
    _say(f"predictor-corrector kick from the ground state: {len(insts)} sub-simulations, {N_STEPS} steps")
    out = {}
    for prec in ("fp32", "fp64"):
        dj, _ = _run(insts, u0s, A, prec, wl.dt, propagator="pc")
        out[prec] = dj.mean(axis=0)
    peak = np.max(np.abs(out["fp64"]))
    err = np.max(np.abs(out["fp32"] - out["fp64"])) / peak
    _say(f"  peak |dJ| {peak:.3e}; max |dJ32 - dJ64| / peak = {err:.2e}")
    assert err < 1e-4
    t = wl.dt * np.arange(1, N_STEPS + 1)
    om = np.linspace(0.02, 1.0, 200)
    _, e32 = spectra.dielectric_function(t, out["fp32"][:, 0], wl.field.k0, om)
    _, e64 = spectra.dielectric_function(t, out["fp64"][:, 0], wl.field.k0, om)
    de = np.max(np.abs(e32 - e64)) / np.max(np.abs(e64 - 1.0))
    _say(f"  eps(omega): max |eps32 - eps64| / max |eps64 - 1| = {de:.2e}")
    assert de < 1e-4
