"""Oracle pins of the spectra (Sec. III): the HHG spectrum of Eqs. (16)-(17) and the
paper's W_L window of the linear-response transform (Eq. (13)), each against closed
forms that do not go through the oracle's trapezoid quadrature.  Also the eigenstate
norm through oracle.propagate.norms."""
import numpy as np

from oracle import spectra


def _cos4_window_transform(omega, T):
    """int_0^T e^{i omega t} cos^4(pi (t - T/2) / T) dt in closed form.  With s = t - T/2,
    cos^4(pi s / T) = 3/8 + cos(2 pi s / T) / 2 + cos(4 pi s / T) / 8, and
    int_{-T/2}^{T/2} e^{i omega s} cos(a s) ds = S(omega + a) + S(omega - a),
    S(x) = sin(x T / 2) / x (-> T / 2 at x = 0)."""
    omega = np.asarray(omega, float)

    def S(x):
        safe = np.where(x == 0.0, 1.0, x)
        return np.where(x == 0.0, T / 2, np.sin(x * T / 2) / safe)

    def cos_integral(a):
        return S(omega + a) + S(omega - a)

    body = 3 / 8 * cos_integral(0.0) + cos_integral(2 * np.pi / T) / 2 + cos_integral(4 * np.pi / T) / 8
    return np.exp(1j * omega * T / 2) * body


def test_hhg_window_is_cos4():
    """Eq. (17) with the duration restored: W(t) = cos^4(pi (t - T/2) / T) on (0, T).
    cos^4(pi/4) = 1/4 at t = T/4 and 3T/4 (a cos^2 window would give 1/2), 1 at T/2 and
    0 outside (0, T)."""
    T = 800.0
    w = spectra.hhg_window(np.array([-1.0, 0.0, T / 4, T / 2, 3 * T / 4, T, T + 1]), T)
    np.testing.assert_allclose(w, [0, 0, 0.25, 1, 0.25, 0, 0], rtol=0, atol=1e-15)


def test_hhg_spectrum_of_constant_current_closed_form():
    """I(omega) = omega^2 |FT[W J]|^2 (Eq. (16)).  For J = 1 the transform is that of the
    window, known in closed form; the omega^2 weight, the window's power and its argument
    are all fixed by it.  At omega = 0 the window integrates to 3T/8 (cos^2: T/2)."""
    T = 1000.0
    t = np.arange(0.0, T + 1e-9, 0.05)
    om = np.array([0.003, 0.01, 0.02, 0.05, 0.13, 0.4])
    got = spectra.hhg_spectrum(t, np.ones_like(t), T, om)
    want = om ** 2 * np.abs(_cos4_window_transform(om, T)) ** 2
    np.testing.assert_allclose(got, want, rtol=1e-9, atol=1e-12 * np.max(want))
    w0 = spectra.fourier(t, spectra.hhg_window(t, T), np.array([0.0]))[0]
    np.testing.assert_allclose(w0.real, 3 * T / 8, rtol=1e-12)


def test_hhg_harmonic_ratio():
    """J = a cos(w1 t) + b cos(3 w1 t) with w1 T >> 1: the windowed transform at a harmonic
    n w1 is (c_n / 2) 3T/8 up to the window's far tails, so I(n w1) = (n w1)^2 (c_n / 2)^2
    (3T/8)^2, and I(3 w1) / I(w1) = 9 b^2 / a^2 (the omega^2 weight of Eq. (16))."""
    T = 2000.0
    t = np.arange(0.0, T + 1e-9, 0.02)
    w1, a, b = 0.5, 1.0, 0.3
    j = a * np.cos(w1 * t) + b * np.cos(3 * w1 * t)
    I = spectra.hhg_spectrum(t, j, T, np.array([w1, 3 * w1]))
    np.testing.assert_allclose(I[0], w1 ** 2 * (a / 2) ** 2 * (3 * T / 8) ** 2, rtol=1e-6)
    np.testing.assert_allclose(I[1], (3 * w1) ** 2 * (b / 2) ** 2 * (3 * T / 8) ** 2, rtol=1e-6)
    np.testing.assert_allclose(I[1] / I[0], 9 * b * b / (a * a), rtol=1e-6)


def test_conductivity_wl_window_values():
    """The paper's window W_L(x) = 1 - 3x^2 + 2x^3, x = t / T_W (Eq. (13)).  A current that is
    non-zero at one interior sample t_j only has the transform
    dt W_L(t_j / T_W) e^{i omega t_j} delta J / k0 (trapezoid weight 1), which reads W_L at
    x = 1/4, 1/2, 3/4 (0.84375, 0.5, 0.15625); beyond T_W the window is 0."""
    dt, TW, k0 = 0.5, 100.0, 1e-3
    t = np.arange(0.0, 150.0 + 1e-9, dt)
    om = np.array([0.0, 0.7])
    for x, want in ((0.25, 0.84375), (0.5, 0.5), (0.75, 0.15625), (1.2, 0.0)):
        j = int(round(x * TW / dt))
        dj = np.zeros_like(t)
        dj[j] = 2e-5
        sig = spectra.conductivity(t, dj, k0, om, window_T=TW)
        np.testing.assert_allclose(sig, dt * want * np.exp(1j * om * t[j]) * 2e-5 / k0, rtol=1e-13, atol=1e-18)


def test_conductivity_wl_window_constant_current():
    """Constant delta J = n k0 under W_L: sigma(omega) = n T int_0^1 p(x) e^{i Omega x} dx with
    p = 1 - 3x^2 + 2x^3 and Omega = omega T.  Repeated integration by parts (p(1) = 0,
    p'(0) = p'(1) = 0, p''(0) = -6, p''(1) = 6, p''' = 12) gives
    -1/z + 6 (e^z + 1)/z^3 - 12 (e^z - 1)/z^4 with z = i Omega; at omega = 0 it is n T / 2.
    The trapezoid rule (Sec. III.A transform on t_n = n dt, weight 1/2 at t_0) adds its
    Euler-Maclaurin term dt^2/12 (f'(end) - f'(0)) = -i omega n dt^2 / 12 (the integrand
    e^{i omega t} W_L has slope i omega n at t = 0 and vanishes with its slope at T_W)."""
    n, k0, TW, dt = 0.0296, 1e-3, 400.0, 0.02
    t = np.arange(0.0, 600.0 + 1e-9, dt)
    om = np.array([0.05, 0.2, 0.6, 1.3])
    sig = spectra.conductivity(t, np.full_like(t, n * k0), k0, om, window_T=TW)
    z = 1j * om * TW
    exact = n * TW * (-1 / z + 6 * (np.exp(z) + 1) / z ** 3 - 12 * (np.exp(z) - 1) / z ** 4)
    want = exact - 1j * om * n * dt ** 2 / 12
    np.testing.assert_allclose(sig, want, rtol=1e-9, atol=1e-12 * np.max(np.abs(want)))
    sig0 = spectra.conductivity(t, np.full_like(t, n * k0), k0, np.array([0.0]), window_T=TW)
    np.testing.assert_allclose(sig0.real, n * TW / 2, rtol=1e-7)
