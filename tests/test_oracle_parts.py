"""Oracle pins of the parts: k-point sets, Hartree/LDA, pseudopotentials and
spectra, each against closed forms or textbook routines."""
from fractions import Fraction
import itertools

import numpy as np
import pytest
from scipy import integrate

import workloads as W
from oracle import hxc, kpoints, spectra
from oracle.cell import Cell
from oracle.pseudo import Projectors, local_potential


# ---------------------------------------------------------------- k-points
def test_mp_small_closed_form():
    k = kpoints.monkhorst_pack((2, 1, 3))
    assert k.shape == (6, 3)
    assert set(k[:, 0].tolist()) == {-0.25, 0.25}
    np.testing.assert_allclose(sorted(set(k[:, 2].tolist())), [-1 / 3, 0.0, 1 / 3], atol=1e-16)
    np.testing.assert_array_equal(k[:, 1], 0.0)
    np.testing.assert_array_equal(k[0], [-0.25, 0.0, -1 / 3])  # n1 fastest


@pytest.mark.parametrize("N,M", [(8, 4), (4, 2), (2, 2), (4, 4)])
def test_shift_union_is_dense_grid(N, M):
    dense = set(kpoints.mp_fractions((N * M,) * 3))
    union = []
    for j in itertools.product(range(M), repeat=3):
        q = [kpoints.uniform_shift_fraction(M, jj) for jj in j]
        assert all(0 < x < 1 for x in q)
        union += kpoints.mp_fractions((N,) * 3, q)
    assert len(union) == len(dense) and set(union) == dense
    # the float generator is exact for these dyadic values
    for j in [(0, 1, M - 1), (M - 1, 0, 0)]:
        ks = W.KSpec((N, N, N), (M, M, M), j)
        fl = kpoints.kset(ks)
        q = [kpoints.uniform_shift_fraction(M, jj) for jj in j]
        ex = sorted(kpoints.mp_fractions((N,) * 3, q))
        assert sorted(map(tuple, fl.tolist())) == [tuple(float(x) for x in p) for p in ex]


def test_halton_textbook_values():
    h = kpoints.halton(4)
    np.testing.assert_allclose(h[:3, 0], [1 / 2, 1 / 4, 3 / 4])
    np.testing.assert_allclose(h[:3, 1], [1 / 3, 2 / 3, 1 / 9])
    np.testing.assert_allclose(h[:4, 2], [1 / 5, 2 / 5, 3 / 5, 4 / 5])
    assert np.all((h > 0) & (h < 1))


def test_wrap_half():
    np.testing.assert_array_equal(kpoints.wrap_half([0.5, -0.5, 0.625, -0.625, 1.0]),
                                  [0.5, 0.5, -0.375, 0.375, 0.0])


# ---------------------------------------------------------------- Hartree / LDA
def test_poisson_cosine_closed_form():
    lat, _ = W.diamond8()
    c = Cell(lat, (12, 12, 12))
    r = c.positions()
    G = np.array([1, 2, -1]) @ c.B
    rho = 0.03 + 0.01 * np.cos(r @ G)
    v = hxc.hartree(c, rho)
    np.testing.assert_allclose(v, 4 * np.pi * 0.01 * np.cos(r @ G) / (G @ G), atol=1e-14)


def test_poisson_fft_vs_direct_dft_nonorthogonal():
    lat, _ = W.fcc2()
    c = Cell(lat, (4, 4, 4))
    rho = np.random.default_rng(2).uniform(0, 1, c.shape)
    # direct DFT sum with the same conventions
    N = c.N
    v = np.zeros(c.shape)
    for m1, m2, m3 in itertools.product(*[range(-n // 2, n - n // 2) for n in N]):
        if (m1, m2, m3) == (0, 0, 0) or -N[0] // 2 in (m1,) or -N[1] // 2 == m2 or -N[2] // 2 == m3:
            continue
        G = m1 * c.B[0] + m2 * c.B[1] + m3 * c.B[2]
        ph = np.exp(-2j * np.pi * (m1 * np.arange(N[0])[None, None, :] / N[0]
                                   + m2 * np.arange(N[1])[None, :, None] / N[1]
                                   + m3 * np.arange(N[2])[:, None, None] / N[2]))
        rg = np.sum(rho * ph)
        v = v + np.real(4 * np.pi * rg / (G @ G) * np.conj(ph)) / c.ng
    np.testing.assert_allclose(hxc.hartree(c, rho), v, atol=1e-13)


def test_slater_textbook_constant():
    rs = np.array([0.5, 1.0, 2.0, 5.0])
    rho = 3 / (4 * np.pi * rs ** 3)
    # eps_x = -0.458165 / r_s Ha and v_x = 4/3 eps_x
    np.testing.assert_allclose(hxc.slater_exchange(rho) * rs, -4 / 3 * 0.4581652933, rtol=1e-9)


def test_pz81_potential_is_derivative():
    for rs in (0.3, 0.8, 1.5, 4.0, 10.0):
        rho = 3 / (4 * np.pi * rs ** 3)
        h = rho * 1e-5

        def e(r):
            return r * hxc.pz81_eps(np.cbrt(3 / (4 * np.pi * r)))

        num = (e(rho + h) - e(rho - h)) / (2 * h)
        assert abs(hxc.correlation(np.array([rho]))[0] - num) < 1e-8


def test_pz81_limits():
    # high-density coefficient A = (1 - ln 2) / pi^2 (Gell-Mann--Brueckner)
    assert abs(hxc.PZ_A - (1 - np.log(2)) / np.pi ** 2) < 2e-5
    # the two branches meet at r_s = 1 (energy and potential)
    lo, hi = hxc.pz81_eps(1 - 1e-12), hxc.pz81_eps(1 + 1e-12)
    assert abs(lo - hi) < 1e-4
    assert abs(hxc.pz81_v(1 - 1e-12) - hxc.pz81_v(1 + 1e-12)) < 2e-4
    assert hxc.correlation(np.array([0.0, 1e-31]))[0] == 0.0


# ---------------------------------------------------------------- pseudopotential
def test_local_potential_single_gaussian():
    a = 30.0
    c = Cell(np.eye(3) * a, (16, 16, 16), atom_frac=[[0.5, 0.5, 0.5]],
             species=[W.Species(D=-2.0, w=1.0)])
    v = local_potential(c)
    r = c.positions()
    d2 = np.sum((r - 15.0) ** 2, axis=-1)
    np.testing.assert_allclose(v, -2.0 * np.exp(-d2 / 2.0), atol=1e-40)


def test_local_potential_periodic_images():
    lat, frac = W.diamond8()
    sp = W.Species(D=-1.5, w=1.3)
    c = Cell(lat, (6, 6, 6), frac, np.zeros(8, int), [sp])
    v = local_potential(c)
    # brute force over a wide image range at one grid point
    r0 = c.positions()[1, 2, 3]
    tot = 0.0
    for n in itertools.product(range(-4, 5), repeat=3):
        for t in c.tau:
            d = r0 - t - np.array(n) @ c.A
            dd = d @ d
            if dd < (15 * sp.w) ** 2:
                tot += sp.D * np.exp(-dd / (2 * sp.w ** 2))
    assert abs(v[1, 2, 3] - tot) < 1e-13


def test_projector_normalisation_fine_grid():
    """sum_r |f_lm|^2 dV tends to the radial integral of the shifted-cut Gaussian."""
    sp = W.Species(D=-1.0, w=1.0)
    a = 9.6
    c = Cell(np.eye(3) * a, (48, 48, 48), atom_frac=[[0.5, 0.5, 0.5]], species=[sp])
    pr = Projectors(c)
    f = pr.atoms[0]["f"]
    rc, Rc = sp.rc, sp.Rc
    gc = np.exp(-Rc ** 2 / (2 * rc ** 2))
    ns2 = 1 / (np.pi ** 1.5 * rc ** 3)
    np2 = 2 / (np.pi ** 1.5 * rc ** 5)
    s_int = integrate.quad(lambda r: 4 * np.pi * r * r * ns2 * (np.exp(-r * r / (2 * rc * rc)) - gc) ** 2, 0, Rc)[0]
    p_int = integrate.quad(lambda r: 4 * np.pi / 3 * r ** 4 * np2 * (np.exp(-r * r / (2 * rc * rc)) - gc) ** 2, 0, Rc)[0]
    assert 0.9 < s_int < 1.0
    assert abs(np.sum(f[0] ** 2) * c.dV - s_int) < 1e-4
    for i in range(1, 4):
        assert abs(np.sum(f[i] ** 2) * c.dV - p_int) < 1e-4
    # s and p are orthogonal
    assert abs(np.sum(f[0] * f[1]) * c.dV) < 1e-10
    # uncut Gaussians would be normalised: s_int -> 1 as Rc -> infinity
    full = integrate.quad(lambda r: 4 * np.pi * r * r * ns2 * np.exp(-r * r / rc ** 2), 0, 50)[0]
    assert abs(full - 1) < 1e-10


# ---------------------------------------------------------------- spectra
def test_drude_closed_form():
    """Free electrons: delta J(t) = n k0 for t >= 0, so with damping gamma,
    sigma(omega) = n / (gamma - i omega) and eps = 1 - 4 pi n / (omega (omega + i gamma))."""
    n, k0, gamma, dt = 0.0296, 1e-3, 0.005, 0.02
    t = np.arange(0, 4000.0, dt)
    om = np.array([0.1, 0.3, 0.6, 1.0])
    sig = spectra.conductivity(t, np.full_like(t, n * k0), k0, om, gamma)
    np.testing.assert_allclose(sig, n / (gamma - 1j * om), rtol=1e-4)
    eps = spectra.dielectric(sig, om)
    drude = 4 * np.pi * n / (om * (om + 1j * gamma))
    np.testing.assert_allclose(eps, 1 - drude, rtol=0, atol=1e-4 * np.max(np.abs(drude)))


def test_fourier_of_gaussian():
    t = np.arange(0, 200.0, 0.02)
    s, t0 = 7.0, 100.0
    f = np.exp(-(t - t0) ** 2 / (2 * s * s))
    om = np.array([0.0, 0.1, 0.2, 0.35])
    want = s * np.sqrt(2 * np.pi) * np.exp(1j * om * t0) * np.exp(-om ** 2 * s * s / 2)
    np.testing.assert_allclose(spectra.fourier(t, f, om), want, atol=1e-10)


def test_hhg_window_and_peak():
    T = 1000.0
    t = np.arange(0, T, 0.05)
    w = spectra.hhg_window(t, T)
    assert abs(spectra.hhg_window(np.array([T / 2]), T)[0] - 1) < 1e-15
    assert w[0] == 0.0
    om0 = 0.2
    om = np.linspace(0.05, 0.8, 76)
    I = spectra.hhg_spectrum(t, np.sin(om0 * t), T, om)
    assert abs(om[np.argmax(I)] - om0) < 0.011


def test_standard_error():
    x = np.array([[1.0], [2.0], [3.0], [4.0]])
    assert abs(spectra.standard_error(x)[0] - np.std([1, 2, 3, 4], ddof=1) / 2) < 1e-15


@pytest.mark.parametrize("axis,base,N", [(0, 2, 3), (1, 3, 2), (2, 5, 4)])
def test_halton_two_step_average_closed_form(axis, base, N):
    """Two-step average (Eq. (9)) of f(k) = cos(2 pi N k_d) over Halton-shifted MP grids
    (Eq. (10), Sec. II.B).  On every shifted grid f = (-1)^(N+1) cos(2 pi q_m) (the
    N-point grid aliases this frequency), and the radical inverses of m = 0..B^j - 1 are
    the points i / B^j, whose cosines sum to 0; without m = 0 the sum over
    m = 1..B^j - 1 is -1.  So the average over N_H = B^j - 1 shifts is
    (-1)^N / (B^j - 1)."""
    coarse = [1, 1, 1]
    coarse[axis] = N
    for j in (1, 2):
        n_h = base ** j - 1
        tot = 0.0
        for m in range(1, n_h + 1):
            k = kpoints.kset(W.KSpec(tuple(coarse), halton_index=m))
            tot += np.mean(np.cos(2 * np.pi * N * k[:, axis]))
        assert abs(tot / n_h - (-1) ** N / n_h) < 1e-12


def test_explicit_shift_is_eq10():
    q = (0.3, 0.05, 0.9)
    k = kpoints.kset(W.KSpec((2, 3, 1), shift_q=q))
    ref = [[(2 * n1 - 3 + 2 * q[0]) / 4, (2 * n2 - 4 + 2 * q[1]) / 6, (2 - 2 + 2 * q[2]) / 2]
           for n2 in (1, 2, 3) for n1 in (1, 2)]
    np.testing.assert_allclose(k, kpoints.wrap_half(ref), rtol=0, atol=1e-15)


def test_nh_convergence_scaled_copies():
    """delta J_m = c_m g(t): eps is affine in delta J, so eps(N_H) - 1 = mean(c_1..c_N)
    (eps_g - 1) and the standard error of its real and imaginary parts is
    std(c_1..c_N) / sqrt(N) |Re, Im (eps_g - 1)|."""
    t = np.arange(0.0, 100.0, 0.05)
    g = 1e-5 * np.exp(-0.01 * t) * np.sin(0.3 * t)
    c = np.array([1.0, 3.0, -2.0, 0.5, 4.0, 2.5])
    om = np.linspace(0.1, 1.0, 7)
    eg = spectra.dielectric(spectra.conductivity(t, g, 1e-3, om), om) - 1.0
    rows = spectra.nh_convergence(t, c[:, None] * g[None, :], 1e-3, om, [1, 2, 6])
    for n, eps, sem in rows:
        np.testing.assert_allclose(eps - 1.0, c[:n].mean() * eg, rtol=1e-11, atol=1e-14)
        s = c[:n].std(ddof=1) / np.sqrt(n) if n > 1 else 0.0
        np.testing.assert_allclose(sem.real, s * np.abs(eg.real), rtol=1e-10, atol=1e-14)
        np.testing.assert_allclose(sem.imag, s * np.abs(eg.imag), rtol=1e-10, atol=1e-14)
