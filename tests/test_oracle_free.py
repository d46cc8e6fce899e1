"""Oracle pins: free electrons (v_ion = v_Hxc = 0) against closed forms.

A grid plane wave e^{i G.r} is an exact eigenvector of the finite-difference
kinetic operator [p + kappa]^2/2 of Eq. (2).  With theta_d the phase advance per
grid step along a_d, D1 -> i s(theta), D2 -> lambda(theta) with
s = (8 sin t - sin 2t)/6, lambda = (32 cos t - 2 cos 2t - 30)/12, so the
symbol is computed here from trigonometry alone; one Taylor-4 step multiplies
the wave by T4(-i eps dt) = sum_{m<=4} (-i eps dt)^m / m!, and the current
(Eqs. (5)-(6)) of the G = 0 state is -n (k + A).
"""
import numpy as np
import pytest

import workloads as W
from oracle import cell as C
from oracle import propagate as P
from oracle.hamiltonian import System


def free_instance(cellname, grid, nb=1, kspec=((1, 1, 1),)):
    lat, _ = W.CELLS[cellname]()
    return W.Instance(cell=cellname, lattice=lat, grid=grid, atom_frac=np.zeros((0, 3)),
                      atom_species=np.zeros(0, int), species=[], kspec=W.KSpec(*kspec),
                      n_bands=nb)


def plane_wave(cell, m):
    r = cell.positions()
    G = np.asarray(m, float) @ cell.B
    return np.exp(1j * r @ G) / np.sqrt(cell.omega)


def fd_symbol(lattice, N, kappa, m):
    """Symbol of the FD operator for the wave with integer frequencies m.

    Uses the dual basis of the grid steps h_d = a_d / N_d (so that
    grad = sum_d e_d d/ds_d with e_d . h_e = delta_de), built by solving the
    linear system rather than from reciprocal vectors.
    """
    H = np.asarray(lattice, float) / np.asarray(N, float)[:, None]  # rows h_d
    E = np.linalg.solve(H, np.eye(3)).T  # rows e_d, E @ H.T = I
    th = 2 * np.pi * np.asarray(m, float) / np.asarray(N, float)
    s = (8 * np.sin(th) - np.sin(2 * th)) / 6
    lam = (32 * np.cos(th) - 2 * np.cos(2 * th) - 30) / 12
    eps = 0.5 * kappa @ kappa
    for d in range(3):
        eps += -0.5 * (E[d] @ E[d]) * lam[d] + (kappa @ E[d]) * s[d]
        for e in range(3):
            if e != d:
                eps += 0.5 * (E[d] @ E[e]) * s[d] * s[e]
    return eps


@pytest.mark.parametrize("cellname,grid", [("diamond8", (8, 8, 8)), ("fcc2", (8, 8, 8)),
                                            ("diamond8", (6, 8, 10))])
def test_plane_wave_symbol(cellname, grid):
    inst = free_instance(cellname, grid)
    s = System(inst)
    rng = np.random.default_rng(0)
    for trial in range(4):
        m = rng.integers(-3, 4, size=3)
        kappa = rng.uniform(-0.3, 0.3, size=3)
        u = plane_wave(s.cell, m)
        hu = s.apply_h(kappa, 0.0, u)
        eps = fd_symbol(s.cell.A, s.cell.N, kappa, m)
        np.testing.assert_allclose(hu, eps * u, rtol=0, atol=1e-12 * max(1, abs(eps)) / np.sqrt(s.cell.omega))


def test_fd_continuum_limit_nonorthogonal():
    """As h -> 0 the FD symbol tends to |kappa + G|^2 / 2 with 4th-order error."""
    lat, _ = W.fcc2()
    kappa = np.array([0.11, -0.07, 0.05])
    m = np.array([1, -1, 2])
    B = 2 * np.pi * np.linalg.inv(lat).T
    exact = 0.5 * np.sum((kappa + m @ B) ** 2)
    errs = []
    for n in (16, 32, 64):
        errs.append(abs(fd_symbol(lat, (n, n, n), kappa, m) - exact))
        inst = free_instance("fcc2", (n, n, n))
        if n == 16:
            s = System(inst)
            u = plane_wave(s.cell, m)
            hu = s.apply_h(kappa, 0.0, u)
            ratio = np.vdot(u, hu) / np.vdot(u, u)
            assert abs(ratio - fd_symbol(lat, (n, n, n), kappa, m)) < 1e-12
    # halving h divides the error by ~16
    assert 12 < errs[0] / errs[1] < 20 and 12 < errs[1] / errs[2] < 20


def test_fd_order_of_accuracy():
    """D1 and D2 of a smooth periodic function converge at 4th order."""
    errs1, errs2 = [], []
    for n in (16, 32):
        x = np.arange(n) * 2 * np.pi / n
        f = np.exp(np.sin(x))[None, None, :]
        d1 = C.D1(f, 0)[0, 0] * n / (2 * np.pi)
        d2 = C.D2(f, 0)[0, 0] * (n / (2 * np.pi)) ** 2
        errs1.append(np.max(np.abs(d1 - np.cos(x) * f[0, 0])))
        errs2.append(np.max(np.abs(d2 - (np.cos(x) ** 2 - np.sin(x)) * f[0, 0])))
    assert 12 < errs1[0] / errs1[1] < 20
    assert 12 < errs2[0] / errs2[1] < 20


def test_taylor_step_closed_form():
    """u -> T4(-i eps dt) u exactly for an eigen-plane-wave (no Hxc)."""
    inst = free_instance("diamond8", (8, 8, 8))
    s = System(inst)
    kappa = np.array([0.13, -0.07, 0.21])
    m = (1, 2, -1)
    u = plane_wave(s.cell, m)[None]
    eps = fd_symbol(s.cell.A, s.cell.N, kappa, m)
    for dt in (0.02, 0.05):
        z = -1j * eps * dt
        t4 = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
        out = P.taylor_step(s, kappa, 0.0, u, dt)
        np.testing.assert_allclose(out, t4 * u, rtol=0, atol=1e-14)


def test_free_electron_current_and_kick():
    """G = 0 orbitals at every k: J = -n (k + A); after a kick delta J = n k0."""
    inst = free_instance("diamond8", (8, 8, 8), nb=1, kspec=((2, 2, 2),))
    s = System(inst)
    u = np.stack([plane_wave(s.cell, (0, 0, 0))[None] for _ in range(s.nk)])
    n = 2.0 / s.cell.omega  # one doubly occupied band
    A = np.array([-1e-3, 0.0, 0.0])
    J = P.current(s, A, u)
    kbar = np.mean(s.k_cart, axis=0)
    np.testing.assert_allclose(J, -n * (kbar + A), atol=1e-18)
    run = P.Run(s, u, 0.02, "none")
    dj = run.run(np.array([[A, A]] * 3)) - run.J_pre
    np.testing.assert_allclose(dj[:, 0], n * 1e-3, rtol=1e-12)
    np.testing.assert_allclose(dj[:, 1:], 0.0, atol=1e-18)


def test_density_counts_electrons():
    """sum_r rho dV = sum_b f_b for orthonormal orbitals (Eq. (3))."""
    import workloads as Wl
    sp = Wl.draw_species(np.random.default_rng(1))
    inst = Wl.make_instance("diamond8", (6, 6, 6), 5, [sp], Wl.KSpec((2, 1, 1)))
    s = System(inst)
    u = Wl.random_orbitals(3, s.nk, 5, inst.grid, inst.omega)
    assert abs(np.sum(P.density(s, u)) * s.cell.dV - 10.0) < 1e-12


def test_uniform_density_scf_phase():
    """Uniform rho: v_H = 0 and v_xc is the constant LDA value, which simply
    adds to the plane-wave eigenvalue in every Taylor step."""
    from oracle import hxc
    inst = free_instance("diamond8", (8, 8, 8), nb=1, kspec=((1, 1, 1),))
    s = System(inst)
    m = (0, 0, 0)
    u = plane_wave(s.cell, m)[None, None]
    n = 2.0 / s.cell.omega
    vxc = hxc.slater_exchange(np.array([n]))[0] + hxc.correlation(np.array([n]))[0]
    kap = np.array([0.0, 0.0, 0.0])
    A = np.array([0.02, 0.0, 0.0])
    run = P.Run(s, u, 0.02, "scf")
    np.testing.assert_allclose(run.v_hxc, vxc, atol=1e-14)
    run.run(np.array([[A, A]] * 2))
    eps = fd_symbol(s.cell.A, s.cell.N, kap + A, m) + vxc
    z = -1j * eps * 0.02
    t4 = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    np.testing.assert_allclose(run.u, t4 ** 2 * u, atol=1e-14)
