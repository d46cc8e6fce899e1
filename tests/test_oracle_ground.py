"""Oracle pins for the ground-state preparation by imaginary-time propagation:
the Taylor-4 step of exp(-tau h) on eigenvectors and against the exact
exponential, the Cholesky orthonormalisation, free electrons against the
closed-form finite-difference spectrum, and the converged self-consistent
result against the independent dense-diagonalisation route."""
import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import ground as G
from oracle.hamiltonian import System
from oracle.propagate import density


def _species():
    return W.draw_species(np.random.default_rng(3))


def _free(grid, nb, kf):
    lat, _ = W.CELLS["diamond8"]()
    inst = W.Instance(cell="diamond8", lattice=lat, grid=grid, atom_frac=np.zeros((0, 3)),
                      atom_species=np.zeros(0, int), species=[], kspec=W.KSpec((1, 1, 1)), n_bands=nb)
    return System(inst, k_frac=np.array([kf]))


def test_itime_step_on_eigenvectors_and_against_expm():
    """On an eigenvector of h the step multiplies by sum_{m<=4} (-tau e)^m / m!; on a
    general vector it differs from exp(-tau H) u by at most the Taylor remainder
    (tau |e|_max)^5 / 5! |u| (H Hermitian)."""
    inst = W.make_instance("diamond8", (4, 4, 4), 2, [_species()], W.KSpec((1, 1, 1)))
    s = System(inst)
    v = np.random.default_rng(1).uniform(-0.3, 0.0, s.cell.shape)
    kap = s.k_cart[0] + np.array([0.05, -0.02, 0.01])
    H = s.dense_h(kap, v)
    H = 0.5 * (H + H.conj().T)
    e, X = np.linalg.eigh(H)
    tau = 0.3
    for j in (0, 17, 63):
        u = X[:, j].reshape((1,) + s.cell.shape)
        got = G.imaginary_time_step(s, kap, v, u, tau)
        x = -tau * e[j]
        f = 1 + x + x ** 2 / 2 + x ** 3 / 6 + x ** 4 / 24
        np.testing.assert_allclose(got, f * u, rtol=0, atol=1e-12)
    u = np.random.default_rng(2).standard_normal((1,) + s.cell.shape) + 0j
    got = G.imaginary_time_step(s, kap, v, u, tau).ravel()
    ref = scipy.linalg.expm(-tau * H) @ u.ravel()
    bound = (tau * np.max(np.abs(e))) ** 5 / 120 * np.linalg.norm(u)
    err = np.linalg.norm(got - ref)
    assert err <= bound * 1.0001 and err > 1e-6 * bound  # a real remainder, inside its bound


def test_orthonormalise_cholesky_properties():
    rng = np.random.default_rng(4)
    u = rng.standard_normal((5, 4, 4, 4)) + 1j * rng.standard_normal((5, 4, 4, 4))
    dV = 0.37
    q = G.orthonormalise(u, dV)
    Q = q.reshape(5, -1).T
    U = u.reshape(5, -1).T
    np.testing.assert_allclose(Q.conj().T @ Q * dV, np.eye(5), atol=1e-13)
    # same span, Gram-Schmidt order: Q^H U dV = L^H is upper triangular, positive diagonal
    R = Q.conj().T @ U * dV
    assert np.max(np.abs(np.tril(R, -1))) < 1e-12
    assert np.all(np.real(np.diag(R)) > 0) and np.max(np.abs(np.imag(np.diag(R)))) < 1e-12
    np.testing.assert_allclose(Q @ R, U, atol=1e-12)


def test_itime_free_electrons_closed_form():
    """No atoms, no Hxc: the iteration converges to the span of the lowest plane waves,
    whose band-energy sum is that of the lowest finite-difference symbols (sorted from
    the closed form of the stencil, computed here from trigonometry)."""
    grid = (6, 6, 6)
    kf = np.array([0.11, 0.23, -0.17])
    nb = 4
    s = _free(grid, nb, kf)
    N = np.array(grid)
    H = s.cell.A / N[:, None]
    E = np.linalg.solve(H, np.eye(3)).T
    kap = s.k_cart[0]
    sym = []
    for m in np.ndindex(*grid):
        m = np.array(m) - (np.array(m) > N // 2) * N
        th = 2 * np.pi * m / N
        sd = (8 * np.sin(th) - np.sin(2 * th)) / 6
        lam = (32 * np.cos(th) - 2 * np.cos(2 * th) - 30) / 12
        eps = 0.5 * kap @ kap
        for d in range(3):
            eps += -0.5 * (E[d] @ E[d]) * lam[d] + (kap @ E[d]) * sd[d]
            for e in range(3):
                if e != d:
                    eps += 0.5 * (E[d] @ E[e]) * sd[d] * sd[e]
        sym.append(eps)
    sym = np.sort(sym)
    assert sym[nb] - sym[nb - 1] > 0.05  # a gap above the filled span
    u0 = W.random_orbitals(6, 1, nb, grid, s.cell.omega)
    u, rho, v, res = G.imaginary_time_scf(s, u0, 0.9, 1.0, 300, hxc_mode="none")
    e_sum = G.subspace_energy(s, v, u)
    assert abs(e_sum - np.sum(sym[:nb])) < 1e-10
    assert res[-1] < 1e-8 and res[-1] < 1e-6 * res[0]


def test_itime_scf_equals_dense_diagonalisation():
    inst = W.make_instance("diamond8", (6, 6, 6), 4, [_species()], W.KSpec((2, 1, 1)))
    s = System(inst)
    u_d, eps, v_d, r_d = G.scf(s, tol=1e-12)
    rho_d = density(s, u_d)
    u0 = W.random_orbitals(5, s.nk, s.nb, inst.grid, inst.omega)
    u, rho, v, res = G.imaginary_time_scf(s, u0, 1.0, 0.6, 150)
    assert np.sum(np.abs(rho - rho_d)) * s.cell.dV < 1e-10
    assert np.max(np.abs(v - v_d)) < 1e-9
    assert abs(G.subspace_energy(s, v, u) - np.mean(np.sum(eps, axis=1))) < 1e-10
    assert res[-1] < 1e-12 and res[0] > 1e-3
