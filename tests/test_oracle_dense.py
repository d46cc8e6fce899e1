"""Oracle pins by brute force on a 6^3 grid (all 8 atoms of the diamond cell).

The dense h_kappa is assembled here a second way -- Kronecker products of 1-D
circulant difference matrices, an explicit loop over grid points and atom
images for the projectors -- and compared with the oracle's stencil
application.  Then the Taylor-4 step is checked against the dense Taylor
polynomial and against the exact exponential expm(-i H dt) within the Taylor
remainder bound, and the per-step norm of eigenstates against the closed form
|T4(-i x)|^2 = 1 - x^6/72 + x^8/576 (Eq. (1) propagated by a 4th-order
expansion).
"""
import itertools

import numpy as np
import pytest
import scipy.linalg

import workloads as W
from oracle import propagate as P
from oracle.hamiltonian import System


def small_system(grid=(6, 6, 6), nk=(1, 1, 1), nb=4, seed=11):
    sp = W.draw_species(np.random.default_rng(seed))
    inst = W.make_instance("diamond8", grid, nb, [sp], W.KSpec(nk))
    return System(inst), sp


def circulant(n, coef):
    M = np.zeros((n, n))
    for off, c in coef.items():
        for i in range(n):
            M[i, (i + off) % n] += c
    return M


def dense_by_kron(sys, sp, kappa, v):
    N1, N2, N3 = sys.cell.N
    a = sys.cell.A[0, 0]
    h = a / np.array([N1, N2, N3])
    D1 = {1: 2 / 3, -1: -2 / 3, 2: -1 / 12, -2: 1 / 12}
    D2 = {0: -2.5, 1: 4 / 3, -1: 4 / 3, 2: -1 / 12, -2: -1 / 12}
    I = [np.eye(N1), np.eye(N2), np.eye(N3)]

    def along(d, M):  # flat index p = i1 + N1 (i2 + N2 i3)
        mats = [I[2], I[1], I[0]]
        mats[2 - d] = M
        return np.kron(np.kron(mats[0], mats[1]), mats[2])

    ng = N1 * N2 * N3
    H = 0.5 * (kappa @ kappa) * np.eye(ng, dtype=complex)
    for d, n in enumerate((N1, N2, N3)):
        H += -0.5 / h[d] ** 2 * along(d, circulant(n, D2))
        H += -1j * kappa[d] / h[d] * along(d, circulant(n, D1))
    H += np.diag(v.ravel())
    # projectors by explicit loops
    rc, Rc = sp.rc, sp.Rc
    ns = (np.pi ** 1.5 * rc ** 3) ** -0.5
    npn = (np.pi ** 1.5 * rc ** 5 / 2) ** -0.5
    gcut = np.exp(-Rc ** 2 / (2 * rc ** 2))
    dV = sys.cell.omega / ng
    for tau in sys.cell.atom_frac @ sys.cell.A:
        P = np.zeros((4, ng), dtype=complex)
        for i3, i2, i1 in itertools.product(range(N3), range(N2), range(N1)):
            r = np.array([i1 * h[0], i2 * h[1], i3 * h[2]])
            x = r - tau
            x = x - a * np.round(x / a)  # minimum image in the cubic cell
            dist2 = x @ x
            if dist2 >= Rc ** 2:
                continue
            gval = np.exp(-dist2 / (2 * rc ** 2)) - gcut
            p = i1 + N1 * (i2 + N2 * i3)
            ph = np.exp(-1j * kappa @ x)
            P[:, p] = ph * gval * np.array([ns, npn * x[0], npn * x[1], npn * x[2]])
        E = np.array([sp.Es, sp.Ep, sp.Ep, sp.Ep])
        H += dV * (P.T * E) @ P.conj()
    return H


def test_dense_matches_stencil():
    sys, sp = small_system()
    kappa = np.array([0.13, -0.07, 0.21])
    v = np.random.default_rng(3).uniform(-1, 0, sys.cell.shape)
    Hs = sys.dense_h(kappa, v)
    Hk = dense_by_kron(sys, sp, kappa, sys.v_loc + v)
    assert np.max(np.abs(Hs - Hs.conj().T)) < 1e-14 * np.max(np.abs(Hs))
    np.testing.assert_allclose(Hs, Hk, rtol=0, atol=1e-13)


def test_taylor_vs_dense_and_expm():
    sys, sp = small_system()
    kappa = np.array([0.05, 0.2, -0.1])
    v = np.random.default_rng(4).uniform(-1, 0, sys.cell.shape)
    H = sys.dense_h(kappa, v)
    u = W.random_orbitals(5, 1, 4, sys.cell.N, sys.cell.omega)[0]
    dt = 0.02
    got = P.taylor_step(sys, kappa, v, u, dt)
    flat = u.reshape(4, -1).T
    X = -1j * dt * H
    T4 = np.eye(len(H)) + X + X @ X / 2 + X @ X @ X / 6 + X @ X @ X @ X / 24
    want = (T4 @ flat).T.reshape(u.shape)
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-13 * np.max(np.abs(u)))
    exact = (scipy.linalg.expm(X) @ flat).T.reshape(u.shape)
    hn = np.linalg.norm(H, 2) * dt
    bound = hn ** 5 / 120 * np.max(np.linalg.norm(flat, axis=0))
    assert np.max(np.linalg.norm((got - exact).reshape(4, -1), axis=1)) <= bound


def test_norm_of_eigenstates():
    sys, sp = small_system()
    kappa = np.zeros(3)
    v = np.zeros(sys.cell.shape)
    H = sys.dense_h(kappa, v)
    e, vec = np.linalg.eigh(H)
    dt = 0.05
    for j in (0, len(e) // 2, len(e) - 1):
        u = (vec[:, j] / np.sqrt(sys.cell.dV)).reshape((1,) + sys.cell.shape)
        n0 = P.norms(sys, u)[0]
        assert abs(n0 - 1.0) < 1e-12  # eigh's unit vectors scaled by 1/sqrt(dV)
        for _ in range(10):
            u = P.taylor_step(sys, kappa, v, u, dt)
        x = e[j] * dt
        want = (1 - x ** 6 / 72 + x ** 8 / 576) ** 10 * n0
        assert abs(P.norms(sys, u)[0] - want) < 1e-12
