"""Oracle pins by invariants of the method.

* Current operator (Eqs. (5)-(6)): pi = (1/i)[r, h] = d h_kappa / d kappa, so the
  per-k band sum of <u|pi|u> equals the kappa-derivative of <u|h_kappa|u>
  (central difference; exact for the quadratic kinetic part).
* Time reversal: conj(h_kappa) = h_{-kappa}, so propagating (conj u, -kappa,
  -dt, -A) gives conj of the orbitals of (u, kappa, dt, A), the same density and
  the negated current; with a k-set closed under k -> -k and u_{-k} = conj u_k,
  J(t < 0) vanishes.
* Two-step decomposition (Sec. II.B): with the Hxc potential frozen the
  k-points decouple, so 2^3 uniform shifts of a 2^3 coarse grid run as 8
  independent simulations reproduce the direct 4^3 Monkhorst-Pack run
  orbital by orbital, and the shift-averaged current equals the direct one.
"""
import numpy as np

import workloads as W
from oracle import kpoints
from oracle import propagate as P
from oracle.hamiltonian import System
from oracle.hxc import v_hxc as hxc_potential


def system(grid=(6, 6, 6), kspec=W.KSpec((1, 1, 1)), nb=3, seed=21, k_frac=None):
    sp = W.draw_species(np.random.default_rng(seed))
    inst = W.make_instance("diamond8", grid, nb, [sp], kspec)
    return System(inst, k_frac=k_frac)


def test_current_is_energy_derivative():
    s = system(k_frac=np.array([[0.1, -0.2, 0.3]]))
    u = W.random_orbitals(8, 1, s.nb, s.cell.N, s.cell.omega)
    v = np.random.default_rng(1).uniform(-0.5, 0.0, s.cell.shape)
    kappa0 = s.k_cart[0] + np.array([0.01, -0.02, 0.005])

    def energy(kap):
        hu = s.apply_h(kap, v, u[0])
        return np.sum(s.occ * np.real(np.sum(np.conj(u[0]) * hu, axis=(1, 2, 3)))) * s.cell.dV

    Jk = P.current_k(s, kappa0, u[0])
    for j in range(3):
        dk = np.zeros(3)
        dk[j] = 1e-4
        num = (energy(kappa0 + dk) - energy(kappa0 - dk)) / 2e-4
        assert abs(num - Jk[j]) < 1e-8 * max(1.0, abs(Jk[j]))


def test_current_without_projectors_changes():
    """The non-local term is not negligible here, so the pin above covers it."""
    s = system(k_frac=np.array([[0.1, -0.2, 0.3]]))
    u = W.random_orbitals(8, 1, s.nb, s.cell.N, s.cell.omega)
    full = P.current_k(s, s.k_cart[0], u[0])
    s.proj.atoms = []
    local = P.current_k(s, s.k_cart[0], u[0])
    assert np.max(np.abs(full - local)) > 1e-3 * np.max(np.abs(full))


def test_time_reversal_identity():
    kf = np.array([[0.125, -0.375, 0.25], [-0.25, 0.125, 0.375]])
    s = system(k_frac=kf)
    sm = system(k_frac=-kf)
    u = W.random_orbitals(9, 2, s.nb, s.cell.N, s.cell.omega)
    A = np.array([[[0.01, -0.02, 0.03], [0.012, -0.018, 0.031]]] * 4)
    r1 = P.Run(s, u, 0.02, "scf")
    r2 = P.Run(sm, np.conj(u), -0.02, "scf")
    J1 = r1.run(A)
    J2 = r2.run(-A)
    np.testing.assert_allclose(r2.u, np.conj(r1.u), rtol=0, atol=1e-13)
    np.testing.assert_allclose(J2, -J1, rtol=0, atol=1e-15)
    np.testing.assert_allclose(P.density(sm, r2.u), P.density(s, r1.u), rtol=0, atol=1e-13)


def test_time_reversal_zero_current():
    kf = kpoints.monkhorst_pack((2, 2, 2))
    half = [i for i in range(8) if i < 4]
    s = system(k_frac=kf, nb=2)
    u = np.empty((8, 2) + s.cell.shape, complex)
    base = W.random_orbitals(10, 4, 2, s.cell.N, s.cell.omega)
    for i in half:
        j = [jj for jj in range(8) if np.allclose(kf[jj], -kf[i])][0]
        u[i] = base[i]
        u[j] = np.conj(base[i])
    J = P.current(s, np.zeros(3), u)
    assert np.max(np.abs(J)) < 1e-17


def test_two_step_equals_dense_with_frozen_hxc():
    grid = (6, 6, 6)
    dense = system(grid, W.KSpec((4, 4, 4)), nb=2)
    n_dense = dense.nk
    u_dense = W.random_orbitals(12, n_dense, 2, grid, dense.cell.omega)
    v_frozen = hxc_potential(dense.cell, P.density(dense, u_dense))
    A = np.array([[[-1e-3, 0, 0], [-1e-3, 0, 0]]] * 3)
    rd = P.Run(dense, u_dense, 0.02, "frozen", v_frozen)
    Jd = rd.run(A)
    per_shift, pre_shift = [], []
    seen = 0
    for j3 in range(2):
        for j2 in range(2):
            for j1 in range(2):
                sub = system(grid, W.KSpec((2, 2, 2), (2, 2, 2), (j1, j2, j3)), nb=2)
                # locate each shifted k in the dense list (exact binary equality)
                idx = [int(np.nonzero(np.all(dense.k_frac == kk, axis=1))[0][0]) for kk in sub.k_frac]
                rs = P.Run(sub, u_dense[idx], 0.02, "frozen", v_frozen)
                per_shift.append(rs.run(A))
                pre_shift.append(rs.J_pre)
                assert np.array_equal(rs.u, rd.u[idx])
                seen += len(idx)
    assert seen == n_dense
    # Eq. (9): the plain mean over the N_H = 8 sub-simulations equals the direct 4^3 run
    np.testing.assert_allclose(P.two_step_average(per_shift), Jd, rtol=1e-14, atol=1e-19)
    np.testing.assert_allclose(P.two_step_average(pre_shift), rd.J_pre, rtol=1e-14, atol=1e-19)
    # and it is the mean of the induced currents too (delta J_m = J_m - J_m^pre, per shift)
    dj = [j - p for j, p in zip(per_shift, pre_shift)]
    np.testing.assert_allclose(P.two_step_average(dj), Jd - rd.J_pre, rtol=1e-12, atol=1e-19)
