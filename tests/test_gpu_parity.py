"""GPU parity: the HIP path (through the C ABI) against the CPU FP64 oracle.

Bars: FP64 path within 1e-10 of the peak |delta J| (and 1e-12-level agreement
of single Hamiltonian applications); FP32 path within 1e-4 of the peak
|delta J|.  Invariants that hold exactly are checked bitwise on the GPU:
two-step sub-grids with frozen Hxc reproduce the direct dense-k run orbital by
orbital, and an instance inside a batch equals the same instance run alone.
"""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import propagate as OP
from oracle.hamiltonian import System
from oracle.hxc import v_hxc as oracle_vhxc

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tdks():
    import torch

    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2112_00920_amd as mod

    mod._lib.load()
    return mod


def species(seed=1):
    return W.draw_species(np.random.default_rng(seed))


CASES = {
    # name: (cell, grid, bands, kspec)
    "d8_6": ("diamond8", (6, 6, 6), 4, W.KSpec((2, 1, 1))),
    "d8_12": ("diamond8", (12, 12, 12), 3, W.KSpec((2, 1, 1))),
    "d8_8x10x12": ("diamond8", (8, 10, 12), 2, W.KSpec((1, 2, 1))),
    "fcc2_8": ("fcc2", (8, 8, 8), 3, W.KSpec((2, 2, 1))),
    "s16_8x8x16": ("super16", (8, 8, 16), 3, W.KSpec((1, 1, 2))),
    "d8_16": ("diamond8", (16, 16, 16), 2, W.KSpec((1, 1, 2))),
    # FP64: the per-column-image tables in device memory (they do not fit the LDS beside the orbital)
    "d8_20": ("diamond8", (20, 20, 20), 2, W.KSpec((1, 2, 1))),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(CASES))
def test_apply_h(tdks, name, precision):
    cell, grid, nb, ks = CASES[name]
    _say(f"apply_h {name} {precision}")
    inst = W.make_instance(cell, grid, nb, [species()], ks)
    sysm = System(inst)
    w = W.random_orbitals(5, sysm.nk, nb, grid, inst.omega)
    A = np.array([0.013, -0.021, 0.008])
    with tdks.Propagator([inst], precision=precision, hxc_mode="none") as prop:
        got = prop.apply_h(0, w, A)
        assert np.array_equal(prop.vloc(0), prop.vloc(0))
        np.testing.assert_allclose(prop.vloc(0), sysm.v_loc, rtol=0, atol=1e-13)
    want = np.stack([sysm.apply_h(sysm.k_cart[k] + A, 0.0, w[k]) for k in range(sysm.nk)])
    err = np.max(np.abs(got - want)) / np.max(np.abs(want))
    if precision == "fp64":
        _say(f"  rel err {err:.2e}")
        assert err < 1e-13
        return
    # FP32 bar from the arithmetic: the FP32 path rounds w to FP32 and sums the stencil,
    # potential and projector terms in FP32. Rounding the input alone changes the FP64
    # result by s_in (computed here with the oracle); the sums' own roundings are of the same
    # order, since the terms exceed the result by the same kinetic conditioning, which grows
    # as 1/h^2 with the grid. Bar: 10 s_in.
    w32 = w.astype(np.complex64).astype(np.complex128)
    want32 = np.stack([sysm.apply_h(sysm.k_cart[k] + A, 0.0, w32[k]) for k in range(sysm.nk)])
    s_in = np.max(np.abs(want32 - want)) / np.max(np.abs(want))
    _say(f"  rel err {err:.2e}; input rounding alone {s_in:.2e} (bar 10x)")
    assert err < 10 * s_in


def run_gpu(tdks, insts, u0s, A, precision="fp64", hxc="scf", frozen=None, k_fracs=None, **kw):
    with tdks.Propagator(insts, k_fracs=k_fracs, precision=precision, hxc_mode=hxc, v_hxc_frozen=frozen,
                         **kw) as prop:
        for i, u in enumerate(u0s):
            prop.load_orbitals(i, u)
        jpre = prop.current_pre()
        prop.step(A)
        dj = prop.current()
        us = [prop.get_orbitals(i) for i in range(len(insts))]
        rhos = [prop.density(i) for i in range(len(insts))]
        return dj, us, rhos, jpre, prop.tiling()


def run_oracle(inst, u0, A, hxc="scf", frozen=None, k_frac=None):
    sysm = System(inst, k_frac=k_frac)
    r = OP.Run(sysm, u0, 0.02, hxc, frozen)
    J = r.run(A)
    return J - r.J_pre, r.u, OP.density(sysm, r.u), r.J_pre


STEP_CASES = {
    # name: (cell, grid, bands, kspec, steps, options)
    "d8_8_scf": ("diamond8", (8, 8, 8), 4, W.KSpec((2, 1, 1)), 12, {}),
    "d8_8_nograph": ("diamond8", (8, 8, 8), 4, W.KSpec((2, 1, 1)), 5, {"graph_steps": -1}),
    "d8_8_ragged_groups": ("diamond8", (8, 8, 8), 5, W.KSpec((3, 1, 1)), 6,
                           {"bands_per_group": 2, "k_per_group": 2}),
    "d8_12": ("diamond8", (12, 12, 12), 4, W.KSpec((2, 2, 2)), 6, {}),
    "fcc2_8": ("fcc2", (8, 8, 8), 3, W.KSpec((2, 2, 2)), 6, {}),
    "s16_8x8x16": ("super16", (8, 8, 16), 6, W.KSpec((1, 1, 2)), 4, {}),
    "d8_16": ("diamond8", (16, 16, 16), 3, W.KSpec((1, 1, 2)), 4, {}),
    "s16_16x16x32": ("super16", (16, 16, 32), 2, W.KSpec((1, 1, 2)), 3, {}),
    "d8_20_split_bands": ("diamond8", (20, 20, 20), 16, W.KSpec((1, 1, 1)), 3, {}),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(STEP_CASES))
def test_steps_vs_oracle(tdks, name, precision):
    cell, grid, nb, ks, steps, opts = STEP_CASES[name]
    _say(f"steps {name} {precision}")
    inst = W.make_instance(cell, grid, nb, [species()], ks)
    nk = int(np.prod(ks.coarse))
    u0 = W.random_orbitals(7, nk, nb, grid, inst.omega)
    A = W.Field("kick", 1e-3).table(steps, 0.02)
    dj, us, rhos, jpre, til = run_gpu(tdks, [inst], [u0], A, precision, **opts)
    dj_o, u_o, rho_o, jpre_o = run_oracle(inst, u0, A)
    peak = np.max(np.abs(dj_o))
    err = np.max(np.abs(dj[0] - dj_o)) / peak
    uerr = np.max(np.abs(us[0] - u_o))
    rerr = np.max(np.abs(rhos[0] - rho_o)) / np.max(rho_o)
    _say(f"  tiling {til}  dJ err {err:.2e}  u err {uerr:.2e}  rho err {rerr:.2e}")
    if precision == "fp64":
        assert err < 1e-10 and rerr < 1e-11 and uerr < 1e-10
        np.testing.assert_allclose(jpre[0], jpre_o, rtol=0, atol=1e-14)
    else:
        assert err < 1e-4 and rerr < 1e-5


def test_two_step_equals_dense_frozen_hxc(tdks):
    """4^3 MP run directly vs its 2^3 shifted 2^3 sub-grids as 8 instances (frozen Hxc)."""
    _say("two-step vs dense, frozen Hxc")
    grid = (8, 8, 8)
    sp = species()
    dense = W.make_instance("diamond8", grid, 2, [sp], W.KSpec((4, 4, 4)))
    kd = tdks.kpoints.from_spec(dense.kspec)
    u_dense = W.random_orbitals(12, 64, 2, grid, dense.omega)
    v_frozen = np.random.default_rng(3).uniform(-0.4, 0.0, (8, 8, 8))
    A = W.Field("kick", 1e-3).table(5, 0.02)
    subs, u_subs, idxs = [], [], []
    for j3 in range(2):
        for j2 in range(2):
            for j1 in range(2):
                s = W.make_instance("diamond8", grid, 2, [sp], W.KSpec((2, 2, 2), (2, 2, 2), (j1, j2, j3)), group=7)
                ks = tdks.kpoints.from_spec(s.kspec)
                idx = [int(np.nonzero(np.all(kd == kk, axis=1))[0][0]) for kk in ks]
                subs.append(s)
                u_subs.append(u_dense[idx])
                idxs.append(idx)
    dj_d, us_d, _, _, _ = run_gpu(tdks, [dense], [u_dense], A, "fp64", "frozen", [v_frozen])
    with tdks.Propagator(subs, precision="fp64", hxc_mode="frozen", v_hxc_frozen=[v_frozen] * 8) as prop:
        for i, u in enumerate(u_subs):
            prop.load_orbitals(i, u)
        prop.step(A)
        dj_g = prop.current(per="group")
        for i in range(8):
            assert np.array_equal(prop.get_orbitals(i), us_d[0][idxs[i]]), f"sub-grid {i} differs"
    np.testing.assert_allclose(dj_g[0], dj_d[0], rtol=1e-13, atol=1e-18)


def test_batched_equals_alone(tdks):
    _say("batched vs alone")
    sp = species()
    grid = (8, 8, 8)
    insts = [W.make_instance("diamond8", grid, 3, [sp], W.KSpec((2, 1, 1), (2, 2, 2), (j, 1, 0)), group=j)
             for j in range(2)]
    insts.append(W.make_instance("diamond8", (6, 6, 6), 2, [sp], W.KSpec((1, 1, 1)), group=5))
    u0s = [W.random_orbitals(20 + i, inst.n_k, inst.n_bands, inst.grid, inst.omega) for i, inst in enumerate(insts)]
    A = W.Field("kick", 1e-3).table(4, 0.02)
    for prec in ("fp64", "fp32"):
        dj_b, us_b, rho_b, _, _ = run_gpu(tdks, insts, u0s, A, prec)
        for i in range(len(insts)):
            dj_a, us_a, rho_a, _, _ = run_gpu(tdks, [insts[i]], [u0s[i]], A, prec)
            assert np.array_equal(us_a[0], us_b[i]), (prec, i)
            assert np.array_equal(dj_a[0], dj_b[i]), (prec, i)
            assert np.array_equal(rho_a[0], rho_b[i]), (prec, i)


def test_time_reversal_on_gpu(tdks):
    _say("time reversal")
    sp = species()
    grid = (8, 8, 8)
    kf = np.array([[0.125, -0.375, 0.25], [-0.25, 0.125, 0.375]])
    inst = W.make_instance("diamond8", grid, 3, [sp], W.KSpec((2, 1, 1)))
    u0 = W.random_orbitals(9, 2, 3, grid, inst.omega)
    A = np.array([[[0.01, -0.02, 0.03], [0.012, -0.018, 0.031]]] * 4)
    with tdks.Propagator([inst], k_fracs=[kf], precision="fp64", dt=0.02) as p1, \
            tdks.Propagator([inst], k_fracs=[-kf], precision="fp64", dt=-0.02) as p2:
        p1.load_orbitals(0, u0)
        p2.load_orbitals(0, np.conj(u0))
        p1.step(A)
        p2.step(-A)
        np.testing.assert_allclose(p2.get_orbitals(0), np.conj(p1.get_orbitals(0)), rtol=0, atol=1e-13)
        j1 = p1.current() + p1.current_pre()[:, None, :]
        j2 = p2.current() + p2.current_pre()[:, None, :]
        np.testing.assert_allclose(j2, -j1, rtol=0, atol=1e-16)
        np.testing.assert_allclose(p2.density(0), p1.density(0), rtol=0, atol=1e-13)


def test_free_electron_closed_form_on_gpu(tdks):
    _say("free electrons")
    lat, _ = W.diamond8()
    inst = W.Instance(cell="diamond8", lattice=lat, grid=(8, 8, 8), atom_frac=np.zeros((0, 3)),
                      atom_species=np.zeros(0, np.int32), species=[], kspec=W.KSpec((2, 2, 2)), n_bands=1)
    omega = inst.omega
    u = np.ones((8, 1, 8, 8, 8), complex) / np.sqrt(omega)
    A = W.Field("kick", 1e-3).table(3, 0.02)
    with tdks.Propagator([inst], precision="fp64", hxc_mode="none") as prop:
        prop.load_orbitals(0, u)
        prop.step(A)
        dj = prop.current()[0]
        n = 2.0 / omega
        np.testing.assert_allclose(dj[:, 0], n * 1e-3, rtol=1e-12)
        np.testing.assert_allclose(dj[:, 1:], 0.0, atol=1e-18)
        kc = np.asarray(tdks.kpoints.mp_grid((2, 2, 2))) @ (2 * np.pi * np.linalg.inv(lat).T)
        uf = prop.get_orbitals(0)
        for k in range(8):
            eps = 0.5 * np.sum((kc[k] + A[0, 0]) ** 2)
            z = -1j * eps * 0.02
            t4 = 1 + z + z * z / 2 + z ** 3 / 6 + z ** 4 / 24
            np.testing.assert_allclose(uf[k], t4 ** 3 * u[k], rtol=0, atol=1e-14)


def test_diamond8_g12_mp2_fp64(tdks):
    """The 8-atom 12^3 cell with 16 bands on the 2^3 MP grid, 20 SCF steps after a kick."""
    wl = W.config("diamond8_g12_mp2")
    inst = wl.instances[0]
    _say("diamond8 12^3 2^3 MP 16 bands, 20 steps FP64")
    u0 = W.random_orbitals(1, 8, 16, inst.grid, inst.omega)
    A = wl.field.table(20, wl.dt)
    dj, us, rhos, jpre, til = run_gpu(tdks, [inst], [u0], A, "fp64")
    dj_o, u_o, rho_o, _ = run_oracle(inst, u0, A)
    err = np.max(np.abs(dj[0] - dj_o)) / np.max(np.abs(dj_o))
    _say(f"  tiling {til} dJ err {err:.2e}")
    assert err < 1e-10


def test_pulse_time_varying_field(tdks):
    """sin^2 pulse: A(t_n + dt/2) != A(t_{n+1}), so propagation and current use different kappa."""
    _say("sin^2 pulse, FP64 and FP32")
    inst = W.make_instance("diamond8", (8, 8, 8), 3, [species()], W.KSpec((2, 1, 1), (2, 2, 2), (1, 0, 1)))
    u0 = W.random_orbitals(31, 2, 3, inst.grid, inst.omega)
    fld = W.Field("pulse", direction=(0.6, 0.0, 0.8), A0=0.5, omega=0.3, T=0.4)
    A = fld.table(16, 0.02)
    assert np.max(np.abs(A[:, 0] - A[:, 1])) > 1e-3
    dj_o, u_o, rho_o, _ = run_oracle(inst, u0, A)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
        dj, us, rhos, _, _ = run_gpu(tdks, [inst], [u0], A, prec)
        err = np.max(np.abs(dj[0] - dj_o)) / np.max(np.abs(dj_o))
        _say(f"  {prec} dJ err {err:.2e}")
        assert err < tol


def test_uneven_batch_one_context(tdks):
    """fcc2 (61-point stencil), cubic cells on two grids and a 1x1x2 supercell in one context."""
    _say("uneven batch")
    sp = species(5)
    insts = [
        W.make_instance("fcc2", (8, 8, 8), 4, [sp], W.KSpec((2, 2, 2)), group=0),
        W.make_instance("diamond8", (8, 8, 8), 5, [sp], W.KSpec((2, 1, 1), (2, 2, 2), (1, 1, 0)), group=1),
        W.make_instance("diamond8", (10, 10, 10), 5, [sp], W.KSpec((2, 1, 1), (2, 2, 2), (0, 1, 1)), group=1),
        W.make_instance("super16", (8, 8, 16), 6, [sp], W.KSpec((1, 1, 2)), group=2),
    ]
    u0s = [W.random_orbitals(40 + i, inst.n_k, inst.n_bands, inst.grid, inst.omega) for i, inst in enumerate(insts)]
    A = W.Field("kick", 1e-3).table(5, 0.02)
    for prec, tol in (("fp64", 1e-10), ("fp32", 1e-4)):
        with tdks.Propagator(insts, precision=prec) as prop:
            for i, u in enumerate(u0s):
                prop.load_orbitals(i, u)
            prop.step(A)
            dj = prop.current()
            djg = prop.current(per="group")
        refs = []
        for i, inst in enumerate(insts):
            dj_o, _, _, _ = run_oracle(inst, u0s[i], A)
            refs.append(dj_o)
            err = np.max(np.abs(dj[i] - dj_o)) / np.max(np.abs(dj_o))
            _say(f"  {prec} instance {i} ({inst.cell} {inst.grid}) dJ err {err:.2e}")
            assert err < tol
        np.testing.assert_allclose(djg[1], 0.5 * (dj[1] + dj[2]), rtol=1e-13, atol=1e-20)


def test_eigenstate_norm_closed_form_on_gpu(tdks):
    """Orbitals that are eigenvectors of the dense h lose norm per step as |T4(-i eps dt)|^2."""
    _say("eigenstate norm")
    inst = W.make_instance("diamond8", (6, 6, 6), 3, [species()], W.KSpec((1, 1, 1)))
    sysm = System(inst)
    H = sysm.dense_h(sysm.k_cart[0], 0.0)
    e, vec = np.linalg.eigh(0.5 * (H + H.conj().T))
    sel = [0, 100, 215]
    u0 = (vec[:, sel].T / np.sqrt(sysm.cell.dV)).reshape(1, 3, 6, 6, 6)
    dt, n = 0.05, 10
    A = np.zeros((n, 2, 3))
    with tdks.Propagator([inst], precision="fp64", dt=dt, hxc_mode="none") as prop:
        prop.load_orbitals(0, u0)
        prop.step(A)
        nr = prop.norms(0)[0]
    for j, s in enumerate(sel):
        x = e[s] * dt
        assert abs(nr[j] - (1 - x ** 6 / 72 + x ** 8 / 576) ** n) < 1e-12


def test_concurrent_classes_graph_equals_eager(tdks):
    """Four shape classes, whose launches run concurrently on forked streams: 18 steps through
    16-step graphs (fork and join captured as parallel branches) against eager launches, bitwise
    (the classes write disjoint data, so their overlap cannot change a bit)."""
    _say("concurrent shape classes: graph vs eager")
    sp = species(6)
    insts = [
        W.make_instance("fcc2", (8, 8, 8), 3, [sp], W.KSpec((2, 1, 1)), group=0),
        W.make_instance("diamond8", (8, 8, 8), 4, [sp], W.KSpec((2, 1, 1)), group=1),
        W.make_instance("diamond8", (10, 10, 10), 3, [sp], W.KSpec((1, 1, 1)), group=1),
        W.make_instance("super16", (8, 8, 16), 4, [sp], W.KSpec((1, 1, 2)), group=2),
    ]
    u0s = [W.random_orbitals(60 + i, inst.n_k, inst.n_bands, inst.grid, inst.omega) for i, inst in enumerate(insts)]
    A = W.Field("kick", 1e-3).table(18, 0.02)
    out = {}
    for gs in (16, -1):
        with tdks.Propagator(insts, precision="fp32", graph_steps=gs) as prop:
            for i, u in enumerate(u0s):
                prop.load_orbitals(i, u)
            prop.step(A)
            out[gs] = (prop.current(), [prop.get_orbitals(i) for i in range(len(insts))])
    for i in range(len(insts)):
        assert np.array_equal(out[16][0][i], out[-1][0][i]), i
        assert np.array_equal(out[16][1][i], out[-1][1][i]), i
