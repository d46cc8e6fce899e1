"""Ground-state preparation on the GPU (tdks_ground_state) through the C ABI against
the oracle's imaginary-time route, step by step: orbitals, density, v_Hxc, J_pre
and the residual after a few iterations on a batch of two different cells (FP64
to 1e-10; FP32 to its rounding), the converged state against the independent
dense-diagonalisation SCF ground state, a kick propagated from it against the
oracle's kick from its own ground state, the frozen-potential mode, and the
argument and state errors."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import ground as G
from oracle import propagate as OP
from oracle.hamiltonian import System
from oracle.propagate import density

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def tdks():
    import torch
    import paper_2112_00920_amd as tdks

    assert torch.cuda.is_available()
    return tdks


def _species():
    return W.draw_species(np.random.default_rng(3))


def _batch():
    sp = _species()
    return [W.make_instance("diamond8", (8, 8, 8), 3, [sp], W.KSpec((2, 1, 1))),
            W.make_instance("fcc2", (8, 8, 8), 2, [sp], W.KSpec((2, 2, 1)), group=1)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("n_iter", [1, 4])
def test_iterations_vs_oracle(tdks, precision, n_iter):
    insts = _batch()
    u0s = [W.random_orbitals(60 + i, inst.n_k, inst.n_bands, inst.grid, inst.omega) for i, inst in enumerate(insts)]
    tau, mix = 0.12, 0.5  # the fcc cell's kinetic bound allows tau <= 0.138
    _say(f"ground state {precision}: {n_iter} iterations, tau {tau}, mix {mix}")
    with tdks.Propagator(insts, precision=precision) as p:
        for i, u in enumerate(u0s):
            p.load_orbitals(i, u)
        res = p.ground_state(n_iter, tau, mix)
        got = [(p.get_orbitals(i), p.density(i), p.vhxc(i)) for i in range(len(insts))]
        jpre = p.current_pre()
    for i, inst in enumerate(insts):
        s = System(inst)
        u0 = u0s[i]
        if precision == "fp32":  # the GPU loaded FP32-rounded orbitals
            u0 = u0.astype(np.complex64).astype(np.complex128)
        u, rho, v, r = G.imaginary_time_scf(s, u0, tau, mix, n_iter)
        j = OP.current(s, np.zeros(3), u)
        eu = np.max(np.abs(got[i][0] - u))
        er = np.max(np.abs(got[i][1] - rho)) / np.max(rho)
        ev = np.max(np.abs(got[i][2] - v))
        ej = np.max(np.abs(jpre[i] - j))
        eres = abs(res[i] - r[-1]) / r[-1]
        _say(f"  instance {i} ({inst.cell}): u {eu:.2e}, rho {er:.2e}, v {ev:.2e}, J_pre {ej:.2e}, "
             f"residual {res[i]:.3e} (rel err {eres:.2e})")
        if precision == "fp64":
            assert eu < 1e-10 and er < 1e-12 and ev < 1e-11 and ej < 1e-12 and eres < 1e-9
        else:
            assert eu < 2e-5 and er < 2e-6 and ev < 1e-6 and ej < 1e-8 and eres < 1e-3


def test_converged_state_and_kick_vs_dense_ground_state(tdks):
    """6^3 cell, 4 bands, 2 k: 150 iterations reach the dense-diagonalisation SCF ground
    state; a kick from it gives the oracle's delta J from its own ground state."""
    inst = W.make_instance("diamond8", (6, 6, 6), 4, [_species()], W.KSpec((2, 1, 1)))
    s = System(inst)
    u_d, eps, v_d, _ = G.scf(s, tol=1e-12)
    rho_d = density(s, u_d)
    u0 = W.random_orbitals(5, s.nk, s.nb, inst.grid, inst.omega)
    A = W.Field("kick", 1e-3).table(10, 0.02)
    with tdks.Propagator([inst], precision="fp64") as p:
        p.load_orbitals(0, u0)
        res = p.ground_state(150, 0.8, 0.5)
        rho, v = p.density(0), p.vhxc(0)
        u_g = p.get_orbitals(0)
        p.step(A)
        dj = p.current()[0]
    drho = np.sum(np.abs(rho - rho_d)) * s.cell.dV
    e_g = G.subspace_energy(s, v, u_g)
    e_d = np.mean(np.sum(eps, axis=1))
    _say(f"  residual {res[0]:.2e}; sum|rho - rho_dense| dV {drho:.2e}; band energy {e_g:.12f} vs {e_d:.12f}")
    assert res[0] < 1e-12 and drho < 1e-10 and abs(e_g - e_d) < 1e-10
    assert np.max(np.abs(v - v_d)) < 1e-9
    r = OP.Run(s, u_d, 0.02, "scf")
    ref = r.run(A) - r.J_pre
    err = np.max(np.abs(dj - ref)) / np.max(np.abs(ref))
    _say(f"  kick from the ground state: max |dJ - dJ_oracle| / peak = {err:.2e} (peak {np.max(np.abs(ref)):.3e})")
    assert err < 1e-8


def test_frozen_potential_mode(tdks):
    inst = _batch()[0]
    s = System(inst)
    v_fr = np.random.default_rng(9).uniform(-0.3, 0.0, inst.grid[::-1])
    u0 = W.random_orbitals(61, inst.n_k, inst.n_bands, inst.grid, inst.omega)
    with tdks.Propagator([inst], precision="fp64", hxc_mode="frozen", v_hxc_frozen=[v_fr]) as p:
        p.load_orbitals(0, u0)
        res = p.ground_state(3, 0.3, 0.5)
        ug = p.get_orbitals(0)
    u, rho, v, r = G.imaginary_time_scf(s, u0, 0.3, 0.5, 3, hxc_mode="frozen", v_hxc_frozen=v_fr)
    assert np.max(np.abs(ug - u)) < 1e-10 and abs(res[0] - r[-1]) < 1e-9 * r[-1]


def test_errors(tdks):
    from paper_2112_00920_amd import _lib

    inst = _batch()[0]
    with tdks.Propagator([inst], precision="fp64") as p:
        with pytest.raises(_lib.TdksError) as e:
            p.ground_state(2, 0.3, 0.5)
        assert e.value.code == _lib.E_STATE
        p.load_orbitals(0, W.random_orbitals(62, inst.n_k, inst.n_bands, inst.grid, inst.omega))
        for bad in ((-1, 0.3, 0.5), (2, 0.0, 0.5), (2, 0.3, 0.0), (2, 0.3, 1.5), (2, 50.0, 0.5)):
            with pytest.raises(_lib.TdksError) as e:
                p.ground_state(*bad)
            assert e.value.code == _lib.E_ARG
        assert p.ground_state(0, 0.3, 0.5).shape == (1,)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_ragged_grid_and_many_bands(tdks, precision):
    """A 7^3 grid (z-segments of unequal length in the imaginary-time kernel) and 20
    bands (the orthonormalisation's tiles of 64 points and its full 2 x 256 Gram
    entries per thread) against the oracle's route, 2 iterations."""
    sp = _species()
    insts = [W.make_instance("diamond8", (7, 7, 7), 3, [sp], W.KSpec((2, 1, 1))),
             W.make_instance("diamond8", (8, 8, 8), 20, [sp], W.KSpec((1, 1, 1)), group=1)]
    u0s = [W.random_orbitals(80 + i, inst.n_k, inst.n_bands, inst.grid, inst.omega) for i, inst in enumerate(insts)]
    with tdks.Propagator(insts, precision=precision) as p:
        til = p.tiling()
        for i, u in enumerate(u0s):
            p.load_orbitals(i, u)
        res = p.ground_state(2, 0.2, 0.5)
        got = [p.get_orbitals(i) for i in range(len(insts))]
    _say(f"  {precision}: tiling {til}")
    for i, inst in enumerate(insts):
        u0 = u0s[i]
        if precision == "fp32":
            u0 = u0.astype(np.complex64).astype(np.complex128)
        u, rho, v, r = G.imaginary_time_scf(System(inst), u0, 0.2, 0.5, 2)
        eu = np.max(np.abs(got[i] - u))
        _say(f"  {precision} instance {i} ({inst.grid}, {inst.n_bands} bands): u err {eu:.2e}, residual {res[i]:.3e}")
        assert eu < (1e-10 if precision == "fp64" else 2e-5)
        assert abs(res[i] - r[-1]) < (1e-9 if precision == "fp64" else 1e-3) * r[-1]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_padded_block_grid(tdks, precision):
    """A 20^3 grid: 800 column segments of 10 points in a block padded to 1024 threads,
    whose extra waves own no segment but take projection, coefficient and current tasks; the
    imaginary-time kernel and the orthonormalisation against the oracle's route, 2 iterations."""
    sp = _species()
    inst = W.make_instance("diamond8", (20, 20, 20), 4, [sp], W.KSpec((2, 1, 1)))
    u0 = W.random_orbitals(91, inst.n_k, inst.n_bands, inst.grid, inst.omega)
    tau = 0.05  # the 20^3 kinetic bound (about 30 Ha) allows tau below 0.09
    with tdks.Propagator([inst], precision=precision) as p:
        til = p.tiling()
        p.load_orbitals(0, u0)
        res = p.ground_state(2, tau, 0.5)
        got = p.get_orbitals(0)
    _say(f"  {precision}: tiling {til}")
    assert til["block"] == 1024 and til["zl"] == 10
    if precision == "fp32":
        u0 = u0.astype(np.complex64).astype(np.complex128)
    u, rho, v, r = G.imaginary_time_scf(System(inst), u0, tau, 0.5, 2)
    eu = np.max(np.abs(got - u))
    _say(f"  {precision}: u err {eu:.2e}, residual {res[0]:.3e}")
    assert eu < (1e-10 if precision == "fp64" else 2e-5)
    assert abs(res[0] - r[-1]) < (1e-9 if precision == "fp64" else 1e-3) * r[-1]


@pytest.mark.parametrize("bands", [(1, 16), (17, 32)])
def test_band_counts_at_block_edges(tdks, bands):
    """Band counts at the edges of the orthonormalisation's 16-band blocks: one band and
    a full block (one block), one past a block and the maximum of 32 (two blocks; the
    launch takes the larger count's variant), FP64 against the oracle's route."""
    sp = _species()
    insts = [W.make_instance("diamond8", (8, 8, 8), nb, [sp], W.KSpec((1, 1, 1)), group=g)
             for g, nb in enumerate(bands)]
    u0s = [W.random_orbitals(90 + i, inst.n_k, inst.n_bands, inst.grid, inst.omega) for i, inst in enumerate(insts)]
    with tdks.Propagator(insts, precision="fp64") as p:
        for i, u in enumerate(u0s):
            p.load_orbitals(i, u)
        res = p.ground_state(2, 0.2, 0.5)
        got = [p.get_orbitals(i) for i in range(len(insts))]
    for i, inst in enumerate(insts):
        u, rho, v, r = G.imaginary_time_scf(System(inst), u0s[i], 0.2, 0.5, 2)
        eu = np.max(np.abs(got[i] - u))
        _say(f"  {inst.n_bands} bands: u err {eu:.2e}, residual {res[i]:.3e}")
        assert eu < 1e-10
        assert abs(res[i] - r[-1]) < 1e-9 * r[-1]
