"""Edge cases of the GPU path, through the C ABI: zero-step and split calls, a
single band at the Gamma point on a small grid, a k-point on
the zone boundary, two species, the longest grid axis the kernels accept, grids
whose a_3 size the z-segment length does not divide (ragged segments), and the
state error of stepping before loading."""
import sys

import numpy as np
import pytest

import workloads as W
from oracle import propagate as OP
from oracle.hamiltonian import System

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


def _species(seed=3):
    return W.draw_species(np.random.default_rng(seed))


def _oracle(inst, u0, A, k_frac=None):
    sysm = System(inst, k_frac=k_frac)
    r = OP.Run(sysm, u0, 0.02, "scf")
    J = r.run(A)
    return J - r.J_pre, r.u


def _gpu(tdks, inst, u0, A, precision, k_frac=None, **kw):
    with tdks.Propagator([inst], k_fracs=None if k_frac is None else [k_frac], precision=precision, **kw) as p:
        p.load_orbitals(0, u0)
        p.step(A)
        return p.current()[0], p.get_orbitals(0)


def _check(name, dj, u, dj_o, u_o, precision):
    peak = np.max(np.abs(dj_o))
    err = np.max(np.abs(dj - dj_o)) / peak
    uerr = np.max(np.abs(u - u_o))
    _say(f"  {name} {precision}: dJ err {err:.2e}, u err {uerr:.2e}")
    if precision == "fp64":
        assert err < 1e-10 and uerr < 1e-10
    else:
        assert err < 1e-4 and uerr < 1e-5


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_zero_and_split_step_calls(tdks, precision):
    """n = 0 is a no-op; 5 + 0 + 7 + 4 steps equal one call of 16 bitwise (graph chunks of 16,
    ragged tails and single-step graphs mixed)."""
    inst = W.make_instance("diamond8", (8, 8, 8), 3, [_species()], W.KSpec((2, 1, 1)))
    u0 = W.random_orbitals(11, 2, 3, inst.grid, inst.omega)
    A = W.Field("kick", 1e-3).table(16, 0.02)
    with tdks.Propagator([inst], precision=precision) as p:
        p.load_orbitals(0, u0)
        p.step(A[:0])
        assert p.steps_done == 0 and p.current().shape == (1, 0, 3)
        p.step(A)
        one, u_one = p.current(), p.get_orbitals(0)
    with tdks.Propagator([inst], precision=precision) as p:
        p.load_orbitals(0, u0)
        for a, b in ((0, 5), (5, 5), (5, 12), (12, 16)):
            p.step(A[a:b])
        split, u_split = p.current(), p.get_orbitals(0)
    assert np.array_equal(one, split) and np.array_equal(u_one, u_split)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_single_band_gamma_smallest_grid(tdks, precision):
    """One band at k = 0 on a 6^3 grid."""
    inst = W.make_instance("diamond8", (6, 6, 6), 1, [_species()], W.KSpec((1, 1, 1)))
    u0 = W.random_orbitals(12, 1, 1, inst.grid, inst.omega, mmax=1)
    A = W.Field("kick", 1e-3).table(6, 0.02)
    dj, u = _gpu(tdks, inst, u0, A, precision)
    dj_o, u_o = _oracle(inst, u0, A)
    _check("1 band, Gamma, 6^3", dj, u, dj_o, u_o, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_zone_boundary_k(tdks, precision):
    """A single k-point at (1/2, 1/2, 1/2), where kappa is largest."""
    inst = W.make_instance("diamond8", (8, 8, 8), 2, [_species()], W.KSpec((1, 1, 1)))
    kf = np.array([[0.5, 0.5, 0.5]])
    u0 = W.random_orbitals(13, 1, 2, inst.grid, inst.omega)
    A = W.Field("kick", 1e-3).table(6, 0.02)
    dj, u = _gpu(tdks, inst, u0, A, precision, k_frac=kf)
    dj_o, u_o = _oracle(inst, u0, A, k_frac=kf)
    _check("k = (1/2, 1/2, 1/2)", dj, u, dj_o, u_o, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_two_species(tdks, precision):
    """Alternating species on the 8-atom cell (different local depths, projector energies
    and radii)."""
    sp1, sp2 = _species(3), _species(4)
    sp2 = W.Species(D=sp2.D, w=sp2.w, rc=1.0, Rc=3.2, Es=sp2.Es, Ep=sp2.Ep)
    inst = W.make_instance("diamond8", (8, 8, 8), 3, [sp1, sp2], W.KSpec((2, 1, 1)))
    inst.atom_species = np.array([0, 1, 0, 1, 1, 0, 1, 0], dtype=np.int32)
    u0 = W.random_orbitals(14, 2, 3, inst.grid, inst.omega)
    A = W.Field("kick", 1e-3).table(6, 0.02)
    dj, u = _gpu(tdks, inst, u0, A, precision)
    dj_o, u_o = _oracle(inst, u0, A)
    _check("two species", dj, u, dj_o, u_o, precision)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_longest_axis(tdks, precision):
    """The 16-atom supercell on an 8 x 8 x 32 grid (32 = the longest axis accepted)."""
    inst = W.make_instance("super16", (8, 8, 32), 2, [_species()], W.KSpec((1, 1, 1)))
    u0 = W.random_orbitals(15, 1, 2, inst.grid, inst.omega)
    A = W.Field("kick", 1e-3).table(4, 0.02)
    dj, u = _gpu(tdks, inst, u0, A, precision)
    dj_o, u_o = _oracle(inst, u0, A)
    _check("8x8x32", dj, u, dj_o, u_o, precision)


def test_step_before_load_is_a_state_error(tdks):
    from paper_2112_00920_amd import _lib

    inst = W.make_instance("diamond8", (8, 8, 8), 2, [_species()], W.KSpec((1, 1, 1)))
    with tdks.Propagator([inst], precision="fp64") as p:
        with pytest.raises(_lib.TdksError) as e:
            p.step(W.Field("kick", 1e-3).table(1, 0.02))
        assert e.value.code == _lib.E_STATE


RAGGED_CASES = {
    # grids whose a_3 size is not a multiple of the chosen z-segment length
    "d8_15": ("diamond8", (15, 15, 15), 2, W.KSpec((1, 1, 2))),  # the paper's grid size
    "d8_7": ("diamond8", (7, 7, 7), 3, W.KSpec((2, 1, 1))),
    "d8_12x12x13": ("diamond8", (12, 12, 13), 2, W.KSpec((1, 1, 1))),
    "fcc2_7": ("fcc2", (7, 7, 7), 2, W.KSpec((2, 2, 1))),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(RAGGED_CASES))
def test_ragged_z_segments(tdks, name, precision):
    cell, grid, nb, ks = RAGGED_CASES[name]
    inst = W.make_instance(cell, grid, nb, [_species()], ks)
    nk = int(np.prod(ks.coarse))
    u0 = W.random_orbitals(16, nk, nb, grid, inst.omega)
    A = W.Field("kick", 1e-3).table(4, 0.02)
    with tdks.Propagator([inst], precision=precision) as p:
        til = p.tiling()
        p.load_orbitals(0, u0)
        p.step(A)
        dj, u = p.current()[0], p.get_orbitals(0)
    _say(f"  {name} {precision}: tiling {til}")
    assert grid[2] % til["zl"] != 0 or grid[2] < til["zl"]
    dj_o, u_o = _oracle(inst, u0, A)
    _check(name, dj, u, dj_o, u_o, precision)


LONG_SEGMENT_CASES = {
    # grid, threads per workgroup: one z-segment of 8 or 10 points per column (the FP32 kernel
    # then sums the Taylor series by Horner's rule and reads the potential from memory)
    "d8_8_zl8": ((8, 8, 8), 64),
    "d8_10_zl10": ((10, 10, 10), 128),
}


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("name", list(LONG_SEGMENT_CASES))
def test_long_z_segments(tdks, name, precision):
    grid, block = LONG_SEGMENT_CASES[name]
    inst = W.make_instance("diamond8", grid, 3, [_species()], W.KSpec((2, 1, 1)))
    u0 = W.random_orbitals(17, inst.n_k, inst.n_bands, grid, inst.omega)
    A = W.Field("kick", 1e-3).table(4, 0.02)
    with tdks.Propagator([inst], precision=precision, block_size=block) as p:
        til = p.tiling()
        p.load_orbitals(0, u0)
        p.step(A)
        dj, u = p.current()[0], p.get_orbitals(0)
    _say(f"  {name} {precision}: tiling {til}")
    assert til["zl"] == grid[2]
    dj_o, u_o = _oracle(inst, u0, A)
    _check(name, dj, u, dj_o, u_o, precision)
