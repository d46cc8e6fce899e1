"""Oracle pins for the predictor-corrector propagator (Hxc at the mid-step): with a
frozen or zero potential it is the explicit step, bit for bit; with SCF Hxc its
error in the current falls as dt^2 where the explicit step's falls as dt (the
explicit step holds v_Hxc[rho(t_n)] over the step), both measured against the same
system run with a 16 times smaller step."""
import numpy as np

import workloads as W
from oracle import propagate as P
from oracle.hamiltonian import System


def _system():
    sp = W.draw_species(np.random.default_rng(3))
    inst = W.make_instance("diamond8", (6, 6, 6), 2, [sp], W.KSpec((1, 1, 1)))
    return System(inst), inst


def test_pc_equals_explicit_without_scf():
    s, inst = _system()
    u0 = W.random_orbitals(7, s.nk, s.nb, inst.grid, inst.omega)
    A = W.Field("kick", 1e-3).table(6, 0.05)
    v_fr = np.random.default_rng(2).uniform(-0.3, 0.0, s.cell.shape)
    for mode, v in (("frozen", v_fr), ("none", None)):
        a = P.Run(s, u0, 0.05, mode, v)
        b = P.Run(s, u0, 0.05, mode, v, propagator="pc")
        assert np.array_equal(a.run(A), b.run(A)) and np.array_equal(a.u, b.u)


def _j_at(s, u0, dt, T, prop):
    n = int(round(T / dt))
    r = P.Run(s, u0, dt, "scf", propagator=prop)
    A = np.zeros((n, 2, 3))
    return r.run(A)[-1]


def test_pc_second_order_in_the_hxc_coupling():
    """Random (non-stationary) orbitals make the density and v_Hxc move from the start,
    so the Hxc coupling error dominates the Taylor-4 truncation at these steps."""
    s, inst = _system()
    u0 = W.random_orbitals(8, s.nk, s.nb, inst.grid, inst.omega)
    T = 0.8
    ref = _j_at(s, u0, 0.00625, T, "pc")
    e = {p: [np.max(np.abs(_j_at(s, u0, dt, T, p) - ref)) for dt in (0.05, 0.025)] for p in ("taylor", "pc")}
    r_exp = e["taylor"][0] / e["taylor"][1]
    r_pc = e["pc"][0] / e["pc"][1]
    assert 1.8 < r_exp < 2.2, e
    assert r_pc > 3.5, e
    assert e["pc"][1] < 0.2 * e["taylor"][1], e
