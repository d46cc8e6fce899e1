"""The k-parallel driver of the oracle (oracle.pool) against the oracle's own Run: the same
per-k arithmetic, only the order of the k-sums of Eqs. (3) and (5) differs, so the currents
agree to rounding (SCF, with a field)."""
import numpy as np

import workloads as W
from oracle import propagate as P
from oracle.hamiltonian import System
from oracle.pool import PoolRun


def test_pool_equals_run():
    sp = W.draw_species(np.random.default_rng(4))
    inst = W.make_instance("diamond8", (6, 6, 6), 3, [sp], W.KSpec((2, 2, 1), (2, 2, 2), (1, 0, 1)))
    sysm = System(inst)
    u0 = W.random_orbitals(8, sysm.nk, 3, inst.grid, inst.omega)
    A = W.Field("pulse", A0=0.5, omega=0.3, T=2.0).table(6, 0.02, start=20)
    ref = P.Run(sysm, u0, 0.02, "scf")
    j_ref = ref.run(A)
    with PoolRun(sysm, u0, 0.02, "scf", workers=3) as pr:
        assert len(pr.blocks) == 3
        j = pr.run(A)
        np.testing.assert_allclose(pr.J_pre, ref.J_pre, rtol=0, atol=1e-14 * np.max(np.abs(ref.J_pre)) + 1e-18)
        np.testing.assert_allclose(j, j_ref, rtol=0, atol=1e-13 * np.max(np.abs(j_ref)))
        np.testing.assert_allclose(pr.orbitals(), ref.u, rtol=0, atol=1e-12)
