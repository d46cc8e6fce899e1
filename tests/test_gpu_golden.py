"""GPU parity at the configurations' lengths and full k-sets, through the C ABI.

* The 12^3 plain-method workload (8 k, 16 bands) for all of its 500 steps in FP64 against
  the oracle run inline, and in FP32 against the same oracle run.
* One instance of each of the other workloads at its full k-set for 50 steps against the
  golden induced currents of tests/golden (written by make_golden.py with the oracle):
  the plain 512-k instance, one two-step sub-simulation (512 k), one HHG sub-simulation on
  20^3 at the peak of the pulse (64 k), and one instance of each kind of the uneven batch.
  FP64 and FP32 each (on 20^3 and 16x16x32 the FP64 kernel keeps its per-column-image
  tables in device memory).
* The two-step batch in FP64 at full size in the benchmark's FP64 tiling (4 k-points per
  workgroup), sampled against the oracle, and the 4-k grouping against 1-k grouping.

Bars (error = max_n |dJ_gpu - dJ_ref| / max_n |dJ_ref|): 1e-10 for FP64, 1e-4 for FP32.
"""
import os
import sys

import numpy as np
import pytest

import workloads as W
from oracle import propagate as OP
from oracle.hamiltonian import System
from oracle.hxc import v_hxc as oracle_vhxc

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.join(HERE, "golden"))
import make_golden as G  # noqa: E402

BARS = {"fp64": 1e-10, "fp32": 1e-4}


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


def _gpu_dj(tdks, inst, u0, A, dt, precision, **opt):
    with tdks.Propagator([inst], precision=precision, dt=dt, **opt) as prop:
        prop.load_orbitals(0, u0)
        prop.step(A)
        return prop.current()[0], prop.current_pre()[0], prop.tiling()


@pytest.fixture(scope="module")
def c1_oracle():
    wl = W.config("diamond8_g12_mp2")
    inst = wl.instances[0]
    u0 = W.random_orbitals(2000, inst.n_k, inst.n_bands, inst.grid, inst.omega)
    A = wl.field.table(wl.steps, wl.dt)
    _say(f"c1 oracle: {wl.steps} FP64 steps of 8 k x 16 bands on 12^3 (single process)")
    run = OP.Run(System(inst), u0, wl.dt, "scf")
    J = run.run(A)
    return inst, u0, A, wl.dt, J - run.J_pre, run.J_pre


@pytest.mark.timeout(600)
@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_c1_full_length(tdks, c1_oracle, precision):
    inst, u0, A, dt, dj_ref, jpre_ref = c1_oracle
    _say(f"c1 full length on the GPU, {precision}")
    dj, jpre, til = _gpu_dj(tdks, inst, u0, A, dt, precision, norm_stride=50)
    assert dj.shape == dj_ref.shape == (500, 3)
    err = np.max(np.abs(dj - dj_ref)) / np.max(np.abs(dj_ref))
    _say(f"  tiling {til}; 500 steps: max |dJ - oracle| / peak = {err:.2e} (bar {BARS[precision]:g})")
    assert err <= BARS[precision]
    if precision == "fp64":
        np.testing.assert_allclose(jpre, jpre_ref, rtol=0, atol=1e-10 * np.max(np.abs(dj_ref)))


GOLDEN = {
    "c2_plain_g16_mp8": ("fp64", "fp32"),
    "c3_twostep_sub27": ("fp64", "fp32"),
    "c4_hhg_sub21_peak": ("fp64", "fp32"),  # 20^3: FP64 with the column tables in device memory
    "c5_uneven_fcc2": ("fp64", "fp32"),
    "c5_uneven_cubic16": ("fp64", "fp32"),
    "c5_uneven_cubic20": ("fp64", "fp32"),
    "c5_uneven_super16": ("fp64", "fp32"),  # 16x16x32: same
}


@pytest.mark.timeout(300)
@pytest.mark.parametrize("case,precision", [(c, p) for c, ps in GOLDEN.items() for p in ps])
def test_golden_full_k(tdks, case, precision):
    recipe, jpre_ref, dj_ref = G.read(case)
    _say(f"golden {case} {precision}: {recipe}")
    inst, u0, A, dt = G.inputs(recipe)
    dj, jpre, til = _gpu_dj(tdks, inst, u0, A, dt, precision)
    assert dj.shape == dj_ref.shape
    peak = np.max(np.abs(dj_ref))
    err = np.max(np.abs(dj - dj_ref)) / peak
    _say(f"  {inst.n_k} k x {inst.n_bands} bands, tiling {til}: {len(dj)} steps, "
         f"max |dJ - golden| / peak = {err:.2e} (peak {peak:.2e}, bar {BARS[precision]:g})")
    assert err <= BARS[precision]
    if precision == "fp64":
        np.testing.assert_allclose(jpre, jpre_ref, rtol=0, atol=1e-10 * max(peak, np.max(np.abs(jpre_ref))))


@pytest.mark.timeout(600)
def test_two_step_full_size_fp64_sampled(tdks):
    """The whole two-step batch in FP64 in the benchmark's FP64 tiling (512 threads,
    z-segments of 8, 4 k-points per workgroup): sampled orbitals after one step against the
    oracle's step, and the current of the sub-simulation against the oracle's from the GPU
    state; then a second step, whose v_Hxc comes from the first step's density summed in
    4-k groups."""
    wl = W.config("twostep_g16_mp8_s4")
    insts = wl.instances
    inst_id = 19
    A = wl.field.table(2, wl.dt)
    _say("full-size two-step FP64: loading 64 sub-simulations")
    with tdks.Propagator(insts, precision="fp64", dt=wl.dt) as prop:
        u_keep = None
        for i, inst in enumerate(insts):
            u = W.random_orbitals_torch(5000 + i, inst.n_k, inst.n_bands, inst.grid, inst.omega)
            prop.load_orbitals(i, u)
            if i == inst_id:
                u_keep = u.cpu().numpy()
            del u
        til = prop.tiling()
        _say(f"  tiling {til}; two steps")
        assert til["k_per_group"] == 4 and til["zl"] == 8 and til["block"] == 512
        prop.step(A[:1])
        u1 = prop.get_orbitals(inst_id)
        vh1 = prop.vhxc(inst_id)
        prop.step(A[1:])
        u2 = prop.get_orbitals(inst_id)
        dj = prop.current()[inst_id]
    sysm = System(insts[inst_id])
    v0 = oracle_vhxc(sysm.cell, OP.density(sysm, u_keep))
    rng = np.random.default_rng(9)
    for k in rng.choice(512, 4, replace=False):
        ref = OP.taylor_step(sysm, sysm.k_cart[k] + A[0, 0], v0, u_keep[k], wl.dt)
        err = np.max(np.abs(u1[k] - ref)) / np.max(np.abs(ref))
        ref2 = OP.taylor_step(sysm, sysm.k_cart[k] + A[1, 0], vh1, u1[k], wl.dt)
        err2 = np.max(np.abs(u2[k] - ref2)) / np.max(np.abs(ref2))
        _say(f"  k {k}: orbital rel err step 1 {err:.2e}, step 2 {err2:.2e}")
        assert err < 1e-12 and err2 < 1e-12
    rho1 = OP.density(sysm, u1)
    assert np.max(np.abs(vh1 - oracle_vhxc(sysm.cell, rho1))) < 1e-11
    J0 = OP.current(sysm, np.zeros(3), u_keep)
    J2 = OP.current(sysm, A[1, 1], u2)
    err = np.max(np.abs(dj[1] - (J2 - J0)))
    _say(f"  current after 2 steps: |dJ_gpu - dJ_oracle(gpu state)| = {err:.2e}")
    assert err < 1e-10 * np.max(np.abs(J2 - J0)) + 1e-16


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_k_grouping_matches_single_k(tdks, precision):
    """Four k-points per workgroup (forced) against one: the same per-orbital arithmetic,
    the density summed in another order, so the currents agree to rounding."""
    sp = W.draw_species(np.random.default_rng(3))
    insts = [W.make_instance("diamond8", (8, 8, 8), 3, [sp], W.KSpec((4, 2, 1), (2, 2, 2), (j, 0, 1)))
             for j in range(2)]
    u0s = [W.random_orbitals(60 + i, inst.n_k, 3, (8, 8, 8), inst.omega) for i, inst in enumerate(insts)]
    A = W.Field("kick", 1e-3).table(12, 0.02)
    res = {}
    for kpg in (1, 4):
        _say(f"k grouping {kpg}, {precision}")
        with tdks.Propagator(insts, precision=precision, k_per_group=kpg) as prop:
            for i, u in enumerate(u0s):
                prop.load_orbitals(i, u)
            assert prop.tiling()["k_per_group"] == kpg
            prop.step(A)
            res[kpg] = prop.current()
    peak = np.max(np.abs(res[1]))
    err = np.max(np.abs(res[4] - res[1])) / peak
    _say(f"  max |dJ(4 k) - dJ(1 k)| / peak = {err:.2e}")
    assert err < (1e-12 if precision == "fp64" else BARS["fp32"])
