"""The tiling autotuner on the two-step workload's grid: it measures the library's
tilings on a sample, returns options the library accepts, and a run with them gives
the same current as the default tiling (to the FP32 bar)."""
import sys

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def test_autotune_two_step_sample(tmp_path):
    import paper_2112_00920_amd as tdks
    from paper_2112_00920_amd import autotune

    wl = W.config("twostep_g16_mp8_s4")
    insts = wl.instances[:8]
    best = autotune.tune(insts, "fp32", steps=2, cache=str(tmp_path / "tune.json"), verbose=True)
    print(f"autotune choice: {best}", flush=True)
    assert best and {"block_size", "waves_per_simd", "bands_per_group"} <= set(best)
    # cached: the second call returns the stored choice
    assert autotune.tune(insts, "fp32", cache=str(tmp_path / "tune.json")) == best
    inst = insts[0]
    kf = np.asarray(tdks.kpoints.from_spec(inst.kspec))[:8]
    u0 = W.random_orbitals(21, len(kf), inst.n_bands, inst.grid, inst.omega)
    A = wl.field.table(3, wl.dt)
    res = []
    for opts in ({}, best):
        with tdks.Propagator([inst], k_fracs=[kf], precision="fp32", dt=wl.dt, **opts) as p:
            p.load_orbitals(0, u0)
            p.step(A)
            res.append(p.current()[0])
    peak = np.max(np.abs(res[0]))
    assert np.max(np.abs(res[1] - res[0])) < 1e-4 * peak


def test_autotune_per_class_uneven_sample(tmp_path):
    """Per-class tuning of an uneven sample (fcc2 16^3 with 4 bands, diamond8 20^3 with 16
    bands): one rule per class, accepted by the library, and a run with the rules gives the
    same currents as the default tilings to the FP32 bar."""
    import paper_2112_00920_amd as tdks
    from paper_2112_00920_amd import autotune

    wl = W.config("uneven40")
    pick = {}
    for inst in wl.instances:
        pick.setdefault((inst.cell, tuple(inst.grid)), inst)
    insts = [pick[("fcc2", (16, 16, 16))], pick[("diamond8", (20, 20, 20))]]
    rules = autotune.tune_classes(insts, "fp32", steps=2, min_items=256, cache=str(tmp_path / "tune.json"),
                                  verbose=True, max_candidates=8)
    print(f"per-class rules: {rules}", flush=True)
    assert len(rules) == 2 and {tuple(r["grid"]) for r in rules} == {(16, 16, 16), (20, 20, 20)}
    assert [r["nonorth"] for r in rules] == [1, 0]
    u0s = [W.random_orbitals_torch(80 + i, inst.n_k, inst.n_bands, inst.grid, inst.omega)
           for i, inst in enumerate(insts)]
    A = wl.field.table(3, wl.dt)
    res = []
    for r in (None, rules):
        with tdks.Propagator(insts, precision="fp32", dt=wl.dt, tiling_rules=r) as p:
            for i, u in enumerate(u0s):
                p.load_orbitals(i, u)
            p.step(A)
            res.append(p.current())
    peak = np.max(np.abs(res[0]))
    assert np.max(np.abs(res[1] - res[0])) < 1e-4 * peak
