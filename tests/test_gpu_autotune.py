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
