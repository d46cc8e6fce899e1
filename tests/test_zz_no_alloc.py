"""GPU test of the allocation-free step (tdks_step_noalloc) through the C ABI.

Its output is compared with tdks_step's on the same inputs, to the FP64 bar (1e-10 of the
peak |delta J|) and the FP32 bar (1e-4), on two calls in a row, the second with a smaller
input (a smaller context, then fewer steps on the first); the two use the same kernels and
the same reduction order, so the currents, orbitals and densities are also bitwise equal.
A context whose partial sums exceed the static scratch array is rejected with
E_UNSUPPORTED.  Each case prints its name before it touches the GPU.
"""
import sys

import numpy as np
import pytest

import workloads as W

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


def _insts(big):
    sp = W.draw_species(np.random.default_rng(2))
    if big:
        return [W.make_instance("diamond8", (8, 8, 8), 3, [sp], W.KSpec((2, 1, 1), (2, 2, 2), (j, 1, 0)), group=0)
                for j in range(2)] + [W.make_instance("fcc2", (8, 8, 8), 2, [sp], W.KSpec((2, 1, 1)), group=1)]
    return [W.make_instance("diamond8", (6, 6, 6), 2, [sp], W.KSpec((1, 1, 1)), group=0)]


def _orbitals(insts, seed):
    return [W.random_orbitals(seed + i, inst.n_k, inst.n_bands, inst.grid, inst.omega)
            for i, inst in enumerate(insts)]


def _compare(prop_ref, prop_na, dj_ref, j_na, precision, label):
    dj_na = j_na - prop_na.current_pre()[:, None, :]
    peak = np.max(np.abs(dj_ref))
    err = np.max(np.abs(dj_na - dj_ref)) / peak
    bar = 1e-10 if precision == "fp64" else 1e-4
    _say(f"  {label}: max |dJ_noalloc - dJ_step| / peak = {err:.2e} (bar {bar:g}); "
         f"bitwise {np.array_equal(dj_na, dj_ref)}")
    assert err <= bar
    assert np.array_equal(dj_na, dj_ref)
    for i in range(prop_ref.n_inst):
        assert np.array_equal(prop_na.get_orbitals(i), prop_ref.get_orbitals(i)), (label, i)
        assert np.array_equal(prop_na.density(i), prop_ref.density(i)), (label, i)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_noalloc_step_matches_step(tdks, precision):
    import torch

    A = W.Field("kick", 1e-3).table(9, 0.02)
    cases = [("first call, 3 instances (two 8^3 cubic, one 8^3 fcc), 6 steps", True, 6),
             ("second call, smaller input: 1 instance on 6^3, 3 steps", False, 3)]
    for label, big, n in cases:
        _say(f"noalloc {precision}: {label}")
        insts = _insts(big)
        u0s = _orbitals(insts, 50 if big else 70)
        with tdks.Propagator(insts, precision=precision) as ref, \
                tdks.Propagator(insts, precision=precision) as na:
            for i, u in enumerate(u0s):
                ref.load_orbitals(i, u)
                na.load_orbitals(i, u)
            ref.step(A[:n])
            dj_ref = ref.current()
            A_dev = torch.tensor(A[:n], dtype=torch.float64, device="cuda").contiguous()
            j_dev = torch.full((len(insts), n, 3), float("nan"), dtype=torch.float64, device="cuda")
            na.step_noalloc(A_dev, j_dev)
            torch.cuda.synchronize()
            _compare(ref, na, dj_ref, j_dev.cpu().numpy(), precision, label)
            np.testing.assert_array_equal(na.check(), 0)
            with pytest.raises(tdks.TdksError) as ei:  # no trace rows for these steps
                na.current()
            assert ei.value.code == tdks._lib.E_STATE
            if big:
                # continuing on the same context with fewer steps (the step counter goes on)
                _say(f"noalloc {precision}: continued call, 2 more steps")
                ref.step(A[n:n + 2])
                dj_ref2 = ref.current()[:, n:]
                A2 = torch.tensor(A[n:n + 2], dtype=torch.float64, device="cuda").contiguous()
                j2 = torch.full((len(insts), 2, 3), float("nan"), dtype=torch.float64, device="cuda")
                na.step_noalloc(A2, j2)
                torch.cuda.synchronize()
                assert na.steps_done == n + 2
                _compare(ref, na, dj_ref2, j2.cpu().numpy(), precision, "continued call")


def test_noalloc_rejects_contexts_beyond_the_scratch(tdks):
    """Three 512-k instances on 16^3 need 3 x 512 x (8 x 4096 + 32) bytes of partial sums,
    more than the 32 MiB array: E_UNSUPPORTED before any launch (nothing loaded)."""
    import torch

    _say("noalloc: context beyond the scratch array")
    sp = W.draw_species(np.random.default_rng(2))
    insts = [W.make_instance("diamond8", (16, 16, 16), 2, [sp], W.KSpec((8, 8, 8)), group=0) for _ in range(3)]
    with tdks.Propagator(insts, precision="fp32") as p:
        A_dev = torch.zeros((2, 2, 3), dtype=torch.float64, device="cuda")
        j_dev = torch.zeros((3, 2, 3), dtype=torch.float64, device="cuda")
        with pytest.raises(tdks.TdksError) as ei:
            p.step_noalloc(A_dev, j_dev)
        assert ei.value.code == tdks._lib.E_UNSUPPORTED
        assert "32" in str(ei.value) or "scratch" in str(ei.value)
