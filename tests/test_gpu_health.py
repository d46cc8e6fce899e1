"""GPU tests of the numeric health check inside the step and of the recording stride.

The Taylor-4 step multiplies the squared norm of every eigencomponent of the Hermitian
h_kappa by |T4(-i x)|^2 = 1 - x^6/72 + x^8/576 (Eq. 1 expanded to 4th order), which is <= 1
while |x| = |dt lambda| <= 2 sqrt 2.  The device checks every step that the current and the
charge are finite and that the charge stays within the bounds this implies, and with a norm
stride every orbital's norm too; tdks_check (and tdks_current) report the first violation
per instance.  Each test prints its case before it touches the GPU.
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


def _batch():
    sp = W.draw_species(np.random.default_rng(1))
    return [W.make_instance("diamond8", (8, 8, 8), 3, [sp], W.KSpec((2, 1, 1), (2, 2, 2), (j, 1, 0)), group=0)
            for j in range(2)]


def _decode(rec):
    rec = int(rec)
    return rec >> 32, (rec >> 4) & 0xFFFFFFF, rec & 15


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("norm_stride", [0, 1])
def test_nan_instance_flagged_and_others_untouched(tdks, precision, norm_stride):
    """NaN orbitals in instance 0 of a batch: the first step flags instance 0 (non-finite),
    instance 1 stays healthy and bitwise equal to the same instance run alone; the next
    tdks_step call reports the violation."""
    _say(f"health: NaN instance, {precision}, norm_stride {norm_stride}")
    insts = _batch()
    u1 = W.random_orbitals(31, insts[1].n_k, 3, (8, 8, 8), insts[1].omega)
    bad = np.full((insts[0].n_k, 3, 8, 8, 8), np.nan, dtype=complex)
    A = W.Field("kick", 1e-3).table(6, 0.02)
    with tdks.Propagator(insts, precision=precision, norm_stride=norm_stride) as prop:
        prop.load_orbitals(0, bad)
        prop.load_orbitals(1, u1)
        prop.step(A[:3])
        with pytest.raises(tdks.TdksError) as ei:
            prop.check()
        assert ei.value.code == tdks._lib.E_NUMERIC
        assert "instance 0, step 1" in str(ei.value), str(ei.value)
        step, orb, code = _decode(ei.value.info[0])
        assert step == 1 and code == 1
        assert int(ei.value.info[1]) == 0
        with pytest.raises(tdks.TdksError) as e2:  # the next step call refuses
            prop.step(A[3:])
        assert e2.value.code == tdks._lib.E_NUMERIC
        with pytest.raises(tdks.TdksError):
            prop.current()
        u_b = prop.get_orbitals(1)
        rho_b = prop.density(1)
        j_b = prop.current_at([0.0, 0.0, 0.0])[1]
    with tdks.Propagator([insts[1]], precision=precision, norm_stride=norm_stride) as alone:
        alone.load_orbitals(0, u1)
        alone.step(A[:3])
        assert int(alone.check()[0]) == 0
        assert np.array_equal(alone.get_orbitals(0), u_b)
        assert np.array_equal(alone.density(0), rho_b)
        assert np.array_equal(alone.current_at([0.0, 0.0, 0.0])[0], j_b)


@pytest.mark.parametrize("norm_stride,codes", [(0, (2, 1)), (1, (4, 1))])
def test_unstable_step_flagged(tdks, norm_stride, codes):
    """dt = 1 puts the top of the FD spectrum at x = dt lambda > 2 sqrt 2, where
    |T4(-i x)|^2 > 1: the norm grows and the check flags it (charge above its value at the
    load, or with the per-orbital check an orbital's norm; non-finite once it overflows)."""
    _say(f"health: unstable dt, norm_stride {norm_stride}")
    insts = _batch()[:1]
    u0 = W.random_orbitals(32, insts[0].n_k, 3, (8, 8, 8), insts[0].omega)
    A = W.Field("kick", 1e-3).table(12, 1.0)
    with tdks.Propagator(insts, precision="fp64", dt=1.0, norm_stride=norm_stride) as prop:
        prop.load_orbitals(0, u0)
        prop.step(A)
        with pytest.raises(tdks.TdksError) as ei:
            prop.check()
    step, orb, code = _decode(ei.value.info[0])
    _say(f"  flagged at step {step}, code {code}, orbital field {orb}: {ei.value}")
    assert code in codes and 1 <= step <= 12
    if code == 4:
        assert orb >= 1 and "band" in str(ei.value)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_healthy_runs_pass_and_record_stride(tdks, precision):
    """A kick and a strong pulse on a batch with both checks every step raise nothing; with
    record_stride 4 the recorded currents are bitwise those of every 4th step of the
    every-step run, and the health record stays clean after 2 + 38 steps (split calls)."""
    _say(f"health: healthy run, record stride, {precision}")
    insts = _batch()
    u0s = [W.random_orbitals(40 + i, inst.n_k, 3, (8, 8, 8), inst.omega) for i, inst in enumerate(insts)]
    pulse = W.Field("pulse", A0=0.03 / 0.0285, omega=0.0285, T=1653.7)
    for field, start in ((W.Field("kick", 1e-3), 0), (pulse, 41342)):  # the pulse at its peak
        A = field.table(40, 0.02, start=start)
        res = {}
        for stride in (1, 4):
            with tdks.Propagator(insts, precision=precision, norm_stride=1, record_stride=stride) as prop:
                for i, u in enumerate(u0s):
                    prop.load_orbitals(i, u)
                prop.step(A[:2])
                prop.step(A[2:])
                assert prop.steps_done == 40
                np.testing.assert_array_equal(prop.check(), 0)
                res[stride] = prop.current()
        assert res[4].shape == (2, 10, 3)
        assert np.array_equal(res[4], res[1][:, 3::4]), field.kind
