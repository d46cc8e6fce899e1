"""Host-side library code against the oracle: k-point generation (bit-exact) and
the spectra used for the two-step average (Eqs. (8)-(10), (12)-(16))."""
import numpy as np
import pytest

import workloads as W
from oracle import kpoints as ok
from oracle import spectra as osp
from paper_2112_00920_amd import kpoints as pk
from paper_2112_00920_amd import spectra as ps


@pytest.mark.parametrize("coarse,shifts", [((2, 2, 2), None), ((8, 8, 8), None), ((3, 1, 2), None),
                                           ((8, 8, 8), (4, 4, 4)), ((4, 4, 4), (2, 2, 2)), ((6, 6, 6), None)])
def test_kpoints_bit_exact(coarse, shifts):
    idxs = [None] if shifts is None else [(0, 0, 0), (1 % shifts[0], 2 % shifts[1], 3 % shifts[2]), tuple(s - 1 for s in shifts)]
    for idx in idxs:
        spec = W.KSpec(coarse, shifts, idx)
        assert np.array_equal(pk.from_spec(spec), ok.kset(spec))


def test_halton_matches_oracle():
    assert np.array_equal(pk.halton_shifts(20), ok.halton(20))


def test_two_step_union_is_dense_grid():
    dense = {tuple(x) for x in pk.mp_grid((8, 8, 8)).tolist()}
    union = []
    for j3 in range(2):
        for j2 in range(2):
            for j1 in range(2):
                union += [tuple(x) for x in pk.shifted_grid((4, 4, 4), (2, 2, 2), (j1, j2, j3)).tolist()]
    assert len(union) == 512 and set(union) == dense


def test_spectra_match_oracle():
    rng = np.random.default_rng(0)
    t = np.arange(0, 200.0, 0.02)
    dj = rng.standard_normal(len(t)) * 1e-5
    om = np.linspace(0.05, 1.0, 20)
    s1, e1 = ps.dielectric_function(t, dj, 1e-3, om, 0.005)
    s2 = osp.conductivity(t, dj, 1e-3, om, 0.005)
    np.testing.assert_allclose(s1, s2, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(e1, osp.dielectric(s2, om), rtol=1e-12)
    np.testing.assert_allclose(ps.hhg_spectrum(t, dj, 150.0, om), osp.hhg_spectrum(t, dj, 150.0, om),
                               rtol=1e-10, atol=1e-30)
    m, sem = ps.group_mean_and_sem(np.stack([dj, 2 * dj, 3 * dj]))
    np.testing.assert_allclose(sem, osp.standard_error(np.stack([dj, 2 * dj, 3 * dj])), rtol=1e-12)


@pytest.mark.parametrize("name", ["twostep_g16_mp8_halton64", "twostep_g16_mp8_random64"])
def test_halton_and_random_shift_ksets_bit_exact(name):
    for inst in W.config(name).instances:
        assert np.array_equal(pk.from_spec(inst.kspec), ok.kset(inst.kspec))


def test_kspec_errors():
    with pytest.raises(ValueError):
        pk.from_spec(W.KSpec((2, 2, 2), (2, 2, 2), (0, 0, 0), halton_index=3))
    with pytest.raises(ValueError):
        pk.from_spec(W.KSpec((2, 2, 2), halton_index=0))
    with pytest.raises(ValueError):
        pk.from_spec(W.KSpec((2, 2, 2), shift_q=(0.5, 1.0, 0.2)))


def test_nh_convergence_matches_oracle():
    rng = np.random.default_rng(3)
    t = np.arange(0, 100.0, 0.02)
    dj = rng.standard_normal((9, len(t), 3)) * 1e-5
    om = np.linspace(0.05, 1.0, 15)
    rows = ps.nh_convergence(t, dj, 1e-3, om, axis=1)
    assert [r["n_h"] for r in rows] == [1, 2, 4, 8, 9]
    ref = osp.nh_convergence(t, dj[:, :, 1], 1e-3, om, [1, 2, 4, 8, 9])
    for r, (n, eps, sem) in zip(rows, ref):
        assert r["n_h"] == n
        np.testing.assert_allclose(r["eps"], eps, rtol=1e-12)
        np.testing.assert_allclose(r["eps_sem"].real, sem.real, rtol=1e-10, atol=1e-15)
        np.testing.assert_allclose(r["eps_sem"].imag, sem.imag, rtol=1e-10, atol=1e-15)
        np.testing.assert_allclose(r["dj_mean"], dj[:n, :, 1].mean(axis=0), rtol=1e-12)
    assert rows[-1]["dev"] == 0.0


def test_harness_table_rows():
    from paper_2112_00920_amd import harness

    rng = np.random.default_rng(11)
    t = np.arange(1, 501) * 0.02
    dj = rng.standard_normal((5, len(t), 3)) * 1e-5
    om = np.linspace(0.1, 1.0, 9)
    rows = harness.table(t, dj, 1e-3, om)
    assert [r["n_h"] for r in rows] == [1, 2, 4, 5]
    assert rows[0]["mean_sem_im_eps"] == 0.0 and rows[-1]["max_dev_eps"] == 0.0
    full = ps.nh_convergence(t, dj, 1e-3, om)
    for r, f in zip(rows, full):
        assert r["max_dev_eps"] == f["dev"]
        assert abs(r["max_sem_im_eps"] - float(np.max(f["eps_sem"].imag))) == 0.0
