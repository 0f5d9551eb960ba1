"""Resident targets / rotation lists and the distance-field scorer vs the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2502_00115_amd import synth
from parity import check_selection, compare_records

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2502_00115_amd import dses  # noqa: E402


def test_resident_equals_plain_bitwise():
    p = synth.make_c1(2)
    plain = dses.register(p.src, p.tgt, p.rotations, p.eps, records=True)
    T = dses.Target(p.tgt)
    S = dses.RotationSet(p.rotations)
    res = dses.register_resident(T, S, p.src, p.eps, records=True)
    assert plain.records.tobytes() == res.records.tobytes()
    assert plain.rot_index == res.rot_index and plain.error == res.error
    # a second call reuses the cached grid and order
    res2 = dses.register_resident(T, S, p.src, p.eps, records=True)
    assert res2.records.tobytes() == res.records.tobytes()


@pytest.mark.parametrize("res", [16, 37, 64])
def test_distance_field_matches_oracle(res):
    p = synth.make_c1(3)
    r = np.float32(0.05)
    T = dses.Target(p.tgt, df_trunc=float(r), df_res=res)
    fld, lo, h = T.field()
    ref = oracle.df_build(p.tgt, r, res)
    np.testing.assert_array_equal(lo, ref.lo)
    np.testing.assert_array_equal(h, ref.h)
    np.testing.assert_allclose(fld.astype(np.float64), ref.field, rtol=0, atol=1e-6)


@pytest.mark.parametrize("metric", ["trunc_l2", "tls", "inliers"])
def test_df_scoring_matches_oracle(metric):
    p = synth.make_c1(6)
    tau = 0.05
    r = np.float32(max(p.eps, tau))
    res = 48
    T = dses.Target(p.tgt, df_trunc=float(r), df_res=res)
    S = dses.RotationSet(p.rotations)
    got = dses.register_resident(T, S, p.src, p.eps, metric, tau=tau, scorer="df", records=True)
    df = oracle.df_build(p.tgt, r, res)
    ref = oracle.records(p.src, p.tgt, p.rotations, p.eps, metric=metric, tau=tau, df=df)
    rep = compare_records(got.records, ref, len(p.src), metric=metric, label=f"df/{metric}")
    check_selection(got, rep, p.eps, label=f"df/{metric}")


def test_df_rejects_mismatched_truncation_and_l1():
    p = synth.make_c1(1)
    T = dses.Target(p.tgt, df_trunc=0.08, df_res=16)
    S = dses.RotationSet(p.rotations[:8])
    with pytest.raises(dses.DsesError) as e:
        dses.register_resident(T, S, p.src, p.eps, scorer="df")
    assert e.value.status == dses.DSES_E_INVAL
    with pytest.raises(dses.DsesError):
        dses.register_resident(T, S, p.src, 0.08, "trunc_l1", scorer="df")
    # AUTO uses the field only when its truncation matches max(eps, tau)
    auto = dses.register_resident(T, S, p.src, 0.08, records=True)
    df = dses.register_resident(T, S, p.src, 0.08, scorer="df", records=True)
    assert auto.records.tobytes() == df.records.tobytes()


def test_df_error_within_lipschitz_bound_of_exact():
    p = synth.make_c1_exact(2)
    res = 64
    T = dses.Target(p.tgt, df_trunc=p.eps, df_res=res)
    S = dses.RotationSet(p.rotations)
    exact = dses.register_resident(T, S, p.src, p.eps, scorer="grid", records=True)
    approx = dses.register_resident(T, S, p.src, p.eps, scorer="df", records=True)
    _, _, h = T.field()
    bound = len(p.src) * 0.5 * float(np.linalg.norm(h.astype(np.float64))) + 1e-4
    np.testing.assert_array_equal(exact.records["bin"], approx.records["bin"])
    assert np.all(np.abs(exact.records["error"] - approx.records["error"]) <= bound)
    assert approx.rot_index == p.true_index


def test_lds_atomic_probe_runs():
    free = dses.measure_lds_atomics("conflict_free")
    rnd = dses.measure_lds_atomics("random")
    for r in (free, rnd):
        assert r["adds_per_s"] > 1e11 and r["per_cu_per_cycle"] > 0.0
    assert rnd["adds_per_s"] <= free["adds_per_s"] * 1.05
