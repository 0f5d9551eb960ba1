"""Metric variants: truncated Lp (p < 1) and the votes-only ranking of Thm. 3.

Lp tolerance: the float32 query carries <= 6e-7 of distance error (see parity.py);
rho = min(d, tau)^p amplifies it by p d^(p-1), <= 16 for d >= 1e-6 at p = 0.5, so a
record's error may differ by 1e-5 |err| + 1e-5 N.  The votes ranking is integer:
bit-exact."""
import numpy as np
import pytest

import oracle
from paper_2502_00115_amd import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2502_00115_amd import dses  # noqa: E402


def _lp_tol(err, n):
    return 1e-5 * np.abs(err) + 1e-5 * n


@pytest.mark.parametrize("lp", [0.5, 0.75])
@pytest.mark.parametrize("scorer", ["brute", "grid"])
@pytest.mark.parametrize("seed", [0, 1])
def test_truncated_lp_matches_oracle(lp, scorer, seed):
    p = synth.make_c1(seed)
    n = len(p.src)
    g = dses.register(p.src, p.tgt, p.rotations, p.eps, metric="trunc_lp", lp=lp, scorer=scorer,
                      records=True)
    orc = oracle.records(p.src, p.tgt, p.rotations, p.eps, metric="trunc_lp", p=lp)
    v = orc["valid"].astype(bool)
    np.testing.assert_array_equal(g.records["votes"], orc["votes"])
    np.testing.assert_array_equal(g.records["bin"][v], orc["bin"][v])
    dinl = np.abs(g.records["inliers"][v].astype(np.int64) - orc["inliers"][v])
    assert np.all(dinl <= orc["boundary"][v])
    eg, eo = g.records["error"][v].astype(np.float64), orc["error"][v]
    bad = np.abs(eg - eo) > _lp_tol(eo, n)
    assert not bad.any(), (eg[bad][:4], eo[bad][:4])
    err = np.where(v, orc["error"], np.inf)
    best = int(np.argmin(err))
    admissible = np.nonzero(err <= err[best] + 2 * _lp_tol(err[best], n))[0]
    assert g.rot_index in admissible


def test_truncated_lp_distance_field_matches_oracle_field():
    p = synth.make_c1(2)
    T = dses.Target(p.tgt, df_trunc=p.eps, df_res=64)
    S = dses.RotationSet(p.rotations)
    g = dses.register_resident(T, S, p.src, p.eps, metric="trunc_lp", lp=0.5, scorer="df",
                               records=True)
    df = oracle.df_build(p.tgt, p.eps, 64)
    orc = oracle.records(p.src, p.tgt, p.rotations, p.eps, metric="trunc_lp", p=0.5, df=df)
    v = orc["valid"].astype(bool)
    np.testing.assert_array_equal(g.records["votes"], orc["votes"])
    eg, eo = g.records["error"][v].astype(np.float64), orc["error"][v]
    assert np.all(np.abs(eg - eo) <= _lp_tol(eo, len(p.src)))


@pytest.mark.parametrize("seed", range(4))
def test_votes_ranking_bit_exact(seed):
    p = synth.make_c1(seed)
    g = dses.register(p.src, p.tgt, p.rotations, p.eps, metric="votes", records=True, top_k=8)
    orc = oracle.records(p.src, p.tgt, p.rotations, p.eps, metric="votes")
    np.testing.assert_array_equal(g.records["votes"], orc["votes"])
    v = orc["valid"].astype(bool)
    np.testing.assert_array_equal(g.records["bin"][v], orc["bin"][v])
    np.testing.assert_array_equal(g.records["inliers"][v], orc["inliers"][v])
    assert np.all(g.records["error"][v] == 0.0)
    assert g.rot_index == oracle.select(orc)
    assert g.votes == int(orc["votes"].max()) and g.inliers == g.votes and g.error == 0.0
    np.testing.assert_array_equal(g.top["rot_index"], oracle.topk(orc, 8))


def test_votes_resident_and_rejections():
    p = synth.make_c2(3)
    rots = p.rotations[::9].copy()
    T, S = dses.Target(p.tgt), dses.RotationSet(rots)
    a = dses.register_resident(T, S, p.src, p.eps, metric="votes")
    b = dses.register(p.src, p.tgt, rots, p.eps, metric="votes")
    assert a.rot_index == b.rot_index and a.votes == b.votes
    with pytest.raises(dses.DsesError):
        dses.register(p.src, p.tgt, rots, p.eps, metric="votes", q=0.5)
    with pytest.raises(dses.DsesError):
        dses.register_batch([{"src": p.src, "tgt": p.tgt, "rotations": rots, "eps": p.eps,
                              "metric": "votes"}])
