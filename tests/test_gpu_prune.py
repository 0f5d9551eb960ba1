"""q-pruned scoring (the pruning step of Alg. 2): vote every rotation, score only
those with M_k >= q M*.  Votes and bins against the oracle's definition (within its
fragility intervals), the scored set exactly the rule applied to the votes, scored
errors within tolerance, selection inside the oracle's admissible set restricted
to the scored rotations."""
import numpy as np
import pytest

import oracle
from paper_2502_00115_amd import synth
from parity import check_selection, compare_records, err_tol

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2502_00115_amd import dses  # noqa: E402


def _gpu_mask(votes, q):
    """The pruning rule applied to a list of vote counts (M_k >= q M*, compared in
    double precision on the counts and the float q)."""
    votes = votes.astype(np.float64)
    return (votes > 0) & (votes >= np.float64(np.float32(q)) * votes.max())


def _check(g, orc, q, n, delta, label):
    # votes and bins of every rotation: the definition's, within its fragility ranges
    # (the scores of the unscored rotations are not compared)
    probe = g.records.copy()
    mask = _gpu_mask(probe["votes"], q)
    # the scored set is exactly the rule applied to the GPU's votes; when every vote
    # is pinned to the oracle's count it is the oracle's own set
    scored = np.isfinite(probe["error"])
    np.testing.assert_array_equal(scored, mask, err_msg=f"{label}: scored set")
    if np.array_equal(probe["votes"], orc["votes"]):
        np.testing.assert_array_equal(mask, oracle.prune_mask(orc, q), err_msg=label)
    assert np.all(probe["inliers"][~mask] == 0)
    rep = compare_records(probe[mask], orc[mask], n, label=label)
    unscored = ~mask & (probe["votes"] > 0)
    if unscored.any():
        # unscored candidates carry their vote: compared with the metric ignored
        rv = compare_records(probe[unscored], orc[unscored], n, scores=False,
                             label=f"{label} (unscored)")
        assert rv["rotations"] == int(unscored.sum())
    check_selection(g, rep, delta, label=label)


@pytest.mark.parametrize("seed", range(4))
@pytest.mark.parametrize("q", [0.5, 0.9, 1.0])
def test_pruned_c1_matches_oracle(seed, q):
    p = synth.make_c1(seed)
    g = dses.register(p.src, p.tgt, p.rotations, p.eps, records=True, q=q)
    orc = oracle.records(p.src, p.tgt, p.rotations, p.eps)
    _check(g, orc, q, len(p.src), p.eps, f"c1 seed {seed} q {q}")


@pytest.mark.parametrize("scorer", ["brute", "grid"])
def test_tiny_q_equals_full_scoring_bitwise(scorer):
    p = synth.make_c1(5)
    full = dses.register(p.src, p.tgt, p.rotations, p.eps, records=True, scorer=scorer)
    tiny = dses.register(p.src, p.tgt, p.rotations, p.eps, records=True, scorer=scorer, q=1e-7)
    assert full.records.tobytes() == tiny.records.tobytes()
    assert full.rot_index == tiny.rot_index


def test_pruned_resident_distance_field_and_topk():
    p = synth.make_c2(2)
    sel = np.arange(0, len(p.rotations), 11)
    rots = p.rotations[sel].copy()
    T = dses.Target(p.tgt, df_trunc=p.eps, df_res=128)
    S = dses.RotationSet(rots)
    g = dses.register_resident(T, S, p.src, p.eps, scorer="df", records=True, q=0.8, top_k=8)
    M = g.records["votes"].max()
    keep = (g.records["votes"] > 0) & (g.records["votes"].astype(np.float64)
                                       >= np.float64(np.float32(0.8)) * M)
    np.testing.assert_array_equal(np.isfinite(g.records["error"]), keep)
    full = dses.register_resident(T, S, p.src, p.eps, scorer="df", records=True)
    np.testing.assert_array_equal(g.records["votes"], full.records["votes"])
    assert g.records["error"][keep].tobytes() == full.records["error"][keep].tobytes()
    # the selection is the full run's best among the kept rotations
    e = np.where(keep, full.records["error"], np.inf)
    order = sorted(np.nonzero(keep)[0], key=lambda k: (e[k], -full.records["inliers"][k], k))
    assert g.rot_index == order[0]
    np.testing.assert_array_equal(g.top["rot_index"][:min(8, len(order))], order[:8])


def test_pruned_c2_sampled_against_oracle():
    p = synth.make_c2(0)
    g = dses.register(p.src, p.tgt, p.rotations, p.eps, records=True, q=0.85)
    M = g.records["votes"].max()
    keep = np.nonzero(np.isfinite(g.records["error"]))[0]
    assert len(keep) < len(p.rotations)
    assert np.all(g.records["votes"][keep].astype(np.float64) >= np.float64(np.float32(0.85)) * M)
    which = keep[:: max(1, len(keep) // 40)]
    orc = oracle.records(p.src, p.tgt, p.rotations, p.eps, which=which)
    compare_records(g.records[which], orc, len(p.src), label="c2 q 0.85")
    # M* of the pruned run is the largest count of the unpruned run
    full = dses.register(p.src, p.tgt, p.rotations, p.eps, records=True)
    assert full.records["votes"].tobytes() == g.records["votes"].tobytes()
    e = g.records["error"][keep]
    assert abs(float(np.min(e)) - g.error) <= err_tol(g.error, len(p.src))
