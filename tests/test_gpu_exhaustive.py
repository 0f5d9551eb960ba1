"""Alg. 1 (pure exhaustive search over rotations x lattice translations) on the GPU:
per-rotation best translations against the oracle's Alg. 1, the brute-force and
cell-grid scorers bitwise equal, and never worse than the DSES candidate."""
import numpy as np
import pytest

import oracle
from paper_2502_00115_amd import synth
from parity import err_tol

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2502_00115_amd import dses  # noqa: E402


def _compare(g, orc, n, label):
    np.testing.assert_array_equal(g.records["votes"], 1)
    eg = g.records["error"].astype(np.float64)
    eo = orc["error"]
    tol = err_tol(eo, n)
    assert np.all(np.abs(eg - eo) <= tol), (label, np.max(np.abs(eg - eo) - tol))
    same = np.all(g.records["bin"] == orc["bin"], axis=1)
    # a different translation only on a near tie of the rotation's best error
    assert np.all(same | (eg <= eo + 2 * tol)), label
    assert np.all(np.abs(g.records["inliers"][same].astype(np.int64) - orc["inliers"][same])
                  <= orc["boundary"][same]), label
    err = orc["error"]
    best = int(np.argmin(err))
    assert g.rot_index in np.nonzero(err <= err[best] + 2 * err_tol(err[best], n))[0], label


@pytest.mark.parametrize("seed", range(3))
def test_exhaustive_tiny_matches_oracle(seed):
    p = synth.make_tiny(seed, n=6, m=8, k=3, delta=0.125)
    g = dses.register_exhaustive(p.src, p.tgt, p.rotations, p.eps, t_min=-0.5, t_max=0.5,
                                 records=True, scorer="brute")
    orc = oracle.exhaustive(p.src, p.tgt, p.rotations, p.eps, t_min=-0.5, t_max=0.5)
    _compare(g, orc, len(p.src), f"tiny {seed}")


@pytest.mark.parametrize("metric", ["trunc_l2", "tls"])
def test_exhaustive_c1_matches_oracle_and_scorers_agree(metric):
    p = synth.make_c1(3)
    rots = p.rotations[-48:]                      # includes the true rotation (last)
    box = dict(t_min=-0.3, t_max=0.3)
    g = dses.register_exhaustive(p.src, p.tgt, rots, p.eps, metric, records=True,
                                 scorer="grid", **box)
    b = dses.register_exhaustive(p.src, p.tgt, rots, p.eps, metric, records=True,
                                 scorer="brute", **box)
    assert g.records.tobytes() == b.records.tobytes()
    orc = oracle.exhaustive(p.src, p.tgt, rots, p.eps, metric=metric, **box)
    _compare(g, orc, len(p.src), f"c1 {metric}")
    # DSES scores one of these translations per rotation
    d = dses.register(p.src, p.tgt, rots, p.eps, metric, records=True, **box)
    v = d.records["votes"] > 0
    assert np.all(g.records["error"][v] <= d.records["error"][v] + err_tol(d.records["error"][v],
                                                                          len(p.src)))


def test_exhaustive_rejects_unsupported_options():
    p = synth.make_tiny(0)
    with pytest.raises(dses.DsesError):
        dses.register_exhaustive(p.src, p.tgt, p.rotations, p.eps, metric="votes")
    big = np.zeros((12289, 3), np.float32)
    with pytest.raises(dses.DsesError):
        dses.register_exhaustive(big, p.tgt, p.rotations, p.eps)
