"""Comparison of HIP-path results with the CPU oracle (test helper).

Tolerances (float32 kernel vs float64 oracle):
  * mode bins and vote counts: bit-exact (both take the bin decision in float32
    by the same documented formula);
  * inliers: may differ only by points whose oracle distance is within 1e-6 of
    eps (reported by the oracle as `boundary`);
  * error: |gpu - oracle| <= 1e-5 |oracle| + 1e-6 sqrt(N).  A float32 query
    q = R x + t carries about 1-3 ulp of error per coordinate, i.e. <= ~6e-7 in a
    distance and ~2.5e-7 rms; summed with random signs over N points that is
    ~2.5e-7 sqrt(N), bounded here with a 4x margin, plus the 1e-5 relative term
    the registration contract states;
  * selected rotation: equal to the oracle's when the oracle's minimum is unique
    beyond twice the error tolerance, else inside that admissible set;
  * translation: |t_gpu - t_oracle| <= 1e-5 max(|t_oracle|, delta).
"""
import numpy as np


def err_tol(err, n):
    return 1e-5 * np.abs(err) + 1e-6 * np.sqrt(n)


def compare_records(gpu, orc, n, metric="trunc_l2", label=""):
    """Per-rotation parity; returns a small report dict."""
    assert len(gpu) == len(orc), label
    valid_o = orc["valid"].astype(bool)
    valid_g = gpu["votes"] > 0
    np.testing.assert_array_equal(valid_g, valid_o, err_msg=f"{label}: validity")
    np.testing.assert_array_equal(gpu["votes"], orc["votes"], err_msg=f"{label}: votes")
    np.testing.assert_array_equal(gpu["bin"][valid_o], orc["bin"][valid_o],
                                  err_msg=f"{label}: mode bins")
    dinl = np.abs(gpu["inliers"][valid_o].astype(np.int64) - orc["inliers"][valid_o])
    assert np.all(dinl <= orc["boundary"][valid_o]), f"{label}: inliers beyond boundary points"
    eg = gpu["error"][valid_o].astype(np.float64)
    eo = orc["error"][valid_o]
    if metric == "inliers":
        assert np.all(np.abs(eg - eo) <= orc["boundary"][valid_o]), f"{label}: L0 error"
        worst = float(np.max(np.abs(eg - eo), initial=0.0))
    else:
        bad = np.abs(eg - eo) > err_tol(eo, n)
        assert not bad.any(), (f"{label}: error mismatch at {np.nonzero(bad)[0][:5]}: "
                               f"gpu {eg[bad][:5]} oracle {eo[bad][:5]}")
        worst = float(np.max(np.abs(eg - eo) / np.maximum(err_tol(eo, n), 1e-30), initial=0.0))
    return {"rotations": int(len(orc)), "invalid": int((~valid_o).sum()),
            "boundary_points": int(orc["boundary"].sum()), "worst_err_over_tol": worst}


def check_selection(got, orc_recs, n, delta, metric="trunc_l2", which=None, label=""):
    """got: dses.Registration; orc_recs: oracle records over `which` (default: all)."""
    which = np.arange(len(orc_recs)) if which is None else np.asarray(which)
    valid = orc_recs["valid"].astype(bool)
    err = np.where(valid, orc_recs["error"], np.inf)
    best = int(np.argmin(err))
    tol = (orc_recs["boundary"].max() + 1e-9) if metric == "inliers" else err_tol(err[best], n)
    admissible = which[err <= err[best] + 2 * tol]
    assert got.rot_index in admissible, (f"{label}: gpu picked {got.rot_index}, oracle best "
                                         f"{which[best]} (admissible {admissible[:8]})")
    if len(admissible) == 1:
        assert got.rot_index == which[best], label
    pos = int(np.nonzero(which == got.rot_index)[0][0])
    r = orc_recs[pos]
    t_orc = r["bin"].astype(np.float64) * float(np.float32(delta))
    assert np.all(np.abs(got.t - t_orc) <= 1e-5 * np.maximum(np.abs(t_orc), delta)), label
    assert abs(got.inliers - int(r["inliers"])) <= int(r["boundary"]), label
    if metric != "inliers":
        assert abs(got.error - r["error"]) <= err_tol(r["error"], n), label
    return len(admissible)
