"""Comparison of HIP-path results with the CPU oracle (test helper).

The oracle evaluates Alg. 2 by its definition in double precision (see
oracle/dses_oracle.c): every pair votes for floor((y - R x)/delta + 1/2), and a
pair within the fragility margin mu of a bin face may go either way for any
evaluation accurate to mu.  The bar, per rotation:

  * validity: the GPU has a vote exactly where the oracle surely has one
    (lo_max >= 1) and none where it surely has none;
  * mode: for a pinned rotation the GPU's bin is the oracle's b*; for an
    ambiguous one it is an admissible bin (cnt + in >= max over bins of cnt - out),
    checked by re-running the oracle's vote for that rotation;
  * votes: the GPU's count of its bin lies in [cnt - out, cnt + in] of that bin
    and is at least max over bins of (cnt - out);
  * inliers: may differ only by points whose oracle distance is within 1e-6 of
    eps (reported by the oracle as `boundary`) or whose distance-field voxel is
    fragile (`inl_frag`);
  * error: within [err_lo - tol, err_hi + tol] of the oracle's score of the GPU's
    bin (err_lo = err_hi = the score for exact scorers), with
    tol = 1e-5 |err| + 1e-6 sqrt(N): a float32 query q = R x + t carries about
    1-3 ulp of error per coordinate, i.e. <= ~6e-7 in a distance and ~2.5e-7 rms;
    summed with random signs over N points that is ~2.5e-7 sqrt(N), bounded here
    with a 4x margin, plus the 1e-5 relative term the registration contract states;
  * selected rotation: inside the admissible winner set W = {k : err_lo_k - tol
    <= min_k' (err_hi_k' + tol)} over the oracle's scores of the GPU's bins, equal
    to the oracle's unique choice when |W| = 1;
  * translation: |t_gpu - delta b| <= 1e-5 max(|delta b|, delta) for the GPU's bin b.

A secondary, labelled check (`compare_library_formula`) compares bins and votes
bit for bit with the library's documented fixed-point bin formula.
"""
import numpy as np

import oracle


def err_tol(err, n):
    return 1e-5 * np.abs(err) + 1e-6 * np.sqrt(n)


def compare_records(gpu, orc, n, metric="trunc_l2", label="", tol=None, scores=True):
    """Per-rotation parity of GPU records (dses RECORD_DTYPE) with oracle Records.

    tol: a function (err, n) -> tolerance, or an array of absolute tolerances, one
    per record (default err_tol).  scores=False compares validity, modes and votes
    only (candidates left unscored).  Returns a report dict with, per compared
    rotation, the oracle's score of the GPU's bin ('err', 'err_lo', 'err_hi', 'inl',
    'bnd', 'ifr'; inf / 0 where the GPU has no candidate), the range of counts of
    the GPU's bin ('vlo', 'vhi') and counts of ambiguous rotations."""
    assert len(gpu) == len(orc), label
    tol = err_tol if tol is None else tol
    if not callable(tol):
        arr = np.asarray(tol, np.float64)
        assert arr.shape == (len(gpu),), label
        tol = _PerRecordTol(arr)
    ctx = orc.ctx
    rot = orc["rot"].astype(np.int64)
    gv = gpu["votes"] > 0
    ov = orc["valid"].astype(bool)
    pinned = orc["pinned"].astype(bool)
    lo_max = orc["lo_max"].astype(np.int64)
    surely_valid = lo_max >= 1
    surely_invalid = pinned & ~ov
    bad = np.nonzero((gv & surely_invalid) | (~gv & surely_valid))[0]
    assert bad.size == 0, f"{label}: validity differs at rotations {rot[bad][:5]}"

    g_votes = gpu["votes"].astype(np.int64)
    same = gv & ov & np.all(gpu["bin"] == orc["bin"], axis=1)
    bad = np.nonzero(pinned & ov & ~same)[0]
    assert bad.size == 0, (f"{label}: pinned mode differs at rotations {rot[bad][:5]}: "
                           f"gpu {gpu['bin'][bad][:3].tolist()} oracle {orc['bin'][bad][:3].tolist()}")
    lo = orc["votes_lo"].astype(np.int64)
    hi = orc["votes_hi"].astype(np.int64)
    ok = (g_votes >= lo) & (g_votes <= hi) & (g_votes >= lo_max)
    bad = np.nonzero(same & ~ok)[0]
    assert bad.size == 0, (f"{label}: votes outside [cnt - out, cnt + in] at rotations "
                           f"{rot[bad][:5]}: gpu {g_votes[bad][:5]} range "
                           f"{list(zip(lo[bad][:5], hi[bad][:5]))}")

    vlo = np.where(gv, lo, 0)
    vhi = np.where(gv, hi, 0)
    # rotations where the GPU took another (necessarily ambiguous) bin
    moved = np.nonzero(gv & ~same)[0]
    for u in moved:
        _, blo, bhi, L = oracle.bin_bounds(ctx, rot[u], gpu["bin"][u])
        vlo[u], vhi[u] = blo, bhi
        v = int(g_votes[u])
        assert bhi > 0 and bhi >= L, (f"{label}: rotation {rot[u]}: gpu bin "
                                      f"{gpu['bin'][u].tolist()} is not an admissible mode "
                                      f"(hi {bhi} < {L})")
        assert blo <= v <= bhi and v >= L, (f"{label}: rotation {rot[u]}: gpu votes {v} "
                                            f"outside [{blo}, {bhi}] / below {L}")

    # the oracle's score of the GPU's bin
    err = np.where(gv, orc["error"], np.inf)
    err_lo = np.where(gv, orc["err_lo"], np.inf)
    err_hi = np.where(gv, orc["err_hi"], np.inf)
    inl = np.where(gv, orc["inliers"], 0).astype(np.int64)
    bnd = np.where(gv, orc["boundary"], 0).astype(np.int64)
    ifr = np.where(gv, orc["inl_frag"], 0).astype(np.int64)
    if not scores:
        return {"rot": rot, "gpu_valid": gv, "vlo": vlo, "vhi": vhi,
                "gpu_bin": gpu["bin"].copy(), "rotations": int(len(orc)),
                "ambiguous": int((~pinned).sum()), "moved": int(moved.size)}
    if metric == "votes":
        inl = np.where(gv, g_votes, 0)
        err = np.where(gv, 0.0, np.inf)
        err_lo, err_hi = err.copy(), err.copy()
        bad = np.nonzero(gv & ((gpu["inliers"].astype(np.int64) != g_votes)
                               | (gpu["error"] != 0.0)))[0]
        assert bad.size == 0, f"{label}: votes ranking records at rotations {rot[bad][:5]}"
    elif moved.size:
        sc = oracle.score_bins(ctx, rot[moved], gpu["bin"][moved])
        err[moved], err_lo[moved], err_hi[moved] = sc["error"], sc["err_lo"], sc["err_hi"]
        inl[moved], bnd[moved], ifr[moved] = sc["inliers"], sc["boundary"], sc["inl_frag"]

    dinl = np.abs(gpu["inliers"].astype(np.int64) - inl)
    bad = np.nonzero(gv & (dinl > bnd + ifr))[0]
    assert bad.size == 0, (f"{label}: inliers beyond boundary points at rotations {rot[bad][:5]}:"
                           f" gpu {gpu['inliers'][bad][:5]} oracle {inl[bad][:5]}")
    eg = gpu["error"].astype(np.float64)
    tol_arr = np.zeros(len(gpu))
    if metric == "inliers":
        # error = N - inliers: the same allowance as the inlier count
        tol_arr = (bnd + ifr).astype(np.float64)
        bad = np.nonzero(gv & (np.abs(eg - err) > bnd + ifr))[0]
        worst = float(np.max(np.abs(eg - err)[gv], initial=0.0))
    elif metric == "votes":
        bad = np.zeros(0, np.int64)
        worst = 0.0
    else:
        t_lo = tol(err_lo, n)
        t_hi = tol(err_hi, n)
        tol_arr = np.where(gv, np.maximum(t_lo, t_hi), 0.0)
        with np.errstate(invalid="ignore"):
            outside = (eg < err_lo - t_lo) | (eg > err_hi + t_hi)
        bad = np.nonzero(gv & outside)[0]
        with np.errstate(invalid="ignore", divide="ignore"):
            dev = np.maximum(err_lo - eg, eg - err_hi) / np.maximum(tol(err, n), 1e-30)
        worst = float(np.max(dev[gv], initial=0.0))
    assert bad.size == 0, (f"{label}: error mismatch at rotations {rot[bad][:5]}: "
                           f"gpu {eg[bad][:5]} oracle {err[bad][:5]} "
                           f"[{err_lo[bad][:5]}, {err_hi[bad][:5]}]")
    return {"rot": rot, "gpu_valid": gv, "err": err, "err_lo": err_lo, "err_hi": err_hi,
            "inl": inl, "bnd": bnd, "ifr": ifr, "vlo": vlo, "vhi": vhi, "tol_arr": tol_arr,
            "gpu_bin": gpu["bin"].copy(),
            "rotations": int(len(orc)), "invalid": int((~gv).sum()),
            "ambiguous": int((~pinned).sum()), "moved": int(moved.size),
            "fragile_pairs": int(orc["frag"].sum()), "boundary_points": int(bnd.sum()),
            "worst_err_over_tol": worst, "metric": metric, "n": n}


class _PerRecordTol:
    """An array of absolute tolerances in the place of a tolerance function."""

    def __init__(self, arr):
        self.arr = arr

    def __call__(self, err, n):
        return self.arr


def admissible_winners(rep, among=None):
    """W over the compared rotations (optionally restricted to a boolean mask)."""
    ok = rep["gpu_valid"] if among is None else (rep["gpu_valid"] & among)
    if not ok.any():
        return rep["rot"][:0]
    if rep["metric"] == "votes":
        # ranked by the mode count (Thm. 3): a rotation can win when its count can
        # reach the largest count some rotation surely has
        best_lo = int(np.max(np.where(ok, rep["vlo"], -1)))
        return rep["rot"][ok & (rep["vhi"] >= best_lo)]
    lo = rep["err_lo"] - rep["tol_arr"]
    hi = rep["err_hi"] + rep["tol_arr"]
    best_hi = float(np.min(np.where(ok, hi, np.inf)))
    return rep["rot"][ok & (lo <= best_hi)]


def check_selection(got, rep, delta, label="", among=None):
    """got: dses.Registration; rep: compare_records() report over rotations that
    include every candidate the selection could have taken (all of them, or a set
    holding the GPU's own best candidates)."""
    W = admissible_winners(rep, among)
    assert got.rot_index in W, (f"{label}: gpu picked {got.rot_index}, admissible "
                                f"{W[:8]} (oracle best score "
                                f"{np.min(np.where(rep['gpu_valid'], rep['err'], np.inf))})")
    if len(W) == 1:
        assert got.rot_index == W[0], label
    pos = int(np.nonzero(rep["rot"] == got.rot_index)[0][0])
    b = rep["gpu_bin"][pos].astype(np.float64)
    t_orc = b * float(np.float32(delta))
    assert np.all(np.abs(got.t - t_orc) <= 1e-5 * np.maximum(np.abs(t_orc), delta)), label
    assert abs(got.inliers - int(rep["inl"][pos])) <= int(rep["bnd"][pos] + rep["ifr"][pos]), label
    if rep["metric"] not in ("inliers", "votes"):
        t = rep["tol_arr"][pos]
        assert rep["err_lo"][pos] - t <= got.error <= rep["err_hi"][pos] + t, label
    return len(W)


def compare_library_formula(gpu, src, tgt, rotations, eps, which=None, label="", zbits=15, **kw):
    """SECONDARY, labelled check of the kernel's arithmetic: bins and votes bit for bit
    equal to the library's documented fixed-point bin formula (z at 2^-zbits bins:
    15 with 16-bit counters, 16 with 32-bit ones)."""
    ref = oracle.records(src, tgt, rotations, eps, which=which,
                         vote="lib" if zbits == 15 else "lib32", metric="votes", **kw)
    np.testing.assert_array_equal(gpu["votes"], ref["votes"],
                                  err_msg=f"{label}: votes (library fixed-point formula)")
    v = ref["valid"].astype(bool)
    np.testing.assert_array_equal(gpu["bin"][v], ref["bin"][v],
                                  err_msg=f"{label}: bins (library fixed-point formula)")
