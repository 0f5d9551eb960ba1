"""CPU oracle for DSES -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it.

The arithmetic lives in ``dses_oracle.c`` (plain C, IEEE double throughout).
This module marshals numpy arrays through ctypes and derives the fragility
margins from the inputs' magnitudes.

Paper steps covered (Cheng et al., arXiv 2502.00115):
  * ``vote64``    -- Lemma 2 / Eq. (5) and the first loop of Alg. 2 by the
                     definition: every pair votes for floor((y - R x)/delta + 1/2),
                     with the counts of pairs within a margin of a bin face, the
                     mode and whether it is pinned.
  * ``nn``        -- Eq. (1)/(2) nearest-neighbour distance, brute force.
  * ``records``   -- Alg. 2 with q = 0: every candidate {R, t*} scored.
  * ``score_bins``-- the error loop of Alg. 2 for given (rotation, bin) pairs.
  * ``select``    -- the argmin return of Alg. 2.
  * ``exhaustive``-- Alg. 1 over the same rotations and lattice.
  * ``df_build``  -- voxel distance field of the reference cloud (scoring
                     variant; not in the paper, defined in the library header).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build_oracle

METRICS = {"trunc_l2": 0, "inliers": 1, "tls": 2, "trunc_l1": 3, "trunc_lp": 4, "votes": 5}
DF_LOOKUPS = {"nearest": 0, "trilinear": 1}
# vote= of records(): the definition, or the library's formulas with z at 2^-15 / 2^-16 bins
_LIB_ZBITS = {"f64": 0, "lib": 15, "lib32": 16}

RECORD_DTYPE = np.dtype([("bin", "<i4", (3,)), ("votes", "<u4"), ("inliers", "<i4"),
                         ("boundary", "<i4"), ("error", "<f8"), ("valid", "<i4"),
                         ("rot", "<i4"), ("votes_lo", "<u4"), ("votes_hi", "<u4"),
                         ("lo_max", "<u4"), ("pinned", "<i4"), ("frag", "<i4"),
                         ("inl_frag", "<i4"), ("err_lo", "<f8"), ("err_hi", "<f8")])
assert RECORD_DTYPE.itemsize == 80

# float32 unit roundoff
_U32 = 2.0 ** -24

_lib = None


def lib():
    global _lib
    if _lib is None:
        # DSES_ORACLE_LIB: a prebuilt variant of this library (the sanitizer test's)
        path = os.environ.get("DSES_ORACLE_LIB") or build_oracle(force=False)
        L = C.CDLL(path)
        fp, dp, ip, up = (C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                          C.POINTER(C.c_uint32))
        i32, f32, f64, vp = C.c_int32, C.c_float, C.c_double, C.c_void_p
        L.orc_box.argtypes = [f32, fp, fp, ip, ip]
        L.orc_box.restype = C.c_int
        L.orc_vote64.argtypes = [fp, i32, fp, i32, fp, f32, f64, ip, ip, up, up, up, ip]
        L.orc_vote64.restype = C.c_int
        L.orc_vote_lib.argtypes = [fp, i32, fp, i32, fp, f32, i32, ip, ip, up, ip]
        L.orc_vote_lib.restype = C.c_uint32
        L.orc_nn.argtypes = [dp, i32, fp, i32, i32, dp]
        L.orc_nn.restype = None
        L.orc_df_build.argtypes = [fp, i32, f32, i32, i32, fp, fp, fp, dp]
        L.orc_df_build.restype = C.c_int
        L.orc_records.argtypes = [fp, i32, fp, i32, fp, i32, ip, i32, f32, f32, f32, fp, fp,
                                  i32, f32, f64, i32, dp, i32, fp, fp, fp, i32, f64, i32, vp]
        L.orc_records.restype = C.c_int
        L.orc_score_bins.argtypes = [fp, i32, fp, i32, fp, i32, ip, ip, i32, f32, f32, f32, i32,
                                     f32, i32, dp, i32, fp, fp, fp, i32, f64, i32, vp]
        L.orc_score_bins.restype = C.c_int
        L.orc_df_query.argtypes = [dp, i32, dp, i32, f32, fp, fp, i32, f64, dp, dp, dp]
        L.orc_df_query.restype = C.c_int
        L.orc_select.argtypes = [vp, i32]
        L.orc_select.restype = C.c_int32
        L.orc_exhaustive.argtypes = [fp, i32, fp, i32, fp, i32, f32, f32, f32, fp, fp, i32, f32,
                                     i32, vp]
        L.orc_exhaustive.restype = C.c_int
        _lib = L
    return _lib


def _f32(a, shape_last=None):
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
    if shape_last is not None:
        a = a.reshape(-1, shape_last)
    return a


def _p(a, t):
    return a.ctypes.data_as(C.POINTER(t))


def _box_args(t_min, t_max):
    t_min = _f32(np.broadcast_to(np.asarray(-1.0 if t_min is None else t_min, np.float32), 3))
    t_max = _f32(np.broadcast_to(np.asarray(1.0 if t_max is None else t_max, np.float32), 3))
    return t_min, t_max


def box(delta, t_min=None, t_max=None):
    """Lattice range of the translation box: (k_lo[3], size[3])."""
    t_min, t_max = _box_args(t_min, t_max)
    k_lo = np.zeros(3, np.int32)
    size = np.zeros(3, np.int32)
    if lib().orc_box(C.c_float(delta), _p(t_min, C.c_float), _p(t_max, C.c_float),
                     _p(k_lo, C.c_int32), _p(size, C.c_int32)):
        raise ValueError("invalid translation box")
    return k_lo, size


# ---------------------------------------------------------------------------
# fragility margins
# ---------------------------------------------------------------------------
def vote_margin(src, tgt, delta, t_min=None, t_max=None):
    """Fragility margin mu of the bin decision, in bin units: 1e-4.

    The library takes the decision on integers: the reference coordinate y/delta
    + 1/2 - k_lo and the rotated source coordinate (R x)/delta, each evaluated in
    double and rounded to a multiple of 2^-16 bins (2^-15 on z with 16-bit
    counters), are subtracted exactly.  Each rounding moves a value by at most half
    a unit, so u + 1/2 is off by at most 2^-15 bins plus double rounding (below
    1e-9 bins at any admitted coordinate), whatever the magnitudes: mu = 1e-4
    covers it three times over.  The arguments are kept for the callers that pass
    a problem; the margin does not depend on them.
    """
    return 1e-4


def df_margin(src, df, t_min=None, t_max=None):
    """Fragility margin of the nearest-voxel decision, in voxel units: a float32
    query q = R x + t and (q - lo) * (1/h) take a handful of roundings of
    magnitudes bounded by |x|, |t|, |q| <= |x| + |t| and |lo|, each relative
    2^-24, plus the rounding of 1/h and of the product (at most res voxels)."""
    t_min, t_max = _box_args(t_min, t_max)
    x = float(np.linalg.norm(_f32(src, 3).astype(np.float64), axis=1).max(initial=0.0))
    t = float(max(np.abs(t_min).max(), np.abs(t_max).max()))
    lo = float(np.abs(df.lo).max())
    h = float(np.min(df.h))
    return max(1e-4, 32 * _U32 * (2 * x + 2 * t + lo + 1.0) / h + 4 * _U32 * df.res)


# ---------------------------------------------------------------------------
# vote of one rotation
# ---------------------------------------------------------------------------
def vote64(src, tgt, R, delta, t_min=None, t_max=None, mu=None):
    """Vote of one rotation by the definition (Lemma 2, Alg. 2's first loop).

    Returns (cnt, out, in, info): dense (size_x, size_y, size_z) arrays of the
    counts, the fragile pairs counted in a bin that may belong elsewhere, the
    fragile pairs that may belong to a bin; info = dict(mode, M, lo, hi, lo_max,
    pinned, frag, mu)."""
    src, tgt = _f32(src, 3), _f32(tgt, 3)
    R = _f32(R).reshape(9)
    k_lo, size = box(delta, t_min, t_max)
    if mu is None:
        mu = vote_margin(src, tgt, delta, t_min, t_max)
    shape = tuple(int(s) for s in size)
    cnt, out, inn = (np.zeros(shape, np.uint32) for _ in range(3))
    info = np.zeros(9, np.int32)
    rc = lib().orc_vote64(_p(src, C.c_float), len(src), _p(tgt, C.c_float), len(tgt),
                          _p(R, C.c_float), C.c_float(delta), C.c_double(mu),
                          _p(k_lo, C.c_int32), _p(size, C.c_int32), _p(cnt, C.c_uint32),
                          _p(out, C.c_uint32), _p(inn, C.c_uint32), _p(info, C.c_int32))
    if rc:
        raise ValueError("oracle rejected the input")
    return cnt, out, inn, {"mode": tuple(int(v) for v in info[:3]), "M": int(info[3]),
                           "lo": int(info[4]), "hi": int(info[5]), "lo_max": int(info[6]),
                           "pinned": bool(info[7]), "frag": int(info[8]), "mu": mu,
                           "k_lo": k_lo, "size": size}


def vote_lib(src, tgt, R, delta, t_min=None, t_max=None, zbits=15):
    """SECONDARY: the vote by the library's documented fixed-point bin formula, z at
    2^-zbits bins (15 with 16-bit counters, 16 with 32-bit ones): dense counts,
    mode, M.  Used only for a labelled bit-exactness check."""
    src, tgt = _f32(src, 3), _f32(tgt, 3)
    R = _f32(R).reshape(9)
    k_lo, size = box(delta, t_min, t_max)
    hist = np.zeros(tuple(int(s) for s in size), np.uint32)
    mode = np.zeros(3, np.int32)
    M = lib().orc_vote_lib(_p(src, C.c_float), len(src), _p(tgt, C.c_float), len(tgt),
                           _p(R, C.c_float), C.c_float(delta), int(zbits), _p(k_lo, C.c_int32),
                           _p(size, C.c_int32), _p(hist, C.c_uint32), _p(mode, C.c_int32))
    return hist, mode, int(M)


def vote(src, tgt, R, delta, t_min=None, t_max=None):
    """Vote array (size_x, size_y, size_z) of one rotation by the definition, its
    mode bin and frequency M."""
    cnt, _, _, info = vote64(src, tgt, R, delta, t_min, t_max)
    return cnt, np.array(info["mode"], np.int32), info["M"]


def nn(q, tgt, l1=False):
    """Brute-force nearest-neighbour distances (double) of queries q to the reference."""
    q = np.ascontiguousarray(np.asarray(q, np.float64).reshape(-1, 3))
    tgt = _f32(tgt, 3)
    out = np.zeros(len(q), np.float64)
    lib().orc_nn(_p(q, C.c_double), len(q), _p(tgt, C.c_float), len(tgt), int(bool(l1)),
                 _p(out, C.c_double))
    return out


class DistanceField:
    def __init__(self, lo, h, inv, field, r, res):
        self.lo, self.h, self.inv, self.field, self.r, self.res = lo, h, inv, field, r, res


def df_build(tgt, r, res, threads=0) -> DistanceField:
    tgt = _f32(tgt, 3)
    lo, h, inv = (np.zeros(3, np.float32) for _ in range(3))
    field = np.zeros((res, res, res), np.float64)
    if lib().orc_df_build(_p(tgt, C.c_float), len(tgt), C.c_float(r), res, threads,
                          _p(lo, C.c_float), _p(h, C.c_float), _p(inv, C.c_float),
                          _p(field, C.c_double)):
        raise ValueError("invalid distance-field request")
    return DistanceField(lo, h, inv, field, np.float32(r), res)


def df_query(df: DistanceField, q, lookup="nearest", mu=1e-4):
    """Field values at double queries q (n x 3) by the lookup's definition: returns
    (D, Dmin, Dmax), the last two over the voxels a query within mu voxel units of a
    face may fall in (equal to D for the trilinear lookup)."""
    q = np.ascontiguousarray(np.asarray(q, np.float64).reshape(-1, 3))
    D, Dmin, Dmax = (np.zeros(len(q)) for _ in range(3))
    rc = lib().orc_df_query(_p(q, C.c_double), len(q), _p(df.field, C.c_double), df.res,
                            C.c_float(df.r), _p(df.lo, C.c_float), _p(df.h, C.c_float),
                            DF_LOOKUPS[lookup], C.c_double(mu), _p(D, C.c_double),
                            _p(Dmin, C.c_double), _p(Dmax, C.c_double))
    if rc:
        raise ValueError("oracle rejected the input")
    return D, Dmin, Dmax


class Records(np.ndarray):
    """Oracle records (RECORD_DTYPE) that remember the problem they were computed
    for (``ctx``), so that a candidate's admissible bins can be queried later."""

    def __new__(cls, arr, ctx):
        obj = np.asarray(arr).view(cls)
        obj.ctx = ctx
        return obj

    def __array_finalize__(self, obj):
        self.ctx = getattr(obj, "ctx", None)


def _df_args(df, eps, tau):
    if df is None:
        return None, 0, None, None, None
    if not np.isclose(df.r, max(np.float32(eps), np.float32(tau))):
        raise ValueError("distance field truncation must be max(eps, tau)")
    return (_p(df.field, C.c_double), df.res, _p(df.lo, C.c_float), _p(df.h, C.c_float),
            _p(df.inv, C.c_float))


def records(src, tgt, rotations, eps, *, delta=None, tau=None, t_min=None, t_max=None,
            metric="trunc_l2", p=0.5, which=None, df: DistanceField | None = None,
            df_lookup="nearest", vote="f64", mu=None, mu_df=None, threads=0) -> Records:
    """One Alg. 2 candidate record per rotation (or per listed rotation index).

    vote="f64" (default): the definition in double with fragility intervals;
    vote="lib" / "lib32": the SECONDARY library formulas (fixed-point bins with z at
    2^-15 / 2^-16 bins, single-precision voxels), for labelled bit-exactness checks."""
    src, tgt = _f32(src, 3), _f32(tgt, 3)
    rots = _f32(rotations, 9)
    delta = eps if delta is None else delta
    tau = eps if tau is None else tau
    t_min, t_max = _box_args(t_min, t_max)
    if which is not None:
        which = np.ascontiguousarray(np.asarray(which, np.int32))
        count = len(which)
    else:
        count = len(rots)
    if mu is None:
        mu = vote_margin(src, tgt, delta, t_min, t_max)
    if mu_df is None:
        mu_df = df_margin(src, df, t_min, t_max) if df is not None else 0.0
    out = np.zeros(count, RECORD_DTYPE)
    fld_p, res, lo_p, h_p, inv_p = _df_args(df, eps, tau)
    rc = lib().orc_records(_p(src, C.c_float), len(src), _p(tgt, C.c_float), len(tgt),
                           _p(rots, C.c_float), len(rots),
                           None if which is None else _p(which, C.c_int32), count,
                           C.c_float(eps), C.c_float(delta), C.c_float(tau),
                           _p(t_min, C.c_float), _p(t_max, C.c_float), METRICS[metric],
                           C.c_float(p), C.c_double(mu), _LIB_ZBITS[vote], fld_p, res, lo_p,
                           h_p, inv_p, DF_LOOKUPS[df_lookup], C.c_double(mu_df), threads,
                           out.ctypes.data)
    if rc:
        raise ValueError("oracle rejected the input")
    ctx = dict(src=src, tgt=tgt, rots=rots, eps=eps, delta=delta, tau=tau, t_min=t_min,
               t_max=t_max, metric=metric, p=p, df=df, df_lookup=df_lookup, vote=vote, mu=mu,
               mu_df=mu_df, threads=threads)
    return Records(out, ctx)


def score_bins(ctx, rot, bins, threads=0):
    """Score the candidates {R_rot[u], delta * bins[u]} of a problem (the ``ctx`` of
    a Records array) with its metric and scorer; no vote.  Returns RECORD_DTYPE."""
    rot = np.ascontiguousarray(np.atleast_1d(np.asarray(rot, np.int32)))
    bins = np.ascontiguousarray(np.asarray(bins, np.int32).reshape(-1, 3))
    assert len(rot) == len(bins)
    out = np.zeros(len(rot), RECORD_DTYPE)
    if ctx["metric"] == "votes":
        raise ValueError("the votes ranking does not score")
    if len(rot) == 0:
        return out
    fld_p, res, lo_p, h_p, inv_p = _df_args(ctx["df"], ctx["eps"], ctx["tau"])
    rc = lib().orc_score_bins(_p(ctx["src"], C.c_float), len(ctx["src"]),
                              _p(ctx["tgt"], C.c_float), len(ctx["tgt"]),
                              _p(ctx["rots"], C.c_float), len(ctx["rots"]), _p(rot, C.c_int32),
                              _p(bins, C.c_int32), len(rot), C.c_float(ctx["eps"]),
                              C.c_float(ctx["delta"]), C.c_float(ctx["tau"]),
                              METRICS[ctx["metric"]], C.c_float(ctx["p"]),
                              _LIB_ZBITS[ctx["vote"]], fld_p, res, lo_p, h_p, inv_p,
                              DF_LOOKUPS[ctx["df_lookup"]], C.c_double(ctx["mu_df"]),
                              threads or ctx["threads"], out.ctypes.data)
    if rc:
        raise ValueError("oracle rejected the input")
    return out


def rescore(recs: Records, **changes) -> Records:
    """The same candidates (the vote does not depend on the scorer) scored again with
    changed scoring parameters (df, df_lookup, metric, tau, p, mu_df): copies the vote
    fields and scores every valid rotation's mode bin anew."""
    ctx = dict(recs.ctx)
    ctx.update(changes)
    if "df" in changes and "mu_df" not in changes:
        ctx["mu_df"] = (df_margin(ctx["src"], ctx["df"], ctx["t_min"], ctx["t_max"])
                        if ctx["df"] is not None else 0.0)
    out = np.asarray(recs).copy()
    v = np.nonzero(out["valid"] != 0)[0]
    if ctx["metric"] == "votes":
        out["inliers"][v] = out["votes"][v]
        out["error"][v] = out["err_lo"][v] = out["err_hi"][v] = 0.0
        out["boundary"][v] = out["inl_frag"][v] = 0
    elif v.size:
        sc = score_bins(ctx, out["rot"][v], out["bin"][v])
        for f in ("inliers", "boundary", "error", "err_lo", "err_hi", "inl_frag"):
            out[f][v] = sc[f]
    return Records(out, ctx)


def bin_bounds(ctx, rot, bin_):
    """For rotation `rot` of a problem: (cnt, lo, hi, lo_max) of bin `bin_` (lattice
    units), i.e. the definition's count, the range [cnt - out, cnt + in] of counts
    any evaluation accurate to mu gives it, and max over bins of cnt - out.  A bin
    is an admissible mode iff hi >= lo_max (and hi > 0)."""
    cnt, out, inn, info = vote64(ctx["src"], ctx["tgt"], ctx["rots"][int(rot)], ctx["delta"],
                                 ctx["t_min"], ctx["t_max"], mu=ctx["mu"])
    c = np.asarray(bin_, np.int64) - info["k_lo"]
    if np.any(c < 0) or np.any(c >= info["size"]):
        return 0, 0, 0, info["lo_max"]
    c = tuple(int(v) for v in c)
    return int(cnt[c]), int(cnt[c] - out[c]), int(cnt[c] + inn[c]), info["lo_max"]


def exhaustive(src, tgt, rotations, eps, *, delta=None, tau=None, t_min=None, t_max=None,
               metric="trunc_l2", p=0.5, threads=0):
    """Alg. 1: per rotation the best lattice translation of the box (records with
    votes = 1); select() over them gives the exhaustive optimum."""
    src, tgt = _f32(src, 3), _f32(tgt, 3)
    rots = _f32(rotations, 9)
    delta = eps if delta is None else delta
    tau = eps if tau is None else tau
    t_min, t_max = _box_args(t_min, t_max)
    out = np.zeros(len(rots), RECORD_DTYPE)
    rc = lib().orc_exhaustive(_p(src, C.c_float), len(src), _p(tgt, C.c_float), len(tgt),
                              _p(rots, C.c_float), len(rots), C.c_float(eps), C.c_float(delta),
                              C.c_float(tau), _p(t_min, C.c_float), _p(t_max, C.c_float),
                              METRICS[metric], C.c_float(p), threads, out.ctypes.data)
    if rc:
        raise ValueError("oracle rejected the input")
    return out


def select(recs) -> int:
    recs = np.ascontiguousarray(recs, RECORD_DTYPE)
    return int(lib().orc_select(recs.ctypes.data, len(recs)))


def topk(recs, k) -> np.ndarray:
    """The k best candidates in the selection order of the return step of Alg. 2
    (smaller error, then more inliers, then lower index) over the rotations with at
    least one in-box vote: the definition written out as a sort.  Returns rotation
    indices, -1 past the number of valid rotations."""
    recs = np.ascontiguousarray(recs, RECORD_DTYPE)
    valid = [q for q in range(len(recs)) if recs["valid"][q]]
    order = sorted(valid, key=lambda q: (float(recs["error"][q]), -int(recs["inliers"][q]), q))
    out = np.full(k, -1, np.int64)
    out[:min(k, len(order))] = order[:k]
    return out


def prune_mask(recs, q) -> np.ndarray:
    """Rotations scored under the pruning of Alg. 2 (Sec. IV-B): valid, with mode
    count M_k >= q M*, M* the largest count; the comparison in double precision of
    the counts and the single-precision q (the reading of the paper's "M >= q M*")."""
    recs = np.ascontiguousarray(recs, RECORD_DTYPE)
    votes = recs["votes"].astype(np.float64)
    mstar = float(votes.max()) if len(votes) else 0.0
    return recs["valid"].astype(bool) & (votes >= np.float64(np.float32(q)) * mstar)


def register(src, tgt, rotations, eps, q=0.0, **kw):
    """Full Alg. 2: returns a dict {R, t, rot_index, inliers, error, votes, records}."""
    recs = records(src, tgt, rotations, eps, **kw)
    if q > 0.0:
        pruned = np.asarray(recs).copy()
        pruned["valid"] = prune_mask(recs, q)
        best = select(pruned)
    else:
        best = select(recs)
    delta = kw.get("delta") or eps
    rots = _f32(rotations, 9)
    if best < 0:
        return {"rot_index": -1, "records": recs}
    r = recs[best]
    return {"R": rots[best].reshape(3, 3).astype(np.float64),
            "t": r["bin"].astype(np.float64) * float(np.float32(delta)),
            "rot_index": best, "inliers": int(r["inliers"]), "error": float(r["error"]),
            "votes": int(r["votes"]), "boundary": int(r["boundary"]),
            "pinned": bool(r["pinned"]), "records": recs}


def nthreads_default() -> int:
    return os.cpu_count() or 1
