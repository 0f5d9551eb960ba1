"""CPU oracle for DSES -- test infrastructure only.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports it.

The arithmetic lives in ``dses_oracle.c`` (plain C, double precision except for
the two float-decided integers described there).  This module only marshals
numpy arrays through ctypes.

Paper steps covered (Cheng et al., arXiv 2502.00115):
  * ``vote``      -- Lemma 2 / Eq. (5) and the first loop of Alg. 2: mode of the
                     rounded rotated pair translations, with its frequency M.
  * ``nn``        -- Eq. (1)/(2) nearest-neighbour distance, brute force.
  * ``records``   -- Alg. 2 with q = 0: every candidate {R, t*} scored.
  * ``select``    -- the argmin return of Alg. 2.
  * ``df_build``  -- voxel distance field of the reference cloud (scoring
                     variant; not in the paper, defined in the library header).
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from .build import LIB, build_oracle

METRICS = {"trunc_l2": 0, "inliers": 1, "tls": 2, "trunc_l1": 3, "trunc_lp": 4, "votes": 5}

RECORD_DTYPE = np.dtype([("bin", "<i4", (3,)), ("votes", "<u4"), ("inliers", "<i4"),
                         ("boundary", "<i4"), ("error", "<f8"), ("valid", "<i4"),
                         ("pad", "<i4")])
assert RECORD_DTYPE.itemsize == 40

_lib = None


def lib():
    global _lib
    if _lib is None:
        path = build_oracle(force=False)
        L = C.CDLL(path)
        fp, dp, ip, up = (C.POINTER(C.c_float), C.POINTER(C.c_double), C.POINTER(C.c_int32),
                          C.POINTER(C.c_uint32))
        L.orc_box.argtypes = [C.c_float, fp, fp, ip, ip]
        L.orc_box.restype = C.c_int
        L.orc_vote.argtypes = [fp, C.c_int32, fp, C.c_int32, fp, C.c_float, ip, ip, up, ip]
        L.orc_vote.restype = C.c_uint32
        L.orc_nn.argtypes = [dp, C.c_int32, fp, C.c_int32, C.c_int32, dp]
        L.orc_nn.restype = None
        L.orc_df_build.argtypes = [fp, C.c_int32, C.c_float, C.c_int32, C.c_int32, fp, fp, fp, dp]
        L.orc_df_build.restype = C.c_int
        L.orc_records.argtypes = [fp, C.c_int32, fp, C.c_int32, fp, C.c_int32, ip, C.c_int32,
                                  C.c_float, C.c_float, C.c_float, fp, fp, C.c_int32, C.c_float,
                                  dp, C.c_int32, fp, fp, C.c_int32, C.c_void_p]
        L.orc_records.restype = C.c_int
        L.orc_select.argtypes = [C.c_void_p, C.c_int32]
        L.orc_exhaustive.argtypes = [fp, C.c_int32, fp, C.c_int32, fp, C.c_int32, C.c_float,
                                     C.c_float, C.c_float, fp, fp, C.c_int32, C.c_float,
                                     C.c_int32, C.c_void_p]
        L.orc_exhaustive.restype = C.c_int
        L.orc_select.restype = C.c_int32
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


def vote(src, tgt, R, delta, t_min=None, t_max=None):
    """Vote array (size_x, size_y, size_z) of one rotation, its mode bin and frequency M."""
    src, tgt = _f32(src, 3), _f32(tgt, 3)
    R = _f32(R).reshape(9)
    k_lo, size = box(delta, t_min, t_max)
    hist = np.zeros(tuple(int(s) for s in size), np.uint32)
    mode = np.zeros(3, np.int32)
    M = lib().orc_vote(_p(src, C.c_float), len(src), _p(tgt, C.c_float), len(tgt),
                       _p(R, C.c_float), C.c_float(delta), _p(k_lo, C.c_int32),
                       _p(size, C.c_int32), _p(hist, C.c_uint32), _p(mode, C.c_int32))
    return hist, mode, int(M)


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


def records(src, tgt, rotations, eps, *, delta=None, tau=None, t_min=None, t_max=None,
            metric="trunc_l2", p=0.5, which=None, df: DistanceField | None = None, threads=0):
    """One Alg. 2 candidate record per rotation (or per listed rotation index)."""
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
    out = np.zeros(count, RECORD_DTYPE)
    if df is not None:
        if not np.isclose(df.r, max(np.float32(eps), np.float32(tau))):
            raise ValueError("distance field truncation must be max(eps, tau)")
        fld, res, lo, inv = df.field, df.res, df.lo, df.inv
        fld_p, lo_p, inv_p = _p(fld, C.c_double), _p(lo, C.c_float), _p(inv, C.c_float)
    else:
        fld_p, res, lo_p, inv_p = None, 0, None, None
    rc = lib().orc_records(_p(src, C.c_float), len(src), _p(tgt, C.c_float), len(tgt),
                           _p(rots, C.c_float), len(rots),
                           None if which is None else _p(which, C.c_int32), count,
                           C.c_float(eps), C.c_float(delta), C.c_float(tau),
                           _p(t_min, C.c_float), _p(t_max, C.c_float), METRICS[metric],
                           C.c_float(p), fld_p, res, lo_p, inv_p, threads, out.ctypes.data)
    if rc:
        raise ValueError("oracle rejected the input")
    return out


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
        pruned = recs.copy()
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
            "votes": int(r["votes"]), "boundary": int(r["boundary"]), "records": recs}


def nthreads_default() -> int:
    return os.cpu_count() or 1
