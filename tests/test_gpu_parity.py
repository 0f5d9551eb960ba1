"""Parity of the HIP path (called through the C ABI) with the CPU oracle."""
import numpy as np
import pytest

import oracle
from paper_2502_00115_amd import synth
from parity import check_selection, compare_library_formula, compare_records

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2502_00115_amd import dses  # noqa: E402


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def run_both(p, metric="trunc_l2", scorer="auto", device=True, **kw):
    if device:
        got = dses.register(_dev(p.src), _dev(p.tgt), _dev(p.rotations), p.eps, metric,
                            scorer=scorer, records=True, **kw)
    else:
        got = dses.register(p.src, p.tgt, p.rotations, p.eps, metric, scorer=scorer,
                            records=True, **kw)
    ref = oracle.records(p.src, p.tgt, p.rotations, p.eps, metric=metric,
                         delta=kw.get("delta_t"), tau=kw.get("tau"), t_min=kw.get("t_min"),
                         t_max=kw.get("t_max"))
    return got, ref


@pytest.mark.parametrize("seed", range(16))
def test_c1_records_and_selection(seed):
    p = synth.make_c1(seed)
    got, ref = run_both(p)
    rep = compare_records(got.records, ref, len(p.src), label=p.name)
    check_selection(got, rep, p.eps, label=p.name)
    # secondary, labelled: the kernel's arithmetic is the documented float formula
    compare_library_formula(got.records, p.src, p.tgt, p.rotations, p.eps, label=p.name)
    print(p.name, {k: v for k, v in rep.items() if np.isscalar(v)})


@pytest.mark.parametrize("seed", range(8))
def test_exact_recovery(seed):
    p = synth.make_c1_exact(seed)
    got = dses.register(_dev(p.src), _dev(p.tgt), _dev(p.rotations), p.eps)
    assert got.rot_index == p.true_index
    np.testing.assert_allclose(got.t, p.t_true, atol=1e-6)
    assert got.inliers == len(p.src)
    assert got.error <= len(p.src) * 1e-6


@pytest.mark.parametrize("metric", ["trunc_l2", "tls", "inliers", "trunc_l1"])
@pytest.mark.parametrize("scorer", ["brute", "grid"])
def test_metrics_and_scorers(metric, scorer):
    p = synth.make_c1(21)
    got, ref = run_both(p, metric=metric, scorer=scorer, tau=0.04)
    rep = compare_records(got.records, ref, len(p.src), metric=metric,
                          label=f"{metric}/{scorer}")
    check_selection(got, rep, p.eps, label=f"{metric}/{scorer}")


def test_brute_and_grid_scorers_are_bitwise_equal():
    p = synth.make_c1(3)
    a = dses.register(p.src, p.tgt, p.rotations, p.eps, scorer="brute", records=True)
    b = dses.register(p.src, p.tgt, p.rotations, p.eps, scorer="grid", records=True)
    assert a.records.tobytes() == b.records.tobytes()


@pytest.mark.parametrize("case", ["far_outliers", "saturating_cell_index"])
def test_grid_scorer_queries_far_outside_the_grid(case):
    """Queries whose cell index lies far outside the cell grid (or saturates the
    float-to-int conversion) find no neighbours there, exactly as brute force."""
    rng = np.random.default_rng(77)
    if case == "far_outliers":
        p = synth.make_c1(5)
        src = p.src.copy()
        src[::7] = rng.uniform(-300.0, 300.0, size=src[::7].shape).astype(np.float32)
        eps, kw = p.eps, {}
        tgt, rots = p.tgt, p.rotations[:64]
    else:
        # a 1e-4-wide reference cluster, cell pitch ~1e-6: sources a few thousand
        # units away put (q - lo) / pitch near 1e10, beyond the int32 range
        tgt = (rng.uniform(0.0, 1.0e-4, size=(64, 3)) + 0.1).astype(np.float32)
        src = np.concatenate([tgt[:24] - 0.1, rng.uniform(-5.0e3, 5.0e3, size=(24, 3))])
        src = src.astype(np.float32)
        eps, kw = 1.0e-6, {"delta_t": 0.25}
        rots = synth.hopf_grid(0)[:24].reshape(-1, 9).astype(np.float32)
    pb = synth.Problem(src, tgt, rots, eps, np.eye(3), np.zeros(3))
    g, ref = run_both(pb, scorer="grid", **kw)
    b = dses.register(src, tgt, rots, eps, scorer="brute", records=True, **kw)
    assert g.records.tobytes() == b.records.tobytes()
    compare_records(g.records, ref, len(src), label=case)


def test_host_and_device_pointers_agree():
    p = synth.make_c1(4)
    a = dses.register(p.src, p.tgt, p.rotations, p.eps, records=True)
    b = dses.register(_dev(p.src), _dev(p.tgt), _dev(p.rotations), p.eps, records=True)
    assert a.records.tobytes() == b.records.tobytes()
    assert a.rot_index == b.rot_index and a.error == b.error


def test_deterministic_repeat():
    p = synth.make_c1(5)
    a = dses.register(p.src, p.tgt, p.rotations, p.eps, records=True)
    b = dses.register(p.src, p.tgt, p.rotations, p.eps, records=True)
    assert a.records.tobytes() == b.records.tobytes()


def test_runs_on_a_side_stream():
    p = synth.make_c1(6)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        a = dses.register(_dev(p.src), _dev(p.tgt), _dev(p.rotations), p.eps, records=True)
    b = dses.register(p.src, p.tgt, p.rotations, p.eps, records=True)
    assert a.records.tobytes() == b.records.tobytes()


# ---------------------------------------------------------------------------
# vote layouts: 16, 32 or 64 reference points per lane group
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,m,k", [(1, 1, 2), (37, 15, 5), (717, 1024, 24), (300, 1000, 9),
                                   (16384, 130, 2), (4100, 1777, 3)])
def test_lane_group_layouts(n, m, k):
    """Every lane-group size gives the oracle's records, bit-identical to the
    others (ragged group counts, windows shorter than a block, one point)."""
    rng = np.random.default_rng(n * 13 + m)
    tgt = rng.uniform(-0.8, 0.8, (m, 3)).astype(np.float32)
    src = (tgt[rng.integers(0, m, n)] + rng.normal(0, 0.01, (n, 3))).astype(np.float32)
    rots = synth.random_rotations(rng, k).reshape(-1, 9).astype(np.float32)
    rots[0] = np.eye(3, dtype=np.float32).reshape(9)
    p = synth.Problem(src, tgt, rots, 0.03, np.eye(3), np.zeros(3))
    ref = oracle.records(p.src, p.tgt, p.rotations, p.eps)
    first = None
    for lg in (16, 32, 64, 0):
        got = dses.register(_dev(p.src), _dev(p.tgt), _dev(p.rotations), p.eps,
                            records=True, lane_group=lg)
        compare_records(got.records, ref, n, label=f"lane_group={lg}")
        if first is None:
            first = got.records.tobytes()
        assert got.records.tobytes() == first, lg


# ---------------------------------------------------------------------------
# ragged sizes, boxes and counter widths
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("n,m,k", [(1, 1, 1), (1, 300, 7), (65, 1, 5), (65, 1023, 33),
                                   (130, 77, 9), (1025, 40, 3), (2100, 260, 4),
                                   # past the points each thread keeps in registers while
                                   # sorting, the largest sorted source, the first unsorted
                                   (4200, 700, 3), (16384, 130, 2), (16385, 100, 2)])
def test_ragged_sizes(n, m, k):
    rng = np.random.default_rng(n * 7 + m)
    tgt = rng.uniform(-0.8, 0.8, (m, 3)).astype(np.float32)
    src = (tgt[rng.integers(0, m, n)] + rng.normal(0, 0.01, (n, 3))).astype(np.float32)
    rots = synth.random_rotations(rng, k).reshape(-1, 9).astype(np.float32)
    rots[0] = np.eye(3, dtype=np.float32).reshape(9)
    p = synth.Problem(src, tgt, rots, 0.05, np.eye(3), np.zeros(3))
    got, ref = run_both(p)
    rep = compare_records(got.records, ref, n, label=f"{n}x{m}x{k}")
    check_selection(got, rep, p.eps, label=f"{n}x{m}x{k}")


@pytest.mark.parametrize("delta,box", [(0.02, 1.0), (0.011, 0.6), (0.05, 2.5), (0.1, 0.05)])
def test_multi_slab_and_small_boxes(delta, box):
    """Boxes from a single bin up to 227^3 bins (many LDS slabs)."""
    p = synth.make_c1(7)
    which = slice(0, 96)
    p.rotations = p.rotations[which].copy()
    got, ref = run_both(p, delta_t=delta, t_min=-box, t_max=box)
    compare_records(got.records, ref, len(p.src), label=f"delta {delta} box {box}")


def test_asymmetric_box():
    p = synth.make_c1(8)
    got, ref = run_both(p, t_min=[-0.3, -1.0, 0.0], t_max=[0.9, 0.2, 0.75])
    compare_records(got.records, ref, len(p.src))


@pytest.mark.parametrize("spread", [0.5, 3.0])
def test_coarse_source_buckets(spread):
    """A box 4,001 bins long in x (delta 1 mm) and references spread over +-spread:
    the sources' reachable x range (about 5,000 or 10,000 bins) no longer fits 4
    buckets per bin, so the sort uses 1 or 1/2 bucket per bin."""
    rng = np.random.default_rng(31)
    tgt = rng.uniform(-0.5, 0.5, (300, 3)).astype(np.float32)
    tgt[:, 0] *= 2 * spread
    src = (tgt[rng.integers(0, 300, 200)] + rng.normal(0, 0.0005, (200, 3))).astype(np.float32)
    rots = np.vstack([np.eye(3).reshape(1, 9), synth.random_rotations(rng, 3).reshape(-1, 9)])
    p = synth.Problem(src, tgt, rots.astype(np.float32), 0.02, np.eye(3), np.zeros(3))
    box = dict(delta_t=0.001, t_min=[-2.0, -0.02, -0.02], t_max=[2.0, 0.02, 0.02])
    got, ref = run_both(p, **box)
    assert ref["votes"][0] > 50
    compare_records(got.records, ref, len(src), label=f"spread {spread}")


def test_32bit_counters_when_16bit_could_overflow():
    """300 source points on one spot and 400 reference points on another: one bin gets
    300*400 = 120,000 > 2^16 votes, so the library must use 32-bit counters."""
    rng = np.random.default_rng(9)
    src = np.tile(np.float32([[0.1, 0.2, 0.3]]), (300, 1))
    tgt = np.vstack([np.tile(np.float32([[0.4, -0.1, 0.2]]), (400, 1)),
                     rng.uniform(-1, 1, (50, 3)).astype(np.float32)])
    rots = np.vstack([np.eye(3).reshape(1, 9), synth.random_rotations(rng, 3).reshape(-1, 9)])
    p = synth.Problem(src, tgt, rots.astype(np.float32), 0.05, np.eye(3), np.zeros(3))
    got, ref = run_both(p)
    assert ref["votes"][0] == 120000
    compare_records(got.records, ref, len(src))


def test_no_vote_in_box_is_nocandidate():
    src = np.zeros((4, 3), np.float32)
    tgt = np.full((5, 3), 0.9, np.float32)
    with pytest.raises(dses.DsesError) as e:
        dses.register(src, tgt, np.eye(3, dtype=np.float32).reshape(1, 9), 0.05,
                      t_min=-0.2, t_max=0.2)
    assert e.value.status == dses.DSES_E_NOCANDIDATE


@pytest.mark.parametrize("device", [False, True])
def test_invalid_inputs_are_rejected(device):
    p = synth.make_c1(1)
    bad = p.src.copy()
    bad[3, 1] = np.nan
    rots = p.rotations.copy()
    rots[2, 0] = 2.0
    f = _dev if device else (lambda a: a)
    for s, t, r in [(bad, p.tgt, p.rotations), (p.src, p.tgt, rots)]:
        with pytest.raises(dses.DsesError) as e:
            dses.register(f(s), f(t), f(r), p.eps)
        assert e.value.status == dses.DSES_E_INVAL
    with pytest.raises(dses.DsesError):
        dses.register(p.src, p.tgt, p.rotations, -1.0)


# ---------------------------------------------------------------------------
# full-size object-scale registration (36,864-rotation grid)
# ---------------------------------------------------------------------------
def _angle_deg(Ra, Rb):
    c = (np.trace(np.asarray(Ra, np.float64).T @ np.asarray(Rb, np.float64)) - 1) / 2
    return float(np.degrees(np.arccos(np.clip(c, -1, 1))))


def _nearest_to_truth(p):
    R = p.rotations.reshape(-1, 3, 3).astype(np.float64)
    c = (np.einsum("kij,ij->k", R, p.R_true) - 1) / 2
    return int(np.argmax(c))


def test_c2_sampled_records_and_selection():
    p = synth.make_c2(0)
    got = dses.register(_dev(p.src), _dev(p.tgt), _dev(p.rotations), p.eps, records=True)
    rng = np.random.default_rng(0)
    recs = got.records
    top = np.argsort(np.where(recs["votes"] > 0, recs["error"], np.inf))[:16]
    which = np.unique(np.concatenate([rng.choice(len(p.rotations), 384, replace=False), top]))
    ref = oracle.records(p.src, p.tgt, p.rotations, p.eps, which=which)
    rep = compare_records(recs[which], ref, len(p.src), label="c2 sample")
    # within the compared set (which holds the GPU's 16 best) the GPU's choice is admissible
    check_selection(got, rep, p.eps, label="c2 sample")
    print(f"c2: rot {got.rot_index} angle to truth {_angle_deg(got.R, p.R_true):.2f} deg, "
          f"t {got.t} vs {p.t_true}; ambiguous {rep['ambiguous']} moved {rep['moved']}")


@pytest.mark.slow
@pytest.mark.parametrize("seed", range(4))
def test_c2_full_grid_every_rotation(seed):
    """All 36,864 candidates of an object-scale registration against the oracle, one
    by one, and the selection against the oracle's admissible winners over the whole
    grid."""
    p = synth.make_c2(seed)
    got = dses.register(_dev(p.src), _dev(p.tgt), _dev(p.rotations), p.eps, records=True)
    ref = oracle.records(p.src, p.tgt, p.rotations, p.eps)
    rep = compare_records(got.records, ref, len(p.src), label=f"c2 seed {seed}")
    nW = check_selection(got, rep, p.eps, label=f"c2 seed {seed}")
    print(f"c2 seed {seed}: rot {got.rot_index} (|W| = {nW}) angle to truth "
          f"{_angle_deg(got.R, p.R_true):.2f} deg; ambiguous {rep['ambiguous']} "
          f"moved {rep['moved']} fragile pairs {rep['fragile_pairs']}")


# ---------------------------------------------------------------------------
# full-size scene-scale registration (294,912-rotation grid), the bench's launch,
# with the exact cell-grid scorer and with the 128^3 distance field
# ---------------------------------------------------------------------------
@pytest.mark.slow
def test_c5_full_size_sampled_records_and_selection():
    p = synth.make_c5(0)
    n = len(p.src)
    got = dses.register(_dev(p.src), _dev(p.tgt), _dev(p.rotations), p.eps, records=True)
    recs = got.records
    assert int((recs["votes"] > 0).sum()) == got.n_valid
    T = dses.Target(p.tgt, df_trunc=p.eps, df_res=128)
    S = dses.RotationSet(p.rotations)
    gdf = dses.register_resident(T, S, p.src, p.eps, scorer="df", records=True)
    # the vote does not depend on the scorer
    assert gdf.records["votes"].tobytes() == recs["votes"].tobytes()
    assert gdf.records["bin"].tobytes() == recs["bin"].tobytes()
    rng = np.random.default_rng(5)
    top = np.argsort(np.where(recs["votes"] > 0, recs["error"], np.inf))[:16]
    top_df = np.argsort(np.where(recs["votes"] > 0, gdf.records["error"], np.inf))[:16]
    truth = _nearest_to_truth(p)
    which = np.unique(np.concatenate([rng.choice(len(p.rotations), 2048, replace=False), top,
                                      top_df, [truth]]))
    ref = oracle.records(p.src, p.tgt, p.rotations, p.eps, which=which)
    rep = compare_records(recs[which], ref, n, label="c5 grid")
    check_selection(got, rep, p.eps, label="c5 grid")
    df = oracle.df_build(p.tgt, p.eps, 128)
    ref_df = oracle.rescore(ref, df=df)
    rep_df = compare_records(gdf.records[which], ref_df, n, label="c5 df")
    check_selection(gdf, rep_df, p.eps, label="c5 df")
    print(f"c5: grid rot {got.rot_index} ({_angle_deg(got.R, p.R_true):.2f} deg), df rot "
          f"{gdf.rot_index} ({_angle_deg(gdf.R, p.R_true):.2f} deg), nearest grid rotation "
          f"{truth}; ambiguous {rep['ambiguous']} of {len(which)}, moved {rep['moved']}")
