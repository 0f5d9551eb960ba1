"""Batched registration and the serving loop: identical results alone and in the mix,
graph replays, admission by memory, and oracle parity on sampled rotations."""
import time

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


def _small_c3(count=6, k=384, seed=0):
    probs = synth.make_c3(seed, count=count)
    for p in probs:
        p.rotations = p.rotations[:k].copy()
    return probs


def _as_dict(p, **kw):
    d = {"src": p.src, "tgt": p.tgt, "rotations": p.rotations, "eps": p.eps}
    d.update(kw)
    return d


def _same(a, b):
    assert a.rot_index == b.rot_index
    assert a.error == b.error and a.inliers == b.inliers and a.votes == b.votes
    np.testing.assert_array_equal(a.t, b.t)


@pytest.mark.parametrize("use_graph", [False, True])
def test_batch_equals_alone_bitwise(use_graph):
    probs = _small_c3()
    alone = [dses.register(p.src, p.tgt, p.rotations, p.eps, records=True) for p in probs]
    got, st = dses.register_batch([_as_dict(p) for p in probs], use_graph=use_graph,
                                  records=True)
    assert st == [0] * len(probs)
    for a, b in zip(alone, got):
        _same(a, b)
        assert a.records.tobytes() == b.records.tobytes()


def test_graph_replays_match_eager_every_time():
    probs = _small_c3(count=5, k=256, seed=1)
    eager = [dses.register(p.src, p.tgt, p.rotations, p.eps, records=True) for p in probs]
    for rep in range(4):
        got, st = dses.register_batch([_as_dict(p) for p in probs], use_graph=True, records=True)
        assert st == [0] * len(probs)
        for a, b in zip(eager, got):
            assert a.records.tobytes() == b.records.tobytes(), f"replay {rep}"
        # the program's own eager work between replays
        x = dses.register(probs[rep].src, probs[rep].tgt, probs[rep].rotations, probs[rep].eps)
        _same(x, eager[rep])
        torch.cuda.synchronize()


def test_batch_with_different_shapes_between_replays():
    a = _small_c3(count=3, k=200, seed=2)
    b = _small_c3(count=7, k=300, seed=3)
    for probs in (a, b, a):
        eager = [dses.register(p.src, p.tgt, p.rotations, p.eps) for p in probs]
        got, st = dses.register_batch([_as_dict(p) for p in probs], use_graph=True)
        assert st == [0] * len(probs)
        for x, y in zip(eager, got):
            _same(x, y)


def test_batch_resident_and_device_inputs():
    probs = _small_c3(count=4, k=256, seed=4)
    T = [dses.Target(p.tgt) for p in probs]
    S = [dses.RotationSet(p.rotations) for p in probs]
    alone = [dses.register(p.src, p.tgt, p.rotations, p.eps) for p in probs]
    got, st = dses.register_batch([{"src": p.src, "target": t, "rotset": s, "eps": p.eps}
                                   for p, t, s in zip(probs, T, S)])
    assert st == [0] * len(probs)
    for x, y in zip(alone, got):
        _same(x, y)
    dev = lambda a: torch.from_numpy(a).cuda()  # noqa: E731
    got2, st2 = dses.register_batch([{"src": dev(p.src), "tgt": dev(p.tgt),
                                      "rotations": dev(p.rotations), "eps": p.eps}
                                     for p in probs])
    assert st2 == [0] * len(probs)
    for x, y in zip(alone, got2):
        _same(x, y)


def test_batch_reports_bad_problem_and_runs_the_rest():
    probs = _small_c3(count=3, k=128, seed=5)
    bad = probs[1].src.copy()
    bad[0, 0] = np.nan
    items = [_as_dict(probs[0]), _as_dict(probs[1], src=bad), _as_dict(probs[2])]
    got, st = dses.register_batch(items)
    assert st[0] == 0 and st[2] == 0 and st[1] == dses.DSES_E_INVAL
    _same(got[0], dses.register(probs[0].src, probs[0].tgt, probs[0].rotations, probs[0].eps))
    _same(got[2], dses.register(probs[2].src, probs[2].tgt, probs[2].rotations, probs[2].eps))


def test_batch_parity_with_oracle_on_sampled_rotations():
    probs = synth.make_c3(6, count=4)
    got, st = dses.register_batch([_as_dict(p) for p in probs], records=True)
    assert st == [0] * len(probs)
    rng = np.random.default_rng(1)
    for p, g in zip(probs, got):
        which = np.sort(rng.choice(len(p.rotations), 48, replace=False))
        ref = oracle.records(p.src, p.tgt, p.rotations, p.eps, which=which)
        compare_records(g.records[which], ref, len(p.src), label=p.name)


# ---------------------------------------------------------------------------
# serving
# ---------------------------------------------------------------------------
def _serving_setup(n_targets=2, n_req=6, k=512, seed=0):
    rng = np.random.default_rng(seed)
    tg = synth.make_c4_targets(seed, count=n_targets)
    rots = synth.hopf_grid(3)[rng.permutation(36864)[:k]].reshape(-1, 9).astype(np.float32)
    targets = [dses.Target(t) for t, _ in tg]
    rotset = dses.RotationSet(rots)
    reqs = []
    for i in range(n_req):
        tid, src = synth.make_c4_request(100 + i, tg)
        reqs.append((tid, src[: 300 + 97 * i]))
    return targets, rotset, rots, reqs


def test_server_results_equal_alone():
    targets, rotset, rots, reqs = _serving_setup()
    alone = [dses.register_resident(targets[t], rotset, src, 0.03) for t, src in reqs]
    srv = dses.Server()
    ids = [srv.submit(targets[t], rotset, src, 0.03) for t, src in reqs]
    for rid, a in zip(ids, alone):
        _same(srv.wait(rid, timeout_ms=60000), a)
    # a second wave arriving while the first is still on the device
    ids = [srv.submit(targets[t], rotset, src, 0.03) for t, src in reqs[:3]]
    ids += [srv.submit(targets[t], rotset, src, 0.03) for t, src in reqs[3:]]
    for rid, a in zip(ids, alone):
        _same(srv.wait(rid, timeout_ms=60000), a)
    srv.close()


def test_server_requests_spanning_many_slices_equal_alone():
    # slices of 10^7 pairs: each request's rotations are counted to completion
    # across many slices on both slice streams before its workgroup selects it
    targets, rotset, rots, reqs = _serving_setup(n_req=4, k=192, seed=9)
    alone = [dses.register_resident(targets[t], rotset, src, 0.03) for t, src in reqs]
    srv = dses.Server(slice_mpairs=10)
    ids = [srv.submit(targets[t], rotset, src, 0.03) for t, src in reqs]
    for rid, a in zip(ids, alone):
        _same(srv.wait(rid, timeout_ms=120000), a)
    srv.close()


def test_server_memory_admission_serialises_when_budget_fits_one():
    targets, rotset, rots, reqs = _serving_setup(n_req=3, k=256, seed=1)
    # a request needs 12 N + 24 K bytes (rounded); budget fits exactly one at a time
    need = max(((12 * len(s) + 255) // 256) * 256 + ((24 * 256 + 255) // 256) * 256
               for _, s in reqs)
    srv = dses.Server(memory_budget=need + 256)
    ids = [srv.submit(targets[t], rotset, src, 0.03) for t, src in reqs]
    res = [srv.wait(r, timeout_ms=60000) for r in ids]
    for (t, src), got in zip(reqs, res):
        _same(got, dses.register_resident(targets[t], rotset, src, 0.03))
    timing = [(g.queue_s, g.total_s) for g in res]
    # requests were admitted one after another: each later one waited in the queue
    for (q0, tot0), (q1, _) in zip(timing, timing[1:]):
        assert q1 >= q0
    assert timing[-1][0] > 0.0
    srv.close()


def test_server_rejects_requests_larger_than_the_budget():
    targets, rotset, _, reqs = _serving_setup(n_req=1, k=256, seed=2)
    srv = dses.Server(memory_budget=4096)
    with pytest.raises(dses.DsesError) as e:
        srv.submit(targets[0], rotset, reqs[0][1], 0.03)
    assert e.value.status == dses.DSES_E_NOMEM
    with pytest.raises(dses.DsesError) as e:
        srv.wait(12345, timeout_ms=0)
    assert e.value.status == dses.DSES_E_STATE
    srv.close()


def test_server_poll_and_timeout():
    targets, rotset, _, reqs = _serving_setup(n_req=1, k=2048, seed=3)
    srv = dses.Server()
    rid = srv.submit(targets[0], rotset, reqs[0][1], 0.03)
    assert srv.poll(rid) in (0, 1)
    while srv.poll(rid) == 0:
        time.sleep(0.005)
    assert srv.poll(rid) == 1
    q, tot = srv.timing(rid)            # finished, not yet consumed
    assert 0.0 <= q <= tot
    got = srv.wait(rid, timeout_ms=60000)
    assert got.rot_index >= 0 and got.queue_s == q and got.total_s == tot
    # the wait consumed the request: its id is forgotten
    assert srv.poll(rid) == dses.DSES_E_STATE
    for call in (lambda: srv.wait(rid, timeout_ms=0), lambda: srv.timing(rid),
                 lambda: srv.cancel(rid)):
        with pytest.raises(dses.DsesError) as e:
            call()
        assert e.value.status == dses.DSES_E_STATE
    srv.close()


def test_server_cancel_withdraws_a_queued_request():
    targets, rotset, _, reqs = _serving_setup(n_req=3, k=256, seed=9)
    # room for one request at a time: the later ones wait in the queue
    need = max(((12 * len(s) + 255) // 256) * 256 + ((24 * 256 + 255) // 256) * 256
               for _, s in reqs)
    srv = dses.Server(memory_budget=need + 256)
    ids = [srv.submit(targets[t], rotset, src, 0.03) for t, src in reqs]
    srv.cancel(ids[2])
    with pytest.raises(dses.DsesError) as e:
        srv.wait(ids[2], timeout_ms=0)
    assert e.value.status == dses.DSES_E_STATE
    for rid, (t, src) in zip(ids[:2], reqs[:2]):
        _same(srv.wait(rid, timeout_ms=60000),
              dses.register_resident(targets[t], rotset, src, 0.03))
    srv.close()


def test_served_non_default_options_equal_alone():
    """Per-request options (pitch, truncation, box, scorer, records, top-k) give the
    result a lone resident registration gives with the same options."""
    targets, rotset, rots, reqs = _serving_setup(n_targets=2, n_req=4, k=640, seed=10)
    opts = [dict(delta_t=0.025, tau=0.04, t_min=[-0.8, -0.9, -0.7], t_max=[0.9, 0.8, 0.85]),
            dict(scorer="brute", tau=0.05),
            dict(delta_t=0.035, t_min=-0.6, t_max=0.6),
            dict()]
    srv = dses.Server()
    ids = [srv.submit(targets[t], rotset, src, 0.03, "tls" if i == 1 else "trunc_l2",
                      records=True, top_k=8, **o)
           for i, ((t, src), o) in enumerate(zip(reqs, opts))]
    for i, (rid, (t, src), o) in enumerate(zip(ids, reqs, opts)):
        got = srv.wait(rid, timeout_ms=60000)
        alone = dses.register_resident(targets[t], rotset, src, 0.03,
                                       "tls" if i == 1 else "trunc_l2", records=True, top_k=8,
                                       **{k: v for k, v in o.items()})
        _same(got, alone)
        assert got.records.tobytes() == alone.records.tobytes(), i
        assert got.top.tobytes() == alone.top.tobytes(), i
    srv.close()


def test_served_df_mix_matches_oracle():
    """Serving workload: requests of different sizes against two resident targets with
    128^3 distance fields, the later ones submitted while earlier ones run.  Each
    result equals its lone registration bit for bit; records on sampled rotations and
    the selection match the oracle's distance-field scoring."""
    rng = np.random.default_rng(12)
    tg = synth.make_c4_targets(3, count=8)
    pick = [int(np.argmin([len(t) for t, _ in tg])), int(np.argsort([len(t) for t, _ in tg])[1])]
    tgts = [tg[i][0] for i in pick]
    rots = synth.hopf_grid(3)[rng.permutation(36864)[:2048]].reshape(-1, 9).astype(np.float32)
    eps = 0.03
    targets = [dses.Target(t, df_trunc=eps, df_res=128) for t in tgts]
    rotset = dses.RotationSet(rots)
    shapes = [tg[i][1] for i in pick]
    reqs = []
    for i in range(5):
        tid = i % 2
        _, src = synth.make_c4_request(200 + i, [(tgts[tid], shapes[tid])])
        reqs.append((tid, src))
    assert len({len(s) for _, s in reqs}) == len(reqs)      # every request its own size
    srv = dses.Server()
    ids = [srv.submit(targets[t], rotset, src, eps, records=True) for t, src in reqs[:2]]
    time.sleep(0.01)
    ids += [srv.submit(targets[t], rotset, src, eps, records=True) for t, src in reqs[2:]]
    served = [srv.wait(r, timeout_ms=120000) for r in ids]
    srv.close()
    fields = [oracle.df_build(t, eps, 128) for t in tgts]
    for i, ((t, src), g) in enumerate(zip(reqs, served)):
        alone = dses.register_resident(targets[t], rotset, src, eps, scorer="df", records=True)
        _same(g, alone)
        assert g.records.tobytes() == alone.records.tobytes(), i
        recs = g.records
        top = np.argsort(np.where(recs["votes"] > 0, recs["error"], np.inf))[:8]
        which = np.unique(np.concatenate([rng.choice(len(rots), 40, replace=False), top]))
        ref = oracle.records(src, tgts[t], rots, eps, which=which, df=fields[t])
        rep = compare_records(recs[which], ref, len(src), label=f"served df {i}")
        check_selection(g, rep, eps, label=f"served df {i}")


def test_batch_with_distance_field_targets_matches_oracle():
    """Batched registration against resident targets scored by their distance fields:
    equal to lone calls, and sampled records and selections match the oracle's
    distance-field scoring (nearest and trilinear lookups)."""
    probs = _small_c3(count=4, k=384, seed=11)
    eps = 0.03
    fields = [oracle.df_build(p.tgt, eps, 64) for p in probs]
    T = [dses.Target(p.tgt, df_trunc=eps, df_res=64) for p in probs]
    S = [dses.RotationSet(p.rotations) for p in probs]
    rng = np.random.default_rng(2)
    for lookup in ("nearest", "trilinear"):
        got, st = dses.register_batch([{"src": p.src, "target": t, "rotset": s, "eps": eps}
                                       for p, t, s in zip(probs, T, S)], scorer="df",
                                      records=True, df_lookup=lookup)
        assert st == [0] * len(probs)
        for p, t, s, g, df in zip(probs, T, S, got, fields):
            alone = dses.register_resident(t, s, p.src, eps, scorer="df", records=True,
                                           df_lookup=lookup)
            _same(g, alone)
            assert g.records.tobytes() == alone.records.tobytes()
            top = np.argsort(np.where(g.records["votes"] > 0, g.records["error"], np.inf))[:8]
            which = np.unique(np.concatenate([rng.choice(len(p.rotations), 48, replace=False),
                                              top]))
            ref = oracle.records(p.src, p.tgt, p.rotations, eps, which=which, df=df,
                                 df_lookup=lookup)
            rep = compare_records(g.records[which], ref, len(p.src), label=f"{p.name} {lookup}")
            check_selection(g, rep, eps, label=f"{p.name} {lookup}")


@pytest.mark.slow
def test_c3_selection_over_full_grids_matches_oracle():
    """Four instances of the 64-registration batch, every rotation of their grids
    compared with the oracle and each selection inside the oracle's admissible set."""
    probs = synth.make_c3(0)
    got, st = dses.register_batch([_as_dict(p) for p in probs], records=True)
    assert st == [0] * len(probs)
    cost = [len(p.src) * len(p.tgt) * len(p.rotations) for p in probs]
    for i in np.argsort(cost)[:4]:
        p, g = probs[i], got[i]
        ref = oracle.records(p.src, p.tgt, p.rotations, p.eps)
        rep = compare_records(g.records, ref, len(p.src), label=p.name)
        nW = check_selection(g, rep, p.eps, label=p.name)
        print(f"{p.name}: n {len(p.src)} m {len(p.tgt)} k {len(p.rotations)} rot {g.rot_index} "
              f"|W| {nW} ambiguous {rep['ambiguous']} moved {rep['moved']}")


def test_server_many_concurrent_clients():
    import threading
    targets, rotset, _, reqs = _serving_setup(n_targets=2, n_req=8, k=384, seed=4)
    alone = [dses.register_resident(targets[t], rotset, src, 0.03) for t, src in reqs]
    srv = dses.Server()
    out = [None] * len(reqs)

    def client(i):
        t, src = reqs[i]
        time.sleep(0.002 * i)
        out[i] = srv.wait(srv.submit(targets[t], rotset, src, 0.03), timeout_ms=60000)

    th = [threading.Thread(target=client, args=(i,)) for i in range(len(reqs))]
    for t in th:
        t.start()
    for t in th:
        t.join()
    for a, b in zip(alone, out):
        _same(a, b)
    srv.close()


def test_autotune_keeps_results_and_caches_the_layout():
    probs = _small_c3(count=5, k=512, seed=7)
    items = [_as_dict(p) for p in probs]
    base, st = dses.register_batch(items, records=True)
    assert st == [0] * len(probs)
    tuned, st = dses.register_batch(items, autotune=True, records=True)
    assert st == [0] * len(probs)
    cfg = dses.batch_last_config()
    assert cfg["source"] == "tuned" and cfg["candidates"] >= 8
    assert cfg["items_per_cu"] in (6, 12, 24, 48, 96) and cfg["vote_parts"] in (0, 1, 2, 4, 8)
    assert cfg["sweep_ms"] > 0.0
    for a, b in zip(base, tuned):
        _same(a, b)
        assert a.records.tobytes() == b.records.tobytes()
    # the same class of batch reuses the tuned layout, in a graph replay too
    again, st = dses.register_batch(items, use_graph=True, records=True)
    assert st == [0] * len(probs)
    cfg2 = dses.batch_last_config()
    assert cfg2["source"] == "tuned-cache"
    assert (cfg2["items_per_cu"], cfg2["vote_parts"]) == (cfg["items_per_cu"], cfg["vote_parts"])
    for a, b in zip(base, again):
        assert a.records.tobytes() == b.records.tobytes()


@pytest.mark.parametrize("vote_parts", [1, 2, 3, 8, 16])
def test_vote_window_split_does_not_change_results(vote_parts):
    # references of 512..4096 points: 8..64 lane groups of 64, each group's source
    # window split into vote_parts units (an uneven 3 and more parts than points included)
    probs = _small_c3(count=4, k=256, seed=8)
    alone = [dses.register(p.src, p.tgt, p.rotations, p.eps, records=True) for p in probs]
    got, st = dses.register_batch([_as_dict(p) for p in probs], vote_parts=vote_parts,
                                  tile_rot=7, records=True)
    assert st == [0] * len(probs)
    cfg = dses.batch_last_config()
    assert cfg["source"] == "caller" and cfg["vote_parts"] == vote_parts
    for a, b in zip(alone, got):
        assert a.records.tobytes() == b.records.tobytes()
