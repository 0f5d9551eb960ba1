"""Allocation failures forced from the host with dses_debug_fail_allocs.

Every allocation the library makes, device or pinned host, goes through one
place that the hook can make fail.  Each entry point must then report the
failure (DSES_E_NOMEM or DSES_E_DEVICE), leave the objects it was given usable,
and give the same results as before once allocations succeed again; the
no-allocation entry point must run with every allocation failing.  No kernel
is launched on a failed allocation, so these tests never touch a bad address.
"""
import numpy as np
import pytest
import torch

from paper_2502_00115_amd import dses, synth

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

FAILED = (dses.DSES_E_NOMEM, dses.DSES_E_DEVICE)


@pytest.fixture(autouse=True)
def _injection_off_afterwards():
    yield
    dses.debug_fail_allocs(0, 0)


def _same(a, b):
    assert a.rot_index == b.rot_index and a.inliers == b.inliers and a.votes == b.votes
    assert a.error == b.error and a.n_valid == b.n_valid
    assert np.array_equal(a.R, b.R) and np.array_equal(a.t, b.t)


def _fails(fn):
    with pytest.raises(dses.DsesError) as e:
        fn()
    assert e.value.status in FAILED, e.value


def test_resident_objects_fail_cleanly_at_every_allocation():
    p = synth.make_c1(5)
    ref_t = dses.Target(p.tgt, df_trunc=p.eps, df_res=24)
    ref_r = dses.RotationSet(p.rotations)
    ref = dses.register_resident(ref_t, ref_r, p.src, p.eps, scorer="df")
    # a target with a distance field makes several allocations: fail each in turn
    failures = 0
    for skip in range(6):
        dses.debug_fail_allocs(skip, 1)
        try:
            t = dses.Target(p.tgt, df_trunc=p.eps, df_res=24)
        except dses.DsesError as e:
            assert e.status in FAILED, e
            failures += 1
            t = None
        finally:
            dses.debug_fail_allocs(0, 0)
        if t is not None:                   # the failure fell after its allocations
            _same(dses.register_resident(t, ref_r, p.src, p.eps, scorer="df"), ref)
            t.close()
    assert failures >= 1
    dses.debug_fail_allocs(0, 1)
    _fails(lambda: dses.RotationSet(p.rotations))
    dses.debug_fail_allocs(0, 0)
    _same(dses.register_resident(ref_t, dses.RotationSet(p.rotations), p.src, p.eps,
                                 scorer="df"), ref)


def test_resident_registration_recovers_after_failed_staging():
    p = synth.make_c1(6)
    fresh = dses.Target(p.tgt)
    rots = dses.RotationSet(p.rotations)
    ref = dses.register_resident(fresh, rots, p.src, p.eps)
    t = dses.Target(p.tgt)
    # the new target's first registration stages it (device allocations)
    dses.debug_fail_allocs(0, 1000)
    _fails(lambda: dses.register_resident(t, rots, p.src, p.eps))
    dses.debug_fail_allocs(0, 0)
    _same(dses.register_resident(t, rots, p.src, p.eps), ref)
    _same(dses.register_resident(t, rots, p.src, p.eps), ref)


def test_batch_recovers_after_failed_growth():
    probs = [synth.make_c1(100 + i) for i in range(96)]   # more instances than before
    items = [{"src": q.src, "tgt": q.tgt, "rotations": q.rotations, "eps": q.eps} for q in probs]
    alone = [dses.register(q.src, q.tgt, q.rotations, q.eps) for q in probs[:8]]
    dses.debug_fail_allocs(0, 1000)
    _fails(lambda: dses.register_batch(items, use_graph=False))
    dses.debug_fail_allocs(0, 0)
    for use_graph in (False, True):
        res, st = dses.register_batch(items, use_graph=use_graph)
        assert all(s == dses.DSES_OK for s in st)
        for a, b in zip(res[:8], alone):
            _same(a, b)


def test_server_creation_fails_cleanly_at_every_allocation():
    p = synth.make_c1(7)
    t, r = dses.Target(p.tgt), dses.RotationSet(p.rotations)
    ref = dses.register_resident(t, r, p.src, p.eps)
    created = 0
    for skip in range(0, 24, 3):
        dses.debug_fail_allocs(skip, 1)
        try:
            srv = dses.Server(memory_budget=64 << 20, max_inflight=8)
        except dses.DsesError as e:
            assert e.status in FAILED, e
            continue
        finally:
            dses.debug_fail_allocs(0, 0)
        created += 1
        srv.close()
    assert created < 8                      # at least one creation met the failure
    srv = dses.Server(memory_budget=64 << 20, max_inflight=8)
    try:
        _same(srv.wait(srv.submit(t, r, p.src, p.eps), timeout_ms=60000), ref)
    finally:
        srv.close()


def test_noalloc_runs_with_every_allocation_failing():
    p = synth.make_c2(4)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")  # noqa: E731
    s, t, r = dev(p.src), dev(p.tgt), dev(p.rotations)
    ref = dses.register(s, t, r, p.eps)
    first = dses.register_noalloc(s, t, r, p.eps)   # sets up the scratch address
    torch.cuda.synchronize()
    dses.debug_fail_allocs(0, 1 << 30)
    for _ in range(2):
        got = dses.register_noalloc(s, t, r, p.eps)
        torch.cuda.synchronize()
        _same(got, ref)
    _same(first, ref)
