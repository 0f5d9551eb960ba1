"""dses_register_noalloc against dses_register: the same kernels on buffers taken
from the library's static device scratch array.  Two calls in a row (the second
smaller, so it runs on the larger call's leftovers in the array), each compared
bit for bit with dses_register and against the oracle; a call that needs more than
the array is refused with DSES_E_NOMEM."""
import numpy as np
import pytest
import torch

import oracle
from paper_2502_00115_amd import dses, synth
from parity import check_selection, compare_records

pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def _same(a, b):
    assert a.rot_index == b.rot_index and a.inliers == b.inliers and a.votes == b.votes
    assert a.error == b.error and a.n_valid == b.n_valid
    assert np.array_equal(a.R, b.R) and np.array_equal(a.t, b.t)


def test_noalloc_equals_register_on_two_calls_in_a_row():
    big = synth.make_c2(1)
    small = synth.make_c1(3)
    for p, sample in ((big, 384), (small, None)):
        s, t, r = _dev(p.src), _dev(p.tgt), _dev(p.rotations)
        got = dses.register_noalloc(s, t, r, p.eps, records=True)
        ref = dses.register(s, t, r, p.eps, records=True)
        torch.cuda.synchronize()
        _same(got, ref)
        assert got.records.tobytes() == ref.records.tobytes(), p.name
        # the oracle's bar, on every rotation of the small call and on sampled
        # rotations (plus the GPU's best) of the large one
        recs = got.records
        if sample is None:
            which = np.arange(len(p.rotations))
        else:
            rng = np.random.default_rng(7)
            top = np.argsort(np.where(recs["votes"] > 0, recs["error"], np.inf))[:16]
            which = np.unique(np.concatenate([rng.choice(len(p.rotations), sample,
                                                         replace=False), top]))
        orc = oracle.records(p.src, p.tgt, p.rotations, p.eps, which=which)
        rep = compare_records(recs[which], orc, len(p.src), label=f"noalloc {p.name}")
        check_selection(got, rep, p.eps, label=f"noalloc {p.name}")


def test_noalloc_without_records_and_with_options():
    p = synth.make_c1(5)
    s, t, r = _dev(p.src), _dev(p.tgt), _dev(p.rotations)
    kw = dict(delta_t=0.04, tau=0.06, t_min=-0.9, t_max=0.9)
    got = dses.register_noalloc(s, t, r, p.eps, "tls", **kw)
    ref = dses.register(s, t, r, p.eps, "tls", **kw)
    _same(got, ref)


def test_noalloc_refuses_calls_beyond_the_array():
    cap = dses.noalloc_scratch_bytes()
    assert cap == 64 << 20
    p = synth.make_c1(0)
    k = cap // 24 + 1024                      # the records alone exceed the array
    r = _dev(p.rotations[:1]).expand(k, 9).contiguous()
    with pytest.raises(dses.DsesError) as e:
        dses.register_noalloc(_dev(p.src), _dev(p.tgt), r, p.eps)
    assert e.value.status == dses.DSES_E_NOMEM and "MiB" in str(e.value)
    # the array is still usable afterwards
    s, t, rr = _dev(p.src), _dev(p.tgt), _dev(p.rotations)
    _same(dses.register_noalloc(s, t, rr, p.eps), dses.register(s, t, rr, p.eps))


def test_noalloc_rejects_host_pointers_and_unsupported_options():
    p = synth.make_c1(0)
    with pytest.raises(ValueError):
        dses.register_noalloc(p.src, p.tgt, p.rotations, p.eps)
    s, t, r = _dev(p.src), _dev(p.tgt), _dev(p.rotations)
    with pytest.raises(dses.DsesError) as e:
        dses.register_noalloc(s, t, r, p.eps, scorer="df")
    assert e.value.status == dses.DSES_E_INVAL
