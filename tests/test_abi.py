"""The C ABI library builds, loads, and exports what include/dses.h declares (CPU only)."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "dses.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dses_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2502_00115_amd import dses
    if not os.path.exists(dses.LIB_PATH):
        from paper_2502_00115_amd import build_lib
        build_lib.build()
    return dses.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["dses_register", "dses_register_batch", "dses_target_create",
                 "dses_rotations_create", "dses_server_create", "dses_server_submit",
                 "dses_server_wait", "dses_last_error"]:
        assert must in names


def test_library_exports_every_declared_symbol(libpath):
    out = subprocess.check_output(["nm", "-D", "--defined-only", libpath]).decode()
    exported = set(re.findall(r"\bT (dses_[a-z_]+)\b", out))
    missing = [n for n in _declared() if n not in exported]
    assert not missing, missing


def test_binding_lists_match_header():
    from paper_2502_00115_amd import dses
    assert sorted(dses.EXPORTED) == _declared()


def test_library_is_gfx950_code_object(libpath):
    out = subprocess.check_output(["strings", libpath]).decode(errors="replace")
    assert "gfx950" in out


def test_argument_errors_need_no_gpu(libpath):
    import numpy as np
    from paper_2502_00115_amd import dses
    cases = [
        (np.zeros((0, 3)), np.zeros((4, 3)), np.eye(3).reshape(1, 9), 0.05, {}),
        (np.zeros((3, 3)), np.zeros((4, 3)), np.eye(3).reshape(1, 9), 0.0, {}),
        (np.zeros((3, 3)), np.zeros((4, 3)), np.eye(3).reshape(1, 9), float("nan"), {}),
        (np.zeros((3, 3)), np.zeros((4, 3)), np.eye(3).reshape(1, 9), 0.05,
         {"t_min": 1.0, "t_max": -1.0}),
        (np.zeros((3, 3)), np.zeros((4, 3)), np.eye(3).reshape(1, 9), 0.05,
         {"scorer": "df"}),
    ]
    for s, t, r, eps, kw in cases:
        with pytest.raises(dses.DsesError) as e:
            dses.register(s, t, r, eps, **kw)
        assert e.value.status == dses.DSES_E_INVAL, (kw, e.value)
    with pytest.raises(ValueError):
        dses.register(np.zeros((4, 2)), np.zeros((4, 3)), np.eye(3).reshape(1, 9), 0.05)
    # the allocation-failure hook checks its arguments on the host
    for skip, count in ((-1, 1), (0, -1)):
        with pytest.raises(dses.DsesError) as e:
            dses.debug_fail_allocs(skip, count)
        assert e.value.status == dses.DSES_E_INVAL
    dses.debug_fail_allocs(0, 0)
    for q in (-0.1, 1.5, float("nan")):
        with pytest.raises(dses.DsesError) as e:
            dses.register(np.zeros((3, 3)), np.zeros((4, 3)), np.eye(3).reshape(1, 9), 0.05, q=q)
        assert e.value.status == dses.DSES_E_INVAL, (q, e.value)
    for lg in (-1, 8, 48, 128):
        with pytest.raises(dses.DsesError) as e:
            dses.register(np.zeros((3, 3)), np.zeros((4, 3)), np.eye(3).reshape(1, 9), 0.05,
                          lane_group=lg)
        assert e.value.status == dses.DSES_E_INVAL, (lg, e.value)
    item = {"src": np.zeros((3, 3)), "tgt": np.zeros((4, 3)),
            "rotations": np.eye(3).reshape(1, 9), "eps": 0.05}
    for kw in ({"vote_parts": 17}, {"vote_parts": -1}, {"tile_rot": -2}):
        with pytest.raises(dses.DsesError) as e:
            dses.register_batch([item], **kw)
        assert e.value.status == dses.DSES_E_INVAL, (kw, e.value)
    with pytest.raises(dses.DsesError) as e:
        dses.Server(slice_mpairs=-1)
    assert e.value.status == dses.DSES_E_INVAL


def test_options_size_and_df_lookup_checked_on_the_host(libpath):
    """dses_options is versioned by struct_size: a size below the oldest layout or
    above the current one is rejected, the older layout (without df_lookup) is
    accepted; an unknown df_lookup is rejected before any device work."""
    import ctypes as C
    import numpy as np
    import torch
    from paper_2502_00115_amd import dses
    L = dses.lib()
    src = np.zeros((3, 3), np.float32)
    tgt = np.zeros((4, 3), np.float32)
    rot = np.eye(3, dtype=np.float32).reshape(1, 9)

    def call(o):
        res = dses.Result()
        return L.dses_register(src.ctypes.data, 3, tgt.ctypes.data, 4, rot.ctypes.data, 1,
                               C.c_float(0.05), 0, C.byref(o), C.byref(res))

    o = dses.Options()
    o.struct_size = C.sizeof(dses.Options)
    o.df_lookup = 2
    assert call(o) == dses.DSES_E_INVAL
    for size in (8, C.sizeof(dses.Options) + 4):
        o = dses.Options()
        o.struct_size = size
        assert call(o) == dses.DSES_E_INVAL, size
    o = dses.Options()
    o.struct_size = dses.Options.df_lookup.offset
    o.df_lookup = 7            # not read: beyond the declared size
    expect = dses.DSES_OK if torch.cuda.is_available() else dses.DSES_E_DEVICE
    assert call(o) in (expect, dses.DSES_E_NOCANDIDATE)
    bo = dses.BatchOpts(C.sizeof(dses.BatchOpts), 0, 0, 0, 0, 0, None, 5)
    probs = (dses.Problem * 1)()
    probs[0].src, probs[0].n = src.ctypes.data, 3
    probs[0].tgt, probs[0].m = tgt.ctypes.data, 4
    probs[0].rotations, probs[0].k = rot.ctypes.data, 1
    probs[0].eps = 0.05
    res = (dses.Result * 1)()
    st = (C.c_int32 * 1)()
    assert L.dses_register_batch(probs, 1, C.byref(bo), res, st) == dses.DSES_E_INVAL


def test_no_device_is_a_loud_error(libpath):
    import numpy as np
    import torch
    from paper_2502_00115_amd import dses
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(dses.DsesError) as e:
        dses.register(np.zeros((3, 3)), np.zeros((4, 3)), np.eye(3).reshape(1, 9), 0.05)
    assert e.value.status == dses.DSES_E_DEVICE


def test_euler_rotation_grid_needs_no_gpu(libpath):
    import numpy as np
    from scipy.spatial.transform import Rotation
    from paper_2502_00115_amd import dses
    K, step = 2, float(np.float32(np.deg2rad(3.0)))
    C = Rotation.from_euler("xyz", [5, 40, -70], degrees=True).as_matrix().astype(np.float32)
    a = np.arange(-K, K + 1) * step
    ref = np.stack([C.astype(np.float64) @ Rotation.from_euler("ZYX", [t, p, x]).as_matrix()
                    for t in a for p in a for x in a])
    got = dses.euler_grid(K, step, C).reshape(-1, 3, 3)
    np.testing.assert_allclose(got, ref, atol=1e-6)
    for bad_step in (0.0, float("nan")):
        with pytest.raises(dses.DsesError):
            dses.euler_grid(K, bad_step)
