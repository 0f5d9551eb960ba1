"""Checks of the seeded input generators (no registration arithmetic involved)."""
import numpy as np
import pytest

from paper_2502_00115_amd import synth


def _geodesic(Ra, Rb):
    c = (np.einsum("...ij,...ij->...", Ra, Rb) - 1.0) / 2.0
    return np.arccos(np.clip(c, -1, 1))


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_hopf_grid_is_a_rotation_grid(level):
    R = synth.hopf_grid(level)
    assert R.shape == (72 * 8 ** level, 3, 3)
    np.testing.assert_allclose(np.einsum("kji,kjl->kil", R, R), np.broadcast_to(np.eye(3), R.shape),
                               atol=1e-12)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)


def test_hopf_grid_refines_uniformly():
    rng = np.random.default_rng(0)
    probe = synth.random_rotations(rng, 400)
    cover = []
    for level in (0, 1, 2):
        G = synth.hopf_grid(level)
        d = np.array([_geodesic(G, p[None]).min() for p in probe])
        cover.append(d.max())
        own = np.array([np.sort(_geodesic(G, g[None]))[1] for g in G[:: max(1, len(G) // 200)]])
        assert own.min() > 0.2 * (np.pi / 2 ** level) / 3        # no near-duplicates
    assert cover[1] < 0.7 * cover[0] and cover[2] < 0.7 * cover[1]


def test_healpix_count_and_equal_area_rings():
    for nside in (1, 2, 4):
        th, ph = synth.healpix_centers(nside)
        assert len(th) == 12 * nside ** 2
        z = np.cos(th)
        assert abs(z.mean()) < 1e-12        # symmetric about the equator


def test_random_rotations_are_rotations():
    R = synth.random_rotations(np.random.default_rng(1), 100)
    np.testing.assert_allclose(np.linalg.det(R), 1.0, atol=1e-12)


@pytest.mark.parametrize("seed", [0, 1])
def test_c1_layout_and_truth(seed):
    p = synth.make_c1(seed)
    assert p.src.shape == (64, 3) and p.tgt.shape == (256, 3) and p.rotations.shape == (577, 9)
    assert p.src.dtype == np.float32 and p.rotations.dtype == np.float32
    np.testing.assert_allclose(p.rotations[p.true_index].reshape(3, 3), p.R_true, atol=1e-6)
    assert np.max(np.linalg.norm(p.tgt, axis=1)) == pytest.approx(1.0, abs=1e-6)
    q = p.src.astype(float) @ p.R_true.T + p.t_true
    d = np.min(np.linalg.norm(q[:, None] - p.tgt[None].astype(float), axis=2), axis=1)
    assert d.max() < 0.05                           # sigma = 0.005 jitter only


def test_c1_exact_is_exact():
    p = synth.make_c1_exact(0)
    R = p.rotations[p.true_index].reshape(3, 3).astype(float)
    q = p.src.astype(float) @ R.T + p.t_true
    d = np.min(np.linalg.norm(q[:, None] - p.tgt[None].astype(float), axis=2), axis=1)
    assert d.max() < 1e-6
    np.testing.assert_allclose(p.t_true / p.eps, np.round(p.t_true / p.eps), atol=1e-12)


def test_c2_c5_shapes():
    p = synth.make_c2(0)
    assert p.src.shape == (717, 3) and p.tgt.shape == (1024, 3) and p.rotations.shape == (36864, 9)
    assert np.max(np.linalg.norm(p.tgt, axis=1)) <= 1.0 + 1e-6
    p5 = synth.make_c5(0, grid_level=2)
    assert p5.src.shape == (4096, 3) and p5.tgt.shape == (16384, 3)


def test_c3_distribution():
    batch = synth.make_c3(0, count=8)
    for p in batch:
        m, n, k = len(p.tgt), len(p.src), len(p.rotations)
        assert 512 <= m <= 4096 and 0.29 * m <= n <= 0.81 * m and 4608 <= k <= 36864


def test_generators_are_deterministic():
    a, b = synth.make_c2(1), synth.make_c2(1)
    np.testing.assert_array_equal(a.src, b.src)
    np.testing.assert_array_equal(a.tgt, b.tgt)


def test_euler_grid_matches_scipy_intrinsic_zyx():
    from scipy.spatial.transform import Rotation
    K, step = 3, float(np.float32(np.deg2rad(2.5)))
    C = Rotation.from_euler("xyz", [10, -20, 30], degrees=True).as_matrix()
    a = np.arange(-K, K + 1) * step
    ref = np.stack([C @ Rotation.from_euler("ZYX", [t, p, x]).as_matrix()
                    for t in a for p in a for x in a])
    np.testing.assert_allclose(synth.euler_grid(K, step, C), ref, atol=1e-12)


def test_local_workload_truth_is_inside_the_search_range():
    p = synth.make_local(1)
    ang = np.rad2deg(np.arccos(np.clip((np.trace(p.R_true) - 1) / 2, -1, 1)))
    assert ang < 7.0 and np.all(np.abs(p.t_true) < p.meta["t_box"])
