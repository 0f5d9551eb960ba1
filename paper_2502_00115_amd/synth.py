"""Seeded synthetic inputs for DSES registration workloads.

This module only draws inputs: point clouds, rigid transforms and rotation
lists.  It holds none of the registration arithmetic (no voting, no binning,
no nearest-neighbour scoring), so both the HIP path and the CPU oracle may take
their inputs from here.

The clouds follow the paper's simulated-data protocol (Sec. V-A): objects
normalised into the unit sphere, source and reference sampled independently
from the same surface, Gaussian jitter clipped to +/-0.05 per axis, a random
half-space cut that keeps a fixed fraction of the source, and a random rigid
transform applied to the source.  The paper runs this on ModelNet40 meshes,
which are not available here; seeded ellipsoids and unions of boxes and
ellipsoids stand in for them.

Conventions
-----------
* Point clouds are float32 arrays of shape (n, 3), row-major xyz.
* A rotation list is a float32 array of shape (k, 9), row-major 3x3 matrices
  that map the source frame into the reference frame (applied as R x + t).
* The source is built as ``x = R_a y + t_a``; the registration answer is
  ``R = R_a^T`` and ``t = -R_a^T t_a``.
* Every generator takes a ``seed`` and uses ``numpy.random.default_rng``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "quat_to_matrix", "random_rotations", "hopf_grid",
    "healpix_centers", "ellipsoid_shape", "multi_primitive_shape",
    "sample_surface", "make_c1", "make_c1_exact", "make_c2", "make_c3",
    "make_c4_targets", "make_c4_request", "make_c5", "make_tiny",
]


@dataclass
class Problem:
    """One registration instance."""
    src: np.ndarray            # (N, 3) float32, partial source X
    tgt: np.ndarray            # (M, 3) float32, full reference Y
    rotations: np.ndarray      # (K, 9) float32 candidate rotations
    eps: float                 # inlier threshold = translation bin size
    R_true: np.ndarray         # (3, 3) float64 ground-truth rotation
    t_true: np.ndarray         # (3,) float64 ground-truth translation
    true_index: int = -1       # index of R_true in ``rotations`` (-1: not on the list)
    name: str = ""
    meta: dict = field(default_factory=dict)


# --------------------------------------------------------------------------
# rotations
# --------------------------------------------------------------------------
def quat_to_matrix(q: np.ndarray) -> np.ndarray:
    """Unit quaternions (w, x, y, z), shape (..., 4) -> rotation matrices (..., 3, 3)."""
    q = np.asarray(q, dtype=np.float64)
    q = q / np.linalg.norm(q, axis=-1, keepdims=True)
    w, x, y, z = q[..., 0], q[..., 1], q[..., 2], q[..., 3]
    R = np.empty(q.shape[:-1] + (3, 3))
    R[..., 0, 0] = 1 - 2 * (y * y + z * z)
    R[..., 0, 1] = 2 * (x * y - w * z)
    R[..., 0, 2] = 2 * (x * z + w * y)
    R[..., 1, 0] = 2 * (x * y + w * z)
    R[..., 1, 1] = 1 - 2 * (x * x + z * z)
    R[..., 1, 2] = 2 * (y * z - w * x)
    R[..., 2, 0] = 2 * (x * z - w * y)
    R[..., 2, 1] = 2 * (y * z + w * x)
    R[..., 2, 2] = 1 - 2 * (x * x + y * y)
    return R


def random_rotations(rng: np.random.Generator, k: int) -> np.ndarray:
    """k rotations uniform on SO(3): normalised 4-D Gaussians as unit quaternions."""
    return quat_to_matrix(rng.standard_normal((k, 4)))


def healpix_centers(nside: int) -> tuple[np.ndarray, np.ndarray]:
    """Centres (theta, phi) of the 12*nside^2 HEALPix pixels, ring scheme.

    Written from the pixel-centre equations of Gorski et al. (2005): polar-cap
    rings with 4i pixels, an equatorial belt of 4*nside pixels per ring with
    alternating half-pixel phase shifts, south cap mirrored.
    """
    zs, phis = [], []
    n2 = nside * nside
    for i in range(1, nside):                      # north polar cap
        z = 1.0 - i * i / (3.0 * n2)
        for j in range(1, 4 * i + 1):
            zs.append(z)
            phis.append(math.pi / (2.0 * i) * (j - 0.5))
    for i in range(nside, 3 * nside + 1):          # equatorial belt
        z = 4.0 / 3.0 - 2.0 * i / (3.0 * nside)
        s = (i - nside + 1) % 2
        for j in range(1, 4 * nside + 1):
            zs.append(z)
            phis.append(math.pi / (2.0 * nside) * (j - s / 2.0))
    for i in range(nside - 1, 0, -1):              # south polar cap
        z = -(1.0 - i * i / (3.0 * n2))
        for j in range(1, 4 * i + 1):
            zs.append(z)
            phis.append(math.pi / (2.0 * i) * (j - 0.5))
    z = np.asarray(zs)
    return np.arccos(np.clip(z, -1, 1)), np.asarray(phis)


def hopf_grid(level: int) -> np.ndarray:
    """Uniform SO(3) grid of 72 * 8**level rotations, shape (K, 3, 3), float64.

    Hopf-fibration construction of Yershova et al. (2010): a HEALPix grid on
    the base sphere S^2 (nside = 2**level) times a uniform grid of
    6 * 2**level angles on the fibre S^1, mapped to unit quaternions by the Hopf
    coordinates (cos(th/2)cos(psi/2), cos(th/2)sin(psi/2),
    sin(th/2)cos(phi+psi/2), sin(th/2)sin(phi+psi/2)).
    """
    nside = 2 ** level
    theta, phi = healpix_centers(nside)
    m = 6 * 2 ** level
    psi = (np.arange(m) + 0.5) * (2.0 * math.pi / m)
    th = theta[:, None] / 2.0
    ph = phi[:, None]
    ps = psi[None, :] / 2.0
    q = np.stack(np.broadcast_arrays(
        np.cos(th) * np.cos(ps),
        np.cos(th) * np.sin(ps),
        np.sin(th) * np.cos(ph + ps),
        np.sin(th) * np.sin(ph + ps)), axis=-1).reshape(-1, 4)
    return quat_to_matrix(q)


# --------------------------------------------------------------------------
# shapes and surface sampling
# --------------------------------------------------------------------------
@dataclass
class _Prim:
    kind: str                  # "ellipsoid" or "box"
    center: np.ndarray         # (3,)
    half: np.ndarray           # (3,) semi-axes / half-sizes
    rot: np.ndarray            # (3, 3) local -> world

    def area(self) -> float:
        a, b, c = self.half
        if self.kind == "box":
            return 8.0 * (a * b + b * c + a * c)
        p = 1.6075                                 # Knud Thomsen's approximation
        return 4 * math.pi * (((a * b) ** p + (a * c) ** p + (b * c) ** p) / 3.0) ** (1 / p)

    def sample(self, rng: np.random.Generator, n: int) -> np.ndarray:
        if n <= 0:
            return np.zeros((0, 3))
        loc = _sample_ellipsoid_local(rng, n, self.half) if self.kind == "ellipsoid" \
            else _sample_box_local(rng, n, self.half)
        return loc @ self.rot.T + self.center

    def inside(self, pts: np.ndarray, shrink: float = 1e-9) -> np.ndarray:
        loc = (pts - self.center) @ self.rot
        if self.kind == "box":
            return np.all(np.abs(loc) < self.half * (1 - shrink), axis=1)
        return np.sum((loc / self.half) ** 2, axis=1) < (1 - shrink)


def _sample_ellipsoid_local(rng, n, half):
    """Area-uniform points on an axis-aligned ellipsoid (rejection on the area element)."""
    a, b, c = half
    gmax = max(b * c, a * c, a * b)
    out = []
    have = 0
    while have < n:
        u = rng.standard_normal((2 * (n - have) + 16, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        g = np.sqrt((b * c * u[:, 0]) ** 2 + (a * c * u[:, 1]) ** 2 + (a * b * u[:, 2]) ** 2)
        keep = rng.random(len(u)) < g / gmax
        pts = u[keep] * half
        out.append(pts)
        have += len(pts)
    return np.concatenate(out)[:n]


def _sample_box_local(rng, n, half):
    """Area-uniform points on the surface of an axis-aligned box."""
    a, b, c = half
    areas = np.array([b * c, b * c, a * c, a * c, a * b, a * b])
    face = rng.choice(6, size=n, p=areas / areas.sum())
    uv = rng.uniform(-1, 1, size=(n, 2))
    pts = np.empty((n, 3))
    for f in range(6):
        sel = face == f
        axis, sign = f // 2, (1.0 if f % 2 == 0 else -1.0)
        others = [i for i in range(3) if i != axis]
        pts[sel, axis] = sign * half[axis]
        pts[sel, others[0]] = uv[sel, 0] * half[others[0]]
        pts[sel, others[1]] = uv[sel, 1] * half[others[1]]
    return pts


@dataclass
class Shape:
    prims: list
    center: np.ndarray
    scale: float

    def world(self, pts: np.ndarray) -> np.ndarray:
        return (pts - self.center) / self.scale


def _finish_shape(rng, prims) -> Shape:
    probe = sample_surface(rng, Shape(prims, np.zeros(3), 1.0), 20000)
    center = probe.mean(axis=0)
    scale = float(np.max(np.linalg.norm(probe - center, axis=1)))
    return Shape(prims, center, scale)


def ellipsoid_shape(rng: np.random.Generator) -> Shape:
    """Ellipsoid with semi-axes U[0.3, 1] in a random orientation, unit-sphere normalised."""
    half = rng.uniform(0.3, 1.0, size=3)
    prim = _Prim("ellipsoid", np.zeros(3), half, random_rotations(rng, 1)[0])
    return Shape([prim], np.zeros(3), float(half.max()))


def multi_primitive_shape(rng: np.random.Generator, n_prims: int | None = None) -> Shape:
    """Union of 3-6 boxes / ellipsoids (centres U[-.5,.5]^3, half-sizes U[.15,.5])."""
    if n_prims is None:
        n_prims = int(rng.integers(3, 7))
    prims = []
    for _ in range(n_prims):
        kind = "box" if rng.random() < 0.5 else "ellipsoid"
        prims.append(_Prim(kind, rng.uniform(-0.5, 0.5, 3), rng.uniform(0.15, 0.5, 3),
                           random_rotations(rng, 1)[0]))
    return _finish_shape(rng, prims)


def sample_surface(rng: np.random.Generator, shape: Shape, n: int) -> np.ndarray:
    """n area-uniform points on the outer surface of the union, in normalised coordinates."""
    areas = np.array([p.area() for p in shape.prims])
    out, have = [], 0
    while have < n:
        want = int(1.3 * (n - have)) + 32
        counts = rng.multinomial(want, areas / areas.sum())
        for pi, (prim, cnt) in enumerate(zip(shape.prims, counts)):
            pts = prim.sample(rng, int(cnt))
            keep = np.ones(len(pts), dtype=bool)
            for qi, other in enumerate(shape.prims):
                if qi != pi:
                    keep &= ~other.inside(pts)
            out.append(pts[keep])
            have += int(keep.sum())
    pts = np.concatenate(out)
    pts = pts[rng.permutation(len(pts))[:n]]
    return shape.world(pts)


# --------------------------------------------------------------------------
# corruption: noise, cuts, outliers, transforms
# --------------------------------------------------------------------------
def jitter(rng, pts, sigma, clip=0.05):
    if sigma <= 0:
        return pts.copy()
    noise = rng.normal(0.0, sigma, size=pts.shape)
    if clip is not None:
        noise = np.clip(noise, -clip, clip)
    return pts + noise


def halfspace_keep(rng, pts, keep_frac):
    """Indices of the points kept by a random-direction half-space shifted to keep a fraction."""
    d = rng.standard_normal(3)
    d /= np.linalg.norm(d)
    proj = pts @ d
    n_keep = int(round(keep_frac * len(pts)))
    order = np.argsort(-proj, kind="stable")
    return np.sort(order[:n_keep])


def add_outliers(rng, pts, frac, lo, hi):
    """Replace a fraction of the points by uniform points in the box [lo, hi]."""
    pts = pts.copy()
    n_out = int(round(frac * len(pts)))
    if n_out:
        idx = rng.choice(len(pts), size=n_out, replace=False)
        pts[idx] = rng.uniform(lo, hi, size=(n_out, 3))
    return pts


def random_transform(rng, t_range=0.5):
    R = random_rotations(rng, 1)[0]
    t = rng.uniform(-t_range, t_range, size=3)
    return R, t


def _apply(R, t, pts):
    return pts @ R.T + t


def _f32(a):
    return np.ascontiguousarray(np.asarray(a, dtype=np.float32))


def _rotlist(R):
    return _f32(np.asarray(R).reshape(-1, 9))


def euler_grid(K: int, step: float, center=None) -> np.ndarray:
    """(2K+1)^3 rotations C Rz(theta) Ry(phi) Rx(xi), theta, phi, xi in
    {-K step, ..., K step}, theta slowest (the loop order of the Euler
    parameterisation of Alg. 2; intrinsic z-y-x is the library's reading)."""
    C = np.eye(3) if center is None else np.asarray(center, np.float64).reshape(3, 3)
    a = (np.arange(-K, K + 1) * np.float64(np.float32(step)))
    th, ph, xi = np.meshgrid(a, a, a, indexing="ij")
    th, ph, xi = th.ravel(), ph.ravel(), xi.ravel()
    ct, st, cp, sp, cx, sx = np.cos(th), np.sin(th), np.cos(ph), np.sin(ph), np.cos(xi), np.sin(xi)
    z = np.zeros_like(th)
    Rz = np.stack([ct, -st, z, st, ct, z, z, z, z + 1], -1).reshape(-1, 3, 3)
    Ry = np.stack([cp, z, sp, z, z + 1, z, -sp, z, cp], -1).reshape(-1, 3, 3)
    Rx = np.stack([z + 1, z, z, z, cx, -sx, z, sx, cx], -1).reshape(-1, 3, 3)
    return C @ Rz @ Ry @ Rx


def _euler_one(th, ph, xi):
    ct, st, cp, sp, cx, sx = np.cos(th), np.sin(th), np.cos(ph), np.sin(ph), np.cos(xi), np.sin(xi)
    Rz = np.array([[ct, -st, 0], [st, ct, 0], [0, 0, 1]])
    Ry = np.array([[cp, 0, sp], [0, 1, 0], [-sp, 0, cp]])
    Rx = np.array([[1, 0, 0], [0, cx, -sx], [0, sx, cx]])
    return Rz @ Ry @ Rx


# --------------------------------------------------------------------------
# workloads
# --------------------------------------------------------------------------
def make_c1(seed: int) -> Problem:
    """Plain DSES: 256-pt ellipsoid target, 64-pt noisy half-cut source, 576 random
    rotations plus the true one at a seeded position; eps = 0.05."""
    rng = np.random.default_rng(seed)
    shape = ellipsoid_shape(rng)
    prim = shape.prims[0]
    tgt = prim.sample(rng, 256)
    tgt = tgt - tgt.mean(axis=0)
    tgt = tgt / np.max(np.linalg.norm(tgt, axis=1))
    d = rng.standard_normal(3)
    side = np.nonzero(tgt @ d >= 0)[0]
    pick = rng.choice(side, size=min(64, len(side)), replace=False)
    part = jitter(rng, tgt[pick], 0.005, clip=None)
    Ra, ta = random_transform(rng)
    src = _apply(Ra, ta, part)
    rots = random_rotations(rng, 576)
    pos = int(rng.integers(0, 577))
    rots = np.insert(rots, pos, Ra.T, axis=0)
    return Problem(_f32(src), _f32(tgt), _rotlist(rots), 0.05, Ra.T, -Ra.T @ ta, pos, f"c1-s{seed}")


def make_c1_exact(seed: int, delta: float = 0.05, n_src: int = 64, n_tgt: int = 256,
                  n_rot: int = 576) -> Problem:
    """Exact-recovery variant of C1: noise-free exact subset, answer t on the delta lattice.

    The source is ``R*^T (y - t*)`` for a subset of the target, with ``R*`` on the
    rotation list and ``t*`` a multiple of ``delta``; the answer is {R*, t*}.
    """
    rng = np.random.default_rng(seed)
    shape = ellipsoid_shape(rng)
    tgt = shape.prims[0].sample(rng, n_tgt)
    tgt = tgt - tgt.mean(axis=0)
    tgt = tgt / np.max(np.linalg.norm(tgt, axis=1))
    tgt32 = _f32(tgt).astype(np.float64)
    d = rng.standard_normal(3)
    side = np.nonzero(tgt32 @ d >= 0)[0]
    pick = rng.choice(side, size=min(n_src, len(side)), replace=False)
    Rs = random_rotations(rng, 1)[0]
    Rs32 = _f32(Rs).astype(np.float64)
    t_star = np.round(rng.uniform(-0.5, 0.5, size=3) / delta) * delta
    src = (tgt32[pick] - t_star) @ Rs32          # rows of R*^T (y - t*)
    rots = random_rotations(rng, n_rot)
    pos = int(rng.integers(0, n_rot + 1))
    rots = np.insert(rots, pos, Rs32, axis=0)
    return Problem(_f32(src), _f32(tgt32), _rotlist(rots), delta, Rs32, t_star, pos,
                   f"c1x-s{seed}")


def _partial_source(rng, shape, n_sample, keep_frac, sigma, outlier_frac, t_range=0.5):
    src = sample_surface(rng, shape, n_sample)
    src = src[halfspace_keep(rng, src, keep_frac)]
    src = jitter(rng, src, sigma, clip=0.05)
    lo, hi = src.min(axis=0), src.max(axis=0)
    src = add_outliers(rng, src, outlier_frac, lo, hi)
    Ra, ta = random_transform(rng, t_range)
    return _apply(Ra, ta, src), Ra, ta


def make_c2(seed: int, grid_level: int = 3) -> Problem:
    """Object-scale registration: 1,024-pt multi-primitive target, 717-pt partial source
    (70% cut of an independent 1,024-pt sample), sigma 0.01 clipped at 0.05, 10%
    outliers, 36,864-rotation Hopf grid; eps = 0.03."""
    rng = np.random.default_rng(1000 + seed)
    shape = multi_primitive_shape(rng)
    tgt = sample_surface(rng, shape, 1024)
    src, Ra, ta = _partial_source(rng, shape, 1024, 0.7, 0.01, 0.10)
    rots = hopf_grid(grid_level)
    return Problem(_f32(src), _f32(tgt), _rotlist(rots), 0.03, Ra.T, -Ra.T @ ta, -1,
                   f"c2-s{seed}")


def make_c3(seed: int, count: int = 64) -> list[Problem]:
    """Batch of registrations: target sizes log-uniform 512-4096, source 30-80% of the
    target by a half-space cut, 0-30% outliers, and the first K of a seeded permutation of
    the 36,864-rotation grid with K log-uniform in [4,608, 36,864]; eps = 0.03."""
    rng = np.random.default_rng(3000 + seed)
    grid = hopf_grid(3)
    out = []
    for b in range(count):
        m = int(round(math.exp(rng.uniform(math.log(512), math.log(4096)))))
        shape = multi_primitive_shape(rng)
        tgt = sample_surface(rng, shape, m)
        frac = rng.uniform(0.3, 0.8)
        src, Ra, ta = _partial_source(rng, shape, m, frac, 0.01, rng.uniform(0.0, 0.3))
        k = int(round(math.exp(rng.uniform(math.log(4608), math.log(36864)))))
        perm = rng.permutation(len(grid))[:k]
        out.append(Problem(_f32(src), _f32(tgt), _rotlist(grid[perm]), 0.03, Ra.T, -Ra.T @ ta,
                           -1, f"c3-s{seed}-{b}"))
    return out


def make_c4_targets(seed: int, count: int = 8) -> list[np.ndarray]:
    """Resident reference clouds for serving: M log-uniform in [2,048, 8,192]."""
    rng = np.random.default_rng(4000 + seed)
    tg = []
    for _ in range(count):
        m = int(round(math.exp(rng.uniform(math.log(2048), math.log(8192)))))
        shape = multi_primitive_shape(rng)
        tg.append((_f32(sample_surface(rng, shape, m)), shape))
    return tg


def make_c4_request(seed: int, targets) -> tuple[int, np.ndarray]:
    """One serving request: a target id and a 256-4,096-pt source with 20% outliers."""
    rng = np.random.default_rng(5000 + seed)
    tid = int(rng.integers(0, len(targets)))
    _, shape = targets[tid]
    n = int(round(math.exp(rng.uniform(math.log(256), math.log(4096)))))
    src, _, _ = _partial_source(rng, shape, int(round(n / 0.7)), 0.7, 0.01, 0.20)
    return tid, _f32(src[:n])


def make_c5(seed: int, grid_level: int = 4) -> Problem:
    """Scene-scale: 16,384-pt six-primitive target, 4,096-pt partial source (sigma 0.005,
    20% outliers), 294,912-rotation Hopf grid; eps = 0.02."""
    rng = np.random.default_rng(6000 + seed)
    shape = multi_primitive_shape(rng, 6)
    tgt = sample_surface(rng, shape, 16384)
    src, Ra, ta = _partial_source(rng, shape, int(round(4096 / 0.7)) + 1, 0.7, 0.005, 0.20)
    src = src[:4096]
    rots = hopf_grid(grid_level)
    return Problem(_f32(src), _f32(tgt), _rotlist(rots), 0.02, Ra.T, -Ra.T @ ta, -1,
                   f"c5-s{seed}")


def make_local(seed: int, K: int = 10, step_deg: float = 0.5) -> Problem:
    """Local registration with an initial guess (stand-in for the paper's on-robot
    gripper pose correction, whose clouds are not available): a multi-primitive
    object of radius 0.1 m (metres), 2,048 reference points, a 70% partial view of
    an independent 2,048-point sample with 1 mm noise (clipped at 5 mm) and 10%
    outliers, displaced by a rotation of up to 4 degrees per Euler angle and a
    translation of up to 1.2 cm per axis.  Rotations: the Euler grid of +-K step
    around the identity (default +-5 degrees in 0.5-degree steps, 9,261 rotations);
    translation box +-1.6 cm; eps = delta = 2 mm."""
    rng = np.random.default_rng(6000 + seed)
    shape = multi_primitive_shape(rng)
    tgt = 0.1 * sample_surface(rng, shape, 2048)
    src = 0.1 * sample_surface(rng, shape, 2048)
    src = src[halfspace_keep(rng, src, 0.7)]
    src = jitter(rng, src, 0.001, clip=0.005)
    src = add_outliers(rng, src, 0.10, src.min(axis=0), src.max(axis=0))
    Ra = _euler_one(*rng.uniform(-np.deg2rad(4.0), np.deg2rad(4.0), size=3))
    ta = rng.uniform(-0.012, 0.012, size=3)
    src = _apply(Ra, ta, src)
    rots = euler_grid(K, np.deg2rad(step_deg))
    return Problem(_f32(src), _f32(tgt), _rotlist(rots), 0.002, Ra.T, -Ra.T @ ta, -1,
                   f"local-s{seed}", {"t_box": 0.016})


def make_tiny(seed: int, n: int = 6, m: int = 8, k: int = 4, delta: float = 0.0625,
              spread: float = 0.5) -> Problem:
    """Tiny random instance for brute-force checks (coordinates within +/-spread)."""
    rng = np.random.default_rng(9000 + seed)
    tgt = rng.uniform(-spread, spread, size=(m, 3))
    src = rng.uniform(-spread, spread, size=(n, 3))
    rots = random_rotations(rng, k)
    return Problem(_f32(src), _f32(tgt), _rotlist(rots), delta, np.eye(3), np.zeros(3), -1,
                   f"tiny-s{seed}")
