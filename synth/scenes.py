"""Seeded synthetic aerial scenes, cameras and pose sets.

Every array is produced with numpy's PCG64 generator.  The workloads stand in
for the paper's remote-sensing datasets (Mill 19-Rubble, Xi-MSTS, Sec. 4.1 and
Table 1), which are not available: a 1 km^2 heightfield with box "buildings",
Gaussian primitives carrying centre, rotation, scale, opacity, colour and a
feature vector (the primitive of Sec. 3.1), seen from a downward-looking UAV
camera at 100-300 m altitude.

Conventions (shared by the renderer and the oracle, stated once here):
  * means (N,3) float32, world metres, Z up.
  * log_scales (N,3) float32: per-axis log of the standard deviation.
  * quats (N,4) float32 in (w, x, y, z) order, not necessarily unit length.
  * opacities (N,) float32, already in [0, 1].
  * sh (N, (deg+1)^2, 3) float32, coefficient-major, RGB last.
  * feat (N, D) uint16: bfloat16 bit patterns.
  * pose: (12,) float32, row-major [R | t] mapping world to camera,
    x_c = R x_w + t, camera axes x right, y down, z forward.
  * camera: pinhole fx, fy, cx, cy in pixels; pixel (i, j) has its centre at
    (i + 0.5, j + 0.5).

The DC colour coefficient is drawn uniformly on [-sqrt(pi), sqrt(pi)]: with the
real degree-0 harmonic 1/(2 sqrt(pi)) and the +0.5 colour offset this makes the
degree-0 colour uniform on [0, 1].
"""
from __future__ import annotations

import dataclasses
import math
from typing import Optional

import numpy as np
from scipy.spatial.transform import Rotation

SQRT_PI = math.sqrt(math.pi)


# --------------------------------------------------------------------------
# containers
# --------------------------------------------------------------------------
@dataclasses.dataclass
class Scene:
    means: np.ndarray
    log_scales: np.ndarray
    quats: np.ndarray
    opacities: np.ndarray
    sh: np.ndarray
    sh_degree: int
    feat: Optional[np.ndarray] = None          # (N, D) uint16 bf16 bits
    part_offsets: Optional[np.ndarray] = None  # (n_parts + 1,) int64

    @property
    def n(self) -> int:
        return int(self.means.shape[0])

    @property
    def feat_dim(self) -> int:
        return 0 if self.feat is None else int(self.feat.shape[1])

    def subset(self, idx) -> "Scene":
        idx = np.asarray(idx)
        return Scene(
            means=np.ascontiguousarray(self.means[idx]),
            log_scales=np.ascontiguousarray(self.log_scales[idx]),
            quats=np.ascontiguousarray(self.quats[idx]),
            opacities=np.ascontiguousarray(self.opacities[idx]),
            sh=np.ascontiguousarray(self.sh[idx]),
            sh_degree=self.sh_degree,
            feat=None if self.feat is None else np.ascontiguousarray(self.feat[idx]),
        )

    def copy(self) -> "Scene":
        return Scene(
            means=self.means.copy(), log_scales=self.log_scales.copy(),
            quats=self.quats.copy(), opacities=self.opacities.copy(),
            sh=self.sh.copy(), sh_degree=self.sh_degree,
            feat=None if self.feat is None else self.feat.copy(),
            part_offsets=None if self.part_offsets is None else self.part_offsets.copy(),
        )


@dataclasses.dataclass
class Camera:
    fx: float
    fy: float
    cx: float
    cy: float
    width: int
    height: int


# --------------------------------------------------------------------------
# bf16 bit helpers (round to nearest even)
# --------------------------------------------------------------------------
def f32_to_bf16_bits(x: np.ndarray) -> np.ndarray:
    b = np.ascontiguousarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    rounded = (b + 0x7FFF + ((b >> 16) & 1)) >> 16
    return rounded.astype(np.uint16)


def bf16_bits_to_f32(b: np.ndarray) -> np.ndarray:
    return (np.asarray(b, dtype=np.uint32) << 16).view(np.float32)


# --------------------------------------------------------------------------
# primitive draws
# --------------------------------------------------------------------------
def _terrain_height(x, y):
    return 8.0 * np.sin(x / 23.0) * np.cos(y / 31.0)


def _unit_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q.astype(np.float32)


def _sigmoid_opacity(rng, n):
    return (1.0 / (1.0 + np.exp(-rng.standard_normal(n)))).astype(np.float32)


def _sh(rng, n, degree):
    k = (degree + 1) ** 2
    sh = np.empty((n, k, 3), dtype=np.float32)
    sh[:, 0, :] = rng.uniform(-SQRT_PI, SQRT_PI, size=(n, 3))
    if k > 1:
        sh[:, 1:, :] = rng.normal(0.0, 0.2, size=(n, k - 1, 3))
    return sh


def _features(rng, n, dim):
    f = rng.standard_normal((n, dim)).astype(np.float32)
    f /= np.linalg.norm(f, axis=1, keepdims=True).astype(np.float32)
    return f32_to_bf16_bits(f)


def terrain_scene(n, extent, seed, sh_degree=0, feat_dim=0, noise=0.5,
                  centre=(0.0, 0.0)) -> Scene:
    """n Gaussians on z = 8 sin(x/23) cos(y/31) + N(0, noise) over a square of
    side `extent` metres centred at `centre`."""
    rng = np.random.Generator(np.random.PCG64(seed))
    x = rng.uniform(-extent / 2, extent / 2, n) + centre[0]
    y = rng.uniform(-extent / 2, extent / 2, n) + centre[1]
    z = _terrain_height(x, y) + rng.normal(0.0, noise, n)
    means = np.stack([x, y, z], axis=1).astype(np.float32)
    log_scales = rng.normal(-0.5, 0.3, (n, 3)).astype(np.float32)
    quats = _unit_quats(rng, n)
    opac = _sigmoid_opacity(rng, n)
    sh = _sh(rng, n, sh_degree)
    feat = _features(rng, n, feat_dim) if feat_dim else None
    return Scene(means, log_scales, quats, opac, sh, sh_degree, feat)


def _building_points(rng, n_boxes, per_box, extent, centre):
    """Points uniform (area-weighted) on the 4 walls and the roof of boxes."""
    pts = np.empty((n_boxes * per_box, 3))
    cx = rng.uniform(-extent / 2 + 20, extent / 2 - 20, n_boxes) + centre[0]
    cy = rng.uniform(-extent / 2 + 20, extent / 2 - 20, n_boxes) + centre[1]
    sx = rng.uniform(8.0, 30.0, n_boxes)
    sy = rng.uniform(8.0, 30.0, n_boxes)
    hz = rng.uniform(5.0, 40.0, n_boxes)
    yaw = rng.uniform(0.0, math.pi / 2, n_boxes)
    base = _terrain_height(cx, cy)
    for b in range(n_boxes):
        areas = np.array([sx[b] * hz[b], sx[b] * hz[b], sy[b] * hz[b], sy[b] * hz[b], sx[b] * sy[b]])
        face = rng.choice(5, size=per_box, p=areas / areas.sum())
        a = rng.uniform(-0.5, 0.5, per_box)
        h = rng.uniform(0.0, 1.0, per_box)
        lx = np.where(face == 0, a * sx[b], np.where(face == 1, a * sx[b],
             np.where(face == 2, -0.5 * sx[b], np.where(face == 3, 0.5 * sx[b], a * sx[b]))))
        ly = np.where(face == 0, -0.5 * sy[b], np.where(face == 1, 0.5 * sy[b],
             np.where(face <= 3, a * sy[b], rng.uniform(-0.5, 0.5, per_box) * sy[b])))
        lz = np.where(face == 4, hz[b], h * hz[b])
        c, s = math.cos(yaw[b]), math.sin(yaw[b])
        sl = slice(b * per_box, (b + 1) * per_box)
        pts[sl, 0] = cx[b] + c * lx - s * ly
        pts[sl, 1] = cy[b] + s * lx + c * ly
        pts[sl, 2] = base[b] + lz
    return pts


def aerial_scene(n_total, extent, seed, sh_degree=3, feat_dim=32, n_boxes=2000,
                 per_box=50, centre=(0.0, 0.0)) -> Scene:
    """Terrain plus box buildings: n_total Gaussians, n_boxes*per_box of them on
    the buildings' walls and roofs."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n_b = n_boxes * per_box
    n_t = n_total - n_b
    x = rng.uniform(-extent / 2, extent / 2, n_t) + centre[0]
    y = rng.uniform(-extent / 2, extent / 2, n_t) + centre[1]
    z = _terrain_height(x, y) + rng.normal(0.0, 0.5, n_t)
    terrain = np.stack([x, y, z], axis=1)
    bpts = _building_points(rng, n_boxes, per_box, extent, centre) if n_boxes else np.zeros((0, 3))
    means = np.concatenate([terrain, bpts]).astype(np.float32)
    n = means.shape[0]
    log_scales = rng.normal(-0.5, 0.3, (n, 3)).astype(np.float32)
    quats = _unit_quats(rng, n)
    opac = _sigmoid_opacity(rng, n)
    sh = _sh(rng, n, sh_degree)
    feat = _features(rng, n, feat_dim) if feat_dim else None
    return Scene(means, log_scales, quats, opac, sh, sh_degree, feat)


def partitioned_scene(n_total, extent, seed, cells_per_side=4, sh_degree=0, feat_dim=32,
                      boxes_per_km2=2000, per_box=50) -> Scene:
    """A square scene of side `extent` stored as cells_per_side^2 contiguous
    spatial partitions (row-major cells), each drawn like `aerial_scene`."""
    cells = cells_per_side * cells_per_side
    cell = extent / cells_per_side
    n_cell = n_total // cells
    boxes = int(round(boxes_per_km2 * (cell / 1000.0) ** 2))
    parts = []
    for c in range(cells):
        cxy = (-extent / 2 + (c % cells_per_side + 0.5) * cell,
               -extent / 2 + (c // cells_per_side + 0.5) * cell)
        parts.append(aerial_scene(n_cell, cell, seed * 100 + c, sh_degree, feat_dim,
                                  n_boxes=boxes, per_box=per_box, centre=cxy))
    offs = np.zeros(cells + 1, dtype=np.int64)
    offs[1:] = np.cumsum([p.n for p in parts])
    cat = lambda f: np.ascontiguousarray(np.concatenate([getattr(p, f) for p in parts]))
    return Scene(cat("means"), cat("log_scales"), cat("quats"), cat("opacities"), cat("sh"),
                 sh_degree, cat("feat") if feat_dim else None, part_offsets=offs)


# --------------------------------------------------------------------------
# cameras and poses
# --------------------------------------------------------------------------
def down_pose(centre_xy, altitude, tilt_rotvec_xy=(0.0, 0.0), yaw=0.0) -> np.ndarray:
    """World->camera [R|t] (12 float32) of a camera `altitude` metres above the
    terrain at centre_xy, looking straight down (camera z = -world Z), then
    yawed about world Z and tilted by a rotation vector in the world xy plane."""
    cx, cy = centre_xy
    C = np.array([cx, cy, float(_terrain_height(cx, cy)) + altitude])
    r_down = np.diag([1.0, -1.0, -1.0])                      # camera -> world, nadir
    r_tilt = Rotation.from_rotvec([tilt_rotvec_xy[0], tilt_rotvec_xy[1], 0.0]).as_matrix()
    r_yaw = Rotation.from_rotvec([0.0, 0.0, yaw]).as_matrix()
    r_cw = r_yaw @ r_tilt @ r_down
    R = r_cw.T
    t = -R @ C
    return np.concatenate([R, t[:, None]], axis=1).reshape(12).astype(np.float32)


def perturb_poses(pose, count, seed, sigma_t, sigma_rot_deg) -> np.ndarray:
    """`count` poses T' = Exp-free perturbation of a seed pose: camera centre
    moved by N(0, sigma_t) metres per axis and orientation rotated by a
    rotation vector ~ N(0, sigma_rot) per axis (applied in the world frame)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    P = np.asarray(pose, dtype=np.float64).reshape(3, 4)
    R, t = P[:, :3], P[:, 3]
    C = -R.T @ t
    out = np.empty((count, 12), dtype=np.float32)
    for k in range(count):
        dC = rng.normal(0.0, sigma_t, 3)
        dR = Rotation.from_rotvec(np.deg2rad(rng.normal(0.0, sigma_rot_deg, 3))).as_matrix()
        Rk = R @ dR.T
        Ck = C + dC
        out[k] = np.concatenate([Rk, (-Rk @ Ck)[:, None]], axis=1).reshape(12)
    return out


# --------------------------------------------------------------------------
# the workloads of the tests and the benchmark
# --------------------------------------------------------------------------
def terrain_20k_view(k=0):
    """20k Gaussians on a 200 m heightfield, SH0, no features, 256x192 view
    from 120 m with +/-10 deg tilt; 16 px tiles."""
    seed = 1000 + k
    scene = terrain_scene(20_000, 200.0, seed, sh_degree=0, feat_dim=0)
    rng = np.random.Generator(np.random.PCG64(seed + 500))
    tilt = np.deg2rad(rng.uniform(-10.0, 10.0, 2))
    pose = down_pose((0.0, 0.0), 120.0, tilt, rng.uniform(0, 2 * math.pi))
    cam = Camera(220.0, 220.0, 128.0, 96.0, 256, 192)
    return scene, pose[None], cam


def _aerial_pose(rng, max_tilt_deg, alt_lo=100.0, alt_hi=300.0, span=200.0):
    ang = math.radians(rng.uniform(0.0, max_tilt_deg))
    d = rng.uniform(0, 2 * math.pi)
    return down_pose((rng.uniform(-span, span), rng.uniform(-span, span)),
                     rng.uniform(alt_lo, alt_hi),
                     (ang * math.cos(d), ang * math.sin(d)), rng.uniform(0, 2 * math.pi))


_AERIAL_CACHE = {}


def aerial_1m_scene(k=0):
    key = ("aerial_1m", k)
    if key not in _AERIAL_CACHE:
        _AERIAL_CACHE.clear()
        _AERIAL_CACHE[key] = aerial_scene(1_000_000, 1000.0, 2000 + k, sh_degree=3, feat_dim=32)
    return _AERIAL_CACHE[key]


def aerial_1m_1080p(k=0):
    """1M Gaussians (900k terrain + 2000 buildings x 50), SH3, 32-d bf16
    features, 1920x1080 view, fx=1500, altitude U(100,300) m, tilt <= 30 deg."""
    scene = aerial_1m_scene(k)
    rng = np.random.Generator(np.random.PCG64(2000 + k + 500))
    pose = _aerial_pose(rng, 30.0)
    cam = Camera(1500.0, 1500.0, 960.0, 540.0, 1920, 1080)
    return scene, pose[None], cam


def aerial_1m_64_views(k=0, count=64, with_seed=False):
    """The config-2 scene seen by 64 poses perturbed from a seed pose by
    N(0,5 m) and N(0,3 deg), rendered at 960x540 with fx=750.  with_seed
    also returns the seed (query) pose."""
    scene = aerial_1m_scene(k)
    rng = np.random.Generator(np.random.PCG64(3000 + k))
    seed_pose = _aerial_pose(rng, 30.0)
    poses = perturb_poses(seed_pose, count, 3000 + k + 1, 5.0, 3.0)
    cam = Camera(750.0, 750.0, 480.0, 270.0, 960, 540)
    if with_seed:
        return scene, poses, cam, seed_pose
    return scene, poses, cam


def differentiable_200k(k=0):
    """200k Gaussians over 447x447 m (about 1/m^2), SH0 + 32-d features,
    640x480, fx=500, 120 m.  Returns (scene, true pose, start pose, camera):
    the start pose is the true pose offset by N(0,2 m) and N(0,2 deg)."""
    seed = 4000 + k
    scene = terrain_scene(200_000, 447.0, seed, sh_degree=0, feat_dim=32)
    rng = np.random.Generator(np.random.PCG64(seed + 500))
    tilt = np.deg2rad(rng.uniform(-10.0, 10.0, 2))
    truth = down_pose((0.0, 0.0), 120.0, tilt, rng.uniform(0, 2 * math.pi))
    start = perturb_poses(truth, 1, seed + 1, 2.0, 2.0)[0]
    cam = Camera(500.0, 500.0, 320.0, 240.0, 640, 480)
    return scene, truth[None], start[None], cam


def fd_subset_5k(k=0):
    """The finite-difference subset: 5k Gaussians over 80x80 m, 128x96,
    fx=220, 120 m; SH0 + 32-d features."""
    seed = 4100 + k
    scene = terrain_scene(5_000, 80.0, seed, sh_degree=0, feat_dim=32)
    rng = np.random.Generator(np.random.PCG64(seed + 500))
    tilt = np.deg2rad(rng.uniform(-10.0, 10.0, 2))
    pose = down_pose((0.0, 0.0), 120.0, tilt, rng.uniform(0, 2 * math.pi))
    cam = Camera(220.0, 220.0, 64.0, 48.0, 128, 96)
    return scene, pose[None], cam


def partitioned_8m(k=0, n_total=8_000_000, queries=16):
    """8M Gaussians over 4x4 km in 16 spatial partitions (buildings pro rata),
    16 query poses; levels 480x270 / 960x540 / 1920x1080 with fx 375/750/1500.
    Returns (scene, true poses, start poses, cameras)."""
    seed = 5000 + k
    scene = partitioned_scene(n_total, 4000.0, seed, cells_per_side=4, sh_degree=0, feat_dim=32)
    rng = np.random.Generator(np.random.PCG64(seed + 500))
    truth = np.stack([_aerial_pose(rng, 30.0, span=1600.0) for _ in range(queries)])
    start = np.stack([perturb_poses(truth[q], 1, seed + 10 + q, 5.0, 3.0)[0] for q in range(queries)])
    cams = [Camera(375.0, 375.0, 240.0, 135.0, 480, 270),
            Camera(750.0, 750.0, 480.0, 270.0, 960, 540),
            Camera(1500.0, 1500.0, 960.0, 540.0, 1920, 1080)]
    return scene, truth, start, cams


def tiny_scene(n, seed, width=64, height=48, sh_degree=0, feat_dim=0, extent=None, altitude=40.0,
               fx=None):
    """A small random scene and a nadir-ish view of it for exhaustive checks.
    The scene spans the camera footprint plus a margin so that Gaussians cross
    the image border."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fx = fx if fx is not None else 0.9 * width
    if extent is None:
        extent = 1.2 * width / fx * altitude
    x = rng.uniform(-extent / 2, extent / 2, n)
    y = rng.uniform(-extent / 2, extent / 2, n)
    z = rng.normal(0.0, 2.0, n)
    means = np.stack([x, y, z], axis=1).astype(np.float32)
    log_scales = (rng.normal(-0.5, 0.3, (n, 3)) + math.log(altitude / 120.0 * 8)).astype(np.float32)
    quats = _unit_quats(rng, n)
    opac = _sigmoid_opacity(rng, n)
    sh = _sh(rng, n, sh_degree)
    feat = _features(rng, n, feat_dim) if feat_dim else None
    scene = Scene(means, log_scales, quats, opac, sh, sh_degree, feat)
    tilt = np.deg2rad(rng.uniform(-10.0, 10.0, 2))
    pose = down_pose((0.0, 0.0), altitude, tilt, rng.uniform(0, 2 * math.pi))
    # down_pose measures altitude above the heightfield; re-centre on z = 0
    P = pose.reshape(3, 4).astype(np.float64)
    C = np.array([0.0, 0.0, altitude])
    P[:, 3] = -P[:, :3] @ C
    cam = Camera(float(fx), float(fx), width / 2.0, height / 2.0, width, height)
    return scene, P.reshape(12).astype(np.float32)[None], cam


def feature_maps(count, dim, height, width, seed, layout="planar") -> np.ndarray:
    """`count` 2D feature maps of `dim` channels (the training views' image
    features that Gaussians are scored against): N(0, 1) float32, planar
    (count, dim, height, width) or interleaved (count, height, width, dim)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    m = rng.standard_normal((count, dim, height, width), dtype=np.float32)
    if layout == "interleaved":
        m = np.ascontiguousarray(m.transpose(0, 2, 3, 1))
    return m


def matching_maps(dim, coarse_h, coarse_w, seed, shift=(3, 5), noise=0.3):
    """Query and rendered feature maps for coarse-to-fine matching, as bf16
    bits: fine maps (dim, 8 coarse_h, 8 coarse_w) of N(0, 1) features, the
    rendered one the query's moved by `shift` = (dx, dy) fine pixels plus
    N(0, noise) (fresh features where it moves in from outside), and coarse
    maps that are the fine maps' 8 x 8 means.  Returns (q_coarse, r_coarse,
    q_fine, r_fine)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    Hf, Wf = 8 * coarse_h, 8 * coarse_w
    q = rng.standard_normal((dim, Hf, Wf), dtype=np.float32)
    r = rng.standard_normal((dim, Hf, Wf), dtype=np.float32)
    dx, dy = shift
    ys = slice(max(dy, 0), Hf + min(dy, 0))
    xs = slice(max(dx, 0), Wf + min(dx, 0))
    ys_src = slice(max(-dy, 0), Hf + min(-dy, 0))
    xs_src = slice(max(-dx, 0), Wf + min(-dx, 0))
    r[:, ys, xs] = q[:, ys_src, xs_src] + noise * rng.standard_normal(q[:, ys_src, xs_src].shape, dtype=np.float32)
    pool = lambda f: f.reshape(dim, coarse_h, 8, coarse_w, 8).mean(axis=(2, 4))
    return (f32_to_bf16_bits(pool(q)), f32_to_bf16_bits(pool(r)), f32_to_bf16_bits(q), f32_to_bf16_bits(r))
