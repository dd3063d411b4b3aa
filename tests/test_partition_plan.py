"""Host side of partition streaming (CPU): the partition boxes and the
per-pose plan of which partitions a batch may see, against the oracle's
per-Gaussian projection; argument checks of the cache."""
import math

import numpy as np
import pytest

import synth

CAM = synth.Camera(220.0, 220.0, 128.0, 96.0, 256, 192)


@pytest.fixture(scope="module")
def hg():
    import paper_2507_15683_amd as hg
    return hg


@pytest.fixture(scope="module")
def scene():
    return synth.partitioned_scene(48_000, 800.0, 7, cells_per_side=4, sh_degree=0, feat_dim=0,
                                   boxes_per_km2=300, per_box=50)


def _poses(count, seed, span=400.0):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        ang, d = math.radians(rng.uniform(0, 35)), rng.uniform(0, 2 * math.pi)
        out.append(synth.down_pose((rng.uniform(-span, span), rng.uniform(-span, span)), rng.uniform(40, 260),
                                   (ang * math.cos(d), ang * math.sin(d)), rng.uniform(0, 2 * math.pi)))
    return np.stack(out)


def test_boxes_contain_every_support_ball(hg, scene):
    """Each box is the smallest float box around the balls of radius
    3.33 exp(max log-scale): it contains them all and touches them to within
    float rounding on every side."""
    b = hg.host_partition_bounds(scene)
    offs = scene.part_offsets
    for k in range(len(offs) - 1):
        sl = slice(offs[k], offs[k + 1])
        m = scene.means[sl].astype(np.float64)
        r = 3.33 * np.exp(scene.log_scales[sl].astype(np.float64).max(axis=1))
        lo, hi = (m - r[:, None]).min(axis=0), (m + r[:, None]).max(axis=0)
        assert (b[k, :3] <= lo).all() and (b[k, 3:] >= hi).all()
        np.testing.assert_allclose(b[k, :3], lo, rtol=0, atol=1e-4 * (1 + np.abs(lo)).max())
        np.testing.assert_allclose(b[k, 3:], hi, rtol=0, atol=1e-4 * (1 + np.abs(hi)).max())


def test_plan_covers_every_visible_gaussian(hg, scene):
    """Every partition holding a Gaussian whose footprint the oracle's FP64
    projection puts on the image is planned, for poses all over the scene;
    and the plan is not trivially everything."""
    import oracle
    b = hg.host_partition_bounds(scene)
    poses = _poses(24, 3)
    plan = hg.partition_plan(b, poses, hg.Intrinsics.of(CAM))
    part_of = np.repeat(np.arange(len(scene.part_offsets) - 1), np.diff(scene.part_offsets))
    skipped = 0
    for p in range(len(poses)):
        vis = oracle.project(scene, poses[p], CAM)["visible"].astype(bool)
        need = np.unique(part_of[vis])
        assert plan[p, need].all(), (p, need, np.nonzero(plan[p])[0])
        skipped += int((plan[p] == 0).sum())
    assert skipped > 0.5 * plan.size  # a 256x192 view from <= 260 m sees a few of the 16 cells


def test_margin_grows_the_plan_and_backward_views_see_nothing(hg, scene):
    b = hg.host_partition_bounds(scene)
    poses = _poses(16, 4)
    K = hg.Intrinsics.of(CAM)
    p0 = hg.partition_plan(b, poses, K)
    p1 = hg.partition_plan(b, poses, K, motion_margin=60.0)
    assert (p1 >= p0).all() and p1.sum() > p0.sum()
    # a camera above the scene looking up: every box is behind it
    up = synth.down_pose((0.0, 0.0), 300.0).reshape(3, 4).astype(np.float64)
    flip = np.diag([1.0, -1.0, -1.0])
    T = np.concatenate([flip @ up[:, :3], (flip @ up[:, 3])[:, None]], axis=1).reshape(12).astype(np.float32)
    assert hg.partition_plan(b, T[None], K).sum() == 0


def test_empty_partition_is_never_planned(hg, scene):
    """A partition with no Gaussians gets an empty box (min > max), which no
    pose sees."""
    s = synth.Scene(scene.means, scene.log_scales, scene.quats, scene.opacities, scene.sh, 0, None,
                    part_offsets=np.concatenate([[0], scene.part_offsets]).astype(np.int64))
    b = hg.host_partition_bounds(s)
    assert (b[0, :3] > b[0, 3:]).all()
    plan = hg.partition_plan(b, _poses(8, 5), hg.Intrinsics.of(CAM))
    assert plan[:, 0].sum() == 0


def test_cache_arguments_rejected_on_host(hg, scene):
    """Bad partition tables and slot counts fail before anything touches a
    device."""
    import ctypes
    from paper_2507_15683_amd import _lib
    lib = _lib.load()
    hs, keep = hg._host_scene(scene)
    h = ctypes.c_void_p()
    for slots in (0, 17, 65):
        assert lib.hgsr_pcache_create(ctypes.byref(h), ctypes.byref(hs), slots) == 1
    bad = np.array(scene.part_offsets, dtype=np.int64)
    bad[3], bad[4] = bad[4], bad[3]
    s2 = synth.Scene(scene.means, scene.log_scales, scene.quats, scene.opacities, scene.sh, 0, None,
                     part_offsets=bad)
    hs2, keep2 = hg._host_scene(s2)
    assert lib.hgsr_pcache_create(ctypes.byref(h), ctypes.byref(hs2), 4) == 1
    assert b"decrease" in lib.hgsr_last_error()
    b = hg.host_partition_bounds(scene)
    K = hg.Intrinsics.of(CAM)
    with pytest.raises(hg.HgsrError):
        hg.partition_plan(b, np.full(12, np.nan, dtype=np.float32), K)
    with pytest.raises(hg.HgsrError):
        hg.partition_plan(b, _poses(1, 6), K, motion_margin=-1.0)
