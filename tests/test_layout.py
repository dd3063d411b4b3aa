"""Spatial (Morton) order of a scene, computed on the host (CPU)."""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def hg():
    import paper_2507_15683_amd as hg
    return hg


def test_cube_corners_follow_the_bit_interleave(hg):
    """The 8 corners of a cube, shuffled: Morton order puts corner
    (x, y, z) in {0, 1}^3 at position x + 2y + 4z."""
    corners = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], dtype=np.float32)
    shuf = np.random.default_rng(0).permutation(8)
    perm = hg.spatial_order(corners[shuf])
    got = corners[shuf][perm]
    np.testing.assert_array_equal(got, corners)


def test_permutation_within_partitions_and_local(hg):
    sc = synth.partitioned_scene(48_000, 800.0, 7, cells_per_side=4, sh_degree=0, feat_dim=0,
                                 boxes_per_km2=300, per_box=50)
    perm = hg.spatial_order(sc.means, sc.part_offsets)
    assert np.array_equal(np.sort(perm), np.arange(sc.n))
    offs = sc.part_offsets
    for k in range(len(offs) - 1):
        seg = perm[offs[k]:offs[k + 1]]
        assert seg.min() >= offs[k] and seg.max() < offs[k + 1]
    # consecutive Gaussians are neighbours: far shorter steps than in the given order
    step = lambda m: np.linalg.norm(np.diff(m.astype(np.float64), axis=0), axis=1).mean()
    assert step(sc.means[perm]) < 0.1 * step(sc.means)


def test_ties_and_bad_arguments(hg):
    m = np.zeros((5, 3), dtype=np.float32)       # all equal: index order
    assert list(hg.spatial_order(m)) == [0, 1, 2, 3, 4]
    with pytest.raises(hg.HgsrError):
        hg.spatial_order(m, np.array([0, 3, 2, 5], dtype=np.int64))


def test_spatial_layout_permutes_every_array_together(hg):
    sc = synth.tiny_scene(300, 5, feat_dim=8, sh_degree=1)[0]
    out, perm = hg.spatial_layout(sc)
    for f in ("means", "log_scales", "quats", "opacities", "sh", "feat"):
        np.testing.assert_array_equal(getattr(out, f), getattr(sc, f)[perm])
    assert out.sh_degree == sc.sh_degree
