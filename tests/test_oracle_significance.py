"""Pins of the oracle's significance scoring (Sec. 3.2, Eq. 4-6) and of its
render visibility check, against closed forms, the oracle's brute-force
renderer, finite differences of the rendered image and the renderer's own
projection.  CPU only."""
import math

import numpy as np

import synth
from synth import Camera, Scene
from oracle import significance as sg

Y00 = 1.0 / (2.0 * math.sqrt(math.pi))


def _scene(means, sigmas, opac, feat):
    n = len(means)
    sh = np.zeros((n, 1, 3), dtype=np.float32)
    sh[:, 0, :] = (0.6 - 0.5) / Y00
    ls = np.log(np.repeat(np.asarray(sigmas, np.float64)[:, None], 3, 1))
    q = np.tile([1.0, 0.0, 0.0, 0.0], (n, 1))
    return Scene(np.asarray(means, np.float32), ls.astype(np.float32), q.astype(np.float32),
                 np.asarray(opac, np.float32), sh, 0, synth.f32_to_bf16_bits(np.asarray(feat, np.float32)))


def _pose(t):
    return np.array([1, 0, 0, t[0], 0, 1, 0, t[1], 0, 0, 1, t[2]], dtype=np.float64)


def test_closed_form_views(oracle_lib):
    """Hand-built scene with known visibility and cosines over three views:
    A is visible in all three with cosines 1, -1 and 1/2 (S = 1/6, M = 3);
    B sits behind four nearly opaque occluders (never blended); C is below the 1/255
    gate; D's mean projects left of the image in views 0 and 2 though its
    footprint reaches into it (blended, not visible) and inside in view 1; E is
    behind the camera; F projects inside in views 0 and 2 only."""
    cam = Camera(100.0, 100.0, 32.0, 24.0, 64, 48)
    D = 8
    rng = np.random.default_rng(5)
    feat = rng.normal(0, 1, (10, D))
    # distinct depths everywhere (equal depths of two overlapping Gaussians
    # are order near-ties, which make pixels fragile)
    means = [[-0.93, 0.31, 10.0],        # A: U = 22.7, V = 27.1
             [0.5, -0.5, 20.0],          # B: U = 34.5, V = 21.5
             [-0.5, 0.5, 10.2],          # C
             [-3.4125, 0.1, 10.5],       # D: U = -0.5, V = 24.95
             [0.0, 0.0, -5.0],           # E
             [2.9925, 0.095, 9.5],       # F: U = 63.5, V = 25
             [0.275, -0.275, 11.0], [0.3125, -0.3125, 12.5], [0.35, -0.35, 14.0], [0.4, -0.4, 16.0]]  # on B's ray
    sig = [0.05, 0.1, 0.05, 0.2, 0.05, 0.05, 2.0, 2.0, 2.0, 2.0]
    opa = [0.8, 0.5, 0.003, 0.8, 0.8, 0.8, 0.97, 0.97, 0.97, 0.97]
    sc = _scene(means, sig, opa, feat)
    poses = np.stack([_pose((0, 0, 0)), _pose((0.2, 0, 0)), _pose((0, 0.3, 0))])
    Hf, Wf = 12, 16                                  # 4x4-pixel cells
    maps = rng.normal(0, 1, (3, D, Hf, Wf)).astype(np.float32)
    fA = sg.bf16_to_f64(sc.feat[0])
    v = rng.normal(0, 1, D)
    v -= (v @ fA) / (fA @ fA) * fA
    v *= math.sqrt(3.0) * np.linalg.norm(fA) / np.linalg.norm(v)
    maps[0][:, 6, 5] = fA                            # view 0: U 22.7, V 27.1 -> cell (5, 6): cos 1
    maps[1][:, 6, 6] = -fA                           # view 1: U 24.7 -> cell (6, 6): cos -1
    maps[2][:, 7, 5] = fA + v                        # view 2: V 30.1 -> cell (5, 7): cos 1/2
    r = sg.significance(sc, poses, cam, maps)
    assert r["count"][0] == 3
    assert abs(r["score_sum"][0] - 0.5) < 1e-6 and abs(r["score"][0] - 0.5 / 3) < 1e-6
    assert r["count"][1] == 0 and r["count"][2] == 0 and r["count"][4] == 0
    assert list(r["visible"][:, 3]) == [False, True, False]
    assert list(r["visible"][:, 5]) == [True, False, True]
    # D is blended (it contributes) although its mean is outside the image
    c, _, _ = oracle_lib.contrib(sc, poses[0], cam)
    assert c[3] and not c[1] and not c[2] and not c[4]
    # F's two cosines, straight from the cells it falls in: view 0 (U 63.5,
    # V 25) -> cell (15, 6); view 2 (V 25 + 30/9.5 = 28.16) -> cell (15, 7)
    fF = sg.bf16_to_f64(sc.feat[5])
    want = 0.0
    for i, cy in ((0, 6), (2, 7)):
        ft = maps[i][:, cy, 15].astype(np.float64)
        want += fF @ ft / (np.linalg.norm(fF) * np.linalg.norm(ft) + 1e-8)
    assert abs(r["score_sum"][5] - want) < 1e-12
    assert r["count"][5] == 2 and abs(r["score"][5] - want / 2) < 1e-12   # Eq. 6 divides by M, not by the views
    assert not r["exempt"][:, :6].any()


def test_visibility_is_the_support_of_the_rgb_gradient(oracle_lib):
    """The render-mask algorithm marks a Gaussian visible when the summed RGB
    has a nonzero gradient with respect to its mean.  Moving a mean by 1e-6 m
    changes the oracle's rendered image exactly when the Gaussian is blended
    somewhere (opacities kept below the 0.99 clamp, where a blended Gaussian
    has a zero alpha gradient)."""
    checked = 0
    for seed in range(6):
        sc, P, cam = synth.tiny_scene(40 + 10 * seed, 40 + seed, feat_dim=4)
        sc.opacities[:] = np.minimum(sc.opacities, 0.9)
        c, robust, touched = oracle_lib.contrib(sc, P[0], cam)
        base = oracle_lib.render(sc, P[0], cam)["rgb"].sum()
        for j in range(sc.n):
            if touched[j] and not robust[j]:
                continue
            moved = False
            for k in range(3):
                m64 = sc.means.astype(np.float64)
                m64[j, k] += 1e-6
                moved |= oracle_lib.render(sc, P[0], cam, overrides={"means": m64})["rgb"].sum() != base
            assert moved == bool(c[j]), (seed, j)
            checked += 1
    assert checked > 200



def test_projection_is_the_renderers_pinhole(oracle_lib):
    """The algorithm's projection (homogeneous point, pose, perspective
    division, K) agrees with the renderer's projected means and depths."""
    for seed in range(4):
        sc, P, cam = synth.tiny_scene(150, 70 + seed)
        U, V, d = sg.project_means(sc.means, P[0], cam)
        p = oracle_lib.project(sc, P[0], cam)
        front = d > 0.2
        np.testing.assert_allclose(U[front], p["u"][front], rtol=1e-12, atol=1e-9)
        np.testing.assert_allclose(V[front], p["v"][front], rtol=1e-12, atol=1e-9)
        np.testing.assert_allclose(d, p["z"], rtol=1e-12, atol=1e-12)


def test_contrib_is_the_union_of_brute_force_blend_lists(oracle_lib):
    """A Gaussian contributes exactly when the brute-force renderer (one
    global depth sort, every Gaussian at every pixel) blends it at some pixel;
    robust contributions are contributions."""
    for seed in range(8):
        sc, P, cam = synth.tiny_scene(60 + 20 * seed, 90 + seed, feat_dim=4 if seed % 2 else 0)
        r = oracle_lib.render(sc, P[0], cam, mode="brute", want_lists=True, list_cap=256)
        lists = r["lists"]
        want = np.zeros(sc.n, dtype=bool)
        want[lists[lists >= 0]] = True
        for tile in (8, 16):
            c, robust, touched = oracle_lib.contrib(sc, P[0], cam, tile=tile)
            assert np.array_equal(c, want), (seed, tile)
            assert not (robust & ~c).any()
            # a pixel's walk reaches every Gaussian it blends
            frag = r["fragile"].reshape(-1)
            on_frag = np.zeros(sc.n, dtype=bool)
            fl = lists[frag]
            on_frag[fl[fl >= 0]] = True
            assert not (on_frag & ~touched).any()


def test_cell_rule_on_a_non_integer_grid():
    """(U, V) reads the cell that contains it: with W = 64 and Wf = 10 (6.4 px
    per cell) and H = 48, Hf = 5 (9.6 px), points at known positions read the
    cells k with 6.4 k <= U < 6.4 (k + 1); the image's right and bottom
    borders are excluded.  One-hot maps identify the cell read."""
    W, H, Wf, Hf = 64, 48, 10, 5
    Dm = Wf * Hf
    fmap = np.zeros((Dm, Hf, Wf))
    for cy in range(Hf):
        for cx in range(Wf):
            fmap[cy * Wf + cx, cy, cx] = 1.0
    feat = np.arange(1, Dm + 1, dtype=np.float64)[None, :].repeat(9, 0)
    U = np.array([0.0, 6.39, 6.41, 12.9, 63.99, 64.0, -0.01, 30.0, 30.0])
    V = np.array([0.0, 9.59, 9.61, 19.3, 47.99, 10.0, 10.0, 48.0, 47.5])
    cos, inside, near = sg.sample_cosines(feat, U, V, fmap, W, H, edge_px=1e-3)
    assert list(inside) == [True, True, True, True, True, False, False, False, True]
    norm = np.linalg.norm(feat[0])
    got = np.rint(cos[inside] * norm).astype(int) - 1          # the one-hot channel read
    want = []
    for u, v in zip(U[inside], V[inside]):
        cx = int(np.floor(u / 6.4)); cy = int(np.floor(v / 9.6))
        want.append(cy * Wf + cx)
    assert list(got) == want
    assert near[0] and near[5] and near[7]                     # on the border
    assert not near[1] and not near[3]
    # near a cell border from either side: 5e-4 px below the border at
    # U = 19.2 is near, 5e-3 px below it is not (the default tolerance,
    # 1e-3 px); the same on the upper side of the border at V = 19.2
    U2 = np.array([19.1995, 19.195, 30.0, 30.0])
    V2 = np.array([14.4, 14.4, 19.2005, 19.205])
    _, _, near2 = sg.sample_cosines(feat[:4], U2, V2, fmap, W, H)
    assert list(near2) == [True, False, True, False]


def test_significance_invariances(oracle_lib):
    """Permuting the Gaussians permutes every output; reordering the views
    leaves the sums unchanged up to rounding and the counts exactly."""
    sc, P, cam = synth.tiny_scene(300, 123, feat_dim=8)
    poses = synth.perturb_poses(P[0].reshape(12), 3, 5, 0.5, 2.0)
    maps = np.random.default_rng(3).normal(0, 1, (3, 8, cam.height // 2, cam.width // 2))
    r = sg.significance(sc, poses, cam, maps)
    assert r["count"].max() >= 1 and (r["count"] > 0).sum() > 30
    perm = np.random.default_rng(4).permutation(sc.n)
    rp = sg.significance(sc.subset(perm), poses, cam, maps)
    for k in ("score_sum", "count", "score"):
        assert np.array_equal(rp[k], r[k][perm]), k
    rv = sg.significance(sc, poses[::-1], cam, maps[::-1])
    assert np.array_equal(rv["count"], r["count"])
    np.testing.assert_allclose(rv["score_sum"], r["score_sum"], rtol=0, atol=1e-12)


def test_contrib_flags_follow_the_blended_lists(oracle_lib):
    """contrib marks the Gaussians blended at some pixel, robust those blended
    at some pixel that is not fragile: recomputed here from the render's own
    per-pixel blended lists and fragile map."""
    for seed in (3, 8):
        sc, P, cam = synth.tiny_scene(150, seed)
        r = oracle_lib.render(sc, P[0], cam, want_lists=True)
        c, robust, _ = oracle_lib.contrib(sc, P[0], cam)
        want_c = np.zeros(sc.n, bool)
        want_r = np.zeros(sc.n, bool)
        nb = r["nblend"].reshape(-1)
        frag = r["fragile"].reshape(-1)
        for pix in np.nonzero(nb)[0]:
            ids = r["lists"][pix, :nb[pix]]
            want_c[ids] = True
            if not frag[pix]:
                want_r[ids] = True
        assert want_r.any() and (want_c & ~want_r).sum() < want_c.sum()
        assert np.array_equal(c.astype(bool), want_c)
        assert np.array_equal(robust.astype(bool), want_r)


def test_fragile_only_visibility_is_exempt(oracle_lib):
    """A pair whose visibility rests only on fragile pixels is exempt: a
    Gaussian of opacity float32(1/255) centred on a pixel centre is blended
    at that pixel alone, where its alpha is within the FP32 error of the
    gate.  Its mean is inside the image, away from cell borders."""
    cam = Camera(100.0, 100.0, 32.5, 24.5, 64, 48)
    rng = np.random.default_rng(3)
    sc = _scene([[0.0, 0.0, 10.0], [0.5, 0.3, 12.0]], [1.0, 0.3], [1 / 255, 0.8], rng.normal(0, 1, (2, 8)))
    maps = rng.normal(0, 1, (1, 8, 12, 16)).astype(np.float32)
    c, robust, touched = oracle_lib.contrib(sc, _pose((0, 0, 0)), cam)
    assert c[0] and not robust[0] and touched[0]
    r = sg.significance(sc, _pose((0, 0, 0))[None], cam, maps)
    assert r["visible"][0, 0] and r["exempt"][0, 0]
    assert r["visible"][0, 1] and not r["exempt"][0, 1]
