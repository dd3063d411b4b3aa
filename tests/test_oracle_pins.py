"""Pins of the FP64 oracle against closed forms, library routines, brute force
and invariants -- chosen so that a dropped term, a wrong sign or index, or a
transposed operand in the oracle fails at least one of them.  CPU only."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from synth import Camera, Scene

Y00 = 1.0 / (2.0 * math.sqrt(math.pi))  # textbook real SH, l = 0


def _one(means, log_scales, quats, opac, rgb, feat=None, sh_degree=0):
    n = len(means)
    K = (sh_degree + 1) ** 2
    sh = np.zeros((n, K, 3), dtype=np.float32)
    sh[:, 0, :] = (np.asarray(rgb, dtype=np.float64) - 0.5) / Y00
    return Scene(np.asarray(means, np.float32).reshape(n, 3), np.asarray(log_scales, np.float32).reshape(n, 3),
                 np.asarray(quats, np.float32).reshape(n, 4), np.asarray(opac, np.float32).reshape(n),
                 sh, sh_degree, None if feat is None else synth.f32_to_bf16_bits(np.asarray(feat, np.float32)))


IDENT = np.array([1, 0, 0, 0, 0, 1, 0, 0, 0, 0, 1, 0], dtype=np.float32)


def _closed_alpha(cam, o, s2, u=None, v=None):
    u = cam.cx if u is None else u
    v = cam.cy if v is None else v
    jj, ii = np.mgrid[0:cam.height, 0:cam.width]
    d2 = (ii + 0.5 - u) ** 2 + (jj + 0.5 - v) ** 2
    a = np.minimum(0.99, o * np.exp(-d2 / (2 * s2)))
    return np.where(a >= 1 / 255, a, 0.0)


# ------------------------------------------------------------------ projection
def test_isotropic_closed_form(oracle_lib):
    """One camera-facing isotropic Gaussian on the optical axis:
    s^2 = (f sigma / z)^2 + 0.3 and alpha = min(0.99, o exp(-d^2 / 2 s^2))."""
    cam = Camera(100.0, 100.0, 32.0, 24.0, 64, 48)
    sigma, z, o = 0.5, 10.0, 0.8
    c = np.array([0.2, 0.6, 0.9])
    f = np.linspace(-1, 1, 8).astype(np.float32) / 2
    q = Rotation.random(random_state=3).as_quat()  # any rotation of an isotropic Gaussian
    sc = _one([[0, 0, z]], [[math.log(sigma)] * 3], [[q[3], q[0], q[1], q[2]]], [o], [c], feat=[f])
    sigma, o = math.exp(float(sc.log_scales[0, 0])), float(sc.opacities[0])  # the stored float32 values
    c = sc.sh[0, 0].astype(np.float64) * Y00 + 0.5
    r = oracle_lib.render(sc, IDENT, cam)
    s2 = (cam.fx * sigma / z) ** 2 + 0.3
    a = _closed_alpha(cam, o, s2)
    np.testing.assert_allclose(r["alpha"], a, rtol=0, atol=1e-12)
    np.testing.assert_allclose(r["rgb"], c[:, None, None] * a[None], atol=1e-12)
    np.testing.assert_allclose(r["depth"], np.where(a > 0, z, 0.0), atol=1e-12)
    fb = synth.bf16_bits_to_f32(synth.f32_to_bf16_bits(f)).astype(np.float64)
    np.testing.assert_allclose(r["feat"], fb[:, None, None] * a[None], atol=1e-12)
    p = oracle_lib.project(sc, IDENT, cam)
    np.testing.assert_allclose([p["cov_xx"][0], p["cov_xy"][0], p["cov_yy"][0]], [s2, 0, s2], rtol=1e-12, atol=1e-12)


def test_anisotropic_axis_and_quaternion_order(oracle_lib):
    """A 90-degree turn about z swaps the x and y variances (w,x,y,z order);
    the world covariance equals scipy's rotation of diag(s^2)."""
    cam = Camera(100.0, 120.0, 32.0, 24.0, 64, 48)
    s = np.array([0.3, 0.7, 1.1])
    z = 10.0
    h = math.sqrt(0.5)
    sc = _one([[0, 0, z], [0, 0, z]], [np.log(s)] * 2, [[h, 0, 0, h], [h, h, 0, 0]], [0.5, 0.5], [[0.5] * 3] * 2)
    p = oracle_lib.project(sc, IDENT, cam)
    np.testing.assert_allclose([p["cov_xx"][0], p["cov_yy"][0], p["cov_xy"][0]],
                               [(cam.fx / z) ** 2 * s[1] ** 2 + 0.3, (cam.fy / z) ** 2 * s[0] ** 2 + 0.3, 0.0],
                               rtol=1e-6, atol=1e-9)
    np.testing.assert_allclose([p["cov_xx"][1], p["cov_yy"][1]],
                               [(cam.fx / z) ** 2 * s[0] ** 2 + 0.3, (cam.fy / z) ** 2 * s[2] ** 2 + 0.3], rtol=1e-6)
    rng = np.random.default_rng(0)
    n = 50
    q = rng.standard_normal((n, 4))
    ls = rng.normal(-0.5, 0.3, (n, 3))
    sc = _one(rng.normal(0, 1, (n, 3)) + [0, 0, 10], ls, q, np.full(n, 0.5), np.full((n, 3), 0.5))
    p = oracle_lib.project(sc, IDENT, cam)
    qf = sc.quats.astype(np.float64)
    Rm = Rotation.from_quat(np.concatenate([qf[:, 1:], qf[:, :1]], axis=1)).as_matrix()
    S2 = np.exp(2 * sc.log_scales.astype(np.float64))
    Sw = np.einsum("nij,nj,nkj->nik", Rm, S2, Rm)
    got = np.stack([p["cov3_xx"], p["cov3_xy"], p["cov3_xz"], p["cov3_yy"], p["cov3_yz"], p["cov3_zz"]], 1)
    want = np.stack([Sw[:, 0, 0], Sw[:, 0, 1], Sw[:, 0, 2], Sw[:, 1, 1], Sw[:, 1, 2], Sw[:, 2, 2]], 1)
    np.testing.assert_allclose(got, want, rtol=1e-10, atol=1e-12)


def _rand_pose(seed):
    rng = np.random.default_rng(seed)
    R = Rotation.random(random_state=seed).as_matrix()
    C = rng.normal(0, 3, 3)
    t = -R @ C
    return np.concatenate([R, t[:, None]], 1).reshape(12)


def test_projection_matches_pinhole_and_ewa_jacobian(oracle_lib):
    """u, v = K (X/Z) (the pinhole map of Algorithm 1); Sigma' - 0.3 I equals
    J Sigma_c J^T with J the numerical Jacobian of that map (unclamped case)."""
    cam = Camera(150.0, 140.0, 40.0, 30.0, 80, 60)
    rng = np.random.default_rng(1)
    pose = _rand_pose(7)
    R, t = pose.reshape(3, 4)[:, :3], pose.reshape(3, 4)[:, 3]
    n = 40
    # place Gaussians in front of the camera inside the view
    dirs = np.stack([rng.uniform(-0.2, 0.2, n), rng.uniform(-0.15, 0.15, n), np.ones(n)], 1)
    depth = rng.uniform(5, 20, n)
    mc = dirs * depth[:, None]
    mw = (mc - t) @ R  # R^T (mc - t)
    sc = _one(mw, rng.normal(-1, 0.3, (n, 3)), rng.standard_normal((n, 4)), np.full(n, 0.7), np.full((n, 3), 0.5))
    mw = sc.means.astype(np.float64)
    p = oracle_lib.project(sc, pose, cam)
    mc = mw @ R.T + t
    K = np.array([[cam.fx, 0, cam.cx], [0, cam.fy, cam.cy], [0, 0, 1]])
    uvw = (K @ (mc / mc[:, 2:3]).T).T
    np.testing.assert_allclose(p["u"], uvw[:, 0], rtol=1e-12)
    np.testing.assert_allclose(p["v"], uvw[:, 1], rtol=1e-12)
    np.testing.assert_allclose(p["z"], mc[:, 2], rtol=1e-12)

    def pix(x):
        return np.array([cam.fx * x[0] / x[2] + cam.cx, cam.fy * x[1] / x[2] + cam.cy])

    for i in range(n):
        Sw = np.array([[p["cov3_xx"][i], p["cov3_xy"][i], p["cov3_xz"][i]],
                       [p["cov3_xy"][i], p["cov3_yy"][i], p["cov3_yz"][i]],
                       [p["cov3_xz"][i], p["cov3_yz"][i], p["cov3_zz"][i]]])
        Sc = R @ Sw @ R.T
        h = 1e-5 * mc[i, 2]
        J = np.stack([(pix(mc[i] + h * e) - pix(mc[i] - h * e)) / (2 * h) for e in np.eye(3)], 1)
        S2 = J @ Sc @ J.T
        got = np.array([[p["cov_xx"][i] - 0.3, p["cov_xy"][i]], [p["cov_xy"][i], p["cov_yy"][i] - 0.3]])
        np.testing.assert_allclose(got, S2, rtol=1e-6, atol=1e-9 * np.abs(S2).max())
        conic = np.linalg.inv(S2 + 0.3 * np.eye(2))
        np.testing.assert_allclose([p["conic_a"][i], p["conic_b"][i], p["conic_c"][i]],
                                   [conic[0, 0], conic[0, 1], conic[1, 1]], rtol=1e-6,
                                   atol=1e-8 * np.abs(conic).max())


@pytest.mark.parametrize("axis", [0, 1])
def test_guard_clamp_freezes_jacobian(oracle_lib, axis):
    """Inside 1.3x the half field of view Sigma' is the EWA form with the
    pinhole Jacobian; beyond it the Jacobian is evaluated at the clamp, so
    moving the Gaussian further out leaves Sigma' unchanged while the projected
    mean keeps moving."""
    cam = Camera(100.0, 110.0, 32.0, 24.0, 64, 48)
    z = 10.0
    tan = 32 / 100.0 if axis == 0 else 24 / 110.0
    ratios = [1.2, 1.3, 1.5, 3.0]
    pos = [[r * tan * z, 0.5, z] if axis == 0 else [0.5, r * tan * z, z] for r in ratios]
    sc = _one(pos, [[0.0, -0.5, 0.3]] * 4, [[0.9, 0.1, 0.3, 0.2]] * 4, [0.6] * 4, [[0.5] * 3] * 4)
    p = oracle_lib.project(sc, IDENT, cam)
    for k in ("cov_xx", "cov_xy", "cov_yy"):
        np.testing.assert_allclose(p[k][1:], p[k][1], rtol=1e-6)
    uv = p["u"] if axis == 0 else p["v"]
    assert uv[1] < uv[2] < uv[3]

    def pix(x):
        return np.array([cam.fx * x[0] / x[2] + cam.cx, cam.fy * x[1] / x[2] + cam.cy])

    for i in (0, 1):  # at and inside the guard band the Jacobian is the pinhole one
        m = sc.means[i].astype(np.float64)
        Sw = np.array([[p["cov3_xx"][i], p["cov3_xy"][i], p["cov3_xz"][i]],
                       [p["cov3_xy"][i], p["cov3_yy"][i], p["cov3_yz"][i]],
                       [p["cov3_xz"][i], p["cov3_yz"][i], p["cov3_zz"][i]]])
        h = 1e-6 * z
        J = np.stack([(pix(m + h * e) - pix(m - h * e)) / (2 * h) for e in np.eye(3)], 1)
        S2 = J @ Sw @ J.T
        np.testing.assert_allclose([p["cov_xx"][i] - 0.3, p["cov_xy"][i], p["cov_yy"][i] - 0.3],
                                   [S2[0, 0], S2[0, 1], S2[1, 1]], rtol=1e-5)


def test_alpha_clamped_at_099(oracle_lib):
    """alpha = min(0.99, o e^{-q/2}): an opaque Gaussian centred on a pixel
    centre gives exactly 0.99 there."""
    cam = Camera(100.0, 100.0, 32.5, 24.5, 64, 48)
    sc = _one([[0, 0, 10]], [[0.0] * 3], [[1, 0, 0, 0]], [1.0], [[1, 1, 1]])
    r = oracle_lib.render(sc, IDENT, cam)
    assert r["alpha"][24, 32] == 0.99
    assert r["alpha"].max() == 0.99


# ------------------------------------------------------------------ blending
def test_over_operator_two_gaussians(oracle_lib):
    """Two Gaussians on the axis: rgb = c1 a1 + c2 a2 (1 - a1), alpha =
    1 - (1-a1)(1-a2), depth = weighted mean of z; input order irrelevant."""
    cam = Camera(100.0, 100.0, 32.0, 24.0, 64, 48)
    z1, z2, s1, s2_, o1, o2 = 10.0, 14.0, 0.4, 0.9, 0.7, 0.6
    c1, c2 = np.array([1.0, 0.2, 0.1]), np.array([0.1, 0.3, 0.9])
    for order in ([0, 1], [1, 0]):
        means = np.array([[0, 0, z1], [0, 0, z2]])[order]
        sc = _one(means, np.log([[s1] * 3, [s2_] * 3])[order], [[1, 0, 0, 0]] * 2, np.array([o1, o2])[order],
                  np.array([c1, c2])[order])
        r = oracle_lib.render(sc, IDENT, cam)
        i1, i2 = order.index(0), order.index(1)
        f1, f2 = float(sc.opacities[i1]), float(sc.opacities[i2])
        g1, g2 = math.exp(float(sc.log_scales[i1, 0])), math.exp(float(sc.log_scales[i2, 0]))
        c1 = sc.sh[i1, 0].astype(np.float64) * Y00 + 0.5
        c2 = sc.sh[i2, 0].astype(np.float64) * Y00 + 0.5
        a1 = _closed_alpha(cam, f1, (cam.fx * g1 / z1) ** 2 + 0.3)
        a2 = _closed_alpha(cam, f2, (cam.fx * g2 / z2) ** 2 + 0.3)
        np.testing.assert_allclose(r["rgb"], c1[:, None, None] * a1 + c2[:, None, None] * a2 * (1 - a1), atol=1e-12)
        A = 1 - (1 - a1) * (1 - a2)
        np.testing.assert_allclose(r["alpha"], A, atol=1e-12)
        dep = np.divide(a1 * z1 + a2 * (1 - a1) * z2, A, out=np.zeros_like(A), where=A > 0)
        np.testing.assert_allclose(r["depth"], dep, rtol=1e-12, atol=1e-12)


def test_termination_stack(oracle_lib):
    """Five o=0.95 Gaussians centred on a pixel: T = 0.05, 0.0025, 1.25e-4,
    then 6.25e-6 < 1e-4 so the 4th is not blended; alpha = 0.999875."""
    cam = Camera(100.0, 100.0, 32.5, 24.5, 64, 48)
    cols = np.random.default_rng(2).uniform(0, 1, (5, 3))
    sc = _one([[0, 0, 10 + k] for k in range(5)], [[0.0] * 3] * 5, [[1, 0, 0, 0]] * 5, [0.95] * 5, cols)
    r = oracle_lib.render(sc, IDENT, cam)
    o = float(np.float32(0.95))
    assert abs(r["alpha"][24, 32] - (1 - (1 - o) ** 3)) < 1e-12 and abs(r["alpha"][24, 32] - 0.999875) < 1e-7
    assert r["nblend"][24, 32] == 3
    cols = sc.sh[:, 0, :].astype(np.float64) * Y00 + 0.5
    want = sum(cols[k] * o * (1 - o) ** k for k in range(3))
    np.testing.assert_allclose(r["rgb"][:, 24, 32], want, atol=1e-12)


def test_stop_threshold_is_1e4(oracle_lib):
    """The walk stops before blending a Gaussian that would take T below 1e-4
    (Sec. 3.1's tile rasterizer): three o = 0.9 layers leave T = 1e-3; a
    fourth layer of 0.93 would leave 7e-5 (not blended), one of 0.88 leaves
    1.2e-4 (blended)."""
    cam = Camera(100.0, 100.0, 32.5, 24.5, 64, 48)
    cols = np.random.default_rng(7).uniform(0, 1, (4, 3))
    for o4, nb in ((0.93, 3), (0.88, 4)):
        sc = _one([[0, 0, 10 + k] for k in range(4)], [[0.0] * 3] * 4, [[1, 0, 0, 0]] * 4, [0.9] * 3 + [o4], cols)
        o = sc.opacities.astype(np.float64)
        T3 = (1 - o[0]) ** 3
        assert (T3 * (1 - o[3]) < 1e-4) == (nb == 3) and 5e-5 < T3 * (1 - o[3]) < 1.5e-4
        r = oracle_lib.render(sc, IDENT, cam)
        assert r["nblend"][24, 32] == nb
        np.testing.assert_allclose(r["T"][24, 32], T3 * ((1 - o[3]) if nb == 4 else 1.0), rtol=1e-12)


def test_equal_depths_blend_in_index_order(oracle_lib):
    """Two Gaussians at the same depth are taken in index order (the (z, i)
    key): rgb = c0 a + c1 a (1 - a) at their common centre."""
    cam = Camera(100.0, 100.0, 32.5, 24.5, 64, 48)
    c = np.array([[1.0, 0.0, 0.2], [0.0, 1.0, 0.6]])
    for order in ([0, 1], [1, 0]):
        sc = _one([[0, 0, 10]] * 2, [[0.0] * 3] * 2, [[1, 0, 0, 0]] * 2, [0.5, 0.5], c[order])
        col = sc.sh[:, 0, :].astype(np.float64) * Y00 + 0.5
        a = float(sc.opacities[0])
        r = oracle_lib.render(sc, IDENT, cam)
        np.testing.assert_allclose(r["rgb"][:, 24, 32], col[0] * a + col[1] * a * (1 - a), atol=1e-12)


def test_gate_admits_alpha_of_exactly_1_255(oracle_lib):
    """The gate drops alpha < 1/255 only: an FP64 opacity of exactly 1/255
    centred on a pixel centre is blended there (support radius 0), and one
    just below it is not drawn at all."""
    cam = Camera(100.0, 100.0, 32.5, 24.5, 64, 48)
    sc = _one([[0, 0, 10]], [[0.0] * 3], [[1, 0, 0, 0]], [0.5], [[1, 1, 1]])
    r = oracle_lib.render(sc, IDENT, cam, overrides={"opacities": np.array([1 / 255])})
    assert r["nblend"][24, 32] == 1 and r["nblend"].sum() == 1
    assert abs(r["alpha"][24, 32] - 1 / 255) < 1e-15
    r = oracle_lib.render(sc, IDENT, cam, overrides={"opacities": np.array([np.nextafter(1 / 255, 0)])})
    assert r["alpha"].max() == 0


def test_fragile_pixels_mark_decisions_within_fp32_error(oracle_lib):
    """A pixel is fragile where a decision lies within the FP32 error bound of
    going the other way: alpha within it of 1/255 (above or below), T within
    it of 1e-4 at a step, or two blended Gaussians whose depths differ by
    less than their FP32 depth error.  The same decisions far from their
    thresholds leave the pixel robust."""
    cam = Camera(100.0, 100.0, 32.5, 24.5, 64, 48)
    one = _one([[0, 0, 10]], [[0.0] * 3], [[1, 0, 0, 0]], [0.5], [[1, 1, 1]])
    # the gate: the pixel one to the right of the centre (d = 1 px) sees
    # alpha = o exp(-1 / (2 s2)), s2 = (f sigma / z)^2 + 0.3
    s2 = (cam.fx * 1.0 / 10.0) ** 2 + 0.3
    for rel, frag in ((1 + 1e-9, True), (1 - 1e-9, True), (2.0, False)):
        o = rel / 255 * math.exp(0.5 / s2)
        r = oracle_lib.render(one, IDENT, cam, overrides={"opacities": np.array([o])})
        assert bool(r["fragile"][24, 33]) == frag, rel
    # the stop: three layers of 0.9, then a fourth leaving T = 1e-4 (1 +- 1e-9)
    four = _one([[0, 0, 10 + k] for k in range(4)], [[0.0] * 3] * 4, [[1, 0, 0, 0]] * 4, [0.5] * 4, [[1, 1, 1]] * 4)
    T3 = 0.1 ** 3
    for rel, frag in ((1 + 1e-9, True), (1 - 1e-9, True), (0.5, False)):
        o4 = 1 - 1e-4 * rel / T3
        r = oracle_lib.render(four, IDENT, cam, overrides={"opacities": np.array([0.9, 0.9, 0.9, o4])})
        assert bool(r["fragile"][24, 32]) == frag, rel
    # depth order: two blended Gaussians 5e-7 apart at z = 10 (FP32 error of
    # z there ~1e-6), then 1e-3 apart
    two = _one([[0, 0, 10]] * 2, [[0.0] * 3] * 2, [[1, 0, 0, 0]] * 2, [0.5, 0.5], [[1, 0, 0], [0, 1, 0]])
    for dz, frag in ((5e-7, True), (0.0, True), (1e-3, False)):
        m = np.array([[0, 0, 10.0], [0, 0, 10.0 + dz]])
        r = oracle_lib.render(two, IDENT, cam, overrides={"means": m})
        assert bool(r["fragile"][24, 32]) == frag, dz


def test_associativity_front_back(oracle_lib):
    """Compositing the front half and then the back half with 'over' equals
    compositing the whole depth-sorted list (no termination: low opacity)."""
    sc, P, cam = synth.tiny_scene(120, 11, feat_dim=8)
    sc.opacities[:] = np.minimum(sc.opacities, 0.35)
    p = oracle_lib.project(sc, P[0], cam)
    zmed = np.median(p["z"])
    front = np.nonzero(p["z"] < zmed)[0]
    back = np.nonzero(p["z"] >= zmed)[0]
    r = oracle_lib.render(sc, P[0], cam)
    assert r["T"].min() > 1e-3
    rf = oracle_lib.render(sc.subset(front), P[0], cam)
    rb = oracle_lib.render(sc.subset(back), P[0], cam)
    np.testing.assert_allclose(r["rgb"], rf["rgb"] + rf["T"] * rb["rgb"], atol=1e-12)
    np.testing.assert_allclose(r["T"], rf["T"] * rb["T"], atol=1e-12)
    np.testing.assert_allclose(r["feat"], rf["feat"] + rf["T"] * rb["feat"], atol=1e-12)
    Z = r["depth"] * r["alpha"]
    np.testing.assert_allclose(Z, rf["depth"] * rf["alpha"] + rf["T"] * rb["depth"] * rb["alpha"], atol=1e-9)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_brute_force_equals_tiled_bitwise(oracle_lib, tile):
    """The tiled renderer reaches exactly the per-pixel global-sort definition
    (seeds 0-99, N <= 200, 64x48)."""
    for seed in range(100):
        n = 20 + (seed * 37) % 181
        sc, P, cam = synth.tiny_scene(n, seed, feat_dim=4 if seed % 3 == 0 else 0, sh_degree=seed % 4)
        b = oracle_lib.render(sc, P[0], cam, mode="brute")
        t = oracle_lib.render(sc, P[0], cam, mode="tiled", tile=tile, margin=seed % 2)
        for k in ("rgb", "depth", "alpha", "T", "nblend"):
            assert np.array_equal(b[k], t[k]), (seed, k)
        if sc.feat is not None:
            assert np.array_equal(b["feat"], t["feat"])


def test_permutation_invariance(oracle_lib):
    sc, P, cam = synth.tiny_scene(200, 5, feat_dim=4, sh_degree=2)
    r = oracle_lib.render(sc, P[0], cam)
    perm = np.random.default_rng(0).permutation(sc.n)
    r2 = oracle_lib.render(sc.subset(perm), P[0], cam)
    for k in ("rgb", "depth", "alpha", "feat"):
        np.testing.assert_allclose(r[k], r2[k], atol=1e-12)


def test_support_rectangle_is_exact(oracle_lib):
    """Every pixel with alpha >= 1/255 lies in the Gaussian's rectangle, and the
    rectangle is the tightest one: a row and a column of every border hold a
    pixel within the ellipse's bounding box."""
    sc, P, cam = synth.tiny_scene(150, 9)
    p = oracle_lib.project(sc, P[0], cam)
    jj, ii = np.mgrid[0:cam.height, 0:cam.width]
    for i in np.nonzero(p["visible"])[0]:
        dx = ii + 0.5 - p["u"][i]
        dy = jj + 0.5 - p["v"][i]
        q = p["conic_a"][i] * dx * dx + 2 * p["conic_b"][i] * dx * dy + p["conic_c"][i] * dy * dy
        ok = p["o"][i] * np.exp(-0.5 * q) >= 1 / 255
        inside = (ii >= p["px0"][i]) & (ii <= p["px1"][i]) & (jj >= p["py0"][i]) & (jj <= p["py1"][i])
        assert not np.any(ok & ~inside), i
        assert abs(p["rx"][i] - math.sqrt(2 * math.log(255 * p["o"][i]) * p["cov_xx"][i])) < 1e-9


def test_degenerate_cases(oracle_lib):
    cam = Camera(100.0, 100.0, 32.0, 24.0, 64, 48)
    # empty scene -> background
    empty = _one(np.zeros((0, 3)), np.zeros((0, 3)), np.zeros((0, 4)), np.zeros(0), np.zeros((0, 3)))
    r = oracle_lib.render(empty, IDENT, cam, bg=(0.1, 0.2, 0.3))
    np.testing.assert_allclose(r["rgb"][:, 5, 5], [0.1, 0.2, 0.3])
    assert r["alpha"].max() == 0 and r["depth"].max() == 0
    # opacity below 1/255, behind the near plane, behind the camera -> invisible
    sc = _one([[0, 0, 10], [0, 0, 0.1], [0, 0, -5]], [[0.0] * 3] * 3, [[1, 0, 0, 0]] * 3,
              [1 / 255 * 0.99, 0.9, 0.9], [[1, 1, 1]] * 3)
    p = oracle_lib.project(sc, IDENT, cam)
    assert list(p["visible"]) == [0, 0, 0]
    r = oracle_lib.render(sc, IDENT, cam, bg=(0.5, 0.5, 0.5))
    assert r["alpha"].max() == 0
    np.testing.assert_allclose(r["rgb"], 0.5)
    # background is added with the remaining transmittance
    sc = _one([[0, 0, 10]], [[0.0] * 3], [[1, 0, 0, 0]], [0.8], [[1.0, 0.0, 0.0]])
    r0 = oracle_lib.render(sc, IDENT, cam)
    r1 = oracle_lib.render(sc, IDENT, cam, bg=(0.0, 1.0, 0.0))
    np.testing.assert_allclose(r1["rgb"][1], r0["T"], atol=1e-12)


def test_depth_is_camera_z_under_pose(oracle_lib):
    """Depth of a lone Gaussian is its camera-space z (Algorithm 1's depth),
    through a general pose."""
    cam = Camera(100.0, 100.0, 32.0, 24.0, 64, 48)
    pose = _rand_pose(3)
    R, t = pose.reshape(3, 4)[:, :3], pose.reshape(3, 4)[:, 3]
    mc = np.array([0.3, -0.2, 12.0])
    sc = _one([(mc - t) @ R], [[0.0] * 3], [[1, 0, 0, 0]], [0.9], [[0.5] * 3])
    r = oracle_lib.render(sc, pose, cam)
    zc = (R @ sc.means[0].astype(np.float64) + t)[2]
    d = r["depth"][r["alpha"] > 0]
    np.testing.assert_allclose(d, zc, rtol=1e-12)


# ------------------------------------------------------------------ SH
def test_sh_orthonormal_by_quadrature(oracle_lib):
    n_t, n_p = 24, 48
    x, w = np.polynomial.legendre.leggauss(n_t)
    phi = (np.arange(n_p) + 0.5) * 2 * np.pi / n_p
    ct, ph = np.meshgrid(x, phi, indexing="ij")
    st = np.sqrt(1 - ct ** 2)
    dirs = np.stack([st * np.cos(ph), st * np.sin(ph), ct], -1).reshape(-1, 3)
    wts = (w[:, None] * np.full(n_p, 2 * np.pi / n_p)[None]).reshape(-1)
    Y = oracle_lib.sh_basis(3, dirs)
    G = (Y * wts[:, None]).T @ Y
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_convention_matches_scipy(oracle_lib):
    """Real SH = sqrt(2) Re / Im of scipy's complex harmonics (Condon-Shortley
    phase), ordered m = -l..l."""
    from scipy.special import sph_harm_y
    rng = np.random.default_rng(4)
    d = rng.standard_normal((64, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = oracle_lib.sh_basis(3, d)
    theta = np.arccos(d[:, 2])
    phi = np.arctan2(d[:, 1], d[:, 0])
    for l in range(4):
        for m in range(-l, l + 1):
            c = sph_harm_y(l, abs(m), theta, phi)
            want = c.real if m == 0 else (np.sqrt(2) * (c.real if m > 0 else c.imag))
            np.testing.assert_allclose(Y[:, l * l + l + m], want, atol=1e-12)
    # first-order terms are -C y, C z, -C x
    C1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose(Y[:, 1:4], np.stack([-C1 * d[:, 1], C1 * d[:, 2], -C1 * d[:, 0]], 1), atol=1e-12)


def test_sh_degree0_reproduces_colour(oracle_lib):
    sc, P, cam = synth.tiny_scene(50, 2)
    p = oracle_lib.project(sc, P[0], cam)
    want = np.maximum(0, sc.sh[:, 0, :].astype(np.float64) * Y00 + 0.5)
    np.testing.assert_allclose(np.stack([p["r"], p["g"], p["b"]], 1), want, atol=1e-12)
    assert want.min() >= 0 and want.max() <= 1


def test_view_dependent_colour_uses_camera_centre(oracle_lib):
    """A degree-1 coefficient on Y_1,0 (= C1 * d_z) gives colour 0.5 + k C1 d_z
    with d the unit vector from the camera centre to the mean."""
    cam = Camera(100.0, 100.0, 32.0, 24.0, 64, 48)
    pose = _rand_pose(5)
    R, t = pose.reshape(3, 4)[:, :3], pose.reshape(3, 4)[:, 3]
    mw = (np.array([0.1, 0.2, 9.0]) - t) @ R
    sc = _one([mw], [[0.0] * 3], [[1, 0, 0, 0]], [0.9], [[0.5] * 3], sh_degree=1)
    sc.sh[0, 0, :] = 0.0
    sc.sh[0, 2, :] = [1.0, -0.5, 0.25]
    p = oracle_lib.project(sc, pose, cam)
    C = -R.T @ t
    d = sc.means[0].astype(np.float64) - C
    d /= np.linalg.norm(d)
    C1 = math.sqrt(3 / (4 * math.pi))
    np.testing.assert_allclose([p["r"][0], p["g"][0], p["b"][0]],
                               np.maximum(0, 0.5 + np.array([1.0, -0.5, 0.25]) * C1 * d[2]), atol=1e-12)


def test_sh_coefficients_indexed_l2_l_m(oracle_lib):
    """Degree-3 colour: coefficient k = l^2 + l + m multiplies the real
    harmonic Y_lm (scipy's, Condon-Shortley phase) at the unit direction from
    the camera centre to the mean; colour = max(0, 0.5 + sum)."""
    from scipy.special import sph_harm_y
    cam = Camera(100.0, 100.0, 32.0, 24.0, 64, 48)
    pose = _rand_pose(9)
    R, t = pose.reshape(3, 4)[:, :3], pose.reshape(3, 4)[:, 3]
    mw = (np.array([0.7, -0.4, 8.0]) - t) @ R
    sc = _one([mw], [[0.0] * 3], [[1, 0, 0, 0]], [0.9], [[0.5] * 3], sh_degree=3)
    rng = np.random.default_rng(11)
    sc.sh[0] = rng.uniform(-0.3, 0.3, (16, 3)).astype(np.float32)
    sc.sh[0, 0, :] = 2.0  # keeps every channel above the clamp
    p = oracle_lib.project(sc, pose, cam)
    d = sc.means[0].astype(np.float64) + R.T @ t
    d /= np.linalg.norm(d)
    theta, phi = np.arccos(d[2]), np.arctan2(d[1], d[0])
    want = np.full(3, 0.5)
    for l in range(4):
        for m in range(-l, l + 1):
            cpx = sph_harm_y(l, abs(m), theta, phi)
            y = cpx.real if m == 0 else np.sqrt(2) * (cpx.real if m > 0 else cpx.imag)
            want += sc.sh[0, l * l + l + m].astype(np.float64) * y
    assert want.min() > 0
    np.testing.assert_allclose([p["r"][0], p["g"][0], p["b"][0]], want, atol=1e-12)


def test_negative_colour_is_clamped_to_zero(oracle_lib):
    """colour = max(0, SH sum + 0.5): a DC term below -0.5 gives 0, and the
    render shows no trace of that channel."""
    cam = Camera(100.0, 100.0, 32.5, 24.5, 64, 48)
    sc = _one([[0, 0, 10]], [[0.0] * 3], [[1, 0, 0, 0]], [0.8], [[-0.4, 0.3, 1.2]])
    p = oracle_lib.project(sc, IDENT, cam)
    assert p["r"][0] == 0.0 and p["g"][0] > 0 and p["b"][0] > 1
    r = oracle_lib.render(sc, IDENT, cam)
    assert r["rgb"][0].max() == 0.0 and r["rgb"][1].max() > 0


def test_fp64_inputs_read_like_fp32(oracle_lib):
    """The FP64 input path (finite differences, exact pins) reads every array
    in the layout of the FP32 one: the same values through either path render
    the same images bit for bit."""
    sc, P, cam = synth.tiny_scene(60, 13, feat_dim=8, sh_degree=3)
    base = oracle_lib.render(sc, P[0], cam)
    feat = synth.bf16_bits_to_f32(sc.feat).astype(np.float64)
    for key, arr in (("means", sc.means), ("opacities", sc.opacities), ("log_scales", sc.log_scales),
                     ("quats", sc.quats), ("sh", sc.sh), ("feat", feat)):
        r = oracle_lib.render(sc, P[0], cam, overrides={key: np.asarray(arr, np.float64)})
        for out in ("rgb", "depth", "alpha", "feat"):
            assert np.array_equal(r[out], base[out]), (key, out)


# ------------------------------------------------------------------ tile lists
@pytest.mark.parametrize("size", [(64, 48, 13), (60, 44, 17)])
def test_tile_lists_follow_the_listing_rule(oracle_lib, size):
    """A visible Gaussian is listed in a tile of its pixel rectangle exactly
    when the tile's rectangle of pixel centres (clipped to the image: the
    ragged size has partial tiles) meets its support ellipse
    q <= 2 ln(255 o); checked here by brute force on a 1/40 px grid of each
    such rectangle (grid minimum vs the listing decision), in (z, index)
    order.  Listing must also be a subset of the rectangle rule."""
    W, H, seed = size
    sc, P, cam = synth.tiny_scene(180, seed, width=W, height=H)
    tile = 16
    p = oracle_lib.project(sc, P[0], cam)
    off, ids, edge = oracle_lib.tile_lists(sc, P[0], cam, tile)
    ntx = (cam.width + tile - 1) // tile
    nty = (cam.height + tile - 1) // tile
    k2 = 2.0 * np.log(255.0 * p["o"])
    dropped = 0
    for ty in range(nty):
        for tx in range(ntx):
            b = ty * ntx + tx
            got = list(ids[off[b]:off[b + 1]])
            rect = [i for i in range(sc.n) if p["visible"][i] and p["px0"][i] // tile <= tx <= p["px1"][i] // tile
                    and p["py0"][i] // tile <= ty <= p["py1"][i] // tile]
            assert set(got) <= set(rect)
            xs = np.arange(tx * tile + 0.5, min((tx + 1) * tile, cam.width) - 0.5 + 1e-9, 1 / 40)
            ys = np.arange(ty * tile + 0.5, min((ty + 1) * tile, cam.height) - 0.5 + 1e-9, 1 / 40)
            X, Y = np.meshgrid(xs, ys)
            want = []
            for i in rect:
                a, bb, c = p["conic_a"][i], p["conic_b"][i], p["conic_c"][i]
                dx, dy = X - p["u"][i], Y - p["v"][i]
                qmin = (a * dx * dx + 2 * bb * dx * dy + c * dy * dy).min()
                # grid spacing bound: |grad q| * spacing / sqrt(2) at most
                slack = 2 * np.sqrt(max(a, c) * k2[i]) * np.sqrt(max(a, c)) / 40
                if qmin <= k2[i]:
                    want.append(i)
                else:
                    assert i not in got or qmin <= k2[i] + slack, (tx, ty, i)
                    if i in got:
                        want.append(i)
            dropped += len(rect) - len(got)
            want.sort(key=lambda i: (p["z"][i], i))
            assert got == want, (tx, ty)
    assert dropped > 0  # the rule is tighter than the rectangle on this scene


def test_edge_flag_marks_an_ellipse_grazing_a_tile_corner(oracle_lib):
    """A Gaussian whose support ellipse passes within the edge tolerance of a
    tile's corner of pixel centres is flagged as a tile-edge Gaussian even
    though its pixel rectangle is far from every tile boundary; moved 0.3 px
    further into that tile it is not flagged."""
    cam = Camera(100.0, 100.0, 32.0, 24.0, 64, 48)
    z, tile, corner = 10.0, 16, 15.5  # tile (0, 0)'s last pixel centre

    def scene_at(t):
        u = v = corner + t  # centre on the corner's diagonal, outside tile 0
        m = [(u - cam.cx) * z / cam.fx, (v - cam.cy) * z / cam.fy, z]
        return _one([m], [[math.log(0.15)] * 3], [[1, 0, 0, 0]], [0.8], [[1, 1, 1]])

    def gap(t):  # q at the corner minus the support threshold
        p = oracle_lib.project(scene_at(t), IDENT, cam)
        dx, dy = corner - p["u"][0], corner - p["v"][0]
        q = p["conic_a"][0] * dx * dx + 2 * p["conic_b"][0] * dx * dy + p["conic_c"][0] * dy * dy
        return q - 2 * np.log(255 * p["o"][0]), p

    lo, hi = 0.0, 8.0
    assert gap(lo)[0] < 0 < gap(hi)[0]
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        lo, hi = (mid, hi) if gap(mid)[0] < 0 else (lo, mid)
    for t, flagged in ((lo - 1e-5, 1), (lo - 0.3, 0)):
        _, p = gap(t)
        for b in (p["bx0"][0], p["bx1"][0], p["by0"][0], p["by1"][0]):  # rectangle far from tile bounds
            assert abs(b - round(b)) > 0.05 or int(round(b)) % tile not in (0, tile - 1)
        off, ids, edge = oracle_lib.tile_lists(scene_at(t), IDENT, cam, tile)
        assert 0 in ids[off[0]:off[1]]  # tile 0 lists it (the corner lies inside the ellipse)
        assert edge[0] == flagged, t


def test_min_q_box_closed_forms_and_grid(oracle_lib):
    rng = np.random.default_rng(5)
    # mean inside -> 0; isotropic axis-aligned -> a * squared distance
    assert oracle_lib.min_q_box(np.array([[2.0, 0.3, 1.0, 5.0, 5.0, 4.0, 6.0, 4.5, 5.5]]))[0] == 0.0
    r = oracle_lib.min_q_box(np.array([[0.5, 0.0, 0.5, 0.0, 0.0, 3.0, 4.0, -1.0, 1.0]]))[0]
    assert abs(r - 0.5 * 9.0) < 1e-15
    r = oracle_lib.min_q_box(np.array([[0.5, 0.0, 0.5, 0.0, 0.0, 3.0, 4.0, 4.0, 6.0]]))[0]
    assert abs(r - 0.5 * 25.0) < 1e-15
    rows = []
    for _ in range(200):
        L = rng.normal(size=(2, 2))
        S = L @ L.T + 0.1 * np.eye(2)
        a, b, c = S[0, 0], S[0, 1], S[1, 1]
        u, v = rng.uniform(-5, 5, 2)
        x0, y0 = rng.uniform(-6, 4, 2)
        x1, y1 = x0 + rng.uniform(0.1, 3), y0 + rng.uniform(0.1, 3)
        rows.append([a, b, c, u, v, x0, x1, y0, y1])
    rows = np.array(rows)
    got = oracle_lib.min_q_box(rows)
    for row, g in zip(rows, got):
        a, b, c, u, v, x0, x1, y0, y1 = row
        X, Y = np.meshgrid(np.linspace(x0, x1, 401), np.linspace(y0, y1, 401))
        dx, dy = X - u, Y - v
        q = a * dx * dx + 2 * b * dx * dy + c * dy * dy
        assert g <= q.min() + 1e-12  # never above any point of the rectangle
        assert q.min() - g <= 1e-3 * (1 + q.min())  # and at the grid's resolution


# ------------------------------------------------------------------ pose tangent and residual
def test_se3_exp_matches_matrix_exponential():
    from scipy.linalg import expm
    from oracle.se3 import exp_se3, hat
    rng = np.random.default_rng(0)
    for _ in range(20):
        xi = rng.normal(0, 0.7, 6)
        X = np.zeros((4, 4))
        X[:3, :3] = hat(xi[3:])
        X[:3, 3] = xi[:3]
        np.testing.assert_allclose(exp_se3(xi), expm(X), atol=1e-12)
    np.testing.assert_allclose(exp_se3(np.zeros(6)), np.eye(4))


def test_residual_gradient_closed_form():
    from oracle.loss import residual, residual_grad
    rng = np.random.default_rng(1)
    rgb, rgbt = rng.uniform(0, 1, (3, 5, 4)), rng.uniform(0, 1, (3, 5, 4))
    f, ft = rng.normal(0, 1, (6, 5, 4)), rng.normal(0, 1, (6, 5, 4))
    gr, gf = residual_grad(rgb, f, rgbt, ft)
    h = 1e-6
    for idx in [(0, 1, 2), (2, 4, 3), (1, 0, 0)]:
        a = rgb.copy(); a[idx] += h
        b = rgb.copy(); b[idx] -= h
        assert abs((residual(a, f, rgbt, ft) - residual(b, f, rgbt, ft)) / (2 * h) - gr[idx]) < 1e-7
    for idx in [(0, 1, 2), (5, 4, 3), (3, 2, 1)]:
        a = f.copy(); a[idx] += h
        b = f.copy(); b[idx] -= h
        assert abs((residual(rgb, a, rgbt, ft) - residual(rgb, b, rgbt, ft)) / (2 * h) - gf[idx]) < 1e-7
    # identical features give zero feature residual
    assert abs(residual(rgbt, ft, rgbt, ft)) < 1e-8


@pytest.mark.parametrize("opaque", [False, True])
def test_frozen_render_reproduces_reference(oracle_lib, opaque):
    """Replaying the blended lists with the decisions frozen reproduces the
    render bit for bit, also where alpha is clamped at 0.99 (opaque case)."""
    sc, P, cam = synth.tiny_scene(150, 21, feat_dim=4)
    if opaque:
        sc.opacities[:] = 1.0
    r = oracle_lib.render(sc, P[0], cam, want_lists=True)
    fz = oracle_lib.render_frozen(sc, P[0], cam, r["lists"], r["nblend"])
    for k in ("rgb", "depth", "alpha", "T", "feat"):
        assert np.array_equal(r[k], fz[k]), k
    if opaque:  # some Gaussian's pair at its nearest pixel centre is clamped
        p = oracle_lib.project(sc, P[0], cam)
        dx = np.floor(p["u"]) + 0.5 - p["u"]
        dy = np.floor(p["v"]) + 0.5 - p["v"]
        q = p["conic_a"] * dx * dx + 2 * p["conic_b"] * dx * dy + p["conic_c"] * dy * dy
        assert ((q < -2 * np.log(0.99)) & (p["visible"] == 1)).any()


def test_translation_identity_of_finite_differences(oracle_lib):
    """Moving every mean by delta equals moving the camera by -delta, so
    dL/drho = R sum_i dL/dmu_i (any SH degree)."""
    from oracle.loss import fd_gradients, residual
    sc, P, cam = synth.tiny_scene(25, 31, feat_dim=4, sh_degree=2)
    pose = P[0].astype(np.float64)
    tgt = oracle_lib.render(sc, synth.perturb_poses(P[0], 1, 99, 0.5, 1.0)[0], cam)
    loss = lambda o: residual(o["rgb"], o["feat"], tgt["rgb"], tgt["feat"])
    g_pose, gp, _ = fd_gradients(sc, pose, cam, loss, h=1e-5, gauss_ids=range(sc.n), params=("means",))
    g_means = gp["means"]
    R = pose.reshape(3, 4)[:, :3]
    want = R @ g_means.sum(0)
    assert np.linalg.norm(want) > 1e-4
    np.testing.assert_allclose(g_pose[:3], want, rtol=1e-5, atol=1e-9)


def test_left_jacobian_against_the_matrix_exponential():
    """The oracle's left Jacobian of SE(3) (its defining series) against
    scipy's matrix exponential and logarithm: the columns of J_l(xi) are
    central differences of log(Exp(xi + h e_k) Exp(xi)^-1); J_l(0) = I; the
    rotation block is the V of Exp's translation; and the first-order rule
    holds for rotations up to 170 degrees with translations of tens of metres."""
    from scipy.linalg import expm, logm
    from oracle.se3 import exp_se3, left_jacobian

    def twist(x):
        M = np.zeros((4, 4))
        M[:3, :3] = np.array([[0, -x[5], x[4]], [x[5], 0, -x[3]], [-x[4], x[3], 0]])
        M[:3, 3] = x[:3]
        return M

    def vee(M):
        return np.r_[M[:3, 3], M[2, 1], M[0, 2], M[1, 0]]

    assert np.array_equal(left_jacobian(np.zeros(6)), np.eye(6))
    rng = np.random.default_rng(4)
    for scale_r, scale_w in ((0.1, 0.01), (3.0, 0.5), (20.0, 2.0), (5.0, np.radians(170))):
        xi = np.r_[rng.normal(0, scale_r, 3), rng.normal(size=3)]
        xi[3:] *= scale_w / np.linalg.norm(xi[3:])
        np.testing.assert_allclose(exp_se3(xi), expm(twist(xi)), atol=1e-12 * max(1.0, scale_r))
        J = left_jacobian(xi)
        h = 1e-6
        base_inv = np.linalg.inv(expm(twist(xi)))
        fd = np.zeros((6, 6))
        for k in range(6):
            e = np.zeros(6)
            e[k] = h
            lp = vee(np.real(logm(expm(twist(xi + e)) @ base_inv)))
            lm = vee(np.real(logm(expm(twist(xi - e)) @ base_inv)))
            fd[:, k] = (lp - lm) / (2 * h)
        np.testing.assert_allclose(J, fd, atol=1e-6 * max(1.0, scale_r))
        # the rotation block is V (Exp's translation is V rho)
        V = exp_se3(np.r_[1.0, 0, 0, xi[3:]])[:3, 3], exp_se3(np.r_[0, 1.0, 0, xi[3:]])[:3, 3], \
            exp_se3(np.r_[0, 0, 1.0, xi[3:]])[:3, 3]
        np.testing.assert_allclose(J[3:, 3:], np.stack(V, 1), atol=1e-12)
        np.testing.assert_allclose(J[:3, :3], np.stack(V, 1), atol=1e-12)
