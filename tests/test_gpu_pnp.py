"""GPU pose solve (Sec. 3.4, Eq. 10: RANSAC over given 3-point samples,
truncated-quadratic refinement), back-projection and Algorithm 2's
consistency check through the C ABI against the FP64 oracle; and the dense
stage end to end (render, match, back-project, solve) on a synthetic scene."""
import math

import numpy as np
import pytest
from scipy.spatial.transform import Rotation

import synth
from gpu_util import log

pytestmark = pytest.mark.gpu

CAM = synth.Camera(800.0, 780.0, 480.0, 270.0, 960, 540)


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2507_15683_amd as hg
    return hg


@pytest.fixture(scope="module")
def op():
    from oracle import pnp
    return pnp


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    return (t if dtype is None else t.to(dtype)).cuda()


def _pose(seed, alt=150.0):
    rng = np.random.default_rng(seed)
    R = Rotation.from_rotvec([math.pi, 0, 0]).as_matrix() @ Rotation.from_rotvec(rng.normal(0, 0.1, 3)).as_matrix()
    C = np.array([rng.normal(0, 5), rng.normal(0, 5), alt])
    T = np.eye(4)
    T[:3, :3] = R.T
    T[:3, 3] = -R.T @ C
    return T


def _problem(seed, n, noise, outliers):
    """float32 correspondences seen by a known pose, with noise and
    outliers, and a prior 2 m / 2 degrees away (all in float32 so that GPU
    and oracle read the same numbers)."""
    from oracle.se3 import exp_se3
    rng = np.random.default_rng(seed)
    T = _pose(seed)
    u = rng.uniform(10, CAM.width - 10, n)
    v = rng.uniform(10, CAM.height - 10, n)
    d = rng.uniform(120, 180, n)
    Xc = np.stack([d * (u - CAM.cx) / CAM.fx, d * (v - CAM.cy) / CAM.fy, d], 1)
    X = (Xc - T[:3, 3]) @ T[:3, :3]
    p = np.stack([u, v], 1) + rng.normal(0, noise, (n, 2))
    out = rng.random(n) < outliers
    p[out] = np.stack([rng.uniform(0, CAM.width, out.sum()), rng.uniform(0, CAM.height, out.sum())], 1)
    T0 = exp_se3(np.r_[rng.normal(0, 1.2, 3), np.radians(rng.normal(0, 1.2, 3))]) @ T
    return (p.astype(np.float32), X.astype(np.float32), T, T0[:3, :].reshape(12).astype(np.float32), out)


@pytest.mark.parametrize("seed,n,noise,outliers,H", [(1, 2000, 0.5, 0.3, 128), (2, 300, 0.0, 0.0, 16),
                                                     (3, 5000, 1.0, 0.5, 256), (4, 7, 0.2, 0.0, 5)])
def test_pnp_parity(hg, op, seed, n, noise, outliers, H):
    """Hypotheses and their inlier counts (up to points within 5e-3 px of
    tau) wherever the oracle's Gauss-Newton fitted its sample exactly (a
    sample with no exact fit lets the iteration wander, and rounding then
    decides where it ends); the winner, the refined pose, and the inliers
    against the FP64 errors at the returned pose."""
    import torch
    log(f"case: pnp seed {seed} n {n} noise {noise} outliers {outliers} H {H}")
    p, X, T, T0, out = _problem(seed, n, noise, outliers)
    samples = np.random.default_rng(100 + seed).integers(0, n, (H, 3)).astype(np.int32)
    tau = 2.0
    p64, X64 = p.astype(np.float64), X.astype(np.float64)
    ref = op.pnp_ransac(p64, X64, CAM, T0.astype(np.float64), samples, tau=tau)
    r = hg.Renderer()
    g = r.pnp(_t(p), _t(X), hg.Intrinsics.of(CAM), _t(T0), _t(samples), tau=tau, want_hyps=True)
    torch.cuda.synchronize()
    counts = g["counts"].cpu().numpy()
    hyps = g["hyp_poses"].cpu().numpy().reshape(H, 3, 4)
    fitted = np.array([ref["valid"][h] and ref["hyp_err"][h][samples[h]].max() < 1e-4 for h in range(H)])
    checked = 0
    for h in np.nonzero(fitted)[0]:
        assert counts[h] >= 0, h
        np.testing.assert_allclose(hyps[h][:, :3], ref["hyps"][h][:, :3], atol=1e-5)
        np.testing.assert_allclose(hyps[h][:, 3], ref["hyps"][h][:, 3], atol=1e-3, rtol=0)
        near = int((np.abs(ref["hyp_err"][h] - tau) < 5e-3).sum())
        assert abs(int(counts[h]) - int(ref["counts"][h])) <= near, (h, counts[h], ref["counts"][h], near)
        checked += 1
    # degenerate samples (a repeated index) are invalid on both sides
    rep = np.array([len(set(s_.tolist())) < 3 for s_ in samples])
    assert not ref["valid"][rep].any() and (counts[rep] == -1).all()
    best = int(g["best"].cpu().numpy()[0])
    top = np.sort(ref["counts"][fitted])[::-1]
    log("hypotheses fitted", checked, "of", H, "valid", int(ref["valid"].sum()), "best", best, ref["best"])
    if len(top) and (len(top) == 1 or top[0] - top[1] > 5) and ref["counts"][ref["best"]] == top[0]:
        assert best == ref["best"]
    pose = g["pose"].cpu().numpy().reshape(3, 4)
    dt = np.abs(pose[:, 3] - ref["pose"][:, 3]).max()
    dR = np.abs(pose[:, :3] - ref["pose"][:, :3]).max()     # (arccos of the trace is blind below ~1e-3 deg)
    inl = g["inliers"].cpu().numpy().astype(bool)
    log("pose diff", float(dt), "m, rotation entries", float(dR), "; inliers", int(g["n_inliers"].cpu().numpy()[0]),
        int(ref["inliers"].sum()))
    assert dt < 5e-3 and dR < 1e-5
    e_own = op.errors(np.vstack([pose.astype(np.float64), [0, 0, 0, 1]]), CAM, X64, p64)
    clear = np.abs(e_own - tau) >= 1e-3
    assert np.array_equal(inl[clear], (e_own < tau)[clear])
    assert int(g["n_inliers"].cpu().numpy()[0]) == int(inl.sum())
    if noise == 0.0 and outliers == 0.0:
        np.testing.assert_allclose(pose, T[:3, :], atol=2e-3)


def test_degenerate_and_empty(hg, op):
    """A repeated index makes a sample invalid (-1); with no valid sample the
    prior pose is returned unrefined and its inliers counted."""
    import torch
    p, X, T, T0, _ = _problem(5, 50, 0.1, 0.0)
    r = hg.Renderer()
    g = r.pnp(_t(p), _t(X), hg.Intrinsics.of(CAM), _t(T0), _t(np.array([[3, 3, 3], [1, 2, 40]], np.int32)))
    assert list(g["counts"].cpu().numpy() >= 0) == [False, True] and int(g["best"].cpu().numpy()[0]) == 1
    g = r.pnp(_t(p), _t(X), hg.Intrinsics.of(CAM), _t(T0), _t(np.array([[7, 7, 7]], np.int32)))
    torch.cuda.synchronize()
    assert int(g["best"].cpu().numpy()[0]) == -1
    np.testing.assert_array_equal(g["pose"].cpu().numpy(), T0)
    ref = op.pnp_ransac(p.astype(np.float64), X.astype(np.float64), CAM, T0.astype(np.float64), [[7, 7, 7]])
    assert int(g["n_inliers"].cpu().numpy()[0]) == int(ref["inliers"].sum())


def test_backprojection_matches_oracle(hg, op):
    rng = np.random.default_rng(21)
    depth = rng.uniform(80, 250, (CAM.height, CAM.width)).astype(np.float32)
    pose = _pose(22)[:3, :].reshape(12).astype(np.float32)
    pix = rng.integers(0, CAM.width * CAM.height, 5000).astype(np.int32)
    g = hg.backproject(_t(depth), _t(pose), hg.Intrinsics.of(CAM), _t(pix)).cpu().numpy()
    want = op.backproject(depth.astype(np.float64), pose.astype(np.float64), CAM, pix)
    np.testing.assert_allclose(g, want, rtol=0, atol=5e-4)


def test_consistency_matches_oracle(hg, op):
    from oracle.se3 import exp_se3
    T = _pose(31)
    for jumps, want in (([1.0, 2.0, 0.5], True), ([1.0, 25.0], False), ([19.0, 19.0, 19.0], True), ([], True)):
        seq = [T]
        for k, deg in enumerate(jumps):
            ax = np.array([0.2, 0.7, -0.3]) / np.linalg.norm([0.2, 0.7, -0.3])
            seq.append(exp_se3(np.r_[0.5, 0, 0, np.radians(deg) * ax]) @ seq[-1])
        poses = np.stack([s[:3, :].reshape(12) for s in seq]).astype(np.float32)
        rel, ang = hg.pose_consistency(_t(poses), 20.0)
        assert bool(rel.cpu().numpy()[0]) == want == op.consistent([q.reshape(3, 4) for q in poses.astype(np.float64)])
        if jumps:
            assert abs(float(ang.cpu().numpy()[0]) - max(jumps)) < 1e-2


def test_dense_stage_end_to_end(hg):
    """Render the query view and a view from a prior 1 m / 1.7 degrees away,
    match their feature maps coarse (8 x 8 means of the fine maps) to fine,
    lift the rendered side with the prior's depth and solve: the solved
    camera centre is closer to the query's than the prior's was."""
    import torch
    from oracle.se3 import exp_se3
    log("case: dense stage end to end")
    sc = synth.terrain_scene(60_000, 240.0, 77, sh_degree=0, feat_dim=32)
    cam = synth.Camera(230.0, 230.0, 128.0, 96.0, 256, 192)
    Tq = np.eye(4)
    Tq[:3, :] = synth.down_pose((0.0, 0.0), 120.0, (0.05, -0.03), 0.7).reshape(3, 4)
    Tp = exp_se3(np.r_[1.0, -0.8, 0.6, np.radians([1.0, -0.8, 1.2])]) @ Tq
    scene = hg.GaussianScene.from_numpy(sc)
    r = hg.Renderer()
    Kq = hg.Intrinsics.of(cam)

    def render(T):
        o = r.render(scene, _t(T[:3, :].reshape(1, 12).astype(np.float32)), Kq, tile=16)
        return o["feat"][0].clone(), o["depth"][0].clone()

    def coarse(f):
        D, H, W = f.shape
        return f.reshape(D, H // 8, 8, W // 8, 8).mean(dim=(2, 4)).to(torch.bfloat16).contiguous()

    q_f, _ = render(Tq)
    p_f, depth = render(Tp)
    m = r.match(coarse(q_f), coarse(p_f), q_f.to(torch.bfloat16).contiguous(), p_f.to(torch.bfloat16).contiguous(),
                tau_coarse=0.1, tau_fine=0.1)
    torch.cuda.synchronize()
    K_c = int(m["n_coarse"].cpu().numpy().view(np.uint32)[0])
    fq = m["fine_query"][: 64 * K_c]
    fr = m["fine_render"][: 64 * K_c]
    ok = fq >= 0
    fq, fr = fq[ok], fr[ok]
    n = int(fq.numel())
    log("coarse matches", K_c, "fine matches", n)
    assert n > 500
    W = cam.width
    p2d = torch.stack([(fq % W).float() + 0.5, (fq // W).float() + 0.5], 1).contiguous()
    pose_p = _t(Tp[:3, :].reshape(12).astype(np.float32))
    x3d = hg.backproject(depth, pose_p, Kq, fr.to(torch.int32).contiguous())
    samples = _t(np.random.default_rng(5).integers(0, n, (512, 3)).astype(np.int32))
    g = r.pnp(p2d, x3d, Kq, pose_p, samples, tau=2.0)
    torch.cuda.synchronize()
    Ts = g["pose"].cpu().numpy().reshape(3, 4).astype(np.float64)
    C = lambda P: -P[:, :3].T @ P[:, 3]
    e0 = np.linalg.norm(C(Tp[:3, :]) - C(Tq[:3, :]))
    e1 = np.linalg.norm(C(Ts) - C(Tq[:3, :]))
    log("camera centre error: prior", float(e0), "m, solved", float(e1), "m; inliers",
        int(g["n_inliers"].cpu().numpy()[0]), "of", n)
    assert int(g["best"].cpu().numpy()[0]) >= 0
    assert e1 < 0.5 * e0


def test_no_correspondences(hg):
    """With no correspondences every sample is invalid: the prior pose comes
    back with no inliers."""
    import torch
    T0 = _pose(41)[:3, :].reshape(12).astype(np.float32)
    r = hg.Renderer()
    empty2 = torch.empty((0, 2), dtype=torch.float32, device="cuda")
    empty3 = torch.empty((0, 3), dtype=torch.float32, device="cuda")
    g = r.pnp(empty2, empty3, hg.Intrinsics.of(CAM), _t(T0), _t(np.array([[0, 1, 2], [3, 4, 5]], np.int32)))
    torch.cuda.synchronize()
    assert (g["counts"].cpu().numpy() == -1).all() and int(g["best"].cpu().numpy()[0]) == -1
    np.testing.assert_array_equal(g["pose"].cpu().numpy(), T0)
    assert int(g["n_inliers"].cpu().numpy()[0]) == 0
    x = hg.backproject(torch.ones((4, 5), device="cuda"), _t(T0), hg.Intrinsics.of(CAM),
                       torch.empty(0, dtype=torch.int32, device="cuda"))
    assert x.shape == (0, 3)
