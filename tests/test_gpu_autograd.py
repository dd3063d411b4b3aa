"""The autograd form of the renderer (torch.autograd.Function around the
render and its backward): the gradient of a torch-written L1 + feature-cosine
residual equals the library backward fed the same output gradients and the
oracle's FP64 central differences; Algorithm 1's visibility check written as
RGB.sum().backward(); a non-zero pose tangent xi (render at Exp(xi) T,
gradient through the left Jacobian) against differences over xi itself; the
retraction and tangent kernels against the oracle's SE(3) formulas; and a
stale backward (another render on the same renderer first) refused."""
import numpy as np
import pytest

import synth
from gpu_util import log, parity, to_np

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hg():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    import paper_2507_15683_amd as hg
    return hg


@pytest.fixture(scope="module")
def orc():
    import oracle
    oracle.build(force=False)
    return oracle


def _t(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _rel(a, b):
    a = np.asarray(a, np.float64).ravel()
    b = np.asarray(b, np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _torch_residual(rgb, feat, rgb_t, feat_t):
    """L = 1/(HW) sum_p [sum_c |rgb - rgb*| + (1 - cos(F, F*))] written in
    torch ops (FP32), summed over poses."""
    import torch
    HW = rgb.shape[-1] * rgb.shape[-2]
    L = (rgb - rgb_t).abs().sum() / HW
    if feat is not None:
        dot = (feat * feat_t).sum(1)
        n = feat.norm(dim=1) * feat_t.norm(dim=1) + 1e-8
        L = L + (1.0 - dot / n).sum() / HW
    return L


def test_autograd_matches_backward_and_finite_differences(hg, orc):
    """FD subset (5k Gaussians, 128x96) against a target at a hidden pose
    offset: torch.autograd.grad of the residual with respect to xi, means and
    opacities equals Renderer.backward fed torch's own dL/d(rgb, feat) (to
    float-atomic ordering, 1e-6 relative), and the pose and 64 Gaussians'
    gradients match the oracle's frozen-decision differences within 1e-3."""
    import torch
    from oracle.loss import fd_gradients, residual_frozen_signs
    sc, P, cam = synth.fd_subset_5k(0)
    hidden = synth.perturb_poses(P[0], 1, 41, 2.0, 2.0)[0]
    tgt = orc.render(sc, hidden, cam)
    rgb_t = _t(tgt["rgb"][None].astype(np.float32))
    feat_t = _t(tgt["feat"][None].astype(np.float32))
    scene = hg.GaussianScene.from_numpy(sc)
    scene.means.requires_grad_(True)
    scene.opacities.requires_grad_(True)
    r = hg.Renderer()
    K = hg.Intrinsics.of(cam)
    xi = torch.zeros((1, 6), dtype=torch.float32, device="cuda", requires_grad=True)
    log("case: autograd residual on the FD subset")
    rgb, depth, alpha, feat = hg.render_differentiable(r, scene, _t(P), K, xi=xi)
    L = _torch_residual(rgb, feat, rgb_t, feat_t)
    g_xi, g_mu, g_o = torch.autograd.grad(L, [xi, scene.means, scene.opacities], retain_graph=True)
    g_rgb, g_feat = torch.autograd.grad(L, [rgb, feat])
    direct = r.backward(dict(rgb=g_rgb, feat=g_feat), want=("pose", "means", "opacities"), P=1, scene=scene)
    for name, a, b in (("pose", g_xi, direct["pose"]), ("means", g_mu, direct["means"]),
                       ("opacities", g_o, direct["opacities"])):
        rel = _rel(to_np(a), to_np(b))
        log(name, "autograd vs backward rel", rel)
        assert rel <= 1e-6, name
    ref = orc.render(sc, P[0], cam, want_lists=True, list_cap=512)
    blended = np.unique(ref["lists"][ref["lists"] >= 0])
    ids = np.random.default_rng(1).choice(blended, 64, replace=False)
    lf = residual_frozen_signs(ref["rgb"], tgt["rgb"], tgt["feat"])
    log("case: oracle FD")
    g_pose, gp, _ = fd_gradients(sc, P[0].astype(np.float64), cam, lf, h=1e-4, gauss_ids=ids,
                                 params=("means", "opacities"))
    for name, g, fd in (("pose", to_np(g_xi)[0], g_pose), ("means", to_np(g_mu)[ids], gp["means"]),
                        ("opacities", to_np(g_o)[ids], gp["opacities"])):
        log(name, "autograd vs FD rel", _rel(g, fd))
        assert _rel(g, fd) <= 1e-3, name


def test_visibility_by_rgb_sum_backward(hg, orc):
    """Algorithm 1's render-visibility test written as RGB.sum().backward():
    the Gaussians whose mean receives a non-zero gradient are blended at some
    pixel (the oracle's blend lists), and xi's gradient equals the library
    backward of an all-ones rgb gradient."""
    import torch
    sc, P, cam = synth.tiny_scene(300, 71, width=96, height=64, feat_dim=8, sh_degree=1)
    scene = hg.GaussianScene.from_numpy(sc)
    scene.means.requires_grad_(True)
    r = hg.Renderer()
    xi = torch.zeros((1, 6), dtype=torch.float32, device="cuda", requires_grad=True)
    log("case: RGB.sum().backward() on a 300-Gaussian 96x64 view")
    rgb, _, _, _ = hg.render_differentiable(r, scene, _t(P), hg.Intrinsics.of(cam), xi=xi)
    rgb.sum().backward()
    nz = np.nonzero(np.abs(to_np(scene.means.grad)).sum(1) > 0)[0]
    ref = orc.render(sc, P[0], cam, want_lists=True, list_cap=512)
    blended = np.unique(ref["lists"][ref["lists"] >= 0])
    log("mean-gradient support", len(nz), "blended (oracle)", len(blended))
    assert set(nz.tolist()) <= set(blended.tolist())
    assert len(nz) >= 0.97 * len(blended)
    r2 = hg.Renderer()
    out = r2.render(scene, _t(P), hg.Intrinsics.of(cam))
    direct = r2.backward(dict(rgb=torch.ones_like(out["rgb"])), want=("pose",))
    assert _rel(to_np(xi.grad), to_np(direct["pose"])) <= 1e-6


def test_nonzero_tangent_against_differences_over_xi(hg, orc):
    """At xi = (0.3, -0.2, 0.5 m, 0.01, -0.02, 0.015 rad) the forward renders
    Exp(xi) T (oracle parity at that pose) and d/dxi matches the oracle's
    central differences over xi itself (the left Jacobian's chain rule)."""
    import torch
    from oracle.loss import fd_tangent_gradient, residual_frozen_signs
    sc, P, cam = synth.fd_subset_5k(0)
    hidden = synth.perturb_poses(P[0], 1, 43, 2.0, 2.0)[0]
    tgt = orc.render(sc, hidden, cam)
    rgb_t = _t(tgt["rgb"][None].astype(np.float32))
    feat_t = _t(tgt["feat"][None].astype(np.float32))
    scene = hg.GaussianScene.from_numpy(sc)
    r = hg.Renderer()
    xi0 = np.array([0.3, -0.2, 0.5, 0.01, -0.02, 0.015])
    xi = _t(xi0[None].astype(np.float32)).requires_grad_(True)
    log("case: non-zero tangent on the FD subset")
    rgb, depth, alpha, feat = hg.render_differentiable(r, scene, _t(P), hg.Intrinsics.of(cam), xi=xi)
    from oracle.se3 import left_perturb
    x32 = xi0.astype(np.float32).astype(np.float64)
    ref = orc.render(sc, left_perturb(P[0].astype(np.float64), x32).astype(np.float32), cam)
    parity(dict(rgb=rgb.detach(), depth=depth.detach(), alpha=alpha.detach(), feat=feat.detach()), ref,
           label="render at Exp(xi) T")
    L = _torch_residual(rgb, feat, rgb_t, feat_t)
    L.backward()
    lf = residual_frozen_signs(ref["rgb"], tgt["rgb"], tgt["feat"])
    g_fd, _ = fd_tangent_gradient(sc, P[0].astype(np.float64), x32, cam, lf, h=1e-4)
    g = to_np(xi.grad)[0]
    log("xi grad", g, "fd", g_fd, "rel", _rel(g, g_fd))
    assert _rel(g, g_fd) <= 1e-3


def test_retraction_and_tangent_kernels_against_oracle(hg):
    """hgsr_pose_retract against Exp(xi) T and hgsr_pose_tangent_grad against
    J_l(xi)^T g of the oracle, for rotations up to 170 degrees; J_l(0) = I
    bit for bit."""
    import torch
    from oracle.se3 import left_jacobian, left_perturb
    rng = np.random.default_rng(8)
    n = 37
    poses = synth.perturb_poses(synth.down_pose((0.0, 0.0), 150.0, (0.1, 0.05), 0.3), n, 9, 5.0, 3.0)
    xi = np.concatenate([rng.normal(0, 3.0, (n, 3)), rng.normal(0, 1.0, (n, 3))], 1)
    xi[:, 3:] *= (rng.uniform(0, np.radians(170), n) / np.linalg.norm(xi[:, 3:], axis=1))[:, None]
    xi[0] = 0.0
    xi = xi.astype(np.float32)
    g = rng.normal(0, 1, (n, 6)).astype(np.float32)
    log("case: retraction / tangent kernels, 37 poses")
    out = to_np(hg.pose_retract(_t(poses.astype(np.float32)), _t(xi)))
    gx = to_np(hg.pose_tangent_grad(_t(xi), _t(g)))
    for p in range(n):
        want = left_perturb(poses[p].astype(np.float32).astype(np.float64), xi[p].astype(np.float64))
        np.testing.assert_allclose(out[p], want, rtol=1e-6, atol=1e-5 * (1 + np.abs(want).max()))
        wg = left_jacobian(xi[p].astype(np.float64)).T @ g[p].astype(np.float64)
        np.testing.assert_allclose(gx[p], wg, rtol=2e-6, atol=1e-6 * np.abs(wg).max())
    assert np.array_equal(gx[0], g[0])


def test_backward_of_a_replaced_render_is_refused(hg):
    """render_differentiable, then another render on the same renderer,
    then .backward() of the first: the library refuses (HGSR_ERR_STATE)
    instead of returning the second render's gradients; the library call
    itself refuses a stale render_id, and accepts the current one."""
    import torch
    sc, P, cam = synth.tiny_scene(200, 72, width=64, height=48, feat_dim=0, sh_degree=0)
    scene = hg.GaussianScene.from_numpy(sc)
    r = hg.Renderer()
    K = hg.Intrinsics.of(cam)
    log("case: stale backward refused")
    rgb, _, _, _ = hg.render_differentiable(r, scene, _t(P), K)
    first = r.render_id()
    r.render(scene, _t(synth.perturb_poses(P[0], 1, 3, 1.0, 1.0)), K)
    assert r.render_id() == first + 1
    with pytest.raises(hg.HgsrError, match="STATE"):
        rgb.sum().backward()
    g1 = dict(rgb=torch.ones((1, 3, cam.height, cam.width), device="cuda"))
    with pytest.raises(hg.HgsrError, match="STATE"):
        r.backward(g1, want=("pose",), render_id=first)
    r.backward(g1, want=("pose",), render_id=first + 1)
    torch.cuda.synchronize()
