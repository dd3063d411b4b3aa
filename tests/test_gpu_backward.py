"""GPU backward against FP64 central finite differences of the oracle (frozen
decisions, h = 1e-4), within 1e-3 relative; visibility (Algorithm 1: only
contributors get gradients); the translation identity; residual kernel
parity; an Adam pose-refinement run; and graph capture of a refinement step."""
import numpy as np
import pytest

import synth
from gpu_util import log, to_np

pytestmark = pytest.mark.gpu
REL = 1e-3


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


def _t(a, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30))


def _check_components(g, fd, what):
    g = np.asarray(g, dtype=np.float64).ravel()
    fd = np.asarray(fd, dtype=np.float64).ravel()
    big = np.abs(fd) > 1e-2 * np.abs(fd).max()
    comp = np.abs(g[big] - fd[big]) / np.abs(fd[big])
    log(f"{what}: rel-norm {_rel(g, fd):.2e}, worst large component {comp.max(initial=0):.2e}")
    assert _rel(g, fd) <= REL, what
    assert comp.max(initial=0) <= 10 * REL, what


def _setup_residual(hg, orc, sc, P, cam, seed):
    """Target = oracle render at a hidden pose offset N(0,2 m), N(0,2 deg)."""
    hidden = synth.perturb_poses(P[0], 1, seed, 2.0, 2.0)[0]
    tgt = orc.render(sc, hidden, cam)
    tgt_rgb = _t(tgt["rgb"][None].astype(np.float32))
    tgt_feat = _t(tgt["feat"][None].astype(np.float32)) if tgt["feat"] is not None else None
    return tgt, tgt_rgb, tgt_feat


def _gpu_grads(hg, sc, P, cam, tgt_rgb, tgt_feat, want):
    r = hg.Renderer()
    scene = hg.GaussianScene.from_numpy(sc)
    out = r.render(scene, _t(P), hg.Intrinsics.of(cam))
    loss, g_rgb, g_feat = hg.residual(out["rgb"], out["feat"], tgt_rgb, tgt_feat)
    grads = r.backward(dict(rgb=g_rgb, feat=g_feat), want=want)
    return {k: to_np(v) for k, v in grads.items()}, out, float(to_np(loss)[0])


def test_residual_kernel_matches_oracle(hg, orc):
    from oracle.loss import residual, residual_grad
    rng = np.random.default_rng(0)
    P, D, H, W = 2, 8, 20, 24
    rgb = rng.uniform(0, 1, (P, 3, H, W)).astype(np.float32)
    rgbt = rng.uniform(0, 1, (P, 3, H, W)).astype(np.float32)
    f = rng.normal(0, 1, (P, D, H, W)).astype(np.float32)
    ft = rng.normal(0, 1, (P, D, H, W)).astype(np.float32)
    f[:, :, 0, 0] = 0.0  # an empty-feature pixel
    log("case: residual kernel P=2 D=8")
    loss, g_rgb, g_feat = hg.residual(_t(rgb), _t(f), _t(rgbt), _t(ft), lam_f=0.7)
    for p in range(P):
        L = residual(rgb[p].astype(np.float64), f[p].astype(np.float64), rgbt[p].astype(np.float64),
                     ft[p].astype(np.float64), lam_f=0.7)
        gr, gf = residual_grad(rgb[p].astype(np.float64), f[p].astype(np.float64), rgbt[p].astype(np.float64),
                               ft[p].astype(np.float64), lam_f=0.7)
        assert abs(to_np(loss)[p] - L) <= 1e-5 * abs(L)
        np.testing.assert_allclose(to_np(g_rgb)[p], gr, atol=1e-9)
        np.testing.assert_allclose(to_np(g_feat)[p], gf, atol=1e-7, rtol=1e-4)


def test_pose_means_opacity_grads_vs_fd(hg, orc):
    """The FD subset: 5k Gaussians, 128x96; residual against a hidden-offset
    target; pose (6), and means/opacities of 64 contributing Gaussians."""
    from oracle.loss import fd_gradients, residual, residual_frozen_signs
    sc, P, cam = synth.fd_subset_5k(0)
    tgt, tgt_rgb, tgt_feat = _setup_residual(hg, orc, sc, P, cam, 41)
    log("case: differentiable_200k FD subset, GPU backward")
    g, out, loss = _gpu_grads(hg, sc, P, cam, tgt_rgb, tgt_feat, ("pose", "means", "opacities"))
    ref = orc.render(sc, P[0], cam, want_lists=True, list_cap=512)
    blended = np.unique(ref["lists"][ref["lists"] >= 0])
    ids = np.random.default_rng(1).choice(blended, 64, replace=False)
    lf = residual_frozen_signs(ref["rgb"], tgt["rgb"], tgt["feat"])
    log("case: oracle FD")
    g_pose, gp, _ = fd_gradients(sc, P[0].astype(np.float64), cam, lf, h=1e-4, gauss_ids=ids,
                                 params=("means", "opacities"))
    log("loss gpu", loss, "oracle", residual(ref["rgb"], ref["feat"], tgt["rgb"], tgt["feat"]), "fragile px",
        int(ref["fragile"].sum()))
    log("pose gpu", g["pose"][0], "fd", g_pose)
    _check_components(g["pose"][0], g_pose, "pose")
    _check_components(g["means"][ids], gp["means"], "means")
    _check_components(g["opacities"][ids], gp["opacities"], "opacities")


def test_depth_alpha_grads_vs_fd(hg, orc):
    """A linear functional of depth, alpha and rgb exercises the depth
    normalisation and the final-transmittance terms of the backward."""
    import torch
    from oracle.loss import fd_gradients, linear_functional
    sc, P, cam = synth.tiny_scene(250, 61, width=72, height=56, feat_dim=8, sh_degree=1)
    rng = np.random.default_rng(2)
    w = dict(depth=rng.normal(0, 1e-2, (cam.height, cam.width)), alpha=rng.normal(0, 1, (cam.height, cam.width)),
             rgb=rng.normal(0, 1, (3, cam.height, cam.width)))
    r = hg.Renderer()
    scene = hg.GaussianScene.from_numpy(sc)
    log("case: linear functional of depth/alpha/rgb, bg=(0.2,0.3,0.4)")
    out = r.render(scene, _t(P), hg.Intrinsics.of(cam), bg=(0.2, 0.3, 0.4))
    go = {k: _t(v[None].astype(np.float32)) for k, v in w.items()}
    grads = r.backward(go, want=("pose", "means", "opacities"))
    ref = orc.render(sc, P[0], cam, want_lists=True, bg=(0.2, 0.3, 0.4))
    blended = np.unique(ref["lists"][ref["lists"] >= 0])
    ids = np.random.default_rng(3).choice(blended, 32, replace=False)
    wf = {k: v.astype(np.float32).astype(np.float64) for k, v in w.items()}
    g_pose, gp, _ = fd_gradients(sc, P[0].astype(np.float64), cam, lambda o: linear_functional(o, wf), h=1e-4,
                                 gauss_ids=ids, params=("means", "opacities"), bg=(0.2, 0.3, 0.4))
    _check_components(to_np(grads["pose"])[0], g_pose, "pose (depth/alpha)")
    _check_components(to_np(grads["means"])[ids], gp["means"], "means (depth/alpha)")
    _check_components(to_np(grads["opacities"])[ids], gp["opacities"], "opacities (depth/alpha)")


def test_shape_colour_feature_grads_vs_fd(hg, orc):
    """log-scales, quaternions, SH (degree 2) and feature vectors."""
    from oracle.loss import fd_gradients, residual, residual_frozen_signs
    sc, P, cam = synth.tiny_scene(220, 71, width=64, height=48, feat_dim=16, sh_degree=2)
    tgt, tgt_rgb, tgt_feat = _setup_residual(hg, orc, sc, P, cam, 72)
    log("case: scales/quats/sh/feat grads")
    g, out, _ = _gpu_grads(hg, sc, P, cam, tgt_rgb, tgt_feat, ("pose", "means", "log_scales", "quats", "sh", "feat"))
    ref = orc.render(sc, P[0], cam, want_lists=True)
    blended = np.unique(ref["lists"][ref["lists"] >= 0])
    ids = np.random.default_rng(4).choice(blended, 12, replace=False)
    lf = residual_frozen_signs(ref["rgb"], tgt["rgb"], tgt["feat"])
    g_pose, gp, _ = fd_gradients(sc, P[0].astype(np.float64), cam, lf, h=1e-4, gauss_ids=ids,
                                 params=("means", "log_scales", "quats", "sh", "feat"))
    _check_components(g["pose"][0], g_pose, "pose (SH2)")
    for k in ("means", "log_scales", "quats", "sh", "feat"):
        _check_components(g[k][ids], gp[k], k)


def test_translation_identity_and_visibility(hg, orc):
    """dL/drho = R sum_i dL/dmu_i (exact for any SH degree), and with
    L = sum(rgb) (Algorithm 1) the Gaussians with a non-zero mean gradient are
    exactly the blended ones (up to Gaussians seen only at fragile pixels)."""
    import torch
    sc, P, cam = synth.tiny_scene(300, 81, width=80, height=60, sh_degree=3)
    r = hg.Renderer()
    scene = hg.GaussianScene.from_numpy(sc)
    log("case: RGB.sum().backward() visibility")
    out = r.render(scene, _t(P), hg.Intrinsics.of(cam))
    grads = r.backward(dict(rgb=torch.ones_like(out["rgb"])), want=("pose", "means"))
    gm = to_np(grads["means"])
    gpose = to_np(grads["pose"])[0]
    R = P[0].reshape(3, 4)[:, :3].astype(np.float64)
    want = R @ gm.sum(0)
    assert np.linalg.norm(gpose[:3] - want) <= 1e-4 * np.linalg.norm(want), (gpose[:3], want)
    ref = orc.render(sc, P[0], cam, want_lists=True)
    lists = ref["lists"]
    frag = ref["fragile"].reshape(-1)
    blended = set(np.unique(lists[lists >= 0]).tolist())
    robust = set(np.unique(lists[~frag][lists[~frag] >= 0]).tolist())
    nonzero = set(np.nonzero(np.linalg.norm(gm, axis=1) > 0)[0].tolist())
    log(f"blended {len(blended)}, robust {len(robust)}, gpu nonzero {len(nonzero)}, fragile px {int(frag.sum())}")
    assert robust <= nonzero
    # a Gaussian the oracle never blends may only get a gradient through a
    # fragile pixel (a decision within FP32 rounding of flipping)
    assert len(nonzero - blended) <= int(frag.sum())


def test_sh3_pose_grad_vs_fd(hg, orc):
    from oracle.loss import fd_gradients, residual, residual_frozen_signs
    sc, P, cam = synth.tiny_scene(260, 91, width=64, height=48, feat_dim=8, sh_degree=3)
    tgt, tgt_rgb, tgt_feat = _setup_residual(hg, orc, sc, P, cam, 92)
    log("case: SH3 pose grad")
    g, _, _ = _gpu_grads(hg, sc, P, cam, tgt_rgb, tgt_feat, ("pose",))
    ref = orc.render(sc, P[0], cam)
    lf = residual_frozen_signs(ref["rgb"], tgt["rgb"], tgt["feat"])
    g_pose, _, _ = fd_gradients(sc, P[0].astype(np.float64), cam, lf, h=1e-4, params=())
    _check_components(g["pose"][0], g_pose, "pose (SH3)")


def test_batched_backward_matches_single(hg, orc):
    """Pose gradients of a batch equal the per-pose ones; Gaussian gradients
    are their sum."""
    import torch
    sc, P, cam = synth.tiny_scene(300, 95, width=64, height=48, feat_dim=8, sh_degree=1)
    Ps = synth.perturb_poses(P[0], 4, 96, 1.0, 2.0)
    scene = hg.GaussianScene.from_numpy(sc)
    r = hg.Renderer()
    log("case: batched backward 4 poses")
    out = r.render(scene, _t(Ps), hg.Intrinsics.of(cam), schedule="tile")
    gb = r.backward(dict(rgb=torch.ones_like(out["rgb"]), feat=torch.ones_like(out["feat"])), want=("pose", "means"))
    acc = np.zeros((sc.n, 3))
    for p in range(4):
        o1 = r.render(scene, _t(Ps[p:p + 1]), hg.Intrinsics.of(cam))
        g1 = r.backward(dict(rgb=torch.ones_like(o1["rgb"]), feat=torch.ones_like(o1["feat"])), want=("pose", "means"))
        assert _rel(to_np(gb["pose"])[p], to_np(g1["pose"])[0]) < 1e-5
        acc += to_np(g1["means"])
    assert _rel(to_np(gb["means"]), acc) < 1e-5


def test_refinement_converges(hg, orc):
    """Config-4 style: 200k Gaussians, 640x480, target rendered at a hidden
    pose offset; 50 Adam steps on the pose tangent reduce the residual and
    the pose error."""
    import torch
    sc, truth, start, cam = synth.differentiable_200k(0)
    log("case: differentiable_200k refinement, oracle target")
    tgt = orc.render(sc, truth[0], cam)
    tgt_rgb = _t(tgt["rgb"][None].astype(np.float32))
    tgt_feat = _t(tgt["feat"][None].astype(np.float32))
    scene = hg.GaussianScene.from_numpy(sc)
    K = hg.Intrinsics.of(cam)
    r = hg.Renderer()
    poses = _t(start.copy())
    m = torch.zeros((1, 6), device="cuda")
    v = torch.zeros((1, 6), device="cuda")
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    losses = []
    for it in range(50):
        out = r.render(scene, poses, K)
        loss, g_rgb, g_feat = hg.residual(out["rgb"], out["feat"], tgt_rgb, tgt_feat)
        g = r.backward(dict(rgb=g_rgb, feat=g_feat), want=("pose",))
        hg.pose_adam(poses, g["pose"], m, v, step, lr_rho=5e-2, lr_phi=2e-3)
        losses.append(float(to_np(loss)[0]))
    fin = to_np(poses)[0].reshape(3, 4)
    tr = truth[0].reshape(3, 4).astype(np.float64)
    st = start[0].reshape(3, 4).astype(np.float64)
    cpos = lambda T: -T[:, :3].T @ T[:, 3]
    e0 = np.linalg.norm(cpos(st) - cpos(tr))
    e1 = np.linalg.norm(cpos(fin) - cpos(tr))
    log(f"loss {losses[0]:.4f} -> {losses[-1]:.4f}; camera-centre error {e0:.3f} m -> {e1:.3f} m; "
        f"steps {int(to_np(step)[0])}")
    assert int(to_np(step)[0]) == 50
    assert losses[-1] < 0.8 * losses[0]
    assert e1 < e0


def test_graph_replay_matches_eager(hg):
    """One refinement step (render, residual, backward, Adam) captured in a
    HIP graph and replayed 5 times (with eager work and synchronisation
    between replays) gives the same poses as the same 5 steps run eagerly."""
    import torch
    sc, P, cam = synth.tiny_scene(300, 99, width=64, height=48, feat_dim=8)
    Ps = synth.perturb_poses(P[0], 3, 100, 1.0, 2.0)
    tg = synth.perturb_poses(P[0], 3, 101, 1.0, 2.0)
    scene = hg.GaussianScene.from_numpy(sc)
    K = hg.Intrinsics.of(cam)

    def make():
        r = hg.Renderer()
        r.reserve(3, K.width, K.height, 16, 4096, 1 << 18, sc.n)
        st = dict(poses=_t(Ps.copy()), m=torch.zeros((3, 6), device="cuda"), v=torch.zeros((3, 6), device="cuda"),
                  step=torch.zeros(1, dtype=torch.int32, device="cuda"))
        st["out"] = r.alloc_outputs(scene, 3, K)
        st["res"] = (torch.empty(3, device="cuda"), torch.empty((3, 3, K.height, K.width), device="cuda"),
                     torch.empty((3, 8, K.height, K.width), device="cuda"))
        st["grads"] = r.alloc_grads(scene, 3, ("pose",))
        return r, st

    rt = hg.Renderer()
    tgt = rt.render(scene, _t(tg), K)
    tgt = {k: (None if v is None else v.clone()) for k, v in tgt.items()}
    opts = rt.opts(schedule="tile")

    def step_fn(r, st, stream):
        r.render_into(scene, st["poses"], K, st["out"], opts, stream=stream)
        hg.residual(st["out"]["rgb"], st["out"]["feat"], tgt["rgb"], tgt["feat"], out=st["res"], stream=stream)
        r.backward(dict(rgb=st["res"][1], feat=st["res"][2]), want=("pose",), P=3, scene=scene, grads=st["grads"],
                   stream=stream)
        hg.pose_adam(st["poses"], st["grads"]["pose"], st["m"], st["v"], st["step"], stream=stream)

    s = torch.cuda.Stream()
    r1, st1 = make()
    with torch.cuda.stream(s):
        step_fn(r1, st1, s)  # warm-up sizes
    s.synchronize()
    assert r1.check_overflow(s) == 0
    r2, st2 = make()
    st1["poses"].copy_(_t(Ps)); st1["m"].zero_(); st1["v"].zero_(); st1["step"].zero_()
    torch.cuda.synchronize()
    log("case: capture one refinement step")
    r1.graph_begin(s)
    step_fn(r1, st1, s)
    r1.graph_end()
    for k in range(5):
        r1.graph_launch(1, s)
        s.synchronize()
        with torch.cuda.stream(s):
            step_fn(r2, st2, s)
        s.synchronize()
        d = np.abs(to_np(st1["poses"]) - to_np(st2["poses"])).max()
        log(f"replay {k}: max |pose graph - eager| = {d:.2e}")
        assert d < 1e-5
    assert int(to_np(st1["step"])[0]) == 5


@pytest.mark.parametrize("D,tile,bf16", [(32, 16, False), (8, 8, False), (0, 32, False), (32, 8, True)])
def test_residual_backward_matches_separate(hg, orc, D, tile, bf16):
    """The residual formed inside the blend backward equals the residual
    kernel followed by the plain backward: loss up to summation order, pose
    and mean gradients to float-atomic rounding."""
    import torch
    sc, P, cam = synth.tiny_scene(500, 40 + D, width=83, height=61, feat_dim=D, sh_degree=1)
    Ps = synth.perturb_poses(P[0], 3, 41, 1.0, 2.0)
    tg = synth.perturb_poses(P[0], 3, 42, 1.0, 2.0)
    scene = hg.GaussianScene.from_numpy(sc)
    K = hg.Intrinsics.of(cam)
    tgt = hg.Renderer().render(scene, _t(tg), K)
    tgt = {k: (None if v is None else v.clone()) for k, v in tgt.items()}
    log(f"case: residual backward D={D} tile={tile} bf16={bf16}")
    r = hg.Renderer()
    a = r.render(scene, _t(Ps), K, tile=tile, feat_bf16=bf16)
    la, g_rgb, g_feat = hg.residual(a["rgb"], a["feat"], tgt["rgb"], tgt["feat"])
    ga = r.backward(dict(rgb=g_rgb, feat=g_feat), want=("pose", "means"))
    ga = {k: to_np(v).copy() for k, v in ga.items()}
    lb, gb = r.residual_backward(tgt["rgb"], tgt["feat"], want=("pose", "means"))
    assert np.allclose(to_np(la), to_np(lb), rtol=1e-5, atol=0)
    assert _rel(to_np(gb["pose"]), ga["pose"]) < 1e-5
    assert _rel(to_np(gb["means"]), ga["means"]) < 1e-5


@pytest.mark.parametrize("tile", [8, 16])
def test_pose_only_residual_backward_matches_full(hg, tile):
    """Without an opacity gradient the residual backward forms eight
    per-splat sums instead of ten (no opacity or depth sum): the loss is
    bitwise that of the full form, pose and mean gradients agree to
    float-atomic rounding."""
    import torch
    sc, P, cam = synth.tiny_scene(700, 91, width=97, height=66, feat_dim=32, sh_degree=3)
    Ps = synth.perturb_poses(P[0], 3, 92, 1.0, 2.0)
    tg = synth.perturb_poses(P[0], 3, 93, 1.0, 2.0)
    scene = hg.GaussianScene.from_numpy(sc)
    K = hg.Intrinsics.of(cam)
    tgt = hg.Renderer().render(scene, _t(tg), K)
    tgt = {k: (None if v is None else v.clone()) for k, v in tgt.items()}
    log(f"case: pose-only residual backward tile={tile}")
    r = hg.Renderer()
    r.render(scene, _t(Ps), K, tile=tile, feat_accum="valu")
    lf, gf = r.residual_backward(tgt["rgb"], tgt["feat"], want=("pose", "means", "opacities"))
    lf = lf.clone()
    gf = {k: to_np(v).copy() for k, v in gf.items()}
    lp, gp = r.residual_backward(tgt["rgb"], tgt["feat"], want=("pose", "means"))
    assert torch.equal(lf, lp)
    assert np.abs(gf["opacities"]).max() > 0
    assert _rel(to_np(gp["pose"]), gf["pose"]) < 1e-5
    assert _rel(to_np(gp["means"]), gf["means"]) < 1e-5


def test_residual_backward_shared_target(hg):
    """One target shared by all poses gives what the same target replicated
    per pose gives (loss bitwise, gradients to float-atomic rounding)."""
    sc, P, cam = synth.tiny_scene(400, 50, width=70, height=52, feat_dim=16, sh_degree=1)
    Ps = synth.perturb_poses(P[0], 4, 51, 1.0, 2.0)
    scene = hg.GaussianScene.from_numpy(sc)
    K = hg.Intrinsics.of(cam)
    q = hg.Renderer().render(scene, _t(P), K)
    one_rgb, one_feat = q["rgb"].clone(), q["feat"].clone()
    rep_rgb = one_rgb.expand(4, -1, -1, -1).contiguous()
    rep_feat = one_feat.expand(4, -1, -1, -1).contiguous()
    log("case: shared vs replicated target")
    r = hg.Renderer()
    r.render(scene, _t(Ps), K)
    la, ga = r.residual_backward(one_rgb, one_feat)
    la, pa = to_np(la).copy(), to_np(ga["pose"]).copy()
    lb, gb = r.residual_backward(rep_rgb, rep_feat)
    assert np.array_equal(la, to_np(lb))
    assert _rel(to_np(gb["pose"]), pa) < 1e-6


@pytest.mark.parametrize("tile", [8, 16])
def test_matrix_core_feature_term_matches_valu(hg, orc, tile):
    """The backward's feature term h = gF . f on the matrix cores (bf16 parts
    of the FP32 pixel gradient, exact products) gives the gradients of the
    per-pixel FP32 dot product up to summation order (and the forward's
    matrix-core feature sum, |delta| <= 1e-7), with the residual formed in the
    prologue and with dL/dfeat images."""
    import torch
    sc, P, cam = synth.tiny_scene(700, 60 + tile, width=97, height=70, feat_dim=32, sh_degree=2)
    Ps = synth.perturb_poses(P[0], 3, 61, 1.0, 2.0)
    tg = synth.perturb_poses(P[0], 3, 62, 1.0, 2.0)
    scene = hg.GaussianScene.from_numpy(sc)
    K = hg.Intrinsics.of(cam)
    tgt = hg.Renderer().render(scene, _t(tg), K)
    tgt = {k: (None if v is None else v.clone()) for k, v in tgt.items()}
    log(f"case: matrix-core feature term, tile {tile}")
    res = {}
    # "mfma": the feature sum of the forward and the feature term of the
    # backward on the matrix cores; "valu": both on the VALU
    for fa in ("valu", "mfma"):
        r = hg.Renderer()
        out = r.render(scene, _t(Ps), K, tile=tile, feat_accum=fa)
        lb, gb = r.residual_backward(tgt["rgb"], tgt["feat"], want=("pose", "means", "opacities"))
        _, g_rgb, g_feat = hg.residual(out["rgb"], out["feat"], tgt["rgb"], tgt["feat"])
        gp = r.backward(dict(rgb=g_rgb, feat=g_feat), want=("pose", "means", "opacities"))
        res[fa] = ({k: to_np(v).copy() for k, v in gb.items()}, {k: to_np(v).copy() for k, v in gp.items()},
                   to_np(lb).copy())
        torch.cuda.synchronize()
    for which in (0, 1):
        for k in ("pose", "means", "opacities"):
            rel = _rel(res["mfma"][which][k], res["valu"][which][k])
            log(which, k, rel)
            assert rel < 1e-5, (which, k, rel)
    np.testing.assert_allclose(res["mfma"][2], res["valu"][2], rtol=1e-6, atol=0)


@pytest.mark.parametrize("tile", [8, 16, 32])
def test_backward_schedules_agree(hg, tile):
    """The blend backward under its persistent work queues (pose-major and
    tile-major) gives the grid launch's gradients -- pose, means, opacities
    and features -- up to float-atomic rounding, for the plain backward and
    for the residual formed inside it."""
    import torch
    sc, P, cam = synth.tiny_scene(600, 70 + tile, width=97, height=71, feat_dim=16, sh_degree=1)
    Ps = synth.perturb_poses(P[0], 5, 71, 1.0, 2.0)
    tg = synth.perturb_poses(P[0], 5, 72, 1.0, 2.0)
    scene = hg.GaussianScene.from_numpy(sc)
    K = hg.Intrinsics.of(cam)
    tgt = hg.Renderer().render(scene, _t(tg), K)
    tgt = {k: (None if v is None else v.clone()) for k, v in tgt.items()}
    want = ("pose", "means", "opacities", "feat")
    res = {}
    for sched in ("grid", "pose", "tile"):
        log(f"case: backward schedule {sched}, tile {tile}, 5 poses")
        r = hg.Renderer()
        out = r.render(scene, _t(Ps), K, tile=tile, schedule=sched)
        g = r.backward(dict(rgb=torch.ones_like(out["rgb"]), feat=torch.ones_like(out["feat"])), want=want)
        g = {k: to_np(v).copy() for k, v in g.items()}
        r.render(scene, _t(Ps), K, tile=tile, schedule=sched)
        loss, gr = r.residual_backward(tgt["rgb"], tgt["feat"], want=("pose", "means"))
        res[sched] = (g, {k: to_np(v).copy() for k, v in gr.items()}, to_np(loss).copy())
        r.close()
    g0, r0, l0 = res["grid"]
    for sched in ("pose", "tile"):
        g1, r1, l1 = res[sched]
        for k in want:
            assert _rel(g1[k], g0[k]) < 1e-5, (sched, k)
        for k in ("pose", "means"):
            assert _rel(r1[k], r0[k]) < 1e-5, (sched, "residual", k)
        assert np.array_equal(l1, l0), (sched, "loss")
