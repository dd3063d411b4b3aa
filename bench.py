"""Benchmark of the splat rasterizer on one MI355X.

Headline (the JSON line's `value`): forward rendering throughput on
1,000,000 Gaussians (900k on a 1x1 km heightfield plus 2,000 box buildings,
SH degree 3, 32-d bf16 features), one 1920x1080 view, fx = 1500, 100-300 m
altitude, tilt <= 30 deg.  A step renders that view (projection, tile
binning, sort, blend: RGB + depth + alpha + 32-channel FP32 feature map).

Beside it, in the same line:
  fwd_bwd     one pose-refinement step (render, L1 + feature-cosine residual,
              backward to the pose, Adam update) over 64 candidate poses of
              the same scene at 960x540: the batched path (autotuned tile and
              schedule, one launch per stage for all poses, the step captured
              in a HIP graph) against the plain single-pose path looped over
              the same poses (eager, no graph).
  partitioned 8M Gaussians in 16 spatial partitions over 4x4 km, 16 query
              poses, three coarse-to-fine levels (480x270, 960x540,
              1920x1080) of 20 batched refinement steps each, every level a
              captured graph; per-step latency p50/p99 and device memory use.
  roofline    the blend kernel's algorithmic bytes per launch over its
              event-timed duration, against HBM peak.
  cpu_baseline the FP64 oracle on the host cores, on a bounded sample.

python bench.py [--gpus 1] [--steps 50] [--warmup 10] [--no-cpu]
                [--no-fwd-bwd] [--no-partitioned]
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# Counter summaries the roofline figures read: each records a hash of the
# sources of the kernels it counted and is used only while they still match.
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "blend_fwd_1080p_1M_traffic.txt")
SQ_FILE = os.path.join(ROOT, "profiles", "render_1080p_1M_sq_counters.md")
REFINE_SQ_FILE = os.path.join(ROOT, "profiles", "refine_64x960x540_1M_sq_counters.md")
CSRC = "paper_2507_15683_amd/csrc/"
BLEND_SOURCES = (CSRC + "blend.hip", CSRC + "hgsr_device.hpp")
REFINE_SOURCES = (CSRC + "blend.hip", CSRC + "backward.hip", CSRC + "hgsr_device.hpp")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(files) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def blend_source_hash() -> str:
    return source_hash(BLEND_SOURCES)


def guarded_fields(path: str, sources, tile: int, feat_accum: str = "valu"):
    """The key: value fields of a committed counter summary, or None when it
    was taken on other sources or another kernel variant."""
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                if ":" in line and not line.startswith(("#", "|", "`", " ")):
                    k, v = line.split(":", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_sha256") != source_hash(sources):
            return None
        if int(kv.get("tile", 0)) != tile or kv.get("feat_accum", "valu") != feat_accum:
            return None
        return kv
    except (OSError, ValueError):
        return None


def measured_valu(tile: int, feat_accum: str):
    """VALU instructions per blend launch from the committed SQ counter
    summary, or None."""
    kv = guarded_fields(SQ_FILE, BLEND_SOURCES, tile, feat_accum)
    try:
        return int(kv["valu_insts_per_dispatch"]) if kv else None
    except (KeyError, ValueError):
        return None


def measured_traffic(tile: int, feat_accum: str):
    """HBM bytes per blend launch from the committed counter summary, or None
    when it was taken on other sources or another kernel variant."""
    kv = guarded_fields(TRAFFIC_FILE, BLEND_SOURCES, tile, feat_accum)
    try:
        return int(kv["traffic_bytes_per_launch"]) if kv else None
    except (KeyError, ValueError):
        return None


_VALU_RATE = None


def valu_rate(hg) -> float:
    """Wave64 FP32 FMA instructions per second the device issues, measured
    live by the library's probe (independent FMA chains over every CU): the
    ceiling the VALU issue fractions are taken against."""
    global _VALU_RATE
    if _VALU_RATE is None:
        import ctypes
        from paper_2507_15683_amd import _lib
        r = ctypes.c_double(0.0)
        _lib.check(_lib.load().hgsr_probe_valu_rate(ctypes.byref(r), None), "hgsr_probe_valu_rate")
        _VALU_RATE = float(r.value)
        log(f"bench: VALU probe {_VALU_RATE:.4g} wave64 FMA/s ({_VALU_RATE / (256 * 2.4e9):.3f} per CU per "
            "cycle at the nominal 2.4 GHz)")
    return _VALU_RATE


def valu_peak_desc(hg) -> dict:
    r = valu_rate(hg)
    return {"wave_fma_per_s": round(r, -6), "per_cu_cycle_at_2p4ghz": round(r / (256 * 2.4e9), 3),
            "source": "hgsr_probe_valu_rate: independent FP32 FMA chains, measured in this run"}


def pct(xs, q):
    import numpy as np
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))


def headline(hg, torch, synth, args):
    """Config: 1M Gaussians, 1920x1080, one pose (forward only)."""
    import ctypes
    log("bench: generating the 1M-Gaussian scene")
    sc, P, cam = synth.aerial_1m_1080p(0)
    # stored in spatial (Morton) order, the library's scene layout (built once
    # at load, outside the timed region): same Gaussians, same image
    scene = hg.GaussianScene.from_numpy(sc, spatial=args.layout == "spatial")
    poses = torch.from_numpy(P).cuda()
    K = hg.Intrinsics.of(cam)
    r = hg.Renderer()
    out = r.alloc_outputs(scene, 1, K)
    log("bench: first render (sizes the workspace)")
    r.render(scene, poses, K, tile=16, sort=args.sort, out=out)
    if args.tile:
        tile, feat_accum = args.tile, ("valu" if args.feat == "auto" else args.feat)
        opts = r.opts(tile=tile, sort=args.sort, feat_accum=feat_accum)
        tuned = None
    else:
        tuned = r.autotune(scene, poses, K, out, sort=args.sort)
        log("bench: autotuned", tuned)
        tile, feat_accum = tuned["tile"], tuned["feat_accum"]
        opts = r.opts(tile=0, sort=args.sort, schedule="auto")
    r.render(scene, poses, K, tile=tile, sort=args.sort, schedule=tuned["schedule"] if tuned else "grid",
             feat_accum=feat_accum, out=out)
    st = r.stats()
    log("bench: stats", st)
    for _ in range(args.warmup):
        r.render_into(scene, poses, K, out, opts)
    torch.cuda.synchronize()
    lib = r.lib
    lib.hgsr_profile_enable(r.ctx, 1)
    ms_acc = (ctypes.c_double * 6)()
    calls = (ctypes.c_int64 * 6)()
    lib.hgsr_profile_read(r.ctx, ms_acc, calls)  # reset
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        r.render_into(scene, poses, K, out, opts)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    lib.hgsr_profile_read(r.ctx, ms_acc, calls)
    lib.hgsr_profile_enable(r.ctx, 0)
    if r.check_overflow() != 0:
        raise RuntimeError("workspace overflow during the timed renders")
    eager_ms = (t1 - t0) / args.steps * 1e3
    W, H, D = cam.width, cam.height, sc.feat_dim
    stage_ms = [ms_acc[k] / max(calls[k], 1) for k in range(3)]

    # the same render captured once as a HIP graph and replayed: every kernel
    # still runs per frame; the host launch gaps between them go away
    gs = torch.cuda.Stream()
    with torch.cuda.stream(gs):
        r.render_into(scene, poses, K, out, opts, stream=gs)
    gs.synchronize()
    r.graph_begin(gs)
    r.render_into(scene, poses, K, out, opts, stream=gs)
    r.graph_end()
    r.graph_launch(args.warmup, gs)
    gs.synchronize()
    torch.cuda.synchronize()
    g0 = time.perf_counter()
    r.graph_launch(args.steps, gs)
    gs.synchronize()
    torch.cuda.synchronize()
    g1 = time.perf_counter()
    if r.check_overflow(gs) != 0:
        raise RuntimeError("workspace overflow during the replayed renders")
    ms = (g1 - g0) / args.steps * 1e3

    # the same view with bf16 feature output
    out16 = r.alloc_outputs(scene, 1, K, feat_bf16=True)
    opts16 = r.opts(tile=0 if not args.tile else tile, sort=args.sort, schedule="auto" if not args.tile else "grid",
                    feat_bf16=True, feat_accum="auto" if not args.tile else feat_accum)
    for _ in range(args.warmup):
        r.render_into(scene, poses, K, out16, opts16)
    torch.cuda.synchronize()
    b0 = time.perf_counter()
    for _ in range(args.steps):
        r.render_into(scene, poses, K, out16, opts16)
    torch.cuda.synchronize()
    b1 = time.perf_counter()
    ms16 = (b1 - b0) / args.steps * 1e3

    # blend: algorithmic bytes per launch = per-pixel outputs (rgb 12 + depth 4
    # + alpha 4 + D*4 feature + 8 saved for the backward) + one read of every
    # visible splat (48 B record + 2*D feature)
    bytes_px = 12 + 4 + 4 + 4 * D + 8
    bytes_blend = W * H * bytes_px + st["visible"] * (48 + 2 * D)
    achieved = bytes_blend / (stage_ms[2] * 1e-3) / 1e9
    traffic = measured_traffic(tile, feat_accum)
    valu = measured_valu(tile, feat_accum)
    res = dict(ms=ms, eager_ms=eager_ms, mpix=W * H / (ms * 1e-3) / 1e6, ms16=ms16, stage_ms=stage_ms, tile=tile,
               feat_accum=feat_accum, tuned=tuned, st=st, W=W, H=H, D=D, n=sc.n)
    res["roofline"] = {"kernel": f"blend_fwd (tile {tile})", "bound": "hbm", "achieved": round(achieved, 1),
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                       "traffic": traffic, "bytes_per_launch": int(bytes_blend),
                       "launch_us": round(stage_ms[2] * 1e3, 2)}
    if valu is not None:
        # the resource that bounds the blend: VALU instruction issue (counted
        # by SQ_INSTS_VALU), against the FMA issue rate measured live
        res["roofline"]["valu"] = {"instructions_per_launch": valu,
                                   "issue_frac": round(valu / (stage_ms[2] * 1e-3) / valu_rate(hg), 4),
                                   "peak": valu_peak_desc(hg)}
    res["cpu_inputs"] = (sc, P, cam)
    del out, out16, r
    return res


def refine_step_fns(hg, scene, K, lam_f=1.0, lr_rho=1e-2, lr_phi=1e-3):
    """One refinement step: render, the residual's gradient formed inside the
    blend backward (no gradient images), backward to the pose, Adam."""
    def step(r, st, opts, stream):
        r.render_into(scene, st["poses"], K, st["out"], opts, stream=stream)
        r.residual_backward(st["tgt_rgb"], st["tgt_feat"], lam_f=lam_f, loss=st["loss"], grads=st["grads"],
                            P=st["poses"].shape[0], scene=scene, stream=stream)
        hg.pose_adam(st["poses"], st["grads"]["pose"], st["m"], st["v"], st["step"], lr_rho=lr_rho, lr_phi=lr_phi,
                     stream=stream)
    return step


def refine_state(hg, torch, r, scene, K, poses, tgt_rgb, tgt_feat):
    NP = poses.shape[0]
    st = dict(poses=poses, tgt_rgb=tgt_rgb, tgt_feat=tgt_feat,
              m=torch.zeros((NP, 6), device="cuda"), v=torch.zeros((NP, 6), device="cuda"),
              step=torch.zeros(1, dtype=torch.int32, device="cuda"))
    st["out"] = r.alloc_outputs(scene, NP, K)
    st["loss"] = torch.empty(NP, device="cuda")
    st["grads"] = r.alloc_grads(scene, NP, ("pose",))
    return st


def reserve_headroom(r, NP, K, n, factor=1.5):
    """Grow the workspace past the last render's needs so that poses moved by
    the captured refinement steps still fit (nothing may allocate under
    capture)."""
    s = r.stats()
    r.reserve(NP, K.width, K.height, s["tile"], int(factor * 2 * s["visible"] / NP) + 4096,
              int(factor * s["keys"]) + 65536, n)


def fwd_bwd(hg, torch, synth, args):
    """64 candidate poses, 960x540, 1M Gaussians: batched + graph vs plain."""
    log("bench: fwd+bwd, 64 poses at 960x540")
    sc, P, cam, seed = synth.aerial_1m_64_views(0, with_seed=True)
    scene = hg.GaussianScene.from_numpy(sc, spatial=args.layout == "spatial")
    K = hg.Intrinsics.of(cam)
    NP = P.shape[0]
    rt = hg.Renderer()
    q = rt.render(scene, torch.from_numpy(seed[None]).cuda(), K)
    # the query view, one target shared by all candidate poses
    tgt_rgb, tgt_feat = q["rgb"].clone(), q["feat"].clone()
    del q, rt
    step_fn = refine_step_fns(hg, scene, K)
    s = torch.cuda.Stream()

    # batched: autotune, size, capture one step, replay
    r = hg.Renderer()
    st = refine_state(hg, torch, r, scene, K, torch.from_numpy(P).cuda(), tgt_rgb, tgt_feat)
    tuned = r.autotune(scene, st["poses"], K, st["out"], with_backward=True)
    log("bench: autotuned (64 poses)", tuned)
    opts = r.opts(tile=0, schedule="auto")
    r.render(scene, st["poses"], K, tile=0, schedule="auto", out=st["out"])
    reserve_headroom(r, NP, K, sc.n)
    # forward-only batched throughput
    with torch.cuda.stream(s):
        for _ in range(3):
            r.render_into(scene, st["poses"], K, st["out"], opts, stream=s)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(args.fb_steps):
        r.render_into(scene, st["poses"], K, st["out"], opts, stream=s)
    e1.record(s)
    s.synchronize()
    fwd_ms = e0.elapsed_time(e1) / args.fb_steps
    with torch.cuda.stream(s):
        step_fn(r, st, opts, s)
    s.synchronize()
    if r.check_overflow(s) != 0:
        raise RuntimeError("workspace overflow in the batched warm-up step")
    st["poses"].copy_(torch.from_numpy(P).cuda())
    st["m"].zero_(); st["v"].zero_(); st["step"].zero_()
    torch.cuda.synchronize()
    r.graph_begin(s)
    step_fn(r, st, opts, s)
    r.graph_end()
    r.graph_launch(2, s)
    s.synchronize()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0.record(s)
    r.graph_launch(args.fb_steps, s)
    e1.record(s)
    s.synchronize()
    t1 = time.perf_counter()
    batched_ms = e0.elapsed_time(e1) / args.fb_steps
    if r.check_overflow(s) != 0:
        raise RuntimeError("workspace overflow during the captured refinement steps")
    loss_b = st["loss"].mean().item()
    # rooflines of the step's two blends, from per-stage event times of
    # eager steps with the captured step's options
    stats = r.stats(s)
    r.profile(True)
    r.profile_read()
    with torch.cuda.stream(s):
        for _ in range(3):
            step_fn(r, st, opts, s)
    s.synchronize()
    prof = r.profile_read()
    r.profile(False)
    del st, r
    W, H, D = cam.width, cam.height, sc.feat_dim
    px = NP * W * H
    vis = stats["visible"]
    fwd_us = prof["blend"][0] / max(prof["blend"][1], 1) * 1e3
    bwd_us = prof["blend_bwd"][0] / max(prof["blend_bwd"][1], 1) * 1e3
    # forward: outputs and saved state per pixel, one read of each visible
    # splat; backward with the residual: saved state, the forward's colour
    # and feature maps and the targets per pixel, each visible splat's record
    # and feature read and its ten gradient sums written
    bytes_fwd = px * (20 + 4 * D + 8) + vis * (48 + 2 * D)
    bytes_bwd = px * (8 + 2 * (12 + 4 * D)) + vis * (48 + 2 * D + 40)
    rate = valu_rate(hg)
    kv = guarded_fields(REFINE_SQ_FILE, REFINE_SOURCES, stats["tile"], tuned["feat_accum"] if tuned else "valu")
    roof = {}
    for name, us, b, key in (("blend_fwd", fwd_us, bytes_fwd, "fwd_valu_insts_per_dispatch"),
                             ("blend_bwd", bwd_us, bytes_bwd, "bwd_valu_insts_per_dispatch")):
        ach = b / (us * 1e-6) / 1e9
        e = {"launch_us": round(us, 1), "hbm": {"bytes_per_launch": int(b), "achieved": round(ach, 1),
                                                "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                                "frac": round(ach / HBM_PEAK_GBS, 4)}}
        if kv and key in kv:
            v = int(kv[key])
            e["valu"] = {"instructions_per_launch": v, "issue_frac": round(v / (us * 1e-6) / rate, 4)}
        roof[name] = e
    step = {"ms": round(batched_ms, 3),
            "hbm_frac": round((bytes_fwd + bytes_bwd) / (batched_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4)}
    if all("valu" in roof[k] for k in roof):
        vt = roof["blend_fwd"]["valu"]["instructions_per_launch"] + roof["blend_bwd"]["valu"]["instructions_per_launch"]
        step["valu_frac"] = round(vt / (batched_ms * 1e-3) / rate, 4)
    roof["step"] = step
    roof["valu_peak"] = valu_peak_desc(hg)
    roof["visible"] = int(vis)

    # plain: one pose at a time, tile 16, grid schedule, eager
    rp = hg.Renderer()
    poses_p = torch.from_numpy(P).cuda()
    per = []
    for p in range(NP):
        stp = refine_state(hg, torch, rp, scene, K, poses_p[p:p + 1], tgt_rgb, tgt_feat)
        per.append(stp)
    # size the workspace on every pose first
    for p in range(NP):
        rp.render(scene, per[p]["poses"], K, tile=16, out=per[p]["out"])
    popts = rp.opts(tile=16, schedule="grid")
    with torch.cuda.stream(s):
        for p in range(NP):
            step_fn(rp, per[p], popts, s)
    s.synchronize()
    e0.record(s)
    with torch.cuda.stream(s):
        for _ in range(args.plain_steps):
            for p in range(NP):
                step_fn(rp, per[p], popts, s)
    e1.record(s)
    s.synchronize()
    plain_ms = e0.elapsed_time(e1) / args.plain_steps
    if rp.check_overflow(s) != 0:
        raise RuntimeError("workspace overflow in the plain loop")
    del per, rp
    return {"workload": "1M Gaussians, 64 candidate poses at 960x540 (fx 750), pose refinement step: render + "
                        "L1/feature-cosine residual + backward to the pose + Adam",
            "batched_graph_ms_per_step": round(batched_ms, 3), "plain_loop_ms_per_step": round(plain_ms, 3),
            "speedup": round(plain_ms / batched_ms, 2), "batched_fwd_ms": round(fwd_ms, 3),
            "batched_fwd_mpix_s": round(NP * W * H / (fwd_ms * 1e-3) / 1e6, 1),
            "steps_timed": args.fb_steps, "plain_steps_timed": args.plain_steps, "autotuned": tuned,
            "mean_loss_after": round(loss_b, 5), "roofline": roof}


def significance(hg, torch, synth, args):
    """Significance scoring (Sec. 3.2, Eq. 4-6): the 1M-Gaussian scene against
    64 training views at 960x540 with 32-channel FP32 maps at image
    resolution, one call per batch of 64 views."""
    import ctypes
    log("bench: significance scoring, 64 views at 960x540")
    sc, P, cam = synth.aerial_1m_64_views(0)
    scene = hg.GaussianScene.from_numpy(sc, spatial=args.layout == "spatial")
    K = hg.Intrinsics.of(cam)
    NP, W, H, D, n = P.shape[0], cam.width, cam.height, sc.feat_dim, sc.n
    poses = torch.from_numpy(P).cuda()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(3100)
    maps = torch.randn((NP, D, H, W), generator=gen, device="cuda", dtype=torch.float32)
    r = hg.Renderer()
    first = r.significance(scene, poses, K, maps, tile=16)       # sizes the workspace
    pairs = int(first["vis_count"].sum().item())
    st = r.stats()
    reserve_headroom(r, NP, K, n, factor=1.1)
    del first
    ssum = torch.zeros(n, dtype=torch.float32, device="cuda")
    cnt = torch.zeros(n, dtype=torch.int32, device="cuda")
    opts = r.opts(tile=16)
    s = torch.cuda.Stream()
    lib = r.lib
    ms_acc = (ctypes.c_double * 6)()
    calls = (ctypes.c_int64 * 6)()
    out = {}
    for layout in ("planar", "interleaved"):
        m = maps if layout == "planar" else maps.permute(0, 2, 3, 1).contiguous()
        for _ in range(2):
            r.significance_into(scene, poses, K, m, ssum, cnt, opts, layout=layout, stream=s)
        s.synchronize()
        lib.hgsr_profile_enable(r.ctx, 1)
        lib.hgsr_profile_read(r.ctx, ms_acc, calls)  # reset
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(args.sig_steps):
            r.significance_into(scene, poses, K, m, ssum, cnt, opts, layout=layout, stream=s)
        e1.record(s)
        s.synchronize()
        lib.hgsr_profile_read(r.ctx, ms_acc, calls)
        lib.hgsr_profile_enable(r.ctx, 0)
        if r.check_overflow(s) != 0:
            raise RuntimeError("workspace overflow during the timed scoring calls")
        # the profiled events sit between the stages and slow them slightly;
        # the batch time comes from an unprofiled run
        e0.record(s)
        for _ in range(args.sig_steps):
            r.significance_into(scene, poses, K, m, ssum, cnt, opts, layout=layout, stream=s)
        e1.record(s)
        s.synchronize()
        ms = e0.elapsed_time(e1) / args.sig_steps
        stage = {k: ms_acc[i] / max(calls[i], 1) for k, i in (("project", 0), ("bin_sort", 1), ("visibility_walk", 2),
                                                             ("score", 5))}
        out[layout] = dict(ms=ms, stage=stage)
        if layout == "interleaved":
            del m
    del maps
    pl, il = out["planar"], out["interleaved"]
    # scoring pass: algorithmic bytes = the P x n visibility bytes, each
    # Gaussian's mean, feature vector and running sum/count once (12 + 2D + 16),
    # and one D-float map vector per visible (view, Gaussian) pair
    score_bytes = NP * n + n * (12 + 2 * D + 16) + pairs * 4 * D
    walk_bytes = NP * n + st["keys"] * 4 + st["visible"] * 48   # flags written, list read, records read
    rl = []
    for name, lay in (("planar", pl), ("interleaved", il)):
        t = lay["stage"]["score"] * 1e-3
        rl.append({"kernel": f"score ({name} maps)", "bound": "hbm", "achieved": round(score_bytes / t / 1e9, 1),
                   "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(score_bytes / t / 1e9 / HBM_PEAK_GBS, 4),
                   "bytes_per_launch": int(score_bytes), "launch_us": round(lay["stage"]["score"] * 1e3, 2)})
    return {"workload": "1M Gaussians (32-d features) scored against 64 views at 960x540, 32-channel FP32 maps at "
                        "image resolution: visibility walk + Eq. 4 cosine at the projected mean + per-Gaussian sums",
            "ms_per_batch": round(pl["ms"], 3), "views_per_s": round(NP / (pl["ms"] * 1e-3), 1),
            "mpix_per_s": round(NP * W * H / (pl["ms"] * 1e-3) / 1e6, 1),
            "interleaved_ms_per_batch": round(il["ms"], 3),
            "stages_ms": {k: round(v, 4) for k, v in pl["stage"].items()},
            "interleaved_stages_ms": {k: round(v, 4) for k, v in il["stage"].items()},
            "visible_pairs": pairs, "records": st["visible"], "tile_entries": st["keys"],
            "walk_bytes_per_launch": int(walk_bytes), "roofline_score": rl, "steps_timed": args.sig_steps}


def matching(hg, torch, synth, args):
    """Coarse-to-fine probabilistic mutual matching (Sec. 3.4, Eq. 11) at the
    1080p sizes: 135 x 240 coarse positions (1/8), 1080 x 1920 fine maps,
    32-channel bf16 features; the render a shifted, noisy copy of the query."""
    import numpy as np
    log("bench: matching, 135x240 coarse / 1080x1920 fine")
    Hc, Wc, D = 135, 240, 32
    q_c, r_c, q_f, r_f = synth.matching_maps(D, Hc, Wc, seed=9000, shift=(11, -6), noise=0.3)
    bf = lambda b: torch.from_numpy(b.view(np.int16)).cuda().view(torch.bfloat16)
    qc, rc, qf, rf = bf(q_c), bf(r_c), bf(q_f), bf(r_f)
    r = hg.Renderer()
    s = torch.cuda.Stream()
    out = r.match(qc, rc, qf, rf, stream=s)
    s.synchronize()
    for _ in range(2):
        r.match(qc, rc, qf, rf, out=out, stream=s)
    s.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(args.match_steps):
        r.match(qc, rc, qf, rf, out=out, stream=s)
    e1.record(s)
    s.synchronize()
    ms = e0.elapsed_time(e1) / args.match_steps
    K = int(out["n_coarse"].cpu().numpy().view(np.uint32)[0])
    n_fine = int((out["fine_query"][: 64 * K] >= 0).sum().item())
    N = Hc * Wc
    # the two coarse passes each form the N x N cosine matrix on the matrix
    # cores (2 N^2 D flops per pass)
    tflops = 2 * 2 * N * N * D / (ms * 1e-3) / 1e12
    return {"workload": "coarse-to-fine probabilistic mutual matching, 135x240 coarse positions (1920x1080 / 8), "
                        "1080x1920 fine maps, 32-channel bf16 features, tau 0.1",
            "ms_per_call": round(ms, 3), "coarse_pairs_per_s": round(N * N / (ms * 1e-3), 1),
            "coarse_correspondences": K, "fine_correspondences": n_fine,
            "coarse_matrix_tflop_s": round(tflops, 1), "steps_timed": args.match_steps}


def pose_solve(hg, torch, synth, args):
    """The dense stage's pose solve (Sec. 3.4, Eq. 10) at the size of the
    1080p matching output: 640k 2D-3D correspondences (half of them outliers,
    the inliers with 0.5 px noise) seen at 1920x1080, f = 1500, from 100-300 m,
    1024 RANSAC samples of 3, 10 Gauss-Newton steps per hypothesis and 10
    refinement steps from a prior 2 m / 1.2 degrees away."""
    import numpy as np
    log("bench: pose solve, 640k correspondences, 1024 hypotheses")
    n, H = 640_000, 1024
    cam = synth.Camera(1500.0, 1500.0, 960.0, 540.0, 1920, 1080)
    rng = np.random.Generator(np.random.PCG64(4242))
    pose = synth.down_pose((10.0, -20.0), 200.0, (0.2, -0.1), 0.4).reshape(3, 4).astype(np.float64)
    u = rng.uniform(0, cam.width, n)
    v = rng.uniform(0, cam.height, n)
    d = rng.uniform(150.0, 260.0, n)
    Xc = np.stack([d * (u - cam.cx) / cam.fx, d * (v - cam.cy) / cam.fy, d], 1)
    X = (Xc - pose[:, 3]) @ pose[:, :3]
    p = np.stack([u, v], 1) + rng.normal(0.0, 0.5, (n, 2))
    out = rng.random(n) < 0.5
    p[out] = np.stack([rng.uniform(0, cam.width, out.sum()), rng.uniform(0, cam.height, out.sum())], 1)
    prior = synth.perturb_poses(pose.reshape(12).astype(np.float32), 1, 4243, 1.2, 0.7)[0]
    samples = rng.integers(0, n, (H, 3)).astype(np.int32)
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    p2d, x3d, pr, smp = t(p.astype(np.float32)), t(X.astype(np.float32)), t(prior), t(samples)
    K = hg.Intrinsics.of(cam)
    r = hg.Renderer()
    s = torch.cuda.Stream()
    res = r.pnp(p2d, x3d, K, pr, smp, stream=s)
    s.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(args.pnp_steps):
        r.pnp(p2d, x3d, K, pr, smp, stream=s)
    e1.record(s)
    s.synchronize()
    ms = e0.elapsed_time(e1) / args.pnp_steps
    got = res["pose"].cpu().numpy().reshape(3, 4).astype(np.float64)
    C = lambda P: -P[:, :3].T @ P[:, 3]
    return {"workload": "2D-3D pose solve, 640k correspondences (50% outliers, 0.5 px noise), 1920x1080 f=1500, "
                        "1024 RANSAC samples x 10 Gauss-Newton steps, 10 refinement steps, tau 2 px",
            "ms_per_call": round(ms, 3), "hypothesis_evaluations_per_s": round(n * H / (ms * 1e-3), 1),
            "inliers": int(res["n_inliers"].cpu().numpy()[0]), "true_inliers": int((~out).sum()),
            "centre_error_m": round(float(np.linalg.norm(C(got) - C(pose))), 5), "steps_timed": args.pnp_steps}


def streaming(hg, torch, synth, args):
    """Out-of-core rendering: the partitioned 8M-Gaussian scene (16 cells of
    1 km^2) kept in pinned host memory with a device budget of 6 partitions,
    a flight of 48 query views at 1920x1080 (f = 1500, 150 m) straight across
    the 4 x 4 km area, each view prepared with the next 4 as upcoming views,
    so that the next cell is uploaded while the current view renders; against
    the same views with the whole scene resident."""
    import math
    import numpy as np
    log("bench: out-of-core streaming, 8M Gaussians, 6 of 16 partitions resident, 48 views at 1080p")
    sc = synth.partitioned_8m(0)[0]
    cam = synth.Camera(1500.0, 1500.0, 960.0, 540.0, 1920, 1080)
    K = hg.Intrinsics.of(cam)
    NV, AHEAD, SLOTS = 48, 4, 6
    poses = np.stack([synth.down_pose((-1800.0 + 3600.0 * k / (NV - 1), -1500.0 + 3000.0 * k / (NV - 1)), 150.0,
                                      (0.05, 0.0), math.pi / 5) for k in range(NV)])
    dev_poses = torch.from_numpy(poses).cuda()
    s = torch.cuda.Stream()
    host = hg.spatial_layout(sc)[0] if args.layout == "spatial" else sc
    pc = hg.PartitionCache(host, SLOTS)
    r = hg.Renderer()
    out = None

    def run(timed):
        nonlocal out
        ups = pre = 0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for k in range(NV):
            desc = pc.prepare(poses[k:k + 1], K, ahead=poses[k + 1:k + 1 + AHEAD], stream=s)
            ups += pc.stats["uploads"]
            pre += pc.stats["prefetched"]
            out = r.render(desc, dev_poses[k:k + 1], K, out=out, check_overflow=not timed, stream=s)
        e1.record(s)
        s.synchronize()
        return e0.elapsed_time(e1) / NV, ups, pre

    run(False)                      # sizes the renderer's workspace
    pc.evict_all()
    t0 = pc.stats["total_bytes"]
    ms, ups, pre = run(True)
    if r.check_overflow(s) != 0:
        raise RuntimeError("workspace overflow in the streamed flight")
    gb = (pc.stats["total_bytes"] - t0) / 1e9
    # one cold upload (the 4 partitions of views 10..14), timed on the host (prepare + wait)
    pc.evict_all()
    s.synchronize()
    t = time.perf_counter()
    pc.prepare(poses[10:15], K, stream=s)
    cold = pc.stats
    s.synchronize()
    t_up = time.perf_counter() - t
    dev_bytes = pc.stats["device_bytes"]
    pc.close()
    # the same flight with the whole scene resident
    full = hg.GaussianScene.from_numpy(sc, spatial=args.layout == "spatial")
    r2 = hg.Renderer()
    o2 = r2.render(full, dev_poses[:1], K)
    for k in range(NV):
        r2.render(full, dev_poses[k:k + 1], K, out=o2, stream=s)
    s.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for k in range(NV):
        r2.render(full, dev_poses[k:k + 1], K, out=o2, check_overflow=False, stream=s)
    e1.record(s)
    s.synchronize()
    ms_res = e0.elapsed_time(e1) / NV
    scene_bytes = sum(getattr(sc, f).nbytes for f in ("means", "log_scales", "quats", "opacities", "sh", "feat"))
    del full
    return {"workload": "8M Gaussians in 16 partitions over 4x4 km (SH0, 32-d features) in pinned host memory, "
                        f"{SLOTS} partitions on the device, 48 views at 1920x1080 f=1500 from 150 m crossing the area, "
                        f"each view prepared with the next {AHEAD} as upcoming views",
            "ms_per_view_streamed": round(ms, 3), "ms_per_view_resident": round(ms_res, 3),
            "uploads": ups, "uploads_ahead": pre, "uploaded_gb": round(gb, 3),
            "device_budget_gb": round(dev_bytes / 1e9, 3), "scene_gb": round(scene_bytes / 1e9, 3),
            "cold_upload": {"partitions": cold["uploads"], "gb": round(cold["bytes_uploaded"] / 1e9, 3),
                            "ms": round(t_up * 1e3, 2),
                            "gb_per_s": round(cold["bytes_uploaded"] / 1e9 / t_up, 1)}}


def refine_levels(hg, torch, r, scene, n, poses, truth, cams, lr_rho, lr_phi, iters, s):
    """Coarse-to-fine refinement of `poses` (device, updated in place) against
    targets rendered at `truth`: per level, the step captured once as a HIP
    graph and replayed `iters` times.  Returns per-level records and the
    per-step latencies."""
    NQ = truth.shape[0]
    lat, per_level = [], []
    for lvl, cam in enumerate(cams):
        K = hg.Intrinsics.of(cam)
        step_fn = refine_step_fns(hg, scene, K, lr_rho=lr_rho, lr_phi=lr_phi)
        tgt = r.render(scene, torch.from_numpy(truth).cuda(), K)
        tgt_rgb, tgt_feat = tgt["rgb"], tgt["feat"]
        del tgt
        st = refine_state(hg, torch, r, scene, K, poses, tgt_rgb, tgt_feat)
        tuned = r.autotune(scene, poses, K, st["out"], with_backward=True)
        opts = r.opts(tile=0, schedule="auto")
        r.render(scene, poses, K, tile=0, schedule="auto", out=st["out"])
        reserve_headroom(r, NQ, K, n)
        keep = poses.clone()
        with torch.cuda.stream(s):
            step_fn(r, st, opts, s)  # warm-up (then undone)
        s.synchronize()
        poses.copy_(keep)
        st["m"].zero_(); st["v"].zero_(); st["step"].zero_()
        torch.cuda.synchronize()
        r.graph_begin(s)
        step_fn(r, st, opts, s)
        r.graph_end()
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(iters + 1)]
        losses = []
        ev[0].record(s)
        for k in range(iters):
            r.graph_launch(1, s)
            ev[k + 1].record(s)
            if k == 0:
                losses.append(st["loss"].clone())
        s.synchronize()
        if r.check_overflow(s) != 0:
            raise RuntimeError(f"workspace overflow at level {lvl}")
        ll = [ev[k].elapsed_time(ev[k + 1]) for k in range(iters)]
        lat += ll
        per_level.append({"size": f"{cam.width}x{cam.height}", "tile": tuned["tile"], "schedule": tuned["schedule"],
                          "p50_ms": round(pct(ll, 50), 3), "p99_ms": round(pct(ll, 99), 3),
                          "loss_first": round(losses[0].mean().item(), 5),
                          "loss_last": round(st["loss"].mean().item(), 5)})
        log("bench: level", per_level[-1])
        del st, tgt_rgb, tgt_feat
    return per_level, lat


def centre_errors(poses, truth):
    import numpy as np
    NQ = truth.shape[0]
    T = poses.astype(np.float64).reshape(NQ, 3, 4)
    tr = truth.astype(np.float64).reshape(NQ, 3, 4)
    cpos = lambda A: -np.einsum("qji,qj->qi", A[:, :, :3], A[:, :, 3])
    return np.linalg.norm(cpos(T) - cpos(tr), axis=1)


def partitioned(hg, torch, synth, args):
    """8M Gaussians in 16 partitions, 16 query poses, 3 levels x 20 steps."""
    import numpy as np
    log("bench: partitioned scene (8M Gaussians) generation")
    sc, truth, start, cams = synth.partitioned_8m(0)
    scene = hg.GaussianScene.from_numpy(sc, spatial=args.layout == "spatial")
    s = torch.cuda.Stream()
    r = hg.Renderer()
    poses = torch.from_numpy(start).cuda()
    torch.cuda.synchronize()
    free0, total = torch.cuda.mem_get_info()
    res0 = torch.cuda.memory_reserved()
    torch.cuda.reset_peak_memory_stats()
    t_start = time.perf_counter()
    per_level, lat = refine_levels(hg, torch, r, scene, sc.n, poses, truth, cams, args.part_lr_rho,
                                   args.part_lr_phi, args.part_iters, s)
    wall = time.perf_counter() - t_start
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    res1 = torch.cuda.memory_reserved()
    peak = torch.cuda.max_memory_allocated()
    e0 = centre_errors(start, truth)
    e1 = centre_errors(poses.cpu().numpy(), truth)
    # the same loop from offsets inside the photometric basin of these
    # scenes (random per-Gaussian colour and feature decorrelate within about
    # a metre on the ground)
    near = np.stack([synth.perturb_poses(truth[q], 1, 5600 + q, args.part_near_t, args.part_near_rot)[0]
                     for q in range(truth.shape[0])]).astype(np.float32)
    pn = torch.from_numpy(near).cuda()
    conv_levels, _ = refine_levels(hg, torch, r, scene, sc.n, pn, truth, cams, args.part_near_lr_rho,
                                   args.part_near_lr_phi, args.part_iters, s)
    n0 = centre_errors(near, truth)
    n1 = centre_errors(pn.cpu().numpy(), truth)
    del r
    return {"workload": "8M Gaussians in 16 partitions over 4x4 km, 16 query poses, 3 levels (480x270, 960x540, "
                        f"1920x1080) x {args.part_iters} captured fwd+bwd refinement steps",
            "step_p50_ms": round(pct(lat, 50), 3), "step_p99_ms": round(pct(lat, 99), 3), "levels": per_level,
            "device_mem_in_use_gb": round((total - free1) / 1e9, 2),
            "device_mem_before_gb": round((total - free0) / 1e9, 2),
            "library_workspace_gb": round(((free0 - free1) - (res1 - res0)) / 1e9, 2),
            "torch_peak_allocated_gb": round(peak / 1e9, 2),
            "camera_centre_error_m": {
                "start_median": round(float(np.median(e0)), 3), "final_median": round(float(np.median(e1)), 3),
                "note": "start offsets N(0,5 m), N(0,3 deg) lie outside the photometric basin of these synthetic "
                        "scenes; the timed loop does not localise from there"},
            "convergence_from_near": {
                "start_offsets": f"N(0,{args.part_near_t} m), N(0,{args.part_near_rot} deg)",
                "lr_rho_m": args.part_near_lr_rho, "lr_phi_rad": args.part_near_lr_phi,
                "start_median_m": round(float(np.median(n0)), 3), "final_median_m": round(float(np.median(n1)), 3),
                "improved": int(np.sum(n1 < n0)), "of": int(len(n0)), "levels": conv_levels},
            "wall_s": round(wall, 2)}


def cpu_baseline(synth, sc, P, cam, budget_s):
    """The FP64 oracle on the host cores: frames of the headline scene at the
    headline pose and nearby poses until `budget_s` seconds have passed."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    poses = np.concatenate([P[:1], synth.perturb_poses(P[0], 63, 77, 2.0, 1.0)])
    frames, tested, blended = 0, 0, 0
    c0 = time.perf_counter()
    while frames < len(poses):
        ref = oracle.render(sc, poses[frames], cam, tile=16, margin=0)
        tested += ref["stats"]["tested"]
        blended += ref["stats"]["blended"]
        frames += 1
        if time.perf_counter() - c0 >= budget_s:
            break
    c1 = time.perf_counter()
    W, H = cam.width, cam.height
    return {"value": round(frames * W * H / (c1 - c0) / 1e6, 4), "unit": "Mpix/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": f"{frames} full 1920x1080 frames of the headline scene (headline pose, then nearby poses), "
                      "FP64 tiled oracle", "seconds": round(c1 - c0, 3),
            "oracle_tested_pairs_per_frame": int(tested / frames), "oracle_blended_pairs_per_frame":
                int(blended / frames)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="time budget of the CPU oracle sample")
    ap.add_argument("--tile", type=int, default=0, help="0: autotuned")
    ap.add_argument("--sort", default="bucket")
    ap.add_argument("--feat", choices=["auto", "valu", "mfma"], default="auto",
                    help="feature accumulation with a fixed --tile (auto: the VALU)")
    ap.add_argument("--layout", choices=["spatial", "given"], default="spatial",
                    help="scene storage order: spatial (Morton, the library's layout) or as generated")
    ap.add_argument("--no-fwd-bwd", action="store_true")
    ap.add_argument("--no-partitioned", action="store_true")
    ap.add_argument("--no-significance", action="store_true")
    ap.add_argument("--no-matching", action="store_true")
    ap.add_argument("--match-steps", type=int, default=10)
    ap.add_argument("--no-pose-solve", action="store_true")
    ap.add_argument("--no-streaming", action="store_true")
    ap.add_argument("--pnp-steps", type=int, default=10)
    ap.add_argument("--sig-steps", type=int, default=10)
    ap.add_argument("--fb-steps", type=int, default=20)
    ap.add_argument("--plain-steps", type=int, default=3)
    ap.add_argument("--part-iters", type=int, default=20)
    ap.add_argument("--part-lr-rho", type=float, default=0.3, help="Adam step (m) of the partitioned refinement")
    ap.add_argument("--part-lr-phi", type=float, default=4e-3, help="Adam step (rad) of the partitioned refinement")
    ap.add_argument("--part-near-t", type=float, default=1.0, help="start offset (m) of the convergence run")
    ap.add_argument("--part-near-rot", type=float, default=0.5, help="start offset (deg) of the convergence run")
    ap.add_argument("--part-near-lr-rho", type=float, default=0.05, help="Adam step (m) of the convergence run")
    ap.add_argument("--part-near-lr-phi", type=float, default=1e-3, help="Adam step (rad) of the convergence run")
    ap.add_argument("--only", choices=["headline", "fwd_bwd", "partitioned", "significance", "matching", "pose_solve", "streaming"],
                    default=None,
                    help="run one section and print its result alone (for profiling)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="run only a plain 1 GiB device copy (5 launches), to scale HBM counters")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = 1 << 28  # 1 GiB of float32
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": 4 * n, "copy_bytes_written": 4 * n, "launches": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the renderer shards by pose with "
              "no collective; run one process per GPU instead)", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2507_15683_amd as hg
    import synth

    if args.only == "fwd_bwd":
        print(json.dumps({"fwd_bwd": fwd_bwd(hg, torch, synth, args)}), flush=True)
        return
    if args.only == "partitioned":
        print(json.dumps({"partitioned": partitioned(hg, torch, synth, args)}), flush=True)
        return
    if args.only == "significance":
        print(json.dumps({"significance": significance(hg, torch, synth, args)}), flush=True)
        return
    if args.only == "matching":
        print(json.dumps({"matching": matching(hg, torch, synth, args)}), flush=True)
        return
    if args.only == "streaming":
        print(json.dumps({"streaming": streaming(hg, torch, synth, args)}), flush=True)
        return
    if args.only == "pose_solve":
        print(json.dumps({"pose_solve": pose_solve(hg, torch, synth, args)}), flush=True)
        return
    if args.only == "headline":
        args.no_fwd_bwd = args.no_partitioned = args.no_significance = args.no_matching = True
        args.no_pose_solve = args.no_streaming = args.no_cpu = True
    h = headline(hg, torch, synth, args)
    result = {
        "metric": "rendered Mpix/s at 1080p/1M Gaussians",
        "value": round(h["mpix"], 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(h["ms"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1M Gaussians (SH3, 32-d bf16 features), 1920x1080, one pose, forward render "
                               f"(tile {h['tile']}, {args.sort} sort)", "layout": args.layout,
                   "gaussians": h["n"], "width": h["W"],
                   "height": h["H"], "feat_dim": h["D"], "visible": h["st"]["visible"], "keys": h["st"]["keys"],
                   "autotuned": h["tuned"]},
        "stages_ms": {"project": round(h["stage_ms"][0], 4), "bin_sort": round(h["stage_ms"][1], 4),
                      "blend": round(h["stage_ms"][2], 4)},
        "timing": "K replays of the render captured as one HIP graph, between two device synchronisations",
        "eager": {"ms_per_step": round(h["eager_ms"], 4),
                  "value": round(h["W"] * h["H"] / (h["eager_ms"] * 1e-3) / 1e6, 2), "unit": "Mpix/s"},
        "bf16_feature_out": {"ms_per_step": round(h["ms16"], 4),
                             "value": round(h["W"] * h["H"] / (h["ms16"] * 1e-3) / 1e6, 2), "unit": "Mpix/s"},
        "roofline": h["roofline"],
    }
    torch.cuda.empty_cache()
    if not args.no_fwd_bwd:
        result["fwd_bwd"] = fwd_bwd(hg, torch, synth, args)
        torch.cuda.empty_cache()
    if not args.no_partitioned:
        result["partitioned"] = partitioned(hg, torch, synth, args)
        torch.cuda.empty_cache()
    if not args.no_significance:
        result["significance"] = significance(hg, torch, synth, args)
        torch.cuda.empty_cache()
    if not args.no_matching:
        result["matching"] = matching(hg, torch, synth, args)
        torch.cuda.empty_cache()
    if not args.no_pose_solve:
        result["pose_solve"] = pose_solve(hg, torch, synth, args)
        torch.cuda.empty_cache()
    if not args.no_streaming:
        result["streaming"] = streaming(hg, torch, synth, args)
        torch.cuda.empty_cache()
    if not args.no_cpu:
        log("bench: timing the CPU oracle")
        sc, P, cam = h["cpu_inputs"]
        result["cpu_baseline"] = cpu_baseline(synth, sc, P, cam, args.cpu_seconds)
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
