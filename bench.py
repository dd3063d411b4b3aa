"""Benchmark of the splat rasterizer on one MI355X.

Workload (default): 1,000,000 Gaussians (900k on a 1x1 km heightfield plus
2,000 box buildings, SH degree 3, 32-d bf16 features), one 1920x1080 view,
fx = 1500, 100-300 m altitude, tilt <= 30 deg.  A step renders that view
(projection, tile binning, sort, blend: RGB + depth + alpha + 32-channel FP32
feature map).  Prints one JSON line.

python bench.py [--gpus 1] [--steps 50] [--warmup 10] [--no-cpu]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--tile", type=int, default=16)
    ap.add_argument("--sort", default="bucket")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported (the renderer shards by pose with "
              "no collective; run one process per GPU instead)", file=sys.stderr)
        sys.exit(2)

    import ctypes

    import numpy as np
    import torch

    import paper_2507_15683_amd as hg
    import synth

    def log(*a):
        print(*a, file=sys.stderr, flush=True)

    log("bench: generating the 1M-Gaussian scene")
    sc, P, cam = synth.config2(0)
    scene = hg.GaussianScene.from_numpy(sc)
    poses = torch.from_numpy(P).cuda()
    K = hg.Intrinsics.of(cam)
    r = hg.Renderer()
    out = r.alloc_outputs(scene, 1, K)
    log("bench: first render (sizes the workspace)")
    r.render(scene, poses, K, tile=args.tile, sort=args.sort, out=out)
    st = r.stats()
    log("bench: stats", st)
    opts = r.opts(tile=args.tile, sort=args.sort)
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
    assert r.check_overflow() == 0
    ms = (t1 - t0) / args.steps * 1e3
    W, H, D = cam.width, cam.height, sc.feat_dim
    mpix = W * H / (ms * 1e-3) / 1e6
    stage_ms = [ms_acc[k] / max(calls[k], 1) for k in range(3)]
    # blend: algorithmic bytes per launch = per-pixel outputs (rgb 12 + depth 4
    # + alpha 4 + D*4 feature + 8 saved for the backward) + one read of every
    # visible splat (48 B record + 2*D feature)
    bytes_px = 12 + 4 + 4 + 4 * D + 8
    bytes_blend = W * H * bytes_px + st["visible"] * (48 + 2 * D)
    achieved = bytes_blend / (stage_ms[2] * 1e-3) / 1e9
    result = {
        "metric": "rendered Mpix/s at 1080p/1M Gaussians",
        "value": round(mpix, 2),
        "unit": "Mpix/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "1M Gaussians (SH3, 32-d bf16 features), 1920x1080, one pose, tile "
                               f"{args.tile}, {args.sort} sort", "gaussians": sc.n, "width": W, "height": H,
                   "feat_dim": D, "visible": st["visible"], "keys": st["keys"]},
        "stages_ms": {"project": round(stage_ms[0], 4), "bin_sort": round(stage_ms[1], 4),
                      "blend": round(stage_ms[2], 4)},
        "roofline": {"kernel": "blend_fwd", "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                     "bytes_per_launch": int(bytes_blend)},
    }
    if not args.no_cpu:
        import oracle
        oracle.build(force=False)
        log("bench: timing the CPU oracle on the same 1080p view")
        c0 = time.perf_counter()
        ref = oracle.render(sc, P[0], cam, tile=16, margin=0)
        c1 = time.perf_counter()
        result["cpu_baseline"] = {"value": round(W * H / (c1 - c0) / 1e6, 4), "unit": "Mpix/s",
                                  "cores": oracle.num_threads(), "kind": "oracle",
                                  "sample": "one full 1920x1080 frame of the same scene and pose (FP64, tiled)",
                                  "seconds": round(c1 - c0, 3)}
        result["config"]["oracle_tested_pairs"] = ref["stats"]["tested"]
        result["config"]["oracle_blended_pairs"] = ref["stats"]["blended"]
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
