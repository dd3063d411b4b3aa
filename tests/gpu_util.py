"""Helpers shared by the GPU tests: scene upload and element-wise parity
against the oracle with its fragile-pixel exemption."""
from __future__ import annotations

import sys

import numpy as np

COLOR_TOL = 1e-4   # absolute, colour / alpha / features
DEPTH_RTOL = 1e-4  # relative, depth


def log(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def to_np(t):
    import torch
    if t.dtype == torch.bfloat16:
        t = t.float()
    return t.detach().cpu().numpy().astype(np.float64)


def parity(out, ref, p=0, feat_tol=COLOR_TOL, max_fragile_frac=0.02, label=""):
    """Compare pose p of a GPU render with an oracle render element by
    element, except at the oracle's fragile pixels (a gate, stop or depth-order
    decision within the FP32 error bound).  Returns a summary dict."""
    frag = ref["fragile"]
    ok = ~frag
    rgb = to_np(out["rgb"][p])
    alpha = to_np(out["alpha"][p])
    depth = to_np(out["depth"][p])
    d_rgb = np.abs(rgb - ref["rgb"]).max(axis=0)
    d_a = np.abs(alpha - ref["alpha"])
    d_d = np.abs(depth - ref["depth"]) / np.maximum(np.abs(ref["depth"]), 1e-30)
    d_d[(ref["alpha"] == 0) & (alpha == 0)] = 0.0
    bad = ok & ((d_rgb > COLOR_TOL) | (d_a > COLOR_TOL) | (d_d > DEPTH_RTOL))
    d_f = None
    if out.get("feat") is not None and ref.get("feat") is not None:
        f = to_np(out["feat"][p])
        d_f = np.abs(f - ref["feat"]).max(axis=0)
        bad |= ok & (d_f > feat_tol)
    summary = dict(label=label, pixels=int(frag.size), fragile=int(frag.sum()), bad=int(bad.sum()),
                   max_rgb=float(d_rgb[ok].max(initial=0)), max_alpha=float(d_a[ok].max(initial=0)),
                   max_depth_rel=float(d_d[ok].max(initial=0)),
                   max_feat=float(d_f[ok].max(initial=0)) if d_f is not None else None)
    log("parity", summary)
    if bad.any():
        ys, xs = np.nonzero(bad)
        log("first bad pixels", list(zip(ys[:8].tolist(), xs[:8].tolist())))
    assert not bad.any(), summary
    assert frag.mean() <= max_fragile_frac, summary
    return summary
