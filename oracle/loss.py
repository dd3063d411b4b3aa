"""Refinement residual and finite-difference gradients -- oracle side, FP64.

Residual of one pose (the dense stage compares a rendered package with the
query, Sec. 3.4; the form used here is an L1 photometric term plus a feature
cosine term):
    L = 1/(H W) * sum_p [ sum_c |rgb_c - rgb*_c| + lam_f (1 - cos(F_p, F*_p)) ]
    cos(a, b) = a.b / (|a| |b| + 1e-8),   d|x|/dx = sign(x), sign(0) = 0.
For a batch of poses the residual is the sum of the per-pose residuals.

Finite differences use the frozen-decision renderer of the oracle: the set
and order of Gaussians blended at each pixel are taken from a render at the
reference point and held fixed, which is the smooth piece of the renderer the
analytic gradient differentiates.
"""
from __future__ import annotations

import numpy as np

from . import render, render_frozen
from .se3 import left_perturb

COS_EPS = 1e-8


def residual(rgb, feat, rgb_t, feat_t, lam_f=1.0) -> float:
    H, W = rgb.shape[1:]
    l1 = np.abs(rgb - rgb_t).sum()
    if feat is None or lam_f == 0.0:
        return float(l1 / (H * W))
    dot = (feat * feat_t).sum(axis=0)
    na = np.sqrt((feat * feat).sum(axis=0))
    nb = np.sqrt((feat_t * feat_t).sum(axis=0))
    cos = dot / (na * nb + COS_EPS)
    return float((l1 + lam_f * (1.0 - cos).sum()) / (H * W))


def residual_frozen_signs(rgb_ref, rgb_t, feat_t, lam_f=1.0):
    """The residual with the sign pattern of |rgb - rgb*| taken at a reference
    render and held fixed: the smooth piece of the L1 term that contains the
    reference point (what its gradient sign(rgb - rgb*) differentiates).
    Returns loss_fn(out) for finite differences."""
    sgn = np.sign(rgb_ref - rgb_t)

    def loss(out):
        H, W = out["rgb"].shape[1:]
        l1 = (sgn * (out["rgb"] - rgb_t)).sum()
        if out.get("feat") is None or lam_f == 0.0:
            return float(l1 / (H * W))
        f = out["feat"]
        dot = (f * feat_t).sum(axis=0)
        na = np.sqrt((f * f).sum(axis=0))
        nb = np.sqrt((feat_t * feat_t).sum(axis=0))
        return float((l1 + lam_f * (1.0 - dot / (na * nb + COS_EPS)).sum()) / (H * W))

    return loss


def residual_grad(rgb, feat, rgb_t, feat_t, lam_f=1.0):
    """Closed-form dL/d rgb (3,H,W) and dL/d feat (D,H,W)."""
    H, W = rgb.shape[1:]
    s = 1.0 / (H * W)
    g_rgb = np.sign(rgb - rgb_t) * s
    if feat is None or lam_f == 0.0:
        return g_rgb, None
    dot = (feat * feat_t).sum(axis=0)
    na = np.sqrt((feat * feat).sum(axis=0))
    nb = np.sqrt((feat_t * feat_t).sum(axis=0))
    n = na * nb + COS_EPS
    unit = np.divide(feat, na, out=np.zeros_like(feat), where=na > 0)
    dcos = feat_t / n - (dot * nb / (n * n)) * unit
    return g_rgb, -lam_f * s * dcos


def linear_functional(out, weights) -> float:
    """L = sum over channels of <w_k, out_k> for any subset of outputs (used to
    check the depth and alpha gradients, which the residual does not touch)."""
    return float(sum((out[k] * w).sum() for k, w in weights.items()))


def _param64(scene, name):
    if name == "feat":
        return (np.asarray(scene.feat, dtype=np.uint32) << 16).view(np.float32).astype(np.float64)
    return np.asarray(getattr(scene, name), dtype=np.float64)


def fd_gradients(scene, pose, cam, loss_fn, h=1e-4, gauss_ids=(), params=("means", "opacities"), tile=16,
                 list_cap=512, bg=(0.0, 0.0, 0.0)):
    """Central differences of loss_fn(frozen render) with respect to the 6
    left-perturbation pose coordinates (rho, phi) and, for each id in
    gauss_ids, every component of each named Gaussian parameter.  Returns
    (g_pose (6,), {param: (k, ...) array}, reference render)."""
    ref = render(scene, pose, cam, mode="tiled", tile=tile, bg=bg, want_lists=True, list_cap=list_cap)
    lists, counts = ref["lists"], ref["nblend"]
    base = {p: _param64(scene, p) for p in params}

    def L(pose12, overrides=None):
        out = render_frozen(scene, pose12, cam, lists, counts, bg=bg, overrides=overrides)
        return loss_fn(out)

    g_pose = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        g_pose[k] = (L(left_perturb(pose, e)) - L(left_perturb(pose, -e))) / (2 * h)
    ids = list(gauss_ids)
    out = {}
    for p in params:
        arr = base[p]
        per = arr[0].shape if arr.ndim > 1 else ()
        g = np.zeros((len(ids),) + per)
        for j, i in enumerate(ids):
            for comp in np.ndindex(*per) if per else [()]:
                plus = arr.copy()
                minus = arr.copy()
                plus[(i,) + comp] += h
                minus[(i,) + comp] -= h
                g[(j,) + comp] = (L(pose, {p: plus}) - L(pose, {p: minus})) / (2 * h)
        out[p] = g
    return g_pose, out, ref


def fd_tangent_gradient(scene, pose, xi, cam, loss_fn, h=1e-4, tile=16, list_cap=512, bg=(0.0, 0.0, 0.0)):
    """Central differences of loss_fn(frozen render at Exp(xi) T) with
    respect to the six components of xi itself (not of a perturbation at
    the retracted pose).  Returns (g_xi (6,), reference render at Exp(xi) T)."""
    xi = np.asarray(xi, dtype=np.float64)
    base = left_perturb(pose, xi)
    ref = render(scene, base, cam, mode="tiled", tile=tile, bg=bg, want_lists=True, list_cap=list_cap)
    lists, counts = ref["lists"], ref["nblend"]
    g = np.zeros(6)
    for k in range(6):
        e = np.zeros(6)
        e[k] = h
        lp = loss_fn(render_frozen(scene, left_perturb(pose, xi + e), cam, lists, counts, bg=bg))
        lm = loss_fn(render_frozen(scene, left_perturb(pose, xi - e), cam, lists, counts, bg=bg))
        g[k] = (lp - lm) / (2 * h)
    return g, ref
