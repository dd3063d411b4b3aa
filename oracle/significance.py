"""Significance scoring with the render-gradient visibility check -- FP64
oracle, TEST INFRASTRUCTURE ONLY (the test suite, the smoke check and the
benchmark's CPU-baseline leg use it; the HIP library never does).

Sec. 3.2 scores every Gaussian by how well its feature agrees with the 2D
features of the training views in which it is visible.  For view i with
world->camera pose (R, t), intrinsics K and image size W x H:

  visibility (the render-mask algorithm of Sec. 3.2, "render gradient
  visibility check with projection filtering"):
    M^r[j]   render the view, back-propagate the summed RGB: j is visible when
             its mean receives a nonzero gradient, i.e. when j is blended
             with weight alpha T > 0 at one pixel at least (the oracle's walk
             decides this; see `contrib` in the package);
    (U, V)   homogeneous mean -> camera frame -> divide by the depth -> K;
    M^i[j]   0 <= U < W and 0 <= V < H;
    M        M^i and M^r.
  Eq. 4   S(G_i)_j = F_j . F^t(U, V) / (|F_j| |F^t(U, V)|)  for every j in M;
  Eq. 5   S(G)_j   = sum over the views of S(G_i)_j;
  Eq. 6   S(g_j)   = S(G)_j / M_j, M_j the number of views in which j is
                     visible.

Readings (the paper is silent on them): F^t is a D x Hf x Wf map covering the
image, and (U, V) reads cell (floor(U Wf / W), floor(V Hf / H)) -- the cell
that contains the point, no interpolation; the cosine's denominator gets
+1e-8, as in the refinement residual; S(g_j) = 0 when M_j = 0.

A GPU evaluates these decisions in FP32.  `exempt` marks the (view,
Gaussian) pairs that FP32 rounding may legitimately decide the other way:
visibility decided only at fragile pixels (see `contrib`), or a projected
mean within `edge_px` of the image border or of a cell border.
"""
from __future__ import annotations

import numpy as np

from . import contrib

COS_EPS = 1e-8
EDGE_PX = 1e-3


def bf16_to_f64(bits: np.ndarray) -> np.ndarray:
    """bfloat16 bit patterns -> exact float64 values."""
    b = np.ascontiguousarray(bits, dtype=np.uint16).astype(np.uint32) << 16
    return b.view(np.float32).astype(np.float64)


def project_means(means: np.ndarray, pose, cam):
    """The algorithm's projection of Gaussian means: returns U, V and the
    camera-frame depth (U, V are NaN where the depth is not positive)."""
    X = np.asarray(means, dtype=np.float64)
    Tm = np.asarray(pose, dtype=np.float64).reshape(3, 4)
    homo = np.concatenate([X, np.ones((X.shape[0], 1))], axis=1)
    xc = (Tm @ homo.T).T
    d = xc[:, 2]
    safe = np.where(d > 0.0, d, np.nan)
    xh = xc / safe[:, None]
    K = np.array([[cam.fx, 0.0, cam.cx], [0.0, cam.fy, cam.cy], [0.0, 0.0, 1.0]])
    uv = (K @ xh.T).T
    return uv[:, 0], uv[:, 1], d


def sample_cosines(feat64: np.ndarray, U: np.ndarray, V: np.ndarray, fmap: np.ndarray, width: int, height: int,
                   edge_px: float = EDGE_PX):
    """Eq. 4 for every Gaussian of one view, before the visibility mask.

    feat64 (N, D) Gaussian features; fmap (D, Hf, Wf).  Returns (cos, inside,
    near_edge): cos is NaN where (U, V) is outside the image; near_edge marks
    points within edge_px of the image border or of a cell border."""
    D, Hf, Wf = fmap.shape
    with np.errstate(invalid="ignore"):
        inside = (U >= 0.0) & (U < width) & (V >= 0.0) & (V < height)
    inside &= np.isfinite(U) & np.isfinite(V)
    n = U.shape[0]
    cos = np.full(n, np.nan)
    near = np.zeros(n, dtype=bool)
    idx = np.nonzero(inside)[0]
    u, v = U[idx], V[idx]
    sx, sy = Wf / width, Hf / height
    cx = np.floor(u * sx).astype(np.int64)
    cy = np.floor(v * sy).astype(np.int64)
    ft = fmap[:, cy, cx].T.astype(np.float64)          # (m, D)
    fg = feat64[idx]
    dot = (fg * ft).sum(axis=1)
    na = np.sqrt((fg * fg).sum(axis=1))
    nb = np.sqrt((ft * ft).sum(axis=1))
    cos[idx] = dot / (na * nb + COS_EPS)
    fu, fv = u * sx, v * sy
    du = np.abs(fu - np.round(fu)) / sx
    dv = np.abs(fv - np.round(fv)) / sy
    near[idx] = (du < edge_px) | (dv < edge_px)
    # within edge_px of the image border, inside or outside it
    fin = np.isfinite(U) & np.isfinite(V)
    Uf, Vf = np.where(fin, U, -1e30), np.where(fin, V, -1e30)
    dist_x = np.minimum(np.abs(Uf), np.abs(width - Uf))
    dist_y = np.minimum(np.abs(Vf), np.abs(height - Vf))
    near |= fin & (((dist_x < edge_px) & (Vf > -edge_px) & (Vf < height + edge_px)) |
                   ((dist_y < edge_px) & (Uf > -edge_px) & (Uf < width + edge_px)))
    return cos, inside, near


def view_terms(scene, pose, cam, fmap: np.ndarray, tile: int = 16, near: float = 0.2, edge_px: float = EDGE_PX):
    """One view's visibility M (N,), Eq. 4 cosines (NaN where not in the
    image), and the pairs FP32 may decide differently (`exempt`)."""
    c, robust, touched = contrib(scene, pose, cam, tile=tile, near=near)
    U, V, _ = project_means(scene.means, pose, cam)
    feat64 = bf16_to_f64(scene.feat)
    cos, inside, near_edge = sample_cosines(feat64, U, V, fmap, cam.width, cam.height, edge_px)
    visible = inside & c
    uncertain = (~robust) & touched
    exempt = uncertain | near_edge
    return dict(visible=visible, cos=cos, exempt=exempt, U=U, V=V, contrib=c)


def significance(scene, poses, cam, maps: np.ndarray, tile: int = 16, near: float = 0.2, edge_px: float = EDGE_PX):
    """Eq. 4-6 over the views `poses` (P, 12) with feature maps (P, D, Hf, Wf).

    Returns score_sum (N,) (Eq. 5), count (N,) (the visibility counts M_j),
    score (N,) (Eq. 6), visible (P, N), exempt (P, N)."""
    poses = np.asarray(poses, dtype=np.float64).reshape(-1, 12)
    n = scene.means.shape[0]
    total = np.zeros(n)
    count = np.zeros(n, dtype=np.int64)
    vis = np.zeros((poses.shape[0], n), dtype=bool)
    exempt = np.zeros((poses.shape[0], n), dtype=bool)
    for i, pose in enumerate(poses):
        t = view_terms(scene, pose, cam, maps[i], tile, near, edge_px)
        m = t["visible"]
        total[m] += t["cos"][m]
        count[m] += 1
        vis[i] = m
        exempt[i] = t["exempt"]
    score = np.where(count > 0, total / np.maximum(count, 1), 0.0)
    return dict(score_sum=total, count=count, score=score, visible=vis, exempt=exempt)
