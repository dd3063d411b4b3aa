"""2D-3D pose solve with RANSAC and pose consistency verification -- FP64
oracle, TEST INFRASTRUCTURE ONLY (the test suite, the smoke check and the
benchmark's CPU-baseline leg use it; the HIP library never does).

The dense stage turns fine correspondences into a pose (Sec. 3.4): the
rendered depth lifts each matched rendered pixel to a world point, and
Eq. 10 solves
    {R*, t*}, I* = argmin_{R,t} sum_{i in I} rho(|p_i - pi(K [R|t] g_i)|, tau)
with a robust loss rho of threshold tau (reprojection error in pixels),
pi([x, y, z]) = [x/z, y/z], by PnP with RANSAC; Algorithm 2 then checks the
poses of n rounds for consistency.

Readings (the paper names the solver family but not its steps):
  * back-projection: world point = R_r^T (d K^-1 [u, v, 1]^T - t_r) for the
    rendered pixel's centre (u, v) = (x + 1/2, y + 1/2), its rendered depth
    d (the normalised expected camera z) and the render pose [R_r | t_r];
  * RANSAC hypotheses: each from a minimal sample of 3 correspondences
    (indices given, so that every implementation draws the same samples),
    solved by `gn_iters` Gauss-Newton steps on the 6 reprojection residuals
    from the prior pose T0 (the render pose), with the left update
    T <- Exp(delta) T, delta = -(J^T J)^-1 J^T r; a sample whose normal
    matrix is singular is invalid;
  * score: the number of correspondences with positive depth and
    reprojection error below tau (ties: lowest hypothesis index);
  * rho is the truncated quadratic min(e^2, tau^2): from the best hypothesis,
    `refine_iters` Gauss-Newton steps on the current inlier set, which is
    re-taken before every step; the returned inlier set is the final pose's;
  * Algorithm 2's loop compares T_1 with T_2 on every pass; read as every
    consecutive pair (T_i, T_i+1), "any two" dense results: a pair whose
    rotation differs by more than tau_deg makes the result unreliable.
"""
from __future__ import annotations

import numpy as np

from .se3 import exp_se3


def backproject(depth: np.ndarray, pose12, K, pix: np.ndarray) -> np.ndarray:
    """World points of rendered pixels `pix` (row-major indices into the
    H x W depth map) under the render pose."""
    H, W = depth.shape
    y, x = np.divmod(np.asarray(pix, dtype=np.int64), W)
    u, v = x + 0.5, y + 0.5
    d = depth[y, x].astype(np.float64)
    Xc = np.stack([d * (u - K.cx) / K.fx, d * (v - K.cy) / K.fy, d], axis=1)
    P = np.asarray(pose12, dtype=np.float64).reshape(3, 4)
    R, t = P[:, :3], P[:, 3]
    return (Xc - t) @ R          # R^T (Xc - t) row by row


def project(T: np.ndarray, K, X: np.ndarray):
    """Camera points and pixel coordinates of world points X under T (4x4)."""
    Xc = X @ T[:3, :3].T + T[:3, 3]
    z = Xc[:, 2]
    with np.errstate(divide="ignore", invalid="ignore"):
        u = K.fx * Xc[:, 0] / z + K.cx
        v = K.fy * Xc[:, 1] / z + K.cy
    return Xc, np.stack([u, v], axis=1)


def residual_jacobian(T: np.ndarray, K, X: np.ndarray, p: np.ndarray):
    """Residuals r = pi(K T X) - p (n x 2) and their Jacobians (n x 2 x 6)
    with respect to the left perturbation Exp(xi) T, xi = (rho, phi):
    dXc/dxi = [I, -[Xc]x]."""
    Xc, uv = project(T, K, X)
    r = uv - p
    x, y, z = Xc[:, 0], Xc[:, 1], Xc[:, 2]
    dpi = np.zeros((len(X), 2, 3))
    dpi[:, 0, 0] = K.fx / z
    dpi[:, 0, 2] = -K.fx * x / z**2
    dpi[:, 1, 1] = K.fy / z
    dpi[:, 1, 2] = -K.fy * y / z**2
    dX = np.zeros((len(X), 3, 6))
    dX[:, :, :3] = np.eye(3)
    # -[Xc]x
    dX[:, 0, 4], dX[:, 0, 5] = z, -y
    dX[:, 1, 3], dX[:, 1, 5] = -z, x
    dX[:, 2, 3], dX[:, 2, 4] = y, -x
    return r, np.einsum("nij,njk->nik", dpi, dX), z


def gn_step(T, K, X, p):
    """One Gauss-Newton step on the given correspondences; None if J^T J is
    singular."""
    r, J, _ = residual_jacobian(T, K, X, p)
    Jf = J.reshape(-1, 6)
    A = Jf.T @ Jf
    b = Jf.T @ r.reshape(-1)
    if np.linalg.matrix_rank(A, tol=1e-12 * max(np.abs(A).max(), 1e-300)) < 6:
        return None
    delta = -np.linalg.solve(A, b)
    return exp_se3(delta) @ T


def errors(T, K, X, p):
    Xc, uv = project(T, K, X)
    e = np.sqrt(((uv - p) ** 2).sum(axis=1))
    return np.where(Xc[:, 2] > 0, e, np.inf)


def pnp_ransac(p2d, X3d, K, pose0, samples, tau=2.0, gn_iters=10, refine_iters=10):
    """Eq. 10 by RANSAC over the given 3-point samples (H x 3 indices), then
    truncated-quadratic Gauss-Newton on the inliers.  Returns dict(pose (3x4),
    best, counts (H,), valid (H,), hyps (H, 3, 4), inliers (bool n),
    hyp_err (H, n): every hypothesis' reprojection errors)."""
    p = np.asarray(p2d, dtype=np.float64)
    X = np.asarray(X3d, dtype=np.float64)
    T0 = np.eye(4)
    T0[:3, :] = np.asarray(pose0, dtype=np.float64).reshape(3, 4)
    H = len(samples)
    counts = np.zeros(H, dtype=np.int64)
    valid = np.zeros(H, dtype=bool)
    hyps = np.zeros((H, 3, 4))
    hyp_err = np.full((H, len(p)), np.inf)
    for h, s in enumerate(np.asarray(samples, dtype=np.int64)):
        T = T0.copy()
        ok = True
        for _ in range(gn_iters):
            Tn = gn_step(T, K, X[s], p[s])
            if Tn is None:
                ok = False
                break
            T = Tn
        if not ok:
            continue
        valid[h] = True
        hyps[h] = T[:3, :]
        e = errors(T, K, X, p)
        hyp_err[h] = e
        counts[h] = int((e < tau).sum())
    if not valid.any():          # no hypothesis: the prior pose, no refinement
        inl = errors(T0, K, X, p) < tau
        return dict(pose=T0[:3, :].copy(), best=-1, counts=np.where(valid, counts, -1), valid=valid, hyps=hyps,
                    inliers=inl, hyp_err=hyp_err)
    best = int(np.argmax(np.where(valid, counts, -1)))
    T = np.eye(4)
    T[:3, :] = hyps[best]
    for _ in range(refine_iters):
        inl = errors(T, K, X, p) < tau
        Tn = gn_step(T, K, X[inl], p[inl])
        if Tn is None:
            break
        T = Tn
    inl = errors(T, K, X, p) < tau
    return dict(pose=T[:3, :].copy(), best=best, counts=np.where(valid, counts, -1), valid=valid, hyps=hyps,
                inliers=inl, hyp_err=hyp_err)


def rotation_angle_deg(T1, T2) -> float:
    """Algorithm 2's pose difference: angle of R1 R2^T in degrees, the trace
    clamped to [-1, 3] against rounding."""
    R1 = np.asarray(T1, dtype=np.float64).reshape(3, 4)[:, :3]
    R2 = np.asarray(T2, dtype=np.float64).reshape(3, 4)[:, :3]
    tr = min(3.0, max(np.trace(R1 @ R2.T), -1.0))
    return float(np.degrees(np.arccos((tr - 1.0) / 2.0)))


def consistent(poses, tau_deg=20.0) -> bool:
    """Algorithm 2 over consecutive pairs of the n dense results."""
    return all(rotation_angle_deg(poses[i], poses[i + 1]) <= tau_deg for i in range(len(poses) - 1))
