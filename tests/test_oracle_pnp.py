"""Pins of the oracle's pose solve (Eq. 10 by RANSAC over given 3-point
samples, truncated-quadratic refinement), back-projection and Algorithm 2's
consistency check, against finite differences, exact synthetic geometry and
closed forms.  CPU only."""
import math

import numpy as np
from scipy.spatial.transform import Rotation

from synth import Camera
from oracle import pnp
from oracle.se3 import exp_se3

K = Camera(800.0, 780.0, 480.0, 270.0, 960, 540)


def _pose(seed, alt=150.0):
    rng = np.random.default_rng(seed)
    R = Rotation.from_rotvec([math.pi, 0, 0]).as_matrix() @ Rotation.from_rotvec(rng.normal(0, 0.1, 3)).as_matrix()
    C = np.array([rng.normal(0, 5), rng.normal(0, 5), alt])
    T = np.eye(4)
    T[:3, :3] = R.T
    T[:3, 3] = -R.T @ C
    return T


def _scene(T, n, seed, noise=0.0, outliers=0.0):
    """World points seen by T (on a bumpy ground), their pixels with noise
    and a fraction of random outlier pixels."""
    rng = np.random.default_rng(seed)
    u = rng.uniform(20, K.width - 20, n)
    v = rng.uniform(20, K.height - 20, n)
    d = rng.uniform(120, 180, n)
    Xc = np.stack([d * (u - K.cx) / K.fx, d * (v - K.cy) / K.fy, d], 1)
    X = (Xc - T[:3, 3]) @ T[:3, :3]
    p = np.stack([u, v], 1) + rng.normal(0, noise, (n, 2))
    out = rng.random(n) < outliers
    p[out] = np.stack([rng.uniform(0, K.width, out.sum()), rng.uniform(0, K.height, out.sum())], 1)
    return p, X, out


def test_jacobian_matches_finite_differences():
    T = _pose(1)
    p, X, _ = _scene(T, 20, 2)
    r, J, _ = pnp.residual_jacobian(T, K, X, p)
    h = 1e-6
    for k in range(6):
        e = np.zeros(6); e[k] = h
        rp, _, _ = pnp.residual_jacobian(exp_se3(e) @ T, K, X, p)
        rm, _, _ = pnp.residual_jacobian(exp_se3(-e) @ T, K, X, p)
        np.testing.assert_allclose((rp - rm) / (2 * h), J[:, :, k], rtol=1e-5, atol=1e-6)


def test_three_points_converge_to_the_exact_pose():
    """A noise-free minimal sample from a prior 2 m / 2 degrees away
    reprojects exactly after the Gauss-Newton steps and is the true pose."""
    T = _pose(3)
    p, X, _ = _scene(T, 3, 4)
    T0 = exp_se3(np.r_[np.random.default_rng(5).normal(0, 1.2, 3), np.radians([1.2, -1.0, 1.5])]) @ T
    r = pnp.pnp_ransac(p, X, K, T0[:3, :].reshape(12), [[0, 1, 2]], tau=1.0, gn_iters=10, refine_iters=0)
    assert r["valid"][0] and r["counts"][0] == 3
    np.testing.assert_allclose(r["hyps"][0], T[:3, :], atol=1e-7)


def test_exact_data_with_outliers():
    """0.5 px noise and 30 % outliers: the pose is recovered to a few cm and
    hundredths of a degree, the inlier set is the true one up to outliers
    that land within tau by chance."""
    T = _pose(7)
    p, X, out = _scene(T, 600, 8, noise=0.5, outliers=0.3)
    T0 = exp_se3(np.r_[1.5, -1.0, 2.0, np.radians([1.5, -2.0, 1.0])]) @ T
    samples = np.random.default_rng(9).integers(0, 600, (64, 3))
    r = pnp.pnp_ransac(p, X, K, T0[:3, :].reshape(12), samples, tau=2.0)
    dt = np.linalg.norm(r["pose"][:, 3] - T[:3, 3])
    dR = pnp.rotation_angle_deg(r["pose"].reshape(12), T[:3, :].reshape(12))
    assert dt < 0.05 and dR < 0.05, (dt, dR)
    assert (r["inliers"] & ~out).sum() >= 0.97 * (~out).sum()
    assert (r["inliers"] & out).sum() <= 0.02 * out.sum()
    # the refined pose is the least-squares optimum over its inlier set
    Ts = T.copy()
    for _ in range(30):
        Ts = pnp.gn_step(Ts, K, X[r["inliers"]], p[r["inliers"]])
    np.testing.assert_allclose(r["pose"], Ts[:3, :], atol=1e-7)
    assert r["counts"][r["best"]] == r["counts"][r["valid"]].max()


def test_degenerate_sample_is_invalid():
    """Three identical correspondences give a singular normal matrix."""
    T = _pose(11)
    p, X, _ = _scene(T, 5, 12)
    r = pnp.pnp_ransac(p, X, K, T[:3, :].reshape(12), [[1, 1, 1], [0, 2, 4]], tau=1.0)
    assert not r["valid"][0] and r["valid"][1] and r["best"] == 1


def test_backprojection_round_trip():
    """Points projected to pixel centres with their camera z written into a
    depth map come back exactly."""
    T = _pose(13)
    rng = np.random.default_rng(14)
    x = rng.integers(0, K.width, 50); y = rng.integers(0, K.height, 50)
    pix = y * K.width + x
    d = rng.uniform(100, 200, 50)
    depth = np.zeros((K.height, K.width))
    depth[y, x] = d
    X = pnp.backproject(depth, T[:3, :].reshape(12), K, pix)
    Xc, uv = pnp.project(T, K, X)
    np.testing.assert_allclose(Xc[:, 2], d, rtol=1e-12)
    np.testing.assert_allclose(uv, np.stack([x + 0.5, y + 0.5], 1), atol=1e-9)


def test_consistency_check_closed_forms():
    """The angle of R1 R2^T: a turn of theta about any axis gives theta; equal
    rotations give 0 (the clamp keeps arccos defined); a 25 degree jump
    between two consecutive results makes the sequence unreliable."""
    T = _pose(15)
    for theta in (0.5, 10.0, 19.9, 90.0, 179.0):
        Rz = Rotation.from_rotvec(np.radians(theta) * np.array([0.3, -0.5, 0.81]) /
                                  np.linalg.norm([0.3, -0.5, 0.81])).as_matrix()
        T2 = T.copy(); T2[:3, :3] = Rz @ T[:3, :3]
        assert abs(pnp.rotation_angle_deg(T2[:3, :].reshape(12), T[:3, :].reshape(12)) - theta) < 1e-6
    assert pnp.rotation_angle_deg(T[:3, :].reshape(12), T[:3, :].reshape(12)) == 0.0
    small = [exp_se3(np.r_[0, 0, 0, 0.01 * k, 0, 0]) @ T for k in range(3)]
    assert pnp.consistent([s[:3, :] for s in small])
    jump = small[:2] + [exp_se3(np.r_[0, 0, 0, 0, 0, np.radians(25)]) @ small[1]]
    assert not pnp.consistent([s[:3, :] for s in jump])


def test_refinement_retakes_the_inlier_set_until_it_is_a_fixed_point():
    """Eq. 10's truncated quadratic min(e^2, tau^2) is minimised by
    Gauss-Newton on the inlier set re-taken before each step.  With 1 px
    noise and only 6 samples the best hypothesis fits a noisy triple, so its
    inlier set differs from the converged one.  The returned set is the
    returned pose's own set (errors < tau), one more re-taken Gauss-Newton
    step leaves the pose where it is (the pose is the least-squares optimum
    of exactly the set it selects), and the truncated cost does not exceed
    the best hypothesis'.  Refining on the hypothesis' set alone ends at the
    optimum of a different set, which the next re-taken step moves by
    centimetres."""
    tau = 2.0
    for seed in (0, 1, 3, 5):
        T = _pose(20 + seed)
        p, X, _ = _scene(T, 400, 21 + seed, noise=1.0, outliers=0.3)
        T0 = exp_se3(np.r_[1.5, -1.0, 2.0, np.radians([1.5, -2.0, 1.0])]) @ T
        samples = np.random.default_rng(22 + seed).integers(0, 400, (6, 3))
        r = pnp.pnp_ransac(p, X, K, T0[:3, :].reshape(12), samples, tau=tau)
        hyp_inl = r["hyp_err"][r["best"]] < tau
        assert (hyp_inl != r["inliers"]).sum() >= 30, seed   # the case the check is about
        Tr = np.eye(4)
        Tr[:3, :] = r["pose"]
        e = pnp.errors(Tr, K, X, p)
        np.testing.assert_array_equal(r["inliers"], e < tau)
        Tn = pnp.gn_step(Tr, K, X[r["inliers"]], p[r["inliers"]])
        assert np.abs(Tn - Tr).max() < 1e-8, seed
        Th = np.eye(4)
        Th[:3, :] = r["hyps"][r["best"]]
        cost = lambda M: np.minimum(pnp.errors(M, K, X, p) ** 2, tau * tau).sum()
        assert cost(Tr) <= cost(Th), seed


def test_score_counts_errors_below_tau_in_front_of_the_camera():
    """The RANSAC score of the exact pose: correspondences with reprojection
    error below tau and positive depth.  Three exact, three 1.5 px off
    (counted at tau = 2), three 3 px off (not counted), one world point
    behind the camera on the ray of its pixel (error 0, not counted), two
    more exact: 8.  Two identical samples tie and the lower index wins."""
    T = _pose(7)
    p, X, _ = _scene(T, 12, 8)
    p[3:6] += [1.5, 0.0]
    p[6:9] += [0.0, 3.0]
    Xc9 = X[9] @ T[:3, :3].T + T[:3, 3]
    X[9] = (-Xc9 - T[:3, 3]) @ T[:3, :3]  # same pixel, negative depth
    r = pnp.pnp_ransac(p, X, K, T[:3, :].reshape(12), [[0, 1, 2], [0, 1, 2]], tau=2.0, gn_iters=3,
                       refine_iters=0)
    assert list(r["counts"]) == [8, 8] and r["best"] == 0
    want = np.array([1] * 6 + [0] * 4 + [1] * 2, dtype=bool)
    assert np.array_equal(r["inliers"], want)
    e = r["hyp_err"][0]
    np.testing.assert_allclose(e[3:6], 1.5, atol=1e-6)
    np.testing.assert_allclose(e[6:9], 3.0, atol=1e-6)
    assert np.isinf(e[9])
