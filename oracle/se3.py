"""SE(3) pose tangent used by the pose gradient -- oracle side, FP64, TEST
INFRASTRUCTURE ONLY.

The pose gradient is taken with respect to a left perturbation of the
world->camera pose, T <- Exp(xi) T, xi = (rho, phi) with translation first.
Exp is the closed form of the matrix exponential of the 4x4 twist
[[phi^, rho], [0, 0]] (Rodrigues for the rotation, V rho for the translation).
A loss of the poses Exp(xi) T has d/dxi = J_l(xi)^T dL/d(delta), J_l the left
Jacobian, Exp(xi + dxi) = Exp(J_l(xi) dxi) Exp(xi) to first order; by
definition J_l(xi) = sum_{n >= 0} ad(xi)^n / (n + 1)! with the adjoint
ad(rho, phi) = [[phi^, rho^], [0, phi^]].
"""
from __future__ import annotations

import numpy as np


def hat(w):
    return np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])


def exp_se3(xi) -> np.ndarray:
    """4x4 matrix Exp(xi) for xi = (rho, phi)."""
    xi = np.asarray(xi, dtype=np.float64)
    rho, phi = xi[:3], xi[3:]
    th = float(np.linalg.norm(phi))
    K = hat(phi)
    if th < 1e-12:
        R = np.eye(3) + K
        V = np.eye(3) + 0.5 * K
    else:
        a = np.sin(th) / th
        b = (1.0 - np.cos(th)) / th**2
        c = (th - np.sin(th)) / th**3
        R = np.eye(3) + a * K + b * K @ K
        V = np.eye(3) + b * K + c * K @ K
    T = np.eye(4)
    T[:3, :3] = R
    T[:3, 3] = V @ rho
    return T


def left_perturb(pose12, xi) -> np.ndarray:
    """Return Exp(xi) * T as 12 doubles, T given as a row-major [R|t]."""
    T = np.eye(4)
    T[:3, :] = np.asarray(pose12, dtype=np.float64).reshape(3, 4)
    return (exp_se3(xi) @ T)[:3, :].reshape(12)


def ad_se3(xi) -> np.ndarray:
    """6x6 adjoint of the twist (rho, phi): [[phi^, rho^], [0, phi^]]."""
    xi = np.asarray(xi, dtype=np.float64)
    A = np.zeros((6, 6))
    A[:3, :3] = hat(xi[3:])
    A[:3, 3:] = hat(xi[:3])
    A[3:, 3:] = hat(xi[3:])
    return A


def left_jacobian(xi, terms: int = 60) -> np.ndarray:
    """J_l(xi) as its defining series sum_n ad^n / (n + 1)!."""
    A = ad_se3(xi)
    M = np.eye(6)
    J = np.eye(6)
    for n in range(1, terms):
        M = M @ A / (n + 1)
        J = J + M
    return J
