"""Gradient refinement of poses, stated plainly for the oracle.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

Adam (Kingma and Ba, ICLR 2015) ascends logL on the pose tangent: with
g = d logL/d(dt, dw), m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, and the
bias-corrected step s = lr (m/(1-b1^k)) / (sqrt(v/(1-b2^k)) + eps), the
pose moves by t <- t + s_t and R <- exp([s_w]x) R (the same tangent
convention as the pose adjoint).

Retraction: xi = (dt, w) moves a base pose to (exp([w]x) R, t + dt).  Since
exp([w + e]x) = exp([J(w) e]x) exp([w]x) to first order in e, with the left
Jacobian J(w) = I + (1 - cos th)/th^2 [w]x + (th - sin th)/th^3 [w]x^2
(th = |w|), a tangent gradient g_w at the retracted pose becomes J(w)^T g_w
with respect to w.
"""

from __future__ import annotations

import numpy as np


def rotvec_exp(w: np.ndarray) -> np.ndarray:
    """Rotation matrix of the rotation vector w (Rodrigues' formula)."""
    th = float(np.linalg.norm(w))
    if th == 0.0:
        return np.eye(3)
    k = w / th
    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
    return np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * (K @ K)


def adam_pose_step(poses, grad, state, it, lr_t, lr_r, b1=0.9, b2=0.999, eps=1e-8):
    """One step for poses [N,4,4], grad [N,>=6], state [N,12] (m, v); returns updated copies."""
    P = np.array(poses, dtype=np.float64, copy=True)
    S = np.array(state, dtype=np.float64, copy=True)
    g = np.asarray(grad, dtype=np.float64)[:, :6]
    m, v = S[:, :6], S[:, 6:]
    m[:] = b1 * m + (1 - b1) * g
    v[:] = b2 * v + (1 - b2) * g * g
    lr = np.array([lr_t] * 3 + [lr_r] * 3)
    s = lr * (m / (1 - b1**it)) / (np.sqrt(v / (1 - b2**it)) + eps)
    for n in range(P.shape[0]):
        P[n, :3, 3] += s[n, :3]
        P[n, :3, :3] = rotvec_exp(s[n, 3:]) @ P[n, :3, :3]
    return P, S


def left_jacobian(w: np.ndarray) -> np.ndarray:
    """J(w) of the rotation exponential (identity at w = 0)."""
    w = np.asarray(w, dtype=np.float64)
    th = float(np.linalg.norm(w))
    if th == 0.0:
        return np.eye(3)
    K = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]])
    return np.eye(3) + (1 - np.cos(th)) / th**2 * K + (th - np.sin(th)) / th**3 * (K @ K)


def retract(base, xi):
    """Poses [N,4,4] = (exp([w_n]x) R_b, t_b + dt_n); base [N,4,4] or [4,4]."""
    xi = np.asarray(xi, dtype=np.float64)
    B = np.asarray(base, dtype=np.float64)
    B = np.broadcast_to(B, (xi.shape[0], 4, 4)) if B.ndim == 2 or B.shape[0] == 1 else B
    out = np.array(B, dtype=np.float64, copy=True)
    for n in range(xi.shape[0]):
        out[n, :3, :3] = rotvec_exp(xi[n, 3:]) @ B[n, :3, :3]
        out[n, :3, 3] = B[n, :3, 3] + xi[n, :3]
    return out


def retract_grad(xi, g_tan, dlogL=None):
    """d/d xi [N,6] of sum_n dlogL_n f_n(retract(base, xi)_n) given the tangent
    gradients g_tan [N,>=6] = (d/d dt, d/d dw) of f_n at the retracted poses."""
    xi = np.asarray(xi, dtype=np.float64)
    g = np.asarray(g_tan, dtype=np.float64)
    u = np.ones(xi.shape[0]) if dlogL is None else np.asarray(dlogL, dtype=np.float64)
    out = np.empty((xi.shape[0], 6))
    for n in range(xi.shape[0]):
        out[n, :3] = u[n] * g[n, :3]
        out[n, 3:] = u[n] * (left_jacobian(xi[n, 3:]).T @ g[n, 3:6])
    return out
