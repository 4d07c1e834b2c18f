"""Gradient refinement of poses, stated plainly for the oracle.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

Adam (Kingma and Ba, ICLR 2015) ascends logL on the pose tangent: with
g = d logL/d(dt, dw), m = b1 m + (1-b1) g, v = b2 v + (1-b2) g^2, and the
bias-corrected step s = lr (m/(1-b1^k)) / (sqrt(v/(1-b2^k)) + eps), the
pose moves by t <- t + s_t and R <- exp([s_w]x) R (the same tangent
convention as the pose adjoint).
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
