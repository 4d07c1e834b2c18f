"""Pins of the oracle's Adam pose step: the first bias-corrected step moves
every coordinate by the learning rate in the direction of the gradient, the
rotation update is scipy's rotation-vector exponential, and the step keeps
rotations orthonormal."""

import numpy as np
from scipy.spatial.transform import Rotation

from oracle.refine import adam_pose_step, rotvec_exp
from workloads import random_poses


def test_first_adam_step_has_the_learning_rate_as_length():
    rng = np.random.default_rng(0)
    P = random_poses(rng, 5, 0.8, 0.02)
    g = rng.normal(0, 100, (5, 8))
    Q, S = adam_pose_step(P, g, np.zeros((5, 12)), 1, lr_t=1e-3, lr_r=1e-2, eps=0.0)
    np.testing.assert_allclose(Q[:, :3, 3] - P[:, :3, 3], 1e-3 * np.sign(g[:, :3]), rtol=1e-12)
    for n in range(5):
        dR = Q[n, :3, :3] @ P[n, :3, :3].T
        np.testing.assert_allclose(Rotation.from_matrix(dR).as_rotvec(), 1e-2 * np.sign(g[n, 3:6]), rtol=1e-9)
    np.testing.assert_allclose(S[:, :6], 0.1 * g[:, :6])


def test_rotation_exponential_matches_scipy_and_stays_orthonormal():
    rng = np.random.default_rng(1)
    for _ in range(20):
        w = rng.normal(0, 1, 3)
        R = rotvec_exp(w)
        np.testing.assert_allclose(R, Rotation.from_rotvec(w).as_matrix(), atol=1e-14)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
