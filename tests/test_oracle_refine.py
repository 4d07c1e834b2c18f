"""Pins of the oracle's Adam pose step: the first bias-corrected step moves
every coordinate by the learning rate in the direction of the gradient, the
rotation update is scipy's rotation-vector exponential, and the step keeps
rotations orthonormal."""

import numpy as np
from scipy.spatial.transform import Rotation

from oracle.refine import adam_pose_step, left_jacobian, retract, retract_grad, rotvec_exp
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


def _smooth_f(P, a, B):
    """A smooth function of a pose: a . t + trace(B R)."""
    return float(a @ P[:3, 3] + np.trace(B @ P[:3, :3]))


def test_retract_grad_matches_finite_differences_through_the_retraction():
    rng = np.random.default_rng(41)
    a, B = rng.normal(size=3), rng.normal(size=(3, 3))
    base = np.eye(4)
    base[:3, :3] = rotvec_exp(rng.normal(size=3))
    base[:3, 3] = rng.normal(size=3)
    for scale in (0.0, 0.3, 2.5):
        xi = rng.normal(size=(1, 6)) * scale
        P = retract(base, xi)[0]
        # tangent gradient at the retracted pose: perturb by exp([d]x) R, t + d
        g = np.zeros(6)
        e = 1e-6
        for k in range(6):
            d = np.zeros(6)
            d[k] = e
            fp = _smooth_f(retract(P, d[None])[0], a, B)
            fm = _smooth_f(retract(P, -d[None])[0], a, B)
            g[k] = (fp - fm) / (2 * e)
        want = np.zeros(6)
        for k in range(6):
            d = np.zeros(6)
            d[k] = e
            want[k] = (_smooth_f(retract(base, xi + d)[0], a, B) - _smooth_f(retract(base, xi - d)[0], a, B)) / (2 * e)
        got = retract_grad(xi, g[None], np.array([1.0]))[0]
        np.testing.assert_allclose(got, want, rtol=1e-6, atol=1e-7)
        np.testing.assert_allclose(retract_grad(xi, g[None], np.array([-2.0]))[0], -2.0 * want, rtol=1e-6, atol=2e-7)


def test_left_jacobian_closed_forms():
    assert np.array_equal(left_jacobian(np.zeros(3)), np.eye(3))
    rng = np.random.default_rng(42)
    w = rng.normal(size=3)
    # J(w) w = w, and J(w) of a half turn about z in closed form
    np.testing.assert_allclose(left_jacobian(w) @ w, w, rtol=1e-12)
    Jz = left_jacobian(np.array([0.0, 0.0, np.pi]))
    np.testing.assert_allclose(Jz, [[0, -2 / np.pi, 0], [2 / np.pi, 0, 0], [0, 0, 1]], atol=1e-12)
