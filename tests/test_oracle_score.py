"""Pins of the oracle's windowed likelihood (eq. (1), truncated to a window
as in Sec. III-B's scoring strategy) against closed forms, invariants and
scipy's Gaussian density."""

import numpy as np
import pytest
from scipy.spatial.transform import Rotation
from scipy.stats import multivariate_normal

import oracle
from oracle import tiny


def _random_images(rng, H, W, N, frac_obs=0.8, frac_rend=0.6, spread=0.01):
    base = np.stack(np.meshgrid(np.linspace(-0.1, 0.1, W), np.linspace(-0.08, 0.08, H)), -1)
    z = 0.7 + 0.02 * rng.standard_normal((H, W))
    obs = np.concatenate([base * z[..., None], z[..., None]], -1)
    obs[rng.random((H, W)) > frac_obs] = 0.0
    rend = np.repeat(np.concatenate([base * z[..., None], z[..., None]], -1)[None], N, 0)
    rend = rend + spread * rng.standard_normal(rend.shape)
    rend[rng.random((N, H, W)) > frac_rend] = 0.0
    return obs, rend


def test_outlier_only_likelihood_is_uniform_density():
    # p_out = 1: every valid pixel has density 1/V, whatever is rendered
    rng = np.random.default_rng(0)
    obs, rend = _random_images(rng, 9, 11, 3)
    V = 2.5
    logL, l1 = oracle.score(obs, rend, sigma=0.004, p_out=1.0, V=V, window=5)
    n_valid = int((obs[..., 2] > 0).sum())
    np.testing.assert_allclose(logL, -n_valid * np.log(V), rtol=1e-13)
    np.testing.assert_allclose(l1, n_valid * np.log(V), rtol=1e-13)


def test_rigid_transform_of_both_images_leaves_score_unchanged():
    rng = np.random.default_rng(1)
    obs, rend = _random_images(rng, 10, 12, 4)
    R = Rotation.from_rotvec([0.1, -0.2, 0.05]).as_matrix()
    t = np.array([0.05, -0.03, 0.4])

    def move(x):
        y = x @ R.T + t
        return np.where(x[..., 2:3] > 0, y, 0.0)

    a, _ = oracle.score(obs, rend, 0.006, 0.05, 1.0, 5)
    b, _ = oracle.score(move(obs), move(rend), 0.006, 0.05, 1.0, 5)
    np.testing.assert_allclose(a, b, rtol=1e-12)


def test_full_window_equals_untruncated_eq1_with_scipy_density():
    rng = np.random.default_rng(2)
    H, W = 6, 5
    obs, rend = _random_images(rng, H, W, 2, spread=0.004)
    r = 2 * max(H, W) - 1
    logL, _ = oracle.score(obs, rend, 0.005, 0.1, 1.7, r)
    for n in range(2):
        ref = tiny.loglik_untruncated(obs, rend[n], 0.005, 0.1, V=1.7)
        np.testing.assert_allclose(logL[n], ref, rtol=1e-11)


def test_single_pixel_closed_form():
    q_obs = np.array([[[0.01, -0.02, 0.8]]])
    q_r = np.array([[[0.012, -0.017, 0.805]]])
    sigma, p, V = 0.004, 0.2, 3.0
    logL, _ = oracle.score(q_obs, q_r[None], sigma, p, V, 1)
    dens = multivariate_normal(mean=q_r[0, 0], cov=sigma**2 * np.eye(3)).pdf(q_obs[0, 0])
    np.testing.assert_allclose(logL[0], np.log(p / V + (1 - p) * dens), rtol=1e-13)


@pytest.mark.parametrize("window", [1, 3, 5, 7])
def test_window_reaches_exactly_h_pixels(window):
    h = (window - 1) // 2
    H, W = 9, 13
    obs = np.zeros((H, W, 3))
    obs[4, 6] = [0.0, 0.0, 0.8]
    sigma, p, V = 0.003, 0.01, 1.0
    M = H * W
    peak = np.log(p / V + (1 - p) / M * (2 * np.pi * sigma**2) ** -1.5)
    for dr, dc in [(0, h), (h, 0), (-h, -h), (h, -h), (0, h + 1), (h + 1, 0), (-h - 1, 0)]:
        rend = np.zeros((1, H, W, 3))
        rend[0, 4 + dr, 6 + dc] = obs[4, 6]  # same point, another pixel
        logL, _ = oracle.score(obs, rend, sigma, p, V, window)
        inside = max(abs(dr), abs(dc)) <= h
        np.testing.assert_allclose(logL[0], peak if inside else np.log(p / V), rtol=1e-13)


def test_pixels_without_rendered_neighbours_contribute_log_outlier_density():
    rng = np.random.default_rng(4)
    H, W = 12, 14
    obs, rend = _random_images(rng, H, W, 1, frac_obs=1.0, frac_rend=1.0)
    rend[:, 4:, :] = 0.0
    rend[:, :, 5:] = 0.0  # rendered points only in the top-left 4x5 block
    p, V, r = 0.03, 1.3, 3
    full, _ = oracle.score(obs, rend, 0.005, p, V, r)
    near = obs.copy()
    near[6:, :] = 0.0
    near[:, 7:] = 0.0  # keep only observed pixels whose window can touch the block
    part, _ = oracle.score(near, rend, 0.005, p, V, r, M=H * W)
    n_far = int((obs[..., 2] > 0).sum() - (near[..., 2] > 0).sum())
    np.testing.assert_allclose(full - part, n_far * np.log(p / V), rtol=1e-12)


def test_counters_pairs_and_observed():
    rng = np.random.default_rng(6)
    obs, rend = _random_images(rng, 7, 8, 2)
    _, _, cnt = oracle.score(obs, rend, 0.005, 0.1, 1.0, 3, counters=True)
    assert np.all(cnt[:, oracle.C_OBS] == (obs[..., 2] > 0).sum())
    assert np.all(cnt[:, oracle.C_RPIX] == (rend[..., 2] > 0).reshape(2, -1).sum(1))
    # brute count of pairs
    for n in range(2):
        pairs = 0
        for i in range(7):
            for j in range(8):
                if obs[i, j, 2] <= 0:
                    continue
                blk = rend[n, max(0, i - 1):i + 2, max(0, j - 1):j + 2, 2]
                pairs += int((blk > 0).sum())
        assert cnt[n, oracle.C_PAIR] == pairs
