"""Pins of the oracle's normalise-and-sample step and the coarse-to-fine
proposal (Sec. III-B): Philox known answers, exact weights for equal
logits, Gumbel-max frequencies against softmax, grid layout against numpy,
and the proposal density of a partition schedule."""

import copy
import itertools
import os

import numpy as np
import pytest
from scipy.stats import chisquare

import oracle
from oracle.c2f import c2f, final_cell_volume, partition_schedule
from workloads import GridSpec, make_config, pose_matrix

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        v = [int(x, 16) for x in line.split()]
        rows.append((v[0:4], v[4:6], tuple(v[6:10])))
    return rows


@pytest.mark.parametrize("row", range(3))
def test_philox_known_answers(row):
    ctr, key, out = _kat()[row]
    assert oracle.philox(ctr, key) == out


def test_uniforms_are_odd_multiples_of_2_pow_minus_24():
    for i in range(2000):
        u = oracle.uniform(12345, i, 7, 3, 0, i % 4)
        m = u * 2**24
        assert 0 < u < 1 and m == int(m) and int(m) % 2 == 1


def test_equal_logits_give_uniform_weights_and_weights_sum_to_one():
    w, idx, logw = oracle.sample(np.full(37, -123.4), 5, seed=1)
    np.testing.assert_allclose(w, 1.0 / 37, rtol=1e-14)
    np.testing.assert_allclose(logw, -np.log(37), rtol=1e-14)
    rng = np.random.default_rng(0)
    L = rng.normal(0, 30, 1000)
    w, _, _ = oracle.sample(L, 1, seed=2)
    np.testing.assert_allclose(w.sum(), 1.0, rtol=1e-13)
    np.testing.assert_allclose(np.log(w), L - L.max() - np.log(np.exp(L - L.max()).sum()), atol=1e-12)


def test_gumbel_max_frequencies_follow_softmax():
    L = np.array([0.0, 1.0, -0.5, 2.0, 0.3])
    K = 100_000
    w, idx, _ = oracle.sample(L, K, seed=99)
    counts = np.bincount(idx, minlength=len(L))
    assert chisquare(counts, K * w).pvalue > 1e-3


def test_grid_layout_matches_numpy_linspace_order():
    wl = make_config(0)
    P = oracle.enumerate_grid(wl.grid)
    assert P.shape == (256, 4, 4)
    lx = np.linspace(-0.05, 0.05, 8)
    lz = np.linspace(-0.05, 0.05, 4)
    for ix, iy, iz in [(0, 0, 0), (7, 7, 3), (3, 5, 1), (1, 0, 2)]:
        n = (ix * 8 + iy) * 4 + iz
        np.testing.assert_allclose(P[n, :3, 3], wl.true_pose[:3, 3] + [lx[ix], lx[iy], lz[iz]], atol=1e-15)
        np.testing.assert_array_equal(P[n, :3, :3], np.eye(3))
    g = GridSpec(center=pose_matrix(np.eye(3), (0, 0, 1)), half_extent=(0.04, 0.04, 0), count=(10, 10, 1),
                 rotations=np.stack([np.eye(3), np.diag([1.0, -1.0, -1.0]), np.eye(3)[[1, 2, 0]]]))
    Q = oracle.enumerate_grid(g)
    assert Q.shape == (300, 4, 4)
    np.testing.assert_array_equal(Q[100 * 2 + 37, :3, :3], np.eye(3)[[1, 2, 0]])
    np.testing.assert_allclose(Q[100 * 1 + 37, :3, 3], [np.linspace(-0.04, 0.04, 10)[3],
                                                         np.linspace(-0.04, 0.04, 10)[7], 1.0], atol=1e-15)


def test_rotation_perturbations_are_rotations_within_the_angle():
    axes = []
    for r in range(400):
        R = oracle.perturbation(7, 2, r, 0.3)
        np.testing.assert_allclose(R @ R.T, np.eye(3), atol=1e-14)
        assert abs(np.linalg.det(R) - 1) < 1e-14
        ang = np.arccos(np.clip((np.trace(R) - 1) / 2, -1, 1))
        assert ang <= 0.3 + 1e-12
        if r == 0:
            np.testing.assert_array_equal(R, np.eye(3))
        else:
            w = np.array([R[2, 1] - R[1, 2], R[0, 2] - R[2, 0], R[1, 0] - R[0, 1]])
            axes.append(w / np.linalg.norm(w))
    # axis uniform on the sphere: mean near 0, second moment near I/3
    A = np.array(axes)
    assert np.abs(A.mean(0)).max() < 0.12
    np.testing.assert_allclose(A.T @ A / len(A), np.eye(3) / 3, atol=0.06)


def _partition_problem():
    base = GridSpec(center=pose_matrix(np.eye(3), (0, 0, 0.8)), half_extent=(0.06, 0.0, 0.0), count=(3, 1, 1))
    stages = partition_schedule(base, [(3, 1, 1), (2, 1, 1), (2, 1, 1)])
    x0 = 0.013
    score = lambda P: -((P[:, 0, 3] - x0) ** 2) / (2 * 0.02**2)
    return base, stages, score


def test_partition_schedule_proposal_density_integrates_to_one():
    base, stages, score = _partition_problem()
    # walk every path of the schedule; the final cells must tile the initial
    # region exactly and the path probabilities must sum to one
    leaves, probs = [], []

    def walk(centre, t, logp):
        P = oracle.enumerate_grid(stages[t], center=centre, stage=t)
        L = score(P)
        w = np.exp(L - L.max())
        w /= w.sum()
        for i in range(P.shape[0]):
            if t + 1 < len(stages):
                walk(P[i], t + 1, logp + np.log(w[i]))
            else:
                leaves.append(P[i, 0, 3])
                probs.append(np.exp(logp + np.log(w[i])))

    walk(base.center, 0, 0.0)
    vol = final_cell_volume(stages)
    np.testing.assert_allclose(sorted(leaves), -0.06 + vol * (np.arange(12) + 0.5), atol=1e-15)
    np.testing.assert_allclose(np.sum(probs), 1.0, rtol=1e-14)
    np.testing.assert_allclose(np.sum(np.array(probs) / vol) * vol, 1.0, rtol=1e-14)
    # the sampler's own log q for a drawn path equals that path's probability
    poses, logq, idx, _ = c2f(score, base.center, stages, K=8, seed=5)
    for k in range(8):
        j = int(np.argmin(np.abs(np.array(leaves) - poses[k, 0, 3])))
        np.testing.assert_allclose(np.exp(logq[k]), probs[j], rtol=1e-12)


def test_flat_likelihood_draws_final_cells_uniformly():
    base, stages, _ = _partition_problem()
    flat = lambda P: np.zeros(P.shape[0])
    poses, logq, idx, _ = c2f(flat, base.center, stages, K=6000, seed=3)
    cells = np.round((poses[:, 0, 3] + 0.06) / 0.01 - 0.5).astype(int)
    counts = np.bincount(cells, minlength=12)
    assert chisquare(counts).pvalue > 1e-3
    np.testing.assert_allclose(logq, -np.log(12), rtol=1e-13)


def test_c2f_rotation_stages_compose_around_chosen_centres():
    base = GridSpec(center=pose_matrix(np.eye(3), (0, 0, 0.8)), half_extent=(0.02, 0.02, 0.0), count=(3, 3, 1),
                    n_rot=4, rot_max_angle=0.2)
    st = [copy.deepcopy(base), copy.deepcopy(base)]
    st[1].half_extent = (0.005, 0.005, 0.0)
    st[1].rot_max_angle = 0.05
    target = np.array([0.011, -0.004, 0.8])
    score = lambda P: -np.sum((P[:, :3, 3] - target) ** 2, 1) / (2 * 0.003**2)
    poses, logq, idx, hist = c2f(score, base.center, st, K=4, seed=11)
    P0 = oracle.enumerate_grid(st[0], seed=11, stage=0)
    for k in range(4):
        c = P0[idx[0, k]]
        P1 = oracle.enumerate_grid(st[1], seed=11, stage=1, center=c)
        np.testing.assert_array_equal(poses[k], P1[idx[1, k]])
        assert np.all(logq[k] <= 0)
