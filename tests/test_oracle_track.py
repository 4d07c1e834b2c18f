"""Pins of the oracle's tracking frame (oracle/track.py): a noiseless
observation is found exactly when the grid holds the truth, a flat
likelihood resolves every tie to the first hypothesis, the first Adam step
has the closed-form size, and near ties are followed."""

import numpy as np

import oracle
from oracle import track
from workloads import Camera, GridSpec, ScoreParams, pose_matrix, voxel_blob, voxel_mesh


def scene(seed=5):
    rng = np.random.default_rng(seed)
    meshes = [voxel_mesh(voxel_blob(60, rng, radius=0.03)), voxel_mesh(voxel_blob(50, rng, radius=0.03))]
    cam = Camera(60.0, 60.0, 24.0, 18.0, 36, 48)
    truth = [pose_matrix(np.eye(3), (-0.03, 0.0, 0.5)), pose_matrix(np.eye(3), (0.035, 0.01, 0.52))]
    d, _ = oracle.render([(v, t, P) for (v, t), P in zip(meshes, truth)], cam)
    return meshes, [track.round32(P) for P in truth], cam, track.round32(oracle.unproject(d[0], cam))


def test_noiseless_truth_on_the_grid_is_found():
    meshes, truth, cam, obs = scene()
    sp = ScoreParams(sigma=0.003, p_out=0.01, outlier_volume=1.0, window=3)
    start = [P.copy() for P in truth]
    start[0][:3, 3] += (0.01, -0.005, 0.005)  # on the grid below: offsets in steps of 5 mm
    spec = GridSpec(center=np.eye(4), half_extent=(0.015, 0.015, 0.015), count=(7, 7, 7))
    out = track.track_frame(meshes, start, obs, cam, sp, [spec])
    np.testing.assert_allclose(out[0], truth[0], atol=1e-7)
    np.testing.assert_allclose(out[1], truth[1], atol=1e-7)


def test_flat_likelihood_takes_the_first_hypothesis_at_every_stage():
    meshes, truth, cam, obs = scene()
    sp = ScoreParams(sigma=0.003, p_out=1.0, outlier_volume=1.0, window=3)
    stages = [GridSpec(center=np.eye(4), half_extent=(0.02, 0.01, 0.03), count=(3, 3, 3), n_rot=4,
                       rot_max_angle=0.2),
              GridSpec(center=np.eye(4), half_extent=(0.004, 0.002, 0.001), count=(2, 2, 2), n_rot=3,
                       rot_max_angle=0.1)]
    out = track.track_frame(meshes, truth, obs, cam, sp, stages)
    for o in range(2):
        want = truth[o].copy()
        want[:3, 3] -= np.array([0.024, 0.012, 0.031])  # index 0: the lowest offset of each axis, identity rotation
        np.testing.assert_allclose(out[o], want, atol=1e-7)
    ends = track.search_ends(meshes, truth, 0, stages, obs, cam, sp, tol=0.0, limit=2)
    assert len(ends) == 4
    np.testing.assert_allclose(ends[0], out[0], atol=1e-7)
    assert not np.allclose(ends[1], ends[0])


def test_first_adam_step_moves_each_coordinate_by_its_rate():
    meshes, truth, cam, obs = scene()
    sp = ScoreParams(sigma=0.003, p_out=0.01, outlier_volume=1.0, window=3)
    start = [P.copy() for P in truth]
    start[0][:3, 3] += (0.004, -0.003, 0.002)
    start = [track.round32(P) for P in start]
    d, ids = oracle.render(track.scene_objects(meshes, start, 0, start[0][None]), cam)
    dr, _, _ = oracle.score_grad(obs, oracle.unproject(d, cam), sp.sigma, sp.p_out, 1.0, 3)
    g = oracle.render_grad(meshes[0][0], meshes[0][1], start[0][None], cam, ids, d, dr)[0]
    Q = track.refine(meshes, start, 0, obs, cam, sp, 1, 1e-3, 1e-2)
    # Adam's first step is lr g / (|g| + eps): the rate times the gradient's sign
    np.testing.assert_allclose(Q[:3, 3] - start[0][:3, 3], 1e-3 * np.sign(g[:3]), atol=2e-8)
    from oracle.refine import rotvec_exp

    np.testing.assert_allclose(Q[:3, :3], rotvec_exp(1e-2 * np.sign(g[3:])) @ start[0][:3, :3], atol=1e-7)
    # ascent: the translation moves back along x and z (the object shows no
    # face turned along y here, so the frozen-visibility gradient has no y part)
    assert np.sign(g[0]) == -1 and np.sign(g[2]) == -1 and g[1] == 0
