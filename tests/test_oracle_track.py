"""Pins of the oracle's tracking frame (oracle/track.py): a noiseless
observation is found exactly when the grid holds the truth, a flat
likelihood resolves every tie to the first hypothesis, the first Adam step
has the closed-form size, and near ties are followed; the occlusion
handling counts seen pixels exactly on squares of known footprint, keeps
or replaces updates by the last motion in the pinned order, and widens the
next search."""

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


def square(x0, x1, y0, y1):
    """A camera-facing square [x0, x1] x [y0, y1] at z = 0 of its frame (two
    triangles, wound to face the camera)."""
    v = np.array([[x0, y0, 0.0], [x1, y0, 0.0], [x1, y1, 0.0], [x0, y1, 0.0]])
    t = np.array([[0, 2, 1], [0, 3, 2]], dtype=np.int32)
    return v, t


def test_seen_fraction_counts_pixels_in_front_and_confirmed_by_the_observation():
    # A square covering pixel columns 10..29 and rows 10..29 at 0.5 m (edges a
    # quarter pixel outside those pixels' centres), and an occluder at 0.4 m
    # covering columns 10..19 of it: half the square's 400 pixels are in
    # front; alone all are; behind a larger occluder none.  The observation
    # must confirm each pixel within the tolerance: moving the right half of
    # the observed square back 2 cm (tolerance 1 cm) or blanking it halves
    # the fraction.
    cam = Camera(60.0, 60.0, 24.0, 18.0, 36, 48)
    z, zo = 0.5, 0.4

    def span(a, b, zz):  # pixel edges a - 0.25 .. b + 1.25 as metric coordinates at depth zz
        return (a - 0.25 - cam.cx) / cam.fx * zz, (b + 1.25 - cam.cx) / cam.fx * zz

    def vspan(a, b, zz):
        return (a - 0.25 - cam.cy) / cam.fy * zz, (b + 1.25 - cam.cy) / cam.fy * zz

    target = square(*span(10, 29, z), *vspan(10, 29, z))
    half = square(*span(8, 19, zo), *vspan(8, 31, zo))
    whole = square(*span(5, 35, zo), *vspan(5, 33, zo))
    at = lambda zz: pose_matrix(np.eye(3), (0.0, 0.0, zz))
    d = oracle.render([(target[0], target[1], at(z))], cam)[0][0]
    assert int((d > 0).sum()) == 400
    obs = oracle.unproject(d, cam)
    seen = lambda meshes, poses, o, ob: track.seen_fraction(meshes, poses, o, cam, ob, 0.01)
    assert seen([target], [at(z)], 0, obs) == 1.0
    assert seen([target, half], [at(z), at(zo)], 0, obs) == 0.5
    assert seen([target, whole], [at(z), at(zo)], 0, obs) == 0.0
    back = oracle.unproject(np.where(np.arange(cam.W) >= 20, d + 0.02 * (d > 0), d), cam)
    assert seen([target], [at(z)], 0, back) == 0.5
    blank = oracle.unproject(np.where(np.arange(cam.W) >= 20, 0.0, d), cam)
    assert seen([target], [at(z)], 0, blank) == 0.5
    # a larger tolerance takes the moved half back
    assert track.seen_fraction([target], [at(z)], 0, cam, back, 0.03) == 1.0
    # observed two pixels to the right: columns 10 and 11 see no observed
    # point of their own; a 5 x 5 window finds one two (column 10) or one
    # (column 11) pixel away, 0.5 m x 2/60 = 16.7 mm or 8.3 mm from theirs
    shift = oracle.unproject(np.roll(d, 2, axis=1), cam)
    assert track.seen_fraction([target], [at(z)], 0, cam, shift, 0.02, window=1) == 0.9
    assert track.seen_fraction([target], [at(z)], 0, cam, shift, 0.02, window=5) == 1.0
    assert track.seen_fraction([target], [at(z)], 0, cam, shift, 0.01, window=5) == 0.95
    # the occluder itself is never behind; its observed depth here is the
    # target's, 10 cm away, so none of it is confirmed
    assert seen([target, half], [at(z), at(zo)], 1, obs) == 0.0
    # off screen: nothing drawn
    assert seen([target], [pose_matrix(np.eye(3), (5.0, 0.0, z))], 0, obs) == 0.0


def rot_z(deg):
    a = np.deg2rad(deg)
    return np.array([[np.cos(a), -np.sin(a), 0.0], [np.sin(a), np.cos(a), 0.0], [0.0, 0.0, 1.0]])


def rot_x(deg):
    a = np.deg2rad(deg)
    return np.array([[1.0, 0.0, 0.0], [0.0, np.cos(a), -np.sin(a)], [0.0, np.sin(a), np.cos(a)]])


def test_gate_keeps_visible_updates_and_moves_hidden_objects_by_the_last_motion():
    # The kept motion is a turn about the camera's x axis applied on the left
    # of an orientation turned about z (the two do not commute, so the order
    # of the product is pinned) and a 1 cm step.
    g = track.Gating.start(1, min_visible=0.3, widen=2.5)
    prev = pose_matrix(rot_z(20.0), (0.1, 0.0, 0.8))
    new = pose_matrix(rot_x(10.0) @ rot_z(20.0), (0.11, -0.01, 0.8))
    out = track.gate_update(g, 0, prev, new, seen=0.3)  # at the threshold: kept
    np.testing.assert_array_equal(out, new)
    np.testing.assert_allclose(g.dR[0], rot_x(10.0), atol=1e-15)
    np.testing.assert_allclose(g.dt[0], (0.01, -0.01, 0.0), atol=1e-15)
    assert (g.dropped[0], g.scale[0]) == (0, 1.0)
    # hidden twice: each frame the object turns 10 more degrees and moves 1 cm
    # further, whatever the search proposed
    junk = pose_matrix(rot_z(-70.0), (0.5, 0.5, 2.0))
    out = track.gate_update(g, 0, new, junk, seen=0.29)
    np.testing.assert_allclose(out, pose_matrix(rot_x(20.0) @ rot_z(20.0), (0.12, -0.02, 0.8)), atol=1e-15)
    assert (g.dropped[0], g.scale[0]) == (1, 2.5)
    out = track.gate_update(g, 0, out, junk, seen=0.0)
    np.testing.assert_allclose(out, pose_matrix(rot_x(30.0) @ rot_z(20.0), (0.13, -0.03, 0.8)), atol=1e-15)
    assert (g.dropped[0], g.scale[0]) == (2, 2.5)
    # seen again: the update stands and the search box shrinks back
    back = pose_matrix(rot_z(52.0), (0.135, -0.03, 0.8))
    np.testing.assert_array_equal(track.gate_update(g, 0, out, back, seen=0.9), back)
    assert (g.dropped[0], g.scale[0]) == (0, 1.0)


def test_a_hidden_object_keeps_still_and_the_next_search_widens():
    # Object 0 straight behind a square filling the view: its update is
    # dropped (no motion yet, so it stays put), the square is updated, and
    # the next frame's first stage is the plain grid with its translation
    # offsets scaled by widen.
    meshes, truth, cam, obs = scene()
    wall = square(-0.2, 0.2, -0.2, 0.2)
    meshes = [meshes[0], wall]
    poses = [truth[0], track.round32(pose_matrix(np.eye(3), (0.0, 0.0, 0.4)))]
    d, _ = oracle.render([(v, t, P) for (v, t), P in zip(meshes, poses)], cam)
    obs = track.round32(oracle.unproject(d[0], cam))
    sp = ScoreParams(sigma=0.003, p_out=0.01, outlier_volume=1.0, window=3)
    spec = GridSpec(center=np.eye(4), half_extent=(0.01, 0.01, 0.01), count=(3, 3, 3))
    g = track.Gating.start(2, min_visible=0.2, widen=3.0)
    assert track.seen_fraction(meshes, poses, 0, cam, obs, 3 * sp.sigma) == 0.0
    out = track.track_frame(meshes, poses, obs, cam, sp, [spec], gating=g)
    np.testing.assert_array_equal(out[0], poses[0])
    # the wall fills the view, so only its depth is observable: found, and kept
    assert abs(out[1][2, 3] - poses[1][2, 3]) < 1e-7
    assert g.dropped == [1, 0] and g.scale == [3.0, 1.0]
    wide = oracle.enumerate_grid(track.scaled(spec, 3.0), center=poses[0])
    plain = oracle.enumerate_grid(spec, center=poses[0])
    np.testing.assert_allclose(wide[:, :3, 3] - poses[0][:3, 3], 3.0 * (plain[:, :3, 3] - poses[0][:3, 3]),
                               atol=1e-9)
