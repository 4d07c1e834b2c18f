"""The seeded synthetic inputs: geometry conventions, determinism and the
shapes the configurations state."""

import numpy as np

import oracle
from workloads import box_mesh, make_config, voxel_blob, voxel_mesh


def test_voxel_triangles_wind_outward():
    rng = np.random.default_rng(0)
    centres = voxel_blob(10, rng)
    verts, tris = voxel_mesh(centres)
    for t in range(tris.shape[0]):
        a, b, c = verts[tris[t]]
        n = np.cross(b - a, c - a)
        centroid = (a + b + c) / 3
        assert np.dot(n, centroid - centres[t // 12]) > 0
        assert abs(np.linalg.norm(n) - 0.01**2) < 1e-15  # half of a 1 cm face, doubled
    bv, bt = box_mesh((0.1, 0.2, 0.3))
    assert np.allclose(bv.max(0) - bv.min(0), [0.1, 0.2, 0.3])


def test_blob_voxels_are_distinct_lattice_cells_in_the_ball():
    rng = np.random.default_rng(1)
    c = voxel_blob(2000, rng)
    cells = np.round(c / 0.01).astype(int)
    assert len({tuple(x) for x in cells}) == 2000
    assert np.all(np.linalg.norm(c, axis=1) <= 0.10 + 1e-12)


def test_configs_are_deterministic_and_shaped_as_stated():
    a, b = make_config(0), make_config(0)
    np.testing.assert_array_equal(a.verts, b.verts)
    np.testing.assert_array_equal(a.noise["gauss"], b.noise["gauss"])
    assert a.tris.shape == (6000, 3) and a.grid.N == 256
    assert (a.camera.H, a.camera.W) == (48, 64)
    c1 = make_config(1, render=oracle.render_depth_fn)
    assert c1.tris.shape == (24000, 3) and c1.grid.N == 5000
    assert (c1.camera.H, c1.camera.W) == (120, 160)
    np.testing.assert_allclose(c1.true_pose[:3, :3], c1.grid.rotations[0])
    # the occluder hides 20% +- 0.5% of the object's pixels at the true pose
    obj = oracle.render([(c1.verts, c1.tris, c1.true_pose)], c1.camera)[0][0] > 0
    occ = oracle.render([c1.occluder], c1.camera)[0][0] > 0
    assert abs((obj & occ).sum() / obj.sum() - 0.20) <= 0.005
    assert c1.occluder[2][2, 3] - 0.03 == np.float64(0.6) or abs(c1.occluder[2][2, 3] - 0.63) < 1e-12


def test_camera_pan_keeps_the_object_centred_and_moves_a_little_per_frame():
    from workloads import camera_pan_sequence

    (v, t), P, cam, noise = camera_pan_sequence(res=50, n_frames=120)
    assert t.shape == ((10 * 6 * 17 + 27) * 12 + 2, 3) and P.shape == (120, 4, 4) and (cam.H, cam.W) == (50, 50)
    for T in P:
        np.testing.assert_allclose(T[:3, :3] @ T[:3, :3].T, np.eye(3), atol=1e-12)
        assert abs(T[0, 3]) < 1e-12 and abs(T[1, 3]) < 1e-12 and 0.54 <= T[2, 3] <= 0.66  # origin on the axis
        up = T[:3, :3] @ np.array([0.0, 0.0, 1.0])
        assert up[1] < -0.4  # scene +z points up in the image (image y runs down)
    step_t = np.linalg.norm(np.diff(P[:, :3, 3], axis=0), axis=1)
    step_r = [np.degrees(np.arccos(np.clip((np.trace(P[i + 1, :3, :3] @ P[i, :3, :3].T) - 1) / 2, -1, 1)))
              for i in range(119)]
    assert step_t.max() < 0.006 and max(step_r) < 1.5
    # same object and path at every resolution; noise drawn per resolution
    (v2, _), P2, cam2, noise2 = camera_pan_sequence(res=25, n_frames=120)
    np.testing.assert_array_equal(v, v2)
    np.testing.assert_array_equal(P, P2)
    assert noise2[0]["gauss"].shape == (25, 25) and cam2.fx * 2 == cam.fx
    # the object rests on the table: its lowest voxel face is at the table's height
    obj = v[:-4]
    assert abs(obj[:, 2].min() - v[-4:, 2].max()) < 1e-12
