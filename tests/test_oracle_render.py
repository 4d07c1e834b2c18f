"""Pins of the oracle's renderer against things other than itself.

Renderer = Alg. 1's DepthRenderer call and the point-cloud conversion of
Sec. III-A (iii), under the conventions stated in the oracle's header.
"""

import numpy as np
import pytest

import oracle
from oracle import tiny
from workloads import Camera, box_mesh, pose_matrix, random_poses, tiny_scene, voxel_blob, voxel_mesh


def _cases():
    out = []
    for seed in range(4):
        rng = np.random.default_rng(100 + seed)
        verts, tris, cam = tiny_scene(rng, 20, 12, 16, f=120.0)
        P = random_poses(rng, 2, 0.5, 0.02)
        out.append((verts, tris, cam, P))
    # a pose close to the camera: some triangles cross the near plane and are dropped
    rng = np.random.default_rng(7)
    verts, tris, cam = tiny_scene(rng, 30, 12, 16, f=12.0)
    out.append((verts, tris, cam, random_poses(rng, 2, 0.035, 0.003)))
    return out


@pytest.mark.parametrize("case", range(5))
def test_plain_scan_matches_bruteforce_ray_casting(case):
    verts, tris, cam, P = _cases()[case]
    depth, ids = oracle.render([(verts, tris, P)], cam)
    for n in range(P.shape[0]):
        bd, bi = tiny.render_bruteforce(verts, tris, P[n], cam)
        assert (ids[n] >= 0).sum() > 0
        np.testing.assert_array_equal(ids[n], bi)
        np.testing.assert_allclose(depth[n], bd, rtol=0, atol=1e-12)


def test_closed_form_axis_aligned_cube():
    s, z0 = 0.1, 0.6
    cam = Camera(50.0, 50.0, 16.25, 12.0, 24, 32)
    verts, tris = box_mesh((s, s, s))
    depth, ids = oracle.render([(verts, tris, pose_matrix(np.eye(3), (0, 0, z0)))], cam)
    front = z0 - s / 2
    c = np.arange(cam.W) + 0.5
    r = np.arange(cam.H) + 0.5
    X = (c[None, :] - cam.cx) / cam.fx + 0 * r[:, None]
    Y = (r[:, None] - cam.cy) / cam.fy + 0 * c[None, :]
    inside = (np.abs(X) * front <= s / 2) & (np.abs(Y) * front <= s / 2)
    assert inside.sum() == 90  # 9 columns x 10 rows
    assert np.all(ids[0][~inside] == -1) and np.all(depth[0][~inside] == 0)
    np.testing.assert_allclose(depth[0][inside], front, rtol=0, atol=1e-15)
    # the -z face is split along the diagonal from corner (-,-) to (+,+):
    # triangle 8 holds the side y > x, triangle 9 the side y < x
    expect = np.where(Y > X, 8, 9)
    np.testing.assert_array_equal(ids[0][inside], expect[inside])


def test_pose_equals_pretransformed_vertices():
    rng = np.random.default_rng(11)
    verts, tris = voxel_mesh(voxel_blob(60, rng, radius=0.05))
    cam = Camera(80.0, 80.0, 20.3, 15.1, 30, 40)
    P = random_poses(rng, 3, 0.6, 0.03)
    d1, i1 = oracle.render([(verts, tris, P)], cam)
    for n in range(3):
        vt = verts @ P[n, :3, :3].T + P[n, :3, 3]
        d2, i2 = oracle.render([(vt, tris, np.eye(4))], cam)
        np.testing.assert_array_equal(i1[n], i2[0])
        np.testing.assert_allclose(d1[n], d2[0], rtol=0, atol=1e-12)


def test_composition_of_two_meshes_is_nearest_surface():
    rng = np.random.default_rng(5)
    va, ta = voxel_mesh(voxel_blob(30, rng, radius=0.04))
    vb, tb = box_mesh((0.05, 0.05, 0.05))
    cam = Camera(60.0, 60.0, 16.4, 12.2, 24, 32)
    Pa = pose_matrix(np.eye(3), (0.0, 0.0, 0.5))
    Pb = pose_matrix(np.eye(3), (0.02, 0.0, 0.4))
    d, i = oracle.render([(va, ta, Pa), (vb, tb, Pb)], cam)
    da, ia = tiny.render_bruteforce(va, ta, Pa, cam)
    db, ib = tiny.render_bruteforce(vb, tb, Pb, cam, id_offset=ta.shape[0])
    da[da == 0] = np.inf
    db[db == 0] = np.inf
    exp_d = np.minimum(da, db)
    exp_i = np.where(db < da, ib, ia)
    exp_d[np.isinf(exp_d)] = 0
    np.testing.assert_array_equal(i[0], exp_i)
    np.testing.assert_allclose(d[0], exp_d, atol=1e-12)


def test_counters_and_unprojection():
    rng = np.random.default_rng(3)
    verts, tris, cam = tiny_scene(rng, 15, 12, 16, f=100.0)
    P = random_poses(rng, 2, 0.5, 0.01)
    d, i, cnt = oracle.render([(verts, tris, P)], cam, counters=True)
    assert np.all(cnt[:, oracle.C_VERT] == verts.shape[0])
    assert np.all(cnt[:, oracle.C_TRI] == tris.shape[0])
    assert np.all(cnt[:, oracle.C_FRONT] <= tris.shape[0])
    assert np.all(cnt[:, oracle.C_FRAG] >= (i >= 0).reshape(2, -1).sum(1))
    xyz = oracle.unproject(d, cam)
    # each point lies on its pixel's ray at the rendered depth
    np.testing.assert_array_equal(xyz[..., 2], d)
    cc = (np.arange(cam.W) + 0.5 - cam.cx) / cam.fx
    np.testing.assert_allclose(xyz[..., 0], d * cc[None, None, :], rtol=1e-15, atol=0)
