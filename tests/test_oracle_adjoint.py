"""Pins of the oracle's adjoint: central finite differences in FP64 on the
frozen-visibility forward, and closed forms for a frontal face.

The adjoint differentiates eq. (1), truncated to a window (Sec. III-B), with
respect to the rendered points, sigma, p_out and the 6-DoF pose (update
R <- exp([dw]x) R, t <- t + dt) with triangle visibility held fixed."""

import numpy as np
from scipy.spatial.transform import Rotation

import oracle
from workloads import Camera, box_mesh, pose_matrix, random_poses, voxel_blob, voxel_mesh


def _scene(seed=0, N=2):
    rng = np.random.default_rng(seed)
    verts, tris = voxel_mesh(voxel_blob(40, rng, radius=0.05))
    cam = Camera(90.0, 90.0, 16.3, 12.4, 24, 32)
    P = random_poses(rng, N, 0.6, 0.01)
    truth = random_poses(rng, 1, 0.6, 0.005)[0]
    truth[:3, :3] = P[0, :3, :3]
    d, _ = oracle.render([(verts, tris, truth)], cam)
    obs = oracle.unproject(d[0] + 0.001 * rng.standard_normal(d[0].shape) * (d[0] > 0), cam)
    return verts, tris, cam, P, obs


def _perturb(P, k, h):
    Q = P.copy()
    if k < 3:
        Q[k, 3] += h
    else:
        w = np.zeros(3)
        w[k - 3] = h
        Q[:3, :3] = Rotation.from_rotvec(w).as_matrix() @ P[:3, :3]
    return Q


def test_score_adjoint_matches_central_differences():
    rng = np.random.default_rng(1)
    H, W = 6, 7
    z = 0.7 + 0.003 * rng.standard_normal((H, W))
    obs = np.stack([0.01 * rng.standard_normal((H, W)), 0.01 * rng.standard_normal((H, W)), z], -1)
    rend = obs[None] + 0.003 * rng.standard_normal((1, H, W, 3))
    rend[0, rng.random((H, W)) < 0.3] = 0.0
    obs[rng.random((H, W)) < 0.2] = 0.0
    sig, p, V, r = 0.004, 0.05, 1.2, 3
    dq, ds, dp = oracle.score_grad(obs, rend, sig, p, V, r)
    f = lambda s=sig, pp=p, q=rend: oracle.score(obs, q, s, pp, V, r)[0][0]
    h = 1e-7
    np.testing.assert_allclose(ds[0], (f(s=sig + h) - f(s=sig - h)) / (2 * h), rtol=2e-6)
    np.testing.assert_allclose(dp[0], (f(pp=p + 1e-6) - f(pp=p - 1e-6)) / 2e-6, rtol=2e-6)
    for (i, j, c) in [(0, 0, 0), (2, 3, 2), (5, 6, 1), (3, 1, 2)]:
        if rend[0, i, j, 2] <= 0:
            continue
        qp, qm = rend.copy(), rend.copy()
        qp[0, i, j, c] += 1e-7
        qm[0, i, j, c] -= 1e-7
        np.testing.assert_allclose(dq[0, i, j, c], (f(q=qp) - f(q=qm)) / 2e-7, rtol=2e-5, atol=1e-3)


def test_pose_adjoint_matches_frozen_visibility_differences():
    verts, tris, cam, P, obs = _scene()
    sig, p, V, r = 0.003, 0.01, 1.0, 5
    depth, ids = oracle.render([(verts, tris, P)], cam)
    xyz = oracle.unproject(depth, cam)
    dq, _, _ = oracle.score_grad(obs, xyz, sig, p, V, r)
    g = oracle.render_grad(verts, tris, P, cam, ids, depth, dq)

    def logL_frozen(Q, n):
        dz = oracle.render_frozen(verts, tris, Q[None], cam, ids[n][None])
        return oracle.score(obs, oracle.unproject(dz, cam), sig, p, V, r)[0][0]

    h = 1e-7
    for n in range(P.shape[0]):
        fd = np.array([(logL_frozen(_perturb(P[n], k, h), n) - logL_frozen(_perturb(P[n], k, -h), n)) / (2 * h)
                       for k in range(6)])
        np.testing.assert_allclose(g[n], fd, rtol=1e-5, atol=1e-4 * np.abs(fd).max())


def test_frontal_face_depth_derivatives_closed_form():
    # a cube facing the camera: its visible face is the plane z = z0 - s/2,
    # so moving the cube along z moves every visible depth by the same
    # amount, while sliding it sideways or spinning it about the optical axis
    # leaves depths unchanged
    s, z0 = 0.1, 0.6
    cam = Camera(50.0, 50.0, 16.25, 12.0, 24, 32)
    verts, tris = box_mesh((s, s, s))
    P = pose_matrix(np.eye(3), (0.0, 0.0, z0))
    depth, ids = oracle.render([(verts, tris, P)], cam)
    rows, cols = np.nonzero(ids[0] >= 0)
    for rr, cc in [(rows[0], cols[0]), (rows[len(rows) // 2], cols[len(rows) // 2])]:
        dq = np.zeros((1, cam.H, cam.W, 3))
        # d logL / d q_j = e_z: then g_j = d_z = 1, so d_pose is dz_j/d(pose)
        dq[0, rr, cc, 2] = 1.0
        g = oracle.render_grad(verts, tris, P[None], cam, ids, depth, dq)[0]
        np.testing.assert_allclose(g[2], 1.0, rtol=1e-14)
        np.testing.assert_allclose(g[[0, 1, 5]], 0.0, atol=1e-14)


def test_pure_outlier_model_has_zero_pose_gradient():
    verts, tris, cam, P, obs = _scene(seed=3)
    depth, ids = oracle.render([(verts, tris, P)], cam)
    xyz = oracle.unproject(depth, cam)
    dq, ds, dp = oracle.score_grad(obs, xyz, 0.003, 1.0, 1.0, 5)
    assert np.all(dq == 0.0) and np.all(ds == 0.0)
    g = oracle.render_grad(verts, tris, P, cam, ids, depth, dq)
    assert np.all(g == 0.0)
    # with p_out = 1 every valid pixel contributes d/dp ln(p/V + (1-p)S/M) = 1 - V S/M
    n_valid = (obs[..., 2] > 0).sum()
    assert np.all(dp <= n_valid + 1e-9)
