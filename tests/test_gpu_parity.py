"""Parity of the HIP library against the FP64 oracle, element by element on
identical seeded inputs (float32 values, widened to float64 for the oracle).

Bars (from the stated targets):
  * render: >= 99.9% of (hypothesis, pixel) pairs have equal triangle ids,
    and there both are empty or |dz| <= 1e-5 m;
  * logL: |logL_gpu - logL_64| <= 1e-4 * sum_i |l_i| (the L1 mass of the
    per-pixel terms);
  * adjoint: ||g_gpu - g_64|| <= 1e-3 ||g_64|| + 1e-6 per hypothesis;
  * samples: equal wherever the oracle's top-two gap of logL + G exceeds
    1e-4 (absolute, for given logits) or 1e-4 of the L1 mass (for scored
    hypotheses): FP32 Gumbel noise and FP32 logL error stay well below it.
"""

import numpy as np
import pytest
import torch

import oracle
from workloads import Camera, make_config, pose_matrix, random_poses, voxel_blob, voxel_mesh

pytestmark = pytest.mark.gpu

LOGL_RTOL = 1e-4


def say(*a):
    print(*a, flush=True)


@pytest.fixture(scope="module")
def b3d():
    import paper_2312_08715_amd as b

    assert torch.cuda.is_available(), "GPU tests need a device"
    b.load_library()
    return b


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


_cache = {}


def workload(k):
    if k not in _cache:
        wl = make_config(k, render=oracle.render_depth_fn)
        wl.verts = f32(wl.verts)
        obs = f32(oracle.observed_xyz(wl))
        P = f32(oracle.enumerate_grid(wl.grid, seed=wl.seeds["hyp"]))
        _cache[k] = (wl, obs, P)
    return _cache[k]


def agree(gz, gtri, od, oi):
    """Per pixel: same triangle, or two surfaces at the same depth (a tie
    between coplanar faces, where either id is a correct answer)."""
    return (gtri == oi) | ((gtri >= 0) & (oi >= 0) & (np.abs(gz - od) <= 1e-5))


def clean_hypotheses(gz, gtri, od, oi):
    return np.all(agree(gz, gtri, od, oi).reshape(gz.shape[0], -1), axis=1)


def render_compare(gxyz, gtri, od, oi):
    gz = gxyz[..., 2]
    same = gtri == oi
    frac = same.mean()
    both = same & (oi >= 0)
    dz = np.abs(gz[both] - od[both]).max() if both.any() else 0.0
    empty_ok = np.all(gz[same & (oi < 0)] == 0)
    return frac, dz, empty_ok


@pytest.mark.parametrize("k", [0, 1])
def test_render_batch_matches_oracle(b3d, k):
    wl, obs, P = workload(k)
    say(f"render parity: config {k}, N={P.shape[0]}")
    mesh = b3d.Mesh(wl.verts, wl.tris)
    K = b3d.intrinsics_of(wl.camera)
    xyz, tri = b3d.render_batch(mesh, dev(P), K)
    torch.cuda.synchronize()
    sel = np.arange(P.shape[0]) if k == 0 else np.random.default_rng(0).choice(P.shape[0], 400, replace=False)
    od, oi = oracle.render([(wl.verts, wl.tris, P[sel])], wl.camera)
    gx = xyz[torch.as_tensor(sel, device="cuda")].cpu().numpy()
    gt = tri[torch.as_tensor(sel, device="cuda")].cpu().numpy()
    frac, dz, empty_ok = render_compare(gx, gt, od, oi)
    say(f"  id agreement {frac:.6f}, max |dz| {dz:.3g}")
    assert frac >= 0.999 and dz <= 1e-5 and empty_ok
    # x, y are the depth times the pixel ray
    cc = ((np.arange(wl.camera.W) + 0.5 - wl.camera.cx) / wl.camera.fx).astype(np.float32)
    np.testing.assert_allclose(gx[..., 0], gx[..., 2] * cc[None, None, :], rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("k", [0, 1])
def test_score_matches_oracle_on_identical_point_images(b3d, k):
    wl, obs, P = workload(k)
    sel = np.arange(P.shape[0]) if k == 0 else np.random.default_rng(1).choice(P.shape[0], 300, replace=False)
    say(f"score parity: config {k}, {len(sel)} hypotheses")
    od, _ = oracle.render([(wl.verts, wl.tris, P[sel])], wl.camera)
    rend = f32(oracle.unproject(od, wl.camera))
    s = wl.score
    L64, l1 = oracle.score(obs, rend, s.sigma, s.p_out, s.outlier_volume, s.window)
    p = b3d.score_params(s.sigma, s.p_out, s.outlier_volume, s.window)
    Lg = b3d.score(dev(obs), dev(rend), p).cpu().numpy().astype(np.float64)
    err = np.abs(Lg - L64) / l1
    # the kernel without the workspace's valid-pixel list (taken when W is not a multiple of 4)
    Lp = b3d.score(dev(obs), dev(rend), p, workspace=False).cpu().numpy().astype(np.float64)
    errp = np.abs(Lp - L64) / l1
    say(f"  max rel-L1 error {err.max():.3g} (without the workspace {errp.max():.3g})")
    assert err.max() <= LOGL_RTOL and errp.max() <= LOGL_RTOL


def _scene(b3d, wl, obs, mesh=None):
    mesh = mesh or b3d.Mesh(wl.verts, wl.tris)
    s = wl.score
    scene = b3d.Scene(mesh, b3d.intrinsics_of(wl.camera), b3d.score_params(s.sigma, s.p_out, s.outlier_volume,
                                                                          s.window))
    o = dev(obs)
    scene.set_observed(o)
    return scene, mesh, o


def _oracle_logL(wl, obs, P, chunk=500):
    s = wl.score
    outs, l1s, ids, ds = [], [], [], []
    for i in range(0, P.shape[0], chunk):
        d, idn = oracle.render([(wl.verts, wl.tris, P[i:i + chunk])], wl.camera)
        L, l1 = oracle.score(obs, oracle.unproject(d, wl.camera), s.sigma, s.p_out, s.outlier_volume, s.window)
        outs.append(L)
        l1s.append(l1)
        ids.append(idn)
        ds.append(d)
    return np.concatenate(outs), np.concatenate(l1s), np.concatenate(ids), np.concatenate(ds)


@pytest.mark.parametrize("k", [0, 1])
def test_fused_render_score_matches_oracle_and_split_path(b3d, k):
    wl, obs, P = workload(k)
    say(f"fused parity: config {k}, N={P.shape[0]}")
    scene, mesh, o = _scene(b3d, wl, obs)
    Pd = dev(P)
    Lf = b3d.render_score(scene, Pd).cpu().numpy().astype(np.float64)
    xyz, tri = b3d.render_batch(mesh, Pd, b3d.intrinsics_of(wl.camera))
    s = wl.score
    Ls = b3d.score(o, xyz, b3d.score_params(s.sigma, s.p_out, s.outlier_volume, s.window)).cpu().numpy()
    L64, l1, oid, od = _oracle_logL(wl, obs, P)
    # fused equals the split composition up to FP32 rounding
    assert np.max(np.abs(Lf - Ls) / l1) <= 1e-5
    gt = tri.cpu().numpy()
    clean = clean_hypotheses(xyz[..., 2].cpu().numpy(), gt, od, oid)
    err = np.abs(Lf - L64) / l1
    say(f"  hypotheses with identical ids: {clean.mean():.4f}; max rel-L1 err (clean) {err[clean].max():.3g},"
        f" (all) {err.max():.3g}")
    say(f"  clean fraction {clean.mean():.4f}")
    assert clean.mean() >= 0.99
    assert err[clean].max() <= LOGL_RTOL
    # the oracle re-scoring the GPU's own point images
    sel = np.arange(0, P.shape[0], max(1, P.shape[0] // 200))
    Lr, l1r = oracle.score(obs, xyz[torch.as_tensor(sel, device="cuda")].cpu().numpy().astype(np.float64),
                           s.sigma, s.p_out, s.outlier_volume, s.window)
    assert np.max(np.abs(Lf[sel] - Lr) / l1r) <= LOGL_RTOL
    # bitwise repeatable
    Lf2 = b3d.render_score(scene, Pd).cpu().numpy()
    assert np.array_equal(Lf2, Lf.astype(np.float32))


def test_autotuned_tile_keeps_results_and_cache_round_trips(b3d, tmp_path):
    wl, obs, P = workload(1)
    sel = np.arange(0, P.shape[0], 25)
    say(f"autotune: config 1, {len(sel)} hypotheses")
    scene, mesh, o = _scene(b3d, wl, obs)
    Pd = dev(P[sel])
    L0, G0 = b3d.render_score(scene, Pd, grad=True)
    cache = str(tmp_path / "tiles.json")
    z = scene.autotune(Pd, grad=True, cache=cache)
    say(f"  chosen depth-buffer capacity {z} keys")
    # every tile shape gives bitwise the same results
    L1, G1 = b3d.render_score(scene, Pd, grad=True)
    assert torch.equal(L1, L0) and torch.equal(G1, G0)
    lo, hi, cur = scene.tile_limits()
    assert lo <= cur <= hi and cur == z
    scene.set_tile(lo)  # the smallest: bands of two rows
    L3, G3 = b3d.render_score(scene, Pd, grad=True)
    assert torch.equal(L3, L0) and torch.equal(G3, G0)
    # a second scene of the same shape class takes the cached choice without timing
    scene2, _, _ = _scene(b3d, wl, obs, mesh=mesh)
    assert scene2.autotune(Pd, grad=True, cache=cache) == z
    # capacities outside the LDS budget or below one band are refused; 0 restores the default
    with pytest.raises(b3d.B3DError):
        scene2.set_tile(lo - 1)
    with pytest.raises(b3d.B3DError):
        scene2.set_tile(hi + 1)
    scene2.set_tile(0)
    assert torch.equal(b3d.render_score(scene2, Pd), L0)


def test_autograd_score_through_the_retraction_matches_oracle(b3d):
    from oracle.refine import retract, retract_grad

    wl, obs, P = workload(0)
    sel = np.arange(0, P.shape[0], 16)
    say(f"autograd B3DScore: config 0, {len(sel)} hypotheses")
    scene, mesh, o = _scene(b3d, wl, obs)
    rng = np.random.default_rng(77)
    xi = f32(rng.normal(size=(len(sel), 6)) * np.array([0.005] * 3 + [0.05] * 3))
    base = P[sel]
    s = wl.score
    sigma = torch.tensor(s.sigma * 1.25, dtype=torch.float32, requires_grad=True)
    p_out = torch.tensor(s.p_out, dtype=torch.float32, requires_grad=True)
    xi_t = dev(xi).requires_grad_(True)
    logL = b3d.B3DScore.apply(xi_t, dev(base), sigma, p_out, scene)
    dl = f32(rng.normal(1.0, 0.3, len(sel)))
    logL.backward(dev(dl))
    # oracle: retract in FP64 from the same FP32 inputs, score and adjoints there
    sg, po = float(sigma.detach()), float(p_out.detach())
    Pr = retract(base, xi)
    Pg = b3d.pose_retract(dev(base), dev(xi)).cpu().numpy()
    assert np.max(np.abs(Pg - Pr)) <= 1e-6
    od, oi = oracle.render([(wl.verts, wl.tris, Pr)], wl.camera)
    rend = oracle.unproject(od, wl.camera)
    L64, l1 = oracle.score(obs, rend, sg, po, s.outlier_volume, s.window)
    dr, ds, dp = oracle.score_grad(obs, rend, sg, po, s.outlier_volume, s.window)
    gp = oracle.render_grad(wl.verts, wl.tris, Pr, wl.camera, oi, od, dr)
    assert np.max(np.abs(logL.detach().cpu().numpy() - L64) / l1) <= LOGL_RTOL
    want = retract_grad(xi, gp, dl)
    got = xi_t.grad.cpu().numpy()
    xyz, tri = b3d.render_batch(mesh, dev(Pg), b3d.intrinsics_of(wl.camera))
    clean = clean_hypotheses(xyz[..., 2].cpu().numpy(), tri.cpu().numpy(), od, oi)
    say(f"  clean fraction {clean.mean():.4f}")
    assert clean.mean() >= 0.99
    for n in np.nonzero(clean)[0]:
        assert np.linalg.norm(got[n] - want[n]) <= 1e-3 * np.linalg.norm(want[n]) + 1e-6, (n, got[n], want[n])
    if clean.all():
        assert abs(float(sigma.grad) - np.sum(dl * ds)) <= 1e-3 * np.sum(np.abs(dl * ds)) + 1e-3
        assert abs(float(p_out.grad) - np.sum(dl * dp)) <= 1e-4 * np.sum(np.abs(dl * dp)) + 1e-3
    # the scene took the new sigma; the window cannot change
    assert scene.params.sigma == np.float32(s.sigma * 1.25)
    with pytest.raises(b3d.B3DError):
        scene.set_params(b3d.score_params(s.sigma, s.p_out, s.outlier_volume, s.window + 2))


def test_score_backward_matches_oracle(b3d):
    wl, obs, P = workload(0)
    sel = np.arange(0, 256, 8)
    say(f"score_backward parity: config 0, {len(sel)} hypotheses")
    od, _ = oracle.render([(wl.verts, wl.tris, P[sel])], wl.camera)
    rend = f32(oracle.unproject(od, wl.camera))
    s = wl.score
    dl = f32(np.random.default_rng(3).normal(1.0, 0.5, len(sel)))
    dr64, ds64, dp64 = oracle.score_grad(obs, rend, s.sigma, s.p_out, s.outlier_volume, s.window, dlogL=dl)
    p = b3d.score_params(s.sigma, s.p_out, s.outlier_volume, s.window)
    for ws in (True, False):  # with the workspace's valid-pixel list, and without
        dr, ds, dp = b3d.score_backward(dev(obs), dev(rend), p, dlogL=dev(dl), workspace=ws)
        dr, ds, dp = dr.cpu().numpy(), ds.cpu().numpy(), dp.cpu().numpy()
        for n in range(len(sel)):
            e = np.linalg.norm(dr[n] - dr64[n])
            assert e <= 1e-3 * np.linalg.norm(dr64[n]) + 1e-6, (n, e)
        np.testing.assert_allclose(ds, ds64, rtol=1e-3, atol=1e-3 * np.abs(ds64).max())
        np.testing.assert_allclose(dp, dp64, rtol=1e-4)


def test_render_backward_matches_oracle(b3d):
    wl, obs, P = workload(0)
    sel = np.arange(0, 256, 16)
    say(f"render_backward parity: config 0, {len(sel)} hypotheses")
    od, oi = oracle.render([(wl.verts, wl.tris, P[sel])], wl.camera)
    rend = oracle.unproject(od, wl.camera)
    s = wl.score
    dr64, _, _ = oracle.score_grad(obs, rend, s.sigma, s.p_out, s.outlier_volume, s.window)
    dr32 = f32(dr64)
    g64 = oracle.render_grad(wl.verts, wl.tris, P[sel], wl.camera, oi, od, dr32)
    mesh = b3d.Mesh(wl.verts, wl.tris)
    g = b3d.render_backward(mesh, dev(P[sel]), b3d.intrinsics_of(wl.camera), dev(oi, torch.int32),
                            dev(dr32)).cpu().numpy()
    for n in range(len(sel)):
        assert np.linalg.norm(g[n] - g64[n]) <= 1e-3 * np.linalg.norm(g64[n]) + 1e-6


@pytest.mark.parametrize("k", [0, 1])
def test_fused_adjoint_matches_oracle(b3d, k):
    wl, obs, P = workload(k)
    sel = np.arange(0, P.shape[0], 8 if k == 0 else 50)
    say(f"fused adjoint parity: config {k}, {len(sel)} hypotheses")
    scene, mesh, o = _scene(b3d, wl, obs)
    Ps = P[sel]
    logL, G = b3d.render_score(scene, dev(Ps), grad=True)
    G = G.cpu().numpy()
    xyz, tri = b3d.render_batch(mesh, dev(Ps), b3d.intrinsics_of(wl.camera))
    s = wl.score
    od, oi = oracle.render([(wl.verts, wl.tris, Ps)], wl.camera)
    rend = oracle.unproject(od, wl.camera)
    dr, ds, dp = oracle.score_grad(obs, rend, s.sigma, s.p_out, s.outlier_volume, s.window)
    gp = oracle.render_grad(wl.verts, wl.tris, Ps, wl.camera, oi, od, dr)
    clean = clean_hypotheses(xyz[..., 2].cpu().numpy(), tri.cpu().numpy(), od, oi)
    say(f"  clean hypotheses {clean.mean():.3f}")
    say(f"  clean fraction {clean.mean():.4f}")
    assert clean.mean() >= 0.99
    for n in np.nonzero(clean)[0]:
        assert np.linalg.norm(G[n, :6] - gp[n]) <= 1e-3 * np.linalg.norm(gp[n]) + 1e-6, (n, G[n, :6], gp[n])
        assert abs(G[n, 6] - ds[n]) <= 1e-3 * abs(ds[n]) + 1e-3
        assert abs(G[n, 7] - dp[n]) <= 1e-4 * abs(dp[n]) + 1e-3


def test_fused_adjoint_at_the_image_border_matches_oracle(b3d):
    # objects straddling each edge and corner of the image: the gather of
    # d logL / d z then clips its window at the border (the clamped path)
    wl, obs, P = workload(0)
    cam = wl.camera
    Q = []
    for n, (u, v) in enumerate([(1.0, cam.cy), (cam.W - 1.0, cam.cy), (cam.cx, 1.0), (cam.cx, cam.H - 1.0),
                                 (0.0, 0.0), (cam.W, cam.H)]):
        q = P[(37 * n) % P.shape[0]].copy()
        z = q[2, 3]
        q[0, 3] = (u - cam.cx) * z / cam.fx
        q[1, 3] = (v - cam.cy) * z / cam.fy
        Q.append(q)
    Q = f32(np.stack(Q))
    say(f"fused adjoint at the border: {len(Q)} hypotheses")
    scene, mesh, o = _scene(b3d, wl, obs)
    logL, G = b3d.render_score(scene, dev(Q), grad=True)
    G = G.cpu().numpy()
    xyz, tri = b3d.render_batch(mesh, dev(Q), b3d.intrinsics_of(cam))
    s = wl.score
    od, oi = oracle.render([(wl.verts, wl.tris, Q)], cam)
    # every pose leaves part of the object outside the image and part inside
    drawn = (oi >= 0).reshape(len(Q), -1).sum(1)
    assert np.all(drawn > 0), drawn
    rend = oracle.unproject(od, cam)
    L64, l1 = oracle.score(obs, rend, s.sigma, s.p_out, s.outlier_volume, s.window)
    dr, ds, dp = oracle.score_grad(obs, rend, s.sigma, s.p_out, s.outlier_volume, s.window)
    gp = oracle.render_grad(wl.verts, wl.tris, Q, cam, oi, od, dr)
    clean = clean_hypotheses(xyz[..., 2].cpu().numpy(), tri.cpu().numpy(), od, oi)
    say(f"  clean {clean.sum()} of {len(Q)}; drawn pixels {drawn.tolist()}")
    assert clean.sum() >= len(Q) - 1
    assert np.max((np.abs(logL.cpu().numpy() - L64) / l1)[clean]) <= LOGL_RTOL
    for n in np.nonzero(clean)[0]:
        assert np.linalg.norm(G[n, :6] - gp[n]) <= 1e-3 * np.linalg.norm(gp[n]) + 1e-6, (n, G[n, :6], gp[n])
        assert abs(G[n, 6] - ds[n]) <= 1e-3 * abs(ds[n]) + 1e-3
        assert abs(G[n, 7] - dp[n]) <= 1e-4 * abs(dp[n]) + 1e-3


def test_enumerate_matches_oracle(b3d):
    wl, _, _ = workload(1)
    g, rots = b3d.grid_of(wl.grid)
    Pg = b3d.enumerate_grid(g).cpu().numpy()
    Po = oracle.enumerate_grid(wl.grid)
    np.testing.assert_allclose(Pg, Po, atol=2e-7)
    from workloads import GridSpec

    spec = GridSpec(center=pose_matrix(np.eye(3), (0.01, -0.02, 0.7)), half_extent=(0.02, 0.01, 0.005),
                    count=(5, 3, 2), cell_centres=True, n_rot=37, rot_max_angle=0.4)
    g2, _ = b3d.grid_of(spec)
    Pg2 = b3d.enumerate_grid(g2, seed=77, stage=3).cpu().numpy()
    Po2 = oracle.enumerate_grid(spec, seed=77, stage=3)
    np.testing.assert_allclose(Pg2, Po2, atol=2e-6)


def test_sampler_matches_oracle(b3d):
    rng = np.random.default_rng(5)
    N, K, seed, stage = 5000, 64, 4001, 2
    L = f32(rng.normal(0, 3, N))
    w, idx, lw = b3d.sample(dev(L), K, seed, stage)
    w, idx, lw = w.cpu().numpy(), idx.cpu().numpy(), lw.cpu().numpy()
    w64, idx64, lw64 = oracle.sample(L, K, seed, stage)
    np.testing.assert_allclose(w, w64, rtol=2e-5, atol=1e-9)
    agree = 0
    for k in range(K):
        G = np.array([-np.log(-np.log(oracle.uniform(seed, n, k, stage, 0))) for n in range(N)])
        v = np.sort(L + G)
        if v[-1] - v[-2] > 1e-4:
            assert idx[k] == idx64[k]
            agree += 1
    assert agree >= K - 1
    np.testing.assert_allclose(lw[idx == idx64], lw64[idx == idx64], atol=1e-4)
    # segmented: P segments with their own counters
    Ls = f32(rng.normal(0, 2, (3, 700)))
    _, i2, _ = b3d.sample(dev(Ls), 1, seed, 1)
    for p in range(3):
        _, ip, _ = oracle.sample(Ls[p], 1, seed, 1, k0=p)
        assert i2[p, 0].item() == ip[0]


def _gumbel(seed, N, draw, stage):
    """The oracle's Gumbel noise of one categorical draw: -ln(-ln u), u from
    the Philox counter (n, draw, stage, 0)."""
    u = np.array([oracle.uniform(seed, n, draw, stage, 0) for n in range(N)])
    return -np.log(-np.log(u))


C2F_DRAW_GAP = 1e-4  # a draw is decided when its top-two gap of logL + G exceeds this times the L1 mass
C2F_LOGQ_RTOL = 1e-5  # log q and log weights, relative to the L1 mass of the scores they come from


def test_c2f_step_matches_oracle(b3d):
    # Three stages, 32 particles, on a posterior flattened (sigma 4 cm,
    # p_out 0.9) so that the particles spread over many cells: the oracle runs
    # its own chain of stages (oracle.c2f), and every particle whose draws so
    # far agree is compared stage by stage: its cell probabilities, and its
    # draw wherever the oracle's top-two gap of logL + Gumbel is above the
    # tolerance; at the end its pose and log q.
    # Both sides must score the same poses: on this object (voxel faces on a
    # 1 cm lattice, seen square on) a pose moved by one FP32 rounding puts
    # hundreds of pixel centres on the other side of an edge (logL moves by up
    # to 1% of its L1 mass), so the schedule uses dyadic offsets around a
    # dyadic centre and explicit rotations: the FP32 enumeration is then exact.
    wl, obs, _ = workload(0)
    from oracle.c2f import c2f
    from oracle.refine import rotvec_exp
    from workloads import GridSpec

    sig, po, V, r = 0.04, 0.9, wl.score.outlier_volume, wl.score.window
    mesh = b3d.Mesh(wl.verts, wl.tris)
    scene = b3d.Scene(mesh, b3d.intrinsics_of(wl.camera), b3d.score_params(sig, po, V, r))
    scene.set_observed(dev(obs))
    rots = f32(np.stack([np.eye(3)] + [rotvec_exp(np.array(w)) for w in
                                       ([0.12, 0, 0], [0, -0.12, 0.05], [0.04, 0.08, -0.1])]))
    centre = pose_matrix(np.eye(3), (2.0 ** -7, -2.0 ** -7, 0.8125))
    st = [GridSpec(center=centre, half_extent=(2.0 ** -4,) * 3, count=(5, 5, 5), rotations=rots),
          GridSpec(center=centre, half_extent=(2.0 ** -6,) * 3, count=(5, 5, 5)),
          GridSpec(center=centre, half_extent=(2.0 ** -8,) * 3, count=(3, 3, 3))]
    K, seed = 32, 4000
    grids = [b3d.grid_of(g) for g in st]  # (grid, rotations tensor): the tensors outlive the call
    sched = b3d.make_schedule([g for g, _ in grids])
    poses, logq, idx, W = b3d.c2f_step(scene, centre, sched, K, seed, weights=True)
    poses, logq, idx = poses.cpu().numpy(), logq.cpu().numpy().astype(np.float64), idx.cpu().numpy()
    W = [w.cpu().numpy().astype(np.float64) for w in W]
    say(f"c2f: {len(st)} stages, K={K}, sigma {sig}, p_out {po}")

    l1_of = {}

    def score_fn(Pq):
        assert np.array_equal(Pq, f32(Pq))  # exact in FP32: both sides score identical poses
        d, _ = oracle.render([(wl.verts, wl.tris, Pq)], wl.camera)
        L, l1 = oracle.score(obs, oracle.unproject(d, wl.camera), sig, po, V, r)
        l1_of[len(l1_of)] = l1
        return L

    P64, lq64, idx64, hist = c2f(score_fn, centre, st, K, seed)
    l1s = [l1_of[0]] + [np.stack([l1_of[1 + (t - 1) * K + k] for k in range(K)]) for t in range(1, len(st))]
    say(f"  gpu paths {len({tuple(c) for c in idx.T.tolist()})} distinct, oracle "
        f"{len({tuple(c) for c in idx64.T.tolist()})} distinct, {len(set(idx64[0].tolist()))} at stage 0")
    assert len({tuple(c) for c in idx64.T.tolist()}) >= 16  # the test is not degenerate
    same = np.ones(K, dtype=bool)  # particles whose draws agree so far
    decided = 0
    lq_bound = np.zeros(K)
    worst_w = 0.0
    for t in range(len(st)):
        for k in range(K):
            if not same[k]:
                continue
            L = hist[t] if t == 0 else hist[t][k]
            l1 = (l1s[t] if t == 0 else l1s[t][k]).max()
            w64 = np.exp(L - L.max())
            w64 /= w64.sum()
            wg = W[t] if t == 0 else W[t][k]
            worst_w = max(worst_w, np.max(np.abs(wg - w64) / (w64 + 1e-30)))
            assert np.all(np.abs(wg - w64) <= C2F_LOGQ_RTOL * l1 * w64 + 1e-7), (t, k)
            v = np.sort(L + _gumbel(seed, L.shape[0], k, t))
            lq_bound[k] += C2F_LOGQ_RTOL * l1
            if v[-1] - v[-2] > C2F_DRAW_GAP * l1:
                assert idx[t, k] == idx64[t, k], (t, k)
                decided += 1
            same[k] &= idx[t, k] == idx64[t, k]
    say(f"  {decided} of {K * len(st)} draws gap-decided; {same.sum()} of {K} particles agree at every stage; "
        f"worst relative weight error {worst_w:.3g}")
    assert decided >= 0.9 * K * len(st)
    assert same.sum() >= 0.9 * K
    np.testing.assert_allclose(poses[same], P64[same], atol=1e-6)
    assert np.all(np.abs(logq[same] - lq64[same]) <= lq_bound[same] + 1e-5)


def test_banded_render_and_fused_path_on_a_large_close_object(b3d):
    # the object covers more pixels than one LDS buffer holds: the kernels
    # process it in bands of rows
    rng = np.random.default_rng(9)
    verts, tris = voxel_mesh(voxel_blob(1500, rng))
    verts = f32(verts)
    cam = Camera(300.0, 300.0, 160.2, 119.7, 240, 320)
    P = f32(random_poses(rng, 24, 0.35, 0.02))
    say("banded parity: 320x240, object at 0.35 m")
    mesh = b3d.Mesh(verts, tris)
    K = b3d.intrinsics_of(cam)
    xyz, tri = b3d.render_batch(mesh, dev(P), K)
    od, oi = oracle.render([(verts, tris, P)], cam)
    frac, dz, ok = render_compare(xyz.cpu().numpy(), tri.cpu().numpy(), od, oi)
    assert frac >= 0.999 and dz <= 1e-5 and ok
    truth = P[0].copy()
    d, _ = oracle.render([(verts, tris, truth)], cam)
    obs = f32(oracle.unproject(d[0] + 0.002 * rng.standard_normal(d[0].shape) * (d[0] > 0), cam))
    scene = b3d.Scene(mesh, K, b3d.score_params(0.003, 0.01, 1.0, 5))
    scene.set_observed(dev(obs))
    Lf, G = b3d.render_score(scene, dev(P), grad=True)
    Lf = Lf.cpu().numpy()
    L64, l1 = oracle.score(obs, oracle.unproject(od, cam), 0.003, 0.01, 1.0, 5)
    clean = clean_hypotheses(xyz[..., 2].cpu().numpy(), tri.cpu().numpy(), od, oi)
    say(f"  clean fraction {clean.mean():.4f}")
    assert clean.mean() >= 0.99
    assert np.max((np.abs(Lf - L64) / l1)[clean]) <= LOGL_RTOL
    Ls = b3d.score(dev(obs), xyz, b3d.score_params(0.003, 0.01, 1.0, 5)).cpu().numpy()
    assert np.max(np.abs(Lf - Ls) / l1) <= 1e-5
    dr, ds, dp = oracle.score_grad(obs, oracle.unproject(od, cam), 0.003, 0.01, 1.0, 5)
    gp = oracle.render_grad(verts, tris, P, cam, oi, od, dr)
    G = G.cpu().numpy()
    for n in np.nonzero(clean)[0]:
        assert np.linalg.norm(G[n, :6] - gp[n]) <= 1e-3 * np.linalg.norm(gp[n]) + 1e-6


def test_static_background_scene_matches_oracle(b3d):
    rng = np.random.default_rng(12)
    va, ta = voxel_mesh(voxel_blob(300, rng, radius=0.06))
    vb, tb = voxel_mesh(voxel_blob(200, rng, radius=0.05))
    va, vb = f32(va), f32(vb)
    cam = Camera(150.0, 150.0, 80.0, 60.0, 120, 160)
    Pb = f32(random_poses(rng, 1, 0.75, 0.0)[0])
    Pb[:3, 3] = [0.05, 0.02, 0.75]
    truth = f32(random_poses(rng, 1, 0.8, 0.0)[0])
    truth[:3, 3] = [-0.02, 0.0, 0.8]
    d, _ = oracle.render([(va, ta, truth), (vb, tb, Pb)], cam)
    obs = f32(oracle.unproject(d[0] + 0.002 * rng.standard_normal(d[0].shape) * (d[0] > 0), cam))
    P = f32(random_poses(rng, 64, 0.8, 0.04))
    say("background scene parity: 2 objects, 64 hypotheses")
    ma, mb = b3d.Mesh(va, ta), b3d.Mesh(vb, tb)
    K = b3d.intrinsics_of(cam)
    # the static object alone must render as the oracle does
    xb, tb_ = b3d.render_batch(mb, dev(Pb[None]), K)
    odb, oib = oracle.render([(vb, tb, Pb)], cam)
    assert clean_hypotheses(xb[..., 2].cpu().numpy(), tb_.cpu().numpy(), odb, oib).all()
    scene = b3d.Scene(ma, K, b3d.score_params(0.003, 0.01, 1.0, 5))
    scene.set_background([mb], Pb[None])
    scene.set_observed(dev(obs))
    Lf, G = b3d.render_score(scene, dev(P), grad=True)
    xa, ta_ = b3d.render_batch(ma, dev(P), K)
    oda, oia = oracle.render([(va, ta, P)], cam)
    clean = clean_hypotheses(xa[..., 2].cpu().numpy(), ta_.cpu().numpy(), oda, oia)
    od, oi = oracle.render([(va, ta, P), (vb, tb, Pb)], cam)
    L64, l1 = oracle.score(obs, oracle.unproject(od, cam), 0.003, 0.01, 1.0, 5)
    err = np.abs(Lf.cpu().numpy() - L64) / l1
    say(f"  clean {clean.mean():.3f}; max rel-L1 err (clean) {err[clean].max():.3g}")
    say(f"  clean fraction {clean.mean():.4f}")
    assert clean.mean() >= 0.99 and err[clean].max() <= LOGL_RTOL
    dr, ds, dp = oracle.score_grad(obs, oracle.unproject(od, cam), 0.003, 0.01, 1.0, 5)
    G = G.cpu().numpy()
    np.testing.assert_allclose(G[clean, 7], dp[clean], rtol=1e-3)
    np.testing.assert_allclose(G[clean, 6], ds[clean], rtol=2e-3, atol=1e-3 * np.abs(ds).max())
    gp = oracle.render_grad(va, ta, P, cam, oi, od, dr)
    for n in np.nonzero(clean)[0]:
        assert np.linalg.norm(G[n, :6] - gp[n]) <= 1e-3 * np.linalg.norm(gp[n]) + 1e-6


def _midpoints(b3d, sigma_max, A, B):
    """The oracle's midpoint nodes; the library's (b3d_noise_midpoints) must
    be their FP32 values."""
    from oracle.noise import midpoints

    sig, po = midpoints(sigma_max, A, B)
    gs, gp = b3d.noise_grid_midpoints(sigma_max, A, B)
    assert np.array_equal(gs, sig.astype(np.float32)) and np.array_equal(gp, po.astype(np.float32))
    return sig, po


def _grid_compare(b3d, scene, P, obs, rend64, clean, sig, po, V, window):
    """GPU noise-grid logL and marginal vs the oracle's on FP64 renders."""
    from oracle.noise import score_grid

    sig32, po32 = f32(sig), f32(po)
    scene.set_noise_grid(sig32, po32)
    marg, Lg = b3d.render_score_marginal(scene, dev(P), grid=True)
    marg, Lg = marg.cpu().numpy().astype(np.float64), Lg.cpu().numpy().astype(np.float64)
    L64, marg64 = score_grid(obs, rend64, sig32, po32, V=V, window=window)
    l1 = np.stack([np.stack([oracle.score(obs, rend64, float(s), float(p), V, window)[1] for p in po32], -1)
                   for s in sig32], -2)
    err = np.abs(Lg - L64) / l1
    say(f"  noise grid {len(sig)}x{len(po)}: max rel-L1 err per point (clean) {err[clean].max():.3g}")
    assert err[clean].max() <= LOGL_RTOL
    assert np.all(np.abs(marg - marg64)[clean] <= LOGL_RTOL * l1.max(axis=(1, 2))[clean])
    # bitwise repeatable, and the marginal is the weighted log-sum-exp of the grid values
    assert np.array_equal(b3d.render_score_marginal(scene, dev(P)).cpu().numpy(), marg.astype(np.float32))
    lse = np.log(np.exp(Lg.reshape(len(P), -1) - Lg.max(axis=(1, 2))[:, None]).sum(1) / Lg[0].size) + Lg.max(axis=(1, 2))
    assert np.allclose(marg, lse, rtol=0, atol=1e-3 + 1e-6 * np.abs(lse))


def test_noise_grid_marginal_matches_oracle(b3d):
    wl, obs, P = workload(0)
    say(f"noise grid parity: config 0, {P.shape[0]} hypotheses")
    scene, mesh, o = _scene(b3d, wl, obs)
    xyz, tri = b3d.render_batch(mesh, dev(P), b3d.intrinsics_of(wl.camera))
    L64, l1, oid, od = _oracle_logL(wl, obs, P)
    clean = clean_hypotheses(xyz[..., 2].cpu().numpy(), tri.cpu().numpy(), od, oid)
    say(f"  clean fraction {clean.mean():.4f}")
    assert clean.mean() >= 0.99
    s = wl.score
    # deviation counts the kernel compiles for (2, 3) and the general path (6)
    for A, B in ((3, 3), (2, 3), (6, 2)):
        sig, po = _midpoints(b3d, 0.012, A, B)
        say(f"  grid {A} x {B}")
        _grid_compare(b3d, scene, P, obs, oracle.unproject(od, wl.camera), clean, sig, po, s.outlier_volume,
                      s.window)
    # a grid of one point is the plain score
    scene.set_noise_grid([s.sigma], [s.p_out], log_w=[[0.0]])
    m1 = b3d.render_score_marginal(scene, dev(P)).cpu().numpy().astype(np.float64)
    assert np.max(np.abs(m1 - b3d.render_score(scene, dev(P)).cpu().numpy()) / l1) <= 1e-5
    # limits of the grid are refused
    with pytest.raises(b3d.B3DError):
        scene.set_noise_grid(np.full(9, 0.005), [0.1])
    with pytest.raises(b3d.B3DError):
        scene.set_noise_grid([0.005, 0.006, 0.007], np.full(6, 0.1))


def test_noise_grid_at_paper_scale_matches_oracle_on_sampled_hypotheses(b3d):
    # the launch the bench times: 4 x 4 grid over all 5000 hypotheses
    wl, obs, P = workload(1)
    say(f"noise grid parity: config 1, N={P.shape[0]}, 4x4 grid, every 25th hypothesis checked")
    scene, mesh, o = _scene(b3d, wl, obs)
    sig, po = _midpoints(b3d, 0.01, 4, 4)
    scene.set_noise_grid(f32(sig), f32(po))
    marg, Lg = b3d.render_score_marginal(scene, dev(P), grid=True)
    sel = np.arange(0, P.shape[0], 25)
    sub, _, _ = _scene(b3d, wl, obs, mesh=mesh)
    xyz, tri = b3d.render_batch(mesh, dev(P[sel]), b3d.intrinsics_of(wl.camera))
    _, _, oid, od = _oracle_logL(wl, obs, P[sel])
    clean = clean_hypotheses(xyz[..., 2].cpu().numpy(), tri.cpu().numpy(), od, oid)
    say(f"  clean fraction {clean.mean():.4f}")
    assert clean.mean() >= 0.99
    s = wl.score
    _grid_compare(b3d, sub, P[sel], obs, oracle.unproject(od, wl.camera), clean, sig, po, s.outlier_volume, s.window)
    # the full launch agrees with the launch over the sample, bit for bit
    m_sub, L_sub = b3d.render_score_marginal(sub, dev(P[sel]), grid=True)
    assert torch.equal(marg[torch.as_tensor(sel, device="cuda")], m_sub)
    assert torch.equal(Lg[torch.as_tensor(sel, device="cuda")], L_sub)
    # and bands of two rows give the same bits as the default depth-buffer tile
    lo, _, _ = sub.tile_limits()
    sub.set_tile(lo)
    m_lo, L_lo = b3d.render_score_marginal(sub, dev(P[sel]), grid=True)
    assert torch.equal(m_lo, m_sub) and torch.equal(L_lo, L_sub)


def test_noise_grid_with_static_background_matches_oracle(b3d):
    rng = np.random.default_rng(13)
    va, ta = voxel_mesh(voxel_blob(300, rng, radius=0.06))
    vb, tb = voxel_mesh(voxel_blob(200, rng, radius=0.05))
    va, vb = f32(va), f32(vb)
    cam = Camera(150.0, 150.0, 80.0, 60.0, 120, 160)
    Pb = f32(random_poses(rng, 1, 0.75, 0.0)[0])
    Pb[:3, 3] = [0.05, 0.02, 0.75]
    truth = f32(random_poses(rng, 1, 0.8, 0.0)[0])
    truth[:3, 3] = [-0.02, 0.0, 0.8]
    d, _ = oracle.render([(va, ta, truth), (vb, tb, Pb)], cam)
    obs = f32(oracle.unproject(d[0] + 0.002 * rng.standard_normal(d[0].shape) * (d[0] > 0), cam))
    P = f32(random_poses(rng, 48, 0.8, 0.04))
    say("noise grid with background: 2 objects, 48 hypotheses")
    ma, mb = b3d.Mesh(va, ta), b3d.Mesh(vb, tb)
    K = b3d.intrinsics_of(cam)
    scene = b3d.Scene(ma, K, b3d.score_params(0.003, 0.01, 1.0, 5))
    scene.set_background([mb], Pb[None])
    scene.set_observed(dev(obs))
    xa, ta_ = b3d.render_batch(ma, dev(P), K)
    oda, oia = oracle.render([(va, ta, P)], cam)
    clean = clean_hypotheses(xa[..., 2].cpu().numpy(), ta_.cpu().numpy(), oda, oia)
    od, oi = oracle.render([(va, ta, P), (vb, tb, Pb)], cam)
    sig, po = _midpoints(b3d, 0.01, 4, 4)
    _grid_compare(b3d, scene, P, obs, oracle.unproject(od, cam), clean, sig, po, 1.0, 5)


def test_edge_cases(b3d):
    wl, obs, P = workload(0)
    mesh = b3d.Mesh(wl.verts, wl.tris)
    K = b3d.intrinsics_of(wl.camera)
    scene, _, o = _scene(b3d, wl, obs, mesh)
    # N = 0 is a no-op
    e = torch.empty((0, 4, 4), device="cuda")
    assert b3d.render_score(scene, e).numel() == 0
    # object behind the camera or far outside the view renders nothing
    Q = P[:3].copy()
    Q[0, 2, 3] = -0.8
    Q[1, 0, 3] = 5.0
    Q[2, 2, 3] = 0.005  # straddles the near plane: triangles crossing it are dropped
    xyz, tri = b3d.render_batch(mesh, dev(Q), K)
    od, oi = oracle.render([(wl.verts, wl.tris, Q)], wl.camera)
    assert np.array_equal(tri.cpu().numpy()[:2], oi[:2]) and np.all(oi[:2] == -1)
    assert np.all(xyz.cpu().numpy()[:2] == 0)
    # triangles a few millimetres from the camera project to thousands of
    # pixels, where single-precision edge functions flip more centres
    frac, dz, ok = render_compare(xyz.cpu().numpy()[2:], tri.cpu().numpy()[2:], od[2:], oi[2:])
    say(f"  near-plane pose: id agreement {frac:.5f}")
    assert frac >= 0.99 and ok
    L = b3d.render_score(scene, dev(Q)).cpu().numpy()
    s = wl.score
    L64, l1 = oracle.score(obs, oracle.unproject(od, wl.camera), s.sigma, s.p_out, s.outlier_volume, s.window)
    assert np.max((np.abs(L - L64) / l1)[:2]) <= LOGL_RTOL
    # ragged batch sizes
    for n in (1, 3, 257):
        Pn = P[np.arange(n) % P.shape[0]]
        Ln = b3d.render_score(scene, dev(Pn)).cpu().numpy()
        L0 = b3d.render_score(scene, dev(P)).cpu().numpy()
        assert np.array_equal(Ln, L0[np.arange(n) % P.shape[0]])
    # the fused kernel's limits: a very wide image, or rays beyond |x/z| = 1e3, are refused
    with pytest.raises(b3d.B3DError):
        b3d.Scene(mesh, b3d.Intrinsics(600.0, 600.0, 1024.0, 60.0, 0.01, 120, 2048), b3d.score_params(0.003, 0.01, 1.0, 5))
    with pytest.raises(b3d.B3DError):
        b3d.Scene(mesh, b3d.Intrinsics(0.05, 0.05, 80.0, 60.0, 0.01, 120, 160), b3d.score_params(0.003, 0.01, 1.0, 5))
    # invalid arguments are rejected before any launch
    with pytest.raises(b3d.B3DError):
        b3d.score(o, xyz, b3d.score_params(wl.score.sigma, 0.0, 1.0, 3))
    with pytest.raises(b3d.B3DError):
        b3d.score(o, xyz, b3d.score_params(wl.score.sigma, 0.1, 1.0, 4))


def test_multi_scene_batch_equals_per_scene_calls(b3d):
    # scenes of different image sizes, meshes and hypothesis counts in
    # launches of up to eight scenes each (here two, on two streams): every
    # result equals the per-scene call's bit for bit (the per-hypothesis body
    # is the same and no result depends on the tile the batch caps), run
    # eagerly twice and replayed from a captured graph with eager work in
    # between
    rng = np.random.default_rng(21)
    items, refs, keep = [], [], []
    sizes = [(120, 160), (180, 240), (240, 320), (120, 160), (180, 240), (120, 160), (240, 320), (120, 160),
             (180, 240), (120, 160), (120, 160)]
    for k, (H, W) in enumerate(sizes):
        v, t = voxel_mesh(voxel_blob(int(rng.integers(300, 1500)), rng))
        cam = Camera(W * 0.9375, W * 0.9375, W / 2, H / 2, H, W)
        truth = random_poses(rng, 1, 0.8, 0.0)[0]
        d, _ = oracle.render([(v, t, truth)], cam)
        obs = oracle.unproject(d[0] + 0.002 * rng.standard_normal(d[0].shape) * (d[0] > 0), cam)
        m = b3d.Mesh(v, t)
        sc = b3d.Scene(m, b3d.intrinsics_of(cam), b3d.score_params(0.003, 0.01, 1.0, 5))
        o = dev(obs)
        sc.set_observed(o)
        P = random_poses(rng, int(rng.integers(20, 200)), 0.8, 0.03)
        P[:, :3, :3] = truth[:3, :3]
        Pd = dev(P)
        keep += [m, o]
        items.append((sc, Pd))
        refs.append(b3d.render_score(sc, Pd, grad=True))
    say(f"batch: {len(items)} scenes, {sum(p.shape[0] for _, p in items)} hypotheses")
    batch = b3d.Batch(items, grad=True)
    L, G = batch.run()
    torch.cuda.synchronize()
    for k, ((Lr, Gr), Lb, Gb) in enumerate(zip(refs, L, G)):
        assert torch.equal(Lb, Lr) and torch.equal(Gb, Gr), f"scene {k}: batch differs from the per-scene call"
    say("  batch results bitwise equal to per-scene calls")
    L2, _ = batch.run()
    torch.cuda.synchronize()
    for a, (Lr, _) in zip(L2, refs):
        assert torch.equal(a, Lr)
    for a in L:
        a.fill_(0.0)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        batch.run()
    for rep in range(3):
        x = b3d.render_score(items[0][0], items[0][1])  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        ok = all(torch.equal(Lb, Lr) and torch.equal(Gb, Gr) for (Lr, Gr), Lb, Gb in zip(refs, L, G))
        say(f"  graph replay {rep}: equal to the per-scene calls {ok}")
        assert ok and torch.equal(x, refs[0][0])


def _batch_scene(rng, H, W, vox):
    """A scene of the many-scenes mix: object 0 (the moving one) 0.8 m ahead,
    the others as static background at seeded poses, observed through the
    oracle's FP64 render with 2 mm noise and 3% outliers."""
    from workloads import observation_noise, pose_matrix, shoemake_rotations

    cam = Camera(W * 0.9375, W * 0.9375, W / 2.0, H / 2.0, H, W)
    objs = []
    for k, nv in enumerate(vox):
        v, t = voxel_mesh(voxel_blob(nv, rng))
        pos = (0.0, 0.0, 0.8) if k == 0 else (rng.uniform(-0.2, 0.2), rng.uniform(-0.15, 0.15),
                                              rng.uniform(0.8, 1.2))
        objs.append((f32(v), t, f32(pose_matrix(shoemake_rotations(1, rng)[0], pos))))
    nz = observation_noise(H, W, rng, 0.002, 0.03)
    d = oracle.render(objs, cam)[0][0]
    d = np.where(d > 0, d + nz["gauss"], 0.0)
    d = np.where(nz["outlier_mask"], nz["outlier_depth"], d)
    return objs, cam, f32(oracle.unproject(d, cam))


def test_multi_scene_batch_matches_oracle(b3d):
    # The many-scenes mix as one batch: two scenes of each image
    # size (160x120, 240x180, 320x240) with 2-4 objects, the others drawn as
    # static background; hypotheses of object 0 on the benchmark's grid
    # (10x10 translations over +-2 cm x layers x 10 rotations within 10
    # degrees).  Forward + adjoint of 100 sampled hypotheses per scene (200
    # per image size) against the oracle's composite render, score and
    # gradients; every hypothesis checked for logL on identical-id
    # hypotheses, gradients likewise.
    from workloads import GridSpec

    rng = np.random.default_rng(303)
    shapes = [(120, 160, [2000, 700]), (180, 240, [1200, 900, 600]), (240, 320, [1500, 500, 800, 1000]),
              (120, 160, [900, 1500, 500, 600]), (180, 240, [2500, 800]), (240, 320, [700, 2000, 600])]
    sc_p = (0.003, 0.01, 1.0, 5)
    items, keep, cases = [], [], []
    for i, (H, W, vox) in enumerate(shapes):
        objs, cam, obs = _batch_scene(rng, H, W, vox)
        meshes = [b3d.Mesh(v, t) for v, t, _ in objs]
        scene = b3d.Scene(meshes[0], b3d.intrinsics_of(cam), b3d.score_params(*sc_p))
        scene.set_background(meshes[1:], np.stack([P for _, _, P in objs[1:]]))
        o = dev(obs)
        scene.set_observed(o)
        nz = int(rng.integers(1, 4))
        spec = GridSpec(center=objs[0][2], half_extent=(0.02, 0.02, 0.02), count=(10, 10, nz), n_rot=10,
                        rot_max_angle=np.deg2rad(10.0))
        P = f32(oracle.enumerate_grid(spec, seed=3003 + i, stage=0))
        items.append((scene, dev(P)))
        keep += [meshes, o]
        cases.append((objs, cam, obs, P))
    say(f"batch vs oracle: {len(items)} scenes, {sum(c[3].shape[0] for c in cases)} hypotheses")
    batch = b3d.Batch(items, grad=True)
    Lb, Gb = batch.run()
    torch.cuda.synchronize()
    for (objs, cam, obs, P), (sc, Pd), L, G in zip(cases, items, Lb, Gb):
        sel = np.sort(rng.choice(P.shape[0], 100, replace=False))
        Ps = P[sel]
        v0, t0, _ = objs[0]
        od, oi = oracle.render([(v0, t0, Ps)] + [(v, t, Q) for v, t, Q in objs[1:]], cam)
        rend = oracle.unproject(od, cam)
        L64, l1 = oracle.score(obs, rend, *sc_p)
        dr, ds, dp = oracle.score_grad(obs, rend, *sc_p)
        gp = oracle.render_grad(v0, t0, Ps, cam, oi, od, dr)
        # identical ids: the GPU's render of object 0 against the oracle's
        xa, ta = b3d.render_batch(sc.mesh, dev(Ps), b3d.intrinsics_of(cam))
        oda, oia = oracle.render([(v0, t0, Ps)], cam)
        clean = clean_hypotheses(xa[..., 2].cpu().numpy(), ta.cpu().numpy(), oda, oia)
        Lg = L.cpu().numpy()[sel].astype(np.float64)
        Gg = G.cpu().numpy()[sel].astype(np.float64)
        err = np.abs(Lg - L64) / l1
        say(f"  {cam.W}x{cam.H}, {len(objs)} objects, N={P.shape[0]}: clean {clean.mean():.3f}, "
            f"max rel-L1 logL err (clean) {err[clean].max():.3g}")
        assert clean.mean() >= 0.99 and err[clean].max() <= LOGL_RTOL
        for n in np.nonzero(clean)[0]:
            assert np.linalg.norm(Gg[n, :6] - gp[n]) <= 1e-3 * np.linalg.norm(gp[n]) + 1e-6, (n, Gg[n, :6], gp[n])
            assert abs(Gg[n, 6] - ds[n]) <= 1e-3 * abs(ds[n]) + 1e-3
            assert abs(Gg[n, 7] - dp[n]) <= 1e-4 * abs(dp[n]) + 1e-3


def test_adam_pose_step_matches_oracle(b3d):
    from oracle.refine import adam_pose_step

    rng = np.random.default_rng(31)
    P = f32(random_poses(rng, 40, 0.8, 0.03))
    g = f32(rng.normal(0, 1e4, (40, 8)))
    st = np.zeros((40, 12))
    Pd, gd, sd = dev(P), dev(g), dev(st)
    b1, b2, eps = (float(np.float32(x)) for x in (0.9, 0.999, 1e-8))
    lr_t, lr_r = float(np.float32(1e-3)), float(np.float32(1e-2))
    for it in (1, 2, 3):
        b3d.adam_pose_step(Pd, gd, sd, it, lr_t, lr_r, b1, b2, eps)
        P, st = adam_pose_step(P, g, st, it, lr_t, lr_r, b1, b2, eps)
    np.testing.assert_allclose(Pd.cpu().numpy(), P, atol=2e-6)
    np.testing.assert_allclose(sd.cpu().numpy(), st, rtol=1e-5, atol=1e-3)


def test_refine_poses_equals_score_and_adam_launched_in_turn(b3d):
    wl, obs, P = workload(0)
    sel = np.arange(0, P.shape[0], 32)
    say(f"refine_poses: config 0, {len(sel)} poses, 6 steps")
    scene, mesh, o = _scene(b3d, wl, obs)
    b1, b2, eps = 0.9, 0.999, 1e-8
    A = dev(P[sel])
    b3d.refine_poses(scene, A, 6, 1e-3, 1e-2, b1, b2, eps)
    B = dev(P[sel])
    st = torch.zeros((len(sel), 12), dtype=torch.float32, device="cuda")
    for it in range(1, 7):
        _, G = b3d.render_score(scene, B, grad=True)
        b3d.adam_pose_step(B, G, st, it, 1e-3, 1e-2, b1, b2, eps)
    np.testing.assert_allclose(A.cpu().numpy(), B.cpu().numpy(), rtol=0, atol=1e-6)
    # the steps moved the poses
    assert not np.allclose(A.cpu().numpy(), P[sel])


def test_refine_poses_follows_the_oracle_adam_chain(b3d):
    # Eight Adam steps on logL from FP32 start poses, in lockstep with the
    # oracle's chain (FP64 render, score, pose gradient and Adam): at every
    # step the GPU's fused gradient at the oracle's current poses (rounded to
    # FP32) against the oracle's, and the GPU's Adam update from the oracle's
    # state against the oracle's update.  The two chains are not compared
    # free-running: logL is only piecewise smooth in the pose (a pixel changes
    # triangle where an edge crosses its centre; on this object's lattice of
    # voxel faces many centres lie exactly on edges), so poses that differ by
    # one rounding can take different steps.  The one-workgroup refinement
    # (b3d_refine_poses) is compared over one step, from the same start, and
    # equals the launch-by-launch chain (the test below).
    from oracle.refine import adam_pose_step

    wl, obs, P = workload(0)
    s = wl.score
    sel = np.arange(0, P.shape[0], 11)
    n = 8
    c32 = [float(np.float32(x)) for x in (1e-3, 1e-2, 0.9, 0.999, 1e-8)]
    say(f"refine vs oracle Adam chain: config 0, {len(sel)} poses, {n} steps in lockstep")
    scene, mesh, o = _scene(b3d, wl, obs)
    Q = P[sel].copy()
    st = np.zeros((len(sel), 12))
    worst_g, worst_p, n_clean = 0.0, 0.0, 0
    K = b3d.intrinsics_of(wl.camera)
    for it in range(1, n + 1):
        od, oi = oracle.render([(wl.verts, wl.tris, Q)], wl.camera)
        rend = oracle.unproject(od, wl.camera)
        dr, _, _ = oracle.score_grad(obs, rend, s.sigma, s.p_out, s.outlier_volume, s.window)
        g64 = oracle.render_grad(wl.verts, wl.tris, Q, wl.camera, oi, od, dr)
        _, G = b3d.render_score(scene, dev(Q), grad=True)
        G = G.cpu().numpy().astype(np.float64)
        xyz, tri = b3d.render_batch(mesh, dev(Q), K)
        clean = clean_hypotheses(xyz[..., 2].cpu().numpy(), tri.cpu().numpy(), od, oi)
        n_clean += clean.sum()
        for m in np.nonzero(clean)[0]:
            e = np.linalg.norm(G[m, :6] - g64[m])
            assert e <= 1e-3 * np.linalg.norm(g64[m]) + 1e-6, (it, m, G[m, :6], g64[m])
            worst_g = max(worst_g, e / np.linalg.norm(g64[m]))
        Qn, stn = adam_pose_step(Q, g64, st, it, *c32)
        Qd, sd = dev(Q), dev(st)
        b3d.adam_pose_step(Qd, dev(g64), sd, it, *c32)
        dp = np.abs(Qd.cpu().numpy() - Qn).max()
        worst_p = max(worst_p, dp)
        assert dp <= 2e-6, (it, dp)
        if it == 1:  # the one-workgroup refinement's first step from the same start
            A = dev(Q)
            b3d.refine_poses(scene, A, 1, *c32)
            d1 = np.abs(A.cpu().numpy() - Qn).max()
            say(f"  refine_poses, one step: max pose diff {d1:.3g}")
            assert d1 <= 2e-6
        Q, st = f32(Qn), f32(stn)
    say(f"  worst relative gradient error {worst_g:.3g} over {n_clean} clean (pose, step) pairs; "
        f"worst Adam update diff {worst_p:.3g}")
    assert n_clean >= 0.99 * len(sel) * n
    moved = np.abs(Q - P[sel]).reshape(len(sel), -1).max(1)
    assert moved.min() >= 1e-2
    # What the eight steps buy: logL at the chain's end minus at its start,
    # by the GPU and by the oracle.  Adam on this piecewise-smooth logL does
    # not raise it for every pose (the oracle's own chain raises 19 of these
    # 24, median +40, worst -27), so the GPU's gains are held to the
    # oracle's rather than each required to be positive.
    def oracle_logL(X):
        od, oi = oracle.render([(wl.verts, wl.tris, X)], wl.camera)
        L, l1 = oracle.score(obs, oracle.unproject(od, wl.camera), s.sigma, s.p_out, s.outlier_volume, s.window)
        xyz, tri = b3d.render_batch(mesh, dev(X), K)
        return L, l1, clean_hypotheses(xyz[..., 2].cpu().numpy(), tri.cpu().numpy(), od, oi)
    (L0, l1a, c0), (L8, l1b, c8) = oracle_logL(f32(P[sel])), oracle_logL(Q)
    gpu = (b3d.render_score(scene, dev(Q)) - b3d.render_score(scene, dev(P[sel]))).cpu().numpy().astype(np.float64)
    both = c0 & c8
    bar = LOGL_RTOL * (l1a + l1b)
    assert both.sum() >= len(sel) - 1  # ids equal to the oracle's at both ends, but for at most one pose
    assert np.all(np.abs(gpu - (L8 - L0))[both] <= bar[both]), np.abs(gpu - (L8 - L0))[both].max()
    assert (L8 > L0).mean() >= 0.75
    say(f"  logL raised for {(gpu > 0).sum()} of {len(sel)} poses (oracle {(L8 > L0).sum()}); median gain "
        f"{np.median(gpu):.1f}")


def test_tracker_graph_replays_match_eager_frames_and_follow_the_objects(b3d):
    from workloads import assemble_observed_depth, tracking_sequence, Workload, ScoreParams, GridSpec

    meshes, paths, cam, noise = tracking_sequence(seed=77, n_frames=6, n_obj=2, vox_range=(300, 600))
    meshes = [(f32(v), t) for v, t in meshes]
    F, M = paths.shape[:2]
    say(f"tracker: {M} objects, {F} frames")
    frames = []
    for f in range(F):
        objs = [(v, t, paths[f, k]) for k, (v, t) in enumerate(meshes)]
        d = oracle.render(objs, cam)[0][0]
        d = np.where(d > 0, d + noise[f]["gauss"], 0.0)
        d = np.where(noise[f]["outlier_mask"], noise[f]["outlier_depth"], d)
        frames.append(dev(f32(oracle.unproject(d, cam))))
    ms = [b3d.Mesh(v, t) for v, t in meshes]
    K = b3d.intrinsics_of(cam)
    p = b3d.score_params(0.003, 0.01, 1.0, 5)
    grid = [b3d.make_grid(np.eye(4), (0.02, 0.02, 0.02), (6, 6, 6), n_rot=8, rot_max_angle=np.deg2rad(5.0)),
            b3d.make_grid(np.eye(4), (0.005, 0.005, 0.005), (3, 3, 3), n_rot=8, rot_max_angle=np.deg2rad(2.0))]
    init = f32(paths[0])
    tg = b3d.Tracker(ms, K, p, grid, init, n_refine=5)
    te = b3d.Tracker(ms, K, p, grid, init, n_refine=5)
    for f in range(1, F):
        tg.frame(frames[f])
        torch.cuda.synchronize()
        te.frame(frames[f], eager=True)
        torch.cuda.synchronize()
        a, b = tg.poses().cpu().numpy(), te.poses().cpu().numpy()
        np.testing.assert_array_equal(a, b)
    est = tg.poses().cpu().numpy()
    for k in range(M):
        err_t = np.linalg.norm(est[k, :3, 3] - paths[-1, k, :3, 3])
        dR = est[k, :3, :3] @ paths[-1, k, :3, :3].T
        err_r = np.degrees(np.arccos(np.clip((np.trace(dR) - 1) / 2, -1, 1)))
        say(f"  object {k}: position error {err_t * 100:.3f} cm, orientation error {err_r:.3f} deg")
        assert err_t < 0.01 and err_r < 5.0
    # checkpoint and resume: a frame's state is the objects' poses (the
    # refinement's moments start from zero every frame), so a tracker created
    # from poses saved after frame 2 continues bit for bit like the original
    tc = b3d.Tracker(ms, K, p, grid, init, n_refine=5)
    for f in range(1, 3):
        tc.frame(frames[f])
    saved = tc.poses().cpu().numpy()
    tr = b3d.Tracker(ms, K, p, grid, saved, n_refine=5)
    for f in range(3, F):
        tc.frame(frames[f])
        tr.frame(frames[f])
        torch.cuda.synchronize()
        np.testing.assert_array_equal(tc.poses().cpu().numpy(), tr.poses().cpu().numpy())
    np.testing.assert_array_equal(tr.poses().cpu().numpy(), est)


def _oracle_stage_best(verts, tris, cam, obs, s, spec, stage, center, tol_rel):
    """Poses of a stage's hypotheses around `center` and the indices whose
    oracle log-likelihood is within tol_rel * L1 of the best, best first."""
    P = oracle.enumerate_grid(spec, seed=0, stage=stage, center=center)
    d, _ = oracle.render([(verts, tris, P)], cam)
    L, l1 = oracle.score(obs, oracle.unproject(d, cam), s.sigma, s.p_out, s.outlier_volume, s.window)
    order = np.argsort(-L, kind="stable")
    ok = [int(j) for j in order if L[j] >= L[order[0]] - tol_rel * l1[j]]
    return P, ok


def _oracle_frame_ends(verts, tris, cam, obs, s, specs, center, tol_rel, stage=0, limit=3):
    """Poses a frame of argmax-per-stage search can end on when near ties
    (within the tolerance) may go either way, the all-best path first."""
    P, ok = _oracle_stage_best(verts, tris, cam, obs, s, specs[stage], stage, center, tol_rel)
    ends = []
    for j in ok[:limit]:
        nxt = f32(P[j]).astype(np.float64)  # the tracker keeps its poses in float32
        ends += [nxt] if stage + 1 == len(specs) else _oracle_frame_ends(verts, tris, cam, obs, s, specs, nxt,
                                                                         tol_rel, stage + 1, limit)
    return ends


@pytest.mark.parametrize("res", [25, 50])
def test_camera_pan_tracker_takes_the_oracles_best_hypothesis_every_stage(b3d, res):
    # a camera circling an object on a table, tracked with four stages of
    # hypotheses per frame and no gradient steps: the oracle runs the same
    # argmax-per-stage search from the known first pose, and every GPU frame
    # must land on the pose the oracle's search ends on; where a stage holds a
    # near tie (within the score tolerance) either candidate is correct, so the
    # oracle follows each tied branch and the GPU's pose must equal the end of
    # one of them, whose (oracle-computed) pose the oracle then continues from
    from workloads import ScoreParams, camera_pan_schedule, camera_pan_sequence

    F = 10
    (v, t), truth, cam, noise = camera_pan_sequence(res=res, n_frames=120)  # its first F frames
    v = f32(v)
    say(f"camera pan tracker: {res}x{res}, {t.shape[0]} triangles, {F} frames")
    s = ScoreParams(sigma=0.003, p_out=0.01, outlier_volume=1.0, window=5)
    frames = []
    for f in range(F):
        d = oracle.render([(v, t, truth[f])], cam)[0][0]
        d = np.where(d > 0, d + noise[f]["gauss"], 0.0)
        d = np.where(noise[f]["outlier_mask"], noise[f]["outlier_depth"], d)
        frames.append(f32(oracle.unproject(d, cam)))
    specs = camera_pan_schedule()
    for g in specs:
        g.rotations = f32(g.rotations).astype(np.float64)  # both sides use the float32 rotations the GPU reads
    grids = [b3d.grid_of(g) for g in specs]  # (grid, rotations tensor): the tensors outlive the tracker
    tr = b3d.Tracker([b3d.Mesh(v, t)], b3d.intrinsics_of(cam), b3d.score_params(s.sigma, s.p_out, s.outlier_volume,
                                                                               s.window),
                     [g for g, _ in grids], f32(truth[:1]), n_refine=0)
    cur = f32(truth[0]).astype(np.float64)
    off_best = 0
    for f in range(1, F):
        tr.frame(dev(frames[f]))
        g = tr.poses().cpu().numpy()[0].astype(np.float64)
        ends = _oracle_frame_ends(v, t, cam, frames[f].astype(np.float64), s, specs, cur, LOGL_RTOL)
        hit = [e for e in ends if np.allclose(e, g, atol=1e-5)]
        assert hit, f"frame {f}: the GPU's pose is none of the ends of the oracle's search"
        off_best += int(hit[0] is not ends[0])
        cur = hit[0]
    say(f"  {F - 1} frames; {off_best} took a tied candidate other than the oracle's first")
    err_t = np.linalg.norm(cur[:3, 3] - truth[F - 1, :3, 3])
    err_r = np.degrees(np.arccos(np.clip((np.trace(cur[:3, :3] @ truth[F - 1, :3, :3].T) - 1) / 2, -1, 1)))
    say(f"  last frame: scene origin off by {err_t * 100:.3f} cm, orientation by {err_r:.3f} deg")
    assert err_t < 0.005 and err_r < 3.0


def test_hot_calls_replay_from_a_captured_graph(b3d):
    # enumerate -> fused render + score + adjoint -> sample, captured once into a
    # graph and replayed several times with eager work in between: every replay
    # must equal the eager results bit for bit (the calls launch only on the
    # caller's stream, allocate nothing and issue no memset)
    wl, obs, P = workload(1)
    scene, mesh, o = _scene(b3d, wl, obs)
    grid, _ = b3d.grid_of(wl.grid)
    seed = wl.seeds["sampler"]
    Pe = b3d.enumerate_grid(grid, seed=seed)
    Le, Ge = b3d.render_score(scene, Pe, grad=True)
    we, ie, lwe = b3d.sample(Le, 64, seed)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):  # warm the allocator on the side stream
        b3d.render_score(scene, b3d.enumerate_grid(grid, seed=seed), grad=True)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        Pg = b3d.enumerate_grid(grid, seed=seed)
        Lg, Gg = b3d.render_score(scene, Pg, grad=True)
        wg, ig, lwg = b3d.sample(Lg, 64, seed)
    for rep in range(3):
        Lx = b3d.render_score(scene, Pe[::7].contiguous())  # eager work between replays
        g.replay()
        torch.cuda.synchronize()
        say(f"  graph replay {rep}: logL equal {torch.equal(Lg, Le)}, samples equal {torch.equal(ig, ie)}")
        assert torch.equal(Pg, Pe) and torch.equal(Lg, Le) and torch.equal(Gg, Ge)
        assert torch.equal(ig, ie) and torch.equal(lwg, lwe) and torch.equal(wg, we)
        assert torch.equal(Lx, Le[::7])
