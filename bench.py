"""Throughput of the batched render-and-score hot path on one MI355X.

One step = one pass of the hot path over one batch of pose hypotheses of the
paper-scale single-object workload (2000 voxels = 24,000 triangles, 160x120
image, fx = fy = 150, 5000 hypotheses = 10x10 translations x 50 rotations,
5x5 window, sigma 3 mm, p_out 0.01):
  enumerate the hypothesis grid -> fused render + windowed likelihood +
  adjoint (d logL / d(pose, sigma, p_out)) -> normalise and draw samples.
Inputs are resident in device memory before timing starts.  The line also
reports the forward-only fused path, the plain split path (render point
images to memory, then score them; with and without the adjoint), the
roofline position of the fused kernel, and the FP64 CPU oracle on the host.

Usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--no-cpu-baseline]
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "pose hypotheses scored/s (render+logL) at 160x120, 24k tris; fwd+adjoint vs plain"

# Algorithmic work in FP32 lane-operations (a transcendental counts 4): 17 per
# vertex transformed, 12 per triangle tested, 27 per camera-facing triangle set
# up, 10 per covered pixel centre, 12 per (observed, rendered) window pair, 6 per
# observed pixel that sees a rendered point; the adjoint adds 10 per pair and 30
# per rendered object pixel.  For the fused kernel the items are counted by its
# instrumented instantiation on the same launch (the work of the algorithm as
# run, after cluster culling); for the plain method they are the oracle's
# counters (every triangle of the mesh).
COST = {"vert": 17, "tri": 12, "front": 27, "frag": 10, "pair": 12, "obs": 6, "adj_pair": 10, "adj_rpix": 30}
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12  # FP32 lane-ops/s, non-packed: 39.3 T
HBM_PEAK_GBPS = 8000.0  # MI355X HBM3E, published

# HBM bytes of one fused forward+adjoint launch on this workload, from two
# rocprofv3 --pmc runs (FETCH_SIZE, WRITE_SIZE in KiB per dispatch) scaled by
# what the same counters read for a plain 256 MiB device copy (FETCH_SIZE x 2.0,
# WRITE_SIZE x 1.0).  Valid only for the kernel sources with this digest:
# after any change to them the figure is reported as null until re-measured.
TRAFFIC = {"sources_sha256": "2651132e3b1803b9ed5bf65ba8c33a08cd01a5da02fc95ec9fba0c607afa7519", "fetch_KiB": 6370.8, "write_KiB": 312.5, "fetch_scale": 2.0, "write_scale": 1.0}
KERNEL_SOURCES = ["k_fused.hip", "b3d_device.hpp", "b3d_launch.hpp"]


def kernel_sources_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2312_08715_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic():
    t = TRAFFIC
    if t["sources_sha256"] is None or t["sources_sha256"] != kernel_sources_digest():
        return None
    return (t["fetch_KiB"] * t["fetch_scale"] + t["write_KiB"] * t["write_scale"]) * 1024.0


def lane_ops(c, adjoint=True):
    f = (COST["vert"] * c["vert"] + COST["tri"] * c["tri"] + COST["front"] * c["front"] + COST["frag"] * c["frag"]
         + COST["pair"] * c["pair"] + COST["obs"] * c["obs"])
    if adjoint:
        f += COST["adj_pair"] * c["pair"] + COST["adj_rpix"] * c["rpix"]
    return f


def counted_work(b3d, scene, P):
    w = b3d.render_score_work(scene, P)
    return {"vert": w["vertices"], "tri": w["triangles"], "front": w["setup"], "frag": w["fragments"],
            "pair": w["pairs"], "obs": w["observed"], "rpix": w["adjoint_pixels"], "exact": w["exact_tests"]}


def build_inputs(b3d, torch, k=1):
    """Workload inputs (config k: 0 small, 1 paper scale), built on the GPU with the library itself."""
    from workloads import assemble_observed_depth, make_config

    def render_depth(objs, cam):
        return gpu_depth(b3d, torch, objs, cam)

    wl = make_config(k, render=render_depth)
    K = b3d.intrinsics_of(wl.camera)
    depth = assemble_observed_depth(render_depth, wl)
    obs = b3d.unproject(torch.as_tensor(depth, dtype=torch.float32, device="cuda"), K)
    return wl, K, obs


def gpu_depth(b3d, torch, objs, cam):
    """Composite depth [H,W] (numpy) of (verts, tris, pose) objects rendered by the library."""
    K = b3d.intrinsics_of(cam)
    z = None
    for v, t, P in objs:
        m = b3d.Mesh(v, t)
        xyz, _ = b3d.render_batch(m, torch.as_tensor(np.asarray(P, np.float32)[None], device="cuda"), K, False)
        zk = xyz[0, ..., 2].cpu().numpy().astype(np.float64)
        z = zk if z is None else np.where((zk > 0) & ((z == 0) | (zk < z)), zk, z)
    return z


def noisy_observation(b3d, torch, depth, noise, cam):
    z = np.where(depth > 0, depth + noise["gauss"], 0.0)
    z = np.where(noise["outlier_mask"], noise["outlier_depth"], z)
    return b3d.unproject(torch.as_tensor(z, dtype=torch.float32, device="cuda"), b3d.intrinsics_of(cam))


def rot_err_deg(Ra, Rb):
    c = (np.trace(Ra @ Rb.T) - 1.0) / 2.0
    return float(np.degrees(np.arccos(np.clip(c, -1.0, 1.0))))


def bench_small(b3d, torch, steps, warmup):
    """The small configuration (500 voxels = 6,000 triangles, 64x48, 256
    hypotheses, 3x3 window): fused forward + adjoint, median of per-launch HIP
    event times.  At 256 hypotheses one launch fills a quarter of the chip's
    workgroup slots, so this measures latency more than throughput."""
    wl, K, obs = build_inputs(b3d, torch, 0)
    s = wl.score
    scene = b3d.Scene(b3d.Mesh(wl.verts, wl.tris), K, b3d.score_params(s.sigma, s.p_out, s.outlier_volume, s.window))
    scene.set_observed(obs)
    grid, _ = b3d.grid_of(wl.grid)
    P = b3d.enumerate_grid(grid, seed=wl.seeds["hyp"])
    stream = torch.cuda.current_stream()
    ts = []
    for i in range(warmup + steps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b3d.render_score(scene, P, grad=True)
        e1.record(stream)
        e1.synchronize()
        if i >= warmup:
            ts.append(e0.elapsed_time(e1) / 1e3)
    t = float(np.median(ts))
    return {"hypotheses": int(P.shape[0]), "value": P.shape[0] / t, "ms": t * 1e3, "unit": "hypotheses/s",
            "note": "fused forward + adjoint, 64x48, 6k triangles, median of HIP event times per launch"}


def bench_throughput_vs_n(b3d, torch, scene, P, ns=(625, 1250, 2500, 5000, 10000, 20000), reps=10):
    """Fused forward + adjoint at several batch sizes of the same workload (the
    5000 paper-scale hypotheses tiled or cut): one GPU's share when the
    hypotheses of a stage are split across g GPUs is N = 5000 / g."""
    stream = torch.cuda.current_stream()
    out = []
    for n in ns:
        Pn = P.repeat((n + P.shape[0] - 1) // P.shape[0], 1, 1)[:n].contiguous()
        for _ in range(2):
            b3d.render_score(scene, Pn, grad=True)
        ts = []
        for _ in range(reps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            b3d.render_score(scene, Pn, grad=True)
            e1.record(stream)
            e1.synchronize()
            ts.append(e0.elapsed_time(e1) / 1e3)
        t = float(np.median(ts))
        out.append({"N": n, "ms": t * 1e3, "hypotheses_per_s": n / t})
    return out


def bench_noise_grid(b3d, torch, scene, P, A=4, B=4, sigma_max=0.01, reps=10):
    """Hierarchical likelihood: logL of every hypothesis under a 4 x 4 grid of
    (sigma, p_out) midpoints and the marginal over it, forward only."""
    sig, po = b3d.noise_grid_midpoints(sigma_max, A, B)
    scene.set_noise_grid(sig, po)
    stream = torch.cuda.current_stream()
    for _ in range(2):
        b3d.render_score_marginal(scene, P, grid=True)
    ts = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        b3d.render_score_marginal(scene, P, grid=True)
        e1.record(stream)
        e1.synchronize()
        ts.append(e0.elapsed_time(e1) / 1e3)
    t = float(np.median(ts))
    # counted work of the same render and windows; each pair adds a scale and an
    # exponential per extra deviation, each observed pixel a logarithm per grid point
    c = counted_work(b3d, scene, P)
    ops = (lane_ops(c, adjoint=False) + 3 * (A - 1) * c["pair"]
           + (COST["obs"] * (A * B - 1) + A) * c["obs"])
    achieved = ops / t / 1e12
    return {"grid": f"{A}x{B}", "value": P.shape[0] / t, "ms": t * 1e3, "unit": "hypotheses/s",
            "roofline": {"bound": "alu", "kernel": "k_render_score_grid", "achieved": achieved,
                         "peak": VALU_PEAK_TOPS, "unit": "TOP/s (FP32 lane-ops)", "frac": achieved / VALU_PEAK_TOPS,
                         "ops_per_hypothesis": ops / P.shape[0]},
            "note": "fused render + windowed likelihood under every grid point + marginal, one launch"}


SMC_STAGE_NOISE = ((0.03, 0.3), (0.01, 0.2), (0.004, 0.1))


def bench_smc(b3d, torch, p=None, n_particles=16, reps=2, seed=4242, stage_noise=SMC_STAGE_NOISE):
    """SMC over the objects of the four-object table scene at 320x240: the
    library is the scene's four meshes, every particle places four objects;
    per object, stage 0 scores 4 types x 6 faces x 512 placement cells, then
    two splits of 64 cells, then the 4 x 4 noise cells over the whole image."""
    from workloads import table_scene

    meshes, poses, table, cam, noise, Tcw = table_scene()
    objs = [(v, t, P) for (v, t), P in zip(meshes, poses)] + [table]
    obs = noisy_observation(b3d, torch, gpu_depth(b3d, torch, objs, cam), noise, cam)
    types = [b3d.Mesh(v, t) for v, t in meshes]
    tv, tt, tT = table
    tmesh = b3d.Mesh(tv, tt)
    counts = ((8, 8, 8), (4, 4, 4), (4, 4, 4))
    n_obj = len(meshes)
    sp = b3d.smc_params(n_particles=n_particles, n_objects=n_obj, counts=counts, sigma_max=0.02, noise_A=4, noise_B=4,
                        sigma0=0.015, p_out0=0.5, ess_threshold=0.5, outlier_volume=1.0, window=5, seed=seed,
                        stage_noise=stage_noise)
    smc = b3d.SMC(types, b3d.table(tT, 1.0, 1.0), b3d.intrinsics_of(cam), sp, fixed=[tmesh],
                  fixed_poses=np.asarray(tT, np.float32)[None])

    def run():
        smc.reset(obs)
        for _ in range(n_obj):
            smc.step()

    run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        run()
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / reps
    n0 = int(np.prod(counts[0])) * 6 * len(types)
    hyp = n_obj * n_particles * (n0 + sum(int(np.prod(c)) for c in counts[1:]))
    r = smc.read()
    best = int(torch.argmax(r["logW"]).item())
    place = r["place"][best].cpu().numpy()
    est = r["poses"][best].cpu().numpy()
    found = []
    for k, ((v, _), P) in enumerate(zip(meshes, poses)):
        c = 0.5 * (v.min(0) + v.max(0))
        ct = P[:3, :3] @ c + P[:3, 3]
        errs = [np.linalg.norm((est[j][:3, :3] @ c + est[j][:3, 3]) - ct) for j in range(n_obj) if place[j, 0] == k]
        found.append(round(100 * min(errs), 2) if errs else None)
    return {"particles": n_particles, "objects": n_obj, "types": len(types), "image": f"{cam.W}x{cam.H}",
            "ms_per_run": t * 1e3, "particle_hypotheses_per_run": hyp, "particle_hypotheses_per_s": hyp / t,
            "scored_per_run": r["scored"], "scored_per_s": r["scored"] / t,
            "map_particle": {"types": place[:, 0].tolist(), "faces": place[:, 1].tolist(),
                             "noise": [round(float(x), 5) for x in r["noise"][best].cpu().numpy()],
                             "centre_error_cm_per_true_object": found},
            "ess_last": float(r["ess"].item()), "stage_noise": stage_noise,
            "note": "reset + 4 SMC stages; placement cells scored by the batched fused kernel (16 particles x "
                    f"{n0} cells at stage 0; particles with equal state share one scoring, hence scored < "
                    "particle hypotheses), noise cells over the whole image, eq. (2)/(3) weights, resampling"}


def bench_batch(b3d, torch, p, n_scenes=64, seed=1003, reps=3, tune=True, size=None, n_hyp=None):
    """Many scenes (1-8 objects of 500-8000 voxels, three image sizes, 1k-20k
    hypotheses each) as one batch (b3d_batch_run), forward + adjoint, against
    the same scenes one launch at a time; depth-buffer tiles from the
    autotuner.
    size, n_hyp: one image size (H, W) and hypothesis count for every scene
    instead of the drawn ones."""
    import tempfile

    from workloads import Camera, observation_noise, pose_matrix, random_scene_batch, shoemake_rotations, voxel_blob, \
        voxel_mesh

    tile_cache = os.path.join(tempfile.mkdtemp(prefix="b3d_tiles_"), "tiles.json")
    rng = np.random.default_rng(seed)
    items, keep = [], []
    for i, sh in enumerate(random_scene_batch(rng, n_scenes)):
        H, W = sh["H"], sh["W"]
        if size is not None:
            H, W = size
        if n_hyp is not None:
            sh["N"] = n_hyp
        cam = Camera(W * 0.9375, W * 0.9375, W / 2.0, H / 2.0, H, W)
        objs = []
        for k, nv in enumerate(sh["voxels"]):
            v, t = voxel_mesh(voxel_blob(nv, rng))
            pos = (0.0, 0.0, 0.8) if k == 0 else (rng.uniform(-0.2, 0.2), rng.uniform(-0.15, 0.15),
                                                  rng.uniform(0.8, 1.2))
            objs.append((v, t, pose_matrix(shoemake_rotations(1, rng)[0], pos)))
        obs = noisy_observation(b3d, torch, gpu_depth(b3d, torch, objs, cam),
                                observation_noise(H, W, rng, 0.002, 0.03), cam)
        meshes = [b3d.Mesh(v, t) for v, t, _ in objs]
        scene = b3d.Scene(meshes[0], b3d.intrinsics_of(cam), p)
        if len(objs) > 1:
            scene.set_background(meshes[1:], np.stack([P for _, _, P in objs[1:]]))
        scene.set_observed(obs)
        # 10 x ny x nz translations over +-2 cm x 10 rotations within 10 degrees
        nz = max(1, int(round(sh["N"] / 1000.0)))
        ny = 10 if sh["N"] >= 1000 else max(1, sh["N"] // 100)
        grid = b3d.make_grid(objs[0][2], (0.02, 0.02, 0.02), (10, ny, nz), n_rot=10, rot_max_angle=np.deg2rad(10.0))
        P = b3d.enumerate_grid(grid, seed=3003 + i)
        if tune:  # the tile of each shape class (image size, window, mesh size), timed once
            scene.autotune(P[:2048], grad=True, cache=tile_cache)
        items.append((scene, P))
        keep += [meshes, obs]
    total = sum(int(P.shape[0]) for _, P in items)
    batch = b3d.Batch(items, grad=True)
    batch.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        batch.run()
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / reps
    for sc, P in items:
        b3d.render_score(sc, P, grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        for sc, P in items:
            b3d.render_score(sc, P, grad=True)
    torch.cuda.synchronize()
    t_seq = (time.perf_counter() - t0) / reps
    # VALU roofline of the batch: every scene's work as the instrumented kernel
    # counts it (culled), priced by the cost table, over the batch's time
    ops = 0.0
    for sc, P in items:
        ops += lane_ops(counted_work(b3d, sc, P), adjoint=True)
    achieved = ops / t_batch / 1e12
    return {"scenes": n_scenes, "hypotheses": total, "value": total / t_batch, "ms": t_batch * 1e3,
            "one_at_a_time": {"value": total / t_seq, "ms": t_seq * 1e3}, "unit": "hypotheses/s",
            "tiles": "autotuned per shape class" if tune else "default",
            "roofline": {"bound": "alu", "kernel": "k_batch<true>", "achieved": achieved, "peak": VALU_PEAK_TOPS,
                         "unit": "TOP/s (FP32 lane-ops)", "frac": achieved / VALU_PEAK_TOPS,
                         "counting": "kernel's own count (instrumented launch per scene) x cost table",
                         "traffic": None},
            "note": "forward + adjoint; launches of eight scenes, one workgroup per hypothesis, on two streams, "
                    "vs one launch per scene"}


def bench_tracking(b3d, torch, p, n_frames=200, min_visible=0.0, widen=1.0):
    """Three objects on smooth SE(3) paths, 160x120, 4% outliers; per frame and
    object two stages of hypotheses (10,000 over +-3 cm x 10 rotations within
    8 deg, then 2,500 over +-7.5 mm x 20 rotations within 3 deg around the best)
    and 10 Adam steps, one HIP graph per frame."""
    from workloads import tracking_sequence

    meshes, paths, cam, noise = tracking_sequence(seed=1004, n_frames=n_frames)
    M = paths.shape[1]
    frames = []
    vis = np.zeros((n_frames, M))  # fraction of each object's pixels not hidden by the others
    for f in range(n_frames):
        objs = [(v, t, paths[f, k]) for k, (v, t) in enumerate(meshes)]
        alone = [gpu_depth(b3d, torch, [o], cam) for o in objs]
        depth = gpu_depth(b3d, torch, objs, cam)
        for k in range(M):
            own = alone[k] > 0
            vis[f, k] = float((own & (alone[k] == depth)).sum()) / max(1, int(own.sum()))
        frames.append(noisy_observation(b3d, torch, depth, noise[f], cam))
    ms = [b3d.Mesh(v, t) for v, t in meshes]
    stages = [b3d.make_grid(np.eye(4), (0.03, 0.03, 0.03), (10, 10, 10), n_rot=10, rot_max_angle=np.deg2rad(8.0)),
              b3d.make_grid(np.eye(4), (0.0075, 0.0075, 0.0075), (5, 5, 5), n_rot=20, rot_max_angle=np.deg2rad(3.0))]
    tr = b3d.Tracker(ms, b3d.intrinsics_of(cam), p, stages, paths[0], n_refine=10, lr_t=1e-3, lr_r=1e-2,
                     min_visible=min_visible, widen=widen)
    est = torch.empty((n_frames, M, 4, 4), dtype=torch.float32, device="cuda")
    gst = torch.zeros((n_frames, M, 3), dtype=torch.float32, device="cuda")
    est[0] = torch.as_tensor(paths[0], dtype=torch.float32)
    tr.frame(frames[1])  # captures the frame graph
    est[1] = tr.poses()
    gst[1] = tr.state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for f in range(2, n_frames):
        tr.frame(frames[f])
        est[f] = tr.poses()
        gst[f] = tr.state()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    E = est.cpu().numpy().astype(np.float64)
    G = gst.cpu().numpy()
    pos = np.linalg.norm(E[1:, :, :3, 3] - paths[1:, :, :3, 3], axis=2) * 100.0
    rot = np.array([[rot_err_deg(E[f, k, :3, :3], paths[f, k, :3, :3]) for k in range(M)] for f in range(1, n_frames)])
    lost = pos > 5.0
    seen = vis[1:] >= 0.5
    def hidden_before_loss(k):
        """The frames just before object k is first lost: the run of frames in
        which it was under 10% visible, and how far its true pose moved then
        (the search reaches 3 cm around the previous estimate)."""
        if not lost[:, k].any():
            return None
        f1 = int(np.argmax(lost[:, k]) + 1)
        f0 = f1
        while f0 > 1 and vis[f0 - 1, k] < 0.1:
            f0 -= 1
        moved = float(np.linalg.norm(paths[f1, k, :3, 3] - paths[f0, k, :3, 3]) * 100.0)
        return {"hidden_from": f0, "frames_hidden": f1 - f0, "true_motion_cm": moved,
                "visibility_at_loss": float(vis[f1, k])}

    per_obj = [{"mean_cm": float(pos[:, k].mean()), "max_cm": float(pos[:, k].max()),
                "frames_over_5cm": int(lost[:, k].sum()),
                "first_over_5cm": int(np.argmax(lost[:, k]) + 1) if lost[:, k].any() else None,
                "frames_under_half_visible": int((~seen[:, k]).sum()),
                "least_visible": float(vis[1:, k].min()),
                "before_loss": hidden_before_loss(k),
                "updates_dropped": int((G[1:, k, 1] > 0).sum())}
               for k in range(M)]
    return {"frames_per_s": (n_frames - 2) / dt, "frames": n_frames, "objects": M, "per_object": per_obj,
            "hypotheses_per_frame": int(M * 12500), "position_error_cm": {"mean": float(pos.mean()),
                                                                           "max": float(pos.max())},
            "orientation_error_deg": {"mean": float(rot.mean()), "max": float(rot.max())},
            "when_at_least_half_visible": {"position_error_cm": {"mean": float(pos[seen].mean()),
                                                                  "median": float(np.median(pos[seen]))},
                                           "orientation_error_deg": {"mean": float(rot[seen].mean()),
                                                                     "median": float(np.median(rot[seen]))}},
            "min_visible": min_visible, "widen": widen,
            "note": "objects pass behind each other; an object hidden for several frames is lost by the local search"
                    + ("" if min_visible <= 0 else "; occlusion handling: updates less than min_visible seen are "
                       "dropped for the last motion, the next first stage widened")}


def bench_camera_pan(b3d, torch, p, resolutions=(25, 50, 100, 200), n_frames=120):
    """The setting of the paper's tracking table (Sec. IV, Table 1): a camera
    circling one object on a table for 120 frames at square resolutions of
    25 to 200 pixels, tracked from the known first pose by four stages of
    hypotheses per frame (1,708 in all: rotations, translations, then two
    joint stages, each around the best of the stage before) and no gradient
    steps, one HIP graph per frame.  The tracked quantity is the scene's pose
    in the camera frame; errors are of the camera's position in the scene
    frame and of its orientation."""
    from workloads import camera_pan_schedule, camera_pan_sequence

    specs = camera_pan_schedule()
    grids = [b3d.grid_of(g) for g in specs]  # (grid, rotations tensor): the tensors outlive the trackers
    per_frame = sum(g.N for g in specs)
    out = {}
    for res in resolutions:
        (v, t), truth, cam, noise = camera_pan_sequence(res=res, n_frames=n_frames)
        frames = [noisy_observation(b3d, torch, gpu_depth(b3d, torch, [(v, t, truth[f])], cam), noise[f], cam)
                  for f in range(n_frames)]
        tr = b3d.Tracker([b3d.Mesh(v, t)], b3d.intrinsics_of(cam), p, [g for g, _ in grids], truth[:1], n_refine=0)
        est = torch.empty((n_frames, 1, 4, 4), dtype=torch.float32, device="cuda")
        est[0] = torch.as_tensor(truth[:1], dtype=torch.float32)
        tr.frame(frames[1])  # captures the frame graph
        est[1] = tr.poses()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for f in range(2, n_frames):
            tr.frame(frames[f])
            est[f] = tr.poses()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        tr.close()
        E = est[:, 0].cpu().numpy().astype(np.float64)
        cam_pos = lambda T: -T[:, :3, :3].transpose(0, 2, 1) @ T[:, :3, 3:4]  # noqa: E731
        pos = np.linalg.norm((cam_pos(E[1:]) - cam_pos(truth[1:]))[..., 0], axis=1) * 100.0
        rot = np.array([rot_err_deg(E[f, :3, :3], truth[f, :3, :3]) for f in range(1, n_frames)])
        out[f"{res}x{res}"] = {"frames_per_s": (n_frames - 2) / dt,
                               "hypotheses_per_s": per_frame * (n_frames - 2) / dt,
                               "position_error_cm": {"mean": float(pos.mean()), "max": float(pos.max())},
                               "orientation_error_deg": {"mean": float(rot.mean()), "max": float(rot.max())}}
    return {"frames": n_frames, "hypotheses_per_frame": per_frame, "triangles": int(t.shape[0]),
            "by_resolution": out}


TABLE_STAGES = [((0.08, 0.08, 0.08), (10, 10, 10), 10, 30.0), ((0.02, 0.02, 0.02), (10, 10, 10), 10, 10.0),
                ((0.005, 0.005, 0.005), (10, 10, 10), 10, 3.0)]


def bench_table_c2f(b3d, torch, p, stages=None):
    """Four objects on a table at 320x240: per object three coarse-to-fine
    stages of 10,000 hypotheses for 16 particles, then 20 Adam steps on the
    survivors with the adjoint.  stages: (half extents, translation counts,
    rotations, rotation cone in degrees) per stage."""
    from workloads import shoemake_rotations, table_scene

    meshes, poses, table, cam, noise, Tcw = table_scene()
    objs = [(v, t, P) for (v, t), P in zip(meshes, poses)] + [table]
    obs = noisy_observation(b3d, torch, gpu_depth(b3d, torch, objs, cam), noise, cam)
    ms = [b3d.Mesh(v, t) for v, t, _ in objs]
    K = b3d.intrinsics_of(cam)
    rng = np.random.default_rng(2002)
    stages = TABLE_STAGES if stages is None else stages
    sched = b3d.make_schedule([b3d.make_grid(np.eye(4), h, n, n_rot=r, rot_max_angle=np.deg2rad(a))
                               for h, n, r, a in stages])
    out, total_h, total_t, tiles = [], 0, 0.0, []
    for k in range(len(meshes)):
        scene = b3d.Scene(ms[k], K, p)
        others = [j for j in range(len(objs)) if j != k]
        scene.set_background([ms[j] for j in others], np.stack([objs[j][2] for j in others]))
        scene.set_observed(obs)
        truth = poses[k]
        # start 3 cm and 15 degrees away from the truth (a detection's error)
        w = rng.normal(size=3)
        w *= np.deg2rad(15.0) / np.linalg.norm(w)
        Kx = np.array([[0, -w[2], w[1]], [w[2], 0, -w[0]], [-w[1], w[0], 0]]) / np.linalg.norm(w)
        th = np.linalg.norm(w)
        dR = np.eye(3) + np.sin(th) * Kx + (1 - np.cos(th)) * Kx @ Kx
        dt = rng.normal(size=3)
        dt *= 0.03 / np.linalg.norm(dt)
        start = truth.copy()
        start[:3, :3] = dR @ truth[:3, :3]
        start[:3, 3] += dt
        # the depth-buffer tile from the autotuner, on the first stage's hypotheses (set-up, not timed)
        h0, n0, r0, a0 = stages[0]
        g0 = b3d.make_grid(start, h0, n0, n_rot=r0, rot_max_angle=np.deg2rad(a0))
        tiles.append(scene.autotune(b3d.enumerate_grid(g0, seed=4002 + k)[:2048], grad=False))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        P, logq, idx = b3d.c2f_step(scene, start, sched, 16, 4002 + k)
        b3d.refine_poses(scene, P, 20, 1e-3, 1e-2)
        L = b3d.render_score(scene, P)
        torch.cuda.synchronize()
        dtm = time.perf_counter() - t0
        best = P[int(torch.argmax(L))].cpu().numpy().astype(np.float64)
        sizes = [int(np.prod(n)) * r for _, n, r, _ in stages]
        n_h = sizes[0] + 16 * sum(sizes[1:]) + 21 * 16
        total_h += n_h
        total_t += dtm
        # is the true pose more likely than the one found?  (if not, an error is
        # the object's near-symmetry under this noise, not a search failure)
        L_truth = float(b3d.render_score(scene, torch.as_tensor(np.asarray(truth, np.float32)[None],
                                                                device="cuda"))[0])
        out.append({"object": k, "triangles": int(meshes[k][1].shape[0]), "ms": dtm * 1e3,
                    "position_error_cm": float(np.linalg.norm(best[:3, 3] - truth[:3, 3]) * 100),
                    "orientation_error_deg": rot_err_deg(best[:3, :3], truth[:3, :3]),
                    "logL_found_minus_truth": float(L.max()) - L_truth})
    return {"hypotheses_per_s": total_h / total_t, "objects": out, "tiles": tiles,
            "note": "3 stages x 10,000 hypotheses (16 particles from stage 2), then 20 Adam steps on 16 poses; "
                    "depth-buffer tiles from the autotuner"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--samples", type=int, default=64, help="draws per step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--fused-only", action="store_true", help="skip the split-path comparison")
    ap.add_argument("--no-extras", action="store_true", help="skip the batch, tracking and table workloads")
    ap.add_argument("--only", choices=["batch", "tracking", "camera_pan", "table", "noise_grid", "smc"],
                    help="run just one of the extra workloads and print its JSON (for profiling)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device copy (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path (hypotheses would shard "
              "across GPUs with one small all-reduce per stage; see the design notes).", file=sys.stderr)
        sys.exit(2)

    import torch

    import paper_2312_08715_amd as b3d

    torch.cuda.set_device(0)
    wl, K, obs = build_inputs(b3d, torch)
    s = wl.score
    p = b3d.score_params(s.sigma, s.p_out, s.outlier_volume, s.window)
    if args.only and args.only != "noise_grid":
        fn = {"batch": bench_batch, "tracking": bench_tracking, "camera_pan": bench_camera_pan,
              "table": bench_table_c2f, "smc": bench_smc}[args.only]
        print(json.dumps({args.only: fn(b3d, torch, p)}), flush=True)
        return
    mesh = b3d.Mesh(wl.verts, wl.tris)
    scene = b3d.Scene(mesh, K, p)
    scene.set_observed(obs)
    grid, rots = b3d.grid_of(wl.grid)
    if args.only == "noise_grid":
        P = b3d.enumerate_grid(grid, seed=wl.seeds["sampler"])
        print(json.dumps({args.only: bench_noise_grid(b3d, torch, scene, P)}), flush=True)
        return
    N = b3d.grid_size(grid)
    seed = wl.seeds["sampler"]
    stream = torch.cuda.current_stream()

    poses = torch.empty((N, 4, 4), dtype=torch.float32, device="cuda")
    kev = []

    def step(timed_kernel=False, grad=True):
        P = b3d.enumerate_grid(grid, seed=seed)
        if timed_kernel:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
        out = b3d.render_score(scene, P, grad=grad)
        if timed_kernel:
            e1.record(stream)
            kev.append((e0, e1))
        logL = out[0] if grad else out
        w, idx, lw = b3d.sample(logL, args.samples, seed)
        return idx

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / steps

    # headline: fused forward + adjoint
    kev.clear()
    t_step = timed(lambda: step(timed_kernel=True), args.steps, args.warmup)
    kev_t = [a.elapsed_time(b) for a, b in kev[args.warmup:]]
    t_kernel = float(np.mean(kev_t)) / 1e3
    t_kernel_median = float(np.median(kev_t)) / 1e3
    # forward only
    t_fwd = timed(lambda: step(grad=False), args.steps, args.warmup)

    # plain split path: point images through device memory
    P = b3d.enumerate_grid(grid, seed=seed)

    split_ev = {}

    def ev(name, fn):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        out = fn()
        e1.record(stream)
        split_ev.setdefault(name, []).append((e0, e1))
        return out

    def split(adj):
        xyz, tri = ev("render_batch_ids" if adj else "render_batch", lambda: b3d.render_batch(mesh, P, K, want_tri=adj))
        L = ev("score", lambda: b3d.score(obs, xyz, p))
        if adj:
            dr, ds, dp = ev("score_backward", lambda: b3d.score_backward(obs, xyz, p))
            ev("render_backward", lambda: b3d.render_backward(mesh, P, K, tri, dr))
        return L

    t_split = t_split_adj = float("nan")
    split_kernels = {}
    if not args.fused_only:
        t_split = timed(lambda: split(False), max(3, args.steps // 4), 1)
        t_split_adj = timed(lambda: split(True), max(3, args.steps // 4), 1)
        _, tri = b3d.render_batch(mesh, P, K, want_tri=True)  # the drawn pixels render_backward reads
        split_kernels = split_rooflines(split_ev, N, wl.camera.H * wl.camera.W, int((tri >= 0).sum()))
        del tri
    if args.copy_calibration:
        src = torch.empty(64 << 20, dtype=torch.float32, device="cuda").fill_(1.0)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    # the chip's peaks, re-measured by microbenchmarks: an FMA loop (lane-ops/s),
    # an HBM triad and an LDS read loop (bytes/s)
    from paper_2312_08715_amd import probe

    valu_measured = probe.probe_fma() / 1e12
    peaks = {"valu_TOPs": valu_measured, "hbm_GBps": probe.probe_hbm() / 1e9, "lds_TBps": probe.probe_lds() / 1e12}
    work = counted_work(b3d, scene, P)
    ops = lane_ops(work, adjoint=True)  # the kernel's own (culled) work
    extras = {}
    if not args.no_extras:
        extras["small_config"] = bench_small(b3d, torch, args.steps, args.warmup)
        extras["throughput_vs_n"] = bench_throughput_vs_n(b3d, torch, scene, P)
        extras["noise_grid_4x4"] = bench_noise_grid(b3d, torch, scene, P)
        for name, fn in (("smc_table_scene", lambda: bench_smc(b3d, torch)),
                         ("batch_64_scenes", lambda: bench_batch(b3d, torch, p)),
                         ("batch_64_small_scenes", lambda: bench_batch(b3d, torch, p, size=(120, 160), n_hyp=1000)),
                         ("tracking_200_frames", lambda: bench_tracking(b3d, torch, p)),
                         ("tracking_200_frames_occlusion_handling",
                          lambda: bench_tracking(b3d, torch, p, min_visible=0.08, widen=2.0)),
                         ("camera_pan_120_frames", lambda: bench_camera_pan(b3d, torch, p)),
                         ("table_c2f_adam", lambda: bench_table_c2f(b3d, torch, p))):
            t0 = time.perf_counter()
            extras[name] = fn()
            print(f"# {name} done in {time.perf_counter() - t0:.1f} s", file=sys.stderr, flush=True)
    cpu, plain_counts = None, None
    if not args.no_cpu_baseline:
        cpu, plain_counts = cpu_baseline(wl, obs.cpu().numpy().astype(np.float64), args.cpu_seconds)
    line = {
        "metric": METRIC,
        "value": N / t_step,
        "unit": "hypotheses/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_step * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "paper-scale single object: 2000 voxels (24k tris), 160x120, 5000 hypotheses "
                               "(10x10 translations x 50 rotations), 5x5 window, fused fwd+adjoint + sampling",
                   "hypotheses": N, "image": "160x120", "triangles": int(wl.tris.shape[0]), "window": s.window,
                   "samples_per_step": args.samples},
        "roofline": roofline_line(t_kernel, t_kernel_median, N, ops, work, plain_counts, valu_measured),
        "fwd_only": {"value": N / t_fwd, "ms_per_step": t_fwd * 1e3},
        "plain_split": {"value": N / t_split, "ms_per_step": t_split * 1e3,
                        "note": "render_batch -> score, point images in HBM",
                        "roofline": split_kernels.get("score")},
        "plain_split_fwd_adjoint": {"value": N / t_split_adj, "ms_per_step": t_split_adj * 1e3,
                                    "note": "render_batch (with ids) -> score -> score_backward -> render_backward",
                                    "roofline": split_kernels.get("score_backward"), "kernels": split_kernels},
        "peaks_measured": peaks,
        "cpu_baseline": cpu,
    }
    line.update(extras)
    print(json.dumps(line), flush=True)


# Algorithmic HBM bytes of each split-path kernel per pixel of every point
# image (one hypothesis's point image is H x W x 12 bytes, its triangle ids
# H x W x 4): render_batch writes points (and ids), score reads points,
# score_backward reads points and writes their gradient.  render_backward
# must read every id but only the point gradients of drawn pixels: 4 bytes a
# pixel plus 12 per drawn pixel (counted on the launch's ids).
SPLIT_BYTES_PER_PIXEL = {"render_batch": 12, "render_batch_ids": 16, "score": 12, "score_backward": 24,
                         "render_backward": 4}
SPLIT_BYTES_PER_DRAWN = {"render_backward": 12}

# HBM bytes per launch of the split kernels on this workload (5000 point
# images of 160x120), from the same two rocprofv3 --pmc runs and copy
# calibration as TRAFFIC (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0, KiB per
# dispatch, mean over the run's dispatches); valid for the sources with this
# digest only.
SPLIT_SOURCES = ["k_render.hip", "k_score.hip", "b3d_device.hpp", "b3d_launch.hpp"]
SPLIT_TRAFFIC = {"sources_sha256": "47fa578138c9ed91af9b40bb4f7f1616b029f8a663451880d268f717caf8b526",
                 "KiB": {"render_batch": [39210.7, 1125996.8], "render_batch_ids": [44446.1, 1500873.9],
                         "score": [563817.4, 166.4], "score_backward": [565346.4, 1126030.5],
                         "render_backward": [244248.0, 234.4]}}


def split_sources_digest() -> str:
    import hashlib

    h = hashlib.sha256()
    for f in SPLIT_SOURCES:
        with open(os.path.join(ROOT, "paper_2312_08715_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def split_rooflines(events, N, HW, drawn):
    """HBM roofline of each split-path kernel from its HIP-event times (warm-up
    excluded), against the 8 TB/s peak; drawn: object pixels over the launch's
    point images."""
    out = {}
    valid = SPLIT_TRAFFIC["sources_sha256"] == split_sources_digest()
    for name, evs in events.items():
        ms = float(np.mean([a.elapsed_time(b) for a, b in evs[1:]])) if len(evs) > 1 else float("nan")
        b = SPLIT_BYTES_PER_PIXEL[name] * HW * N + SPLIT_BYTES_PER_DRAWN.get(name, 0) * drawn
        kib = SPLIT_TRAFFIC["KiB"].get(name)
        traffic = (kib[0] * 2.0 + kib[1] * 1.0) * 1024.0 if valid and kib else None
        out[name] = {"bound": "hbm", "kernel": name, "achieved": b / (ms * 1e-3) / 1e9, "peak": HBM_PEAK_GBPS,
                     "unit": "GB/s", "frac": b / (ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, "bytes": b, "kernel_ms": ms,
                     "traffic": traffic}
    return out


def roofline_line(t_kernel, t_kernel_median, N, ops, work, plain_counts, valu_measured):
    """VALU roofline of the fused kernel.  Algorithmic work per hypothesis is
    the plain method's: the oracle's work counters (every triangle, every
    fragment, every window pair of the definition) priced by the cost table
    (`lane_ops`), from the CPU-baseline leg; the kernel's own, culled count
    (the instrumented launch) is reported beside it.  Without the CPU leg the
    kernel's count stands in."""
    own = {"ops_per_hypothesis": ops / N, "achieved": ops / t_kernel / 1e12,
           "frac": ops / t_kernel / 1e12 / VALU_PEAK_TOPS, "work_per_hypothesis": {k: v / N for k, v in work.items()}}
    plain = lane_ops(plain_counts) if plain_counts else None
    per_h = plain if plain else ops / N
    achieved = per_h * N / t_kernel / 1e12
    return {"bound": "alu", "kernel": "k_render_score<true, 0>", "achieved": achieved, "peak": VALU_PEAK_TOPS,
            "unit": "TOP/s (FP32 lane-ops)", "frac": achieved / VALU_PEAK_TOPS, "traffic": measured_traffic(),
            "counting": "plain method: oracle work counters x cost table" if plain else "kernel's own count",
            "ops_per_hypothesis": per_h, "plain_method_counts_per_hypothesis": plain_counts,
            "kernel_ms": t_kernel * 1e3, "kernel_ms_median": t_kernel_median * 1e3,
            "peak_measured": valu_measured, "frac_of_measured": achieved / valu_measured,
            "kernel_count": own}


def cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(wl, obs64, seconds):
    """The FP64 oracle (render, score, both adjoints) on hypotheses of the same
    workload, in chunks, until about `seconds` of CPU time; all host threads,
    then one thread on a smaller sample."""
    import oracle

    s = wl.score
    P = oracle.enumerate_grid(wl.grid, seed=wl.seeds["hyp"])

    def run(limit, max_done):
        done, t0 = 0, time.perf_counter()
        while done < min(P.shape[0], max_done) and time.perf_counter() - t0 < limit:
            Q = P[done:done + 16]
            d, ids = oracle.render([(wl.verts, wl.tris, Q)], wl.camera)
            xyz = oracle.unproject(d, wl.camera)
            oracle.score(obs64, xyz, s.sigma, s.p_out, s.outlier_volume, s.window)
            dr, ds, dp = oracle.score_grad(obs64, xyz, s.sigma, s.p_out, s.outlier_volume, s.window)
            oracle.render_grad(wl.verts, wl.tris, Q, wl.camera, ids, d, dr)
            done += Q.shape[0]
        return done, time.perf_counter() - t0

    all_threads = oracle.num_threads()
    oracle.set_threads(1)
    one_done, one_dt = run(max(2.0, seconds / 5), 1 << 30)
    oracle.set_threads(all_threads)
    done, t0 = 0, time.perf_counter()
    cnt_sum = np.zeros(oracle.NC)
    chunk = 64
    while done < P.shape[0] and time.perf_counter() - t0 < seconds:
        Q = P[done:done + chunk]
        d, ids, c = oracle.render([(wl.verts, wl.tris, Q)], wl.camera, counters=True)
        xyz = oracle.unproject(d, wl.camera)
        L, l1, c2 = oracle.score(obs64, xyz, s.sigma, s.p_out, s.outlier_volume, s.window, counters=True)
        dr, ds, dp = oracle.score_grad(obs64, xyz, s.sigma, s.p_out, s.outlier_volume, s.window)
        oracle.render_grad(wl.verts, wl.tris, Q, wl.camera, ids, d, dr)
        cnt_sum += (c + c2).sum(0)
        done += Q.shape[0]
    dt = time.perf_counter() - t0
    m = cnt_sum / done
    counts = {"vert": m[oracle.C_VERT], "tri": m[oracle.C_TRI], "front": m[oracle.C_FRONT], "frag": m[oracle.C_FRAG],
              "pair": m[oracle.C_PAIR], "obs": m[oracle.C_OBS_ACTIVE], "rpix": m[oracle.C_RPIX]}
    return ({"value": done / dt, "unit": "hypotheses/s", "cores": oracle.num_threads(), "kind": "oracle",
             "sample": f"first {done} of {P.shape[0]} hypotheses, render+score+adjoint in FP64",
             "cpu": cpu_model(), "host_cpus": os.cpu_count(),
             "single_thread": {"value": one_done / one_dt, "unit": "hypotheses/s",
                               "sample": f"first {one_done} hypotheses, one thread"},
             "other_workloads": cpu_other_workloads()}, counts)


def cpu_other_workloads():
    """The oracle (render + score, forward, all threads) on the small
    configuration (all 256 hypotheses) and on 256 hypotheses of the table
    scene's first coarse-to-fine stage (320x240, the other objects and the
    table as background)."""
    import oracle
    from workloads import make_config, table_scene

    out = {}
    wl = make_config(0, render=oracle.render_depth_fn)
    obs = oracle.observed_xyz(wl)
    P = oracle.enumerate_grid(wl.grid, seed=wl.seeds["hyp"])
    s = wl.score
    t0 = time.perf_counter()
    d, _ = oracle.render([(wl.verts, wl.tris, P)], wl.camera)
    oracle.score(obs, oracle.unproject(d, wl.camera), s.sigma, s.p_out, s.outlier_volume, s.window)
    out["small_config"] = {"value": P.shape[0] / (time.perf_counter() - t0), "unit": "hypotheses/s",
                           "sample": f"all {P.shape[0]} hypotheses, forward"}
    meshes, poses, table, cam, noise, Tcw = table_scene()
    objs = [(v, t, Q) for (v, t), Q in zip(meshes, poses)] + [table]
    d, _ = oracle.render(objs, cam)
    z = np.where(d[0] > 0, d[0] + noise["gauss"], 0.0)
    z = np.where(noise["outlier_mask"], noise["outlier_depth"], z)
    obs = oracle.unproject(z, cam)
    rng = np.random.default_rng(2003)
    k = 3
    P = np.repeat(np.asarray(poses[k])[None], 256, axis=0)
    P[:, :3, 3] += rng.uniform(-0.08, 0.08, size=(256, 3))
    bg = [o for j, o in enumerate(objs) if j != k]
    t0 = time.perf_counter()
    d, _ = oracle.render([(meshes[k][0], meshes[k][1], P)] + bg, cam)
    oracle.score(obs, oracle.unproject(d, cam), 0.003, 0.01, 1.0, 5)
    out["table_scene_stage1"] = {"value": 256 / (time.perf_counter() - t0), "unit": "hypotheses/s",
                                 "sample": "256 hypotheses of the 6000-voxel object within +-8 cm, 320x240, "
                                           "forward with the other objects and the table as background"}
    return out


if __name__ == "__main__":
    main()
