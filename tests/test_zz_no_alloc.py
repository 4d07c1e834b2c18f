"""b3d_c2f_step_noalloc (workspace in the library's fixed device array)
against b3d_c2f_step (caller workspace) through the C ABI: two calls in a
row, the second with a smaller schedule and fewer particles, each equal to
the workspace entry point's results; a schedule above the array's limit is
refused before any launch."""

import ctypes

import numpy as np
import pytest
import torch

import oracle
from workloads import GridSpec, make_config, pose_matrix

pytestmark = pytest.mark.gpu


def f32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def _outputs(b3d, sched, K):
    nw = ctypes.c_int64()
    b3d._call("b3d_c2f_weights_count", ctypes.byref(sched), int(K), ctypes.byref(nw))
    return (torch.full((K, 4, 4), np.nan, device="cuda"), torch.full((K,), np.nan, device="cuda"),
            torch.full((sched.n_stages, K), -7, dtype=torch.int32, device="cuda"),
            torch.full((int(nw.value),), np.nan, device="cuda"))


def test_c2f_step_noalloc_equals_the_workspace_entry_point():
    import paper_2312_08715_amd as b3d

    assert torch.cuda.is_available(), "GPU tests need a device"
    b3d.load_library()
    wl = make_config(0)
    wl.verts = f32(wl.verts)
    obs = f32(oracle.observed_xyz(wl))
    mesh = b3d.Mesh(wl.verts, wl.tris)
    scene = b3d.Scene(mesh, b3d.intrinsics_of(wl.camera), b3d.score_params(0.01, 0.3, 1.0, 3))
    scene.set_observed(dev(obs))
    centre = pose_matrix(np.eye(3), (0.0, 0.0, 0.8))
    big = [GridSpec(center=centre, half_extent=(0.05, 0.05, 0.05), count=(8, 8, 4), n_rot=6, rot_max_angle=0.2),
           GridSpec(center=centre, half_extent=(0.01, 0.01, 0.01), count=(5, 5, 5), n_rot=4, rot_max_angle=0.05)]
    small = [GridSpec(center=centre, half_extent=(0.03, 0.03, 0.03), count=(4, 4, 2), n_rot=2, rot_max_angle=0.1)]
    for specs, K, seed in ((big, 24, 11), (small, 5, 12)):
        grids = [b3d.grid_of(g) for g in specs]
        sched = b3d.make_schedule([g for g, _ in grids])
        P_ref, lq_ref, idx_ref, W_ref = b3d.c2f_step(scene, centre, sched, K, seed, weights=True)
        P, lq, idx, w = _outputs(b3d, sched, K)
        b3d.c2f_step_noalloc(scene, centre, sched, K, seed, P, lq, idx, w)
        torch.cuda.synchronize()
        print(f"no-alloc c2f: {len(specs)} stages, K={K}: idx {idx[-1].tolist()}", flush=True)
        # the same kernels on the same inputs: equal bit for bit
        assert torch.equal(P, P_ref) and torch.equal(lq, lq_ref) and torch.equal(idx, idx_ref)
        assert torch.equal(w, torch.cat([W_ref[0]] + [x.reshape(-1) for x in W_ref[1:]]))
    # a schedule above the fixed array's limit is refused on the host
    huge = [GridSpec(center=centre, half_extent=(0.05, 0.05, 0.05), count=(64, 64, 16), n_rot=4, rot_max_angle=0.2)]
    grids = [b3d.grid_of(g) for g in huge]
    sched = b3d.make_schedule([g for g, _ in grids])
    P, lq, idx, _ = _outputs(b3d, sched, 2)
    with pytest.raises(b3d.B3DError, match="limit"):
        b3d.c2f_step_noalloc(scene, centre, sched, 2, 1, P, lq, idx)
    assert torch.isnan(P).all()  # nothing was launched
