"""Python binding of the b3d HIP library (libb3d.so, gfx950).

Batched render-and-score for coarse-to-fine pose inference after Bayes3D
(arXiv 2312.08715).  This module only marshals arguments: torch tensors
supply device memory and the current HIP stream, and every computation runs
in the library's kernels.  There is no fallback: if the library is missing,
importing works but every call raises ``B3DError``.

The entry points mirror ``include/b3d.h`` one to one.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional, Sequence, Tuple

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_DIR = os.path.join(_HERE, "_lib")
LIB_PATH = os.path.join(LIB_DIR, "libb3d.so")

B3D_MAX_STAGES = 8


class B3DError(RuntimeError):
    pass


class Intrinsics(ctypes.Structure):
    _fields_ = [("fx", ctypes.c_float), ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("z_near", ctypes.c_float), ("H", ctypes.c_int32), ("W", ctypes.c_int32)]


class ScoreParams(ctypes.Structure):
    _fields_ = [("sigma", ctypes.c_float), ("p_out", ctypes.c_float), ("outlier_volume", ctypes.c_float),
                ("norm_M", ctypes.c_float), ("window", ctypes.c_int32)]


class Grid(ctypes.Structure):
    _fields_ = [("center", ctypes.c_float * 16), ("half_extent", ctypes.c_float * 3), ("count", ctypes.c_int32 * 3),
                ("cell_centres", ctypes.c_int32), ("n_rot", ctypes.c_int32), ("rot_max_angle", ctypes.c_float),
                ("rotations", ctypes.c_void_p)]


class BatchItem(ctypes.Structure):
    _fields_ = [("scene", ctypes.c_void_p), ("poses", ctypes.c_void_p), ("N", ctypes.c_int32),
                ("logL_out", ctypes.c_void_p), ("grad_out", ctypes.c_void_p)]


class TrackParams(ctypes.Structure):
    _fields_ = [("n_stages", ctypes.c_int32), ("stages", Grid * B3D_MAX_STAGES), ("n_refine", ctypes.c_int32),
                ("lr_t", ctypes.c_float), ("lr_r", ctypes.c_float), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("min_visible", ctypes.c_float),
                ("widen", ctypes.c_float)]


class Schedule(ctypes.Structure):
    _fields_ = [("n_stages", ctypes.c_int32), ("stages", Grid * B3D_MAX_STAGES)]


class Table(ctypes.Structure):
    _fields_ = [("pose", ctypes.c_float * 16), ("width", ctypes.c_float), ("height", ctypes.c_float)]


class SMCParams(ctypes.Structure):
    _fields_ = [("n_particles", ctypes.c_int32), ("n_objects", ctypes.c_int32), ("n_stages", ctypes.c_int32),
                ("counts", (ctypes.c_int32 * 3) * B3D_MAX_STAGES), ("sigma_max", ctypes.c_float),
                ("noise_A", ctypes.c_int32), ("noise_B", ctypes.c_int32), ("sigma0", ctypes.c_float),
                ("p_out0", ctypes.c_float), ("ess_threshold", ctypes.c_float), ("outlier_volume", ctypes.c_float),
                ("window", ctypes.c_int32), ("norm_M", ctypes.c_float), ("seed", ctypes.c_uint64),
                ("stage_sigma", ctypes.c_float * B3D_MAX_STAGES), ("stage_p_out", ctypes.c_float * B3D_MAX_STAGES)]


class SMCView(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("place", "dphi", "poses", "noise", "logW", "logp", "logL", "choice",
                                               "logq", "logW_pre", "noise_grid", "ancestors", "ess",
                                               "type_post")]


_lib = None

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_U32 = ctypes.c_uint32
_U64 = ctypes.c_uint64

_SIGNATURES = {
    "b3d_last_error": ([], ctypes.c_char_p),
    "b3d_version": ([], ctypes.c_char_p),
    "b3d_mesh_create": ([_P, _I32, _P, _I32, ctypes.POINTER(_P)], ctypes.c_int),
    "b3d_mesh_destroy": ([_P], ctypes.c_int),
    "b3d_mesh_layout_info": ([_P, _I32, _P, _I32, _P], ctypes.c_int),
    "b3d_mesh_info": ([_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)], ctypes.c_int),
    "b3d_unproject": ([_P, _I32, ctypes.POINTER(Intrinsics), _P, _P], ctypes.c_int),
    "b3d_render_batch": ([_P, _P, _I32, ctypes.POINTER(Intrinsics), _P, _P, _P], ctypes.c_int),
    "b3d_score_workspace_size": ([_I32, _I32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "b3d_score": ([_P, _P, _I32, _I32, _I32, ctypes.POINTER(ScoreParams), _P, _P, ctypes.c_size_t, _P], ctypes.c_int),
    "b3d_score_backward": ([_P, _P, _I32, _I32, _I32, ctypes.POINTER(ScoreParams), _P, _P, _P, _P, _P,
                            ctypes.c_size_t, _P], ctypes.c_int),
    "b3d_render_backward": ([_P, _P, _I32, ctypes.POINTER(Intrinsics), _P, _P, _P, _P], ctypes.c_int),
    "b3d_scene_create": ([_P, ctypes.POINTER(Intrinsics), ctypes.POINTER(ScoreParams), ctypes.POINTER(_P)],
                         ctypes.c_int),
    "b3d_scene_destroy": ([_P], ctypes.c_int),
    "b3d_scene_set_background": ([_P, _P, _P, _I32, _P], ctypes.c_int),
    "b3d_scene_set_observed": ([_P, _P, _P], ctypes.c_int),
    "b3d_render_score": ([_P, _P, _I32, _P, _P, _P], ctypes.c_int),
    "b3d_scene_autotune": ([_P, _P, _I32, _I32, ctypes.POINTER(_I32), _P], ctypes.c_int),
    "b3d_scene_set_tile": ([_P, _I32], ctypes.c_int),
    "b3d_scene_set_noise_grid": ([_P, _P, _I32, _P, _I32, _P, _P], ctypes.c_int),
    "b3d_noise_midpoints": ([ctypes.c_double, _I32, _I32, _P, _P], ctypes.c_int),
    "b3d_render_score_marginal": ([_P, _P, _I32, _P, _P, _P], ctypes.c_int),
    "b3d_scene_tile_limits": ([_P, ctypes.POINTER(_I32), ctypes.POINTER(_I32), ctypes.POINTER(_I32)], ctypes.c_int),
    "b3d_render_score_work": ([_P, _P, _I32, _P, _P, _P, _P], ctypes.c_int),
    "b3d_batch_create": ([ctypes.POINTER(BatchItem), _I32, ctypes.POINTER(_P)], ctypes.c_int),
    "b3d_batch_run": ([_P, _P], ctypes.c_int),
    "b3d_batch_destroy": ([_P], ctypes.c_int),
    "b3d_pose_retract": ([_P, _I32, _P, _I32, _P, _P], ctypes.c_int),
    "b3d_pose_retract_backward": ([_P, _P, _P, _I32, _P, _P, _P], ctypes.c_int),
    "b3d_scene_set_params": ([_P, ctypes.POINTER(ScoreParams), _P], ctypes.c_int),
    "b3d_refine_poses": ([_P, _P, _I32, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                          ctypes.c_float, _P], ctypes.c_int),
    "b3d_adam_pose_step": ([_P, _P, _I32, _P, _I32, _I32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                            ctypes.c_float, ctypes.c_float, _P], ctypes.c_int),
    "b3d_tracker_create": ([_P, _I32, ctypes.POINTER(Intrinsics), ctypes.POINTER(ScoreParams),
                            ctypes.POINTER(TrackParams), _P, ctypes.POINTER(_P)], ctypes.c_int),
    "b3d_tracker_frame": ([_P, _P, _P], ctypes.c_int),
    "b3d_tracker_frame_eager": ([_P, _P, _P], ctypes.c_int),
    "b3d_tracker_poses": ([_P, _P, _P], ctypes.c_int),
    "b3d_tracker_state": ([_P, _P, _P], ctypes.c_int),
    "b3d_tracker_destroy": ([_P], ctypes.c_int),
    "b3d_grid_size": ([ctypes.POINTER(Grid)], ctypes.c_int64),
    "b3d_enumerate": ([ctypes.POINTER(Grid), _U64, _I32, _P, _P], ctypes.c_int),
    "b3d_sample": ([_P, _I32, _I32, _I32, _U64, _U32, _U32, _P, _P, _P, _P], ctypes.c_int),
    "b3d_c2f_workspace_size": ([ctypes.POINTER(Schedule), _I32, ctypes.POINTER(ctypes.c_size_t)], ctypes.c_int),
    "b3d_c2f_weights_count": ([ctypes.POINTER(Schedule), _I32, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
    "b3d_c2f_step_noalloc": ([_P, _P, ctypes.POINTER(Schedule), _I32, _U64, _P, _P, _P, _P, _P], ctypes.c_int),
    "b3d_c2f_step": ([_P, _P, ctypes.POINTER(Schedule), _I32, _U64, _P, ctypes.c_size_t, _P, _P, _P, _P, _P],
                     ctypes.c_int),
    "b3d_contact_create": ([_P, _I32, ctypes.POINTER(Table), ctypes.POINTER(_P)], ctypes.c_int),
    "b3d_contact_destroy": ([_P], ctypes.c_int),
    "b3d_contact_poses": ([_P, _P, _P, _I32, _P, _P], ctypes.c_int),
    "b3d_smc_create": ([_P, _I32, _P, _P, _I32, ctypes.POINTER(Table), ctypes.POINTER(Intrinsics),
                        ctypes.POINTER(SMCParams), ctypes.POINTER(_P)], ctypes.c_int),
    "b3d_smc_reset": ([_P, _P, _P], ctypes.c_int),
    "b3d_smc_step": ([_P, _P], ctypes.c_int),
    "b3d_smc_read": ([_P, ctypes.POINTER(SMCView), ctypes.POINTER(_I32), ctypes.POINTER(ctypes.c_int64), _P],
                     ctypes.c_int),
    "b3d_smc_destroy": ([_P], ctypes.c_int),
}


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libb3d.so and declare its signatures (no GPU is touched)."""
    global _lib
    if _lib is None:
        if not os.path.exists(path):
            raise B3DError(f"HIP library not built: {path} is missing (run __graft_entry__.build())")
        L = ctypes.CDLL(path)
        for name, (args, res) in _SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def _call(name: str, *args):
    rc = getattr(load_library(), name)(*args)
    if rc != 0:
        msg = load_library().b3d_last_error().decode(errors="replace")
        raise B3DError(f"{name} failed ({rc}): {msg}")


def _ptr(t: Optional[torch.Tensor], dtype=None) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda:
        raise B3DError("expected a device tensor")
    if not t.is_contiguous():
        raise B3DError("expected a contiguous tensor")
    if dtype is not None and t.dtype != dtype:
        raise B3DError(f"expected {dtype}, got {t.dtype}")
    return t.data_ptr()


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def intrinsics(fx, fy, cx, cy, H, W, z_near=0.01) -> Intrinsics:
    return Intrinsics(float(fx), float(fy), float(cx), float(cy), float(z_near), int(H), int(W))


def intrinsics_of(cam) -> Intrinsics:
    """From an object with fx, fy, cx, cy, H, W (and optionally z_near)."""
    return intrinsics(cam.fx, cam.fy, cam.cx, cam.cy, cam.H, cam.W, getattr(cam, "z_near", 0.01))


def score_params(sigma, p_out, outlier_volume=1.0, window=3, norm_M=0.0) -> ScoreParams:
    return ScoreParams(float(sigma), float(p_out), float(outlier_volume), float(norm_M), int(window))


def version() -> str:
    return load_library().b3d_version().decode()


class Mesh:
    """Device-resident triangle mesh (b3d_mesh_create / b3d_mesh_destroy)."""

    def __init__(self, verts, tris):
        v = np.ascontiguousarray(verts, dtype=np.float32)
        t = np.ascontiguousarray(tris, dtype=np.int32)
        if v.ndim != 2 or v.shape[1] != 3 or t.ndim != 2 or t.shape[1] != 3:
            raise B3DError("verts must be [V,3] and tris [T,3]")
        h = _P()
        _call("b3d_mesh_create", v.ctypes.data, v.shape[0], t.ctypes.data, t.shape[0], ctypes.byref(h))
        self._h = h
        self.V, self.T = v.shape[0], t.shape[0]

    @property
    def handle(self):
        return self._h

    def info(self) -> Tuple[int, int, int]:
        V, T, C = _I32(), _I32(), _I32()
        _call("b3d_mesh_info", self._h, ctypes.byref(V), ctypes.byref(T), ctypes.byref(C))
        return V.value, T.value, C.value

    def close(self):
        if getattr(self, "_h", None):
            load_library().b3d_mesh_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def mesh_layout_info(verts, tris) -> dict:
    """Host-only summary of the device layout b3d_mesh_create would build."""
    v = np.ascontiguousarray(verts, dtype=np.float32)
    t = np.ascontiguousarray(tris, dtype=np.int32)
    info = np.zeros(6, dtype=np.int32)
    _call("b3d_mesh_layout_info", v.ctypes.data, v.shape[0], t.ctypes.data, t.shape[0], info.ctypes.data)
    return dict(zip(("clusters", "visible_clusters", "drawn", "hidden_pairs", "dropped", "quads"), info.tolist()))


def unproject(depth: torch.Tensor, K: Intrinsics) -> torch.Tensor:
    B = depth.numel() // (K.H * K.W)
    out = torch.empty(depth.shape + (3,), dtype=torch.float32, device=depth.device)
    _call("b3d_unproject", _ptr(depth, torch.float32), B, ctypes.byref(K), _ptr(out), _stream())
    return out


def render_batch(mesh: Mesh, poses: torch.Tensor, K: Intrinsics, want_tri: bool = True):
    """Point images [N,H,W,3] (and triangle ids [N,H,W]) of N poses [N,4,4]."""
    N = poses.shape[0]
    xyz = torch.empty((N, K.H, K.W, 3), dtype=torch.float32, device=poses.device)
    tri = torch.empty((N, K.H, K.W), dtype=torch.int32, device=poses.device) if want_tri else None
    _call("b3d_render_batch", mesh.handle, _ptr(poses, torch.float32), N, ctypes.byref(K), _ptr(xyz),
          _ptr(tri), _stream())
    return xyz, tri


_score_ws = {}


def score_workspace(H: int, W: int, device) -> torch.Tensor:
    """The split-path score's workspace for an H x W image (one per device and size, reused)."""
    key = (H, W, str(device))
    if key not in _score_ws:
        nb = ctypes.c_size_t()
        _call("b3d_score_workspace_size", int(H), int(W), ctypes.byref(nb))
        _score_ws[key] = torch.empty(int(nb.value), dtype=torch.uint8, device=device)
    return _score_ws[key]


def score(observed: torch.Tensor, rendered: torch.Tensor, p: ScoreParams, workspace: bool = True) -> torch.Tensor:
    """logL [N] of point images [N,H,W,3] (workspace=False: the kernel without the valid-pixel list)."""
    N, H, W = rendered.shape[0], rendered.shape[1], rendered.shape[2]
    out = torch.empty(N, dtype=torch.float32, device=rendered.device)
    ws = score_workspace(H, W, rendered.device) if workspace else None
    _call("b3d_score", _ptr(observed, torch.float32), _ptr(rendered, torch.float32), N, H, W, ctypes.byref(p),
          _ptr(out), _ptr(ws), 0 if ws is None else ws.numel(), _stream())
    return out


def score_backward(observed, rendered, p: ScoreParams, dlogL=None, want_rendered=True, workspace: bool = True):
    N, H, W = rendered.shape[0], rendered.shape[1], rendered.shape[2]
    dev = rendered.device
    dr = torch.empty_like(rendered) if want_rendered else None
    ds = torch.empty(N, dtype=torch.float32, device=dev)
    dp = torch.empty(N, dtype=torch.float32, device=dev)
    ws = score_workspace(H, W, dev) if workspace else None
    _call("b3d_score_backward", _ptr(observed, torch.float32), _ptr(rendered, torch.float32), N, H, W,
          ctypes.byref(p), _ptr(dlogL, torch.float32), _ptr(dr), _ptr(ds), _ptr(dp), _ptr(ws),
          0 if ws is None else ws.numel(), _stream())
    return dr, ds, dp


def render_backward(mesh: Mesh, poses, K: Intrinsics, tri, d_rendered):
    N = poses.shape[0]
    out = torch.empty((N, 6), dtype=torch.float32, device=poses.device)
    _call("b3d_render_backward", mesh.handle, _ptr(poses, torch.float32), N, ctypes.byref(K),
          _ptr(tri, torch.int32), _ptr(d_rendered, torch.float32), _ptr(out), _stream())
    return out


class Scene:
    """Moving mesh + camera + likelihood parameters + background + observation."""

    def __init__(self, mesh: Mesh, K: Intrinsics, p: ScoreParams):
        h = _P()
        _call("b3d_scene_create", mesh.handle, ctypes.byref(K), ctypes.byref(p), ctypes.byref(h))
        self._h = h
        self.mesh, self.K, self.params = mesh, K, p
        self._keep = []

    @property
    def handle(self):
        return self._h

    def set_background(self, meshes: Sequence[Mesh], poses) -> None:
        n = len(meshes)
        arr = (_P * max(n, 1))(*[m.handle for m in meshes])
        P = np.ascontiguousarray(np.asarray(poses, dtype=np.float32).reshape(n, 16)) if n else np.zeros((1, 16),
                                                                                                         np.float32)
        self._keep = list(meshes)
        _call("b3d_scene_set_background", self._h, arr, P.ctypes.data, n, _stream())

    def set_params(self, p: ScoreParams) -> None:
        """New sigma / p_out / V / normaliser (same window); background terms are recomputed."""
        _call("b3d_scene_set_params", self._h, ctypes.byref(p), _stream())
        self.params = p

    def set_observed(self, observed: torch.Tensor) -> None:
        self._obs = observed  # the scene reads it by reference
        _call("b3d_scene_set_observed", self._h, _ptr(observed, torch.float32), _stream())

    def autotune(self, poses: torch.Tensor, grad: bool = True, cache: Optional[str] = None) -> int:
        """Choose the fused kernel's depth-buffer size for this scene by timing
        the candidates on `poses`; with `cache` (a JSON file), reuse the choice
        recorded for the same shape class (image size, window, mesh size)."""
        import json

        key = f"{self.K.H}x{self.K.W}/w{self.params.window}/T{self.mesh.T}/g{int(bool(grad))}"
        if cache and os.path.exists(cache):
            with open(cache) as f:
                table = json.load(f)
            if key in table:
                _call("b3d_scene_set_tile", self._h, int(table[key]))
                return int(table[key])
        z = _I32()
        _call("b3d_scene_autotune", self._h, _ptr(poses, torch.float32), int(poses.shape[0]), int(bool(grad)),
              ctypes.byref(z), _stream())
        if cache:
            table = {}
            if os.path.exists(cache):
                with open(cache) as f:
                    table = json.load(f)
            table[key] = int(z.value)
            with open(cache, "w") as f:
                json.dump(table, f, indent=1, sort_keys=True)
        return int(z.value)

    def set_noise_grid(self, sigmas, p_outs, log_w=None) -> None:
        """Noise grid of the hierarchical likelihood: sigmas [A] x p_outs [B]
        (grid point a * B + b) with log weights [A, B] (None: equal)."""
        sg = np.ascontiguousarray(np.asarray(sigmas, dtype=np.float32).ravel())
        po = np.ascontiguousarray(np.asarray(p_outs, dtype=np.float32).ravel())
        lw = None if log_w is None else np.ascontiguousarray(np.asarray(log_w, dtype=np.float32).ravel())
        _call("b3d_scene_set_noise_grid", self._h, sg.ctypes.data, sg.size, po.ctypes.data, po.size,
              None if lw is None else lw.ctypes.data, _stream())
        self.noise_grid = (sg.size, po.size)

    def set_tile(self, zcap: int) -> None:
        _call("b3d_scene_set_tile", self._h, int(zcap))

    def tile_limits(self) -> Tuple[int, int, int]:
        """(smallest, largest, current) depth-buffer capacity in keys."""
        lo, hi, cur = _I32(), _I32(), _I32()
        _call("b3d_scene_tile_limits", self._h, ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(cur))
        return int(lo.value), int(hi.value), int(cur.value)

    def close(self):
        if getattr(self, "_h", None):
            load_library().b3d_scene_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def render_score(scene: Scene, poses: torch.Tensor, grad: bool = False):
    """logL [N] (and the adjoint [N,8] when grad) of N poses [N,4,4]."""
    N = poses.shape[0]
    logL = torch.empty(N, dtype=torch.float32, device=poses.device)
    g = torch.empty((N, 8), dtype=torch.float32, device=poses.device) if grad else None
    _call("b3d_render_score", scene.handle, _ptr(poses, torch.float32), N, _ptr(logL), _ptr(g), _stream())
    return (logL, g) if grad else logL


WORK_ITEMS = ("vertices", "triangles", "setup", "fragments", "pairs", "observed", "adjoint_pixels", "exact_tests")


def pose_retract(base: torch.Tensor, xi: torch.Tensor) -> torch.Tensor:
    """Poses [N,4,4] = (exp([w]x) R_b, t_b + dt) for xi [N,6] = (dt, w); base [N,4,4] or [1,4,4]/[4,4]."""
    N = xi.shape[0]
    b = base.reshape(-1, 16)
    out = torch.empty((N, 4, 4), dtype=torch.float32, device=xi.device)
    _call("b3d_pose_retract", _ptr(b, torch.float32), int(b.shape[0]), _ptr(xi, torch.float32), N,
          _ptr(out, torch.float32), _stream())
    return out


def pose_retract_backward(xi: torch.Tensor, grad: torch.Tensor, dlogL: Optional[torch.Tensor] = None):
    """(dxi [N,6], dsp [2]) from render_score's grad [N,8] at the retracted poses: see b3d_pose_retract_backward."""
    N = xi.shape[0]
    dxi = torch.empty((N, 6), dtype=torch.float32, device=xi.device)
    dsp = torch.empty(2, dtype=torch.float32, device=xi.device)
    _call("b3d_pose_retract_backward", _ptr(xi, torch.float32), _ptr(grad, torch.float32),
          None if dlogL is None else _ptr(dlogL, torch.float32), N, _ptr(dxi, torch.float32),
          _ptr(dsp, torch.float32), _stream())
    return dxi, dsp


class B3DScore(torch.autograd.Function):
    """logL [N] of the poses retracted from base_poses by xi [N,6] = (dt, dw),
    differentiable in xi, sigma and p_out (visibility held fixed).

    forward(xi, base_poses, sigma, p_out, scene) -> logL;
    backward(dlogL) -> (dxi, None, dsigma, dp_out, None).
    sigma and p_out (floats or 0-d tensors) replace the scene's values when
    they differ; the window, V and normaliser stay the scene's."""

    @staticmethod
    def forward(ctx, xi, base_poses, sigma, p_out, scene):
        sg, po = float(sigma), float(p_out)
        pr = scene.params
        if sg != pr.sigma or po != pr.p_out:
            scene.set_params(ScoreParams(sg, po, pr.outlier_volume, pr.norm_M, pr.window))
        xi_c = xi.detach().contiguous()
        poses = pose_retract(base_poses.detach().contiguous(), xi_c)
        logL, grad = render_score(scene, poses, grad=True)
        ctx.save_for_backward(xi_c, grad)
        ctx.sp_dev = tuple(v.device if torch.is_tensor(v) else None for v in (sigma, p_out))
        return logL

    @staticmethod
    def backward(ctx, dlogL):
        xi, grad = ctx.saved_tensors
        dxi, dsp = pose_retract_backward(xi, grad, dlogL.contiguous())
        ds, dp = (None if d is None else dsp[k].to(d) for k, d in enumerate(ctx.sp_dev))
        return dxi, None, ds, dp, None


def noise_grid_midpoints(sigma_max: float, A: int, B: int):
    """Cell centres of A equal cells of (0, sigma_max] and B of (0, 1] (b3d_noise_midpoints): with
    equal weights, the midpoint rule for the uniform priors on sigma and p_out."""
    sig = np.zeros(A, dtype=np.float32)
    po = np.zeros(B, dtype=np.float32)
    _call("b3d_noise_midpoints", float(sigma_max), int(A), int(B), sig.ctypes.data, po.ctypes.data)
    return sig, po


def render_score_marginal(scene: Scene, poses: torch.Tensor, grid: bool = False):
    """log marginal over the scene's noise grid [N] (and logL per grid point [N, A, B] when grid)."""
    A, B = scene.noise_grid
    N = poses.shape[0]
    marg = torch.empty(N, dtype=torch.float32, device=poses.device)
    g = torch.empty((N, A, B), dtype=torch.float32, device=poses.device) if grid else None
    _call("b3d_render_score_marginal", scene.handle, _ptr(poses, torch.float32), N, _ptr(g), _ptr(marg), _stream())
    return (marg, g) if grid else marg


def render_score_work(scene: Scene, poses: torch.Tensor) -> dict:
    """Work items of one fused forward+adjoint launch (instrumented kernel)."""
    N = poses.shape[0]
    logL = torch.empty(N, dtype=torch.float32, device=poses.device)
    g = torch.empty((N, 8), dtype=torch.float32, device=poses.device)
    work = torch.zeros(8, dtype=torch.int64, device=poses.device)
    _call("b3d_render_score_work", scene.handle, _ptr(poses, torch.float32), N, _ptr(logL), _ptr(g), _ptr(work),
          _stream())
    return dict(zip(WORK_ITEMS, work.cpu().tolist()))


def make_grid(center, half_extent, count, cell_centres=False, rotations: Optional[torch.Tensor] = None,
              n_rot: int = 1, rot_max_angle: float = 0.0) -> Grid:
    g = Grid()
    c = np.asarray(center, dtype=np.float64).reshape(16)
    for i in range(16):
        g.center[i] = float(c[i])
    for k in range(3):
        g.half_extent[k] = float(half_extent[k])
        g.count[k] = int(count[k])
    g.cell_centres = int(bool(cell_centres))
    if rotations is not None:
        g.n_rot = int(rotations.shape[0])
        g.rotations = _ptr(rotations, torch.float32)
    else:
        g.n_rot = int(n_rot)
        g.rotations = None
    g.rot_max_angle = float(rot_max_angle)
    return g


def grid_of(spec, device="cuda", center=None) -> Tuple[Grid, Optional[torch.Tensor]]:
    """From a workloads.GridSpec; returns the grid and the rotations tensor it references."""
    rots = None
    if spec.rotations is not None:
        rots = torch.as_tensor(np.asarray(spec.rotations, dtype=np.float32).reshape(-1, 9), device=device).contiguous()
    g = make_grid(spec.center if center is None else center, spec.half_extent, spec.count, spec.cell_centres, rots,
                  spec.n_rot, spec.rot_max_angle)
    return g, rots


def grid_size(g: Grid) -> int:
    return int(load_library().b3d_grid_size(ctypes.byref(g)))


def enumerate_grid(g: Grid, seed: int = 0, stage: int = 0, device="cuda") -> torch.Tensor:
    N = grid_size(g)
    if N <= 0:
        raise B3DError("invalid grid")
    out = torch.empty((N, 4, 4), dtype=torch.float32, device=device)
    _call("b3d_enumerate", ctypes.byref(g), int(seed), int(stage), _ptr(out), _stream())
    return out


def sample(logL: torch.Tensor, K: int, seed: int, stage: int = 0, k0: int = 0, weights: bool = True):
    """logL [P,N] or [N] -> weights [P,N], idx [P,K], logw [P,K] (segment axis squeezed for 1-D input)."""
    squeeze = logL.dim() == 1
    L = logL.reshape(1, -1) if squeeze else logL
    P, N = L.shape
    dev = L.device
    w = torch.empty((P, N), dtype=torch.float32, device=dev) if weights else None
    idx = torch.empty((P, K), dtype=torch.int32, device=dev)
    lw = torch.empty((P, K), dtype=torch.float32, device=dev)
    _call("b3d_sample", _ptr(L.contiguous(), torch.float32), P, N, K, int(seed), int(stage), int(k0), _ptr(w),
          _ptr(idx), _ptr(lw), _stream())
    if squeeze:
        return (None if w is None else w[0]), idx[0], lw[0]
    return w, idx, lw


def make_schedule(stages: Sequence[Grid]) -> Schedule:
    if not 1 <= len(stages) <= B3D_MAX_STAGES:
        raise B3DError("schedule needs 1..8 stages")
    s = Schedule()
    s.n_stages = len(stages)
    for i, g in enumerate(stages):
        s.stages[i] = g
    return s


def c2f_step(scene: Scene, center, schedule: Schedule, K: int, seed: int, device="cuda", weights: bool = False):
    """Coarse-to-fine proposal for K particles: poses [K,4,4], logq [K], idx [n_stages,K]
    (and, when weights, the cell probabilities of every stage: a list whose
    entry 0 is [N_0] and entry t >= 1 is [K, N_t])."""
    nb = ctypes.c_size_t()
    _call("b3d_c2f_workspace_size", ctypes.byref(schedule), int(K), ctypes.byref(nb))
    ws = torch.empty(max(int(nb.value), 1), dtype=torch.uint8, device=device)
    c = np.ascontiguousarray(np.asarray(center, dtype=np.float32).reshape(16))
    poses = torch.empty((K, 4, 4), dtype=torch.float32, device=device)
    logq = torch.empty(K, dtype=torch.float32, device=device)
    idx = torch.empty((schedule.n_stages, K), dtype=torch.int32, device=device)
    w = None
    if weights:
        nw = ctypes.c_int64()
        _call("b3d_c2f_weights_count", ctypes.byref(schedule), int(K), ctypes.byref(nw))
        w = torch.empty(int(nw.value), dtype=torch.float32, device=device)
    _call("b3d_c2f_step", scene.handle, c.ctypes.data, ctypes.byref(schedule), int(K), int(seed), _ptr(ws),
          int(nb.value), _ptr(w), _ptr(poses), _ptr(logq), _ptr(idx), _stream())
    if not weights:
        return poses, logq, idx
    per, off = [], 0
    for t in range(schedule.n_stages):
        n = grid_size(schedule.stages[t])
        per.append(w[off:off + n] if t == 0 else w[off:off + K * n].view(K, n))
        off += n if t == 0 else K * n
    return poses, logq, idx, per


def c2f_step_noalloc(scene: Scene, center, schedule: Schedule, K: int, seed: int, poses: torch.Tensor,
                     logq: torch.Tensor, idx: Optional[torch.Tensor] = None,
                     weights: Optional[torch.Tensor] = None) -> None:
    """b3d_c2f_step_noalloc: c2f_step into caller-allocated outputs (poses
    [K,4,4], logq [K], idx [n_stages,K] or None, weights [b3d_c2f_weights_count]
    or None), its workspace in the library's fixed device array."""
    c = np.ascontiguousarray(np.asarray(center, dtype=np.float32).reshape(16))
    _call("b3d_c2f_step_noalloc", scene.handle, c.ctypes.data, ctypes.byref(schedule), int(K), int(seed), _ptr(weights),
          _ptr(poses), _ptr(logq), _ptr(idx), _stream())


class Batch:
    """Many scenes in few launches (b3d_batch_create / b3d_batch_run).

    ``items`` is a list of (scene, poses [N,4,4]); outputs are allocated here:
    ``logL[i]`` [N_i] and, with grad, ``grad[i]`` [N_i, 8]."""

    def __init__(self, items, grad: bool = False):
        self.scenes = [s for s, _ in items]
        self.poses = [P.contiguous() for _, P in items]
        self.logL = [torch.empty(P.shape[0], dtype=torch.float32, device=P.device) for P in self.poses]
        self.grad = [torch.empty((P.shape[0], 8), dtype=torch.float32, device=P.device) for P in self.poses] \
            if grad else None
        arr = (BatchItem * len(items))()
        for i, (s, P) in enumerate(zip(self.scenes, self.poses)):
            arr[i] = BatchItem(s.handle.value if hasattr(s.handle, "value") else s.handle, _ptr(P, torch.float32),
                               int(P.shape[0]), _ptr(self.logL[i]), _ptr(self.grad[i]) if grad else None)
        h = _P()
        _call("b3d_batch_create", arr, len(items), ctypes.byref(h))
        self._h = h

    def run(self):
        _call("b3d_batch_run", self._h, _stream())
        return (self.logL, self.grad) if self.grad is not None else self.logL

    def close(self):
        if getattr(self, "_h", None):
            load_library().b3d_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def refine_poses(scene: Scene, poses: torch.Tensor, n_refine: int, lr_t: float, lr_r: float, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8) -> None:
    """In place: n_refine Adam steps on logL for each pose [N,4,4] (one workgroup per pose)."""
    _call("b3d_refine_poses", scene.handle, _ptr(poses, torch.float32), int(poses.shape[0]), int(n_refine),
          float(lr_t), float(lr_r), float(beta1), float(beta2), float(eps), _stream())


def adam_pose_step(poses: torch.Tensor, grad: torch.Tensor, state: torch.Tensor, it: int, lr_t: float, lr_r: float,
                   beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    """In-place Adam ascent on logL for poses [N,4,4] given grad [N,G>=6] and state [N,12]."""
    N = poses.shape[0]
    _call("b3d_adam_pose_step", _ptr(poses, torch.float32), _ptr(grad, torch.float32), int(grad.shape[1]),
          _ptr(state, torch.float32), N, int(it), float(lr_t), float(lr_r), float(beta1), float(beta2), float(eps),
          _stream())


class Tracker:
    """Graph-captured multi-object tracker (b3d_tracker_*)."""

    def __init__(self, meshes: Sequence[Mesh], K: Intrinsics, p: ScoreParams, grid, init_poses,
                 n_refine: int = 10, lr_t: float = 1e-3, lr_r: float = 1e-2, beta1: float = 0.9,
                 beta2: float = 0.999, eps: float = 1e-8, min_visible: float = 0.0, widen: float = 1.0):
        """grid: one Grid, or a sequence of Grids searched stage by stage each frame.
        min_visible > 0: drop an object's update when less than that fraction
        of its pixels is in front of the others and confirmed by the
        observation (it then moves by its last accepted motion) and widen the
        next frame's stage 0 translations by `widen`."""
        self.meshes = list(meshes)
        M = len(self.meshes)
        arr = (_P * M)(*[m.handle for m in self.meshes])
        P0 = np.ascontiguousarray(np.asarray(init_poses, dtype=np.float32).reshape(M, 16))
        grids = [grid] if isinstance(grid, Grid) else list(grid)
        if not 1 <= len(grids) <= B3D_MAX_STAGES:
            raise B3DError(f"tracker: 1..{B3D_MAX_STAGES} stages")
        st = (Grid * B3D_MAX_STAGES)(*grids)
        tp = TrackParams(len(grids), st, int(n_refine), float(lr_t), float(lr_r), float(beta1), float(beta2),
                         float(eps), float(min_visible), float(widen))
        h = _P()
        _call("b3d_tracker_create", arr, M, ctypes.byref(K), ctypes.byref(p), ctypes.byref(tp), P0.ctypes.data,
              ctypes.byref(h))
        self._h = h
        self.M = M

    def frame(self, observed: torch.Tensor, eager: bool = False) -> None:
        _call("b3d_tracker_frame_eager" if eager else "b3d_tracker_frame", self._h, _ptr(observed, torch.float32),
              _stream())

    def poses(self) -> torch.Tensor:
        out = torch.empty((self.M, 4, 4), dtype=torch.float32, device="cuda")
        _call("b3d_tracker_poses", self._h, _ptr(out), _stream())
        return out

    def state(self) -> torch.Tensor:
        """[M, 3]: seen fraction of the last update, dropped updates in a row, next stage 0 scale."""
        out = torch.empty((self.M, 3), dtype=torch.float32, device="cuda")
        _call("b3d_tracker_state", self._h, _ptr(out), _stream())
        return out

    def close(self):
        if getattr(self, "_h", None):
            load_library().b3d_tracker_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def table(pose, width: float, height: float) -> Table:
    """The table: pose maps its frame (top at z = 0, +z up) to the camera."""
    return Table((ctypes.c_float * 16)(*np.asarray(pose, dtype=np.float32).reshape(16).tolist()), float(width),
                 float(height))


class Contact:
    """A type library placed by contact on a table (b3d_contact_create): every
    type's six resting faces uploaded once."""

    def __init__(self, types: Sequence[Mesh], tbl: Table):
        arr = (_P * len(types))(*[m.handle for m in types])
        h = _P()
        _call("b3d_contact_create", arr, len(types), ctypes.byref(tbl), ctypes.byref(h))
        self._h = h

    @property
    def handle(self):
        return self._h

    def poses(self, place: torch.Tensor, dphi: torch.Tensor) -> torch.Tensor:
        """Camera-frame poses [N,4,4] of objects resting on the table: place [N,2]
        (type, face) int32, dphi [N,3] (dx, dy, dtheta)."""
        N = place.shape[0]
        out = torch.empty((N, 4, 4), dtype=torch.float32, device=place.device)
        _call("b3d_contact_poses", self._h, _ptr(place, torch.int32), _ptr(dphi, torch.float32), N, _ptr(out),
              _stream())
        return out

    def close(self):
        if getattr(self, "_h", None):
            load_library().b3d_contact_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def smc_params(n_particles, n_objects, counts, sigma_max, noise_A, noise_B, sigma0, p_out0, ess_threshold,
               outlier_volume=1.0, window=5, norm_M=0.0, seed=0, stage_noise=None) -> SMCParams:
    """stage_noise: per placement stage (sigma, p_out) at which its cells are
    scored, or None (each particle's current noise at every stage)."""
    if not 1 <= len(counts) <= B3D_MAX_STAGES:
        raise B3DError(f"smc: 1..{B3D_MAX_STAGES} stages")
    c = ((ctypes.c_int32 * 3) * B3D_MAX_STAGES)()
    for t, x in enumerate(counts):
        for k in range(3):
            c[t][k] = int(x[k])
    ss, sp = (ctypes.c_float * B3D_MAX_STAGES)(), (ctypes.c_float * B3D_MAX_STAGES)()
    if stage_noise is not None:
        for t, (s, q) in enumerate(stage_noise):
            ss[t], sp[t] = float(s), float(q)
    return SMCParams(int(n_particles), int(n_objects), len(counts), c, float(sigma_max), int(noise_A), int(noise_B),
                     float(sigma0), float(p_out0), float(ess_threshold), float(outlier_volume), int(window),
                     float(norm_M), int(seed), ss, sp)


class SMC:
    """Sequential Monte Carlo over the objects of a table scene (b3d_smc_*)."""

    def __init__(self, types: Sequence[Mesh], tbl: Table, K: Intrinsics, p: SMCParams,
                 fixed: Sequence[Mesh] = (), fixed_poses=None):
        self.types = list(types)
        self.fixed = list(fixed)
        self.p = p
        arr = (_P * len(self.types))(*[m.handle for m in self.types])
        fx = (_P * max(1, len(self.fixed)))(*[m.handle for m in self.fixed])
        fp = np.ascontiguousarray(np.asarray(fixed_poses if fixed_poses is not None else np.zeros((0, 16)),
                                             dtype=np.float32).reshape(-1, 16))
        h = _P()
        _call("b3d_smc_create", arr, len(self.types), fx, fp.ctypes.data if len(self.fixed) else None,
              len(self.fixed), ctypes.byref(tbl), ctypes.byref(K), ctypes.byref(p), ctypes.byref(h))
        self._h = h
        self._observed = None

    def reset(self, observed: torch.Tensor) -> None:
        self._observed = observed  # read by pointer until the next reset
        _call("b3d_smc_reset", self._h, _ptr(observed, torch.float32), _stream())

    def step(self) -> None:
        _call("b3d_smc_step", self._h, _stream())

    def read(self) -> dict:
        M, n, T = self.p.n_particles, self.p.n_objects, self.p.n_stages
        AB = self.p.noise_A * self.p.noise_B
        d = "cuda"
        out = dict(place=torch.empty((M, n, 2), dtype=torch.int32, device=d),
                   dphi=torch.empty((M, n, 3), dtype=torch.float32, device=d),
                   poses=torch.empty((M, n, 4, 4), dtype=torch.float32, device=d),
                   noise=torch.empty((M, 2), dtype=torch.float32, device=d),
                   logW=torch.empty(M, dtype=torch.float64, device=d),
                   logp=torch.empty(M, dtype=torch.float64, device=d),
                   logL=torch.empty(M, dtype=torch.float32, device=d),
                   choice=torch.empty((T, M), dtype=torch.int32, device=d),
                   logq=torch.empty(M, dtype=torch.float64, device=d),
                   logW_pre=torch.empty(M, dtype=torch.float64, device=d),
                   noise_grid=torch.empty((M, AB), dtype=torch.float32, device=d),
                   ancestors=torch.empty(M, dtype=torch.int32, device=d),
                   ess=torch.empty(1, dtype=torch.float64, device=d),
                   type_post=torch.empty((M, len(self.types)), dtype=torch.float32, device=d))
        v = SMCView(*[_ptr(out[k]) for k, _ in SMCView._fields_])
        k, ns = _I32(), ctypes.c_int64()
        _call("b3d_smc_read", self._h, ctypes.byref(v), ctypes.byref(k), ctypes.byref(ns), _stream())
        torch.cuda.current_stream().synchronize()
        out["placed"] = int(k.value)
        out["scored"] = int(ns.value)
        return out

    def close(self):
        if getattr(self, "_h", None):
            load_library().b3d_smc_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
