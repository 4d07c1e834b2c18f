"""FP64 CPU oracle for the batched render-and-score path (arXiv 2312.08715).

TEST INFRASTRUCTURE ONLY: the plain, slow statement of what the GPU library
computes, written from the paper (Alg. 1's DepthRenderer and
DepthImageLikelihood, eq. (1) with the window truncation of Sec. III-B, and
the coarse-to-fine proposal of Sec. III-B).  Only the tests, the smoke check
and the benchmark's CPU-baseline leg may import it.  It shares no code with
the GPU library and never imports it.

The arithmetic lives in ``b3d_oracle.c`` (double precision, OpenMP over
hypotheses); this module compiles it with gcc and wraps it for numpy.
``tiny.py`` holds numpy brute-force versions used to pin it, and ``c2f.py``
the coarse-to-fine stage loop.
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Iterable, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "b3d_oracle.c")
_BUILD = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_BUILD, "liboracle.so")

NC = 8
C_VERT, C_TRI, C_FRONT, C_FRAG, C_PAIR, C_OBS, C_OBS_ACTIVE, C_RPIX = range(NC)

_lib = None


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (-O2, no fast-math, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        os.makedirs(_BUILD, exist_ok=True)
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE",
                               "-Wall", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def load(path: str):
    """Load an oracle shared library from `path` and declare its signatures."""
    L = ctypes.CDLL(path)
    _declare(L)
    return L


def use_library(L) -> None:
    """Route every oracle call through the already-loaded library L (None =
    the default build).  Used by the tests that plant mistakes in a copy."""
    global _lib
    _lib = L


def lib():
    global _lib
    if _lib is None:
        build()
        _lib = load(_LIB_PATH)
    return _lib


def _declare(L):
    D, I, LL = ctypes.c_double, ctypes.c_int, ctypes.c_longlong
    pd, pi, pl = ctypes.POINTER(D), ctypes.POINTER(I), ctypes.POINTER(LL)
    pu = ctypes.POINTER(ctypes.c_uint32)
    L.orc_render.argtypes = [pd, I, pi, I, I, pd, I, pd, I, I, pd, pi, pl]
    L.orc_render_frozen.argtypes = [pd, I, pi, I, I, pd, I, pd, I, I, pi, pd]
    L.orc_unproject.argtypes = [pd, I, pd, I, I, pd]
    L.orc_score.argtypes = [pd, pd, I, I, I, D, D, D, D, I, pd, pd, pl]
    L.orc_score_grad.argtypes = [pd, pd, I, I, I, D, D, D, D, I, pd, pd, pd, pd]
    L.orc_render_grad.argtypes = [pd, I, pi, I, I, pd, I, pd, I, I, pi, pd, pd, pd]
    L.orc_philox4x32_10.argtypes = [pu, pu, pu]
    L.orc_uniform.argtypes = [ctypes.c_uint64] + [ctypes.c_uint32] * 4 + [I]
    L.orc_uniform.restype = D
    L.orc_sample.argtypes = [pd, I, I, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, pd, pi, pd]
    L.orc_perturbation.argtypes = [ctypes.c_uint64, ctypes.c_uint32, I, D, pd]
    L.orc_enumerate.argtypes = [pd, pd, pi, I, pd, I, D, ctypes.c_uint64, ctypes.c_uint32, pd]
    L.orc_num_threads.restype = I
    L.orc_set_threads.argtypes = [I]
    L.orc_set_threads.restype = None
    for name in ("orc_render", "orc_render_frozen", "orc_unproject", "orc_score", "orc_score_grad",
                 "orc_render_grad", "orc_sample", "orc_enumerate"):
        getattr(L, name).restype = I


def num_threads() -> int:
    return int(lib().orc_num_threads())


def set_threads(n: int) -> None:
    """Threads of the oracle's OpenMP loops from now on."""
    lib().orc_set_threads(int(n))


def _d(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _i(a):
    return np.ascontiguousarray(a, dtype=np.int32)


def _p(a, t=ctypes.c_double):
    return None if a is None else a.ctypes.data_as(ctypes.POINTER(t))


def cam_array(cam) -> np.ndarray:
    return np.array([cam.fx, cam.fy, cam.cx, cam.cy, cam.z_near], dtype=np.float64)


def _check(rc, name):
    if rc != 0:
        raise ValueError(f"{name} rejected its arguments (rc={rc})")


def render(objects: Sequence[Tuple[np.ndarray, np.ndarray, np.ndarray]], cam, counters: bool = False,
           id_offsets: Optional[Sequence[int]] = None):
    """Render a list of (verts [V,3], tris [T,3], poses [N,4,4] or [4,4]).

    All objects must carry the same number of poses (or a single pose, which
    is broadcast).  Triangle ids of object k are offset by the total triangle
    count of objects before it unless ``id_offsets`` is given.
    Returns depth [N,H,W], ids [N,H,W] (and counters [N, NC] if asked).
    """
    Ns = [1 if np.ndim(P) == 2 else np.shape(P)[0] for _, _, P in objects]
    N = max(Ns)
    H, W = cam.H, cam.W
    depth = np.zeros((N, H, W), dtype=np.float64)
    ids = np.full((N, H, W), -1, dtype=np.int32)
    cnt = np.zeros((N, NC), dtype=np.int64)
    ca = cam_array(cam)
    off = 0
    for k, (v, t, P) in enumerate(objects):
        v, t = _d(v), _i(t)
        P = _d(P).reshape(-1, 4, 4)
        if P.shape[0] == 1 and N > 1:
            P = np.ascontiguousarray(np.broadcast_to(P, (N, 4, 4)))
        o = off if id_offsets is None else int(id_offsets[k])
        _check(lib().orc_render(_p(v), v.shape[0], _p(t, ctypes.c_int), t.shape[0], o, _p(P), N, _p(ca), H, W,
                                _p(depth), _p(ids, ctypes.c_int), _p(cnt, ctypes.c_longlong)), "orc_render")
        off += t.shape[0]
    return (depth, ids, cnt) if counters else (depth, ids)


def render_depth_fn(objects, cam) -> np.ndarray:
    """Adapter for the workload builders: depth [H,W] of a list of single-pose objects."""
    return render(objects, cam)[0][0]


def render_frozen(verts, tris, poses, cam, base_ids, id_offset: int = 0, depth: Optional[np.ndarray] = None):
    """Depth on the plane of each pixel's base triangle at the given poses."""
    v, t, P = _d(verts), _i(tris), _d(poses).reshape(-1, 4, 4)
    N = P.shape[0]
    base = _i(np.broadcast_to(base_ids, (N, cam.H, cam.W)))
    out = np.zeros((N, cam.H, cam.W)) if depth is None else _d(depth).copy()
    _check(lib().orc_render_frozen(_p(v), v.shape[0], _p(t, ctypes.c_int), t.shape[0], id_offset, _p(P), N,
                                   _p(cam_array(cam)), cam.H, cam.W, _p(base, ctypes.c_int), _p(out)),
           "orc_render_frozen")
    return out


def unproject(depth, cam) -> np.ndarray:
    """Point image q = z d for a depth image [..., H, W] (empty -> 0)."""
    depth = _d(depth)
    shp = depth.shape
    B = int(np.prod(shp[:-2])) if len(shp) > 2 else 1
    out = np.zeros(shp + (3,), dtype=np.float64)
    _check(lib().orc_unproject(_p(depth), B, _p(cam_array(cam)), cam.H, cam.W, _p(out)), "orc_unproject")
    return out


def score(obs, rend, sigma, p_out, V=1.0, window=3, M=0.0, counters: bool = False):
    """Windowed eq. (1): obs [H,W,3], rend [N,H,W,3] -> logL [N], l1 [N]."""
    obs, rend = _d(obs), _d(rend)
    if rend.ndim == 3:
        rend = rend[None]
    N, H, W, _ = rend.shape
    logL = np.zeros(N)
    l1 = np.zeros(N)
    cnt = np.zeros((N, NC), dtype=np.int64)
    _check(lib().orc_score(_p(obs), _p(rend), N, H, W, float(sigma), float(p_out), float(V), float(M), int(window),
                           _p(logL), _p(l1), _p(cnt, ctypes.c_longlong)), "orc_score")
    return (logL, l1, cnt) if counters else (logL, l1)


def score_grad(obs, rend, sigma, p_out, V=1.0, window=3, M=0.0, dlogL=None, want_rend: bool = True):
    """Adjoint of ``score``: returns d_rend [N,H,W,3] (or None), d_sigma [N], d_pout [N]."""
    obs, rend = _d(obs), _d(rend)
    if rend.ndim == 3:
        rend = rend[None]
    N, H, W, _ = rend.shape
    dl = None if dlogL is None else _d(dlogL)
    dr = np.zeros_like(rend) if want_rend else None
    ds, dp = np.zeros(N), np.zeros(N)
    _check(lib().orc_score_grad(_p(obs), _p(rend), N, H, W, float(sigma), float(p_out), float(V), float(M),
                                int(window), _p(dl), _p(dr), _p(ds), _p(dp)), "orc_score_grad")
    return dr, ds, dp


def render_grad(verts, tris, poses, cam, ids, depth, d_rend, id_offset: int = 0):
    """Pose adjoint (dt, dw) [N,6] of the render with visibility held fixed."""
    v, t, P = _d(verts), _i(tris), _d(poses).reshape(-1, 4, 4)
    N = P.shape[0]
    ids, depth, d_rend = _i(ids), _d(depth), _d(d_rend)
    out = np.zeros((N, 6))
    _check(lib().orc_render_grad(_p(v), v.shape[0], _p(t, ctypes.c_int), t.shape[0], id_offset, _p(P), N,
                                 _p(cam_array(cam)), cam.H, cam.W, _p(ids, ctypes.c_int), _p(depth), _p(d_rend),
                                 _p(out)), "orc_render_grad")
    return out


def philox(ctr: Iterable[int], key: Iterable[int]) -> Tuple[int, int, int, int]:
    c = (ctypes.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (ctypes.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (ctypes.c_uint32 * 4)()
    lib().orc_philox4x32_10(c, k, o)
    return tuple(int(x) for x in o)


def uniform(seed: int, c0: int, c1: int, c2: int, c3: int, word: int = 0) -> float:
    return float(lib().orc_uniform(seed, c0, c1, c2, c3, word))


def sample(logL, K: int, seed: int, stage: int = 0, k0: int = 0):
    """Softmax weights [N], Gumbel-max draws idx [K] and their log weights [K]."""
    logL = _d(logL)
    N = logL.shape[0]
    w = np.zeros(N)
    idx = np.zeros(K, dtype=np.int32)
    logw = np.zeros(K)
    _check(lib().orc_sample(_p(logL), N, K, seed, stage, k0, _p(w), _p(idx, ctypes.c_int), _p(logw)), "orc_sample")
    return w, idx, logw


def perturbation(seed: int, stage: int, r: int, max_angle: float) -> np.ndarray:
    R = np.zeros(9)
    lib().orc_perturbation(seed, stage, r, float(max_angle), _p(R))
    return R.reshape(3, 3)


def enumerate_grid(grid, seed: int = 0, stage: int = 0, center: Optional[np.ndarray] = None) -> np.ndarray:
    """Poses [N,4,4] of a ``workloads.GridSpec`` (optionally around another centre)."""
    c = _d(grid.center if center is None else center)
    half = _d(grid.half_extent)
    cnt = _i(grid.count)
    rots = None if grid.rotations is None else _d(grid.rotations).reshape(-1, 9)
    n_rot = grid.n_rotations
    out = np.zeros((grid.n_trans * n_rot, 4, 4))
    _check(lib().orc_enumerate(_p(c), _p(half), _p(cnt, ctypes.c_int), int(bool(grid.cell_centres)), _p(rots), n_rot,
                               float(grid.rot_max_angle), seed, stage, _p(out)), "orc_enumerate")
    return out


def observed_xyz(wl) -> np.ndarray:
    """Observed point image [H,W,3] of a workload, rendered by the oracle."""
    from workloads import assemble_observed_depth

    return unproject(assemble_observed_depth(render_depth_fn, wl), wl.camera)
