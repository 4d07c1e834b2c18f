"""Seeded synthetic scenes shaped like the paper's tabletop workloads.

The paper's objects are learned voxel models (Fig. 1 caption): a point cloud is
discretised at a fixed resolution and a cube is placed at every occupied cell.
The YCB meshes it uses are not available, so seeded voxel blobs of the same
construction stand in for them. Everything here is random draws and geometry
layout; renders are produced by a caller-supplied function.

Conventions (shared by both sides of every test, stated once here):
  * lengths in metres, 1 voxel = 1 cm cube, 8 unshared vertices and 12
    triangles per voxel, counter-clockwise winding seen from outside;
  * camera frame is +z forward, +x right, +y down; a pose is a 4x4 row-major
    object-to-camera transform;
  * hypothesis grids are described by ``GridSpec`` (centre pose, per-axis
    half-extent and count, delta rotations); expanding a spec into poses is
    the method's first step and is done by each side itself.
"""

from __future__ import annotations

import dataclasses
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

VOXEL = 0.01  # voxel edge, metres

# Corner k of a unit cube has coordinates ((k>>0)&1, (k>>1)&1, (k>>2)&1).
# Each face is two triangles with outward normals (counter-clockwise from
# outside).
_CUBE_TRIS = np.array(
    [
        [0, 4, 6], [0, 6, 2],  # -x
        [1, 3, 7], [1, 7, 5],  # +x
        [0, 1, 5], [0, 5, 4],  # -y
        [2, 6, 7], [2, 7, 3],  # +y
        [0, 2, 3], [0, 3, 1],  # -z
        [4, 5, 7], [4, 7, 6],  # +z
    ],
    dtype=np.int32,
)
_CUBE_CORNERS = np.array([[(k >> 0) & 1, (k >> 1) & 1, (k >> 2) & 1] for k in range(8)], dtype=np.float64)


@dataclasses.dataclass
class Camera:
    """Pinhole intrinsics (pixels) and image size."""

    fx: float
    fy: float
    cx: float
    cy: float
    H: int
    W: int
    z_near: float = 0.01


@dataclasses.dataclass
class GridSpec:
    """A hypothesis grid around a centre pose.

    Hypothesis n = r * (nx*ny*nz) + (ix*ny + iy)*nz + iz has translation
    t_c + (dx[ix], dy[iy], dz[iz]) and rotation dR[r] @ R_c.  Per-axis offsets
    are ``linspace(-h, h, n)`` (``cell_centres=False``; a single sample sits at
    0) or the centres of n equal cells of [-h, h] (``cell_centres=True``, the
    partition form of a coarse-to-fine schedule).  ``rotations`` holds explicit
    delta rotations; when it is None, ``n_rot`` perturbations with angle at
    most ``rot_max_angle`` are drawn from the counter-based generator (index 0
    is the identity).
    """

    center: np.ndarray
    half_extent: Tuple[float, float, float]
    count: Tuple[int, int, int]
    cell_centres: bool = False
    rotations: Optional[np.ndarray] = None
    n_rot: int = 1
    rot_max_angle: float = 0.0

    @property
    def n_trans(self) -> int:
        return int(self.count[0]) * int(self.count[1]) * int(self.count[2])

    @property
    def n_rotations(self) -> int:
        return int(self.rotations.shape[0]) if self.rotations is not None else int(self.n_rot)

    @property
    def N(self) -> int:
        return self.n_trans * self.n_rotations


@dataclasses.dataclass
class ScoreParams:
    sigma: float
    p_out: float
    outlier_volume: float
    window: int
    norm_M: float = 0.0  # <= 0 means H*W


@dataclasses.dataclass
class Workload:
    name: str
    verts: np.ndarray  # [V,3] float64, object frame
    tris: np.ndarray  # [T,3] int32
    camera: Camera
    true_pose: np.ndarray  # [4,4]
    grid: GridSpec
    score: ScoreParams
    noise: dict  # gauss [H,W], outlier_mask [H,W] bool, outlier_depth [H,W]
    occluder: Optional[Tuple[np.ndarray, np.ndarray, np.ndarray]] = None  # verts, tris, pose
    occluder_target: Optional[float] = None
    statics: List[Tuple[np.ndarray, np.ndarray, np.ndarray]] = dataclasses.field(default_factory=list)
    seeds: dict = dataclasses.field(default_factory=dict)


def pose_matrix(R: np.ndarray, t: Sequence[float]) -> np.ndarray:
    P = np.eye(4)
    P[:3, :3] = R
    P[:3, 3] = t
    return P


def voxel_blob(n_vox: int, rng: np.random.Generator, radius: Optional[float] = None) -> np.ndarray:
    """Centres of ``n_vox`` distinct 1 cm lattice cells inside a ball.

    The ball radius is max(10 cm, 1 cm * (6 n / 4 pi)^(1/3)), which keeps the
    occupied fraction at most one half.  Returns [n_vox, 3] float64 centres.
    """
    if radius is None:
        radius = max(0.10, VOXEL * (6.0 * n_vox / (4.0 * np.pi)) ** (1.0 / 3.0))
    m = int(np.floor(radius / VOXEL))
    ax = np.arange(-m, m + 1)
    g = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3)
    inside = g[(g.astype(np.float64) ** 2).sum(1) * VOXEL**2 <= radius**2]
    if n_vox > inside.shape[0]:
        raise ValueError("ball too small for the requested voxel count")
    pick = rng.choice(inside.shape[0], size=n_vox, replace=False)
    return inside[np.sort(pick)].astype(np.float64) * VOXEL


def box_mesh(size: Sequence[float], centre: Sequence[float] = (0.0, 0.0, 0.0)) -> Tuple[np.ndarray, np.ndarray]:
    """Axis-aligned box of the given edge lengths: 8 vertices, 12 triangles."""
    size = np.asarray(size, dtype=np.float64)
    v = (_CUBE_CORNERS - 0.5) * size + np.asarray(centre, dtype=np.float64)
    return v, _CUBE_TRIS.copy()


def voxel_mesh(centres: np.ndarray, edge: float = VOXEL) -> Tuple[np.ndarray, np.ndarray]:
    """One cube per voxel centre; vertices are not shared between voxels."""
    centres = np.asarray(centres, dtype=np.float64)
    n = centres.shape[0]
    verts = centres[:, None, :] + (_CUBE_CORNERS[None, :, :] - 0.5) * edge
    tris = _CUBE_TRIS[None, :, :] + 8 * np.arange(n, dtype=np.int32)[:, None, None]
    return verts.reshape(-1, 3), tris.reshape(-1, 3).astype(np.int32)


def shoemake_rotations(n: int, rng: np.random.Generator) -> np.ndarray:
    """Uniform random rotations by Shoemake's method (Graphics Gems III)."""
    u = rng.random((n, 3))
    a, b = np.sqrt(1.0 - u[:, 0]), np.sqrt(u[:, 0])
    qx, qy = a * np.sin(2 * np.pi * u[:, 1]), a * np.cos(2 * np.pi * u[:, 1])
    qz, qw = b * np.sin(2 * np.pi * u[:, 2]), b * np.cos(2 * np.pi * u[:, 2])
    R = np.empty((n, 3, 3))
    R[:, 0, 0] = 1 - 2 * (qy * qy + qz * qz)
    R[:, 0, 1] = 2 * (qx * qy - qz * qw)
    R[:, 0, 2] = 2 * (qx * qz + qy * qw)
    R[:, 1, 0] = 2 * (qx * qy + qz * qw)
    R[:, 1, 1] = 1 - 2 * (qx * qx + qz * qz)
    R[:, 1, 2] = 2 * (qy * qz - qx * qw)
    R[:, 2, 0] = 2 * (qx * qz - qy * qw)
    R[:, 2, 1] = 2 * (qy * qz + qx * qw)
    R[:, 2, 2] = 1 - 2 * (qx * qx + qy * qy)
    return R


def rotation_grid(n: int, max_angle: float) -> np.ndarray:
    """Small rotations on a lattice of rotation vectors: every (i, j, k) with
    each component one of linspace(-max_angle, max_angle, n) radians, turned
    into a matrix by Rodrigues' formula.  Returns [n^3, 3, 3] float64 in
    lattice order (k fastest); for odd n the middle entry is the identity."""
    ax = np.linspace(-max_angle, max_angle, n) if n > 1 else np.zeros(1)
    out = []
    for a in ax:
        for b in ax:
            for c in ax:
                w = np.array([a, b, c])
                th = np.linalg.norm(w)
                K = np.zeros((3, 3))
                if th > 0:
                    k = w / th
                    K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
                out.append(np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * (K @ K))
    return np.stack(out)


def observation_noise(H: int, W: int, rng: np.random.Generator, depth_noise: float, outlier_frac: float,
                      depth_range: Tuple[float, float] = (0.3, 1.5)) -> dict:
    """Per-pixel draws for the synthetic observation process.

    Every surface pixel gets N(0, depth_noise) added to its depth; then every
    pixel, with probability ``outlier_frac``, is replaced by a depth drawn
    uniformly from ``depth_range``.
    """
    return {
        "gauss": rng.normal(0.0, depth_noise, size=(H, W)),
        "outlier_mask": rng.random((H, W)) < outlier_frac,
        "outlier_depth": rng.uniform(depth_range[0], depth_range[1], size=(H, W)),
    }


RenderFn = Callable[[List[Tuple[np.ndarray, np.ndarray, np.ndarray]], Camera], np.ndarray]


def assemble_observed_depth(render: RenderFn, wl: "Workload") -> np.ndarray:
    """Observed depth image [H,W] for a workload.

    ``render(objects, camera)`` must return the depth image [H,W] of the list
    of (verts, tris, pose) objects (0 where empty).  The object at its true
    pose, the static objects and the occluder (if any) are rendered together;
    surface pixels get the Gaussian draw added; outlier pixels are replaced.
    """
    objs = [(wl.verts, wl.tris, wl.true_pose)] + list(wl.statics)
    if wl.occluder is not None:
        objs.append(wl.occluder)
    z = np.asarray(render(objs, wl.camera), dtype=np.float64)
    z = np.where(z > 0, z + wl.noise["gauss"], 0.0)
    return np.where(wl.noise["outlier_mask"], wl.noise["outlier_depth"], z)


def place_occluder(render: RenderFn, verts: np.ndarray, tris: np.ndarray, pose: np.ndarray, cam: Camera,
                   rng: np.random.Generator, target: float, tol: float, front_z: float = 0.6,
                   thickness: float = 0.06, side: float = 0.2) -> Tuple[np.ndarray, np.ndarray, np.ndarray]:
    """Slide a box occluder across the object until it hides ``target`` of it.

    The box (``side`` x ``side`` x ``thickness``, front face at ``front_z``) is
    turned about the optical axis by a seeded angle and moved along a seeded
    image direction; bisection on the offset stops once the covered fraction of
    the object's pixels is within ``tol`` of ``target``.
    """
    bv, bt = box_mesh((side, side, thickness))
    theta = rng.uniform(0, 2 * np.pi)
    psi = theta + rng.uniform(0.2, 0.6)
    c, s = np.cos(psi), np.sin(psi)
    Rz = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    obj = np.asarray(render([(verts, tris, pose)], cam)) > 0
    n_obj = int(obj.sum())
    if n_obj == 0:
        raise ValueError("object not visible")
    axis_pt = pose[:3, 3] * ((front_z + thickness / 2) / pose[2, 3])
    dirv = np.array([np.cos(theta), np.sin(theta), 0.0])

    def occ_pose(off):
        return pose_matrix(Rz, axis_pt + off * dirv)

    def frac(off):
        occ = np.asarray(render([(bv, bt, occ_pose(off))], cam)) > 0
        return float((occ & obj).sum()) / n_obj

    lo, hi = 0.0, 0.5  # frac(lo) ~ 1, frac(hi) = 0
    for _ in range(80):
        mid = 0.5 * (lo + hi)
        f = frac(mid)
        if abs(f - target) <= tol:
            return bv, bt, occ_pose(mid)
        if f > target:
            lo = mid
        else:
            hi = mid
    raise RuntimeError("occluder bisection did not reach the target coverage")


def _config0() -> Workload:
    k = 0
    rs, ro = np.random.default_rng(1000 + k), np.random.default_rng(2000 + k)
    verts, tris = voxel_mesh(voxel_blob(500, rs, radius=0.10))
    cam = Camera(60.0, 60.0, 32.0, 24.0, 48, 64)
    true_pose = pose_matrix(np.eye(3), (0.0, 0.0, 0.8))
    grid = GridSpec(center=true_pose.copy(), half_extent=(0.05, 0.05, 0.05), count=(8, 8, 4))
    noise = observation_noise(cam.H, cam.W, ro, 0.002, 0.05)
    return Workload("plain-small 64x48 6k tris 256 hyp", verts, tris, cam, true_pose, grid,
                    ScoreParams(0.005, 0.01, 1.0, 3), noise,
                    seeds={"scene": 1000 + k, "obs": 2000 + k, "hyp": 3000 + k, "sampler": 4000 + k})


def _config1() -> Workload:
    k = 1
    rs, ro, rh = (np.random.default_rng(s + k) for s in (1000, 2000, 3000))
    verts, tris = voxel_mesh(voxel_blob(2000, rs))
    cam = Camera(150.0, 150.0, 80.0, 60.0, 120, 160)
    rots = shoemake_rotations(50, rh)
    centre = pose_matrix(np.eye(3), (0.0, 0.0, 0.8))
    true_pose = pose_matrix(rots[0], (0.0, 0.0, 0.8))
    grid = GridSpec(center=centre, half_extent=(0.04, 0.04, 0.0), count=(10, 10, 1), rotations=rots)
    noise = observation_noise(cam.H, cam.W, ro, 0.002, 0.03)
    wl = Workload("plain-paper-scale 160x120 24k tris 5000 hyp", verts, tris, cam, true_pose, grid,
                  ScoreParams(0.003, 0.01, 1.0, 5), noise, occluder_target=0.20,
                  seeds={"scene": 1000 + k, "obs": 2000 + k, "hyp": 3000 + k, "sampler": 4000 + k})
    wl.seeds["occluder_rng"] = ro  # the occluder's draws continue the observation stream
    return wl


def make_config(k: int, render: Optional[RenderFn] = None) -> Workload:
    """Workload k (0: 64x48/6k tris/256 hypotheses; 1: 160x120/24k tris/5000).

    When the workload has an occluder, ``render`` is needed to place it.
    """
    if k == 0:
        return _config0()
    if k == 1:
        wl = _config1()
        ro = wl.seeds.pop("occluder_rng")
        if render is not None:
            wl.occluder = place_occluder(render, wl.verts, wl.tris, wl.true_pose, wl.camera, ro,
                                         target=wl.occluder_target, tol=0.005)
        return wl
    raise ValueError(f"unknown workload {k}")


def tiny_scene(rng: np.random.Generator, n_vox: int, H: int, W: int, f: float = 40.0,
               depth: float = 0.5) -> Tuple[np.ndarray, np.ndarray, Camera]:
    """A few-voxel object and a small camera for brute-force checks."""
    centres = voxel_blob(n_vox, rng, radius=0.04)
    verts, tris = voxel_mesh(centres)
    return verts, tris, Camera(f, f, W / 2.0 + 0.13, H / 2.0 - 0.21, H, W)


def random_poses(rng: np.random.Generator, n: int, depth: float, spread: float) -> np.ndarray:
    """Uniform rotations with translations near (0, 0, depth)."""
    R = shoemake_rotations(n, rng)
    P = np.tile(np.eye(4), (n, 1, 1))
    P[:, :3, :3] = R
    P[:, :3, 3] = rng.uniform(-spread, spread, size=(n, 3)) + np.array([0.0, 0.0, depth])
    return P


def random_scene_batch(rng: np.random.Generator, n_scenes: int):
    """Scene shapes for the many-scenes batch (object counts, voxel counts, sizes, N)."""
    sizes = [(120, 160), (180, 240), (240, 320)]
    out = []
    for _ in range(n_scenes):
        n_obj = int(np.round(np.exp(rng.uniform(np.log(1), np.log(8)))))
        vox = [int(np.round(np.exp(rng.uniform(np.log(500), np.log(8000))))) for _ in range(n_obj)]
        H, W = sizes[rng.integers(0, 3)]
        N = int(np.round(np.exp(rng.uniform(np.log(1000), np.log(20000)))))
        out.append({"n_obj": n_obj, "voxels": vox, "H": H, "W": W, "N": N})
    return out


def smooth_trajectory(rng: np.random.Generator, n_frames: int, start: np.ndarray, max_step_t: float = 0.02,
                      max_step_r: float = np.deg2rad(5.0)) -> np.ndarray:
    """Poses [n_frames, 4, 4]: translation and rotation vector each a sum of
    three seeded sinusoids per axis, scaled so that no frame-to-frame change
    exceeds max_step_t (metres) or max_step_r (radians)."""
    f = np.arange(n_frames, dtype=np.float64)[:, None]
    out = np.tile(np.eye(4), (n_frames, 1, 1))

    def series(cap):
        om = rng.uniform(0.02, 0.15, (3, 3))
        ph = rng.uniform(0, 2 * np.pi, (3, 3))
        amp = rng.uniform(0.3, 1.0, (3, 3))
        x = np.zeros((n_frames, 3))
        for k in range(3):
            x += amp[k] * np.sin(om[k] * f + ph[k])
        step = np.linalg.norm(np.diff(x, axis=0), axis=1).max() if n_frames > 1 else 1.0
        return (x - x[0]) * (0.9 * cap / max(step, 1e-12))

    t = series(max_step_t)
    w = series(max_step_r)
    for i in range(n_frames):
        out[i, :3, 3] = start[:3, 3] + t[i]
        th = np.linalg.norm(w[i])
        K = np.zeros((3, 3))
        if th > 0:
            k = w[i] / th
            K = np.array([[0, -k[2], k[1]], [k[2], 0, -k[0]], [-k[1], k[0], 0]])
        Rw = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * (K @ K)
        out[i, :3, :3] = Rw @ start[:3, :3]
    return out


def tracking_sequence(seed: int = 1004, n_frames: int = 200, n_obj: int = 3, vox_range=(2000, 5000),
                      H: int = 120, W: int = 160, f: float = 150.0, outlier_frac: float = 0.04):
    """Objects moving on smooth seeded SE(3) paths in front of the camera:
    meshes, true poses [F, M, 4, 4], camera, and per-frame noise draws."""
    rng = np.random.default_rng(seed)
    cam = Camera(f, f, W / 2.0, H / 2.0, H, W)
    meshes, paths = [], []
    centres = [(-0.09, 0.0, 0.85), (0.09, 0.02, 0.9), (0.0, -0.05, 0.75), (0.05, 0.08, 0.95)]
    for k in range(n_obj):
        nv = int(rng.integers(vox_range[0], vox_range[1] + 1))
        meshes.append(voxel_mesh(voxel_blob(nv, rng)))
        start = pose_matrix(shoemake_rotations(1, rng)[0], centres[k % len(centres)])
        paths.append(smooth_trajectory(rng, n_frames, start))
    noise = [observation_noise(H, W, rng, 0.002, outlier_frac) for _ in range(n_frames)]
    return meshes, np.stack(paths, 1), cam, noise


def look_at(eye: Sequence[float], target: Sequence[float] = (0.0, 0.0, 0.0),
            up: Sequence[float] = (0.0, 0.0, 1.0)) -> np.ndarray:
    """World-to-camera transform of a camera at `eye` looking at `target`
    with `up` pointing up in the image (+z forward, +x right, +y down)."""
    eye, target, up = (np.asarray(x, dtype=np.float64) for x in (eye, target, up))
    z = target - eye
    z /= np.linalg.norm(z)
    x = np.cross(z, up)
    x /= np.linalg.norm(x)
    y = np.cross(z, x)
    R = np.stack([x, y, z])
    return pose_matrix(R, -R @ eye)


def table_scene(seed: int = 1002, voxels=(800, 1500, 3000, 6000), W: int = 320, H: int = 240, f: float = 300.0,
                distance: float = 0.8, elevation_deg: float = 45.0):
    """Objects resting on a 1 m x 1 m table (world z = 0) seen by a camera
    that looks at the world origin with +z up, at a seeded azimuth.
    Returns meshes, object poses (camera frame), the table (verts, tris,
    pose), the camera, observation noise draws and the camera-from-world pose."""
    rng = np.random.default_rng(seed)
    cam = Camera(f, f, W / 2.0, H / 2.0, H, W)
    az = rng.uniform(0, 2 * np.pi)
    el = np.deg2rad(elevation_deg)
    eye = distance * np.array([np.cos(el) * np.cos(az), np.cos(el) * np.sin(az), np.sin(el)])
    Tcw = look_at(eye)
    meshes, poses = [], []
    slots = [(-0.15, -0.12), (0.14, -0.1), (-0.1, 0.15), (0.15, 0.14)]
    for k, n in enumerate(voxels):
        c = voxel_blob(n, rng)
        v, t = voxel_mesh(c)
        meshes.append((v, t))
        yaw = rng.uniform(0, 2 * np.pi)
        cy, sy = np.cos(yaw), np.sin(yaw)
        Rw = np.array([[cy, -sy, 0.0], [sy, cy, 0.0], [0.0, 0.0, 1.0]])
        lift = -v[:, 2].min()  # rest on the table
        x, y = slots[k % len(slots)]
        Tw = pose_matrix(Rw, (x + rng.uniform(-0.02, 0.02), y + rng.uniform(-0.02, 0.02), lift))
        poses.append(Tcw @ Tw)
    tv = np.array([[-0.5, -0.5, 0.0], [0.5, -0.5, 0.0], [0.5, 0.5, 0.0], [-0.5, 0.5, 0.0]])
    tt = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)  # normal +z, towards the camera
    table = (tv, tt, Tcw.copy())
    noise = observation_noise(H, W, rng, 0.002, 0.03)
    return meshes, poses, table, cam, noise, Tcw


def bottle_voxels(body=(10, 6, 17), cap=(3, 3, 3), cap_shift=(2, 0)) -> np.ndarray:
    """Centres of a solid bottle of 1 cm voxels: a body box of body[0] x
    body[1] x body[2] cells standing on z = 0 with its footprint centred on
    the origin, and a cap box on top shifted by cap_shift cells in x and y.
    The shape has no rotational symmetry about the vertical other than a
    half turn of the body alone, which the shifted cap breaks."""
    def box(n, lo):
        ax = [np.arange(lo[k], lo[k] + n[k]) for k in range(3)]
        return np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(-1, 3)

    b = box(body, (-(body[0] // 2), -(body[1] // 2), 0))
    c = box(cap, (cap_shift[0] - cap[0] // 2, cap_shift[1] - cap[1] // 2, body[2]))
    return (np.concatenate([b, c]).astype(np.float64) + 0.5) * VOXEL


def camera_pan_sequence(seed: int = 1005, n_frames: int = 120, res: int = 100, distance: float = 0.6, sweep_deg: float = 90.0, fov_deg: float = 45.0,
                        outlier_frac: float = 0.04):
    """A camera circling one object that rests on a table (the setting of the
    paper's real-time tracking experiment, Sec. IV and Table 1), at a square
    resolution of res x res.

    The object is a bottle of 1 cm voxels (``bottle_voxels``: a 10 x 6 x 17
    cm body and an off-centre cap, about the size of the paper's mustard
    bottle) at a seeded yaw.  The scene mesh is its voxels plus a 0.5 m x
    0.5 m table quad,
    expressed in a frame whose origin is the point the camera looks at (the
    object's centre), so that camera motion appears as a pose of the whole
    scene in the camera frame.  The camera's azimuth sweeps ``sweep_deg``
    degrees over the sequence, its elevation swings between 25 and 40
    degrees, and its distance varies by +-5 cm.  Returns (verts, tris),
    the true scene poses [n_frames, 4, 4] (camera-from-scene), the camera
    and per-frame noise draws.  The same seed gives the same object and
    path at every resolution; only the noise draws depend on ``res``.
    """
    rng = np.random.default_rng(seed)
    yaw = rng.uniform(0, 2 * np.pi)
    Rz = np.array([[np.cos(yaw), -np.sin(yaw), 0.0], [np.sin(yaw), np.cos(yaw), 0.0], [0.0, 0.0, 1.0]])
    ov, ot = voxel_mesh(bottle_voxels() @ Rz.T)
    centre = np.array([0.0, 0.0, 0.5 * ov[:, 2].max()])  # the bottle's mid-height above the table
    tv = np.array([[-0.25, -0.25, 0.0], [0.25, -0.25, 0.0], [0.25, 0.25, 0.0], [-0.25, 0.25, 0.0]])
    tt = np.array([[0, 1, 2], [0, 2, 3]], dtype=np.int32)
    verts = np.concatenate([ov, tv]) - centre
    tris = np.concatenate([ot, tt + ov.shape[0]]).astype(np.int32)
    az0 = rng.uniform(0, 2 * np.pi)
    ph_el, ph_d = rng.uniform(0, 2 * np.pi, 2)
    s = np.linspace(0.0, 1.0, n_frames)
    az = az0 + np.deg2rad(sweep_deg) * s
    el = np.deg2rad(32.5 + 7.5 * np.sin(2 * np.pi * s + ph_el))
    d = distance + 0.05 * np.sin(2 * np.pi * 1.5 * s + ph_d)
    poses = np.empty((n_frames, 4, 4))
    for i in range(n_frames):
        eye = d[i] * np.array([np.cos(el[i]) * np.cos(az[i]), np.cos(el[i]) * np.sin(az[i]), np.sin(el[i])])
        poses[i] = look_at(eye)
    f = 0.5 * res / np.tan(np.deg2rad(fov_deg) / 2.0)
    cam = Camera(f, f, res / 2.0, res / 2.0, res, res)
    nrng = np.random.default_rng([seed, res])
    noise = [observation_noise(res, res, nrng, 0.002, outlier_frac) for _ in range(n_frames)]
    return (verts, tris), poses, cam, noise


def camera_pan_schedule() -> List[GridSpec]:
    """Per-frame hypothesis stages for tracking ``camera_pan_sequence``, each
    around the best pose of the stage before (1,708 hypotheses a frame):
    rotations alone (5^3 rotation vectors within +-1.2 deg per axis), then
    translations alone (5^3 within +-6 mm), then two joint stages of 3^3
    translations x 3^3 rotations (+-1.5 mm x +-0.4 deg, then +-0.5 mm x
    +-0.15 deg).  Rotations act in the camera frame about the scene origin,
    which is where the camera looks, so the camera's orbit is a rotation the
    first stage can follow."""
    def spec(h, nt, a, nr):
        return GridSpec(np.eye(4), (h, h, h), (nt, nt, nt), rotations=rotation_grid(nr, np.deg2rad(a)))

    return [spec(0.0, 1, 1.2, 5), spec(0.006, 5, 0.0, 1), spec(0.0015, 3, 0.4, 3), spec(0.0005, 3, 0.15, 3)]

