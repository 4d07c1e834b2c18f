"""One frame of multi-object tracking by search and gradient refinement,
stated plainly for the oracle.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

Per frame every object o is updated in turn, the others held fixed at their
current estimates (objects before o already at this frame's values): the
scene is object o at a hypothesised pose in front of the other objects
(rendered jointly; object o's triangle ids first, then the others' in
order).  Each search stage enumerates its grid around o's current pose
(Sec. III-B's coarse-to-fine enumeration around the previous estimate,
random perturbations from the counter-based generator with key 0 and the
stage index as the stage word), scores every hypothesis by eq. (1) with the
window truncation, and moves o to the best one (lowest index among equal
scores): the most probable cell, a deterministic stand-in for a draw.  Then
n_refine Adam steps ascend logL in the pose tangent, the moments starting
from zero each frame (``oracle.refine.adam_pose_step``).

The device keeps poses in single precision, so each chosen pose is rounded
to it before the next stage enumerates around it (``round32``).

``search_ends`` lists every pose a stage-by-stage search can end on when
scores within ``tol`` times the L1 mass of the best hypothesis are taken as
ties: FP32 scores may order such near ties either way, so each is a correct
outcome of the method at that precision.

Occlusion handling (an addition to the method, off unless asked for): after
object o's update, the fraction of the pixels it covers drawn alone at the
new pose that are both in front of the other objects at their current
estimates and have an observed point within 3 sigma of theirs in the
likelihood's window is how much of it the observation confirms
(``seen_fraction``).  Below a threshold the update is
dropped: o takes its previous estimate moved by its last accepted
frame-to-frame motion (``predict``), and the next frame's first stage
searches translations over a wider box (``gate_update``, ``Gating``).  The
observed depth has to take part: a hidden object's best hypothesis is often
a wrong pose in an empty part of the image, where it is in view of the
camera but the observation has nothing there to confirm it.
"""

from __future__ import annotations

import copy
import dataclasses
from typing import Callable, List, Optional, Sequence, Tuple

import numpy as np

from . import enumerate_grid, render, render_grad, score, score_grad, unproject
from .refine import adam_pose_step


def round32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def scene_objects(meshes, poses, o, P):
    """Object o at poses P [N,4,4] in front of the others at `poses`."""
    v, t = meshes[o]
    return [(v, t, P)] + [(meshes[k][0], meshes[k][1], poses[k]) for k in range(len(meshes)) if k != o]


def scaled(spec, scale: float):
    """The grid with its translation half extents times `scale`, each product
    rounded to single precision as the device forms it."""
    if scale == 1.0:
        return spec
    h = tuple(float(np.float32(np.float32(x) * np.float32(scale))) for x in spec.half_extent)
    return dataclasses.replace(spec, half_extent=h)


def stage_scores(meshes, poses, o, spec, stage, obs, cam, sp):
    """Hypotheses of one stage around object o's current pose and their logL, L1."""
    P = enumerate_grid(spec, seed=0, stage=stage, center=round32(poses[o]))
    P = round32(P)
    d, _ = render(scene_objects(meshes, poses, o, P), cam)
    L, l1 = score(obs, unproject(d, cam), sp.sigma, sp.p_out, sp.outlier_volume, sp.window)
    return P, L, l1


def search_ends(meshes, poses, o, stages, obs, cam, sp, tol=0.0, limit=3, stage=0) -> List[np.ndarray]:
    """Poses object o's stage-by-stage argmax search can end on (the plain
    argmax path first); near ties within tol * L1 are followed, at most
    `limit` per stage."""
    P, L, l1 = stage_scores(meshes, poses, o, stages[stage], stage, obs, cam, sp)
    best = int(np.argmax(L))  # the first of equal maxima
    order = [best] + [int(j) for j in np.argsort(-L, kind="stable") if j != best and L[j] >= L[best] - tol * l1[best]]
    ends = []
    for j in order[:limit]:
        nxt = list(poses)
        nxt[o] = P[j]
        if stage + 1 == len(stages):
            ends.append(P[j])
        else:
            ends += search_ends(meshes, nxt, o, stages, obs, cam, sp, tol, limit, stage + 1)
    return ends


def refine(meshes, poses, o, obs, cam, sp, n_refine, lr_t, lr_r, beta1=0.9, beta2=0.999, eps=1e-8):
    """Object o's pose after n_refine Adam steps on logL (moments from zero)."""
    Q = round32(poses[o])[None]
    st = np.zeros((1, 12))
    v, t = meshes[o]
    for it in range(1, n_refine + 1):
        d, ids = render(scene_objects(meshes, poses, o, Q), cam)
        rend = unproject(d, cam)
        dr, _, _ = score_grad(obs, rend, sp.sigma, sp.p_out, sp.outlier_volume, sp.window)
        g = render_grad(v, t, Q, cam, ids, d, dr)
        Q, st = adam_pose_step(Q, g, st, it, lr_t, lr_r, beta1, beta2, eps)
        Q = round32(Q)
    return Q[0]


def track_frame(meshes, poses, obs, cam, sp, stages, n_refine=0, lr_t=1e-3, lr_r=1e-2, beta1=0.9, beta2=0.999,
                eps=1e-8, gating: Optional[Gating] = None) -> np.ndarray:
    """All objects' poses [M,4,4] after one frame (plain argmax search, no ties
    followed); with `gating`, each update passes the occlusion decision."""
    cur = [round32(P) for P in poses]
    for o in range(len(meshes)):
        prev = cur[o]
        st = list(stages)
        if gating is not None:
            st[0] = scaled(st[0], gating.scale[o])
        cur[o] = search_ends(meshes, cur, o, st, obs, cam, sp, tol=0.0, limit=1)[0]
        if n_refine > 0:
            cur[o] = refine(meshes, cur, o, obs, cam, sp, n_refine, lr_t, lr_r, beta1, beta2, eps)
        if gating is not None:
            seen = seen_fraction(meshes, cur, o, cam, obs, 3.0 * sp.sigma, sp.window)
            cur[o] = round32(gate_update(gating, o, prev, cur[o], seen))
    return np.stack(cur)


def seen_fraction(meshes, poses, o, cam, obs, tol: float, window: int = 1) -> float:
    """Of the pixels object o covers drawn alone at poses[o], the fraction
    that are not behind the other objects at their poses (equal depth counts
    as in front) and that the observation confirms: some valid observed point
    (obs [H,W,3], z = 0 invalid) among the window x window pixels centred on
    the pixel lies within distance tol of the object's point there, as the
    likelihood's window looks for one.  0 when o covers no pixel."""
    v, t = meshes[o]
    d_o = render([(v, t, round32(poses[o]))], cam)[0][0]
    drawn = d_o > 0
    n = int(drawn.sum())
    if n == 0:
        return 0.0
    front = drawn
    others = [(meshes[k][0], meshes[k][1], round32(poses[k])) for k in range(len(meshes)) if k != o]
    if others:
        d_b = render(others, cam)[0][0]
        front = drawn & ((d_b <= 0) | (d_o <= d_b))
    q = unproject(d_o, cam)
    ob = np.asarray(obs, dtype=np.float64)
    H, W = d_o.shape
    h = window // 2
    pad = np.zeros((H + 2 * h, W + 2 * h, 3))
    pad[h:h + H, h:h + W] = ob
    seen = np.zeros((H, W), dtype=bool)
    for dy in range(-h, h + 1):
        for dx in range(-h, h + 1):
            oi = pad[h + dy:h + dy + H, h + dx:h + dx + W]
            seen |= (oi[..., 2] > 0) & (np.linalg.norm(oi - q, axis=-1) <= tol)
    return int((front & seen).sum()) / n


@dataclasses.dataclass
class Gating:
    """Per-object occlusion state: the last accepted motion (rotation dR
    applied on the left, translation dt added), dropped updates in a row and
    the first stage's translation scale for the next frame."""

    min_visible: float
    widen: float
    dR: List[np.ndarray]
    dt: List[np.ndarray]
    dropped: List[int]
    scale: List[float]

    @classmethod
    def start(cls, M: int, min_visible: float, widen: float) -> "Gating":
        return cls(min_visible, widen, [np.eye(3) for _ in range(M)], [np.zeros(3) for _ in range(M)], [0] * M,
                   [1.0] * M)


def predict(g: Gating, o: int, prev: np.ndarray) -> np.ndarray:
    """prev moved by object o's kept motion: rotation dR on the left, dt added."""
    P = np.array(prev, dtype=np.float64)
    P[:3, :3] = g.dR[o] @ prev[:3, :3]
    P[:3, 3] = prev[:3, 3] + g.dt[o]
    return P


def gate_update(g: Gating, o: int, prev: np.ndarray, new: np.ndarray, seen: float) -> np.ndarray:
    """Object o's pose after the occlusion decision, given the seen fraction of
    the update; updates g in place.  At least min_visible: the update stands
    and its motion (R_new R_prev^T, t_new - t_prev) is kept; otherwise the
    prediction replaces it and the next first stage widens."""
    if seen >= g.min_visible:
        g.dR[o] = new[:3, :3] @ prev[:3, :3].T
        g.dt[o] = new[:3, 3] - prev[:3, 3]
        g.dropped[o] = 0
        g.scale[o] = 1.0
        return new
    P = predict(g, o, prev)
    g.dropped[o] += 1
    g.scale[o] = g.widen
    return P
