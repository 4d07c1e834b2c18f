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
"""

from __future__ import annotations

import copy
from typing import Callable, List, Sequence, Tuple

import numpy as np

from . import enumerate_grid, render, render_grad, score, score_grad, unproject
from .refine import adam_pose_step


def round32(a):
    return np.asarray(a, dtype=np.float32).astype(np.float64)


def scene_objects(meshes, poses, o, P):
    """Object o at poses P [N,4,4] in front of the others at `poses`."""
    v, t = meshes[o]
    return [(v, t, P)] + [(meshes[k][0], meshes[k][1], poses[k]) for k in range(len(meshes)) if k != o]


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
                eps=1e-8) -> np.ndarray:
    """All objects' poses [M,4,4] after one frame (plain argmax search, no ties followed)."""
    cur = [round32(P) for P in poses]
    for o in range(len(meshes)):
        cur[o] = search_ends(meshes, cur, o, stages, obs, cam, sp, tol=0.0, limit=1)[0]
        if n_refine > 0:
            cur[o] = refine(meshes, cur, o, obs, cam, sp, n_refine, lr_t, lr_r, beta1, beta2, eps)
    return np.stack(cur)
