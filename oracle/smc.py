"""Sequential Monte Carlo over the objects of a table scene, stated plainly for the oracle.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

Scene prior (Alg. 1, scene prior; Sec. III-A (i)).  Object i has a type o_i
uniform over the library O, a contact face c_i uniform over the six faces of
its bounding box, and a planar placement dphi_i = (dx, dy, dtheta) uniform
over the table top less the face's footprint and over a full turn, so

    p(o, c, dphi) = 1/|O| * 1/6 * 1/(W_t - w_oc) * 1/(H_t - h_oc) * 1/(2 pi).

Noise priors (Alg. 1): p_out ~ U(0, 1), sigma ~ U(0, sigma_max).

Readings (the paper gives no more detail than the above):

* The bounding box is the axis-aligned box of the object's vertices in its
  own frame; faces are numbered -x, +x, -y, +y, -z, +z.  Resting on face c
  means the face's outward normal points down the table normal, the face lies
  in the table top (z = 0 of the table frame, +z up) and the footprint's
  centre is at the table frame's origin; dtheta then turns the object about
  the table normal through that centre and (dx, dy) moves it.  dtheta is in
  [0, 2 pi); (dx, dy) ranges over a box of size (W_t - w_oc) x (H_t - h_oc)
  centred on the table's origin.
* Stage i of the SMC sampler (Sec. III-B) proposes the new object by
  coarse-to-fine search over a partition of {types} x {faces} x box(dphi):
  stage 0 splits every (type, face) box into counts[0] equal cells, stage t
  splits the chosen cell into counts[t]; each cell is scored by the target at
  its centre times the cell's volume (its midpoint estimate of the target's
  mass), and since prior density times cell volume is the same for every cell
  of a stage the draw uses softmax(logL).  Stage t scores at a stated
  noise (sigma_t, p_t) when one is given (coarse cells want a wide inlier
  kernel), else at the particle's current estimates (sigma0, p0 for the first
  object); any such choice keeps q exact.  A uniform point of the final cell
  is the proposed dphi.
* The noise is proposed next: A x B equal cells of (0, sigma_max] x (0, 1),
  each scored at its midpoint with the new object at the proposed placement,
  one drawn by softmax, and a uniform point of it taken.
* The proposal density q_i is the product of the draws' probabilities over
  the volume of the final pose cell and over the area of the noise cell.
* log p_i is the windowed eq. (1) log-likelihood of the scene (fixed content
  plus the particle's i objects) at the particle's noise, plus the log prior
  of every object, plus log(1/sigma_max); weights follow eq. (2) for i = 1 and
  eq. (3) after.  Eq. (3) as printed drops the previous stage's noise values
  without a backward-kernel density for them; it is read with the noise prior
  as that kernel (a factor 1/sigma_max from stage 2 on, the same for every
  particle, so normalised weights are as printed), which keeps each stage's
  weights unbiased for that stage's evidence.  With an effective sample size below ess_threshold * M the
  particles are resampled multinomially (Gumbel-max over the log weights) and
  every weight becomes the mean weight.
* Random numbers: categorical draws use the sampler of ``oracle.sample`` with
  stage word (i << 8) | t for the pose stages, (i << 8) | 0x40 for the noise
  and (i << 8) | 0x80 for resampling (draw k0 = particle index); the uniform
  points use Philox4x32-10 counters (m, i, 0, 2) for the placement (words 0, 1,
  2 for dx, dy, dtheta) and (m, i, 1, 2) for the noise (words 0, 1).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Sequence

import numpy as np

from . import sample, uniform

TWO_PI = 2.0 * np.pi

# Rotation taking the outward normal of face c to -z (the table's down).
# Face order: -x, +x, -y, +y, -z, +z.
FACE_ROT = np.array([
    [[0, 0, -1], [0, 1, 0], [1, 0, 0]],
    [[0, 0, 1], [0, 1, 0], [-1, 0, 0]],
    [[1, 0, 0], [0, 0, -1], [0, 1, 0]],
    [[1, 0, 0], [0, 0, 1], [0, -1, 0]],
    [[1, 0, 0], [0, 1, 0], [0, 0, 1]],
    [[1, 0, 0], [0, -1, 0], [0, 0, -1]],
], dtype=np.float64)
FACE_NORMAL = np.array([[-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]], dtype=np.float64)


@dataclass
class Face:
    R: np.ndarray  # 3x3: object frame -> resting frame
    d: np.ndarray  # offset putting the face on z = 0, footprint centred
    w: float       # footprint extent along x
    h: float       # footprint extent along y


def faces_of(verts) -> List[Face]:
    """The six resting frames of an object's bounding box."""
    v = np.asarray(verts, dtype=np.float64)
    lo, hi = v.min(axis=0), v.max(axis=0)
    corners = np.array([[(lo, hi)[i][0], (lo, hi)[j][1], (lo, hi)[k][2]]
                        for i in (0, 1) for j in (0, 1) for k in (0, 1)])
    out = []
    for c in range(6):
        R = FACE_ROT[c]
        q = corners @ R.T
        mn, mx = q.min(axis=0), q.max(axis=0)
        d = -np.array([0.5 * (mn[0] + mx[0]), 0.5 * (mn[1] + mx[1]), mn[2]])
        out.append(Face(R, d, mx[0] - mn[0], mx[1] - mn[1]))
    return out


@dataclass
class Table:
    T: np.ndarray   # table frame -> camera, 4x4
    width: float    # extent along the table frame's x
    height: float   # extent along y


def contact_pose(table: Table, f: Face, dx: float, dy: float, dth: float) -> np.ndarray:
    """Camera-frame pose of an object resting on face f at placement (dx, dy, dth)."""
    c, s = np.cos(dth), np.sin(dth)
    Rz = np.array([[c, -s, 0.0], [s, c, 0.0], [0.0, 0.0, 1.0]])
    P = np.eye(4)
    P[:3, :3] = Rz @ f.R
    P[:3, 3] = Rz @ f.d + np.array([dx, dy, 0.0])
    return np.asarray(table.T, dtype=np.float64) @ P


def root_box(table: Table, f: Face):
    """(lo, hi) of the placement box of a face: centred offsets and a full turn."""
    ax, ay = 0.5 * (table.width - f.w), 0.5 * (table.height - f.h)
    return np.array([-ax, -ay, 0.0]), np.array([ax, ay, TWO_PI])


def log_prior(n_types: int, table: Table, f: Face) -> float:
    """log p(o, c, dphi) for a placement inside the face's box."""
    return -(np.log(n_types) + np.log(6.0) + np.log(table.width - f.w) + np.log(table.height - f.h)
             + np.log(TWO_PI))


def sub_cell(lo, hi, counts, j):
    """Cell j = (ix * ny + iy) * nth + ith of the split of [lo, hi) into counts cells."""
    nx, ny, nt = counts
    i = np.array([j // (ny * nt), (j // nt) % ny, j % nt], dtype=np.float64)
    step = (hi - lo) / np.asarray(counts, dtype=np.float64)
    return lo + i * step, lo + (i + 1.0) * step


@dataclass
class SMCParams:
    counts: Sequence[Sequence[int]]   # cells per axis (dx, dy, dtheta) of each pose stage
    sigma_max: float
    A: int                            # noise cells along sigma
    B: int                            # noise cells along p_out
    sigma0: float
    p0: float
    ess_threshold: float
    seed: int
    stage_noise: Sequence = None      # per pose stage (sigma, p_out) or None: the particle's noise


@dataclass
class Particles:
    place: np.ndarray   # [M, k, 2] type, face
    dphi: np.ndarray    # [M, k, 3]
    poses: np.ndarray   # [M, k, 4, 4]
    noise: np.ndarray   # [M, 2] sigma, p_out
    logW: np.ndarray    # [M]
    logp: np.ndarray    # [M] log target of the current stage
    lprior: np.ndarray  # [M] sum of the objects' log priors
    logL: np.ndarray = field(default=None)  # [M]


def init_particles(M: int, params: SMCParams) -> Particles:
    return Particles(np.zeros((M, 0, 2), np.int32), np.zeros((M, 0, 3)), np.zeros((M, 0, 4, 4)),
                     np.tile([params.sigma0, params.p0], (M, 1)).astype(np.float64), np.zeros(M), np.zeros(M),
                     np.zeros(M), np.zeros(M))


# loglik(m, o, poses [N,4,4], particle objects [(type, pose)], sigma, p_out) -> logL [N]
# (m is the particle; particles with equal objects and noise share one
# evaluation of the stage-0 cells, made with the first of them)
LogLik = Callable[[int, int, np.ndarray, list, float, float], np.ndarray]


def smc_stage(state: Particles, i: int, loglik: LogLik, faces: Sequence[Sequence[Face]], table: Table,
              params: SMCParams):
    """Stage i (1-based) for every particle: propose object i and the noise,
    reweight by eq. (2)/(3), optionally resample.  Returns (new state, diag)."""
    M = state.logW.shape[0]
    n_types = len(faces)
    seed = params.seed
    T = len(params.counts)
    k = state.place.shape[1]
    assert k == i - 1
    n0 = int(np.prod(params.counts[0]))
    choice = np.zeros((T, M), np.int32)
    new_place = np.zeros((M, 2), np.int32)
    new_dphi = np.zeros((M, 3))
    new_pose = np.zeros((M, 4, 4))
    new_noise = np.zeros((M, 2))
    logq = np.zeros(M)
    logL_new = np.zeros(M)
    noise_grid = np.zeros((M, params.A * params.B))
    noise_choice = np.zeros(M, np.int32)
    type_post = np.zeros((M, n_types))
    stage0, stage0_of = {}, []
    for m in range(M):
        objs = [(int(state.place[m, j, 0]), state.poses[m, j]) for j in range(k)]

        def noise_at(t):
            sn = params.stage_noise
            return tuple(sn[t]) if sn is not None and sn[t][0] > 0 else tuple(state.noise[m])
        # pose stage 0: every (type, face) box split into counts[0] cells
        cents, cells = [], []
        for o in range(n_types):
            for c in range(6):
                lo, hi = root_box(table, faces[o][c])
                for j in range(n0):
                    a, b = sub_cell(lo, hi, params.counts[0], j)
                    cells.append((o, c, a, b))
                    cents.append(0.5 * (a + b))
        sig, po = noise_at(0)
        # particles with equal objects and noise score the stage-0 cells alike: once
        key = (float(sig), float(po), tuple((t, Q.tobytes()) for t, Q in objs))
        if key not in stage0:
            stage0[key] = np.concatenate([
                loglik(m, o, np.stack([contact_pose(table, faces[o][cells[n][1]], *cents[n])
                                       for n in range(len(cells)) if cells[n][0] == o]), objs, sig, po)
                for o in range(n_types)])
        L = stage0[key]
        stage0_of.append(L)
        w = np.exp(L - L.max())
        type_post[m] = w.reshape(n_types, -1).sum(axis=1) / w.sum()  # marginal over face and placement
        _, idx, lw = sample(L, 1, seed, stage=(i << 8) | 0, k0=m)
        choice[0, m] = idx[0]
        o, c, lo, hi = cells[idx[0]]
        lq = lw[0]
        # later stages: split the chosen cell
        for t in range(1, T):
            n_t = int(np.prod(params.counts[t]))
            subs = [sub_cell(lo, hi, params.counts[t], j) for j in range(n_t)]
            P = np.stack([contact_pose(table, faces[o][c], *(0.5 * (a + b))) for a, b in subs])
            L = loglik(m, o, P, objs, *noise_at(t))
            _, idx, lw = sample(L, 1, seed, stage=(i << 8) | t, k0=m)
            choice[t, m] = idx[0]
            lo, hi = subs[idx[0]]
            lq += lw[0]
        # a uniform point of the final cell
        u = np.array([uniform(seed, m, i, 0, 2, w) for w in range(3)])
        x = lo + u * (hi - lo)
        lq -= np.log(np.prod(hi - lo))
        pose = contact_pose(table, faces[o][c], *x)
        # noise: midpoint-scored cells of the priors' support, a uniform point of the drawn one
        A, B = params.A, params.B
        g = np.array([loglik(m, o, pose[None], objs, params.sigma_max * (a + 0.5) / A, (b + 0.5) / B)[0]
                      for a in range(A) for b in range(B)])
        noise_grid[m] = g
        _, idx, lw = sample(g, 1, seed, stage=(i << 8) | 0x40, k0=m)
        noise_choice[m] = idx[0]
        a, b = divmod(int(idx[0]), B)
        un = [uniform(seed, m, i, 1, 2, w) for w in range(2)]
        sig_new, p_new = params.sigma_max * (a + un[0]) / A, (b + un[1]) / B
        lq += lw[0] - np.log(params.sigma_max / (A * B))
        new_place[m] = (o, c)
        new_dphi[m] = x
        new_pose[m] = pose
        new_noise[m] = (sig_new, p_new)
        logq[m] = lq
        logL_new[m] = loglik(m, o, pose[None], objs, sig_new, p_new)[0]
    lprior = state.lprior + np.array([log_prior(n_types, table, faces[o][c]) for o, c in new_place])
    logp = logL_new + lprior - np.log(params.sigma_max)
    back = 0.0 if i == 1 else -np.log(params.sigma_max)      # noise prior density of the dropped (sigma, p_out)
    logW_pre = state.logW + logp - state.logp - logq + back   # eq. (2) with logW = logp = 0 before stage 1; eq. (3)
    mx = logW_pre.max()
    e = np.exp(logW_pre - mx)
    ess = e.sum() ** 2 / (e * e).sum()
    _, anc, _ = sample(logW_pre - mx, M, seed, stage=(i << 8) | 0x80, k0=0)
    resampled = bool(ess < params.ess_threshold * M)
    src = anc if resampled else np.arange(M)
    logW = (np.full(M, mx + np.log(e.sum()) - np.log(M)) if resampled else logW_pre.copy())
    new = Particles(
        place=np.concatenate([state.place, new_place[:, None]], axis=1)[src],
        dphi=np.concatenate([state.dphi, new_dphi[:, None]], axis=1)[src],
        poses=np.concatenate([state.poses, new_pose[:, None]], axis=1)[src],
        noise=new_noise[src], logW=logW, logp=logp[src], lprior=lprior[src], logL=logL_new[src])
    diag = dict(choice=choice, logq=logq, logL=logL_new, logp=logp, logW_pre=logW_pre, ess=ess, ancestors=src,
                resampled=resampled, noise_grid=noise_grid, noise_choice=noise_choice, place=new_place,
                dphi=new_dphi, poses=new_pose, noise=new_noise, type_post=type_post, stage0_logL=stage0_of)
    return new, diag


def scene_loglik(obs, cam, types, fixed, V, window, M_norm=0.0) -> LogLik:
    """The likelihood of the method: render the candidate object over the
    fixed content and the particle's objects, score by the windowed eq. (1)."""
    from . import render, score, unproject

    def f(m, o, P, objs, sigma, p_out):
        bg = list(fixed) + [(types[t][0], types[t][1], Q) for t, Q in objs]
        d, _ = render([(types[o][0], types[o][1], P)] + bg, cam)
        L, _ = score(obs, unproject(d, cam), float(sigma), float(p_out), V, window, M_norm)
        return L

    return f
