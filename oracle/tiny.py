"""Brute-force numpy versions used to pin the oracle on tiny inputs.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

* ``render_bruteforce``: for every pixel and every triangle, intersect the
  pixel ray with the triangle (Moller & Trumbore, 1997) with inclusive
  barycentric bounds, and keep the nearest hit (equal depths: smaller id).
  This is an independent route to the plain edge-function scan in the C
  oracle; the same conventions (near-plane drop, back-face test) apply.
* ``loglik_untruncated``: eq. (1) with the inner sum over every rendered
  point (no window), the Gaussian density taken from scipy.
"""

from __future__ import annotations

import numpy as np
from scipy.stats import multivariate_normal


def _rays(cam):
    c = np.arange(cam.W) + 0.5
    r = np.arange(cam.H) + 0.5
    C, R = np.meshgrid(c, r)
    return np.stack([(C - cam.cx) / cam.fx, (R - cam.cy) / cam.fy, np.ones_like(C)], -1)  # [H,W,3]


def render_bruteforce(verts, tris, pose, cam, id_offset=0):
    """Depth [H,W] and ids [H,W] of one mesh at one pose, by ray casting."""
    c = verts @ pose[:3, :3].T + pose[:3, 3]
    d = _rays(cam).reshape(-1, 3)
    depth = np.full(d.shape[0], np.inf)
    ids = np.full(d.shape[0], -1, dtype=np.int64)
    for i, (a, b, e) in enumerate(tris):
        c0, c1, c2 = c[a], c[b], c[e]
        if min(c0[2], c1[2], c2[2]) <= cam.z_near:
            continue
        e1, e2 = c1 - c0, c2 - c0
        if np.dot(np.cross(e1, e2), c0) >= 0.0:
            continue
        pvec = np.cross(d, e2)  # [P,3]
        det = pvec @ e1
        ok = np.abs(det) > 0
        inv = np.where(ok, 1.0 / np.where(ok, det, 1.0), 0.0)
        s = -c0  # ray origin is the camera centre
        u = (pvec @ s) * inv
        qvec = np.cross(s, e1)
        v = (d @ qvec) * inv
        t = (qvec @ e2) * inv
        hit = ok & (u >= 0) & (v >= 0) & (u + v <= 1) & (t > 0)
        idv = id_offset + i
        better = hit & ((t < depth) | ((t == depth) & (idv < ids)))
        depth[better] = t[better]
        ids[better] = idv
    depth[np.isinf(depth)] = 0.0
    return depth.reshape(cam.H, cam.W), ids.reshape(cam.H, cam.W).astype(np.int32)


def loglik_untruncated(obs, rend, sigma, p_out, V=1.0, M=None):
    """Eq. (1) without truncation: sum_i ln(p/V + (1-p)/M sum_j N3(q~_i; q_j, sigma))."""
    obs = obs.reshape(-1, 3)
    rend = rend.reshape(-1, 3)
    if M is None:
        M = obs.shape[0]
    qo = obs[obs[:, 2] > 0]
    qr = rend[rend[:, 2] > 0]
    cov = sigma * sigma * np.eye(3)
    total = 0.0
    for q in qo:
        S = multivariate_normal(mean=q, cov=cov).pdf(qr).sum() if len(qr) else 0.0
        total += np.log(p_out / V + (1.0 - p_out) / M * S)
    return total
