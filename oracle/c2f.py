"""Coarse-to-fine proposal (Sec. III-B, coarse-to-fine schedule, scoring
strategy and the region update), stated plainly for the oracle.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

The region A starts as the first stage's grid around the given centre pose.
At stage t every particle k enumerates stage t's grid around its current
centre, scores each cell at its representative pose (one point per cell,
weight 1, so the cell probabilities are softmax(logL)), draws one cell with
probability proportional to its score, and moves its centre there.  Stage 0
is the same for all particles, so it is scored once and drawn K times.  The
log proposal probability of the discrete choices accumulates in ``logq``;
for a partition schedule (cell-centre grids, each stage splitting the
previous stage's cell) the density of a uniform draw in the final cell is
exp(logq) / volume(final cell).
"""

from __future__ import annotations

import copy
from typing import Callable, List, Sequence

import numpy as np

from . import enumerate_grid, sample


def c2f(score_fn: Callable[[np.ndarray], np.ndarray], center: np.ndarray, stages: Sequence, K: int, seed: int):
    """Run the schedule; ``score_fn(poses [N,4,4]) -> logL [N]``.

    ``stages`` are ``workloads.GridSpec`` objects (their ``center`` is
    ignored).  Returns (poses [K,4,4], logq [K], idx [n_stages, K],
    logL_per_stage list).
    """
    n_st = len(stages)
    idx = np.zeros((n_st, K), dtype=np.int32)
    logL_hist: List[np.ndarray] = []
    P0 = enumerate_grid(stages[0], seed=seed, stage=0, center=center)
    L0 = score_fn(P0)
    logL_hist.append(L0)
    _, i0, lw0 = sample(L0, K, seed, stage=0, k0=0)
    idx[0] = i0
    centres = P0[i0].copy()
    logq = lw0.copy()
    for t in range(1, n_st):
        Ls = []
        for k in range(K):
            P = enumerate_grid(stages[t], seed=seed, stage=t, center=centres[k])
            L = score_fn(P)
            Ls.append(L)
            _, i, lw = sample(L, 1, seed, stage=t, k0=k)
            idx[t, k] = i[0]
            centres[k] = P[i[0]]
            logq[k] += lw[0]
        logL_hist.append(np.stack(Ls))
    return centres, logq, idx, logL_hist


def partition_schedule(base, counts: Sequence[Sequence[int]]):
    """Translation-only partition schedule: stage t splits the previous cell
    into counts[t] cells per axis (cell-centre grids)."""
    out = []
    half = np.asarray(base.half_extent, dtype=np.float64)
    for c in counts:
        g = copy.deepcopy(base)
        g.half_extent = tuple(half.tolist())
        g.count = tuple(int(x) for x in c)
        g.cell_centres = True
        g.rotations = None
        g.n_rot = 1
        out.append(g)
        half = half / np.asarray(c, dtype=np.float64)
    return out


def final_cell_volume(stages) -> float:
    g = stages[-1]
    v = 1.0
    for h, n in zip(g.half_extent, g.count):
        if h > 0:
            v *= 2.0 * h / n
    return v
