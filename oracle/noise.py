"""Hierarchical likelihood over the noise parameters, stated plainly for the oracle.

TEST INFRASTRUCTURE ONLY (see the oracle package docstring).

Alg. 1 puts the priors p_out ~ U(0, 1) and sigma ~ U(0, sigma_max) on the
noise parameters of eq. (1); Sec. IV compares hypotheses under the marginal
over them.  The printed sigma/sigma_max prefactor of eq. (1) is read as the
prior density 1/sigma_max of the uniform prior on sigma.  The marginal is
approximated by a quadrature over a grid of (sigma_a, p_b):

    log p(y | scene) ~= log sum_{a,b} w_ab exp(logL(sigma_a, p_b)),

where logL is the windowed eq. (1) (``oracle.score``) and w_ab are the
quadrature weights including the prior density.  For the midpoint rule on
A equal cells of (0, sigma_max] and B of (0, 1] every w_ab = 1/(A B):
(sigma_max/A) (1/B) cell volume times the prior density 1/sigma_max.
"""

from __future__ import annotations

import numpy as np

import oracle


def midpoints(sigma_max: float, A: int, B: int):
    """Cell centres of A equal cells of (0, sigma_max] and B equal cells of (0, 1]."""
    return sigma_max * (np.arange(A) + 0.5) / A, (np.arange(B) + 0.5) / B


def score_grid(obs, rend, sigmas, p_outs, V=1.0, window=3, M=0.0, log_w=None):
    """logL [N, A, B] under each grid point and the log marginal [N] over the grid.

    log_w [A, B]: log quadrature weights (None: equal weights 1/(A B))."""
    A, B = len(sigmas), len(p_outs)
    rend = np.asarray(rend, dtype=np.float64)
    N = 1 if rend.ndim == 3 else rend.shape[0]
    L = np.empty((N, A, B))
    for a, s in enumerate(sigmas):
        for b, p in enumerate(p_outs):
            L[:, a, b], _ = oracle.score(obs, rend, float(s), float(p), V, window, M)
    lw = np.full((A, B), -np.log(A * B)) if log_w is None else np.asarray(log_w, dtype=np.float64)
    t = (L + lw[None]).reshape(N, -1)
    m = t.max(axis=1)
    marg = m + np.log(np.exp(t - m[:, None]).sum(axis=1))
    return L, marg
