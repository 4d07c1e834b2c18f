"""Pins of the hierarchical likelihood (oracle/noise.py) against closed forms."""

import numpy as np
import pytest

from oracle.noise import midpoints, score_grid

pytestmark = pytest.mark.filterwarnings("ignore")


def one_pixel(dz):
    """A 1x1 observed point and a rendered point dz further along the ray."""
    obs = np.array([[[0.0, 0.0, 0.8]]])
    rend = np.array([[[[0.0, 0.0, 0.8 + dz]]]])
    return obs, rend


def test_p_out_marginal_of_one_pixel_is_exact_under_the_midpoint_rule():
    # for one pixel the likelihood is linear in p_out, so the midpoint rule on
    # (0, 1) integrates it exactly: int_0^1 (p/V + (1-p) N) dp = 1/(2V) + N/2
    sigma, V, dz = 0.004, 2.0, 0.003
    obs, rend = one_pixel(dz)
    N3 = (2 * np.pi * sigma**2) ** -1.5 * np.exp(-dz**2 / (2 * sigma**2))
    for B in (1, 2, 5, 9):
        _, po = midpoints(1.0, 1, B)
        _, marg = score_grid(obs, rend, [sigma], po, V=V, window=1)
        assert np.isclose(marg[0], np.log(1 / (2 * V) + N3 / 2), rtol=1e-12, atol=1e-12)


def test_sigma_marginal_of_one_pixel_converges_to_the_closed_form():
    # with p_out -> 0: (1/s_max) int_0^s_max N3(dz; sigma) dsigma
    #   = (2 pi)^(-3/2) exp(-dz^2 / (2 s_max^2)) / (dz^2 s_max)
    smax, dz = 0.01, 0.004
    obs, rend = one_pixel(dz)
    want = (2 * np.pi) ** -1.5 * np.exp(-dz**2 / (2 * smax**2)) / (dz**2 * smax)
    errs = []
    for A in (250, 1000):
        sig, _ = midpoints(smax, A, 1)
        _, marg = score_grid(obs, rend, sig, [1e-12], V=1.0, window=1)
        errs.append(abs(np.exp(marg[0]) / want - 1))
    assert errs[1] < 2e-5 and errs[1] < errs[0]  # second-order convergence of the midpoint rule


def test_one_point_grid_is_the_plain_score_plus_its_weight():
    import oracle

    rng = np.random.default_rng(5)
    obs = rng.normal(size=(6, 5, 3)) * 0.01 + [0, 0, 0.8]
    rend = rng.normal(size=(3, 6, 5, 3)) * 0.01 + [0, 0, 0.8]
    L, marg = score_grid(obs, rend, [0.005], [0.1], V=1.0, window=3, log_w=np.array([[-0.7]]))
    plain, _ = oracle.score(obs, rend, 0.005, 0.1, 1.0, 3)
    assert np.array_equal(L[:, 0, 0], plain)
    assert np.allclose(marg, plain - 0.7, rtol=1e-15, atol=1e-12)
