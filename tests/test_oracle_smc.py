"""Pins of the SMC oracle (oracle/smc.py): contact geometry, the prior's
normalisation, and the importance-weight identities of eq. (2)-(3)."""

import numpy as np
import pytest

from oracle.smc import (FACE_NORMAL, SMCParams, Table, contact_pose, faces_of, init_particles, log_prior, root_box,
                        smc_stage)

pytestmark = pytest.mark.filterwarnings("ignore")


def random_table(rng):
    a = rng.normal(size=3)
    a /= np.linalg.norm(a)
    th = rng.uniform(0, np.pi)
    K = np.array([[0, -a[2], a[1]], [a[2], 0, -a[0]], [-a[1], a[0], 0]])
    T = np.eye(4)
    T[:3, :3] = np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * K @ K
    T[:3, 3] = rng.normal(size=3)
    return Table(T, 0.9, 0.7)


def box_verts(rng):
    lo = rng.uniform(-0.05, 0.0, size=3) - 0.02
    hi = rng.uniform(0.01, 0.06, size=3)
    return np.array([[(lo, hi)[i][0], (lo, hi)[j][1], (lo, hi)[k][2]] for i in (0, 1) for j in (0, 1) for k in (0, 1)]
                    + list(rng.uniform(lo, hi, size=(20, 3))))


def test_resting_face_lies_on_the_table_centred_and_turned_about_its_normal():
    rng = np.random.default_rng(3)
    table = random_table(rng)
    Tinv = np.linalg.inv(table.T)
    v = box_verts(rng)
    lo, hi = v.min(0), v.max(0)
    for c, f in enumerate(faces_of(v)):
        assert np.isclose(np.linalg.det(f.R), 1.0)
        dx, dy, th = rng.uniform(-0.1, 0.1), rng.uniform(-0.1, 0.1), rng.uniform(0, 2 * np.pi)
        P = Tinv @ contact_pose(table, f, dx, dy, th)  # object -> table frame
        q = v @ P[:3, :3].T + P[:3, 3]
        assert np.isclose(q[:, 2].min(), 0.0, atol=1e-12)  # resting on the top, nothing below it
        # the face's outward normal points down the table normal
        assert np.allclose(P[:3, :3] @ FACE_NORMAL[c], [0, 0, -1], atol=1e-12)
        # the centre of the face is at (dx, dy) on the table top
        axis = c // 2
        fc = 0.5 * (lo + hi)
        fc[axis] = (lo, hi)[c % 2][axis]
        assert np.allclose(P[:3, :3] @ fc + P[:3, 3], [dx, dy, 0.0], atol=1e-12)
        # the footprint is the box's extent along the two other axes
        others = [k for k in range(3) if k != axis]
        assert np.isclose(f.w * f.h, np.prod((hi - lo)[others]))


def test_placement_prior_integrates_to_one():
    rng = np.random.default_rng(4)
    table = random_table(rng)
    types = [faces_of(box_verts(rng)) for _ in range(3)]
    total = 0.0
    for fs in types:
        for f in fs:
            lo, hi = root_box(table, f)
            total += np.exp(log_prior(len(types), table, f)) * np.prod(hi - lo)
    assert np.isclose(total, 1.0, rtol=1e-13)


def _params(seed, thr=0.0, counts=((2, 2, 4), (2, 2, 2), (1, 2, 2))):
    return SMCParams(counts=counts, sigma_max=0.01, A=3, B=2, sigma0=0.008, p0=0.5, ess_threshold=thr, seed=seed)


@pytest.mark.parametrize("thr", [0.0, 2.0])
def test_constant_likelihood_makes_every_weight_the_likelihood(thr):
    # with a flat likelihood every cell of a stage is equally likely, so the
    # proposal density is the prior's (both are 1/(6|O| volume of the box));
    # eq. (2) then gives W_1 = L_1 and eq. (3) W_i = W_{i-1} L_i / L_{i-1}
    rng = np.random.default_rng(5)
    table = random_table(rng)
    types = [faces_of(box_verts(rng)) for _ in range(2)]
    const = {1: -3.25, 2: 7.5}
    params = _params(11, thr)
    st = init_particles(6, params)
    for i in (1, 2):
        st, diag = smc_stage(st, i, lambda m, o, P, objs, s, p: np.full(len(P), const[i]), types, table, params)
        assert np.allclose(st.logW, const[i], rtol=0, atol=1e-11)
        assert diag["resampled"] == (thr > 1)


def test_every_cell_is_scored_at_its_own_face():
    # a likelihood of the pose alone that strongly prefers the object's +z
    # axis pointing up the table normal (face 4, -z, resting): every particle
    # must choose that face, which it can only if each stage-0 cell's pose
    # rests on that cell's face
    rng = np.random.default_rng(9)
    table = random_table(rng)
    Tinv = np.linalg.inv(table.T)
    types = [faces_of(box_verts(rng)) for _ in range(2)]
    params = _params(41)

    def lik(m, o, P, objs, s, p):
        up = np.einsum("ij,njk->nik", Tinv, P)[:, 2, 2]  # table-frame z of the object's z axis
        return 60.0 * up

    st, diag = smc_stage(init_particles(12, params), 1, lik, types, table, params)
    assert np.all(diag["place"][:, 1] == 4)


def test_type_posterior_of_a_type_only_likelihood_is_its_softmax():
    # every type has the same number of stage-0 cells, so a likelihood that
    # depends on the type alone gives posterior softmax over the types
    rng = np.random.default_rng(10)
    table = random_table(rng)
    types = [faces_of(box_verts(rng)) for _ in range(3)]
    a = np.array([0.3, -1.2, 2.0])
    st, diag = smc_stage(init_particles(3, _params(51)), 1, lambda m, o, P, objs, s, p: np.full(len(P), a[o]),
                         types, table, _params(51))
    want = np.exp(a - a.max()) / np.exp(a - a.max()).sum()
    assert np.allclose(diag["type_post"], want[None], rtol=1e-13, atol=0)


@pytest.mark.parametrize("stage_noise", [None, ((0.009, 0.6), (0.002, 0.1))])
def test_weights_are_unbiased_for_the_evidence(stage_noise):
    # E_q[p_1 / q] = integral of p_1 = Z for a likelihood with a closed-form
    # integral: exp(L) = exp(a dx) (1 + 0.5 cos dth) (1 + sigma/sigma_max) (2 - p_out),
    # whatever noise the placement stages score at
    rng = np.random.default_rng(6)
    table = random_table(rng)
    types = [faces_of(box_verts(rng)) for _ in range(2)]
    a = 8.0
    params = _params(21, counts=((2, 2, 2), (2, 1, 1)))
    params.stage_noise = stage_noise
    pose_of = {}

    # the likelihood reads each pose's placement back: contact_pose is wrapped
    # so that every pose it makes is recorded with its (dx, dy, dth)
    import oracle.smc as smc_mod

    real = smc_mod.contact_pose

    def tagged(table_, f, dx, dy, dth):
        P = real(table_, f, dx, dy, dth)
        pose_of[P.tobytes()] = (dx, dy, dth)
        return P

    def loglik2(m, o, P, objs, s, p):
        out = []
        for q in P:
            dx, dy, dth = pose_of[np.asarray(q).tobytes()]
            out.append(a * dx + np.log1p(0.5 * np.cos(dth)) + np.log1p(s / params.sigma_max) + np.log(2.0 - p))
        return np.array(out)

    smc_mod.contact_pose = tagged
    try:
        M = 2000
        st, _ = smc_stage(init_particles(M, params), 1, loglik2, types, table, params)
    finally:
        smc_mod.contact_pose = real
    # Z = sum over (o, c) of 1/(6|O|) * mean of exp(a dx) over the box * 1 * 1.5 * 1.5
    Z = 0.0
    for fs in types:
        for f in fs:
            lo, hi = root_box(table, f)
            half = hi[0]
            Z += (np.sinh(a * half) / (a * half)) / (6 * len(types))
    Z *= 2.25
    W = np.exp(st.logW)
    se = W.std() / np.sqrt(M)
    assert abs(W.mean() - Z) <= 4 * se, (W.mean(), Z, se)
    assert se < 0.05 * Z


def test_resampling_keeps_the_evidence_estimate():
    rng = np.random.default_rng(7)
    table = random_table(rng)
    types = [faces_of(box_verts(rng)) for _ in range(2)]
    params = _params(31, thr=2.0)
    lik = lambda m, o, P, objs, s, p: -50.0 * P[:, 0, 3] ** 2 + np.log(s) + m  # noqa: E731
    st, diag = smc_stage(init_particles(8, params), 1, lik, types, table, params)
    lse = lambda x: x.max() + np.log(np.exp(x - x.max()).sum())  # noqa: E731
    assert diag["resampled"]
    assert np.isclose(lse(st.logW), lse(diag["logW_pre"]), rtol=0, atol=1e-12)
    assert np.allclose(st.logW, st.logW[0])
    # every survivor is a copy of its ancestor's new object
    assert np.array_equal(st.place[:, 0], diag["place"][diag["ancestors"]])
