"""The pins catch plausible mistakes: each mutant below plants one mistake in
a copy of the oracle's C source (compiled on the CPU), and at least one pin
must fail against it.  The pins themselves are the tests of the other
test_oracle_* modules, run here against the mutant."""

import os
import subprocess
import tempfile

import pytest

import oracle

from . import test_oracle_adjoint as adj
from . import test_oracle_render as ren
from . import test_oracle_sampler as smp
from . import test_oracle_score as sco

SRC = os.path.join(os.path.dirname(oracle.__file__), "b3d_oracle.c")

MUTANTS = {
    "inverted coverage test": ("if (w0 > 0.0 || w1 > 0.0 || w2 > 0.0) continue;",
                               "if (w0 < 0.0 || w1 < 0.0 || w2 < 0.0) continue;"),
    "back faces kept instead of front": ("if (!(nc0 < 0.0)) continue; /* back-facing or edge-on */",
                                         "if (!(nc0 > 0.0)) continue;"),
    "pixel centre without the half pixel": ("d[0] = ((double)c + 0.5 - cam[2]) / cam[0];",
                                            "d[0] = ((double)c - cam[2]) / cam[0];"),
    "transposed rotation": ("c[0] = P[0] * v[0] + P[1] * v[1] + P[2] * v[2] + P[3];",
                            "c[0] = P[0] * v[0] + P[4] * v[1] + P[8] * v[2] + P[3];"),
    "inlier weight without (1 - p_out)": ("const double a = p_out / V, b = (1.0 - p_out) / M;\n  const double norm = pow(2.0 * M_PI * sigma * sigma, -1.5);\n  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);\n#pragma omp parallel for schedule(static)\n  for (int n = 0; n < N; ++n) {\n    const double* q = rend + (size_t)n * H * W * 3;\n    double acc",
                                          "const double a = p_out / V, b = 1.0 / M;\n  const double norm = pow(2.0 * M_PI * sigma * sigma, -1.5);\n  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);\n#pragma omp parallel for schedule(static)\n  for (int n = 0; n < N; ++n) {\n    const double* q = rend + (size_t)n * H * W * 3;\n    double acc"),
    "Gaussian normaliser of a 2-D density": ("const double norm = pow(2.0 * M_PI * sigma * sigma, -1.5);\n  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);\n#pragma omp parallel for schedule(static)\n  for (int n = 0; n < N; ++n) {\n    const double* q = rend + (size_t)n * H * W * 3;\n    double acc",
                                             "const double norm = pow(2.0 * M_PI * sigma * sigma, -1.0);\n  const double inv2s2 = 1.0 / (2.0 * sigma * sigma);\n#pragma omp parallel for schedule(static)\n  for (int n = 0; n < N; ++n) {\n    const double* q = rend + (size_t)n * H * W * 3;\n    double acc"),
    "variance read as sigma^2 / 1": ("S += norm * exp(-(dx * dx + dy * dy + dzv * dzv) * inv2s2);",
                                     "S += norm * exp(-(dx * dx + dy * dy + dzv * dzv) * 2.0 * inv2s2);"),
    "window one pixel too wide": ("  const int h = (r - 1) / 2;\n  const double a = p_out / V, b = (1.0 - p_out) / M;\n  const double norm = pow(2.0 * M_PI * sigma * sigma, -1.5);\n  const double inv2s2",
                                  "  const int h = (r + 1) / 2;\n  const double a = p_out / V, b = (1.0 - p_out) / M;\n  const double norm = pow(2.0 * M_PI * sigma * sigma, -1.5);\n  const double inv2s2"),
    "point gradient with the wrong sign": ("const double coef = g * (b / L) * K / s2;", "const double coef = -g * (b / L) * K / s2;"),
    "p_out gradient with a wrong sign": ("dp += (1.0 / V - S / M) / L;", "dp += (1.0 / V + S / M) / L;"),
    "rotation gradient with crossed operands": ("cross3(nn, tq, w);", "cross3(tq, nn, w);"),
    "Gumbel noise with the wrong sign": ("const double v = logL[n] - log(-log(u));", "const double v = logL[n] + log(-log(u));"),
    "Philox multiplier": ("(uint64_t)0xD2511F53u * x[0]", "(uint64_t)0xD2511F55u * x[0]"),
    "cell centres off by half a cell": ("return -h + (2.0 * i + 1.0) * h / n;", "return -h + (2.0 * i) * h / n;"),
}

PINS = [
    lambda: [ren.test_plain_scan_matches_bruteforce_ray_casting(c) for c in range(5)],
    ren.test_closed_form_axis_aligned_cube,
    ren.test_pose_equals_pretransformed_vertices,
    sco.test_outlier_only_likelihood_is_uniform_density,
    sco.test_full_window_equals_untruncated_eq1_with_scipy_density,
    sco.test_single_pixel_closed_form,
    lambda: [sco.test_window_reaches_exactly_h_pixels(w) for w in (1, 3, 5, 7)],
    adj.test_score_adjoint_matches_central_differences,
    adj.test_pose_adjoint_matches_frozen_visibility_differences,
    adj.test_frontal_face_depth_derivatives_closed_form,
    lambda: [smp.test_philox_known_answers(r) for r in range(3)],
    smp.test_gumbel_max_frequencies_follow_softmax,
    smp.test_partition_schedule_proposal_density_integrates_to_one,
]


def _build(src_text, workdir):
    c = os.path.join(workdir, "m.c")
    so = os.path.join(workdir, "m.so")
    open(c, "w").write(src_text)
    subprocess.check_call(["gcc", "-O1", "-fopenmp", "-fPIC", "-shared", "-std=c11", "-D_GNU_SOURCE", "-o", so, c,
                           "-lm"])
    return oracle.load(so)


def _caught():
    for pin in PINS:
        try:
            pin()
        except (AssertionError, ValueError, FloatingPointError):
            return True
    return False


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_every_planted_mistake_fails_a_pin(name):
    old, new = MUTANTS[name]
    text = open(SRC).read()
    assert text.count(old) == 1, f"mutation site for '{name}' not found exactly once"
    with tempfile.TemporaryDirectory() as d:
        mutant = _build(text.replace(old, new), d)
        try:
            oracle.use_library(mutant)
            assert _caught(), f"no pin catches: {name}"
        finally:
            oracle.use_library(None)


def test_the_unmutated_oracle_passes_every_pin():
    with tempfile.TemporaryDirectory() as d:
        oracle.use_library(_build(open(SRC).read(), d))
        try:
            assert not _caught()
        finally:
            oracle.use_library(None)
