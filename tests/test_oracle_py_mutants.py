"""The pins of the oracle's Python modules catch plausible mistakes: each
mutant plants one mistake in a copy of oracle/noise.py, c2f.py, refine.py or
smc.py, and at least one of that module's pins (the tests of
test_oracle_noise, test_oracle_sampler, test_oracle_refine and
test_oracle_smc) must fail against it."""

import importlib
import sys
import types

import pytest

import oracle

from . import test_oracle_noise as noise_pins
from . import test_oracle_refine as refine_pins
from . import test_oracle_sampler as sampler_pins
from . import test_oracle_smc as smc_pins

MUTANTS = {
    "noise": {
        "sigma cells at their right edges": ("return sigma_max * (np.arange(A) + 0.5) / A,",
                                             "return sigma_max * (np.arange(A) + 1.0) / A,"),
        "p_out cells at their left edges": (", (np.arange(B) + 0.5) / B", ", np.arange(B) / B"),
        "grid weights 1/(A + B)": ("-np.log(A * B)", "-np.log(A + B)"),
        "marginal without the shift it subtracted": ("marg = m + np.log(", "marg = np.log("),
    },
    "c2f": {
        "log q not accumulated over stages": ("logq[k] += lw[0]", "logq[k] = lw[0]"),
        "centre not moved to the drawn cell": ("centres[k] = P[i[0]]", "centres[k] = centres[k]"),
        "every particle drawing with one counter": ("_, i, lw = sample(L, 1, seed, stage=t, k0=k)",
                                                    "_, i, lw = sample(L, 1, seed, stage=t, k0=0)"),
        "cells halved instead of split by the counts": ("half = half / np.asarray(c, dtype=np.float64)",
                                                        "half = half / 2.0"),
        "final cell measured by its half-widths": ("v *= 2.0 * h / n", "v *= h / n"),
    },
    "refine": {
        "Adam without bias correction": ("s = lr * (m / (1 - b1**it)) / (np.sqrt(v / (1 - b2**it)) + eps)",
                                         "s = lr * m / (np.sqrt(v) + eps)"),
        "rotation step applied on the right": ("P[n, :3, :3] = rotvec_exp(s[n, 3:]) @ P[n, :3, :3]",
                                               "P[n, :3, :3] = P[n, :3, :3] @ rotvec_exp(s[n, 3:])"),
        "Rodrigues with sin and 1 - cos swapped": ("np.eye(3) + np.sin(th) * K + (1 - np.cos(th)) * (K @ K)",
                                                   "np.eye(3) + (1 - np.cos(th)) * K + np.sin(th) * (K @ K)"),
        "left Jacobian not transposed": ("(left_jacobian(xi[n, 3:]).T @ g[n, 3:6])",
                                         "(left_jacobian(xi[n, 3:]) @ g[n, 3:6])"),
        "left Jacobian's second coefficient over th^2": ("(th - np.sin(th)) / th**3", "(th - np.sin(th)) / th**2"),
        "retraction rotating the translation step": ("out[n, :3, 3] = B[n, :3, 3] + xi[n, :3]",
                                                     "out[n, :3, 3] = B[n, :3, 3] + rotvec_exp(xi[n, 3:]) @ xi[n, :3]"),
    },
    "smc": {
        "resting offset with the wrong sign": ("d = -np.array([0.5 * (mn[0] + mx[0]), 0.5 * (mn[1] + mx[1]), mn[2]])",
                                               "d = np.array([0.5 * (mn[0] + mx[0]), 0.5 * (mn[1] + mx[1]), mn[2]])"),
        "footprint offset not turned": ("P[:3, 3] = Rz @ f.d + np.array([dx, dy, 0.0])",
                                        "P[:3, 3] = f.d + np.array([dx, dy, 0.0])"),
        "prior without the face factor": ("np.log(n_types) + np.log(6.0) +", "np.log(n_types) +"),
        "density of the point in the final cell dropped": ("lq -= np.log(np.prod(hi - lo))", "lq -= 0.0"),
        "noise cell density dropped": ("lq += lw[0] - np.log(params.sigma_max / (A * B))", "lq += lw[0]"),
        "incremental weight without the previous target": ("logW_pre = state.logW + logp - state.logp - logq + back",
                                                           "logW_pre = state.logW + logp - logq + back"),
        "resampled weights summed instead of averaged": ("np.full(M, mx + np.log(e.sum()) - np.log(M))",
                                                         "np.full(M, mx + np.log(e.sum()))"),
        "type posterior summed over the wrong axis": ("w.reshape(n_types, -1).sum(axis=1)",
                                                      "w.reshape(-1, n_types).sum(axis=0)[:n_types]"),
    },
}

PINS = {
    "noise": [noise_pins.test_p_out_marginal_of_one_pixel_is_exact_under_the_midpoint_rule,
              noise_pins.test_sigma_marginal_of_one_pixel_converges_to_the_closed_form,
              noise_pins.test_one_point_grid_is_the_plain_score_plus_its_weight],
    "c2f": [sampler_pins.test_partition_schedule_proposal_density_integrates_to_one,
            sampler_pins.test_flat_likelihood_draws_final_cells_uniformly,
            sampler_pins.test_c2f_rotation_stages_compose_around_chosen_centres],
    "refine": [refine_pins.test_first_adam_step_has_the_learning_rate_as_length,
               refine_pins.test_rotation_exponential_matches_scipy_and_stays_orthonormal,
               refine_pins.test_retract_grad_matches_finite_differences_through_the_retraction,
               refine_pins.test_left_jacobian_closed_forms],
    "smc": [smc_pins.test_resting_face_lies_on_the_table_centred_and_turned_about_its_normal,
            smc_pins.test_placement_prior_integrates_to_one,
            lambda: [smc_pins.test_constant_likelihood_makes_every_weight_the_likelihood(t) for t in (0.0, 2.0)],
            smc_pins.test_every_cell_is_scored_at_its_own_face,
            smc_pins.test_type_posterior_of_a_type_only_likelihood_is_its_softmax,
            lambda: [smc_pins.test_weights_are_unbiased_for_the_evidence(sn)
                     for sn in (None, ((0.009, 0.6), (0.002, 0.1)))],
            smc_pins.test_resampling_keeps_the_evidence_estimate],
}

PIN_MODULES = [noise_pins, refine_pins, sampler_pins, smc_pins]


def mutant_module(sub, old, new):
    real = importlib.import_module(f"oracle.{sub}")
    src = open(real.__file__).read()
    assert src.count(old) == 1, old
    name = f"oracle.{sub}"
    mod = types.ModuleType(name)
    mod.__package__ = "oracle"
    mod.__file__ = real.__file__
    sys.modules[name] = mod  # dataclasses look their module up while the source runs
    try:
        exec(compile(src.replace(old, new), real.__file__, "exec"), mod.__dict__)
    finally:
        sys.modules[name] = real
    return real, mod


def run_pins(sub, real, mod):
    """Run the module's pins with every name they took from the real module
    (and the module itself) pointing at the mutant; the number that fail."""
    saved = []
    for pm in PIN_MODULES:
        for k, v in list(vars(pm).items()):
            if v is real or (hasattr(real, k) and getattr(real, k) is v and not isinstance(v, types.ModuleType)):
                saved.append((pm, k, v))
                setattr(pm, k, mod if v is real else getattr(mod, k))
    sys.modules[f"oracle.{sub}"] = mod
    setattr(oracle, sub, mod)
    failed = 0
    try:
        for pin in PINS[sub]:
            try:
                pin()
            except (AssertionError, KeyError, ValueError, IndexError, FloatingPointError):
                failed += 1
    finally:
        for pm, k, v in saved:
            setattr(pm, k, v)
        sys.modules[f"oracle.{sub}"] = real
        setattr(oracle, sub, real)
    return failed


CASES = [(sub, name) for sub in MUTANTS for name in sorted(MUTANTS[sub])]


@pytest.mark.filterwarnings("ignore")
@pytest.mark.parametrize("sub,name", CASES)
def test_every_planted_mistake_fails_a_pin(sub, name):
    old, new = MUTANTS[sub][name]
    real, mod = mutant_module(sub, old, new)
    assert run_pins(sub, real, mod) > 0, f"no pin catches: {sub}: {name}"


@pytest.mark.filterwarnings("ignore")
@pytest.mark.parametrize("sub", sorted(MUTANTS))
def test_the_unmutated_modules_pass_every_pin(sub):
    # the module rebuilt from its unchanged source, through the same machinery
    first = open(importlib.import_module(f"oracle.{sub}").__file__).read().splitlines()[0]
    real, same = mutant_module(sub, first, first)
    assert run_pins(sub, real, same) == 0
