"""The occlusion-handling pins catch plausible mistakes: each mutant plants
one mistake in a copy of oracle/track.py's source, and at least one of the
tracking pins (test_oracle_track) must fail against it."""

import sys
import types

import pytest

from oracle import track

from . import test_oracle_track as pins

SRC = track.__file__

MUTANTS = {
    "kept rotation applied on the right": ("P[:3, :3] = g.dR[o] @ prev[:3, :3]", "P[:3, :3] = prev[:3, :3] @ g.dR[o]"),
    "kept translation subtracted": ("P[:3, 3] = prev[:3, 3] + g.dt[o]", "P[:3, 3] = prev[:3, 3] - g.dt[o]"),
    "motion taken as R_prev R_new^T": ("g.dR[o] = new[:3, :3] @ prev[:3, :3].T", "g.dR[o] = prev[:3, :3] @ new[:3, :3].T"),
    "threshold itself dropped": ("if seen >= g.min_visible:", "if seen > g.min_visible:"),
    "hidden pixels counted as seen": ("front = drawn & ((d_b <= 0) | (d_o <= d_b))", "front = drawn"),
    "depth alone compared": ("np.linalg.norm(oi - q, axis=-1) <= tol", "np.abs(oi[..., 2] - q[..., 2]) <= tol"),
    "search not widened": ("float(np.float32(np.float32(x) * np.float32(scale)))", "float(np.float32(x))"),
}

PINS = [
    pins.test_seen_fraction_counts_pixels_in_front_and_confirmed_by_the_observation,
    pins.test_gate_keeps_visible_updates_and_moves_hidden_objects_by_the_last_motion,
    pins.test_a_hidden_object_keeps_still_and_the_next_search_widens,
]


def mutant_module(old, new):
    src = open(SRC).read()
    assert src.count(old) == 1, old
    name = "oracle.track_mutant"
    mod = types.ModuleType(name)
    mod.__package__ = "oracle"
    mod.__file__ = SRC
    sys.modules[name] = mod  # the dataclass decorator looks its module up
    try:
        exec(compile(src.replace(old, new), SRC, "exec"), mod.__dict__)
    finally:
        del sys.modules[name]
    return mod


def run_pins(mod):
    failed = 0
    saved = pins.track
    pins.track = mod
    try:
        for pin in PINS:
            try:
                pin()
            except AssertionError:
                failed += 1
    finally:
        pins.track = saved
    return failed


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_every_planted_tracking_mistake_fails_a_pin(name):
    assert run_pins(mutant_module(*MUTANTS[name])) > 0, name


def test_the_unmutated_tracking_oracle_passes_every_pin():
    assert run_pins(mutant_module("def round32(a):", "def round32(a):")) == 0
