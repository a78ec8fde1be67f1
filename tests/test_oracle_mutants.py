"""The oracle's pins are sensitive: every planted mistake (a dropped term, a wrong sign,
a wrong coefficient, a transposed operand, a missing search rule, a wrong tie-break,
a missing cap) built into a copy of the oracle on the CPU fails at least one pin."""
import functools
import os
import types

import pytest

from oracle import oracle as orc
from tests import test_oracle_pins as pins
from tests import test_joint_oracle as joint
from tests import test_particles_oracle as particles
from tests import test_sampler_oracle as sampler

PINS = [
    lambda: pins.test_predict_moments_match_van_loan(),
    lambda: pins.test_pair_loglik_matches_scipy_and_gate(),
    lambda: [pins.test_update_matches_bruteforce(s) for s in range(12)],
    lambda: [pins.test_predict_matches_bruteforce(s) for s in range(8)],
    lambda: pins.test_predict_structural_ties_use_canonical_key(),
    lambda: pins.test_predict_cross_parent_tie_goes_to_lower_rank(),
    lambda: pins.test_single_object_reduces_to_kalman_filter(),
    lambda: pins.test_births_from_unexplained_measurements(),
    lambda: pins.test_truncate_hmax_then_tau_prefix_renormalised(),
    lambda: pins.test_truncate_tau_is_relative_to_the_kept_set(),
    lambda: pins.test_estimate_map_cardinality_not_global_best(),
    lambda: pins.test_estimate_cardinality_tie_goes_to_the_smaller_count(),
    lambda: pins.test_learned_births_restore_the_removed_mass(),
    lambda: sampler.test_categorical_draw_follows_the_normalised_row(),
    lambda: [sampler.test_sampled_children_are_children_with_their_exact_weights(s) for s in range(4)],
    lambda: joint.test_joint_loglik_matches_sequential_kalman(2),
    lambda: [joint.test_reweighted_update_matches_bruteforce(s) for s in range(2)],
    lambda: particles.test_ctrv_without_noise_is_a_line_or_a_circle(),
    lambda: particles.test_update_weights_and_systematic_resampling(),
]

MUTANTS = {
    1: "miss term -gamma|J| dropped",
    2: "Kalman correction with the wrong sign",
    3: "process-noise cross term dt^2/3",
    4: "best-first successor rule (c) missing",
    5: "log|S| without the factor 1/2",
    6: "innovation covariance entries transposed in the gate",
    7: "tie-break by parent rank reversed",
    8: "birth existence not capped",
    9: "estimate returns the globally best hypothesis",
    10: "cardinality tie goes to the larger count",
    11: "no renormalisation after tau",
    12: "tau against the normaliser before the H_max cut",
    13: "removed pairs' mass not restored in the births' clutter probabilities",
    14: "sampled rows normalised without the clutter entry",
    15: "joint likelihood without the shared track uncertainty between detections",
    16: "turning motion bends the wrong way in y",
}


@pytest.mark.parametrize("mutant", sorted(MUTANTS))
def test_planted_mistake_is_caught(mutant, tmp_path, monkeypatch):
    lib = orc.build(out=os.path.join(str(tmp_path), "liboracle_m%d.so" % mutant), mutant=mutant)
    monkeypatch.setattr(pins, "Oracle", functools.partial(orc.Oracle, lib=lib))
    monkeypatch.setattr(sampler, "Oracle", functools.partial(orc.Oracle, lib=lib))
    monkeypatch.setattr(joint, "Oracle", functools.partial(orc.Oracle, lib=lib))
    monkeypatch.setattr(joint, "orc", types.SimpleNamespace(joint_loglik=functools.partial(orc.joint_loglik, lib=lib)))
    monkeypatch.setattr(particles, "orc", types.SimpleNamespace(
        **{f: functools.partial(getattr(orc, f), lib=lib) for f in ("pf_predict", "pf_loglik", "pf_update")}))
    failed = 0
    for pin in PINS:
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed > 0, "planted mistake %d (%s) passed every pin" % (mutant, MUTANTS[mutant])
