"""The convoy benchmark of the paper's Sec. 4.1 (synthetic base track) and the metrics of
Sec. 4.2 (CPU): copies offset in time by delta steps along one closed track, D detections per
object with sigma noise; the Hungarian matching against brute force over permutations; the
cardinality error's definition on hand-made cases."""
import itertools

import numpy as np

from paper_2512_06230_amd import metrics
from paper_2512_06230_amd import scenarios as sc


def test_convoy_copies_follow_the_base_track_with_offsets():
    spec = sc.ConvoySpec(n_obj=7, delta=2, det=5, sigma=0.25, K=548, seed=3)
    scene = sc.make_convoy(spec, n_steps=60)
    base = sc.convoy_track(spec.K, spec.dt, spec.loops)
    assert base.min() > 0.0 and base.max() < 80.0  # inside the 80 x 80 m area
    step = np.linalg.norm(np.diff(np.vstack([base, base[:1]]), axis=0), axis=1)
    assert step.max() < 3.0 * np.median(step)  # closed and smooth: the wrap-around is one step
    for k in (0, 17, 59):
        x = scene.truth_x[k]
        for n in range(spec.n_obj):
            np.testing.assert_allclose(x[n, :2], base[(k + spec.delta * n) % spec.K])
        z = scene.meas[k].astype(np.float64)
        assert z.shape == (spec.n_obj * spec.det, 2)
    # detection noise: sample standard deviation around the truth close to sigma
    res = np.concatenate([scene.meas[k].astype(np.float64).reshape(spec.n_obj, spec.det, 2)
                          - scene.truth_x[k][:, None, :2] for k in range(60)]).reshape(-1)
    assert abs(res.std() - spec.sigma) < 0.02 and abs(res.mean()) < 0.02


def test_matching_is_the_minimum_total_distance():
    rng = np.random.default_rng(5)
    for _ in range(20):
        a = rng.uniform(0, 10, (rng.integers(1, 6), 2))
        b = rng.uniform(0, 10, (rng.integers(1, 6), 2))
        d = metrics.matched_distances(a, b)
        n = min(len(a), len(b))
        best = np.inf
        if len(a) <= len(b):
            for perm in itertools.permutations(range(len(b)), n):
                best = min(best, sum(np.linalg.norm(a[i] - b[j]) for i, j in enumerate(perm)))
        else:
            for perm in itertools.permutations(range(len(a)), n):
                best = min(best, sum(np.linalg.norm(a[j] - b[i]) for i, j in enumerate(perm)))
        assert len(d) == n and abs(d.sum() - best) < 1e-9


def test_cardinality_error_definition():
    assert metrics.cardinality_error([5, 4, 6], [5, 5, 5]) == (0 + 0.2 + 0.2) / 3
    assert metrics.cardinality_error([0], [2]) == 1.0
    est = [np.array([[0.0, 0.0], [3.0, 0.0]]), np.array([[1.0, 1.0]])]
    tru = [np.array([[0.0, 1.0], [3.0, 0.5]]), np.array([[1.0, 1.0], [9.0, 9.0]])]
    assert abs(metrics.matched_error(est, tru) - (0.75 + 0.0) / 2) < 1e-12
