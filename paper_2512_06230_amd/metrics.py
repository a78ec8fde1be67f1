"""Tracking accuracy metrics of the paper's Sec. 4.2, computed on the host from the tracker's
estimates (these are evaluation code, not part of the filter).

* relative cardinality error: |n_hat - n| / n per time point, averaged over the time points;
* matched tracking error: at every time point the minimum-distance matching (Hungarian
  algorithm) between estimated and true positions, and the mean distance of the matched pairs;
  averaged over the time points.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import linear_sum_assignment


def cardinality_error(n_est, n_true) -> float:
    n_est = np.asarray(n_est, np.float64)
    n_true = np.asarray(n_true, np.float64)
    return float(np.mean(np.abs(n_est - n_true) / np.maximum(n_true, 1.0)))


def matched_distances(est_xy, true_xy) -> np.ndarray:
    """Distances of the optimal (minimum total distance) matching of two point sets."""
    a = np.asarray(est_xy, np.float64).reshape(-1, 2)
    b = np.asarray(true_xy, np.float64).reshape(-1, 2)
    if len(a) == 0 or len(b) == 0:
        return np.zeros(0)
    D = np.linalg.norm(a[:, None, :] - b[None, :, :], axis=2)
    r, c = linear_sum_assignment(D)
    return D[r, c]


def matched_error(estimates, truths) -> float:
    """Time average of the per-time-point mean matched distance (time points with an empty
    side are skipped)."""
    per = []
    for e, t in zip(estimates, truths):
        d = matched_distances(e, t)
        if len(d):
            per.append(float(d.mean()))
    return float(np.mean(per)) if per else float("nan")
