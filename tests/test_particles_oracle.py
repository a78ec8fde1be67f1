"""Pins of the oracle's particle form (Sec. 3: weighted particles per track, constant turn
rate and velocity kinematics, likelihood weighting with resampling).  CPU only.

* kinematics: without noise a straight line when the turn rate is zero, a circle of radius
  |v / omega| about a fixed centre otherwise (heading advancing by omega dt per step), and the
  turning formula tends to the straight one as omega -> 0;
* noise: the accelerations drawn by the Box-Muller transform of Philox words are standard
  normal (Kolmogorov-Smirnov against scipy) and uncorrelated;
* association likelihood: one particle gives scipy's normal density; many particles drawn
  from N(m, C) give N(z; m, C + sigma^2 I) within Monte Carlo error; the gate follows the
  weighted moments;
* update: without resampling the weighted mean of particles drawn from N(m, C) is the Kalman
  posterior mean within Monte Carlo error; systematic resampling gives every particle
  floor or ceil of P w_p copies, and weights 1 / P.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import oracle as orc


def _states(rng, n, v=5.0, w=0.0):
    st = np.zeros((5, n))
    st[0] = rng.uniform(0, 50, n)
    st[1] = rng.uniform(0, 50, n)
    st[2] = v
    st[3] = rng.uniform(-math.pi, math.pi, n)
    st[4] = w
    return st


def test_ctrv_without_noise_is_a_line_or_a_circle():
    rng = np.random.default_rng(1)
    st = _states(rng, 50, v=4.0, w=0.0)
    out = orc.pf_predict(st, 0.1, 0.0, 0.0, 1, 0)
    np.testing.assert_allclose(out[0], st[0] + 4.0 * np.cos(st[3]) * 0.1, atol=1e-12)
    np.testing.assert_allclose(out[1], st[1] + 4.0 * np.sin(st[3]) * 0.1, atol=1e-12)
    # turning: every position stays on its circle, the heading advances linearly
    st = _states(rng, 50, v=6.0, w=0.7)
    cx = st[0] - 6.0 / 0.7 * np.sin(st[3])
    cy = st[1] + 6.0 / 0.7 * np.cos(st[3])
    cur = st.copy()
    for k in range(37):
        cur = orc.pf_predict(cur, 0.1, 0.0, 0.0, 1, k)
    np.testing.assert_allclose(np.hypot(cur[0] - cx, cur[1] - cy), 6.0 / 0.7, atol=1e-9)
    np.testing.assert_allclose(cur[3], st[3] + 37 * 0.07, atol=1e-9)
    # the turning formula approaches the straight one
    a = orc.pf_predict(_states(np.random.default_rng(2), 20, 5.0, 2e-4), 0.1, 0.0, 0.0, 1, 0)
    b = orc.pf_predict(_states(np.random.default_rng(2), 20, 5.0, 0.0), 0.1, 0.0, 0.0, 1, 0)
    assert np.max(np.abs(a[:2] - b[:2])) < 1e-5


def test_accelerations_are_standard_normal():
    n = 20000
    st = np.zeros((5, n))
    out = orc.pf_predict(st, 1.0, 1.0, 1.0, 77, 3)
    na = out[2]            # v' = dt nu_a
    nw = out[4]            # omega' = dt nu_w
    for x in (na, nw):
        assert stats.kstest(x, "norm").pvalue > 1e-4
    assert abs(np.corrcoef(na, nw)[0, 1]) < 0.03
    np.testing.assert_allclose(out[0], 0.5 * na, atol=1e-12)  # x' = dt^2/2 nu_a cos 0


def test_association_likelihood_and_gate():
    rng = np.random.default_rng(4)
    sigma, gamma, gate = 0.5, 3.0, 18.42
    st = np.zeros((5, 1))
    st[0, 0], st[1, 0] = 3.0, -1.0
    z = np.array([[3.2, -0.7], [30.0, 30.0]])
    phi = orc.pf_loglik(st, np.zeros(1), 1, 1, z, sigma, gamma, gate)
    ref = math.log(gamma) + stats.multivariate_normal([3.0, -1.0], sigma ** 2 * np.eye(2)).logpdf(z[0])
    assert abs(phi[0, 0] - ref) < 1e-10 and phi[0, 1] == -np.inf
    # a cloud of particles from N(m, C): the Gaussian marginal
    P = 40000
    m = np.array([10.0, 5.0])
    C = np.array([[1.0, 0.3], [0.3, 0.5]])
    xy = rng.multivariate_normal(m, C, P)
    st = np.zeros((5, P))
    st[0], st[1] = xy[:, 0], xy[:, 1]
    lw = np.full(P, -math.log(P))
    z = np.array([[10.5, 5.2], [9.0, 4.0], [12.5, 7.0]])
    phi = orc.pf_loglik(st, lw, 1, P, z, sigma, gamma, gate)
    for i in range(3):
        ref = math.log(gamma) + stats.multivariate_normal(m, C + sigma ** 2 * np.eye(2)).logpdf(z[i])
        assert abs(phi[0, i] - ref) < 0.03, (i, phi[0, i], ref)
    # gate on the weighted moments
    mu = xy.mean(0)
    S = np.cov(xy.T, bias=True) + sigma ** 2 * np.eye(2)
    far = mu + np.array([4.0, 0.0])
    d2 = (far - mu) @ np.linalg.solve(S, far - mu)
    phi = orc.pf_loglik(st, lw, 1, P, far[None], sigma, gamma, d2 * 1.001)
    assert np.isfinite(phi[0, 0])
    phi = orc.pf_loglik(st, lw, 1, P, far[None], sigma, gamma, d2 * 0.999)
    assert phi[0, 0] == -np.inf


def test_update_weights_and_systematic_resampling():
    rng = np.random.default_rng(9)
    P, sigma = 40000, 0.7
    m = np.array([2.0, 1.0])
    C = np.array([[1.5, 0.4], [0.4, 1.0]])
    xy = rng.multivariate_normal(m, C, P)
    st = np.zeros((5, P))
    st[0], st[1] = xy[:, 0], xy[:, 1]
    st[2] = np.arange(P)  # tags the particles
    lw = np.full(P, -math.log(P))
    z = np.array([[2.8, 0.2], [2.4, 0.9]])
    ost, olw, rs, fr = orc.pf_update(st, lw, 1, P, [0], [0, 2], [0, 1], z, sigma, 0.0, 5, 0)
    assert rs[0] == 0 and abs(np.logaddexp.reduce(olw)) < 1e-10
    w = np.exp(olw)
    post = (w[:, None] * ost[:2].T).sum(0)
    R = sigma ** 2 / 2 * np.eye(2)  # two detections: the mean with noise R / 2
    K = C @ np.linalg.inv(C + R)
    ref = m + K @ (z.mean(0) - m)
    assert np.max(np.abs(post - ref)) < 0.02, (post, ref)
    # systematic resampling: copies of particle p are floor or ceil of P w_p
    P = 2000
    st2 = np.zeros((5, P))
    st2[0], st2[1] = rng.normal(0, 1, P), rng.normal(0, 1, P)
    st2[2] = np.arange(P)
    lw2 = np.full(P, -math.log(P))
    ost, olw, rs, fr = orc.pf_update(st2, lw2, 1, P, [0], [0, 1], [0], np.array([[0.3, 0.1]]), 0.5, 1.1, 3, 0)
    assert rs[0] == 1 and np.allclose(olw, -math.log(P))
    a = st2[0] * 0.0 - ((0.3 - st2[0]) ** 2 + (0.1 - st2[1]) ** 2) / (2 * 0.25)
    wp = np.exp(a - np.logaddexp.reduce(a))
    cnt = np.bincount(ost[2].astype(int), minlength=P)
    assert cnt.sum() == P
    assert np.all(cnt >= np.floor(P * wp) - 1e-9) and np.all(cnt <= np.ceil(P * wp) + 1e-9)
    assert np.all(np.diff(ost[2]) >= 0)  # particles copied in order
