"""Pins of the oracle's exact-joint reweighting (the "joint likelihood of the sampled
associations" of Sec. 3 end): a track's detection set S is weighted by the marginal density of
all its detections together, J(S) = integral N(x; m, P) prod_{i in S} N(z_i; H x, R) dx, instead
of the product of the per-detection predictive densities.  CPU only.

* J against two independent routes: quadrature over the position plane (the velocity
  integrates out), and the prediction-error decomposition of sequential Kalman updates;
* one detection: J is the predictive density (scipy);
* the reweighted update against the brute-force children, reweighted here with the
  sequential-Kalman joint likelihood, re-ranked, tau-pruned and renormalised.
"""
import math

import numpy as np
import pytest
from scipy import stats

from oracle import bruteforce as bf
from oracle import oracle as orc
from oracle.oracle import Oracle
from paper_2512_06230_amd import scenarios as sc

BASE = dict(dt=1.0, q=1.0, sigma_z=1.0, p_survive=0.99, det_rate=1.47, clutter_density=2e-3,
            gate_d2=-2.0 * math.log(1e-4), birth_r_max=0.5, birth_rate=0.5, birth_sigma_v=2.0,
            birth_ru_max=0.5, birth_cluster_d=3.0, h_max=64, tau=0.0)


def _track(rng):
    A = rng.normal(0, 0.6, (4, 4))
    P = A @ A.T + np.diag([0.3, 0.4, 0.5, 0.5])
    m = rng.normal(0, 2.0, 4)
    return m, P


def sequential_joint(sigma, z, m, P):
    """log prod_j N(z_j; H m_{j-1}, H P_{j-1} H^T + R), the Kalman filter's innovations."""
    H = np.zeros((2, 4))
    H[0, 0] = H[1, 1] = 1.0
    R = sigma ** 2 * np.eye(2)
    m, P = np.array(m, float), np.array(P, float)
    out = 0.0
    for zj in np.asarray(z, float).reshape(-1, 2):
        S = H @ P @ H.T + R
        out += stats.multivariate_normal(H @ m, S).logpdf(zj)
        K = P @ H.T @ np.linalg.inv(S)
        m = m + K @ (zj - H @ m)
        P = (np.eye(4) - K @ H) @ P
    return out


@pytest.mark.parametrize("n", [1, 2, 3, 5])
def test_joint_loglik_matches_sequential_kalman(n):
    rng = np.random.default_rng(40 + n)
    for _ in range(5):
        m, P = _track(rng)
        sigma = rng.uniform(0.5, 2.0)
        z = m[:2] + rng.normal(0, 1.5, (n, 2))
        got = orc.joint_loglik(sigma, z, m, P)
        assert abs(got - sequential_joint(sigma, z, m, P)) < 1e-9
        if n == 1:
            ref = stats.multivariate_normal(m[:2], P[:2, :2] + sigma ** 2 * np.eye(2)).logpdf(z[0])
            assert abs(got - ref) < 1e-10


def test_joint_loglik_matches_quadrature():
    rng = np.random.default_rng(3)
    m, P = _track(rng)
    sigma = 0.9
    z = m[:2] + rng.normal(0, 1.0, (3, 2))
    # integral over the position plane of N(p; m_p, P_pp) prod_i N(z_i; p, R) (velocity marginalised)
    g = np.linspace(-12.0, 12.0, 1201)
    X, Y = np.meshgrid(m[0] + g, m[1] + g, indexing="ij")
    pts = np.stack([X.ravel(), Y.ravel()], axis=1)
    f = stats.multivariate_normal(m[:2], P[:2, :2]).pdf(pts)
    for zi in z:
        f = f * stats.multivariate_normal(zi, sigma ** 2 * np.eye(2)).pdf(pts)
    quad = f.sum() * (g[1] - g[0]) ** 2
    assert abs(orc.joint_loglik(sigma, z, m, P) - math.log(quad)) < 1e-6


@pytest.mark.parametrize("seed", range(6))
def test_reweighted_update_matches_bruteforce(seed):
    rng = np.random.default_rng(820 + seed)
    st = sc.random_state(rng, n_lab=2 + seed % 2, n_hyp=3, side=6.0, versions=1, p_present=0.9)
    z = sc.measurements_near(rng, st, 1, 6.0, 1.0, det_mean=2.5)[:5]
    K, tau = (1000, 0.0) if seed % 2 == 0 else (6, 1e-3)
    p = dict(BASE, h_max=K, tau=tau)
    o = Oracle(p)
    o.import_state(st)
    o.set_joint(True)
    o.update(0, z)
    out = o.export_state()
    ref = bf.update(st, z, p, K)   # factorised ranking and tau, as the selection
    zz = np.asarray(z, np.float32).astype(np.float64)
    sig = p["sigma_z"]
    rows = []
    moved = 0
    for c in ref["children"]:
        corr = 0.0
        for u in set(x for x in c["theta"] if x >= 0):
            S = [i for i, x in enumerate(c["theta"]) if x == u]
            if len(S) < 2:
                continue
            mu, Pu = st["inst_m"][u], np.asarray(st["inst_P"][u]).reshape(4, 4)
            corr += sequential_joint(sig, zz[S], mu, Pu)
            for i in S:
                corr -= stats.multivariate_normal(mu[:2], Pu[:2, :2] + sig ** 2 * np.eye(2)).logpdf(zz[i])
        moved += abs(corr) > 1e-6
        rows.append((c["logw"] + corr, (c["parent"], tuple(c["theta"]))))
    assert moved > 0  # some kept child holds a track with several detections
    order = sorted(range(len(rows)), key=lambda j: -rows[j][0])   # stable: ties keep the rank
    v = np.array([rows[j][0] for j in order])
    keep = len(v)
    if tau > 0:
        z0 = np.logaddexp.reduce(v)
        keep = 1
        while keep < len(v) and math.exp(v[keep] - z0) >= tau:
            keep += 1
    v = v[:keep] - np.logaddexp.reduce(v[:keep])
    ids = [rows[j][1] for j in order[:keep]]
    got = [(int(a), tuple(int(x) for x in t)) for a, t in zip(out["hyp_parent"], out["theta"])]
    assert got == ids
    np.testing.assert_allclose(out["hyp_logw"], v, atol=1e-9)
