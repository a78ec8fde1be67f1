"""Pins of the FP64 reference of the learned pair proposal (CPU only).

* the bfloat16 rounding against torch's float32 -> bfloat16 conversion (library routine);
* pair features against the oracle's own gate (a second implementation), scipy's
  Mahalanobis distance and the chi-square quantile, and closed forms of the label
  existence probabilities;
* pair marginals, the lost mass of removed pairs and the update without them against
  brute-force enumeration of every association map;
* the hand-derived gradient against central finite differences and torch autograd;
* Adam against its closed forms (constant gradient, zero gradient) and torch.optim.Adam.
"""
import math

import numpy as np
import pytest
import torch
from scipy import stats
from scipy.spatial import distance

from oracle import bruteforce as bf
from oracle import proposal as pp
from oracle.oracle import Oracle
from paper_2512_06230_amd import scenarios as sc

BASE = dict(dt=1.0, q=1.0, sigma_z=1.0, p_survive=0.99, det_rate=1.47, clutter_density=2e-3,
            gate_d2=-2.0 * math.log(1e-4), birth_r_max=0.5, birth_rate=0.5, birth_sigma_v=2.0,
            birth_ru_max=0.5, birth_cluster_d=3.0, h_max=64, tau=0.0)


def _tiny(seed, n_lab=3, n_hyp=4, versions=2):
    rng = np.random.default_rng(seed)
    st = sc.random_state(rng, n_lab=n_lab, n_hyp=n_hyp, side=12.0, versions=versions, p_present=0.75)
    z = sc.measurements_near(rng, st, 2, 12.0, 1.0)[:5]
    return st, z


def _data(seed, n=300):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(0, 18, n), rng.normal(0, 2, n), rng.normal(0, 2, n),
                         rng.uniform(0, 1, n), rng.integers(0, 20, n), rng.integers(1, 12, n)])
    y = rng.uniform(0, 1, n) ** 3
    w = rng.uniform(0.1, 1.0, n)
    params = sc.mlp_init(seed).astype(np.float64)
    params[pp.unpack(np.arange(pp.N_PARAM, dtype=np.float64))["b1"].astype(int)] = rng.normal(0, 0.1, 64)
    return params, pp.feature_norm(X), X, y, w


# --------------------------------------------------------------------------- rounding
def test_bf16_matches_torch_conversion():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.normal(0, 1, 5000), rng.normal(0, 1e3, 2000), rng.uniform(-1e-3, 1e-3, 2000)])
    x = x.astype(np.float32)
    # exact halfway cases: ties go to the even neighbour
    ties = np.array([1 + 2 ** -8, 1 + 3 * 2 ** -8, -(2 + 2 ** -7), 0.75 + 2 ** -9], np.float32)
    x = np.concatenate([x, ties])
    ref = torch.from_numpy(x).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(pp.bf16(x.astype(np.float64)), ref)
    assert pp.bf16(1 + 2 ** -8) == 1.0 and pp.bf16(1 + 3 * 2 ** -8) == 1 + 2 ** -6


# --------------------------------------------------------------------------- features
@pytest.mark.parametrize("seed", range(4))
def test_features_against_gate_scipy_and_closed_forms(seed):
    st, z = _tiny(200 + seed)
    k = 3
    f = pp.pair_features(st, z, k, BASE["sigma_z"], BASE["gate_d2"])
    o = Oracle(BASE)
    o.import_state(st)
    o.update(k, z)
    pr = o.pairs()
    # the same gated pairs, in the same order, as the oracle's update
    np.testing.assert_array_equal(f["u"], pr["u"])
    np.testing.assert_array_equal(f["i"], pr["i"])
    w = np.exp(st["hyp_logw"])
    for row, u, i in zip(f["X"], f["u"], f["i"]):
        S = st["inst_P"][u].reshape(4, 4)[:2, :2] + np.eye(2)
        d = distance.mahalanobis(z[i].astype(np.float64), st["inst_m"][u][:2], np.linalg.inv(S))
        assert abs(row[0] - d * d) < 1e-9 * max(1.0, d * d)
        assert row[0] <= stats.chi2.ppf(0.9999, 2)
        np.testing.assert_allclose(row[1:3], z[i].astype(np.float64) - st["inst_m"][u][:2], atol=1e-12)
        # existence of the label: total weight of the hypotheses holding it
        lab = tuple(st["inst_lab"][u])
        holders = [h for h in range(len(w))
                   if any(tuple(st["inst_lab"][v]) == lab for v in st["hyp_idx"][st["hyp_off"][h]:st["hyp_off"][h + 1]])]
        assert abs(row[3] - w[holders].sum()) < 1e-12
        assert row[4] == k - lab[0]
        assert row[5] == np.sum(f["u"] == u)
    # expected cardinality: sum over labels of r_l equals sum_h w_h |J_h|
    r = pp.label_existence(st)
    card = sum(w[h] * (st["hyp_off"][h + 1] - st["hyp_off"][h]) for h in range(len(w)))
    assert abs(sum(r.values()) - card) < 1e-12


def test_single_hypothesis_labels_exist_with_probability_one():
    rng = np.random.default_rng(5)
    st = sc.random_state(rng, n_lab=4, n_hyp=1, side=12.0, versions=1, p_present=1.0)
    r = pp.label_existence(st)
    assert len(r) == 4 and all(abs(v - 1.0) < 1e-15 for v in r.values())


# --------------------------------------------------------------------------- marginals, lost mass
@pytest.mark.parametrize("seed", range(6))
def test_pair_marginals_match_bruteforce(seed):
    st, z = _tiny(300 + seed, n_lab=2 + seed % 2, n_hyp=3)
    o = Oracle(BASE)
    o.import_state(st)
    o.update(0, z)
    pr = o.pairs()
    ref = bf.update(st, z, BASE, 10)
    for u, i, m, e in zip(pr["u"], pr["i"], pr["mass"], pr["exist"]):
        assert abs(m - ref["pair_mass"].get((int(u), int(i)), 0.0)) < 1e-10
        assert abs(e - ref["exist"].get(int(u), 0.0)) < 1e-10
    y, wt = pp.targets(pr)
    assert np.all((y >= 0) & (y <= 1))
    # summed over instances, the pair marginals of a detection give its non-clutter probability
    for i in range(z.shape[0]):
        assert abs(pr["mass"][pr["i"] == i].sum() - o.diag(len(st["hyp_logw"]))["ru"][i]) < 1e-10


@pytest.mark.parametrize("seed", range(6))
def test_lost_mass_and_reduced_update_match_bruteforce(seed):
    st, z = _tiny(400 + seed, n_lab=2 + seed % 2, n_hyp=3)
    o = Oracle(BASE)
    o.import_state(st)
    o.update(0, z)
    pr = o.pairs()
    rng = np.random.default_rng(seed)
    pick = rng.uniform(size=len(pr["u"])) < 0.4
    skip = list(zip(pr["u"][pick].tolist(), pr["i"][pick].tolist()))
    for K in (3, 1000):
        o2 = Oracle(dict(BASE, h_max=K))
        o2.import_state(st)
        o2.set_skip(np.array([a for a, _ in skip], np.int32), np.array([b for _, b in skip], np.int32))
        o2.update(0, z)
        out = o2.export_state()
        dg = o2.diag(len(st["hyp_logw"]))
        ref = bf.update(st, z, BASE, K, skip=skip)
        assert abs(dg["lost"] - ref["lost"]) < 1e-10
        ch = ref["children"]
        assert len(ch) == len(out["hyp_logw"])
        for h, c in enumerate(ch):
            assert out["hyp_parent"][h] == c["parent"]
            assert tuple(out["theta"][h]) == c["theta"]
            assert abs(out["hyp_logw"][h] - c["logw"]) < 1e-9
            for i, u in enumerate(c["theta"]):
                assert (u, i) not in skip
    # no skipped pair: nothing is lost
    o3 = Oracle(BASE)
    o3.import_state(st)
    o3.update(0, z)
    assert o3.diag(len(st["hyp_logw"]))["lost"] == 0.0


# --------------------------------------------------------------------------- gradient
def test_gradient_matches_finite_differences():
    params, norm, X, y, w = _data(1, n=60)
    loss, g = pp.loss_and_grad(params, norm, X, y, w, bf16_mode=False)
    rng = np.random.default_rng(2)
    idx = np.concatenate([rng.choice(pp.N_PARAM, 300, replace=False), np.arange(pp.N_PARAM - 65, pp.N_PARAM)])
    for j in idx:
        h = 1e-6 * max(1.0, abs(params[j]))
        a, b = params.copy(), params.copy()
        a[j] += h
        b[j] -= h
        fd = (pp.loss_and_grad(a, norm, X, y, w, False)[0] - pp.loss_and_grad(b, norm, X, y, w, False)[0]) / (2 * h)
        assert abs(fd - g[j]) <= 1e-6 * max(1e-3, abs(g[j])) + 1e-9, (j, fd, g[j])


def test_gradient_matches_torch_autograd():
    params, norm, X, y, w = _data(3, n=200)
    loss, g = pp.loss_and_grad(params, norm, X, y, w, bf16_mode=False)
    P = {k: torch.tensor(v, dtype=torch.float64, requires_grad=True) for k, v in pp.unpack(params).items()}
    xs = torch.tensor((X - norm[:6]) / norm[6:], dtype=torch.float64)
    h1 = torch.relu(xs @ P["W1"].T + P["b1"])
    h2 = torch.relu(h1 @ P["W2"].T + P["b2"])
    s = h2 @ P["w3"] + P["b3"][0]
    wt = torch.tensor(w, dtype=torch.float64)
    L = torch.nn.functional.binary_cross_entropy_with_logits(s, torch.tensor(y, dtype=torch.float64),
                                                           weight=wt, reduction="sum") / wt.sum()
    L.backward()
    assert abs(L.item() - loss) < 1e-12
    gt = np.concatenate([P[name].grad.numpy().reshape(-1) for name, _ in pp.SIZES])
    np.testing.assert_allclose(g, gt, rtol=1e-10, atol=1e-14)


def test_bf16_gradient_is_close_to_exact_gradient_of_rounded_weights():
    params, norm, X, y, w = _data(4, n=400)
    _, g16 = pp.loss_and_grad(params, norm, X, y, w, bf16_mode=True)
    _, g64 = pp.loss_and_grad(pp.bf16(params), norm, X, y, w, bf16_mode=False)
    assert np.linalg.norm(g16 - g64) <= 0.05 * np.linalg.norm(g64)


def test_zero_output_layer_gives_log2_loss():
    params, norm, X, y, w = _data(6, n=100)
    p = pp.unpack(params)
    p["w3"][:] = 0.0
    p["b3"][:] = 0.0
    loss, g = pp.loss_and_grad(pp.pack(p), norm, X, y, w)
    assert abs(loss - math.log(2.0)) < 1e-15
    assert abs(g[-1] - (w * (0.5 - y)).sum() / w.sum()) < 1e-15
    assert np.all(g[:pp.N_PARAM - 65] == 0.0)


# --------------------------------------------------------------------------- Adam
def test_adam_closed_forms():
    rng = np.random.default_rng(7)
    th = rng.normal(size=50)
    g = rng.normal(size=50)
    g[:5] = 0.0
    m = np.zeros(50)
    v = np.zeros(50)
    lr = 1e-2
    cur = th.copy()
    for t in range(1, 11):
        cur, m, v = pp.adam_step(cur, m, v, g, t, lr)
    # a constant gradient is followed at exactly lr * g / (|g| + eps) per step
    np.testing.assert_allclose(cur - th, -10 * lr * g / (np.abs(g) + 1e-8), rtol=1e-9, atol=1e-15)
    assert np.all(cur[:5] == th[:5])


def test_adam_matches_torch_optimizer():
    rng = np.random.default_rng(8)
    th0 = rng.normal(size=40)
    grads = rng.normal(size=(6, 40))
    t = torch.tensor(th0, dtype=torch.float64, requires_grad=True)
    opt = torch.optim.Adam([t], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    cur, m, v = th0.copy(), np.zeros(40), np.zeros(40)
    for s in range(6):
        opt.zero_grad()
        t.grad = torch.tensor(grads[s], dtype=torch.float64)
        opt.step()
        cur, m, v = pp.adam_step(cur, m, v, grads[s], s + 1, 3e-3)
    np.testing.assert_allclose(cur, t.detach().numpy(), rtol=1e-12, atol=1e-14)


def test_training_decreases_loss():
    params, norm, X, y, w = _data(9, n=300)
    y = (X[:, 0] < 6.0).astype(np.float64)  # learnable: close pairs associate
    m = np.zeros_like(params)
    v = np.zeros_like(params)
    l0, _ = pp.loss_and_grad(params, norm, X, y, w)
    for t in range(1, 61):
        _, g = pp.loss_and_grad(params, norm, X, y, w)
        params, m, v = pp.adam_step(params, m, v, g, t, 1e-2)
    l1, _ = pp.loss_and_grad(params, norm, X, y, w)
    assert l1 < 0.5 * l0
