"""Pins of the oracle's sampled children (the paper's own hypothesis generator, Sec. 3:
per predicted hypothesis H_up association maps, every measurement drawn independently from
the normalised row of the compatibility matrix over clutter and the hypothesis' tracks; the
distinct maps kept with their exact weights, then tau and H_max).  CPU only.

* the counter-based generator: uniformity (chi-square), distinct outputs for distinct
  counters, dependence on the key;
* the categorical draw: frequencies over many seeds against the normalised rows computed
  from scipy's normal density and the clutter density (chi-square);
* the kept set: every sampled child is a child of the brute-force enumeration, with the
  brute force's weight (renormalised over the kept set); with draws enough to find every
  child of non-negligible proposal probability, the sampled update equals the exact one;
* bookkeeping: draws = H x H_up, distinct maps <= draws, weights normalised, a different
  seed changes the draws, the same seed repeats them.
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


def test_philox_uniforms_are_uniform_and_distinct():
    n = 1 << 15
    u = np.array([orc.philox_uniform(12345, i, 7, 3, 1) for i in range(n)])
    assert np.all((u >= 0.0) & (u < 1.0))
    counts, _ = np.histogram(u, bins=64, range=(0.0, 1.0))
    chi2 = ((counts - n / 64) ** 2 / (n / 64)).sum()
    assert stats.chi2.sf(chi2, 63) > 1e-4, chi2
    # the 128-bit blocks of distinct counters are distinct (the generator is a bijection)
    blocks = {tuple(orc.philox4x32_10([i, 5, 0, 1], [9, 0]).tolist()) for i in range(4096)}
    assert len(blocks) == 4096
    # every output bit flips with probability 1/2 when the key changes by one bit
    a = np.array([orc.philox4x32_10([i, 0, 0, 0], [1, 0]) for i in range(512)], np.uint64)
    b = np.array([orc.philox4x32_10([i, 0, 0, 0], [3, 0]) for i in range(512)], np.uint64)
    flips = np.unpackbits((a ^ b).astype(np.uint32).view(np.uint8)).mean()
    assert abs(flips - 0.5) < 0.02, flips


def _one_cell_state():
    """One hypothesis with three tracks near the origin and one detection between them."""
    st = dict(inst_lab=np.array([[0, 0], [0, 1], [0, 2]], np.int32),
              inst_m=np.array([[0.0, 0.0, 0, 0], [1.5, 0.0, 0, 0], [0.0, 2.0, 0, 0]]),
              inst_P=np.tile(np.diag([0.5, 0.5, 1.0, 1.0]).reshape(1, 16), (3, 1)),
              hyp_logw=np.array([0.0]), hyp_off=np.array([0, 3], np.int32), hyp_idx=np.array([0, 1, 2], np.int32),
              birth_lab=np.zeros((0, 2), np.int32), birth_m=np.zeros((0, 4)), birth_P=np.zeros((0, 16)),
              birth_r=np.zeros(0))
    z = np.array([[0.6, 0.7]], np.float32)
    return st, z


def test_categorical_draw_follows_the_normalised_row():
    st, z = _one_cell_state()
    p = dict(BASE, clutter_density=0.02)
    zz = z.astype(np.float64)[0]
    w = [p["clutter_density"]]  # options in key order: clutter, then tracks by label
    for u in range(3):
        S = st["inst_P"][u].reshape(4, 4)[:2, :2] + p["sigma_z"] ** 2 * np.eye(2)
        w.append(p["det_rate"] * stats.multivariate_normal(st["inst_m"][u][:2], S).pdf(zz))
    prob = np.array(w) / np.sum(w)
    n = 4000
    counts = np.zeros(4)
    for seed in range(n):
        o = Oracle(p)
        o.import_state(st)
        o.set_sampling(1, seed)
        o.update(0, z)
        th = int(o.export_state()["theta"][0][0])
        counts[th + 1] += 1
    chi2 = ((counts - n * prob) ** 2 / (n * prob)).sum()
    assert stats.chi2.sf(chi2, 3) > 1e-4, (counts / n, prob)


def _bf_children(st, z, p):
    ref = bf.update(st, z, p, 10 ** 6)
    return {(c["parent"], tuple(int(x) for x in c["theta"])): c["logw"] for c in ref["children"]}, ref


@pytest.mark.parametrize("seed", range(8))
def test_sampled_children_are_children_with_their_exact_weights(seed):
    rng = np.random.default_rng(600 + seed)
    st = sc.random_state(rng, n_lab=3, n_hyp=3, side=10.0, versions=1, p_present=0.8)
    z = sc.measurements_near(rng, st, 1, 10.0, 1.0)[:4]
    h_up, K = 20, 1000
    p = dict(BASE, h_max=K)
    o = Oracle(p)
    o.import_state(st)
    o.set_sampling(h_up, 99 + seed)
    o.update(0, z)
    out = o.export_state()
    draws, uniq, _ = o.sample_stats()
    H = len(st["hyp_logw"])
    assert draws == H * h_up and len(out["hyp_logw"]) == uniq <= draws
    assert abs(np.exp(out["hyp_logw"]).sum() - 1.0) < 1e-12
    allc, _ = _bf_children(st, z, p)
    keys = [(int(a), tuple(int(x) for x in t)) for a, t in zip(out["hyp_parent"], out["theta"])]
    assert len(set(keys)) == len(keys)
    ref = np.array([allc[k] for k in keys])   # KeyError: not a child
    ref = ref - np.logaddexp.reduce(ref)
    np.testing.assert_allclose(out["hyp_logw"], ref, atol=1e-9)
    assert np.all(np.diff(out["hyp_logw"]) <= 1e-12)  # rank order
    # H_max cut: the best K of the distinct maps
    o2 = Oracle(dict(p, h_max=5))
    o2.import_state(st)
    o2.set_sampling(h_up, 99 + seed)
    o2.update(0, z)
    k2 = [(int(a), tuple(int(x) for x in t)) for a, t in zip(o2.export_state()["hyp_parent"],
                                                            o2.export_state()["theta"])]
    assert k2 == keys[:5]


def test_many_draws_find_the_exact_update():
    """With every child's proposal probability far above 1 / H_up, the sampled set is the
    whole child set, and the update equals the exact (brute-force) one."""
    found = 0
    rng = np.random.default_rng(5)
    for trial in range(40):
        st = sc.random_state(rng, n_lab=2, n_hyp=2, side=4.0, versions=1, p_present=1.0)
        z = sc.measurements_near(rng, st, 0, 4.0, 1.0)[:2]
        p = dict(BASE, clutter_density=0.05, h_max=1000)
        allc, ref = _bf_children(st, z, p)
        # proposal probability of every child: product of its cells' normalised entries
        lw = {}
        for (h, th), v in allc.items():
            lw.setdefault(h, []).append(v)
        ok = True
        for h in range(len(st["hyp_logw"])):
            tracks = st["hyp_idx"][st["hyp_off"][h]:st["hyp_off"][h + 1]]
            for i in range(z.shape[0]):
                w = [p["clutter_density"]] + [p["det_rate"] * ref["dens"][u, i] for u in tracks if ref["gated"][u, i]]
                if min(w) / sum(w) < 0.15:
                    ok = False
        if not ok:
            continue
        o = Oracle(p)
        o.import_state(st)
        o.set_sampling(400, 7 + trial)
        o.update(0, z)
        out = o.export_state()
        keys = [(int(a), tuple(int(x) for x in t)) for a, t in zip(out["hyp_parent"], out["theta"])]
        assert set(keys) == set(allc), trial
        np.testing.assert_allclose(out["hyp_logw"], [allc[k] for k in keys], atol=1e-9)
        found += 1
        if found == 4:
            break
    assert found == 4


def test_seed_changes_and_repeats_the_draws():
    rng = np.random.default_rng(11)
    st = sc.random_state(rng, n_lab=4, n_hyp=4, side=10.0, versions=1, p_present=0.9)
    z = sc.measurements_near(rng, st, 2, 10.0, 1.0)
    res = []
    for seed in (1, 1, 2):
        o = Oracle(dict(BASE, h_max=500))
        o.import_state(st)
        o.set_sampling(8, seed)
        o.update(0, z)
        out = o.export_state()
        res.append([(int(a), tuple(int(x) for x in t)) for a, t in zip(out["hyp_parent"], out["theta"])])
    assert res[0] == res[1]
    assert res[0] != res[2]


# --------------------------------------------------------------------------- sampled prediction
def _pred_state(n_lab, n_hyp, rng, r_birth=()):
    st = sc.random_state(rng, n_lab=n_lab, n_hyp=n_hyp, side=20.0, versions=1, p_present=1.0)
    nb = len(r_birth)
    st["birth_lab"] = np.array([[99, b] for b in range(nb)], np.int32).reshape(-1, 2)
    st["birth_m"] = rng.uniform(0, 20, (nb, 4))
    st["birth_P"] = np.tile(np.eye(4).reshape(1, 16), (nb, 1))
    st["birth_r"] = np.asarray(r_birth, np.float64)
    return st


def test_sampled_prediction_frequencies():
    """One hypothesis, one draw per seed: every track survives with frequency p_S and the
    pending birth joins with frequency r_b (binomial tests)."""
    rng = np.random.default_rng(12)
    st = _pred_state(3, 1, rng, r_birth=[0.3])
    p = dict(BASE, p_survive=0.7, h_max=10)
    n = 3000
    cnt = np.zeros(4)
    for seed in range(n):
        o = Oracle(p)
        o.import_state(st)
        o.set_sampling(1, seed)
        o.predict(0)
        out = o.export_state()
        src = set(out["inst_src"][out["hyp_idx"][out["hyp_off"][0]:out["hyp_off"][1]]].tolist())
        for j in range(3):
            cnt[j] += j in src
        cnt[3] += 3 in src  # the birth is input instance n_inst + 0
    for j, pr in enumerate([0.7, 0.7, 0.7, 0.3]):
        assert stats.binomtest(int(cnt[j]), n, pr).pvalue > 1e-4, (j, cnt[j] / n, pr)


@pytest.mark.parametrize("seed", range(4))
def test_sampled_prediction_with_many_draws_is_the_exact_one(seed):
    """With every survive/die x include/exclude outcome drawn (few dimensions, many draws), the
    sampled prediction keeps them all and equals the brute-force prediction."""
    rng = np.random.default_rng(40 + seed)
    st = _pred_state(2 + seed % 2, 1 + seed % 3, rng, r_birth=[0.4])
    p = dict(BASE, p_survive=0.6, h_max=1000)
    o = Oracle(p)
    o.import_state(st)
    o.set_sampling(600, 5 + seed)
    o.predict(0)
    out = o.export_state()
    ref, _ = bf.predict(st, p, 1000)
    got = {}
    for h in range(len(out["hyp_logw"])):
        src = tuple(sorted(int(x) for x in out["inst_src"][out["hyp_idx"][out["hyp_off"][h]:out["hyp_off"][h + 1]]]))
        got[src] = out["hyp_logw"][h]
    want = {c["src"]: c["logw"] for c in ref}
    assert set(got) == set(want)
    for k in want:
        assert abs(got[k] - want[k]) < 1e-9
