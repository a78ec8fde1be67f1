"""GPU parity of the learned pair proposal: the HIP kernels, through the C ABI, against the
FP64 reference (oracle/proposal.py) and the oracle's update with the same pairs removed.

Tolerances:
* logits: the GPU sums in float32 and the reference in float64, and both round the same
  intermediate values to bfloat16.  A float32 sum that lands on the other side of a bfloat16
  rounding boundary moves one activation by one bfloat16 unit (2^-8 relative), which moves
  the logit by at most a few 1e-2; such flips are rare.  So 99 % of the logits agree to
  1e-4 * max(1, |s|) and all of them to 5e-2 * max(1, |s|).
* loss: 1e-4 relative; gradient: the flips of a few samples out of thousands move it by far
  less than 2e-3 in relative L2 norm.
* removal decisions: thresholds are placed where no reference logit lies within 0.05, so
  both sides remove the same pairs; the updates then agree at the update's bar (log-weights
  within 1e-4 * max(1, |ref|), same hypotheses).
* features, targets and weights: float32 arithmetic on values of order one, 1e-4 relative
  (targets and weights are ratios of posterior masses whose logarithms agree to 1e-4).
Pairs within 1e-4 * G of the gate may be gated differently in FP32 and FP64; instances that
hold one are left out of the comparisons that depend on them.
"""
import ctypes
import math

import numpy as np
import pytest

from oracle import proposal as pp
from oracle.oracle import Oracle, to_f32_state
from paper_2512_06230_amd import scenarios as sc
from tests import parity as pt

pytestmark = pytest.mark.gpu

BASE = dict(dt=1.0, q=1.0, sigma_z=1.0, p_survive=0.99, det_rate=1.47, clutter_density=2e-3,
            gate_d2=-2.0 * math.log(1e-4), birth_r_max=0.5, birth_rate=0.5, birth_sigma_v=2.0,
            birth_ru_max=0.5, birth_cluster_d=3.0, h_max=64, tau=0.0)
K_SCAN = 3


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _tracker(p):
    from paper_2512_06230_amd.glmb import Tracker
    return Tracker(p)


def _case(seed):
    rng = np.random.default_rng(900 + seed)
    st = sc.random_state(rng, n_lab=3 + seed % 4, n_hyp=2 + 3 * (seed % 3), side=20.0, versions=1 + seed % 2)
    z = sc.measurements_near(rng, st, 3 + seed % 3, 20.0, 1.0)
    return to_f32_state(st), z


def _net(seed, X):
    rng = np.random.default_rng(seed)
    params = sc.mlp_init(seed)
    parts = pp.unpack(params.astype(np.float64))
    parts["b1"] = rng.normal(0, 0.2, 64)
    parts["b2"] = rng.normal(0, 0.2, 64)
    parts["w3"] = parts["w3"] * 8.0  # spread the logits so that thresholds fall in clear gaps
    params = pp.pack(parts).astype(np.float32)
    norm = pp.feature_norm(X).astype(np.float32)
    return params, norm


def _ref_logits(params, norm, X):
    s, _ = pp.forward(params.astype(np.float64), norm.astype(np.float64), np.asarray(X, np.float32).astype(np.float64))
    return s


def _gap_threshold(logits, q, margin=0.05):
    """A logit threshold near quantile q with no logit within `margin` of it (or None)."""
    s = np.sort(np.asarray(logits))
    if len(s) < 2:
        return None
    target = np.quantile(s, q)
    mids = [(a + b) / 2 for a, b in zip(s[:-1], s[1:]) if b - a > 2 * margin]
    if not mids:
        return None
    return min(mids, key=lambda c: abs(c - target))


def _prob32(thr_logit):
    return float(np.float32(1.0 / (1.0 + math.exp(-thr_logit))))


# --------------------------------------------------------------------------- features, targets
@pytest.mark.parametrize("seed", range(5))
def test_pair_features_and_targets(torch_cuda, seed):
    st, z = _case(seed)
    p = BASE
    g = _tracker(p)
    g.import_state(st)
    feat, pair, y, w = [g.to_host(a) for a in g.pair_features(K_SCAN, z)]
    g.close()
    ref = pp.pair_features(st, z, K_SCAN, p["sigma_z"], p["gate_d2"])
    o = Oracle(p)
    o.import_state(st)
    o.update(K_SCAN, z)
    pr = o.pairs()
    yo, wo = pp.targets(pr)
    np.testing.assert_array_equal(ref["u"], pr["u"])
    near = pt.near_gate_instances(st, z, p["sigma_z"], p["gate_d2"])
    gk = {(int(a), int(b)): j for j, (a, b) in enumerate(pair)}
    ok = {(int(a), int(b)): j for j, (a, b) in enumerate(zip(ref["u"], ref["i"]))}
    assert len(gk) == len(pair)
    assert {k for k in gk if k[0] not in near} == {k for k in ok if k[0] not in near}
    # listed by instance, then detection
    for a, b in zip(pair[:-1], pair[1:]):
        assert a[0] != b[0] or a[1] < b[1]
    for key, j in ok.items():
        if key[0] in near:
            continue
        a, b = feat[gk[key]], ref["X"][j]
        assert abs(a[0] - b[0]) <= 1e-4 * max(1.0, abs(b[0])), ("d2", key, a, b)
        assert np.all(np.abs(a[1:3] - b[1:3]) <= 1e-4 * np.maximum(1.0, np.abs(b[1:3]))), ("nu", key, a, b)
        assert abs(a[3] - b[3]) <= 1e-5, ("r_label", key, a, b)
        assert a[4] == b[4] and a[5] == b[5], ("age / n_gate", key, a, b)
    if near:
        return  # posterior masses of hypotheses with a near-gate pair may differ
    for key, j in ok.items():
        gi = gk[key]
        assert abs(y[gi] - yo[j]) <= 1e-4 * max(1.0, yo[j]) + 1e-6, ("target", key, y[gi], yo[j])
        assert abs(w[gi] - wo[j]) <= 1e-4 * wo[j] + 1e-7, ("weight", key, w[gi], wo[j])


def test_pair_features_capacity_and_empty(torch_cuda):
    st, z = _case(1)
    g = _tracker(BASE)
    g.import_state(st)
    n = ctypes.c_int32()
    buf = g.to_device(np.zeros(16))
    st_code = g._L.glmb_pair_features(g._ctx, K_SCAN, ctypes.c_void_p(g.to_device(z).data_ptr()), z.shape[0], 1,
                                      ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(buf.data_ptr()),
                                      ctypes.c_void_p(buf.data_ptr()), ctypes.c_void_p(buf.data_ptr()),
                                      ctypes.byref(n))
    assert st_code == -2 and n.value > 1
    feat, pair, y, w = g.pair_features(K_SCAN, np.zeros((0, 2), np.float32))
    assert feat.shape == (0, 6) and pair.shape == (0, 2)
    g.import_state(sc.empty_state())
    feat, pair, y, w = g.pair_features(K_SCAN, z)
    assert feat.shape[0] == 0
    g.close()


# --------------------------------------------------------------------------- network kernels
def _train_data(seed, n):
    rng = np.random.default_rng(seed)
    X = np.column_stack([rng.uniform(0, 18, n), rng.normal(0, 2, n), rng.normal(0, 2, n),
                         rng.uniform(0, 1, n), rng.integers(0, 20, n), rng.integers(1, 12, n)]).astype(np.float32)
    y = (rng.uniform(0, 1, n) ** 3).astype(np.float32)
    w = rng.uniform(0.05, 1.0, n).astype(np.float32)
    return X, y, w


@pytest.mark.parametrize("n", [1, 64, 65, 3001])
def test_network_forward_and_gradient(torch_cuda, n):
    X, y, w = _train_data(n, n)
    params, norm = _net(n, X if n > 1 else np.vstack([X, X + 1]))
    g = _tracker(BASE)
    P = g.to_device(params)
    s = g.to_host(g.mlp_forward(P, norm, g.to_device(X)))
    grad, loss = g.mlp_grad(P, norm, g.to_device(X), g.to_device(y), g.to_device(w))
    grad, loss = g.to_host(grad), float(g.to_host(loss)[0])
    s_ref = _ref_logits(params, norm, X)
    err = np.abs(s - s_ref) / np.maximum(1.0, np.abs(s_ref))
    assert np.mean(err <= 1e-4) >= 0.99 and err.max() <= 5e-2, (np.sort(err)[-5:])
    l_ref, g_ref = pp.loss_and_grad(params.astype(np.float64), norm.astype(np.float64), X.astype(np.float64),
                                    y.astype(np.float64), w.astype(np.float64))
    assert abs(loss - l_ref) <= 1e-4 * abs(l_ref)
    assert np.linalg.norm(grad - g_ref) <= 2e-3 * np.linalg.norm(g_ref)
    # element by element, on the samples whose float32 evaluation takes the same bfloat16
    # rounding and ReLU decisions as the exact one
    keep = ~pp.rounding_sensitive(params, norm, X)
    assert keep.mean() >= 0.9, keep.mean()
    Xk, yk, wk = X[keep], y[keep], w[keep]
    sk = g.to_host(g.mlp_forward(P, norm, g.to_device(Xk)))
    assert np.all(np.abs(sk - s_ref[keep]) <= 1e-4 * np.maximum(1.0, np.abs(s_ref[keep])))
    grad_k, loss_k = g.mlp_grad(P, norm, g.to_device(Xk), g.to_device(yk), g.to_device(wk))
    grad_k, loss_k = g.to_host(grad_k), float(g.to_host(loss_k)[0])
    g.close()
    args = (params.astype(np.float64), norm.astype(np.float64), Xk.astype(np.float64), yk.astype(np.float64),
            wk.astype(np.float64))
    l_k, g_k = pp.loss_and_grad(*args)
    scale = pp.grad_abs_terms(*args)
    assert abs(loss_k - l_k) <= 1e-5 * abs(l_k) + 1e-7
    bad = np.abs(grad_k - g_k) > 3e-5 * scale + 1e-9
    assert not bad.any(), (np.nonzero(bad)[0][:10], grad_k[bad][:5], g_k[bad][:5], scale[bad][:5])


def test_adam_steps(torch_cuda):
    rng = np.random.default_rng(3)
    th = rng.normal(0, 0.3, 4673).astype(np.float32)
    gs = rng.normal(0, 1e-2, (5, 4673)).astype(np.float32)
    g = _tracker(BASE)
    P, Mm, V = g.to_device(th), g.to_device(np.zeros(4673)), g.to_device(np.zeros(4673))
    ref, m, v = th.astype(np.float64), np.zeros(4673), np.zeros(4673)
    for t in range(1, 6):
        G = g.to_device(gs[t - 1])
        g.mlp_adam(P, Mm, V, G, t, 1e-3, 0.9, 0.999, 1e-8)
        ref, m, v = pp.adam_step(ref, m, v, gs[t - 1].astype(np.float64), t, 1e-3)
    out = g.to_host(P)
    g.close()
    np.testing.assert_allclose(out, ref, rtol=1e-5, atol=1e-6)


# --------------------------------------------------------------------------- the learned update
def _oracle_update_with_skip(st, z, p, skip_u, skip_i):
    o = Oracle(p)
    o.import_state(st)
    o.set_skip(skip_u, skip_i)
    o.update(K_SCAN, z)
    return o


@pytest.mark.parametrize("seed", range(6))
def test_learned_update_matches_oracle_with_removed_pairs(torch_cuda, seed):
    st, z = _case(seed)
    ref = pp.pair_features(st, z, K_SCAN, BASE["sigma_z"], BASE["gate_d2"])
    if len(ref["u"]) < 2:
        pytest.skip("too few gated pairs")
    params, norm = _net(seed, ref["X"])
    s_ref = _ref_logits(params, norm, ref["X"])
    thr = _gap_threshold(s_ref, 0.4)
    assert thr is not None
    t = _prob32(thr)
    thr_o = math.log(t / (1.0 - t))
    drop = s_ref < thr_o
    near = pt.near_gate_instances(st, z, BASE["sigma_z"], BASE["gate_d2"])
    skip_parents = pt.parents_with(st, near)
    for K in (5, 64, 1000):
        p = dict(BASE, h_max=K)
        o = _oracle_update_with_skip(st, z, p, ref["u"][drop], ref["i"][drop])
        out_o = o.export_state()
        d_o = o.diag(len(st["hyp_logw"]))
        g = _tracker(p)
        g.import_state(st)
        g.set_proposal(g.to_device(params), norm, t, apply=True, measure=True)
        lost_g = g.proposal_lost(K_SCAN, z, [t])[0]
        g.update(K_SCAN, z)
        stats = g.stats()
        out_g = g.export_state()
        th_g = g.theta(len(out_g["hyp_logw"]), z.shape[0])
        d_g = g.diag(len(st["hyp_logw"]), z.shape[0])
        g.close()
        # the clutter probabilities behind the births (removed mass restored) and the births
        if not near:
            assert np.all(np.abs(d_g["ru"] - d_o["ru"]) <= 1e-4), (d_g["ru"], d_o["ru"])
            if np.all(np.abs(d_o["ru"] - p["birth_ru_max"]) > 1e-3):
                assert out_g["birth_lab"].tolist() == out_o["birth_lab"].tolist()
                np.testing.assert_allclose(out_g["birth_m"], out_o["birth_m"], rtol=1e-4, atol=1e-4)
                np.testing.assert_allclose(out_g["birth_r"], out_o["birth_r"], rtol=1e-4, atol=1e-6)
        if not near:
            assert stats["pairs_removed"] == int(drop.sum())
            assert abs(lost_g - d_o["lost"]) <= 1e-5 + 1e-3 * d_o["lost"], (lost_g, d_o["lost"])
            assert abs(stats["lost_mass"] - d_o["lost"]) <= 1e-5 + 1e-3 * d_o["lost"]
        ids_o = pt.update_ids(out_o, out_o["theta"])
        ids_g = pt.update_ids(out_g, th_g)
        pt.compare_sets(ids_o, out_o["hyp_logw"], ids_g, out_g["hyp_logw"], skip_parents)
        pt.compare_densities(out_o, ids_o, out_g, ids_g, skip_parents)
        # no retained hypothesis uses a removed pair
        removed = set(zip(ref["u"][drop].tolist(), ref["i"][drop].tolist()))
        for row in th_g:
            assert not any((int(u), i) in removed for i, u in enumerate(row) if u >= 0)


@pytest.mark.parametrize("seed", range(3))
def test_lost_mass_at_several_thresholds(torch_cuda, seed):
    st, z = _case(10 + seed)
    if pt.near_gate_instances(st, z, BASE["sigma_z"], BASE["gate_d2"]):
        pytest.skip("a pair sits at the gate")
    ref = pp.pair_features(st, z, K_SCAN, BASE["sigma_z"], BASE["gate_d2"])
    params, norm = _net(50 + seed, ref["X"])
    s_ref = _ref_logits(params, norm, ref["X"])
    ts = []
    for q in (0.1, 0.3, 0.5, 0.7, 0.9):
        thr = _gap_threshold(s_ref, q)
        if thr is not None:
            ts.append(_prob32(thr))
    ts = sorted(set(ts))
    g = _tracker(BASE)
    g.import_state(st)
    g.set_proposal(g.to_device(params), norm, apply=False)
    lost = g.proposal_lost(K_SCAN, z, ts)
    g.close()
    prev = -1.0
    for t, L in zip(ts, lost):
        thr_o = math.log(t / (1.0 - t))
        drop = s_ref < thr_o
        o = _oracle_update_with_skip(st, z, BASE, ref["u"][drop], ref["i"][drop])
        Lo = o.diag(len(st["hyp_logw"]))["lost"]
        assert abs(L - Lo) <= 1e-5 + 1e-3 * Lo, (t, L, Lo)
        assert L >= prev - 1e-6  # more removed pairs never lose less mass
        prev = L


def test_disabled_proposal_is_the_plain_update(torch_cuda):
    st, z = _case(4)
    outs = []
    for mode in ("plain", "disabled"):
        g = _tracker(BASE)
        g.import_state(st)
        if mode == "disabled":
            ref = pp.pair_features(st, z, K_SCAN, BASE["sigma_z"], BASE["gate_d2"])
            params, norm = _net(1, ref["X"])
            g.set_proposal(g.to_device(params), norm, 0.9)
            g.set_proposal(None, None, 0.5)
        g.update(K_SCAN, z)
        outs.append(g.export_state())
        assert g.stats()["pairs_removed"] == 0
        g.close()
    np.testing.assert_array_equal(outs[0]["hyp_logw"], outs[1]["hyp_logw"])
    np.testing.assert_array_equal(outs[0]["inst_m"], outs[1]["inst_m"])


def test_proposal_argument_errors(torch_cuda):
    from paper_2512_06230_amd.glmb import GlmbError
    st, z = _case(2)
    g = _tracker(BASE)
    g.import_state(st)
    params = g.to_device(np.zeros(4673))
    with pytest.raises(GlmbError):
        g.set_proposal(params, np.ones(12), 1.5)
    with pytest.raises(GlmbError):
        g.set_proposal(params, np.zeros(12), 0.5)  # zero standard deviations
    with pytest.raises(GlmbError):
        g.proposal_lost(K_SCAN, z, [0.5])  # no parameters yet
    g.set_proposal(params, np.ones(12), 0.5)
    with pytest.raises(GlmbError):
        g.proposal_lost(K_SCAN, z, [0.5] * 17)
    g.close()


def test_learned_births_equal_plain_births_on_one_hypothesis(torch_cuda):
    """From a state with a single hypothesis, restoring the removed pairs' mass makes the learned
    update's clutter probabilities those of the plain update, so both seed the same births
    (the packaged network at its threshold, on the 500-object scene it was trained for)."""
    torch = torch_cuda
    from paper_2512_06230_amd.proposal import Proposal
    import os
    prop = Proposal.load(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                      "paper_2512_06230_amd", "proposal_n500.npz"))
    spec = sc.spec_for("c3:500")
    scene = sc.make_scene(spec, n_steps=2)
    p = sc.filter_params(spec, 10000, 0.0)
    st = sc.warm_start_state(scene)
    z = torch.as_tensor(scene.meas[0], device="cuda")
    outs = []
    for learned in (False, True):
        g = _tracker(p)
        g.import_state(st)
        if learned:
            g.set_proposal(torch.as_tensor(prop.params, device="cuda"), prop.norm, prop.threshold, apply=True)
        g.update(0, z)
        s = g.stats()
        outs.append((g.export_state(), g.diag(1, int(z.shape[0]))["ru"], s))
        g.close()
    (o_p, ru_p, s_p), (o_l, ru_l, s_l) = outs
    assert s_l["pairs_removed"] > 0.2 * s_l["gated_pairs"], (s_l["pairs_removed"], s_l["gated_pairs"])
    assert np.max(np.abs(ru_l - ru_p)) <= 1e-4, np.max(np.abs(ru_l - ru_p))
    if np.all(np.abs(ru_p - p["birth_ru_max"]) > 1e-3):
        assert o_l["birth_lab"].tolist() == o_p["birth_lab"].tolist()
        np.testing.assert_allclose(o_l["birth_m"], o_p["birth_m"], rtol=1e-4, atol=1e-4)
        np.testing.assert_allclose(o_l["birth_r"], o_p["birth_r"], rtol=1e-4, atol=1e-6)


@pytest.mark.slow
def test_learned_proposal_gains_over_a_tightened_gate(torch_cuda):
    """What the trained network gains over the method without it, at equal lost mass: on a
    held-out 500-object predicted state, the tightest Mahalanobis gate whose retained-set lost
    mass stays <= 1e-3 keeps more pairs than the network at its threshold (whose lost mass obeys
    the same bound)."""
    import os
    import torch
    from paper_2512_06230_amd.glmb import Tracker
    from paper_2512_06230_amd.proposal import Proposal, gate_gain
    prop = Proposal.load(os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                                      "paper_2512_06230_amd", "proposal_n500.npz"))
    spec = sc.spec_for("c3:500", clutter_mean=100.0, seed=2500)
    scene = sc.make_scene(spec, n_steps=4)
    p = sc.filter_params(spec, 10000, 0.0)
    g = Tracker(p)
    g.import_state(sc.warm_start_state(scene))
    for k in range(3):
        g.predict(k)
        g.update(k, torch.as_tensor(scene.meas[k], device="cuda"))
        g.truncate(10000, 0.0)
    g.predict(3)
    st = g.export_state()
    g.close()
    r = gate_gain(p, st, 3, torch.as_tensor(scene.meas[3], device="cuda"), prop)
    print(r, flush=True)
    assert r["lost_mlp"] <= 1e-3 and r["lost_tight_gate"] <= 1e-3
    assert r["pairs_mlp"] < r["pairs_tight_gate"] <= r["pairs_plain"]
