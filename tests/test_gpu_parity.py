"""GPU parity: the HIP library (through its C ABI) against the FP64 oracle on the same
seeded inputs.  Both sides start every compared stage from the same FP32-rounded state."""
import math

import numpy as np
import pytest

from oracle.oracle import Oracle, to_f32_state
from paper_2512_06230_amd import scenarios as sc
from tests import parity as pt

pytestmark = pytest.mark.gpu

BASE = dict(dt=1.0, q=1.0, sigma_z=1.0, p_survive=0.99, det_rate=1.47, clutter_density=2e-3,
            gate_d2=-2.0 * math.log(1e-4), birth_r_max=0.5, birth_rate=0.5, birth_sigma_v=2.0,
            birth_ru_max=0.5, birth_cluster_d=3.0, h_max=64, tau=0.0)


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _tracker(p):
    from paper_2512_06230_amd.glmb import Tracker
    return Tracker(p)


def _update_both(state, z, p, k=0):
    st = to_f32_state(state)
    o = Oracle(p)
    o.import_state(st)
    o.update(k, z)
    out_o = o.export_state()
    d_o = o.diag(len(st["hyp_logw"]))
    g = _tracker(p)
    g.import_state(st)
    near = pt.near_gate_instances(st, z, p["sigma_z"], p["gate_d2"])
    if near:
        # keep only the instances whose gate decisions really differ between FP32 and FP64
        pr = o.pairs()
        ref = set(zip(pr["u"].tolist(), pr["i"].tolist()))
        _, pair, _, _ = g.pair_features(k, z)
        got = set(map(tuple, g.to_host(pair).tolist()))
        near = {u for u, _ in ref ^ got}
    g.near = near
    g.update(k, z)
    out_g = g.export_state()
    M = np.asarray(z).reshape(-1, 2).shape[0]
    th_g = g.theta(len(out_g["hyp_logw"]), M)
    d_g = g.diag(len(st["hyp_logw"]), M)
    stats = g.stats()
    stats["near"] = g.near
    g.close()
    return st, out_o, d_o, out_g, th_g, d_g, stats


def check_update(state, z, p, k=0, full_density=True):
    st, out_o, d_o, out_g, th_g, d_g, stats = _update_both(state, z, p, k)
    skip = pt.parents_with(st, stats["near"])
    keep = np.array([h not in skip for h in range(len(st["hyp_logw"]))])
    if keep.any():
        assert np.all(np.abs(d_g["best"][keep] - d_o["best"][keep]) <= pt.tol(d_o["best"][keep])), "best child"
        assert np.all(np.abs(d_g["logpi"][keep] - d_o["logpi"][keep]) <= pt.tol(d_o["logpi"][keep])), "log pi"
    if not skip:
        assert np.all(np.abs(d_g["ru"] - d_o["ru"]) <= 1e-4), "clutter probabilities"
    ids_o = pt.update_ids(out_o, out_o["theta"])
    ids_g = pt.update_ids(out_g, th_g)
    matched = pt.compare_sets(ids_o, out_o["hyp_logw"], ids_g, out_g["hyp_logw"], skip)
    nd = pt.compare_densities(out_o, ids_o, out_g, ids_g, skip, limit=None if full_density else 200)
    stats["densities_compared"] = nd
    stats["unmatched"] = len(ids_o) - matched
    # births for the next scan (skip when a clutter probability sits at the seed threshold)
    if not skip and np.all(np.abs(d_o["ru"] - p["birth_ru_max"]) > 1e-3):
        assert out_g["birth_lab"].tolist() == out_o["birth_lab"].tolist()
        np.testing.assert_allclose(out_g["birth_m"], out_o["birth_m"], rtol=1e-4, atol=1e-4)
        np.testing.assert_allclose(out_g["birth_P"], out_o["birth_P"], rtol=1e-4, atol=1e-4)
        np.testing.assert_allclose(out_g["birth_r"], out_o["birth_r"], rtol=1e-4, atol=1e-6)
    return matched, stats, out_o, out_g


def check_predict(state, p, k=0):
    st = to_f32_state(state)
    o = Oracle(p)
    o.import_state(st)
    o.predict(k)
    out_o = o.export_state()
    g = _tracker(p)
    g.import_state(st)
    g.predict(k)
    out_g = g.export_state()
    g.close()
    ids_o = pt.predict_ids(out_o)
    ids_g = pt.predict_ids(out_g)
    pt.compare_sets(ids_o, out_o["hyp_logw"], ids_g, out_g["hyp_logw"])
    # predicted moments of every instance, matched by source index
    mo = {int(s): (m, P) for s, m, P in zip(out_o["inst_src"], out_o["inst_m"], out_o["inst_P"])}
    for s, m, P in zip(out_g["inst_src"], out_g["inst_m"], out_g["inst_P"]):
        m0, P0 = mo[int(s)]
        assert np.all(np.abs(m - m0) <= pt.tol(m0)) and np.all(np.abs(P - P0) <= pt.tol(P0))
    return out_o, out_g


# --------------------------------------------------------------------------- tiny / random states
@pytest.mark.parametrize("seed", range(10))
def test_update_random_states(torch_cuda, seed):
    rng = np.random.default_rng(500 + seed)
    st = sc.random_state(rng, n_lab=2 + seed % 5, n_hyp=1 + 3 * (seed % 4), side=20.0, versions=1 + seed % 3)
    z = sc.measurements_near(rng, st, 2 + seed % 4, 20.0, 1.0)
    for K in (1, 5, 64, 1000):
        check_update(st, z, dict(BASE, h_max=K))


def test_update_tau(torch_cuda):
    rng = np.random.default_rng(77)
    st = sc.random_state(rng, n_lab=4, n_hyp=5, side=20.0, versions=2)
    z = sc.measurements_near(rng, st, 3, 20.0, 1.0)
    for tau in (1e-4, 1e-2, 0.3):
        _, _, out_o, out_g = check_update(st, z, dict(BASE, h_max=200, tau=tau))
        assert len(out_g["hyp_logw"]) == len(out_o["hyp_logw"])


@pytest.mark.parametrize("seed", range(6))
def test_predict_random_states(torch_cuda, seed):
    rng = np.random.default_rng(600 + seed)
    st = sc.random_state(rng, n_lab=3 + seed, n_hyp=1 + 2 * seed, side=30.0, versions=1 + seed % 2)
    nb = seed % 4
    st["birth_lab"] = np.array([[9, b] for b in range(nb)], np.int32).reshape(-1, 2)
    st["birth_m"] = rng.uniform(0, 10, (nb, 4))
    st["birth_P"] = np.tile(np.diag([1.0, 1.0, 4.0, 4.0]).reshape(16), (nb, 1))
    st["birth_r"] = rng.uniform(0.05, 0.6, nb)
    for ps in (0.99, 0.6):
        for K in (1, 3, 17, 500):
            check_predict(st, dict(BASE, h_max=K, p_survive=ps), k=3)


# --------------------------------------------------------------------------- scenes (per stage)
def _scene_parity(name, steps, K, tau, warm, seed=0, every=1):
    spec = sc.spec_for(name, seed=seed)
    scene = sc.make_scene(spec, n_steps=steps)
    p = sc.filter_params(spec, K, tau)
    o = Oracle(p)
    o.import_state(sc.warm_start_state(scene) if warm else sc.empty_state())
    total = 0
    for k in range(steps):
        prior = to_f32_state(o.export_state())
        if k % every == 0:
            check_predict(prior, p, k)
        o.import_state(prior)
        o.predict(k)
        pred = to_f32_state(o.export_state())
        if k % every == 0:
            m, _, _, _ = check_update(pred, scene.meas[k], p, k)
            total += m
        o.import_state(pred)
        o.update(k, scene.meas[k])
    return total


def test_scene_c1(torch_cuda):
    assert _scene_parity("c1", 20, 64, 1e-5, warm=False) > 0


def test_scene_c2(torch_cuda):
    assert _scene_parity("c2", 8, 1024, 1e-5, warm=True) > 0


def test_full_size_step(torch_cuda):
    """The benchmarked workload (N=500 objects, H_max=1e4, clutter 100): one prediction and one
    update from a state the oracle produced, compared hypothesis by hypothesis (the track
    densities of every hypothesis found on both sides)."""
    spec = sc.spec_for("c5")
    scene = sc.make_scene(spec, n_steps=2)
    p = sc.filter_params(spec, 10000, 0.0)
    o = Oracle(p)
    o.import_state(sc.warm_start_state(scene))
    o.predict(0)
    o.update(0, scene.meas[0])
    post = to_f32_state(o.export_state())
    check_predict(post, p, 1)
    o.import_state(post)
    o.predict(1)
    pred = to_f32_state(o.export_state())
    matched, stats, out_o, out_g = check_update(pred, scene.meas[1], p, 1)
    print("full size: %d of %d hypotheses matched (%d only near the cut), densities of %d compared"
          % (matched, len(out_o["hyp_logw"]), stats["unmatched"], stats["densities_compared"]), flush=True)
    assert len(out_g["hyp_logw"]) == 10000 and matched > 9000, matched
    assert stats["densities_compared"] == matched


@pytest.mark.slow
def test_scene_c3_n100(torch_cuda):
    assert _scene_parity("c3:100", 3, 1000, 0.0, warm=True) > 0


@pytest.mark.slow
@pytest.mark.parametrize("n_obj,h_max", [(250, 10000), (100, 100000)])
def test_sweep_points_one_step(torch_cuda, n_obj, h_max):
    """Points of the scaling sweep (N objects, clutter 0.2 N, 100x100 m): one prediction and one
    update from a state the oracle produced, compared hypothesis by hypothesis."""
    spec = sc.spec_for("c3:%d" % n_obj)
    scene = sc.make_scene(spec, n_steps=2)
    p = sc.filter_params(spec, h_max, 0.0)
    o = Oracle(p)
    o.import_state(sc.warm_start_state(scene))
    o.predict(0)
    o.update(0, scene.meas[0])
    post = to_f32_state(o.export_state())
    check_predict(post, p, 1)
    o.import_state(post)
    o.predict(1)
    pred = to_f32_state(o.export_state())
    matched, stats, out_o, out_g = check_update(pred, scene.meas[1], p, 1)
    print("N=%d H_max=%d: %d of %d matched, densities of %d compared, search form %d"
          % (n_obj, h_max, matched, len(out_o["hyp_logw"]), stats["densities_compared"], stats["search_form"]),
          flush=True)
    assert len(out_g["hyp_logw"]) == h_max and matched > 0.9 * h_max


# --------------------------------------------------------------------------- edge cases
def test_no_detections(torch_cuda):
    rng = np.random.default_rng(3)
    st = sc.random_state(rng, n_lab=3, n_hyp=4, side=20.0)
    check_update(st, np.zeros((0, 2), np.float32), dict(BASE, h_max=10))


def test_empty_state(torch_cuda):
    z = np.array([[1.0, 2.0], [1.5, 2.2], [40.0, 40.0]], np.float32)
    check_update(sc.empty_state(), z, dict(BASE, h_max=10))
    check_predict(sc.empty_state(), dict(BASE, h_max=10))


def test_wide_gate(torch_cuda):
    """A lost track with a very wide gate: more than 128 detections are compatible with its label."""
    rng = np.random.default_rng(12)
    st = sc.random_state(rng, n_lab=6, n_hyp=5, side=60.0, versions=2)
    st["inst_P"][0] = np.diag([300.0, 300.0, 20.0, 20.0]).reshape(16)
    z = sc.measurements_near(rng, st, 260, 60.0, 1.0)
    for K in (16, 300):
        check_update(st, z, dict(BASE, h_max=K, clutter_density=0.05))


def test_crowded_cell(torch_cuda):
    """Ninety tracks of one hypothesis compete for every detection (cells with 91 options)."""
    rng = np.random.default_rng(31)
    st = sc.random_state(rng, n_lab=90, n_hyp=3, side=4.0, versions=1, p_present=1.0)
    z = sc.measurements_near(rng, st, 0, 4.0, 1.0)[:6]
    for K in (8, 200):
        check_update(st, z, dict(BASE, h_max=K))


def test_small_node_store(torch_cuda):
    """A node store too small for the one-workgroup search: the multi-kernel search with
    threshold raising and compaction must reach the same hypotheses."""
    rng = np.random.default_rng(21)
    st = sc.random_state(rng, n_lab=6, n_hyp=10, side=20.0, versions=2)
    z = sc.measurements_near(rng, st, 4, 20.0, 1.0)
    for cap in (90, 110, 0):  # 90 and 110 overflow the one-workgroup search; 0 = default store
        check_update(st, z, dict(BASE, h_max=64, cap_nodes=cap))


def test_small_node_store_multi_kernel(torch_cuda, monkeypatch):
    """The same small stores on the host-driven multi-kernel levels (the whole-GPU form that
    batched scenes use): threshold raising and node compaction reach the same hypotheses."""
    monkeypatch.setenv("GLMB_SEARCH_FORM", "multi")
    rng = np.random.default_rng(21)
    st = sc.random_state(rng, n_lab=6, n_hyp=10, side=20.0, versions=2)
    z = sc.measurements_near(rng, st, 4, 20.0, 1.0)
    for cap in (90, 110, 0):
        _, stats, _, _ = check_update(st, z, dict(BASE, h_max=64, cap_nodes=cap))
        assert stats["search_form"] == 2, stats


@pytest.mark.parametrize("mode", ["0", "1", "2"])
def test_search_group_bits(torch_cuda, monkeypatch, mode):
    """The one-workgroup search's three ways of rejecting a second pick in one group: item tables
    in global memory with hashed bits and a walk up the picks (0), tables in LDS with hashed bits
    (1), and exact bits when the items carry at most 64 groups (2).  Updates and predictions of
    random states under each against the oracle."""
    monkeypatch.setenv("GLMB_SEARCH_GROUP_BITS", mode)
    for seed in range(4):
        rng = np.random.default_rng(900 + seed)
        st = sc.random_state(rng, n_lab=3 + seed, n_hyp=4 + 3 * seed, side=20.0, versions=2)
        z = sc.measurements_near(rng, st, 3 + seed, 20.0, 1.0)
        for K in (5, 64, 1000):
            check_update(st, z, dict(BASE, h_max=K))
        check_predict(st, dict(BASE, h_max=200))


def test_refine_retry(torch_cuda, monkeypatch, capfd):
    """The update's counting bound raised on purpose above the K-th best child
    (GLMB_DP_BOUND_INFLATE): its search keeps fewer than K children, the update searches again
    from the caller's bound, and the result is still the oracle's."""
    monkeypatch.setenv("GLMB_DP_BOUND_INFLATE", "0.9")
    monkeypatch.setenv("GLMB_TRACE", "1")
    retries = 0
    for seed in range(4):
        rng = np.random.default_rng(700 + seed)
        st = sc.random_state(rng, n_lab=4 + seed, n_hyp=6 + 2 * seed, side=20.0, versions=2)
        z = sc.measurements_near(rng, st, 4 + seed, 20.0, 1.0)
        for K in (5, 20):
            check_update(st, z, dict(BASE, h_max=K))
            retries += capfd.readouterr().err.count("update.refine_retry")
    assert retries > 0


def test_hmax_one(torch_cuda):
    rng = np.random.default_rng(4)
    st = sc.random_state(rng, n_lab=5, n_hyp=6, side=20.0)
    z = sc.measurements_near(rng, st, 2, 20.0, 1.0)
    check_update(st, z, dict(BASE, h_max=1))


def test_nan_detection_is_an_argument_error(torch_cuda):
    from paper_2512_06230_amd.glmb import GlmbError, GLMB_E_ARG
    g = _tracker(BASE)
    z = np.array([[1.0, float("nan")]], np.float32)
    with pytest.raises(GlmbError) as e:
        g.update(0, z)
    assert e.value.status == GLMB_E_ARG
    g.close()


def test_deterministic(torch_cuda):
    spec = sc.spec_for("c1")
    scene = sc.make_scene(spec, n_steps=6)
    p = sc.filter_params(spec, 64, 1e-5)
    runs = []
    for _ in range(2):
        g = _tracker(p)
        for k in range(6):
            g.predict(k)
            g.update(k, scene.meas[k])
        runs.append(g.export_state())
        g.close()
    for key in ("hyp_logw", "inst_m", "inst_P", "hyp_idx"):
        assert np.array_equal(runs[0][key], runs[1][key]), key


def test_truncate_and_estimate(torch_cuda):
    spec = sc.spec_for("c1")
    scene = sc.make_scene(spec, n_steps=8)
    p = sc.filter_params(spec, 64, 0.0)
    o = Oracle(p)
    o.import_state(sc.empty_state())
    for k in range(8):
        o.predict(k)
        o.update(k, scene.meas[k])
    st = to_f32_state(o.export_state())
    for hmax, tau in ((64, 0.0), (10, 0.0), (30, 1e-3), (1, 0.0)):
        oo = Oracle(p)
        oo.import_state(st)
        oo.truncate(hmax, tau)
        g = _tracker(p)
        g.import_state(st)
        g.truncate(hmax, tau)
        a, b = oo.export_state(), g.export_state()
        assert len(a["hyp_logw"]) == len(b["hyp_logw"])
        assert np.all(np.abs(b["hyp_logw"] - a["hyp_logw"]) <= pt.tol(a["hyp_logw"]))
        la, ma, _ = oo.estimate()
        lb, mb = g.estimate()
        assert la.tolist() == lb.tolist()
        np.testing.assert_allclose(mb, ma, rtol=1e-4, atol=1e-4)
        g.close()


def test_unsorted_import_truncate_and_estimate(torch_cuda):
    """A state imported out of rank order is ranked by weight on both sides (stable), so the
    H_max cut and the tau prefix keep the same hypotheses as the oracle."""
    spec = sc.spec_for("c1")
    scene = sc.make_scene(spec, n_steps=6)
    p = sc.filter_params(spec, 64, 0.0)
    o = Oracle(p)
    o.import_state(sc.empty_state())
    for k in range(6):
        o.predict(k)
        o.update(k, scene.meas[k])
    st = to_f32_state(o.export_state())
    rng = np.random.default_rng(5)
    perm = rng.permutation(len(st["hyp_logw"]))
    shuffled = dict(st)
    offs, idx = [0], []
    for h in perm:
        idx.extend(st["hyp_idx"][st["hyp_off"][h]:st["hyp_off"][h + 1]].tolist())
        offs.append(len(idx))
    shuffled["hyp_logw"] = st["hyp_logw"][perm]
    shuffled["hyp_off"] = np.array(offs, np.int32)
    shuffled["hyp_idx"] = np.array(idx, np.int32)
    for hmax, tau in ((64, 0.0), (7, 0.0), (40, 2e-3), (64, 0.05)):
        oo = Oracle(p)
        oo.import_state(shuffled)
        oo.truncate(hmax, tau)
        g = _tracker(p)
        g.import_state(shuffled)
        g.truncate(hmax, tau)
        a, b = oo.export_state(), g.export_state()
        assert len(a["hyp_logw"]) == len(b["hyp_logw"]), (hmax, tau)
        # ties in weight keep the input order on both sides: parents match one to one
        assert a["hyp_parent"].tolist() == b["hyp_parent"].tolist()
        assert np.all(np.abs(b["hyp_logw"] - a["hyp_logw"]) <= pt.tol(a["hyp_logw"]))
        la, ma, _ = oo.estimate()
        lb, mb = g.estimate()
        assert la.tolist() == lb.tolist()
        np.testing.assert_allclose(mb, ma, rtol=1e-4, atol=1e-4)
        g.close()


def test_fingerprint_collisions_resolved(torch_cuda, monkeypatch):
    """(instance, detection set) records are deduplicated on a fingerprint; with the fingerprint
    narrowed to one bit, different sets of one instance collide in almost every update and must
    still become distinct instances (compared with the oracle, densities included)."""
    monkeypatch.setenv("GLMB_REC_HASH_BITS", "1")
    spec = sc.spec_for("c1")
    scene = sc.make_scene(spec, n_steps=8)
    p = sc.filter_params(spec, 64, 1e-5)
    o = Oracle(p)
    o.import_state(sc.empty_state())
    collisions = 0
    for k in range(8):
        o.predict(k)
        pred = to_f32_state(o.export_state())
        _, stats, _, _ = check_update(pred, scene.meas[k], p, k)
        collisions += stats["rec_collisions"]
        o.import_state(pred)
        o.update(k, scene.meas[k])
    assert collisions > 0
