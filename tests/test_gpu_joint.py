"""Exact-joint reweighting on the GPU (glmb_set_joint_reweighting) against the oracle on the
same seeded inputs: the same kept hypotheses, re-ranked by the joint likelihood of every
track's detection set, with the same renormalised log-weights (1e-4 relative) and densities;
alone and together with the sampled children."""
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


def check_joint(state, z, p, k=0, sampling=None):
    from paper_2512_06230_amd.glmb import Tracker
    st = to_f32_state(state)
    o = Oracle(p)
    o.import_state(st)
    o.set_joint(True)
    if sampling:
        o.set_sampling(*sampling)
    o.update(k, z)
    out_o = o.export_state()
    fragile = o.sample_stats()[2] if sampling else []
    g = Tracker(p)
    g.import_state(st)
    g.set_joint_reweighting(True)
    if sampling:
        g.set_sampling(*sampling)
    g.update(k, z)
    out_g = g.export_state()
    M = np.asarray(z).reshape(-1, 2).shape[0]
    th_g = g.theta(len(out_g["hyp_logw"]), M)
    g.close()
    skip = pt.parents_with(st, pt.near_gate_instances(st, z, p["sigma_z"], p["gate_d2"])) | set(fragile)
    ids_o = pt.update_ids(out_o, out_o["theta"])
    ids_g = pt.update_ids(out_g, th_g)
    lw_o, lw_g = np.asarray(out_o["hyp_logw"], np.float64), np.asarray(out_g["hyp_logw"], np.float64)
    if skip:
        common = set(ids_o) & set(ids_g)
        io = np.array([x in common for x in ids_o])
        ig = np.array([x in common for x in ids_g])
        if io.any():
            lw_o = lw_o - np.logaddexp.reduce(lw_o[io])
            lw_g = lw_g - np.logaddexp.reduce(lw_g[ig])
    matched = pt.compare_sets(ids_o, lw_o, ids_g, lw_g, skip)
    pt.compare_densities(out_o, ids_o, out_g, ids_g, skip)
    if not skip:
        # the re-ranked order itself, outside the tolerance band of neighbouring weights
        pos_g = {x: j for j, x in enumerate(ids_g)}
        for j, x in enumerate(ids_o[:-1]):
            y = ids_o[j + 1]
            if x in pos_g and y in pos_g and lw_o[j] - lw_o[j + 1] > 2 * pt.tol(lw_o[j]):
                assert pos_g[x] < pos_g[y], (x, y)
    return matched


@pytest.mark.parametrize("seed", range(8))
def test_joint_reweighting_random_states(torch_cuda, seed):
    rng = np.random.default_rng(900 + seed)
    st = sc.random_state(rng, n_lab=3 + seed % 4, n_hyp=2 + 3 * (seed % 3), side=12.0, versions=1 + seed % 2)
    z = sc.measurements_near(rng, st, 2, 12.0, 1.0, det_mean=2.5)
    for K, tau in ((1000, 0.0), (8, 0.0), (64, 1e-3)):
        matched = check_joint(st, z, dict(BASE, h_max=K, tau=tau))
        assert matched > 0


def test_joint_reweighting_along_a_scene(torch_cuda):
    """The 5-object scene (1-3 detections per object) with joint reweighting on the GPU; at every
    scan its predicted state is updated by both sides, exact and sampled (H_up = 100)."""
    from paper_2512_06230_amd.glmb import Tracker
    spec = sc.spec_for("c1")
    scene = sc.make_scene(spec, n_steps=8)
    p = sc.filter_params(spec, 100, 1e-5)
    g = Tracker(p)
    g.import_state(sc.empty_state())
    g.set_joint_reweighting(True)
    total = 0
    for k in range(8):
        g.predict(k)
        pre = g.export_state()
        total += check_joint(pre, scene.meas[k], p, k)
        total += check_joint(pre, scene.meas[k], p, k, sampling=(100, 31))
        g.update(k, scene.meas[k])
        g.truncate(p["h_max"], p["tau"])
    g.close()
    assert total > 100
