"""Training and calibration of the learned pair proposal, on the GPU.

Every numerical step runs in the library's kernels through the C ABI: the training data
(pair features and the plain update's association probabilities) come from
``glmb_pair_features``, the network is trained with ``glmb_mlp_grad`` and ``glmb_mlp_adam``,
and the threshold is calibrated with ``glmb_proposal_lost``.  This module only moves arrays,
draws the seeded minibatch order, and keeps the bookkeeping (feature statistics over the
collected set, the threshold choice).

Target of a pair (u, i): the posterior probability that detection i belongs to instance u
given that u exists (full posterior of the plain update), weighted by the posterior mass of
the hypotheses holding u.  Loss: weighted binary cross-entropy.  Threshold: the largest value
on a grid whose lost posterior mass versus the plain update (the plain update's retained
mass that the proposal's update does not retain) stays below a bound on every held-out scan;
the lost mass of the full posterior over all association maps is reported beside it.
"""
from __future__ import annotations

import dataclasses
import json
import os
from typing import List, Optional

import numpy as np

from . import scenarios as sc
from .glmb import MLP_NPARAM, Tracker

THRESHOLDS = [1e-7, 3e-7, 1e-6, 3e-6, 1e-5, 3e-5, 1e-4, 3e-4, 1e-3, 3e-3, 1e-2, 2e-2, 5e-2, 0.1, 0.2, 0.4]


@dataclasses.dataclass
class Proposal:
    params: np.ndarray          # float32 [4673]
    norm: np.ndarray            # float32 [12]: feature means, then standard deviations
    threshold: float            # remove a pair when sigmoid(logit) < threshold
    info: dict

    def save(self, path: str):
        np.savez(path, params=self.params, norm=self.norm, threshold=np.float64(self.threshold),
                 info=np.frombuffer(json.dumps(self.info).encode(), dtype=np.uint8))

    @staticmethod
    def load(path: str) -> "Proposal":
        d = np.load(path, allow_pickle=False)
        return Proposal(d["params"].astype(np.float32), d["norm"].astype(np.float32), float(d["threshold"]),
                        json.loads(bytes(d["info"]).decode()))


def _scene_tracker(spec, h_max: int, n_steps: int):
    scene = sc.make_scene(spec, n_steps=n_steps)
    params = sc.filter_params(spec, h_max, 0.0)
    trk = Tracker(params)
    trk.import_state(sc.warm_start_state(scene))
    return scene, trk


def collect(specs: List[sc.SceneSpec], h_max: int, n_steps: int, log=None):
    """Run the plain filter over each scene; at every scan, before the update, record the
    pair features, targets and weights of the predicted state (CUDA tensors, concatenated)."""
    import torch
    feats, ys, ws = [], [], []
    for spec in specs:
        scene, trk = _scene_tracker(spec, h_max, n_steps)
        for k in range(n_steps):
            trk.predict(k)
            z = torch.as_tensor(scene.meas[k], device="cuda")
            f, _, y, w = trk.pair_features(k, z)
            feats.append(f.clone())
            ys.append(y.clone())
            ws.append(w.clone())
            trk.update(k, z)
            trk.truncate(h_max, 0.0)
        trk.close()
        if log:
            log("collected scene seed %d: %d pairs" % (spec.seed, sum(int(f.shape[0]) for f in feats)))
    return torch.cat(feats), torch.cat(ys), torch.cat(ws)


def feature_norm(feat) -> np.ndarray:
    """Per-feature mean and standard deviation of the collected features (host bookkeeping)."""
    X = feat.detach().cpu().numpy().astype(np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return np.concatenate([mu, sd]).astype(np.float32)


def train(trk: Tracker, feat, y, w, epochs: int = 20, batch: int = 8192, lr: float = 2e-3, seed: int = 0,
          log=None):
    """Adam on minibatches; returns (params CUDA tensor, norm, loss history)."""
    import torch
    norm = feature_norm(feat)
    params = torch.as_tensor(sc.mlp_init(seed), device="cuda").contiguous()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    rng = np.random.default_rng(seed)
    n = int(feat.shape[0])
    step = 0
    hist = []
    for ep in range(epochs):
        order = torch.as_tensor(rng.permutation(n), device="cuda")
        tot = 0.0
        nb = 0
        for b0 in range(0, n, batch):
            idx = order[b0:b0 + batch]
            fb = feat.index_select(0, idx).contiguous()
            yb = y.index_select(0, idx).contiguous()
            wb = w.index_select(0, idx).contiguous()
            if float(wb.sum()) <= 0.0:
                continue
            g, loss = trk.mlp_grad(params, norm, fb, yb, wb)
            step += 1
            trk.mlp_adam(params, m, v, g, step, lr)
            tot += float(loss[0])
            nb += 1
        hist.append(tot / max(nb, 1))
        if log:
            log("epoch %d loss %.5f" % (ep, hist[-1]))
    return params, norm, hist


def retained_lost(trk: Tracker, pred_state: dict, k: int, z, params, norm, thresholds):
    """Posterior mass, under the plain update's normalised weights, of the hypotheses the
    plain update retains and the proposal's update (at each threshold) does not, for one
    predicted state; hypotheses are identified by (parent, association map)."""
    M = int(z.shape[0])

    def run(t):
        if t is None:
            trk.set_proposal(params, norm, apply=False)
        else:
            trk.set_proposal(params, norm, t, apply=True)
        trk.import_state(pred_state)
        trk.update(k, z)
        out = trk.export_state()
        th = trk.theta(len(out["hyp_logw"]), M)
        return out, th

    out, th = run(None)
    w = np.exp(out["hyp_logw"].astype(np.float64))
    ref = {(int(p), row.tobytes()): float(x) for p, row, x in zip(out["hyp_parent"], th, w)}
    res = []
    for t in thresholds:
        o2, th2 = run(t)
        keys = set((int(p), row.tobytes()) for p, row in zip(o2["hyp_parent"], th2))
        res.append(sum(x for key, x in ref.items() if key not in keys))
    trk.set_proposal(params, norm, apply=False)
    return np.array(res)


def calibrate(params, norm, specs: List[sc.SceneSpec], h_max: int, n_steps: int, max_lost: float = 1e-3,
              thresholds=THRESHOLDS, log=None):
    """Largest threshold whose retained-set lost mass (see retained_lost) stays <= max_lost on
    every held-out scan of the plain filter's trajectory.  Returns (threshold, worst retained-set
    lost mass per threshold, worst full-posterior lost mass per threshold)."""
    import torch
    worst_ret = np.zeros(len(thresholds))
    worst_full = np.zeros(len(thresholds))
    for spec in specs:
        scene, trk = _scene_tracker(spec, h_max, n_steps)
        probe = Tracker(sc.filter_params(spec, h_max, 0.0))
        trk.set_proposal(params, norm, apply=False)  # loaded for the measurement; updates stay plain
        for k in range(n_steps):
            trk.predict(k)
            z = torch.as_tensor(scene.meas[k], device="cuda")
            worst_full = np.maximum(worst_full, trk.proposal_lost(k, z, thresholds))
            worst_ret = np.maximum(worst_ret, retained_lost(probe, trk.export_state(), k, z, params, norm,
                                                            thresholds))
            trk.update(k, z)
            trk.truncate(h_max, 0.0)
        trk.close()
        probe.close()
        if log:
            log("held-out seed %d: worst retained-set lost mass %s" % (spec.seed, np.array2string(worst_ret, precision=2)))
            log("held-out seed %d: worst full-posterior lost mass %s" % (spec.seed, np.array2string(worst_full, precision=2)))
    ok = [t for t, L in zip(thresholds, worst_ret) if L <= max_lost]
    return (max(ok) if ok else None), worst_ret, worst_full


GATE_GRID = [18.42, 16.0, 14.0, 12.0, 10.0, 9.0, 8.0, 7.0, 6.0, 5.0, 4.0, 3.0, 2.5, 2.0, 1.5, 1.0, 0.5]


def gate_gain(params_filter: dict, pred_state: dict, k: int, z, prop: "Proposal", max_lost: float = 1e-3,
              gates=GATE_GRID):
    """What the learned proposal gains over the method without it, on one predicted state: the
    gated pairs the update keeps (i) with the plain gate, (ii) with the tightest Mahalanobis gate
    of the grid whose retained-set lost mass versus the plain update stays <= max_lost, and
    (iii) with the proposal at its threshold (its lost mass measured the same way)."""
    import torch
    M = int(z.shape[0])

    def update(p, proposal=None):
        t = Tracker(p)
        t.import_state(pred_state)
        if proposal is not None:
            t.set_proposal(torch.as_tensor(proposal.params, device="cuda"), proposal.norm, proposal.threshold,
                           apply=True)
        t.update(k, z)
        out = t.export_state()
        th = t.theta(len(out["hyp_logw"]), M)
        st = t.stats()
        t.close()
        ids = {(int(a), r.tobytes()): float(w) for a, r, w in zip(out["hyp_parent"], th, np.exp(out["hyp_logw"]))}
        return ids, st

    ref, st0 = update(params_filter)

    def lost(ids):
        return float(sum(w for key, w in ref.items() if key not in ids))

    res = dict(pairs_plain=int(st0["gated_pairs"]), gate_plain=float(params_filter["gate_d2"]))
    best = None
    for g in gates:
        if g > params_filter["gate_d2"]:
            continue
        ids, st = update(dict(params_filter, gate_d2=g))
        L = lost(ids)
        if L <= max_lost:
            best = (g, int(st["gated_pairs"]), L)
        else:
            break
    res.update(gate_tight=best[0], pairs_tight_gate=best[1], lost_tight_gate=best[2])
    ids, st = update(params_filter, prop)
    res.update(pairs_mlp=int(st["gated_pairs"] - st["pairs_removed"]), lost_mlp=lost(ids),
               gain_vs_tight_gate=best[1] / max(1, int(st["gated_pairs"] - st["pairs_removed"])))
    return res
