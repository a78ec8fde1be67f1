"""Helpers that compare the HIP library with the FP64 oracle on the same inputs.

Tolerance (FP32 log domain): |gpu - oracle| <= 1e-4 * max(|oracle|, 1) for normalised
log-weights and diagnostics.  Retained hypotheses are compared as sets of identities
(parent index, association map); a hypothesis may be missing on one side only if its
normalised log-weight lies within that tolerance band of the side's cut-off.  Pairs
whose Mahalanobis distance lies within 1e-4*G of the gate G may be gated differently
in FP32 and FP64; parents holding such a pair are excluded from the strict checks and
counted.
"""
from __future__ import annotations

import numpy as np

TOL = 1e-4


def tol(ref):
    return TOL * np.maximum(np.abs(ref), 1.0)


def near_gate_instances(state: dict, z: np.ndarray, sigma: float, gate: float) -> set:
    """Instances (input index) with a detection within 1e-4*G of the gate boundary."""
    z = np.asarray(z, np.float64)
    out = set()
    for u in range(state["inst_m"].shape[0]):
        P = np.asarray(state["inst_P"][u], np.float64).reshape(4, 4)
        S = P[:2, :2] + sigma ** 2 * np.eye(2)
        nu = z - np.asarray(state["inst_m"][u][:2], np.float64)
        d2 = np.einsum("ij,jk,ik->i", nu, np.linalg.inv(S), nu)
        if np.any(np.abs(d2 - gate) <= 1e-4 * gate):
            out.add(u)
    return out


def parents_with(state: dict, insts: set) -> set:
    out = set()
    for h in range(len(state["hyp_logw"])):
        if insts & set(state["hyp_idx"][state["hyp_off"][h]:state["hyp_off"][h + 1]].tolist()):
            out.add(h)
    return out


def compare_sets(ids_o, lw_o, ids_g, lw_g, skip_parents=frozenset()):
    """Identity sets and weights; returns the number of matched hypotheses."""
    lw_o = np.asarray(lw_o, np.float64)
    lw_g = np.asarray(lw_g, np.float64)
    do = {k: v for k, v in zip(ids_o, lw_o)}
    dg = {k: v for k, v in zip(ids_g, lw_g)}
    assert len(do) == len(ids_o) and len(dg) == len(ids_g), "duplicate identities"
    cut_o = lw_o.min() if len(lw_o) else 0.0
    cut_g = lw_g.min() if len(lw_g) else 0.0
    for k in set(do) - set(dg):
        if k[0] in skip_parents:
            continue
        assert do[k] <= cut_o + 2 * tol(cut_o), ("hypothesis missing on the GPU", k, do[k], cut_o)
    for k in set(dg) - set(do):
        if k[0] in skip_parents:
            continue
        assert dg[k] <= cut_g + 2 * tol(cut_g), ("hypothesis only on the GPU", k, dg[k], cut_g)
    matched = 0
    for k in set(do) & set(dg):
        if k[0] in skip_parents:
            continue
        assert abs(dg[k] - do[k]) <= tol(do[k]), ("log-weight", k, dg[k], do[k])
        matched += 1
    return matched


def update_ids(out: dict, theta: np.ndarray):
    return [(int(out["hyp_parent"][h]), tuple(int(x) for x in theta[h])) for h in range(len(out["hyp_logw"]))]


def predict_ids(out: dict):
    ids = []
    for h in range(len(out["hyp_logw"])):
        src = out["inst_src"][out["hyp_idx"][out["hyp_off"][h]:out["hyp_off"][h + 1]]]
        ids.append((tuple(sorted(int(x) for x in src)),))
    return ids


def track_densities(out: dict, h: int) -> dict:
    res = {}
    for j in range(out["hyp_off"][h], out["hyp_off"][h + 1]):
        u = out["hyp_idx"][j]
        res[(int(out["inst_lab"][u][0]), int(out["inst_lab"][u][1]))] = (
            np.asarray(out["inst_m"][u], np.float64), np.asarray(out["inst_P"][u], np.float64))
    return res


def _rows_by_label(out: dict, hs):
    """Instances of hypotheses ``hs`` in label order: (row ids, labels [n,2], instances [n])."""
    off = np.asarray(out["hyp_off"])
    lab = np.asarray(out["inst_lab"]).reshape(-1, 2)
    rid, ins = [], []
    for r, h in enumerate(hs):
        u = np.asarray(out["hyp_idx"][off[h]:off[h + 1]])
        key = lab[u, 0].astype(np.int64) * (1 << 32) + lab[u, 1].astype(np.int64)
        u = u[np.argsort(key, kind="stable")]
        rid.append(np.full(len(u), r))
        ins.append(u)
    rid = np.concatenate(rid) if rid else np.zeros(0, np.int64)
    ins = np.concatenate(ins).astype(np.int64) if ins else np.zeros(0, np.int64)
    return rid, lab[ins] if len(ins) else np.zeros((0, 2), np.int32), ins


def compare_densities(out_o, ids_o, out_g, ids_g, skip_parents=frozenset(), limit=None):
    """Track densities of every hypothesis present on both sides (or the first ``limit``):
    same labels, and means and covariances of each (oracle instance, GPU instance) pair met
    within the tolerance.  Returns the number of hypotheses compared."""
    pos_g = {k: h for h, k in enumerate(ids_g)}
    ho, hg = [], []
    for h, k in enumerate(ids_o):
        if k in pos_g and k[0] not in skip_parents:
            ho.append(h)
            hg.append(pos_g[k])
            if limit and len(ho) >= limit:
                break
    if not ho:
        return 0
    ro, lo, uo = _rows_by_label(out_o, ho)
    rg, lg, ug = _rows_by_label(out_g, hg)
    assert ro.shape == rg.shape and np.array_equal(ro, rg) and np.array_equal(lo, lg), "track labels differ"
    pairs = np.unique(np.stack([uo, ug], axis=1), axis=0)
    mo = np.asarray(out_o["inst_m"], np.float64)[pairs[:, 0]]
    mg = np.asarray(out_g["inst_m"], np.float64)[pairs[:, 1]]
    Po = np.asarray(out_o["inst_P"], np.float64)[pairs[:, 0]]
    Pg = np.asarray(out_g["inst_P"], np.float64)[pairs[:, 1]]
    bm = np.abs(mg - mo) > tol(mo)
    assert not bm.any(), ("mean", pairs[np.nonzero(bm.any(1))[0][:3]], mg[bm][:4], mo[bm][:4])
    bP = np.abs(Pg - Po) > tol(Po)
    assert not bP.any(), ("covariance", pairs[np.nonzero(bP.any(1))[0][:3]], Pg[bP][:4], Po[bP][:4])
    return len(ho)
