"""TEST INFRASTRUCTURE -- FP64 reference of the learned pair proposal.

The proposal is an addition to the update of Sec. 3: a small network scores every gated
(track instance, detection) pair of a predicted GLMB, and the update leaves out the pairs
whose score falls below a threshold, i.e. those whose posterior association probability
is negligible.  Everything here is plain NumPy in float64, written for checking, not speed.

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may import
this module.  It shares no code with the HIP library.

Contents
* ``pair_features``: six numbers per gated pair of a predicted GLMB and a detection set;
* ``forward`` / ``loss_and_grad``: the network 6 -> 64 -> 64 -> 1 with ReLU, optionally with
  the roundings of the GPU form (weights, standardised inputs and both hidden activations
  rounded to bfloat16, every sum exact), a weighted binary cross-entropy on the logit and
  its hand-derived gradient (the roundings pass gradients straight through);
* ``adam_step``: one step of Adam (Kingma & Ba, 2015, Algorithm 1, with bias correction);
* ``targets``: training targets from the oracle's association marginals.

Parameter vector (4673 float values, the layout the HIP library uses too):
  W1[64][6] | b1[64] | W2[64][64] | b2[64] | w3[64] | b3
with W[j][k] the weight from input k to output j.
"""
from __future__ import annotations

import math

import numpy as np

N_IN, N_HID = 6, 64
SIZES = [("W1", (N_HID, N_IN)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
         ("w3", (N_HID,)), ("b3", (1,))]
N_PARAM = sum(int(np.prod(s)) for _, s in SIZES)
FEATURES = ["d2", "nu_x", "nu_y", "r_label", "age", "n_gate"]


def unpack(params: np.ndarray) -> dict:
    params = np.asarray(params, np.float64)
    assert params.shape == (N_PARAM,)
    out, o = {}, 0
    for name, shape in SIZES:
        n = int(np.prod(shape))
        out[name] = params[o:o + n].reshape(shape)
        o += n
    return out


def pack(parts: dict) -> np.ndarray:
    return np.concatenate([np.asarray(parts[name], np.float64).reshape(-1) for name, _ in SIZES])


def bf16(x):
    """Round to the nearest bfloat16 value (8 significant bits), ties to even.

    Values in bfloat16's subnormal range are not treated specially (they do not occur here)."""
    x = np.asarray(x, np.float64)
    m, e = np.frexp(x)  # x = m * 2**e with 0.5 <= |m| < 1
    return np.ldexp(np.rint(m * 256.0) / 256.0, e)


# --------------------------------------------------------------------------- features
def label_existence(state: dict) -> dict:
    """r_l = sum of the weights of the hypotheses that contain label l."""
    w = np.exp(np.asarray(state["hyp_logw"], np.float64))
    lab = np.asarray(state["inst_lab"]).reshape(-1, 2)
    r = {}
    for h in range(len(w)):
        for u in state["hyp_idx"][state["hyp_off"][h]:state["hyp_off"][h + 1]]:
            key = (int(lab[u][0]), int(lab[u][1]))
            r[key] = r.get(key, 0.0) + w[h]
    return r


def pair_features(state: dict, z: np.ndarray, k: int, sigma_z: float, gate_d2: float) -> dict:
    """Features of every gated pair of a predicted GLMB, in (instance, detection) order.

    For instance u with predicted mean m and covariance P, and detection z_i:
      nu = z_i - H m, S = H P H^T + sigma_z^2 I, d2 = nu^T S^-1 nu (gated when d2 <= G);
      r_label = existence probability of u's label in the predicted GLMB;
      age     = k - (birth scan of u's label);
      n_gate  = number of detections gated with u.
    Every instance of the state is scored, as in the oracle's update."""
    z = np.asarray(z, np.float32).astype(np.float64).reshape(-1, 2)
    lab = np.asarray(state["inst_lab"]).reshape(-1, 2)
    r = label_existence(state)
    us, is_, rows = [], [], []
    for u in range(lab.shape[0]):
        m = np.asarray(state["inst_m"][u], np.float64)
        P = np.asarray(state["inst_P"][u], np.float64).reshape(4, 4)
        S = P[:2, :2] + sigma_z * sigma_z * np.eye(2)
        nu = z - m[:2]
        d2 = np.einsum("ij,ij->i", nu, np.linalg.solve(S, nu.T).T)
        g = np.nonzero(d2 <= gate_d2)[0]
        key = (int(lab[u][0]), int(lab[u][1]))
        for i in g:
            us.append(u)
            is_.append(int(i))
            rows.append([d2[i], nu[i, 0], nu[i, 1], r.get(key, 0.0), float(k - key[0]), float(len(g))])
    X = np.asarray(rows, np.float64).reshape(-1, N_IN)
    return dict(u=np.asarray(us, np.int32), i=np.asarray(is_, np.int32), X=X)


def feature_norm(X: np.ndarray) -> np.ndarray:
    """Per-feature mean and standard deviation (12 values); a constant feature gets 1."""
    X = np.asarray(X, np.float64)
    mu = X.mean(axis=0)
    sd = X.std(axis=0)
    sd = np.where(sd > 0, sd, 1.0)
    return np.concatenate([mu, sd])


def targets(pairs: dict) -> tuple:
    """Target p_ui = m_ui / e_u (association probability of the pair given that the
    instance exists) and sample weight e_u, from the oracle's full-posterior marginals
    (m_ui = sum over parents h holding u of pi_h q_hi(u), e_u = sum of those pi_h)."""
    mass = np.asarray(pairs["mass"], np.float64)
    ex = np.asarray(pairs["exist"], np.float64)
    y = np.where(ex > 0, mass / np.where(ex > 0, ex, 1.0), 0.0)
    return np.clip(y, 0.0, 1.0), ex


# --------------------------------------------------------------------------- network
def forward(params: np.ndarray, norm: np.ndarray, X: np.ndarray, bf16_mode: bool = True):
    R = bf16 if bf16_mode else (lambda a: np.asarray(a, np.float64))
    p = {k: R(v) for k, v in unpack(params).items()}
    norm = np.asarray(norm, np.float64)
    xs = R((np.asarray(X, np.float64) - norm[:N_IN]) / norm[N_IN:])
    a1 = xs @ p["W1"].T + p["b1"]
    h1 = R(np.maximum(a1, 0.0))
    a2 = h1 @ p["W2"].T + p["b2"]
    h2 = R(np.maximum(a2, 0.0))
    logit = h2 @ p["w3"] + p["b3"][0]
    cache = dict(p=p, xs=xs, a1=a1, h1=h1, a2=a2, h2=h2)
    return logit, cache


def loss_and_grad(params, norm, X, y, w, bf16_mode: bool = True):
    """Weighted binary cross-entropy on the logit s:
         L = sum_p w_p (softplus(s_p) - y_p s_p) / sum_p w_p
    and its gradient with respect to the parameter vector."""
    y = np.asarray(y, np.float64)
    w = np.asarray(w, np.float64)
    s, c = forward(params, norm, X, bf16_mode)
    W = w.sum()
    sp = np.maximum(s, 0.0) + np.log1p(np.exp(-np.abs(s)))
    loss = float((w * (sp - y * s)).sum() / W)
    ds = w * (1.0 / (1.0 + np.exp(-s)) - y) / W
    p = c["p"]
    g = {}
    g["w3"] = c["h2"].T @ ds
    g["b3"] = np.array([ds.sum()])
    da2 = np.outer(ds, p["w3"]) * (c["a2"] > 0)
    g["W2"] = da2.T @ c["h1"]
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ p["W2"]) * (c["a1"] > 0)
    g["W1"] = da1.T @ c["xs"]
    g["b1"] = da1.sum(axis=0)
    return loss, pack(g)


def adam_step(params, m, v, g, t: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
              eps: float = 1e-8):
    """One Adam step at step number t >= 1; returns (params, m, v)."""
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** t)
    vh = v / (1.0 - beta2 ** t)
    return np.asarray(params, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


def logit_threshold(t: float) -> float:
    """sigma(s) < t  <=>  s < log(t / (1 - t)) for 0 < t < 1."""
    return math.log(t / (1.0 - t))


# --------------------------------------------------------------------------- comparison aids
def _near_bf16_midpoint(v, err):
    """True where a value computed with absolute error up to ``err`` may round to a different
    bfloat16 value than the exact one: within ``err`` of a rounding midpoint, or of zero."""
    v = np.asarray(v, np.float64)
    m, e = np.frexp(np.abs(v))
    ulp = np.ldexp(1.0, e - 8)  # spacing of bfloat16 values around |v|
    t = np.abs(v) / ulp
    mid = (np.floor(t) + 0.5) * ulp
    return (np.abs(np.abs(v) - mid) <= err) | (np.abs(v) <= err)


def _f32_sequential(A, B, bias):
    """float32 sums over k of A[p, k] * B[j, k] + bias[j] taken in index order (the products of
    two bfloat16 values are exact in float32); used only to tell exact sums from rounded ones."""
    A32, B32 = A.astype(np.float32), B.astype(np.float32)
    acc = np.broadcast_to(bias.astype(np.float32), (A.shape[0], B.shape[0])).copy()
    for k in range(A.shape[1]):
        acc = (acc + np.outer(A32[:, k], B32[:, k]).astype(np.float32)).astype(np.float32)
    return acc.astype(np.float64)


def rounding_sensitive(params, norm, X, rel: float = 2e-7) -> np.ndarray:
    """Samples for which a float32 evaluation of the network may take a different bfloat16
    rounding (or ReLU) decision than the exact one: some standardised input or hidden
    pre-activation lies within ``rel`` times the sum of the magnitudes of its terms of a
    rounding midpoint (or of zero, for the ReLU).  A pre-activation that a float32 sum reaches
    exactly (products of bfloat16 values are exact in float32) is not sensitive.  These are the
    samples whose float32 and float64 logits may legitimately differ by one bfloat16 unit of an
    activation."""
    p = {k: bf16(v) for k, v in unpack(params).items()}
    norm = np.asarray(norm, np.float64)
    X = np.asarray(X, np.float64)
    u = (X - norm[:N_IN]) / norm[N_IN:]
    flag = np.any(_near_bf16_midpoint(u, rel * np.abs(u) + 1e-30), axis=1)
    xs = bf16(u)
    a1 = xs @ p["W1"].T + p["b1"]
    s1 = np.abs(xs) @ np.abs(p["W1"]).T + np.abs(p["b1"])
    inexact1 = _f32_sequential(xs, p["W1"], p["b1"]) != a1
    flag |= np.any(_near_bf16_midpoint(a1, rel * s1) & inexact1, axis=1)
    h1 = bf16(np.maximum(a1, 0.0))
    a2 = h1 @ p["W2"].T + p["b2"]
    s2 = np.abs(h1) @ np.abs(p["W2"]).T + np.abs(p["b2"])
    inexact2 = _f32_sequential(h1, p["W2"], p["b2"]) != a2
    flag |= np.any(_near_bf16_midpoint(a2, rel * s2) & inexact2, axis=1)
    return flag


def grad_abs_terms(params, norm, X, y, w) -> np.ndarray:
    """For every parameter, the sum over samples of the magnitudes of the terms whose sum is
    its gradient (the scale of the rounding error of a float32 accumulation)."""
    y = np.asarray(y, np.float64)
    w = np.asarray(w, np.float64)
    s, c = forward(params, norm, X, True)
    ds = np.abs(w * (1.0 / (1.0 + np.exp(-s)) - y) / w.sum())
    p = c["p"]
    g = {}
    g["w3"] = np.abs(c["h2"]).T @ ds
    g["b3"] = np.array([ds.sum()])
    da2 = np.outer(ds, np.abs(p["w3"])) * (c["a2"] > 0)
    g["W2"] = da2.T @ np.abs(c["h1"])
    g["b2"] = da2.sum(axis=0)
    da1 = (da2 @ np.abs(p["W2"])) * (c["a1"] > 0)
    g["W1"] = da1.T @ np.abs(c["xs"])
    g["b1"] = da1.sum(axis=0)
    return pack(g)
