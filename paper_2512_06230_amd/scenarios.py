"""Seeded synthetic scenes for the multi-detection GLMB tracker.

This module only *simulates* the world that the tracker observes: ground-truth
object trajectories, per-object detection clusters and uniform clutter.  It
contains none of the filter's arithmetic, and both the FP64 oracle and the HIP
library consume exactly the arrays it produces (measurements are stored as
float32, the oracle upcasts them).

The structure follows the paper's benchmark (Sec. 4.1): every object yields a
cluster of Gaussian point detections per scan, the detections are presented in
an arbitrary order (the tracker is order invariant), and the scene sizes follow
the configurations used for this build:

* ``c1``   5 objects, 100x100 m, CV motion dt=1 q=1, Pd=0.9, 1-3 detections
           per detected object (Poisson(1.5) clipped), sigma=1 m, clutter
           Poisson(2); 20 scans.
* ``c2``   50 objects, 1000x1000 m, object births Poisson(0.5)/scan, object
           survival 0.99, Poisson(3) detections per object, sigma=2 m,
           clutter Poisson(20); 100 scans.
* ``c3``   c1's generative model with N objects and clutter mean 0.2*N.
* ``c5``   c3 at N=500 (clutter 100).
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional

import numpy as np


@dataclasses.dataclass
class SceneSpec:
    n_obj: int = 5
    side: float = 100.0          # square region [0, side]^2 (reflecting walls)
    n_steps: int = 20
    dt: float = 1.0
    q: float = 1.0               # white-noise acceleration intensity of the truth
    sigma: float = 1.0           # detection noise std (m)
    pd: float = 0.9              # probability that an object is detected at all
    count_mode: str = "clip13"   # "clip13": Poisson(1.5) clipped to [1,3]; "poisson": Poisson(count_mean)
    count_mean: float = 1.5
    clutter_mean: float = 2.0
    birth_rate: float = 0.0      # truth births per scan
    survival: float = 1.0        # truth per-scan survival
    v0_sigma: float = 1.0        # initial velocity std (m/s)
    seed: int = 0


PRESETS = {
    "c1": dict(n_obj=5, side=100.0, n_steps=20, sigma=1.0, pd=0.9, count_mode="clip13",
               count_mean=1.5, clutter_mean=2.0),
    "c2": dict(n_obj=50, side=1000.0, n_steps=100, sigma=2.0, pd=1.0, count_mode="poisson",
               count_mean=3.0, clutter_mean=20.0, birth_rate=0.5, survival=0.99),
}


def spec_for(name: str, **over) -> SceneSpec:
    """Scene spec by preset name ("c1", "c2", "c3:<N>", "c5")."""
    if name.startswith("c3"):
        n = int(name.split(":")[1]) if ":" in name else 100
        base = dict(PRESETS["c1"], n_obj=n, clutter_mean=0.2 * n, n_steps=50)
    elif name == "c5":
        base = dict(PRESETS["c1"], n_obj=500, clutter_mean=100.0, n_steps=50)
    else:
        base = dict(PRESETS[name])
    base.update(over)
    return SceneSpec(**base)


def expected_detections(spec: SceneSpec) -> float:
    """Mean number of detections an existing object yields per scan in the simulator."""
    if spec.count_mode == "clip13":
        lam = spec.count_mean
        p0 = math.exp(-lam)
        p1 = lam * p0
        p2 = lam * lam / 2.0 * p0
        e = 1.0 * (p0 + p1) + 2.0 * p2 + 3.0 * (1.0 - p0 - p1 - p2)
        return spec.pd * e
    return spec.pd * spec.count_mean


@dataclasses.dataclass
class Scene:
    spec: SceneSpec
    meas: List[np.ndarray]            # per scan: float32 [M_k, 2]
    truth_ids: List[np.ndarray]       # per scan: int32 [N_k]
    truth_x: List[np.ndarray]         # per scan: float64 [N_k, 4]
    prior_x: np.ndarray               # float64 [N_0, 4] truth one scan before scan 0
    prior_ids: np.ndarray


def _cv_step(x: np.ndarray, dt: float, q: float, rng: np.random.Generator) -> np.ndarray:
    # sample the exact discretisation of a white-noise-acceleration process per axis
    n = x.shape[0]
    c = np.array([[dt ** 3 / 3.0, dt ** 2 / 2.0], [dt ** 2 / 2.0, dt]]) * q
    L = np.linalg.cholesky(c)
    out = x.copy()
    for ax in range(2):
        w = rng.standard_normal((n, 2)) @ L.T
        out[:, ax] = x[:, ax] + dt * x[:, 2 + ax] + w[:, 0]
        out[:, 2 + ax] = x[:, 2 + ax] + w[:, 1]
    return out


def _reflect(x: np.ndarray, side: float) -> None:
    for ax in range(2):
        lo = x[:, ax] < 0.0
        x[lo, ax] = -x[lo, ax]
        x[lo, 2 + ax] = -x[lo, 2 + ax]
        hi = x[:, ax] > side
        x[hi, ax] = 2.0 * side - x[hi, ax]
        x[hi, 2 + ax] = -x[hi, 2 + ax]
        np.clip(x[:, ax], 0.0, side, out=x[:, ax])


def make_scene(spec: SceneSpec, n_steps: Optional[int] = None) -> Scene:
    rng = np.random.default_rng(spec.seed)
    steps = spec.n_steps if n_steps is None else n_steps
    n0 = spec.n_obj
    pos = rng.uniform(0.0, spec.side, size=(n0, 2))
    vel = rng.normal(0.0, spec.v0_sigma, size=(n0, 2))
    x = np.concatenate([pos, vel], axis=1)
    ids = np.arange(n0, dtype=np.int32)
    next_id = n0
    prior_x = x.copy()
    prior_x[:, 0:2] -= spec.dt * prior_x[:, 2:4]
    prior_ids = ids.copy()
    meas, tids, tx = [], [], []
    for k in range(steps):
        if k > 0:
            x = _cv_step(x, spec.dt, spec.q, rng)
            _reflect(x, spec.side)
            if spec.survival < 1.0 and len(ids):
                keep = rng.uniform(size=len(ids)) < spec.survival
                x, ids = x[keep], ids[keep]
            if spec.birth_rate > 0.0:
                nb = rng.poisson(spec.birth_rate)
                if nb:
                    bp = rng.uniform(0.0, spec.side, size=(nb, 2))
                    bv = rng.normal(0.0, spec.v0_sigma, size=(nb, 2))
                    x = np.concatenate([x, np.concatenate([bp, bv], axis=1)], axis=0)
                    ids = np.concatenate([ids, np.arange(next_id, next_id + nb, dtype=np.int32)])
                    next_id += nb
        zs = []
        for j in range(len(ids)):
            if rng.uniform() >= spec.pd:
                continue
            if spec.count_mode == "clip13":
                c = int(min(max(rng.poisson(spec.count_mean), 1), 3))
            else:
                c = int(rng.poisson(spec.count_mean))
            if c:
                zs.append(x[j, 0:2] + spec.sigma * rng.standard_normal((c, 2)))
        nc = rng.poisson(spec.clutter_mean)
        if nc:
            zs.append(rng.uniform(0.0, spec.side, size=(nc, 2)))
        z = np.concatenate(zs, axis=0) if zs else np.zeros((0, 2))
        z = z[rng.permutation(z.shape[0])]
        meas.append(np.ascontiguousarray(z, dtype=np.float32))
        tids.append(ids.copy())
        tx.append(x.copy())
    return Scene(spec=spec, meas=meas, truth_ids=tids, truth_x=tx, prior_x=prior_x,
                 prior_ids=prior_ids)


# --------------------------------------------------------------------------- convoy (Sec. 4.1)
def convoy_track(K: int = 548, dt: float = 0.1, loops: float = 2.0, center: float = 40.0) -> np.ndarray:
    """A smooth closed ground-truth track standing in for the paper's GPS track (which is not
    available): K positions 0.1 s apart inside an 80 x 80 m area, the closed curve
    (30 cos t + 4 cos 3t, 24 sin t + 5 sin 2t) traversed `loops` times (two loops: about 6.5 m/s,
    three: about 10 m/s), so that time offsets taken modulo K stay on a continuous path."""
    t = 2.0 * math.pi * loops * np.arange(K) / K
    x = center + 30.0 * np.cos(t) + 4.0 * np.cos(3.0 * t)
    y = center + 24.0 * np.sin(t) + 5.0 * np.sin(2.0 * t)
    return np.stack([x, y], axis=1)


@dataclasses.dataclass
class ConvoySpec:
    n_obj: int = 5
    delta: int = 2        # time offset between consecutive copies (steps)
    det: int = 5          # detections per object per step (D)
    sigma: float = 0.25   # detection noise std (m)
    clutter: float = 0.0  # clutter detections per step (lambda = 0 in the paper)
    K: int = 548          # steps of 0.1 s (54.8 s)
    dt: float = 0.1
    loops: float = 3.0    # times the base track goes round its closed curve (about 10 m/s)
    seed: int = 0


def make_convoy(spec: ConvoySpec, n_steps: Optional[int] = None) -> Scene:
    """The paper's benchmark construction (Sec. 4.1): N copies of one track, copy n offset by
    n * delta steps (position at step k is the base track's at (k + n delta) mod K), each
    yielding D detections N(x, sigma^2 I) per step, listed object by object (the tracker is
    invariant to their order).  Velocities in the truth are the track's finite differences."""
    rng = np.random.default_rng(spec.seed)
    base = convoy_track(spec.K, spec.dt, spec.loops)
    vel = (np.roll(base, -1, axis=0) - base) / spec.dt
    steps = spec.K if n_steps is None else n_steps
    ids = np.arange(spec.n_obj, dtype=np.int32)
    meas, tids, tx = [], [], []
    for k in range(steps):
        idx = (k + spec.delta * ids) % spec.K
        x = np.concatenate([base[idx], vel[idx]], axis=1)
        z = [x[j, 0:2] + spec.sigma * rng.standard_normal((spec.det, 2)) for j in range(spec.n_obj)]
        if spec.clutter > 0:
            nc = rng.poisson(spec.clutter)
            if nc:
                z.append(rng.uniform(0.0, 80.0, size=(nc, 2)))
        meas.append(np.ascontiguousarray(np.concatenate(z, axis=0), dtype=np.float32))
        tids.append(ids.copy())
        tx.append(x)
    prior = tx[0].copy()
    prior[:, 0:2] -= spec.dt * prior[:, 2:4]
    cs = SceneSpec(n_obj=spec.n_obj, side=80.0, n_steps=steps, dt=spec.dt, sigma=spec.sigma, pd=1.0,
                   count_mode="poisson", count_mean=float(spec.det), clutter_mean=spec.clutter, seed=spec.seed)
    return Scene(spec=cs, meas=meas, truth_ids=tids, truth_x=tx, prior_x=prior, prior_ids=ids.copy())


def convoy_params(spec: ConvoySpec, h_max: int, tau: float = 1e-5) -> dict:
    """Filter parameters for the convoy: gamma = D, constant-velocity model at dt = 0.1 with
    q = 32 m^2/s^3 (the track turns at up to ~8 m/s^2 at 10 m/s), kappa = 1e-6 per m^2 (no
    clutter, but a clutter option must exist), births from clusters within 3 sigma with a 3 m/s
    velocity spread (chosen on the N = 10 and 20 convoys among q in {2, 8, 32} and spreads in
    {3, 8, 15} m/s)."""
    return dict(
        dt=spec.dt, q=32.0, sigma_z=spec.sigma, p_survive=0.99, det_rate=float(spec.det),
        clutter_density=max(spec.clutter / 6400.0, 1e-6), gate_d2=-2.0 * math.log(1e-4),
        birth_r_max=0.5, birth_rate=0.5, birth_sigma_v=3.0, birth_ru_max=0.5, birth_cluster_d=3.0 * spec.sigma,
        h_max=int(h_max), tau=float(tau),
    )


def filter_params(spec: SceneSpec, h_max: int, tau: float) -> dict:
    """Tracker parameters matched to a simulated scene: gamma = the simulator's mean
    detections per object, kappa = clutter mean / region area, chi-square(2) gate at 0.9999,
    adaptive births seeded from detections with P(not clutter) < 0.5."""
    area = spec.side * spec.side
    return dict(
        dt=spec.dt, q=spec.q, sigma_z=spec.sigma, p_survive=0.99,
        det_rate=expected_detections(spec),
        clutter_density=max(spec.clutter_mean, 1e-3) / area,
        gate_d2=-2.0 * math.log(1e-4),            # chi-square(2) quantile at 0.9999
        birth_r_max=0.5, birth_rate=0.5, birth_sigma_v=2.0, birth_ru_max=0.5,
        birth_cluster_d=3.0 * spec.sigma,
        h_max=int(h_max), tau=float(tau),
    )


def warm_start_state(scene: Scene, vel_sigma: float = 1.0) -> dict:
    """One-hypothesis GLMB holding every object alive at scan 0, placed one scan earlier.

    Labels are (-1, object index).  Covariance is diag(sigma^2, sigma^2, v^2, v^2).
    """
    n = scene.prior_x.shape[0]
    s2 = scene.spec.sigma ** 2
    P = np.zeros((n, 4, 4))
    P[:, 0, 0] = s2
    P[:, 1, 1] = s2
    P[:, 2, 2] = vel_sigma ** 2
    P[:, 3, 3] = vel_sigma ** 2
    return dict(
        inst_lab=np.stack([np.full(n, -1, np.int32), np.arange(n, dtype=np.int32)], axis=1),
        inst_m=scene.prior_x.astype(np.float64),
        inst_P=P.reshape(n, 16),
        hyp_logw=np.zeros(1),
        hyp_off=np.array([0, n], np.int32),
        hyp_idx=np.arange(n, dtype=np.int32),
        birth_lab=np.zeros((0, 2), np.int32), birth_m=np.zeros((0, 4)),
        birth_P=np.zeros((0, 16)), birth_r=np.zeros(0),
    )


def empty_state() -> dict:
    """The GLMB with one hypothesis holding no objects (weight 1)."""
    return dict(
        inst_lab=np.zeros((0, 2), np.int32), inst_m=np.zeros((0, 4)), inst_P=np.zeros((0, 16)),
        hyp_logw=np.zeros(1), hyp_off=np.array([0, 0], np.int32), hyp_idx=np.zeros(0, np.int32),
        birth_lab=np.zeros((0, 2), np.int32), birth_m=np.zeros((0, 4)),
        birth_P=np.zeros((0, 16)), birth_r=np.zeros(0),
    )


def random_state(rng: np.random.Generator, n_lab: int, n_hyp: int, side: float,
                 versions: int = 2, p_present: float = 0.8) -> dict:
    """A synthetic multi-hypothesis GLMB for parity tests of a single stage.

    ``n_lab`` labels, each with up to ``versions`` instances (different histories ->
    slightly different means/covariances); every hypothesis holds a random subset
    of labels, one instance per held label; weights are random and normalised.
    """
    labs, ms, Ps = [], [], []
    inst_of = []
    for l in range(n_lab):
        base = np.array([rng.uniform(0, side), rng.uniform(0, side), rng.normal(), rng.normal()])
        vs = []
        for v in range(versions):
            m = base + np.concatenate([rng.normal(0, 0.3, 2), rng.normal(0, 0.1, 2)])
            A = rng.normal(0, 0.3, (4, 4))
            P = np.diag([1.0, 1.0, 0.5, 0.5]) * rng.uniform(0.5, 1.5) + A @ A.T * 0.1
            vs.append(len(labs))
            labs.append((l // 7, l))
            ms.append(m)
            Ps.append(P.reshape(16))
        inst_of.append(vs)
    rows = set()
    hyp_idx, hyp_off = [], [0]
    tries = 0
    while len(hyp_off) - 1 < n_hyp and tries < 50 * n_hyp:
        tries += 1
        row = []
        for l in range(n_lab):
            if rng.uniform() < p_present:
                row.append(inst_of[l][rng.integers(0, versions)])
        key = tuple(row)
        if key in rows:
            continue
        rows.add(key)
        hyp_idx.extend(row)
        hyp_off.append(len(hyp_idx))
    h = len(hyp_off) - 1
    lw = rng.normal(0, 2.0, h)
    lw = lw - np.log(np.exp(lw - lw.max()).sum()) - lw.max()
    lw = np.sort(lw)[::-1]
    return dict(
        inst_lab=np.array(labs, np.int32).reshape(-1, 2), inst_m=np.array(ms).reshape(-1, 4),
        inst_P=np.array(Ps).reshape(-1, 16), hyp_logw=lw,
        hyp_off=np.array(hyp_off, np.int32), hyp_idx=np.array(hyp_idx, np.int32),
        birth_lab=np.zeros((0, 2), np.int32), birth_m=np.zeros((0, 4)),
        birth_P=np.zeros((0, 16)), birth_r=np.zeros(0),
    )


def measurements_near(rng: np.random.Generator, state: dict, n_clutter: int, side: float,
                      sigma: float, det_mean: float = 1.5) -> np.ndarray:
    """Detections around every label of a state plus uniform clutter (float32)."""
    labs = state["inst_lab"]
    seen = {}
    for u in range(labs.shape[0]):
        key = (int(labs[u, 0]), int(labs[u, 1]))
        if key not in seen:
            seen[key] = u
    zs = []
    for u in seen.values():
        c = rng.poisson(det_mean)
        if c:
            zs.append(state["inst_m"][u, 0:2] + sigma * rng.standard_normal((c, 2)))
    if n_clutter:
        zs.append(rng.uniform(0, side, (n_clutter, 2)))
    z = np.concatenate(zs, axis=0) if zs else np.zeros((0, 2))
    z = z[rng.permutation(z.shape[0])]
    return np.ascontiguousarray(z, dtype=np.float32)


def mlp_init(seed: int, n_in: int = 6, n_hid: int = 64) -> np.ndarray:
    """Seeded initial parameters of the pair-scoring network, in the flat layout
    W1[n_hid][n_in] | b1 | W2[n_hid][n_hid] | b2 | w3[n_hid] | b3 (float32 values).

    Weights are uniform in +-sqrt(6 / fan_in) (He initialisation for ReLU layers; the
    output layer uses +-sqrt(1 / fan_in)); biases start at zero."""
    rng = np.random.default_rng(seed)
    a1, a2, a3 = math.sqrt(6.0 / n_in), math.sqrt(6.0 / n_hid), math.sqrt(1.0 / n_hid)
    parts = [rng.uniform(-a1, a1, n_hid * n_in), np.zeros(n_hid),
             rng.uniform(-a2, a2, n_hid * n_hid), np.zeros(n_hid),
             rng.uniform(-a3, a3, n_hid), np.zeros(1)]
    return np.concatenate(parts).astype(np.float32)


def batch_specs(n_scenes: int = 256, seed: int = 0, n_min: int = 5, n_max: int = 200,
                h_lo: int = 256, h_hi: int = 8192, n_steps: int = 50):
    """Many independent scenes of uneven size: scene s has seed `seed + s`, N ~ U{n_min..n_max}
    objects of the c1 model (100x100 m, clutter Poisson(2)) and H_max = round(exp(U[ln h_lo,
    ln h_hi])).  Returns a list of (SceneSpec, H_max)."""
    rng = np.random.default_rng(10_000 + seed)
    out = []
    for s in range(n_scenes):
        n = int(rng.integers(n_min, n_max + 1))
        h = int(round(math.exp(rng.uniform(math.log(h_lo), math.log(h_hi)))))
        out.append((spec_for("c1", n_obj=n, seed=seed + s, n_steps=n_steps), h))
    return out
