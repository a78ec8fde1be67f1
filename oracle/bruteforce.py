"""TEST INFRASTRUCTURE -- brute-force enumeration of a GLMB time step on tiny scenes.

A second, independent statement of the method used to pin the FP64 oracle.  It shares
no code with ``glmb_oracle.cpp`` and computes things by a different route:

* every association map theta of every predicted hypothesis is enumerated
  explicitly (the space has (T+1)^M members, Sec. 3);
* a child's weight is formed *track by track* as a product of probabilities
  (Poisson detection count of each track times the Gaussian densities of its
  detections from ``scipy.stats``, times kappa per clutter measurement), not as
  the oracle's per-measurement log-sum of Eq. 2 entries;
* posterior track densities use sequential single-detection Kalman updates
  rather than the oracle's one-shot update with the mean detection;
* prediction enumerates every survive/die x include/exclude subset and
  multiplies probabilities.

Only ``tests/`` imports this module.
"""
from __future__ import annotations

import itertools
import math

import numpy as np
from scipy import stats


def cv_matrices(dt: float, q: float):
    F = np.eye(4)
    F[0, 2] = F[1, 3] = dt
    # discretised white-noise acceleration from the Van Loan construction
    from scipy.linalg import expm
    A = np.zeros((8, 8))
    Fc = np.zeros((4, 4))
    Fc[0, 2] = Fc[1, 3] = 1.0
    Gq = np.zeros((4, 4))
    Gq[2, 2] = Gq[3, 3] = q
    A[:4, :4] = -Fc
    A[:4, 4:] = Gq
    A[4:, 4:] = Fc.T
    E = expm(A * dt)
    Fd = E[4:, 4:].T
    Q = Fd @ E[:4, 4:]
    return Fd, 0.5 * (Q + Q.T)


def _key_less(a, b):
    return a < b


def _rank_children(children, K, eps=1e-10):
    """Sort children (value, key, payload) by value desc then key asc; values within
    eps (relative) of each other count as equal.  Returns the first K (all members of
    a tie class straddling the cut are ordered by key)."""
    children = sorted(children, key=lambda c: -c[0])
    groups, cur = [], []
    for c in children:
        if cur and abs(c[0] - cur[0][0]) > eps * max(1.0, abs(cur[0][0])):
            groups.append(cur)
            cur = []
        cur.append(c)
    if cur:
        groups.append(cur)
    out = []
    for g in groups:
        out.extend(sorted(g, key=lambda c: c[1]))
    return out[:K]


def _items_positions(devs):
    """devs: list of (delta, group id, option key) -> dict mapping (group, optkey) -> position."""
    order = sorted(range(len(devs)), key=lambda j: (devs[j][0], devs[j][1], devs[j][2]))
    return {(devs[j][1], devs[j][2]): p for p, j in enumerate(order)}


def predict(state: dict, p: dict, K: int):
    """All survive/die x include/exclude subsets; returns ranked merged hypotheses.

    Output: list of dicts with 'logw' (normalised), 'src' (sorted tuple of source
    instance ids; births are n_inst + b), 'parent' (representative), and the
    predicted instance moments keyed by src id.
    """
    F, Q = cv_matrices(p["dt"], p["q"])
    labs = np.asarray(state["inst_lab"]).reshape(-1, 2)
    n_inst = labs.shape[0]
    moments = {}
    for u in range(n_inst):
        m = F @ np.asarray(state["inst_m"][u])
        P = F @ np.asarray(state["inst_P"][u]).reshape(4, 4) @ F.T + Q
        moments[u] = (m, P, (int(labs[u, 0]), int(labs[u, 1])))
    nb = len(state["birth_r"])
    for b in range(nb):
        m = F @ np.asarray(state["birth_m"][b])
        P = F @ np.asarray(state["birth_P"][b]).reshape(4, 4) @ F.T + Q
        moments[n_inst + b] = (m, P, tuple(int(x) for x in state["birth_lab"][b]))
    ps = p["p_survive"]
    children = []
    for h in range(len(state["hyp_logw"])):
        tracks = list(state["hyp_idx"][state["hyp_off"][h]:state["hyp_off"][h + 1]])
        tracks.sort(key=lambda u: moments[u][2])
        dims = [("t", u, ps) for u in tracks] + [("b", n_inst + b, state["birth_r"][b]) for b in range(nb)]
        # best choice of every dimension and its item position for the canonical key
        devs = []
        for d, (_, _, pr) in enumerate(dims):
            if 0.0 < pr < 1.0:
                devs.append((abs(math.log(pr) - math.log(1.0 - pr)), d, 0))
        pos = _items_positions(devs)
        for choice in itertools.product([True, False], repeat=len(dims)):
            prob = math.exp(state["hyp_logw"][h])
            flips = []
            members = []
            for d, ((kind, src, pr), yes) in enumerate(zip(dims, choice)):
                prob *= pr if yes else (1.0 - pr)
                best_yes = pr >= 1.0 - pr
                if yes != best_yes:
                    flips.append(d)
                if yes:
                    members.append(src)
            if prob <= 0.0:
                continue
            key = (h, len(flips), tuple(sorted(pos[(d, 0)] for d in flips)))
            children.append((math.log(prob), key, tuple(sorted(members))))
    top = _rank_children(children, K)
    merged = {}
    for v, key, mem in top:
        if mem in merged:
            mv, mk = merged[mem]
            merged[mem] = (np.logaddexp(mv, v), min(mk, key))
        else:
            merged[mem] = (v, key)
    items = [(v, k, mem) for mem, (v, k) in merged.items()]
    items = _rank_children(items, len(items))
    z = np.logaddexp.reduce([v for v, _, _ in items])
    return [dict(logw=v - z, src=mem, parent=k[0]) for v, k, mem in items], moments


def update(state: dict, z: np.ndarray, p: dict, K: int, tau: float = 0.0, skip=()):
    """Enumerate every association map of every hypothesis of a *predicted* state.

    ``skip``: (instance, measurement) pairs a proposal removes.  Maps that use one of them
    are left out of the ranking and the marginals; ``lost`` is their share of the mass of
    all maps."""
    z = np.asarray(z, dtype=np.float64).reshape(-1, 2)
    M = z.shape[0]
    labs = np.asarray(state["inst_lab"]).reshape(-1, 2)
    sig2 = p["sigma_z"] ** 2
    gamma, kappa = p["det_rate"], p["clutter_density"]
    gate = stats.chi2.ppf(0.9999, 2) if p.get("gate_from_chi2") else p["gate_d2"]
    U = labs.shape[0]
    lab = [(int(labs[u, 0]), int(labs[u, 1])) for u in range(U)]
    m = [np.asarray(state["inst_m"][u]) for u in range(U)]
    P = [np.asarray(state["inst_P"][u]).reshape(4, 4) for u in range(U)]
    S = [P[u][:2, :2] + sig2 * np.eye(2) for u in range(U)]
    dens = np.zeros((U, M))
    gated = np.zeros((U, M), bool)
    for u in range(U):
        for i in range(M):
            nu = z[i] - m[u][:2]
            d2 = float(nu @ np.linalg.solve(S[u], nu))
            gated[u, i] = d2 <= gate
            dens[u, i] = stats.multivariate_normal(mean=m[u][:2], cov=S[u]).pdf(z[i])
    children = []
    Zh = []
    total_all = 0.0
    pair_mass, exist_mass = {}, {}
    skip = set((int(a), int(b)) for a, b in skip)
    for h in range(len(state["hyp_logw"])):
        tracks = list(state["hyp_idx"][state["hyp_off"][h]:state["hyp_off"][h + 1]])
        tracks.sort(key=lambda u: lab[u])
        w_h = math.exp(state["hyp_logw"][h])
        opts, opts_all = [], []
        for i in range(M):
            opts_all.append([-1] + [u for u in tracks if gated[u, i]])
            opts.append([-1] + [u for u in tracks if gated[u, i] and (u, i) not in skip])
        # best option per measurement and the deviation items for the canonical key
        def lphi(u, i):
            return math.log(kappa) if u < 0 else math.log(gamma * dens[u, i])
        def okey(u):
            return (0, 0, 0) if u < 0 else (1,) + lab[u]
        best = []
        devs = []
        for i in range(M):
            o = sorted(opts[i], key=lambda u: (-lphi(u, i), okey(u)))
            best.append(o[0])
            for u in o[1:]:
                devs.append((lphi(o[0], i) - lphi(u, i), i, okey(u)))
        pos = _items_positions(devs)
        total = 0.0
        for theta in itertools.product(*opts_all):
            prob = w_h
            for u in tracks:
                Su = [i for i in range(M) if theta[i] == u]
                prob *= stats.poisson.pmf(len(Su), gamma) * math.factorial(len(Su))
                for i in Su:
                    prob *= dens[u, i]
            for i in range(M):
                if theta[i] < 0:
                    prob *= kappa
            total_all += prob
            if any((theta[i], i) in skip for i in range(M)):
                continue
            total += prob
            for i in range(M):
                if theta[i] >= 0:
                    pair_mass[(theta[i], i)] = pair_mass.get((theta[i], i), 0.0) + prob
            for u in tracks:
                exist_mass[u] = exist_mass.get(u, 0.0) + prob
            dv = [i for i in range(M) if theta[i] != best[i]]
            key = (h, len(dv), tuple(sorted(pos[(i, okey(theta[i]))] for i in dv)))
            children.append((math.log(prob) if prob > 0 else -np.inf, key, (h, tuple(theta))))
        Zh.append(total)
    Zh = np.array(Zh)
    Ztot = Zh.sum()
    # clutter probability of each measurement under the full posterior
    pc = np.zeros(M)
    for v, key, (h, theta) in children:
        for i in range(M):
            if theta[i] < 0:
                pc[i] += math.exp(v) / Ztot
    top = _rank_children(children, K)
    lz = np.logaddexp.reduce([v for v, _, _ in top])
    if tau > 0:
        keep = 1
        while keep < len(top) and math.exp(top[keep][0] - lz) >= tau:
            keep += 1
        top = top[:keep]
        lz = np.logaddexp.reduce([v for v, _, _ in top])
    out = []
    for v, key, (h, theta) in top:
        tracks = list(state["hyp_idx"][state["hyp_off"][h]:state["hyp_off"][h + 1]])
        dens_out = {}
        for u in tracks:
            mm, PP = m[u].copy(), P[u].copy()
            for i in range(M):
                if theta[i] == u:      # sequential single-detection updates
                    Hm = np.zeros((2, 4))
                    Hm[0, 0] = Hm[1, 1] = 1.0
                    Sk = Hm @ PP @ Hm.T + sig2 * np.eye(2)
                    Kg = PP @ Hm.T @ np.linalg.inv(Sk)
                    mm = mm + Kg @ (z[i] - Hm @ mm)
                    PP = (np.eye(4) - Kg @ Hm) @ PP
            dens_out[lab[u]] = (mm, PP)
        out.append(dict(logw=v - lz, parent=h, theta=tuple(theta), dens=dens_out))
    return dict(children=out, logpi=np.log(Zh / Ztot), ru=1.0 - pc,
                retained=math.exp(lz) / Ztot, Zh=Zh, gated=gated, dens=dens,
                lost=1.0 - Ztot / total_all,
                pair_mass={k: v / Ztot for k, v in pair_mass.items()},
                exist={k: v / Ztot for k, v in exist_mass.items()})
