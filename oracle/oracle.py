"""TEST INFRASTRUCTURE -- ctypes wrapper of the FP64 CPU oracle (``glmb_oracle.cpp``).

Only ``tests/``, ``__graft_entry__.smoke()`` and ``bench.py``'s CPU-baseline leg may
import this module.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "glmb_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

PARAM_ORDER = ["dt", "q", "sigma_z", "p_survive", "det_rate", "clutter_density", "gate_d2",
               "birth_r_max", "birth_rate", "birth_sigma_v", "birth_ru_max", "birth_cluster_d",
               "h_max", "tau"]


def build(force: bool = False, out: str = _LIB, mutant: int = 0) -> str:
    """Compile the oracle with g++ (plain -O2, no fast-math).  ``mutant`` > 0 builds a copy
    with a planted mistake (for the test that the pins catch such mistakes)."""
    if force or mutant or not os.path.exists(out) or os.path.getmtime(out) < os.path.getmtime(_SRC):
        tmp = out + ".tmp"
        subprocess.check_call(["g++", "-O2", "-std=c++17", "-fno-fast-math", "-shared", "-fPIC",
                               "-DORACLE_MUTANT=%d" % mutant, "-o", tmp, _SRC])
        os.replace(tmp, out)
    return out


_libs = {}


def _load(path: str = None):
    if path is None:
        path = build()
    if path not in _libs:
        L = ctypes.CDLL(path)
        vp, ip, dp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int32), \
            ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64)
        L.orc_create.restype = vp
        L.orc_create.argtypes = [dp]
        L.orc_destroy.argtypes = [vp]
        L.orc_set_hmax.argtypes = [vp, ctypes.c_int, ctypes.c_double]
        L.orc_import.argtypes = [vp, ctypes.c_int, ip, dp, dp, ctypes.c_int, dp, ip, ip,
                                 ctypes.c_int, ip, dp, dp, dp]
        L.orc_predict.argtypes = [vp, ctypes.c_int]
        L.orc_update.argtypes = [vp, ctypes.c_int, dp, ctypes.c_int]
        L.orc_truncate.argtypes = [vp, ctypes.c_int, ctypes.c_double]
        L.orc_estimate.argtypes = [vp, ctypes.c_int, ip, ip, dp, dp, ctypes.c_int]
        L.orc_sizes.argtypes = [vp, i64p]
        L.orc_export.argtypes = [vp, ip, dp, dp, ip, ip, ip, dp, ip, ip, ip, ip, ip, dp, dp, dp]
        L.orc_diag.argtypes = [vp, dp, dp, dp, dp]
        L.orc_pairs.argtypes = [vp, ip, ip, dp, dp, dp]
        L.orc_set_skip.argtypes = [vp, ctypes.c_int, ip, ip]
        L.orc_set_sampling.argtypes = [vp, ctypes.c_int, ctypes.c_uint64, ctypes.c_double]
        L.orc_sample_stats.argtypes = [vp, i64p, ip, ctypes.c_int]
        L.orc_sample_stats.restype = ctypes.c_int
        u32p = ctypes.POINTER(ctypes.c_uint32)
        L.orc_philox.argtypes = [u32p, u32p, u32p]
        L.orc_philox_uniform.argtypes = [ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32,
                                         ctypes.c_uint32]
        L.orc_philox_uniform.restype = ctypes.c_double
        L.orc_pf_predict.argtypes = [dp, ctypes.c_int64, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_uint64, ctypes.c_int]
        L.orc_pf_loglik.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, dp, ctypes.c_int, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_double, dp]
        L.orc_pf_update.argtypes = [dp, dp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ip, ip, ip, dp, ctypes.c_double,
                                    ctypes.c_double, ctypes.c_uint64, ctypes.c_int, ctypes.c_double, dp, dp, ip, ip]
        L.orc_set_joint.argtypes = [vp, ctypes.c_int]
        L.orc_joint_loglik.argtypes = [ctypes.c_double, ctypes.c_int, dp, dp, dp]
        L.orc_joint_loglik.restype = ctypes.c_double
        _libs[path] = L
    return _libs[path]


def _i32(a):
    a = np.ascontiguousarray(a, dtype=np.int32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


def _f64(a):
    a = np.ascontiguousarray(a, dtype=np.float64)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


class Oracle:
    """FP64 GLMB time step: predict, update, truncate, estimate, state import/export."""

    def __init__(self, params: dict, lib: str = None):
        L = _load(lib)
        self.params = dict(params)
        arr = np.array([float(params[k]) for k in PARAM_ORDER], dtype=np.float64)
        self._h = L.orc_create(arr.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
        self._L = L

    def __del__(self):
        if getattr(self, "_h", None):
            self._L.orc_destroy(self._h)
            self._h = None

    def set_hmax(self, h_max: int, tau: float):
        self._L.orc_set_hmax(self._h, int(h_max), float(tau))

    def import_state(self, s: dict):
        keep = []
        def I(a):
            a, p = _i32(a)
            keep.append(a)
            return p
        def D(a):
            a, p = _f64(a)
            keep.append(a)
            return p
        n_inst = int(np.asarray(s["inst_lab"]).reshape(-1, 2).shape[0])
        n_hyp = int(len(s["hyp_logw"]))
        n_b = int(np.asarray(s["birth_lab"]).reshape(-1, 2).shape[0])
        rc = self._L.orc_import(self._h, n_inst, I(s["inst_lab"]), D(s["inst_m"]), D(s["inst_P"]),
                                n_hyp, D(s["hyp_logw"]), I(s["hyp_off"]), I(s["hyp_idx"]), n_b,
                                I(s["birth_lab"]), D(s["birth_m"]), D(s["birth_P"]), D(s["birth_r"]))
        assert rc == 0

    def predict(self, k: int):
        assert self._L.orc_predict(self._h, int(k)) == 0

    def update(self, k: int, z: np.ndarray):
        z = np.ascontiguousarray(np.asarray(z, dtype=np.float32).astype(np.float64).reshape(-1, 2))
        assert self._L.orc_update(self._h, int(k), z.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  int(z.shape[0])) == 0

    def truncate(self, h_max: int, tau: float):
        assert self._L.orc_truncate(self._h, int(h_max), float(tau)) == 0

    def sizes(self):
        s = np.zeros(7, np.int64)
        self._L.orc_sizes(self._h, s.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)))
        return dict(n_inst=int(s[0]), n_hyp=int(s[1]), n_birth=int(s[2]), n_idx=int(s[3]),
                    M=int(s[4]), n_S=int(s[5]), n_pairs=int(s[6]))

    def export_state(self) -> dict:
        z = self.sizes()
        ni, nh, nb, nx, M = z["n_inst"], z["n_hyp"], z["n_birth"], z["n_idx"], z["M"]
        out = dict(
            inst_lab=np.zeros((ni, 2), np.int32), inst_m=np.zeros((ni, 4)), inst_P=np.zeros((ni, 16)),
            inst_src=np.zeros(ni, np.int32), S_off=np.zeros(ni + 1, np.int32),
            S_idx=np.zeros(max(z["n_S"], 1), np.int32),
            hyp_logw=np.zeros(nh), hyp_off=np.zeros(nh + 1, np.int32), hyp_idx=np.zeros(max(nx, 1), np.int32),
            hyp_parent=np.zeros(nh, np.int32), theta=np.zeros((nh, max(M, 1)), np.int32),
            birth_lab=np.zeros((nb, 2), np.int32), birth_m=np.zeros((nb, 4)), birth_P=np.zeros((nb, 16)),
            birth_r=np.zeros(nb),
        )
        P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32 if a.dtype == np.int32 else ctypes.c_double))
        self._L.orc_export(self._h, P(out["inst_lab"]), P(out["inst_m"]), P(out["inst_P"]), P(out["inst_src"]),
                           P(out["S_off"]), P(out["S_idx"]), P(out["hyp_logw"]), P(out["hyp_off"]),
                           P(out["hyp_idx"]), P(out["hyp_parent"]), P(out["theta"]), P(out["birth_lab"]),
                           P(out["birth_m"]), P(out["birth_P"]), P(out["birth_r"]))
        out["hyp_idx"] = out["hyp_idx"][:nx]
        out["S_idx"] = out["S_idx"][:z["n_S"]]
        out["theta"] = out["theta"][:, :M]
        return out

    def diag(self, n_parents: int):
        M = self.sizes()["M"]
        best, logpi = np.zeros(n_parents), np.zeros(n_parents)
        ru, scal = np.zeros(max(M, 1)), np.zeros(3)
        P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._L.orc_diag(self._h, P(best), P(logpi), P(ru), P(scal))
        return dict(best=best, logpi=logpi, ru=ru[:M], retained=scal[0], gated=int(scal[1]), lost=scal[2])

    def pairs(self):
        n = self.sizes()["n_pairs"]
        u, i = np.zeros(n, np.int32), np.zeros(n, np.int32)
        phi, mass, ex = np.zeros(n), np.zeros(n), np.zeros(n)
        I = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        D = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
        self._L.orc_pairs(self._h, I(u), I(i), D(phi), D(mass), D(ex))
        return dict(u=u, i=i, phi=phi, mass=mass, exist=ex)

    def set_skip(self, u: np.ndarray, i: np.ndarray):
        u, pu = _i32(u)
        i, pi = _i32(i)
        self._L.orc_set_skip(self._h, int(len(u)), pu, pi)

    def set_sampling(self, h_up: int, seed: int, margin: float = 1e-6):
        """Following updates draw h_up association maps per parent (the paper's generator)
        instead of the exact top-H_max; h_up = 0 restores the exact children."""
        self._L.orc_set_sampling(self._h, int(h_up), int(seed) & 0xFFFFFFFFFFFFFFFF, float(margin))

    def set_joint(self, on: bool):
        """Following updates reweight the kept hypotheses with the joint likelihood of every
        track's detection set (instead of the product of per-detection likelihoods)."""
        self._L.orc_set_joint(self._h, 1 if on else 0)

    def sample_stats(self, cap: int = 1 << 16):
        """(draws, distinct maps, parents with a draw within the margin of a boundary)."""
        c = np.zeros(2, np.int64)
        fr = np.zeros(cap, np.int32)
        n = self._L.orc_sample_stats(self._h, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                     fr.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)), cap)
        return int(c[0]), int(c[1]), fr[:min(n, cap)].tolist()

    def estimate(self, cap: int = 4096):
        n = np.zeros(1, np.int32)
        labs = np.zeros((cap, 2), np.int32)
        means = np.zeros((cap, 4))
        rho = np.zeros(cap + 1)
        rc = self._L.orc_estimate(self._h, int(cap), n.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  labs.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)),
                                  means.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                  rho.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), cap + 1)
        assert rc == 0
        k = int(n[0])
        return labs[:k].copy(), means[:k].copy(), rho


def to_f32_state(s: dict) -> dict:
    """Round a state's floating-point arrays to float32 (and back to float64)."""
    out = dict(s)
    for k in ("inst_m", "inst_P", "hyp_logw", "birth_m", "birth_P", "birth_r"):
        out[k] = np.asarray(s[k], dtype=np.float32).astype(np.float64)
    return out


def philox4x32_10(ctr, key, lib: str = None):
    """The oracle's Philox4x32-10 block: four 32-bit words from a 4-word counter and 2-word key."""
    L = _load(lib)
    c = np.ascontiguousarray(ctr, np.uint32)
    k = np.ascontiguousarray(key, np.uint32)
    out = np.zeros(4, np.uint32)
    P = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32))
    L.orc_philox(P(c), P(k), P(out))
    return out


def philox_uniform(seed: int, a: int, b: int, c: int, stream: int, lib: str = None) -> float:
    return float(_load(lib).orc_philox_uniform(int(seed) & 0xFFFFFFFFFFFFFFFF, a, b, c, stream))


def joint_loglik(sigma: float, z, m, P, lib: str = None) -> float:
    """The oracle's joint log-likelihood of detections z [n, 2] given a track N(m, P)."""
    L = _load(lib)
    z, pz = _f64(np.asarray(z, np.float64).reshape(-1, 2))
    m, pm = _f64(np.asarray(m, np.float64).reshape(4))
    P, pP = _f64(np.asarray(P, np.float64).reshape(16))
    return float(L.orc_joint_loglik(float(sigma), int(z.shape[0]), pz, pm, pP))


# ---- particle form (component-major states [5][n], log weights [n]) ----
def pf_predict(st, dt: float, sigma_a: float, sigma_w: float, seed: int, k: int, lib: str = None):
    """The oracle's constant-turn-rate-and-velocity prediction of every particle (a copy)."""
    out = np.ascontiguousarray(np.array(st, np.float64).reshape(5, -1))
    _load(lib).orc_pf_predict(out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), out.shape[1], float(dt),
                              float(sigma_a), float(sigma_w), int(seed) & 0xFFFFFFFFFFFFFFFF, int(k))
    return out


def pf_loglik(st, lw, U: int, P: int, z, sigma: float, gamma: float, gate: float, lib: str = None):
    """phi [U][M] of particle tracks (-inf outside the gate)."""
    st, pst = _f64(np.asarray(st, np.float64).reshape(5, -1))
    lw, plw = _f64(np.asarray(lw, np.float64).reshape(-1))
    z, pz = _f64(np.asarray(z, np.float64).reshape(-1, 2))
    phi = np.zeros((U, z.shape[0]))
    _load(lib).orc_pf_loglik(pst, plw, U, P, pz, z.shape[0], float(sigma), float(gamma), float(gate),
                             phi.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return phi


def pf_update(st, lw, U: int, P: int, rec_u, rec_off, rec_z, z, sigma: float, ess_frac: float, seed: int, k: int,
              margin: float = 1e-6, lib: str = None):
    """(states [5][R P], log weights [R P], resampled [R], fragile [R]) of the particle update."""
    st, pst = _f64(np.asarray(st, np.float64).reshape(5, -1))
    lw, plw = _f64(np.asarray(lw, np.float64).reshape(-1))
    z, pz = _f64(np.asarray(z, np.float64).reshape(-1, 2))
    ru, pru = _i32(rec_u)
    ro, pro = _i32(rec_off)
    rz, prz = _i32(rec_z if len(rec_z) else np.zeros(1, np.int32))
    R = len(ru)
    ost = np.zeros((5, R * P))
    olw = np.zeros(R * P)
    rs = np.zeros(R, np.int32)
    fr = np.zeros(R, np.int32)
    D = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))
    I = lambda a: a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
    _load(lib).orc_pf_update(pst, plw, U, P, R, pru, pro, prz, pz, float(sigma), float(ess_frac),
                             int(seed) & 0xFFFFFFFFFFFFFFFF, int(k), float(margin), D(ost), D(olw), I(rs), I(fr))
    return ost, olw, rs, fr
