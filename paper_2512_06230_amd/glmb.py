"""Thin ctypes binding of ``libglmb.so`` (the C ABI declared in ``include/glmb.h``).

Argument marshalling only: every step of the filter runs in the library's HIP kernels.
PyTorch supplies device memory (the detections) and the stream.  There is no fallback:
if the library is missing or no GPU is present, construction raises.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libglmb.so")

GLMB_OK, GLMB_E_ARG, GLMB_E_CAPACITY, GLMB_E_NOMEM, GLMB_E_DEVICE, GLMB_E_STATE = 0, -1, -2, -3, -4, -5

EXPORTS = ["glmb_status_string", "glmb_last_error", "glmb_create", "glmb_destroy", "glmb_import_state",
           "glmb_state_sizes", "glmb_export_state", "glmb_predict", "glmb_update", "glmb_truncate",
           "glmb_estimate", "glmb_stats", "glmb_update_diag", "glmb_update_theta", "glmb_set_proposal",
           "glmb_pair_features", "glmb_proposal_lost", "glmb_mlp_forward", "glmb_mlp_grad", "glmb_mlp_adam",
           "glmb_mlp_grad_noalloc", "glmb_set_sampling", "glmb_set_joint_reweighting",
           "glmb_pf_predict", "glmb_pf_loglik", "glmb_pf_update",
           "glmb_batch_create", "glmb_batch_destroy", "glmb_batch_set_schedule", "glmb_batch_scene",
           "glmb_batch_step", "glmb_batch_stats_get", "glmb_batch_last_error"]

MLP_NPARAM, MLP_NFEAT = 4673, 6
MLP_NOALLOC_MAX = 32768
PROPOSAL_APPLY, PROPOSAL_MEASURE = 1, 2


class Params(ctypes.Structure):
    _fields_ = [("dt", ctypes.c_float), ("q", ctypes.c_float), ("sigma_z", ctypes.c_float),
                ("p_survive", ctypes.c_float), ("det_rate", ctypes.c_float), ("clutter_density", ctypes.c_float),
                ("gate_d2", ctypes.c_float), ("birth_r_max", ctypes.c_float), ("birth_rate", ctypes.c_float),
                ("birth_sigma_v", ctypes.c_float), ("birth_ru_max", ctypes.c_float),
                ("birth_cluster_d", ctypes.c_float), ("h_max", ctypes.c_int32), ("tau", ctypes.c_float),
                ("cap_nodes", ctypes.c_int32), ("cap_labels", ctypes.c_int32)]


_I = ctypes.POINTER(ctypes.c_int32)
_F = ctypes.POINTER(ctypes.c_float)


class StateHost(ctypes.Structure):
    _fields_ = [("n_inst", ctypes.c_int32), ("n_hyp", ctypes.c_int32), ("n_idx", ctypes.c_int32),
                ("n_birth", ctypes.c_int32), ("inst_lab", _I), ("inst_m", _F), ("inst_P", _F), ("inst_src", _I),
                ("inst_nz", _I), ("inst_z", _I), ("hyp_logw", _F), ("hyp_off", _I), ("hyp_idx", _I),
                ("hyp_parent", _I), ("birth_lab", _I), ("birth_m", _F), ("birth_P", _F), ("birth_r", _F)]


class StepStats(ctypes.Structure):
    _fields_ = [("n_hyp_in", ctypes.c_int32), ("n_hyp_out", ctypes.c_int32), ("n_meas", ctypes.c_int32),
                ("n_inst_in", ctypes.c_int32), ("n_inst_out", ctypes.c_int32), ("n_labels", ctypes.c_int32),
                ("gated_pairs", ctypes.c_int64), ("option_terms", ctypes.c_int64),
                ("dense_triples", ctypes.c_int64), ("search_nodes", ctypes.c_int32),
                ("search_levels", ctypes.c_int32), ("n_births", ctypes.c_int32),
                ("retained_mass", ctypes.c_double), ("lost_mass", ctypes.c_double),
                ("pairs_removed", ctypes.c_int32), ("stage_ms", ctypes.c_float * 6),
                ("rec_collisions", ctypes.c_int32), ("host_syncs", ctypes.c_int32),
                ("search_form", ctypes.c_int32)]


class BatchStats(ctypes.Structure):
    _fields_ = [("n_scenes", ctypes.c_int32), ("workers", ctypes.c_int32), ("longest_first", ctypes.c_int32),
                ("step_ms", ctypes.c_float), ("scene_updates_per_s", ctypes.c_double),
                ("first_error_scene", ctypes.c_int32)]


_lib = None


def load_library(path: str = LIB_PATH):
    """Load libglmb.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError("libglmb.so is not built: run `python paper_2512_06230_amd/build.py`")
    L = ctypes.CDLL(path)
    vp = ctypes.c_void_p
    L.glmb_status_string.restype = ctypes.c_char_p
    L.glmb_status_string.argtypes = [ctypes.c_int]
    L.glmb_last_error.restype = ctypes.c_char_p
    L.glmb_last_error.argtypes = [vp]
    L.glmb_create.argtypes = [ctypes.POINTER(Params), ctypes.c_int, vp, ctypes.POINTER(vp)]
    L.glmb_destroy.argtypes = [vp]
    L.glmb_import_state.argtypes = [vp, ctypes.POINTER(StateHost)]
    L.glmb_state_sizes.argtypes = [vp, _I, _I, _I, _I]
    L.glmb_export_state.argtypes = [vp, ctypes.POINTER(StateHost)]
    L.glmb_predict.argtypes = [vp, ctypes.c_int32]
    L.glmb_update.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32]
    L.glmb_truncate.argtypes = [vp, ctypes.c_int32, ctypes.c_float]
    L.glmb_estimate.argtypes = [vp, ctypes.c_int32, _I, _I, _F]
    L.glmb_stats.argtypes = [vp, ctypes.POINTER(StepStats)]
    L.glmb_update_diag.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, _F, _F, _F]
    L.glmb_update_theta.argtypes = [vp, ctypes.c_int32, ctypes.c_int32, _I]
    L.glmb_set_proposal.argtypes = [vp, vp, _F, ctypes.c_float, ctypes.c_int32]
    L.glmb_pair_features.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp, vp, _I]
    L.glmb_proposal_lost.argtypes = [vp, ctypes.c_int32, vp, ctypes.c_int32, ctypes.c_int32, _F,
                                     ctypes.POINTER(ctypes.c_double)]
    L.glmb_mlp_forward.argtypes = [vp, vp, _F, vp, ctypes.c_int32, vp]
    L.glmb_mlp_grad.argtypes = [vp, vp, _F, vp, vp, vp, ctypes.c_int32, vp, vp]
    L.glmb_mlp_grad_noalloc.argtypes = [vp, vp, _F, vp, vp, vp, ctypes.c_int32, vp, vp]
    L.glmb_set_sampling.argtypes = [vp, ctypes.c_int32, ctypes.c_uint64]
    L.glmb_set_joint_reweighting.argtypes = [vp, ctypes.c_int32]
    f, i32, u64 = ctypes.c_float, ctypes.c_int32, ctypes.c_uint64
    L.glmb_pf_predict.argtypes = [vp, vp, ctypes.c_int64, f, f, f, u64, i32]
    L.glmb_pf_loglik.argtypes = [vp, vp, vp, i32, i32, vp, i32, f, f, f, vp]
    L.glmb_pf_update.argtypes = [vp, vp, vp, i32, i32, i32, vp, vp, vp, vp, i32, f, f, u64, i32, vp, vp, vp]
    L.glmb_mlp_adam.argtypes = [vp, vp, vp, vp, vp, ctypes.c_int32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float]
    L.glmb_batch_create.argtypes = [ctypes.c_int32, ctypes.POINTER(Params), ctypes.c_int, ctypes.c_int32,
                                    ctypes.POINTER(vp)]
    L.glmb_batch_destroy.argtypes = [vp]
    L.glmb_batch_set_schedule.argtypes = [vp, ctypes.c_int32, ctypes.c_int32]
    L.glmb_batch_scene.argtypes = [vp, ctypes.c_int32, ctypes.POINTER(vp)]
    L.glmb_batch_step.argtypes = [vp, ctypes.c_int32, vp, _I, vp]
    L.glmb_batch_stats_get.argtypes = [vp, ctypes.POINTER(BatchStats)]
    L.glmb_batch_last_error.argtypes = [vp]
    for name in EXPORTS:
        getattr(L, name).restype = ctypes.c_int if name not in ("glmb_status_string", "glmb_last_error",
                                                                "glmb_batch_last_error") else ctypes.c_char_p
    _lib = L
    return L


class GlmbError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__("%s (%d): %s" % (msg, status, msg))
        self.status = status


def _params(p: dict) -> Params:
    return Params(dt=p["dt"], q=p["q"], sigma_z=p["sigma_z"], p_survive=p["p_survive"], det_rate=p["det_rate"],
                  clutter_density=p["clutter_density"], gate_d2=p["gate_d2"], birth_r_max=p["birth_r_max"],
                  birth_rate=p["birth_rate"], birth_sigma_v=p["birth_sigma_v"], birth_ru_max=p["birth_ru_max"],
                  birth_cluster_d=p["birth_cluster_d"], h_max=int(p["h_max"]), tau=float(p["tau"]),
                  cap_nodes=int(p.get("cap_nodes", 0)), cap_labels=int(p.get("cap_labels", 0)))


def _ip(a):
    return a.ctypes.data_as(_I)


def _fp(a):
    return a.ctypes.data_as(_F)


class Tracker:
    """One filter context on a HIP device, driven on a torch stream."""

    def __init__(self, params: dict, device: int = 0, stream=None, _ctx=None, _owner=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the GLMB library runs on the GPU only")
        self._L = load_library()
        self.torch = torch
        self.device = device
        self.params = dict(params)
        if _ctx is not None:  # a context owned by a Batch
            self._ctx = _ctx
            self._owner = _owner
            return
        self.stream = stream if stream is not None else torch.cuda.current_stream(device)
        ctx = ctypes.c_void_p()
        st = self._L.glmb_create(ctypes.byref(_params(params)), device, ctypes.c_void_p(self.stream.cuda_stream),
                                 ctypes.byref(ctx))
        if st != GLMB_OK:
            raise GlmbError(st, "glmb_create: " + self._L.glmb_status_string(st).decode())
        self._ctx = ctx

    def _check(self, st: int, what: str):
        if st != GLMB_OK:
            raise GlmbError(st, "%s: %s" % (what, self._L.glmb_last_error(self._ctx).decode()))

    def close(self):
        if getattr(self, "_ctx", None):
            if getattr(self, "_owner", None) is None:
                self._L.glmb_destroy(self._ctx)
            self._ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---- state
    def import_state(self, s: dict):
        lab = np.ascontiguousarray(np.asarray(s["inst_lab"], np.int32).reshape(-1, 2))
        m = np.ascontiguousarray(np.asarray(s["inst_m"], np.float32).reshape(-1, 4))
        P = np.ascontiguousarray(np.asarray(s["inst_P"], np.float32).reshape(-1, 16))
        lw = np.ascontiguousarray(np.asarray(s["hyp_logw"], np.float32))
        off = np.ascontiguousarray(np.asarray(s["hyp_off"], np.int32))
        idx = np.ascontiguousarray(np.asarray(s["hyp_idx"], np.int32))
        blab = np.ascontiguousarray(np.asarray(s["birth_lab"], np.int32).reshape(-1, 2))
        bm = np.ascontiguousarray(np.asarray(s["birth_m"], np.float32).reshape(-1, 4))
        bP = np.ascontiguousarray(np.asarray(s["birth_P"], np.float32).reshape(-1, 16))
        br = np.ascontiguousarray(np.asarray(s["birth_r"], np.float32))
        h = StateHost(n_inst=lab.shape[0], n_hyp=lw.shape[0], n_idx=idx.shape[0], n_birth=blab.shape[0],
                      inst_lab=_ip(lab), inst_m=_fp(m), inst_P=_fp(P), hyp_logw=_fp(lw), hyp_off=_ip(off),
                      hyp_idx=_ip(idx), birth_lab=_ip(blab), birth_m=_fp(bm), birth_P=_fp(bP), birth_r=_fp(br))
        self._check(self._L.glmb_import_state(self._ctx, ctypes.byref(h)), "glmb_import_state")

    def sizes(self):
        a = [ctypes.c_int32() for _ in range(4)]
        self._check(self._L.glmb_state_sizes(self._ctx, *[ctypes.byref(x) for x in a]), "glmb_state_sizes")
        return dict(n_inst=a[0].value, n_hyp=a[1].value, n_idx=a[2].value, n_birth=a[3].value)

    def export_state(self) -> dict:
        z = self.sizes()
        ni, nh, nx, nb = z["n_inst"], z["n_hyp"], z["n_idx"], z["n_birth"]
        out = dict(inst_lab=np.zeros((ni, 2), np.int32), inst_m=np.zeros((ni, 4), np.float32),
                   inst_P=np.zeros((ni, 16), np.float32), inst_src=np.zeros(ni, np.int32),
                   inst_nz=np.zeros(ni, np.int32), inst_z=np.zeros((ni, 8), np.int32),
                   hyp_logw=np.zeros(nh, np.float32), hyp_off=np.zeros(nh + 1, np.int32),
                   hyp_idx=np.zeros(max(nx, 1), np.int32), hyp_parent=np.zeros(nh, np.int32),
                   birth_lab=np.zeros((nb, 2), np.int32), birth_m=np.zeros((nb, 4), np.float32),
                   birth_P=np.zeros((nb, 16), np.float32), birth_r=np.zeros(nb, np.float32))
        h = StateHost(n_inst=ni, n_hyp=nh, n_idx=max(nx, 1), n_birth=nb, inst_lab=_ip(out["inst_lab"]),
                      inst_m=_fp(out["inst_m"]), inst_P=_fp(out["inst_P"]), inst_src=_ip(out["inst_src"]),
                      inst_nz=_ip(out["inst_nz"]), inst_z=_ip(out["inst_z"]), hyp_logw=_fp(out["hyp_logw"]),
                      hyp_off=_ip(out["hyp_off"]), hyp_idx=_ip(out["hyp_idx"]), hyp_parent=_ip(out["hyp_parent"]),
                      birth_lab=_ip(out["birth_lab"]), birth_m=_fp(out["birth_m"]), birth_P=_fp(out["birth_P"]),
                      birth_r=_fp(out["birth_r"]))
        self._check(self._L.glmb_export_state(self._ctx, ctypes.byref(h)), "glmb_export_state")
        out["hyp_idx"] = out["hyp_idx"][:nx]
        return out

    # ---- the time step
    def predict(self, k: int):
        self._check(self._L.glmb_predict(self._ctx, int(k)), "glmb_predict")

    def update(self, k: int, z):
        """z: torch CUDA float32 tensor [M, 2] (contiguous) or a numpy array (copied to the device)."""
        t = self.torch
        if not isinstance(z, t.Tensor):
            z = t.as_tensor(np.ascontiguousarray(np.asarray(z, np.float32).reshape(-1, 2)), device="cuda")
        if not (z.is_cuda and z.dtype == t.float32 and z.is_contiguous() and z.dim() == 2 and z.shape[1] == 2):
            raise ValueError("detections must be a contiguous CUDA float32 tensor of shape [M, 2]")
        self._z_keep = z
        self._check(self._L.glmb_update(self._ctx, int(k), ctypes.c_void_p(z.data_ptr()), int(z.shape[0])),
                    "glmb_update")

    def truncate(self, h_max: int, tau: float):
        self._check(self._L.glmb_truncate(self._ctx, int(h_max), float(tau)), "glmb_truncate")

    def estimate(self, cap: int = 65536):
        n = ctypes.c_int32()
        labs = np.empty((cap, 2), np.int32)  # the library fills the first n rows
        means = np.empty((cap, 4), np.float32)
        self._check(self._L.glmb_estimate(self._ctx, int(cap), ctypes.byref(n), _ip(labs), _fp(means)),
                    "glmb_estimate")
        return labs[:n.value].copy(), means[:n.value].copy()

    def stats(self) -> dict:
        s = StepStats()
        self._check(self._L.glmb_stats(self._ctx, ctypes.byref(s)), "glmb_stats")
        out = {f: getattr(s, f) for f, _ in StepStats._fields_}
        out["stage_ms"] = list(s.stage_ms)
        return out

    def diag(self, H: int, M: int) -> dict:
        best, logpi = np.zeros(H, np.float32), np.zeros(H, np.float32)
        ru = np.zeros(max(M, 1), np.float32)
        self._check(self._L.glmb_update_diag(self._ctx, int(H), int(M), _fp(best), _fp(logpi), _fp(ru)),
                    "glmb_update_diag")
        return dict(best=best, logpi=logpi, ru=ru[:M])

    def theta(self, n_hyp: int, M: int) -> np.ndarray:
        th = np.zeros((n_hyp, max(M, 1)), np.int32)
        self._check(self._L.glmb_update_theta(self._ctx, int(n_hyp), int(M), _ip(th)), "glmb_update_theta")
        return th[:, :M]

    # ---- learned pair proposal
    def to_device(self, a, dtype=np.float32):
        """A CUDA tensor copy of a host array."""
        return self.torch.as_tensor(np.ascontiguousarray(np.asarray(a, dtype)), device="cuda")

    @staticmethod
    def to_host(t) -> np.ndarray:
        return t.detach().cpu().numpy()

    def _dev(self, a, shape, dtype=None):
        t = self.torch
        dtype = dtype or t.float32
        if not isinstance(a, t.Tensor):
            a = t.as_tensor(np.ascontiguousarray(a), device="cuda")
        if not (a.is_cuda and a.dtype == dtype and a.is_contiguous() and tuple(a.shape) == tuple(shape)):
            raise ValueError("expected a contiguous CUDA %s tensor of shape %s" % (dtype, tuple(shape)))
        return a

    def _z(self, z):
        t = self.torch
        if not isinstance(z, t.Tensor):
            z = t.as_tensor(np.ascontiguousarray(np.asarray(z, np.float32).reshape(-1, 2)), device="cuda")
        return self._dev(z, (z.shape[0], 2))

    @staticmethod
    def _norm(norm):
        n = np.ascontiguousarray(np.asarray(norm, np.float32).reshape(12))
        return n

    def set_sampling(self, h_up: int, seed: int = 0):
        """Following updates keep the distinct maps among h_up drawn per hypothesis (the paper's
        generator) instead of the exact h_max best; h_up = 0 restores the exact update."""
        self._check(self._L.glmb_set_sampling(self._ctx, int(h_up), int(seed) & 0xFFFFFFFFFFFFFFFF),
                    "glmb_set_sampling")

    def set_joint_reweighting(self, on: bool = True):
        """Following updates reweight the kept hypotheses with the joint likelihood of every
        track's detection set (re-ranked, tau, renormalised); False restores the factorised weights."""
        self._check(self._L.glmb_set_joint_reweighting(self._ctx, 1 if on else 0), "glmb_set_joint_reweighting")

    def set_proposal(self, params, norm, threshold: float = 0.5, apply: bool = True, measure: bool = False):
        """params: CUDA float32 [4673] (None unloads the proposal); norm: 12 floats.
        apply: the following updates remove low-scoring pairs; measure: they also report the
        lost posterior mass.  With apply=False the parameters serve proposal_lost only."""
        if params is None:
            self._check(self._L.glmb_set_proposal(self._ctx, None, None, 0.5, 0), "glmb_set_proposal")
            return
        params = self._dev(params, (MLP_NPARAM,))
        n = self._norm(norm)
        flags = (PROPOSAL_APPLY if apply else 0) | (PROPOSAL_MEASURE if measure else 0)
        self._check(self._L.glmb_set_proposal(self._ctx, ctypes.c_void_p(params.data_ptr()), _fp(n),
                                              float(threshold), flags), "glmb_set_proposal")

    def pair_features(self, k: int, z, cap: int = 0):
        """Training data of the current predicted state: (feat [n,6], pair [n,2], target [n],
        weight [n]) as CUDA tensors."""
        t = self.torch
        z = self._z(z)
        cap = max(int(cap), getattr(self, "_pair_cap", 4096))
        for _ in range(2):
            feat = t.empty((cap, MLP_NFEAT), dtype=t.float32, device="cuda")
            pair = t.empty((cap, 2), dtype=t.int32, device="cuda")
            y = t.empty(cap, dtype=t.float32, device="cuda")
            w = t.empty(cap, dtype=t.float32, device="cuda")
            n = ctypes.c_int32()
            st = self._L.glmb_pair_features(self._ctx, int(k), ctypes.c_void_p(z.data_ptr()), int(z.shape[0]), cap,
                                            ctypes.c_void_p(feat.data_ptr()), ctypes.c_void_p(pair.data_ptr()),
                                            ctypes.c_void_p(y.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                                            ctypes.byref(n))
            if st == GLMB_E_CAPACITY and n.value > cap:
                cap = self._pair_cap = n.value
                continue
            self._check(st, "glmb_pair_features")
            m = n.value
            return feat[:m], pair[:m], y[:m], w[:m]
        raise GlmbError(GLMB_E_CAPACITY, "glmb_pair_features: pair count changed between calls")

    def proposal_lost(self, k: int, z, thresholds) -> np.ndarray:
        z = self._z(z)
        thr = np.ascontiguousarray(np.asarray(thresholds, np.float32).reshape(-1))
        out = np.zeros(len(thr), np.float64)
        self._check(self._L.glmb_proposal_lost(self._ctx, int(k), ctypes.c_void_p(z.data_ptr()), int(z.shape[0]),
                                               len(thr), _fp(thr), out.ctypes.data_as(ctypes.POINTER(ctypes.c_double))),
                    "glmb_proposal_lost")
        return out

    def mlp_forward(self, params, norm, feat):
        t = self.torch
        params = self._dev(params, (MLP_NPARAM,))
        feat = self._dev(feat, (feat.shape[0], MLP_NFEAT))
        n = self._norm(norm)
        out = t.empty(feat.shape[0], dtype=t.float32, device="cuda")
        self._check(self._L.glmb_mlp_forward(self._ctx, ctypes.c_void_p(params.data_ptr()), _fp(n),
                                             ctypes.c_void_p(feat.data_ptr()), int(feat.shape[0]),
                                             ctypes.c_void_p(out.data_ptr())), "glmb_mlp_forward")
        return out

    def mlp_grad(self, params, norm, feat, y, w):
        """(grad [4673], loss [1]) CUDA tensors of the weighted cross-entropy."""
        t = self.torch
        params = self._dev(params, (MLP_NPARAM,))
        feat = self._dev(feat, (feat.shape[0], MLP_NFEAT))
        y = self._dev(y, (feat.shape[0],))
        w = self._dev(w, (feat.shape[0],))
        n = self._norm(norm)
        g = t.empty(MLP_NPARAM, dtype=t.float32, device="cuda")
        loss = t.empty(1, dtype=t.float32, device="cuda")
        self._check(self._L.glmb_mlp_grad(self._ctx, ctypes.c_void_p(params.data_ptr()), _fp(n),
                                          ctypes.c_void_p(feat.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                          ctypes.c_void_p(w.data_ptr()), int(feat.shape[0]),
                                          ctypes.c_void_p(g.data_ptr()), ctypes.c_void_p(loss.data_ptr())),
                    "glmb_mlp_grad")
        return g, loss

    def mlp_grad_noalloc(self, params, norm, feat, y, w, grad_out, loss_out):
        """glmb_mlp_grad_noalloc into the caller's CUDA float32 tensors grad_out [4673] and
        loss_out [1]; every input must already be a contiguous CUDA float32 tensor, so that
        nothing is allocated on the way (at most MLP_NOALLOC_MAX samples)."""
        t = self.torch
        n = int(feat.shape[0])
        for a, shape in ((params, (MLP_NPARAM,)), (feat, (n, MLP_NFEAT)), (y, (n,)), (w, (n,)),
                         (grad_out, (MLP_NPARAM,)), (loss_out, (1,))):
            if not (a.is_cuda and a.dtype == t.float32 and a.is_contiguous() and tuple(a.shape) == shape):
                raise ValueError("mlp_grad_noalloc takes contiguous CUDA float32 tensors of the stated shapes")
        nm = self._norm(norm)
        self._check(self._L.glmb_mlp_grad_noalloc(self._ctx, ctypes.c_void_p(params.data_ptr()), _fp(nm),
                                                  ctypes.c_void_p(feat.data_ptr()), ctypes.c_void_p(y.data_ptr()),
                                                  ctypes.c_void_p(w.data_ptr()), n,
                                                  ctypes.c_void_p(grad_out.data_ptr()),
                                                  ctypes.c_void_p(loss_out.data_ptr())), "glmb_mlp_grad_noalloc")

    def mlp_adam(self, params, m, v, g, step: int, lr: float, beta1: float = 0.9, beta2: float = 0.999,
                 eps: float = 1e-8):
        """One Adam step, in place on params, m and v (CUDA float32 [4673] each)."""
        ps = [self._dev(a, (MLP_NPARAM,)) for a in (params, m, v, g)]
        self._check(self._L.glmb_mlp_adam(self._ctx, *[ctypes.c_void_p(a.data_ptr()) for a in ps], int(step),
                                          float(lr), float(beta1), float(beta2), float(eps)), "glmb_mlp_adam")


class Batch:
    """Many independent scenes advanced one time step per call (glmb_batch_*)."""

    def __init__(self, params_list, device: int = 0, workers: int = 4):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU: the GLMB library runs on the GPU only")
        self._L = load_library()
        self.torch = torch
        self.params = [dict(p) for p in params_list]
        arr = (Params * len(self.params))(*[_params(p) for p in self.params])
        b = ctypes.c_void_p()
        st = self._L.glmb_batch_create(len(self.params), arr, device, int(workers), ctypes.byref(b))
        if st != GLMB_OK:
            raise GlmbError(st, "glmb_batch_create: " + self._L.glmb_status_string(st).decode())
        self._b = b
        self.n = len(self.params)

    def _check(self, st: int, what: str):
        if st != GLMB_OK:
            raise GlmbError(st, "%s: %s" % (what, self._L.glmb_batch_last_error(self._b).decode()))

    def scene(self, i: int) -> Tracker:
        """The scene's context as a Tracker (owned by the batch)."""
        ctx = ctypes.c_void_p()
        self._check(self._L.glmb_batch_scene(self._b, int(i), ctypes.byref(ctx)), "glmb_batch_scene")
        return Tracker(self.params[i], _ctx=ctx, _owner=self)

    def set_schedule(self, workers: int, longest_first: bool = True):
        self._check(self._L.glmb_batch_set_schedule(self._b, int(workers), int(bool(longest_first))),
                    "glmb_batch_set_schedule")

    def step(self, k: int, z, z_off):
        """z: CUDA float32 [total, 2] (all scenes' detections, concatenated); z_off: host int [n+1]."""
        t = self.torch
        if not (isinstance(z, t.Tensor) and z.is_cuda and z.dtype == t.float32 and z.is_contiguous()
                and z.dim() == 2 and z.shape[1] == 2):
            raise ValueError("detections must be a contiguous CUDA float32 tensor of shape [total, 2]")
        off = np.ascontiguousarray(np.asarray(z_off, np.int32).reshape(-1))
        if off.shape[0] != self.n + 1:
            raise ValueError("z_off must hold n + 1 offsets")
        self._z_keep = z
        stream = t.cuda.current_stream(z.device).cuda_stream  # where z was written
        self._check(self._L.glmb_batch_step(self._b, int(k), ctypes.c_void_p(z.data_ptr()), _ip(off),
                                            ctypes.c_void_p(stream)), "glmb_batch_step")

    def stats(self) -> dict:
        s = BatchStats()
        self._check(self._L.glmb_batch_stats_get(self._b, ctypes.byref(s)), "glmb_batch_stats_get")
        return {f: getattr(s, f) for f, _ in BatchStats._fields_}

    def close(self):
        if getattr(self, "_b", None):
            self._L.glmb_batch_destroy(self._b)
            self._b = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ---- particle form (stateless calls on torch's current stream) ----------------------------
def _stream_ptr(torch):
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _need(t, dtype, shape, what):
    import torch
    if not (t.is_cuda and t.dtype == dtype and t.is_contiguous() and tuple(t.shape) == tuple(shape)):
        raise ValueError("%s: contiguous CUDA %s tensor of shape %s expected" % (what, dtype, tuple(shape)))
    return ctypes.c_void_p(t.data_ptr())


def pf_predict(state, dt: float, sigma_a: float, sigma_w: float, seed: int, k: int):
    """CTRV prediction of every particle, in place (state: CUDA float32 [5, n])."""
    import torch
    L = load_library()
    n = int(state.shape[1])
    st = L.glmb_pf_predict(_stream_ptr(torch), _need(state, torch.float32, (5, n), "state"), n, float(dt),
                           float(sigma_a), float(sigma_w), int(seed) & 0xFFFFFFFFFFFFFFFF, int(k))
    if st != GLMB_OK:
        raise GlmbError(st, "glmb_pf_predict: " + L.glmb_status_string(st).decode())


def pf_loglik(state, logw, U: int, P: int, z, sigma: float, gamma: float, gate: float):
    """phi [U, M] (CUDA float32) of particle tracks."""
    import torch
    L = load_library()
    M = int(z.shape[0])
    phi = torch.empty((U, M), dtype=torch.float32, device=state.device)
    st = L.glmb_pf_loglik(_stream_ptr(torch), _need(state, torch.float32, (5, U * P), "state"),
                          _need(logw, torch.float32, (U * P,), "logw"), int(U), int(P),
                          _need(z, torch.float32, (M, 2), "z"), M, float(sigma), float(gamma), float(gate),
                          ctypes.c_void_p(phi.data_ptr()))
    if st != GLMB_OK:
        raise GlmbError(st, "glmb_pf_loglik: " + L.glmb_status_string(st).decode())
    return phi


def pf_update(state, logw, U: int, P: int, rec_u, rec_off, rec_z, z, sigma: float, ess_frac: float, seed: int, k: int,
              out=None):
    """(out_state [5, R P], out_logw [R P], resampled [R]) CUDA tensors of the particle update;
    `out` may hold preallocated (out_state, out_logw, resampled)."""
    import torch
    L = load_library()
    R = int(rec_u.shape[0])
    M = int(z.shape[0])
    if out is None:
        out = (torch.empty((5, R * P), dtype=torch.float32, device=state.device),
               torch.empty((R * P,), dtype=torch.float32, device=state.device),
               torch.empty((R,), dtype=torch.int32, device=state.device))
    ost, olw, rs = out
    rz = rec_z if rec_z.numel() else torch.zeros(1, dtype=torch.int32, device=state.device)
    st = L.glmb_pf_update(_stream_ptr(torch), _need(state, torch.float32, (5, U * P), "state"),
                          _need(logw, torch.float32, (U * P,), "logw"), int(U), int(P), R,
                          _need(rec_u, torch.int32, (R,), "rec_u"), _need(rec_off, torch.int32, (R + 1,), "rec_off"),
                          ctypes.c_void_p(rz.data_ptr()), _need(z, torch.float32, (M, 2), "z"), M, float(sigma),
                          float(ess_frac), int(seed) & 0xFFFFFFFFFFFFFFFF, int(k),
                          _need(ost, torch.float32, (5, R * P), "out_state"),
                          _need(olw, torch.float32, (R * P,), "out_logw"), _need(rs, torch.int32, (R,), "resampled"))
    if st != GLMB_OK:
        raise GlmbError(st, "glmb_pf_update: " + L.glmb_status_string(st).decode())
    return ost, olw, rs
