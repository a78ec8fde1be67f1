"""Benchmark of the multi-detection GLMB time step on one MI355X.

A step is one pass of the whole hot path over one scan of synthetic detections:
glmb_predict -> glmb_update -> glmb_truncate -> glmb_estimate, on the N=500-object,
H_max=1e4 workload (100x100 m, clutter 100 per scan, warm start).  All scans are
uploaded to HBM before the timed region.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "GLMB updates/s and hyp·track·meas evals/s, N=500 H_max=1e4; learned vs plain"
HBM_PEAK_GBS = 8000.0       # MI355X HBM3E
FP32_VECTOR_TFLOPS = 157.3  # MI355X FP32 vector: 256 CUs x 128 lanes x 2 flops (FMA) x 2.4 GHz
TRANS_PER_S = 9.8e12        # transcendental (exp / log) rate, assumed a quarter of the unpacked FP32 FMA rate
INST_BYTES = 64             # one track instance record (mean, covariance, label slot, source)


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def stage_roofline(stats, stage):
    """Algorithmic lower bound on each update stage's time (mean over the timed updates), from
    the work the method needs per unit: U1 14 FP32 flops per (instance, detection) pair; U2 one
    read of every hypothesis row (|J| x 4 B) and two floats written per hypothesis (best child,
    log mass) for hypotheses 1..H-1 (the association kernel's share); U4 the predicted rows read,
    the child rows written and one record per new instance; births one exp per (hypothesis,
    detection) cell.  The cut (U3) is a chain of dependent levels: time only."""
    import numpy as np
    H = np.mean([s["n_hyp_in"] for s in stats])
    Ho = np.mean([s["n_hyp_out"] for s in stats])
    M = np.mean([s["n_meas"] for s in stats])
    U = np.mean([s["n_inst_in"] for s in stats])
    Uo = np.mean([s["n_inst_out"] for s in stats])
    J = np.mean([s["dense_triples"] / max(1, s["n_hyp_in"] * s["n_meas"]) for s in stats])
    hbm = HBM_PEAK_GBS * 1e9
    valu = FP32_VECTOR_TFLOPS * 1e12
    out = {}
    f_gate = 14.0 * U * M
    out["gate"] = {"bound": "alu", "work": f_gate, "unit": "FP32 flop", "t_roof_ms": 1e3 * f_gate / valu}
    b_assoc = (H - 1.0) * J * 4.0 + 8.0 * (H - 1.0)
    out["assoc"] = {"bound": "hbm", "work": b_assoc, "unit": "B", "t_roof_ms": 1e3 * b_assoc / hbm}
    out["select"] = {"bound": "latency", "work": None, "unit": None, "t_roof_ms": None}
    b_mat = (H + Ho) * J * 4.0 + Uo * INST_BYTES
    out["materialise"] = {"bound": "hbm", "work": b_mat, "unit": "B", "t_roof_ms": 1e3 * b_mat / hbm}
    x_b = H * M
    out["births"] = {"bound": "trans", "work": x_b, "unit": "exp", "t_roof_ms": 1e3 * x_b / TRANS_PER_S}
    names = ["gate", "assoc", "select", "materialise", "births"]
    for j, n in enumerate(names):
        t = float(stage[j])
        out[n]["measured_ms"] = t
        tr = out[n]["t_roof_ms"]
        out[n]["frac"] = (tr / t) if (tr is not None and t > 0) else None
    t_roof = sum(out[n]["t_roof_ms"] or 0.0 for n in names)
    out["update"] = {"t_roof_ms": t_roof, "measured_ms": float(stage[5]),
                     "frac": t_roof / float(stage[5]) if stage[5] > 0 else None}
    out["mean_tracks_per_hypothesis"] = float(J)
    return out


def accuracy(estimates, truths, cutoff=10.0):
    """Cardinality error and Hungarian-matched position error of the per-scan estimates
    (the metrics of the paper's Sec. 4.2): |n_hat - n| / n, and the mean distance of matched
    (estimate, truth) pairs, pairs farther apart than `cutoff` counted as unmatched."""
    import numpy as np
    from scipy.optimize import linear_sum_assignment
    card, errs, far = [], [], 0
    for (labs, means), tx in zip(estimates, truths):
        n = len(tx)
        card.append(abs(len(means) - n) / max(n, 1))
        if len(means) and n:
            D = np.linalg.norm(np.asarray(means, np.float64)[:, None, :2] - np.asarray(tx)[None, :, :2], axis=2)
            r, c = linear_sum_assignment(np.minimum(D, cutoff))
            d = D[r, c]
            errs.extend(d[d < cutoff].tolist())
            far += int((d >= cutoff).sum()) + abs(len(means) - n)
        else:
            far += max(len(means), n)
    return {"card_rel_err_mean": float(np.mean(card)), "matched_err_mean_m": float(np.mean(errs)) if errs else None,
            "unmatched_per_scan": far / max(1, len(truths)), "cutoff_m": cutoff}



def particle_leg(torch, scene, z, k, P, params, reps=20):
    """The particle form on the benchmark scene's last scan: a cloud of P particles around every
    object (n = N P), CTRV prediction, association log-likelihoods against every detection, and
    the update of one record per object (its detections within 2 m).  Each call is timed with
    events on torch's stream over `reps` launches; bytes are the states and log weights each
    call must read and write (predict 40 B per particle; update 48 B per particle of a record),
    exps one per (gated pair, particle)."""
    import numpy as np
    from paper_2512_06230_amd.glmb import pf_loglik, pf_predict, pf_update
    rng = np.random.default_rng(7)
    tx = scene.truth_x[k]
    U = tx.shape[0]
    st = np.zeros((5, U * P), np.float32)
    st[0] = np.repeat(tx[:, 0], P) + rng.normal(0, 1.0, U * P)
    st[1] = np.repeat(tx[:, 1], P) + rng.normal(0, 1.0, U * P)
    st[2] = np.repeat(np.hypot(tx[:, 2], tx[:, 3]), P) + rng.normal(0, 0.5, U * P)
    st[3] = np.repeat(np.arctan2(tx[:, 3], tx[:, 2]), P) + rng.normal(0, 0.2, U * P)
    st[4] = rng.normal(0, 0.1, U * P)
    lw = np.full(U * P, -np.log(P), np.float32)
    zh = z.cpu().numpy()
    d = np.linalg.norm(zh[None, :, :] - tx[:, None, :2], axis=2)
    rec_u, rec_off, rec_z = [], [0], []
    for u in range(U):
        rec_u.append(u)
        rec_z += np.nonzero(d[u] < 2.0)[0].tolist()
        rec_off.append(len(rec_z))
    T = lambda a: torch.as_tensor(np.asarray(a), device="cuda")
    dst, dlw = T(st), T(lw)
    ru, ro, rz = (T(np.asarray(a, np.int32)) for a in (rec_u, rec_off, rec_z))
    sig, gam, gate = params["sigma_z"], params["det_rate"], params["gate_d2"]
    out = (torch.empty((5, U * P), dtype=torch.float32, device="cuda"), torch.empty(U * P, dtype=torch.float32,
           device="cuda"), torch.empty(U, dtype=torch.int32, device="cuda"))

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    work = dst.clone()
    t_pred = timed(lambda: pf_predict(work, 1.0, 1.0, 0.1, 3, k))
    phi = pf_loglik(dst, dlw, U, P, z, sig, gam, gate)
    gated = int(torch.isfinite(phi).sum())
    t_lik = timed(lambda: pf_loglik(dst, dlw, U, P, z, sig, gam, gate))
    t_upd = timed(lambda: pf_update(dst, dlw, U, P, ru, ro, rz, z, sig, 0.5, 3, k, out=out))
    hbm = HBM_PEAK_GBS * 1e9
    b_pred, b_upd = 40.0 * U * P, 48.0 * U * P
    x_lik = float(gated) * P
    return {"workload": "%d tracks x %d particles (CTRV), %d detections, %d gated pairs, %d update records"
                        % (U, P, zh.shape[0], gated, U),
            "predict": {"ms": t_pred * 1e3, "particles_per_s": U * P / t_pred, "bound": "hbm",
                        "achieved_gbs": b_pred / t_pred / 1e9, "frac": b_pred / t_pred / hbm},
            "loglik": {"ms": t_lik * 1e3, "bound": "trans", "exps_per_s": x_lik / t_lik,
                       "frac": x_lik / t_lik / TRANS_PER_S},
            "update": {"ms": t_upd * 1e3, "bound": "hbm", "achieved_gbs": b_upd / t_upd / 1e9,
                       "frac": b_upd / t_upd / hbm}}


def assoc_source_sha(rec):
    """sha256 of the source region holding the measured kernels (the text between the two
    marker lines named in the traffic record), or None when the file or a marker is gone."""
    import hashlib
    src = os.path.join(ROOT, rec["source"])
    if not os.path.exists(src):
        return None
    text = open(src).read()
    a, b = rec.get("region") or (None, None)
    if not a or not b or a not in text or b not in text:
        return None
    i = text.index(a)
    j = text.index(b, i)
    return hashlib.sha256(text[i:j].encode()).hexdigest()

def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-obj", type=int, default=500)
    ap.add_argument("--h-max", type=int, default=10000)
    ap.add_argument("--clutter", type=float, default=None)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample-hyp", type=int, default=2000,
                    help="the oracle's timed sample: one full step from the GPU's state cut to its best this-many "
                         "hypotheses (with H_max set to the same number); the rate is scaled by this share of H_max")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--batch-scenes", type=int, default=256, help="scenes of the batched leg (0: skip it)")
    ap.add_argument("--particles", type=int, default=4096,
                    help="particles per track of the particle-form leg (0: skip it)")
    ap.add_argument("--convoy-steps", type=int, default=548,
                    help="steps of the paper-setting leg (20-object convoy, H_max 100, H_up 100; 0: skip it)")
    ap.add_argument("--no-autotune-cache", action="store_true")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="first run one device-to-device copy of this many MiB (a known-size kernel that scales "
                         "hardware byte counters)")
    ap.add_argument("--proposal", default=None, help="trained proposal (.npz); default: the packaged one")
    ap.add_argument("--preset", choices=["c3", "c1", "c2"], default="c3",
                    help="c3: N objects in 100x100 m, clutter 0.2 N (default, with --n-obj / --h-max); "
                         "c1: 5 objects, H_max 64, tau 1e-5, empty start; c2: 50 objects in 1000x1000 m with "
                         "births, H_max 1024, tau 1e-5, warm start")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the multi-detection GLMB path runs on a single device "
              "(a scene would shard by ranges of prior-hypothesis rank); run with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2512_06230_amd import scenarios as sc
    from paper_2512_06230_amd.glmb import Tracker

    if args.copy_probe_mib > 0:
        n = args.copy_probe_mib * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    n_scans = args.warmup + args.steps
    tau = 0.0
    if args.preset == "c3":
        clutter = 0.2 * args.n_obj if args.clutter is None else args.clutter
        spec = sc.spec_for("c3:%d" % args.n_obj, clutter_mean=clutter, seed=args.seed)
        workload = "N=%d objects, H_max=%d, clutter %.0f/scan, 100x100 m, warm start, plain update" % (
            args.n_obj, args.h_max, clutter)
    else:
        spec = sc.spec_for(args.preset, seed=args.seed)
        args.n_obj, clutter, tau = spec.n_obj, spec.clutter_mean, 1e-5
        args.h_max = 64 if args.preset == "c1" else 1024
        args.no_learned, args.batch_scenes = True, 0
        workload = ("%s: %d objects, H_max=%d, clutter %.0f/scan, %.0fx%.0f m, tau 1e-5, %s, plain update" % (
            args.preset, spec.n_obj, args.h_max, clutter, spec.side, spec.side,
            "empty start" if args.preset == "c1" else "warm start, object births"))
    scene = sc.make_scene(spec, n_steps=n_scans)
    params = sc.filter_params(spec, args.h_max, tau)
    start = sc.empty_state() if args.preset == "c1" else sc.warm_start_state(scene)
    dev = torch.device("cuda:0")
    # every scan resident in HBM before timing
    zs = [torch.as_tensor(z, device=dev) for z in scene.meas]
    torch.cuda.synchronize()

    def run(proposal=None, measure=False):
        """Warm-up scans, then the timed scans; returns (seconds, per-scan stats)."""
        trk = Tracker(params)
        trk.import_state(start)
        if proposal is not None:
            trk.set_proposal(torch.as_tensor(proposal.params, device=dev), proposal.norm, proposal.threshold,
                             apply=True, measure=measure)

        def step(k):
            trk.predict(k)
            trk.update(k, zs[k])
            trk.truncate(args.h_max, tau)
            return trk.estimate()

        for k in range(args.warmup):
            step(k)
        torch.cuda.synchronize()
        st, est = [], []
        t0 = time.perf_counter()
        for k in range(args.warmup, n_scans):
            est.append(step(k))
            st.append(trk.stats())
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        run.estimates = est
        return el, st, trk

    elapsed, stats, trk = run()
    acc = accuracy(run.estimates, scene.truth_x[args.warmup:n_scans])
    ms_step = 1e3 * elapsed / args.steps
    dense = sum(s["dense_triples"] for s in stats)
    gated = sum(s["option_terms"] for s in stats)
    stage = np.mean(np.array([s["stage_ms"] for s in stats]), axis=0)

    learned = None
    prop_path = args.proposal or os.path.join(ROOT, "paper_2512_06230_amd", "proposal_n500.npz")
    if not args.no_learned and os.path.exists(prop_path):
        from paper_2512_06230_amd.proposal import Proposal
        prop = Proposal.load(prop_path)
        el_l, st_l, trk_l = run(prop)
        trk_l.close()
        # the same scans again, untimed, with the full-posterior lost mass measured at every update
        _, st_m, trk_m = run(prop, measure=True)
        trk_m.close()
        lost = np.array([s["lost_mass"] for s in st_m])
        # lost mass versus the plain update: along the plain trajectory, the plain update's
        # retained mass that the proposal's update does not retain (untimed)
        # and along the learned trajectory (the predicted states the learned filter reaches)
        from paper_2512_06230_amd.proposal import retained_lost
        pw = torch.as_tensor(prop.params, device=dev)
        probe = Tracker(params)
        ret_traj = {}
        gain = None
        for leg in ("plain", "learned"):
            ptrk = Tracker(params)
            ptrk.import_state(start)
            if leg == "learned":
                ptrk.set_proposal(pw, prop.norm, prop.threshold, apply=True)
            r = []
            for k in range(n_scans):
                ptrk.predict(k)
                if k >= args.warmup:
                    r.append(retained_lost(probe, ptrk.export_state(), k, zs[k], pw, prop.norm, [prop.threshold])[0])
                if leg == "plain" and k == n_scans - 1:
                    # what the network gains over the method without it: pairs kept by the plain
                    # gate, by the tightest gate with the same lost-mass bound, and by the network
                    from paper_2512_06230_amd.proposal import gate_gain
                    gain = gate_gain(params, ptrk.export_state(), k, zs[k], prop)
                ptrk.update(k, zs[k])
                ptrk.truncate(args.h_max, 0.0)
            ptrk.close()
            ret_traj[leg] = np.clip(np.array(r), 0.0, 1.0)
        probe.close()
        ret = ret_traj["plain"]
        stage_l = np.mean(np.array([s["stage_ms"] for s in st_l]), axis=0)
        learned = {
            "value": args.steps / el_l, "unit": "GLMB updates/s", "ms_per_step": 1e3 * el_l / args.steps,
            "speedup_vs_plain": elapsed / el_l,
            "update_ms": float(stage_l[5]), "plain_update_ms": float(stage[5]),
            "threshold": prop.threshold,
            "lost_mass_mean": float(ret.mean()), "lost_mass_max": float(ret.max()),
            "lost_mass_definition": "plain update's retained posterior mass absent from the learned update's "
                                    "retained set, per scan, from the plain filter's predicted states",
            "lost_mass_learned_trajectory_mean": float(ret_traj["learned"].mean()),
            "lost_mass_learned_trajectory_max": float(ret_traj["learned"].max()),
            "full_posterior_lost_mass_mean": float(np.clip(lost, 0.0, 1.0).mean()),
            "full_posterior_lost_mass_max": float(np.clip(lost, 0.0, 1.0).max()),
            "n_births_mean": float(np.mean([s["n_births"] for s in st_l])),
            "gain_vs_gate": gain,
            "plain_n_births_mean": float(np.mean([s["n_births"] for s in stats])),
            "pairs_removed_frac": float(sum(s["pairs_removed"] for s in st_l) /
                                        max(1, sum(s["gated_pairs"] for s in st_l))),
            "option_terms_frac": float(sum(s["option_terms"] for s in st_l) / max(1, gated)),
            "evals_per_s": sum(s["dense_triples"] for s in st_l) / el_l,
            "stage_ms": {"gate": float(stage_l[0]), "assoc": float(stage_l[1]), "select": float(stage_l[2]),
                         "materialise": float(stage_l[3]), "births": float(stage_l[4]),
                         "update": float(stage_l[5])},
            "proposal_file": os.path.relpath(prop_path, ROOT),
        }

    convoy_leg = None
    if args.convoy_steps > 0 and args.preset == "c3":
        # the paper's own setting (Sec. 4.1): 20-object convoy, D = 5, sigma = 0.25 m, no clutter,
        # H_max = 100, the paper's generator with H_up = 100 and tau = 1e-5, from an empty state
        from paper_2512_06230_amd import convoy as cv
        r = cv.run(20, 100, 100, 1e-5, 0, 0, args.convoy_steps)
        convoy_leg = {"workload": "synthetic 20-object convoy (delta 2, D 5, sigma 0.25 m, no clutter), H_max 100, "
                                  "sampled children H_up 100, tau 1e-5, empty start, %d steps of 0.1 s" % r["steps"],
                      "update_ms_mean": r["update_ms_mean"], "step_ms_mean": r["step_ms_mean"],
                      "step_ms_max": r["step_ms_max"], "card_rel_err": r["card_rel_err"],
                      "matched_err_m": r["matched_err_m"], "hypotheses_mean": r["hypotheses_mean"],
                      "paper": "update under the 0.1 s real-time budget almost always on an NVIDIA L40S "
                               "(Sec. 4.2, N=20, H_max=100; no number printed)"}

    particle = None
    if args.particles > 0 and args.preset == "c3":
        particle = particle_leg(torch, scene, zs[n_scans - 1], n_scans - 1, args.particles, params)

    batched = None
    if args.batch_scenes > 0:
        from paper_2512_06230_amd.autotune import BatchTuner, workload_key
        from paper_2512_06230_amd.glmb import Batch
        # warm-up steps also serve the schedule tuner when its cache misses; then 50 timed steps of
        # the tuned schedule and, from the same state onwards, 4 steps with one worker (the scenes
        # one after another, one launch sequence per scene) for comparison
        nb_warm, nb_steps, nb_seq = 12, 50, 4
        specs = sc.batch_specs(args.batch_scenes, seed=args.seed, n_steps=nb_warm + nb_steps + nb_seq)
        bscenes = [sc.make_scene(sp, n_steps=nb_warm + nb_steps + nb_seq) for sp, _ in specs]
        bparams = [sc.filter_params(sp, h, 1e-5) for sp, h in specs]
        bz, boff = [], []
        for k in range(nb_warm + nb_steps + nb_seq):  # every scan of every scene resident in HBM
            zk = [bs.meas[k] for bs in bscenes]
            boff.append(np.concatenate([[0], np.cumsum([z.shape[0] for z in zk])]).astype(np.int32))
            bz.append(torch.as_tensor(np.concatenate(zk, axis=0).reshape(-1, 2), device=dev).contiguous())
        batch = Batch(bparams, workers=4)
        for i, bs in enumerate(bscenes):
            batch.scene(i).import_state(sc.warm_start_state(bs))
        cost = sum(h * float(bz[0].shape[0]) / len(bscenes) for _, h in specs)
        tuner = BatchTuner(batch, workload_key(torch.cuda.get_device_name(0), len(bscenes), cost),
                           cache_path=None if args.no_autotune_cache else os.path.join(
                               ROOT, "paper_2512_06230_amd", "autotune_cache.json"))
        for k in range(nb_warm):
            tuner.step(k, bz[k], boff[k])
        torch.cuda.synchronize()
        tb = time.perf_counter()
        for k in range(nb_warm, nb_warm + nb_steps):
            tuner.step(k, bz[k], boff[k])
        torch.cuda.synchronize()
        el_b = time.perf_counter() - tb
        bst = batch.stats()
        batch.set_schedule(1, True)
        torch.cuda.synchronize()
        ts = time.perf_counter()
        for k in range(nb_warm + nb_steps, nb_warm + nb_steps + nb_seq):
            batch.step(k, bz[k], boff[k])
        torch.cuda.synchronize()
        el_s = time.perf_counter() - ts
        batched = {"value": len(bscenes) * nb_steps / el_b, "unit": "scene-updates/s",
                   "ms_per_step": 1e3 * el_b / nb_steps, "scenes": len(bscenes), "steps": nb_steps,
                   "warmup": nb_warm, "workers": bst["workers"], "longest_first": bool(bst["longest_first"]),
                   "workload": "%d scenes: N ~ U{5..200} objects, H_max ~ logU[256, 8192], clutter 2/scan, "
                               "100x100 m, warm start" % len(bscenes),
                   "one_scene_at_a_time": {"value": len(bscenes) * nb_seq / el_s, "ms_per_step": 1e3 * el_s / nb_seq,
                                           "steps": nb_seq, "workers": 1},
                   "speedup_vs_one_scene_at_a_time": (len(bscenes) * nb_steps / el_b) / (len(bscenes) * nb_seq / el_s),
                   "tuner_trials": [{"workers": c[0], "longest_first": c[1], "step_ms": ms} for c, ms in tuner.trials],
                   "mean_h_max": float(np.mean([h for _, h in specs])),
                   "mean_objects": float(np.mean([sp.n_obj for sp, _ in specs]))}
        batch.close()

    # roofline of the dominant kernel: the per-(hypothesis, detection) association kernel, which
    # covers hypotheses 1..H-1 (hypothesis 0's cells come from a one-workgroup kernel before it).
    # Algorithmic HBM bytes per launch: each hypothesis row of |J| instance ids read once (4 B
    # each) and two floats written per hypothesis (its best child's log weight and the log mass
    # of all its children); the duration is the kernel's own, from HIP events around its launch.
    H = np.mean([s["n_hyp_in"] for s in stats])
    M = np.mean([s["n_meas"] for s in stats])
    roof = stage_roofline(stats, stage)
    bytes_assoc = roof["assoc"]["work"]
    t_assoc = float(stage[1]) * 1e-3
    achieved = bytes_assoc / t_assoc / 1e9 if t_assoc > 0 else 0.0
    # measured HBM bytes per launch (rocprofv3 FETCH_SIZE / WRITE_SIZE, scaled by a copy kernel);
    # null once the kernel's source differs from the one the counters were taken with
    traffic = None
    tf = os.path.join(ROOT, "profiles", "k_assoc_n500_h1e4_traffic.json")
    if os.path.exists(tf):
        rec = json.load(open(tf))
        if assoc_source_sha(rec) == rec["source_sha256"] and args.n_obj == 500 and args.h_max == 10000:
            traffic = rec["bytes_per_launch"]
    # measured HBM bytes of the materialisation stage per update (same counters and scaling),
    # null once the materialisation kernels' source differs from the one the counters were taken with
    uf = os.path.join(ROOT, "profiles", "u4_n500_h1e4_traffic.json")
    if os.path.exists(uf) and args.n_obj == 500 and args.h_max == 10000 and args.preset == "c3":
        urec = json.load(open(uf))
        same = assoc_source_sha(urec) == urec["source_sha256"]
        mat = roof["materialise"]
        mat["traffic"] = urec["bytes_per_update"] if same else None
        mat["traffic_frac"] = (urec["bytes_per_update"] / (mat["measured_ms"] * 1e-3) / (HBM_PEAK_GBS * 1e9)
                               if same and mat["measured_ms"] > 0 else None)
    out = {
        "metric": METRIC,
        "value": args.steps / elapsed,
        "unit": "GLMB updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": workload,
                   "n_obj": args.n_obj, "h_max": args.h_max, "clutter_mean": clutter,
                   "mean_detections": float(M), "mean_hypotheses_in": float(H), "parallelism": "single GPU"},
        "evals_per_s": dense / elapsed,
        "update_per_s": 1e3 / float(stage[5]) if stage[5] > 0 else None,
        "gated_evals_per_s": gated / elapsed,
        "stage_ms": {"gate": float(stage[0]), "assoc": float(stage[1]), "select": float(stage[2]),
                     "materialise": float(stage[3]), "births": float(stage[4]), "update": float(stage[5])},
        "roofline": {"kernel": "k_assoc", "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "algorithmic_bytes": bytes_assoc,
                     "traffic_over_algorithmic": (traffic / bytes_assoc) if traffic else None},
        "stage_roofline": roof,
        "host_syncs_per_update": float(np.mean([s["host_syncs"] for s in stats])),
        # the update's exact selection: nodes written, levels, form (0 one workgroup, 1 cooperative
        # whole-GPU launch, 2 host-driven multi-kernel levels)
        "search": {"nodes_mean": float(np.mean([s["search_nodes"] for s in stats])),
                   "levels_mean": float(np.mean([s["search_levels"] for s in stats])),
                   "forms": sorted(set(int(s["search_form"]) for s in stats))},
        "accuracy": acc,
    }
    if learned is not None:
        out["learned"] = learned
    if batched is not None:
        out["batched"] = batched
    if convoy_leg is not None:
        out["convoy"] = convoy_leg
    if particle is not None:
        out["particle"] = particle

    if not args.no_cpu_baseline:
        from oracle.oracle import Oracle
        st = trk.export_state()
        nh = max(1, min(args.cpu_sample_hyp, len(st["hyp_logw"]), args.h_max))
        # the best nh hypotheses (the state lists them in rank order), renormalised by import
        st = dict(st, hyp_logw=st["hyp_logw"][:nh], hyp_off=st["hyp_off"][:nh + 1],
                  hyp_idx=st["hyp_idx"][:st["hyp_off"][nh]])
        o = Oracle(dict(params, h_max=nh))
        o.import_state({k: (np.asarray(v, np.float64) if np.asarray(v).dtype == np.float32 else v)
                        for k, v in st.items() if k not in ("inst_src", "inst_nz", "inst_z", "hyp_parent")})
        kk = n_scans - 1
        # the oracle is single-threaded: pin this thread to one core for the timing
        aff = os.sched_getaffinity(0)
        core = min(aff)
        os.sched_setaffinity(0, {core})
        try:
            tc = time.perf_counter()
            o.predict(kk)
            o.update(kk, scene.meas[kk])
            o.truncate(nh, tau)
            o.estimate()
            tcpu = time.perf_counter() - tc
        finally:
            os.sched_setaffinity(0, aff)
        share = nh / float(args.h_max)
        out["cpu_baseline"] = {"value": share / tcpu, "unit": "GLMB updates/s", "cores": 1,
                               "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
                               "host_cpus_allowed": len(aff), "pinned_core": core, "sample_seconds": tcpu,
                               "sample": "one full step (predict+update+truncate+estimate) of the same workload "
                                         "from the GPU's state after the timed steps cut to its best %d "
                                         "hypotheses (H_max %d), FP64, one thread pinned to one core; rate "
                                         "scaled by %d/%d (work linear in the hypothesis count)"
                                         % (nh, nh, nh, args.h_max)}
    trk.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
