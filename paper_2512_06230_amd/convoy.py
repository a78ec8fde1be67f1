"""The paper's scalability benchmark (Sec. 4.1-4.2) on the GPU: a synthetic convoy of N
copies of one track, D = 5 detections per object per 0.1 s step, sigma = 0.25 m, no clutter,
548 steps; the tracker with the paper's hypothesis generator (H_up = 100 maps per hypothesis,
tau = 1e-5) and H_max hypotheses.  Per run: the time average of the relative cardinality error
and of the Hungarian-matched tracking error, and the mean update and step times; repeated runs
differ in the generator's seed.

    python -m paper_2512_06230_amd.convoy --objects 1 2 5 10 20 --hmax 5 10 25 50 100 --repeats 10
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import metrics
from . import scenarios as sc


def run(n_obj: int, h_max: int, h_up: int = 100, tau: float = 1e-5, data_seed: int = 0, seed: int = 0,
        steps: int = 548, joint: bool = False) -> dict:
    import torch
    from .glmb import Tracker
    spec = sc.ConvoySpec(n_obj=n_obj, seed=data_seed)
    scene = sc.make_convoy(spec, steps)
    p = sc.convoy_params(spec, h_max, tau)
    zs = [torch.as_tensor(z, device="cuda") for z in scene.meas]
    trk = Tracker(p)
    trk.import_state(sc.empty_state())
    if h_up > 0:
        trk.set_sampling(h_up, seed)
    if joint:
        trk.set_joint_reweighting(True)
    torch.cuda.synchronize()
    n_est, est, upd, step_ms, nh = [], [], [], [], []
    for k in range(steps):
        t0 = time.perf_counter()
        trk.predict(k)
        trk.update(k, zs[k])
        trk.truncate(h_max, tau)
        labs, means = trk.estimate()  # synchronises
        step_ms.append(1e3 * (time.perf_counter() - t0))
        s = trk.stats()
        upd.append(s["stage_ms"][5])
        nh.append(s["n_hyp_out"])
        n_est.append(len(labs))
        est.append(means[:, :2])
    trk.close()
    truths = [x[:, :2] for x in scene.truth_x]
    return dict(objects=n_obj, h_max=h_max, h_up=h_up, tau=tau, seed=seed, steps=steps, joint=joint,
                card_rel_err=metrics.cardinality_error(n_est, [len(t) for t in truths]),
                matched_err_m=metrics.matched_error(est, truths),
                update_ms_mean=float(np.mean(upd)), step_ms_mean=float(np.mean(step_ms)),
                step_ms_max=float(np.max(step_ms)), hypotheses_mean=float(np.mean(nh)))


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--objects", type=int, nargs="+", default=[1, 2, 5, 10, 20])
    ap.add_argument("--hmax", type=int, nargs="+", default=[5, 10, 25, 50, 100])
    ap.add_argument("--repeats", type=int, default=10)
    ap.add_argument("--steps", type=int, default=548)
    ap.add_argument("--hup", type=int, default=100, help="maps drawn per hypothesis (0: exact top-H_max)")
    ap.add_argument("--joint", action="store_true", help="exact-joint reweighting of the kept hypotheses")
    ap.add_argument("--out", default=None, help="write every run as a JSON line here")
    a = ap.parse_args(argv)
    f = open(a.out, "w") if a.out else None
    for n in a.objects:
        for h in a.hmax:
            rs = [run(n, h, a.hup, 1e-5, 0, r, a.steps, a.joint) for r in range(a.repeats)]
            for r in rs:
                if f:
                    f.write(json.dumps(r) + "\n")
            agg = {k: (float(np.mean([r[k] for r in rs])), float(np.std([r[k] for r in rs]) / np.sqrt(len(rs))))
                   for k in ("card_rel_err", "matched_err_m", "update_ms_mean", "step_ms_mean")}
            print(json.dumps(dict(objects=n, h_max=h, repeats=len(rs), **{k: v for k, v in agg.items()})),
                  flush=True)
    if f:
        f.close()


if __name__ == "__main__":
    sys.exit(main())
