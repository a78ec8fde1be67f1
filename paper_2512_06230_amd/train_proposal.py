"""Train and calibrate the learned pair proposal on the GPU; writes a .npz file.

    python -m paper_2512_06230_amd.train_proposal --out paper_2512_06230_amd/proposal_n500.npz

Training scenes: 200 scenes of N=200 objects (clutter 40 per scan), H_max=1e3, warm start,
20 scans each, seeds 1000, 1001, ... (optionally also N=500 scenes, seeds 1500, ...).  Threshold: the largest grid value whose lost posterior
mass versus the plain update stays <= 1e-3 on every scan of the held-out scenes (N=500,
clutter 100, H_max=1e4, seeds 2000, ...), i.e. the benchmarked workload on scenes the
benchmark does not use.
"""
from __future__ import annotations

import argparse
import sys
import time

import numpy as np

from . import proposal as pr
from . import scenarios as sc
from .glmb import Tracker


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", required=True)
    ap.add_argument("--train-scenes", type=int, default=200)
    ap.add_argument("--train-scenes-large", type=int, default=0)
    ap.add_argument("--train-steps", type=int, default=20)
    ap.add_argument("--train-n", type=int, default=200)
    ap.add_argument("--train-hmax", type=int, default=1000)
    ap.add_argument("--heldout-scenes", type=int, default=2)
    ap.add_argument("--heldout-steps", type=int, default=6)
    ap.add_argument("--heldout-n", type=int, default=500)
    ap.add_argument("--heldout-hmax", type=int, default=10000)
    ap.add_argument("--epochs", type=int, default=6)
    ap.add_argument("--batch", type=int, default=8192)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--max-lost", type=float, default=1e-3)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)

    def log(msg):
        print("[train] %s" % msg, flush=True)

    t0 = time.time()
    train_specs = [sc.spec_for("c3:%d" % a.train_n, seed=1000 + j) for j in range(a.train_scenes)]
    train_specs += [sc.spec_for("c3:%d" % a.heldout_n, seed=1500 + j) for j in range(a.train_scenes_large)]
    feat, y, w = pr.collect(train_specs, a.train_hmax, a.train_steps, log=log)
    log("training pairs %d (%.1fs)" % (int(feat.shape[0]), time.time() - t0))
    trk = Tracker(sc.filter_params(train_specs[0], a.train_hmax, 0.0))
    params, norm, hist = pr.train(trk, feat, y, w, epochs=a.epochs, batch=a.batch, lr=a.lr, seed=a.seed, log=log)
    trk.close()
    log("trained (%.1fs)" % (time.time() - t0))
    held = [sc.spec_for("c3:%d" % a.heldout_n, seed=2000 + j) for j in range(a.heldout_scenes)]
    thr, worst, worst_full = pr.calibrate(params, norm, held, a.heldout_hmax, a.heldout_steps, a.max_lost, log=log)
    if thr is None:
        log("no threshold keeps the lost mass below %g" % a.max_lost)
        return 1
    info = dict(train_scenes=a.train_scenes, train_steps=a.train_steps, train_n=a.train_n,
                train_hmax=a.train_hmax, train_pairs=int(feat.shape[0]), epochs=a.epochs, batch=a.batch, lr=a.lr,
                seed=a.seed, loss=[float(x) for x in hist], heldout_scenes=a.heldout_scenes,
                heldout_steps=a.heldout_steps, heldout_n=a.heldout_n, heldout_hmax=a.heldout_hmax,
                max_lost=a.max_lost, thresholds=list(pr.THRESHOLDS), worst_lost=[float(x) for x in worst],
                worst_lost_full_posterior=[float(x) for x in worst_full], train_scenes_large=a.train_scenes_large,
                seconds=time.time() - t0)
    pr.Proposal(params.detach().cpu().numpy().astype(np.float32), norm, float(thr), info).save(a.out)
    log("threshold %g, written %s (%.1fs)" % (thr, a.out, time.time() - t0))
    return 0


if __name__ == "__main__":
    sys.exit(main())
