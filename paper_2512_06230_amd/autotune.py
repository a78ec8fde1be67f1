"""Autotuner of the batched step's schedule, with a JSON cache.

The schedule of ``glmb_batch_step`` (number of worker streams, longest-job-first or index
order) changes only the time a step takes, never its result, so the tuner measures each
candidate on the first live steps of a run and keeps the fastest for the rest; the choice is
cached per workload key (device, number of scenes, size bucket of the total cost) so that later
runs start with it.
"""
from __future__ import annotations

import json
import math
import os

HERE = os.path.dirname(os.path.abspath(__file__))
DEFAULT_CACHE = os.path.join(HERE, "autotune_cache.json")
CANDIDATES = [(1, True), (2, True), (4, True), (8, True), (16, True), (16, False)]


def workload_key(device_name: str, n_scenes: int, cost: float) -> str:
    """Device, scene count and the power-of-two bucket of the summed H * M of the scenes."""
    b = int(math.floor(math.log2(max(cost, 1.0))))
    return "%s|scenes=%d|cost=2^%d" % (device_name, n_scenes, b)


class BatchTuner:
    def __init__(self, batch, key: str, cache_path: str = DEFAULT_CACHE, candidates=CANDIDATES):
        self.batch = batch
        self.key = key
        self.cache_path = cache_path
        self.candidates = list(candidates)
        self.cache = {}
        if cache_path and os.path.exists(cache_path):
            with open(cache_path) as f:
                self.cache = json.load(f)
        self.choice = None
        self.trials = []
        hit = self.cache.get(key)
        if hit:
            self.choice = (int(hit["workers"]), bool(hit["longest_first"]))
            batch.set_schedule(*self.choice)

    @property
    def tuned(self) -> bool:
        return self.choice is not None

    def step(self, k: int, z, z_off):
        """One batched step; while untuned, the step measures the next candidate schedule.

        The candidates are measured in a palindromic order (c1 .. cn cn .. c1): the first
        steps of a run grow heavier as the state fills up to H_max, and summing each
        candidate's two times cancels a trend that is linear in the step number."""
        if self.tuned:
            self.batch.step(k, z, z_off)
            return
        seq = self.candidates + self.candidates[::-1]
        cand = seq[len(self.trials)]
        self.batch.set_schedule(*cand)
        self.batch.step(k, z, z_off)
        self.trials.append((cand, float(self.batch.stats()["step_ms"])))
        if len(self.trials) == len(seq):
            total = {}
            for c, ms in self.trials:
                total[c] = total.get(c, 0.0) + ms
            self.choice = min(self.candidates, key=lambda c: total[c])
            self.batch.set_schedule(*self.choice)
            self.cache[self.key] = {"workers": self.choice[0], "longest_first": self.choice[1],
                                    "trials": [{"workers": c[0], "longest_first": c[1], "step_ms": ms}
                                               for c, ms in self.trials]}
            if self.cache_path:
                tmp = self.cache_path + ".tmp"
                with open(tmp, "w") as f:
                    json.dump(self.cache, f, indent=1, sort_keys=True)
                os.replace(tmp, self.cache_path)

    @property
    def warmup_steps(self) -> int:
        """Steps the tuner still needs before its choice is made (0 when cached)."""
        return 0 if self.tuned else 2 * len(self.candidates) - len(self.trials)
