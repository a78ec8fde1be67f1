"""Host logic of the batched step's schedule tuner (no GPU): candidates measured in a
palindromic order, a linear warm-up trend cancelled, the choice cached and reused."""
import json

from paper_2512_06230_amd.autotune import CANDIDATES, BatchTuner


class FakeBatch:
    def __init__(self, cost, trend):
        self.cost, self.trend, self.k, self.sched, self.ms = cost, trend, 0, None, 0.0

    def set_schedule(self, workers, longest_first=True):
        self.sched = (workers, bool(longest_first))

    def step(self, k, z, z_off):
        self.ms = self.cost[self.sched] + self.trend * self.k
        self.k += 1

    def stats(self):
        return {"step_ms": self.ms}


def test_palindromic_order_cancels_a_linear_trend(tmp_path):
    # the true best (8 workers) is measured late; a steep linear growth of the step time would
    # make a one-pass comparison pick an early candidate
    cost = {c: 100.0 for c in CANDIDATES}
    cost[(8, True)] = 90.0
    b = FakeBatch(cost, trend=15.0)
    path = str(tmp_path / "cache.json")
    t = BatchTuner(b, "key", cache_path=path)
    assert t.warmup_steps == 2 * len(CANDIDATES)
    for k in range(2 * len(CANDIDATES)):
        t.step(k, None, None)
    assert t.tuned and t.choice == (8, True) and b.sched == (8, True)
    data = json.load(open(path))
    assert data["key"]["workers"] == 8 and len(data["key"]["trials"]) == 2 * len(CANDIDATES)
    # a new tuner with the same key starts from the cache
    b2 = FakeBatch(cost, trend=0.0)
    t2 = BatchTuner(b2, "key", cache_path=path)
    assert t2.tuned and t2.warmup_steps == 0 and b2.sched == (8, True)
    t2.step(0, None, None)
    assert b2.sched == (8, True)
