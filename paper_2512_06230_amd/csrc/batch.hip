// Batched time step of many independent scenes of uneven size (an addition to the method of
// Sec. 3, which filters one scene).  Host worker threads, each driving its own HIP stream,
// pull scenes in longest-job-first order of a cost estimate and run predict + update +
// truncate on them, so that the small launches and host round trips of one scene overlap with
// the kernels of the others.  Scenes share no data: every scene's result equals its own
// single-scene step bit for bit, whatever the number of workers or the order.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <thread>

#include "ctx.hpp"

struct glmb_batch {
  int device = 0;
  std::vector<glmb_ctx*> ctx;
  std::vector<hipStream_t> streams;
  hipEvent_t ready = nullptr;  // recorded on the caller's stream at every step
  int workers = 1;
  bool ljf = true;
  std::vector<double> cost;  // cost estimate of every scene for the next step
  glmb_batch_stats stats{};
  std::string err;
};

namespace {
glmb_status bfail(glmb_batch* b, glmb_status st, const std::string& msg) {
  if (b) b->err = msg;
  return st;
}
}  // namespace

extern "C" {

const char* glmb_batch_last_error(const glmb_batch* b) { return b ? b->err.c_str() : "null batch"; }

glmb_status glmb_batch_create(int32_t n, const glmb_params* params, int device, int32_t workers, glmb_batch** out) {
  if (n < 1 || !params || !out || workers < 1 || workers > GLMB_BATCH_MAX_WORKERS) return GLMB_E_ARG;
  *out = nullptr;
  glmb_batch* b = new glmb_batch();
  b->device = device;
  b->workers = workers;
  if (hipSetDevice(device) != hipSuccess) {
    delete b;
    return GLMB_E_DEVICE;
  }
  b->streams.resize(GLMB_BATCH_MAX_WORKERS, nullptr);
  for (auto& s : b->streams)
    if (hipStreamCreateWithFlags(&s, hipStreamNonBlocking) != hipSuccess) {
      glmb_batch_destroy(b);
      return GLMB_E_DEVICE;
    }
  if (hipEventCreateWithFlags(&b->ready, hipEventDisableTiming) != hipSuccess) {
    glmb_batch_destroy(b);
    return GLMB_E_DEVICE;
  }
  b->ctx.resize(n, nullptr);
  b->cost.assign(n, 0.0);
  for (int i = 0; i < n; ++i) {
    const glmb_status st = glmb_create(params + i, device, b->streams[0], &b->ctx[i]);
    if (st != GLMB_OK) {
      glmb_batch_destroy(b);
      return st;
    }
    // cooperative launches run one at a time on a device: concurrent scenes use the
    // multi-kernel form of the whole-GPU search, which overlaps across streams
    b->ctx[i]->c.coop_ok = false;
    // scenes overlap across the worker streams already: no side stream per scene
    b->ctx[i]->c.fork_ok = false;
  }
  *out = b;
  return GLMB_OK;
}

glmb_status glmb_batch_destroy(glmb_batch* b) {
  if (!b) return GLMB_E_ARG;
  for (auto* x : b->ctx)
    if (x) glmb_destroy(x);
  for (auto s : b->streams)
    if (s) (void)hipStreamDestroy(s);
  if (b->ready) (void)hipEventDestroy(b->ready);
  delete b;
  return GLMB_OK;
}

glmb_status glmb_batch_set_schedule(glmb_batch* b, int32_t workers, int32_t longest_first) {
  if (!b || workers < 1 || workers > GLMB_BATCH_MAX_WORKERS) return GLMB_E_ARG;
  b->workers = workers;
  b->ljf = longest_first != 0;
  return GLMB_OK;
}

glmb_status glmb_batch_scene(glmb_batch* b, int32_t scene, glmb_ctx** out) {
  if (!b || !out || scene < 0 || scene >= (int)b->ctx.size()) return GLMB_E_ARG;
  *out = b->ctx[scene];
  return GLMB_OK;
}

glmb_status glmb_batch_step(glmb_batch* b, int32_t k, const float* z, const int32_t* z_off, void* caller_stream) {
  if (!b || !z_off) return GLMB_E_ARG;
  const int n = (int)b->ctx.size();
  if (z_off[0] != 0) return bfail(b, GLMB_E_ARG, "z_off[0] must be 0");
  for (int i = 0; i < n; ++i)
    if (z_off[i + 1] < z_off[i]) return bfail(b, GLMB_E_ARG, "z_off must be non-decreasing");
  if (z_off[n] > 0 && !z) return bfail(b, GLMB_E_ARG, "null detections");
  // longest job first on the cost estimate H * M * (1 + gated tracks per detection); the
  // first step, without statistics, uses H * M
  std::vector<int32_t> order(n);
  for (int i = 0; i < n; ++i) {
    order[i] = i;
    if (b->cost[i] <= 0.0) b->cost[i] = (double)b->ctx[i]->c.nhyp * (double)(z_off[i + 1] - z_off[i] + 1);
  }
  if (b->ljf)
    std::stable_sort(order.begin(), order.end(), [&](int32_t x, int32_t y) { return b->cost[x] > b->cost[y]; });
  // the detections may still be in flight on the caller's stream: every worker stream waits
  // for the work queued there before its first launch
  if (hipSetDevice(b->device) != hipSuccess) return bfail(b, GLMB_E_DEVICE, "hipSetDevice failed");
  if (hipEventRecord(b->ready, (hipStream_t)caller_stream) != hipSuccess)
    return bfail(b, GLMB_E_DEVICE, "hipEventRecord on the caller's stream failed");
  for (int w = 0; w < std::min(b->workers, n); ++w)
    if (hipStreamWaitEvent(b->streams[w], b->ready, 0) != hipSuccess)
      return bfail(b, GLMB_E_DEVICE, "hipStreamWaitEvent failed");
  std::atomic<int> next{0};
  std::atomic<int> first_bad{-1};
  std::vector<glmb_status> st(n, GLMB_OK);
  const int W = std::min(b->workers, n);
  auto work = [&](int w) {
    if (hipSetDevice(b->device) != hipSuccess) {
      first_bad.store(-2);
      return;
    }
    for (;;) {
      const int j = next.fetch_add(1);
      if (j >= n) break;
      const int s = order[j];
      glmb_ctx* x = b->ctx[s];
      x->c.s = b->streams[w];
      const int M = z_off[s + 1] - z_off[s];
      glmb_status r = glmb_predict(x, k);
      if (r == GLMB_OK) r = glmb_update(x, k, z ? z + 2 * (size_t)z_off[s] : nullptr, M);
      if (r == GLMB_OK) r = glmb_truncate(x, x->c.p.h_max, x->c.p.tau);
      st[s] = r;
      if (r != GLMB_OK) {
        int expect = -1;
        first_bad.compare_exchange_strong(expect, s);
      }
    }
  };
  const auto t0 = std::chrono::steady_clock::now();
  std::vector<std::thread> pool;
  for (int w = 1; w < W; ++w) pool.emplace_back(work, w);
  work(0);
  for (auto& t : pool) t.join();
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  b->stats.n_scenes = n;
  b->stats.workers = W;
  b->stats.longest_first = b->ljf ? 1 : 0;
  b->stats.step_ms = (float)ms;
  b->stats.scene_updates_per_s = ms > 0 ? 1e3 * n / ms : 0.0;
  b->stats.first_error_scene = first_bad.load();
  if (first_bad.load() == -2) return bfail(b, GLMB_E_DEVICE, "hipSetDevice failed in a worker");
  for (int i = 0; i < n; ++i) {
    const glmb_step_stats& q = b->ctx[i]->c.stats;
    const double M = std::max(1, q.n_meas);
    b->cost[i] = (double)std::max(1, b->ctx[i]->c.nhyp) * M * (1.0 + (double)q.gated_pairs / M);
  }
  if (first_bad.load() >= 0) {
    const int s = first_bad.load();
    return bfail(b, st[s], "scene " + std::to_string(s) + ": " + b->ctx[s]->c.err);
  }
  return GLMB_OK;
}

glmb_status glmb_batch_stats_get(glmb_batch* b, glmb_batch_stats* out) {
  if (!b || !out) return GLMB_E_ARG;
  *out = b->stats;
  return GLMB_OK;
}

}  // extern "C"
