// Filter context: device-resident GLMB state and per-step work buffers.
//
// HBM layout
//   instances   DInst[ninst] (64 B each: mean, upper-triangular covariance, label slot,
//               source index), sorted by label slot so that the instances of one label are
//               contiguous;
//   hypotheses  logw[nhyp] (normalised), ntrk[nhyp], rows[nhyp][stride] with the instance id
//               held for every label slot (-1: label absent); rows are in rank order;
//   labels      host-side table slot -> (birth scan, index), slots in ascending label order;
//   births      pending LMB birth components for the next prediction.
#pragma once

#include <utility>

#include "common.hpp"

namespace glmb {

struct DInst {
  float m[4];
  float P[10];  // P00 P01 P02 P03 P11 P12 P13 P22 P23 P33
  int32_t slot;
  int32_t src;
};
static_assert(sizeof(DInst) == 64, "instance record is one 64-byte line");

struct DBirth {
  float m[4];
  float P[10];
  float r;
  int32_t pad;
};

struct Ctx {
  glmb_params p{};
  int device = 0;
  hipStream_t s = nullptr;
  std::string err;
  bool alive = true;
  bool trace = false;  // GLMB_TRACE=1: print every host-side stage to stderr (flushed)
  hipEvent_t ev[8] = {};  // stage timing events on the context's stream
  bool ev_ok = false;
  // Side stream for work that overlaps the main chain: the births' clutter probabilities run
  // beside the selection and materialisation, the learned proposal's label inputs beside the
  // gate.  Created on first use (default priority); fork[j] are its fork / join events.
  bool fork_ok = true;
  hipStream_t s2 = nullptr;
  hipEvent_t fork[4] = {};
  void side_ready() {
    if (s2) return;
    GLMB_HIP(hipStreamCreateWithFlags(&s2, hipStreamNonBlocking));
    for (auto& e : fork) GLMB_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
  }
  void mark(int i) {
    if (ev_ok) (void)hipEventRecord(ev[i], s);
  }

  // ---- state (host mirrors of the sizes) ----
  std::vector<std::pair<int32_t, int32_t>> slot_lab;   // label of each slot (ascending)
  std::vector<std::pair<int32_t, int32_t>> birth_lab;  // labels of pending births
  int nslot = 0, ninst = 0, nhyp = 0, nbirth = 0, stride = 0;
  DevBuf inst, inst2;          // DInst
  DevBuf inst_nz, inst_z;      // detections of the last update per instance (count, up to 8 indices)
  DevBuf logw, ntrk, rows, hparent;
  DevBuf logw2, ntrk2, rows2;  // double buffers
  DevBuf births, births2;      // DBirth (the update writes the next scan's into births2)
  std::vector<DBirth> birth_host;  // host copy of the pending births, when birth_host_ok
  bool birth_host_ok = false;

  // ---- last update (for diagnostics / exports) ----
  int last_H = 0, last_M = 0, last_stride = 0;
  DevBuf diag_best, diag_logpi, diag_ru;
  DevBuf prev_rows, prev_src;  // predicted rows and instance sources of the last update
  DevBuf child_par, dev_off, dev_i, dev_slot;
  glmb_step_stats stats{};

  // ---- update work buffers ----
  DevBuf z, cmax, gbits, phi, lbits, lpre, llen, loff, lmeas, inst_beg, ccnt, coff, cand, best16, dev1, lserel, tbits, tpre,
      bprime, lzprime, cells, ccount, coff2, it_h, it_delta, it_group, it_opt, it_off, keys, vals32, scal,
      sel_logw, hp_map, first, dmask, exc, cmod, recs, rec_keys, rec_vals, ids, row_mark, ru_part, ru, bt,
      tmp, tk, tv, flags, pre, pmult, pvals, rec_m, ref_b1, ref_opts, ref_top, ref_rest, ref_tot, hopts, ref_sel;
  SelectBufs sb;
  bool sel_multi[2] = {false, false};  // per search site (prediction, update): start on the whole GPU
  bool coop_ok = true;  // cooperative launches allowed (they run one at a time on a device)
  bool force_multi = false;  // every search on the host-driven multi-kernel levels (GLMB_SEARCH_FORM=multi)
  bool force_coop = false;   // every search starts on the whole GPU (GLMB_SEARCH_FORM=coop)
  int group_bits = 2;         // SelectIn::group_bits of every search (GLMB_SEARCH_GROUP_BITS)
  float dp_inflate = 0.f;     // SelectIn::dp_inflate of the update's search (GLMB_DP_BOUND_INFLATE)
  int LW = 1;  // detection-set mask width (32-bit words) of the last gate
  // fingerprint bits of the (instance, detection set) records (16 at most: records of one instance
  // with equal fingerprints are told apart by full comparison)
  uint32_t rec_hash_mask = 0xffffu;
  DevBuf rec_lead;                       // collision path: leader position of every record
  // ---- sampled children (the paper's generator) instead of the exact selection
  int32_t sample_hup = 0;      // association maps drawn per hypothesis (0: exact top-H_max)
  uint64_t sample_seed = 0;    // Philox key
  int32_t sample_unique = 0;   // distinct maps among the last update's draws
  DevBuf s_theta, s_value, s_keys, s_vals, s_flag, s_pre, s_rkeys, s_rvals, s_selv, s_prow, s_hash, s_nt, s_krank,
      s_br;
  // ---- exact-joint reweighting of the kept hypotheses (glmb_set_joint_reweighting)
  bool joint_rw = false;
  bool last_perm = false;  // the last update re-ranked its children: child_perm maps rank -> child
  DevBuf j_corr, j_val, j_keys, child_perm, j_lw, j_tmp, rows3;

  // ---- learned pair proposal
  bool prop_loaded = false, prop_on = false, prop_measure = false;
  float prop_thr = 0.0f;  // logit threshold: pairs with a lower logit are removed
  float prop_t = 0.5f;    // the same threshold as a probability
  float prop_norm[12] = {};
  DevBuf prop_w;          // float32 parameters
  DevBuf pcnt, poff, ppre, pu, pi, plogit, slot_r, slot_part, slot_age, pm_part, pe_part, lz_t, mlp_part;
  DevBuf rmass;  // per detection: removed pairs' likelihood over the most likely hypothesis' instances
  DevBuf lz_r;   // per hypothesis: log mass with the removed pairs restored, then their normaliser
  int32_t* age_pin = nullptr;  // pinned host buffer of the label ages uploaded per update
  int age_cap = 0;
  DevBuf est_buf;  // estimate: presence flags and means of the estimated hypothesis' tracks
};

// opt-in stage trace (host side)
inline void trace(const Ctx& c, const char* stage, long long a = -1, long long b = -1) {
  if (!c.trace) return;
  std::fprintf(stderr, "[glmb] %s %lld %lld\n", stage, a, b);
  std::fflush(stderr);
}

// stages
void stage_predict(Ctx& c, int k);
void stage_update(Ctx& c, int k, const float* z, int M);
void stage_truncate(Ctx& c, int hmax, float tau);
// pieces of the update shared with the proposal
// with pairs: also the gated pairs of the learned update (c.pu / c.pi, count at scal[19]) and
// every instance's gated count (c.pcnt)
void gate_scores(Ctx& c, const float* z, int M, bool pairs = false);
void gate_lists(Ctx& c, int M, bool defer = false);
void assoc_norm(Ctx& c, int M);
// proposal (proposal.hip)
constexpr int kNFeat = 6, kNHid = 64, kNParam = 4673, kMaxThr = 16;
// fixed-point scale of the removed likelihood sums (exp(phi) <= gamma / (2 pi sigma^2) per pair)
constexpr double kRemovedScale = 281474976710656.0;  // 2^48
// the label inputs (existence, age) of the learned update on stream st
void prepare_slots(Ctx& c, int k, hipStream_t st);
// slots_ready: prepare_slots was queued on the side stream, joined by event fork[2]
void proposal_apply(Ctx& c, int k, int M, bool slots_ready = false);
void proposal_lost(Ctx& c, int k, const float* z, int M, const float* thr_prob, int T, double* lost);
int proposal_features(Ctx& c, int k, const float* z, int M, int cap, float* feat, int32_t* pair, float* target,
                      float* weight);
void mlp_forward(Ctx& c, const float* params, const float* norm, const float* feat, int n, float* logit);
void mlp_grad(Ctx& c, const float* params, const float* norm, const float* feat, const float* y, const float* w,
              int n, float* grad, float* loss);
void mlp_adam(Ctx& c, float* params, float* m, float* v, const float* g, int t, float lr, float b1, float b2,
              float eps);
// allocation-free gradient: the partial sums live in a fixed per-device array, whose address
// noalloc_setup (called by glmb_create with the context's device current) looks up once per device
void noalloc_setup(int device);
// sampled prediction (sample.hip): the kept outcomes in rank order, in the form the exact
// prediction's selection leaves them for the merge of identical track sets
struct PredictOut {
  int32_t* crow;     // [n][NS + NB] child rows
  uint64_t* hash;    // [n] row hashes
  int32_t* ntc;      // [n] track counts
  int32_t* parc;     // [n] parent hypotheses
  float* value;      // [n] log weights, rank order
  int32_t* keyrank;  // [n] canonical rank (below `nodes`)
  int nodes;
};
int sample_predict(Ctx& c, int k, int NS, int NB, int U, float ps, const float* br, int K, PredictOut& out);
// sampled children (sample.hip): returns the number of children taken (<= K), their values
// buffer (filled by sample_children_devs) and the kept draws in rank order
int sample_children(Ctx& c, int k, int M, int K, float** sel_value, const uint32_t** kept_draw);
void sample_children_devs(Ctx& c, int M, int nk, const uint32_t* kept_draw, float* sel_value, int32_t* depth,
                          int32_t* ch_h);
void sample_children_list(Ctx& c, int M, int nk, const uint32_t* kept_draw, const int32_t* ch_h, const int32_t* doff,
                          int32_t* dev_i, int32_t* dev_new, int32_t* dev_old);
void mlp_grad_noalloc(Ctx& c, const float* params, const float* norm, const float* feat, const float* y,
                      const float* w, int n, float* grad, float* loss);
void gc_state(Ctx& c);

// F and Q of the constant-velocity model (host constants passed to kernels)
struct CV {
  float dt, a, b, cq;  // Q blocks: a = q dt^3/3, b = q dt^2/2, cq = q dt
};
inline CV cv_of(const glmb_params& p) {
  const double dt = p.dt, q = p.q;
  return CV{(float)dt, (float)(q * dt * dt * dt / 3.0), (float)(q * dt * dt / 2.0), (float)(q * dt)};
}

__device__ __forceinline__ void cv_predict(const CV& cv, float* m, float* P) {
  const float dt = cv.dt;
  const float m0 = m[0] + dt * m[2], m1 = m[1] + dt * m[3];
  m[0] = m0;
  m[1] = m1;
  const float P00 = P[0], P01 = P[1], P02 = P[2], P03 = P[3], P11 = P[4], P12 = P[5], P13 = P[6], P22 = P[7],
              P23 = P[8], P33 = P[9];
  P[0] = P00 + dt * (2.0f * P02) + dt * dt * P22 + cv.a;
  P[1] = P01 + dt * (P03 + P12) + dt * dt * P23;
  P[2] = P02 + dt * P22 + cv.b;
  P[3] = P03 + dt * P23;
  P[4] = P11 + dt * (2.0f * P13) + dt * dt * P33 + cv.a;
  P[5] = P12 + dt * P23;
  P[6] = P13 + dt * P33 + cv.b;
  P[7] = P22 + cv.cq;
  P[8] = P23;
  P[9] = P33 + cv.cq;
}

// the association cells of the last association pass over M detections
inline CellView cells_of(Ctx& c, int M) {
  return CellView{c.best16.as<int16_t>(), c.dev1.as<float>(), c.lserel.as<float>(), c.tbits.as<uint32_t>(),
                  c.tpre.as<uint16_t>(), M, (M + 31) / 32};
}

}  // namespace glmb

// the opaque context of the C ABI
struct glmb_ctx {
  glmb::Ctx c;
};
