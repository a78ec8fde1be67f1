// C ABI of libglmb: argument checks, state import/export, truncation, estimate and
// diagnostics.  Every entry point converts internal errors to a glmb_status.
#include <algorithm>
#include <climits>
#include <cstdlib>
#include <cstring>
#include <map>

#include "ctx.hpp"

namespace glmb {

// ------------------------------------------------------------------ truncation
__device__ __forceinline__ float tsum(float v, float* sh) {
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  __syncthreads();
  if (lane_id() == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  float r = 0.0f;
  for (int j = 0; j < (int)(blockDim.x / kWave); ++j) r += sh[j];
  return r;
}

// one block: normalise the first n weights, keep the prefix before the first weight below tau
// (the first is always kept), renormalise.  The rows are in rank order (weight descending),
// so the prefix is the set of weights >= tau; the maximum is reduced rather than assumed.
// Up to kTruncLds weights are read from HBM once and kept in LDS for the later passes.
constexpr int kTruncLds = 16384;
__global__ __launch_bounds__(1024) void k_truncate(int n, float tau, float* logw, int32_t* nkeep) {
  __shared__ float red[32];
  __shared__ int32_t ired[16];
  __shared__ float lw[kTruncLds];
  const bool cached = n <= kTruncLds;
  float mx = -INFINITY;
  for (int h = threadIdx.x; h < n; h += blockDim.x) {
    const float v = logw[h];
    if (cached) lw[h] = v;
    mx = fmaxf(mx, v);
  }
  for (int d = kWave / 2; d > 0; d >>= 1) mx = fmaxf(mx, __shfl_xor(mx, d, kWave));
  if (lane_id() == 0) red[threadIdx.x / kWave] = mx;
  __syncthreads();
  mx = red[0];
  for (int j = 1; j < (int)(blockDim.x / kWave); ++j) mx = fmaxf(mx, red[j]);
  __syncthreads();
  const float* w = cached ? lw : logw;  // LDS entries written before the barrier above
  float s = 0.0f;
  for (int h = threadIdx.x; h < n; h += blockDim.x) s += __expf(w[h] - mx);
  s = tsum(s, red);
  const float L = mx + __logf(s);
  // first index h >= 1 whose normalised weight is below tau
  int first = n;
  if (tau > 0.0f)
    for (int h = 1 + threadIdx.x; h < n; h += blockDim.x)
      if (__expf(w[h] - L) < tau) {
        first = h;
        break;
      }
  for (int d = kWave / 2; d > 0; d >>= 1) first = min(first, __shfl_xor(first, d, kWave));
  if (lane_id() == 0) ired[threadIdx.x / kWave] = first;
  __syncthreads();
  int keep = ired[0];
  for (int j = 1; j < (int)(blockDim.x / kWave); ++j) keep = min(keep, ired[j]);
  float s2 = 0.0f;
  for (int h = threadIdx.x; h < keep; h += blockDim.x) s2 += __expf(w[h] - mx);
  s2 = tsum(s2, red + 16);
  const float L2 = mx + __logf(s2);
  __syncthreads();
  for (int h = threadIdx.x; h < keep; h += blockDim.x) logw[h] = w[h] - L2;
  if (threadIdx.x == 0) *nkeep = keep;
}

void stage_truncate(Ctx& c, int hmax, float tau) {
  const int n = std::min(c.nhyp, hmax);
  int32_t* scal = need<int32_t>(c.scal, 64);
  GLMB_LAUNCH(k_truncate, 1, 1024, 0, c.s, n, tau, c.logw.as<float>(), scal + 15);
  if (tau <= 0.0f) {  // no weight threshold: the first n are kept, no round trip
    c.nhyp = n;
    return;
  }
  c.nhyp = (int32_t)read_back(c.sb.hs, c.s, {{scal + 15, 1}})[0];
}

// ------------------------------------------------------------------ estimate
// Up to kEstLds hypotheses' weights and track counts are read from HBM once and kept in LDS
// for the passes over the cardinalities.
constexpr int kEstLds = 12288;
__global__ __launch_bounds__(1024) void k_estimate(int H, const float* logw, const int32_t* ntrk, int32_t* out) {
  __shared__ float red[32];
  __shared__ int32_t ired[32];
  __shared__ float lw[kEstLds];
  __shared__ int32_t ln[kEstLds];
  const bool cached = H <= kEstLds;
  // range of track counts
  int lo = INT_MAX, hi = -1;
  for (int h = threadIdx.x; h < H; h += blockDim.x) {
    const int n = ntrk[h];
    if (cached) {
      ln[h] = n;
      lw[h] = logw[h];
    }
    lo = min(lo, n);
    hi = max(hi, n);
  }
  for (int d = kWave / 2; d > 0; d >>= 1) {
    lo = min(lo, __shfl_xor(lo, d, kWave));
    hi = max(hi, __shfl_xor(hi, d, kWave));
  }
  if (lane_id() == 0) {
    ired[threadIdx.x / kWave] = lo;
    ired[16 + threadIdx.x / kWave] = hi;
  }
  __syncthreads();
  lo = INT_MAX;
  hi = -1;
  for (int j = 0; j < (int)(blockDim.x / kWave); ++j) {
    lo = min(lo, ired[j]);
    hi = max(hi, ired[16 + j]);
  }
  __syncthreads();
  const float* wv = cached ? lw : logw;  // LDS entries written before the barriers above
  const int32_t* nv = cached ? ln : ntrk;
  // cardinality distribution, one fixed-order reduction per count; MAP with ties to the smaller
  float best = -1.0f;
  int nbest = lo;
  for (int n = lo; n <= hi; ++n) {
    float s = 0.0f;
    for (int h = threadIdx.x; h < H; h += blockDim.x)
      if (nv[h] == n) s += __expf(wv[h]);
    s = tsum(s, red);
    if (s > best) {
      best = s;
      nbest = n;
    }
  }
  // most likely hypothesis of that size (rows are in rank order)
  int first = INT_MAX;
  for (int h = threadIdx.x; h < H; h += blockDim.x)
    if (nv[h] == nbest) {
      first = h;
      break;
    }
  for (int d = kWave / 2; d > 0; d >>= 1) first = min(first, __shfl_xor(first, d, kWave));
  __syncthreads();
  if (lane_id() == 0) ired[threadIdx.x / kWave] = first;
  __syncthreads();
  if (threadIdx.x == 0) {
    int f = INT_MAX;
    for (int j = 0; j < (int)(blockDim.x / kWave); ++j) f = min(f, ired[j]);
    out[0] = nbest;
    out[1] = f;
  }
}

// mean of every slot's instance in estimated hypothesis res[1] (present[s] = 0 if absent)
__global__ void k_est_gather(int NS, int stride, const int32_t* rows, const DInst* inst, const int32_t* res,
                             int32_t* present, float4* means) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= NS) return;
  const int h = res[1];
  const int u = h >= 0 && h != INT_MAX ? rows[(size_t)h * stride + s] : -1;
  present[s] = u >= 0 ? 1 : 0;
  means[s] = u >= 0 ? make_float4(inst[u].m[0], inst[u].m[1], inst[u].m[2], inst[u].m[3])
                    : make_float4(0.0f, 0.0f, 0.0f, 0.0f);
}

}  // namespace glmb

using glmb::Ctx;
using glmb::DInst;
using glmb::DBirth;
using glmb::Error;
using glmb::stream_sync;

namespace {

glmb_status fail(glmb_ctx* x, glmb_status st, const std::string& msg) {
  if (x) x->c.err = msg;
  return st;
}

template <class F>
glmb_status guarded(glmb_ctx* x, F&& f) {
  if (!x) return GLMB_E_ARG;
  if (!x->c.alive) return fail(x, GLMB_E_STATE, "context is not usable");
  try {
    GLMB_HIP(hipSetDevice(x->c.device));
    f(x->c);
    return GLMB_OK;
  } catch (const Error& e) {
    x->c.err = e.msg;
    if (e.st == GLMB_E_DEVICE) x->c.alive = false;
    return e.st;
  } catch (const std::exception& e) {
    x->c.err = e.what();
    return GLMB_E_STATE;
  }
}

float log_sum_exp(const std::vector<double>& v) {
  double m = -INFINITY;
  for (double x : v) m = std::max(m, x);
  double s = 0.0;
  for (double x : v) s += std::exp(x - m);
  return (float)(m + std::log(s));
}

void upload_state(Ctx& c, const std::vector<std::pair<int32_t, int32_t>>& labs, const std::vector<DInst>& inst,
                  const std::vector<int32_t>& rows, const std::vector<float>& logw, const std::vector<int32_t>& ntrk,
                  const std::vector<DBirth>& births, const std::vector<std::pair<int32_t, int32_t>>& blab,
                  const std::vector<int32_t>* parent = nullptr) {
  hipStream_t s = c.s;
  const int H = (int)logw.size();
  c.slot_lab = labs;
  c.nslot = (int)labs.size();
  c.stride = c.nslot;
  c.ninst = (int)inst.size();
  c.nhyp = H;
  c.nbirth = (int)births.size();
  c.birth_lab = blab;
  c.birth_host = births;
  c.birth_host_ok = true;
  auto up = [&](glmb::DevBuf& b, const void* src, size_t bytes) {
    b.reserve(std::max<size_t>(bytes, 64));
    if (bytes) GLMB_HIP(hipMemcpyAsync(b.p, src, bytes, hipMemcpyHostToDevice, s));
  };
  up(c.inst, inst.data(), inst.size() * sizeof(DInst));
  up(c.rows, rows.data(), rows.size() * sizeof(int32_t));
  up(c.logw, logw.data(), logw.size() * sizeof(float));
  up(c.ntrk, ntrk.data(), ntrk.size() * sizeof(int32_t));
  up(c.births, births.data(), births.size() * sizeof(DBirth));
  std::vector<int32_t> par(H);
  for (int h = 0; h < H; ++h) par[h] = parent ? (*parent)[h] : h;
  up(c.hparent, par.data(), par.size() * sizeof(int32_t));
  GLMB_HIP(stream_sync(s));
}

}  // namespace

extern "C" {

const char* glmb_status_string(glmb_status s) {
  switch (s) {
    case GLMB_OK: return "ok";
    case GLMB_E_ARG: return "invalid argument";
    case GLMB_E_CAPACITY: return "capacity exceeded";
    case GLMB_E_NOMEM: return "device allocation failed";
    case GLMB_E_DEVICE: return "HIP error";
    case GLMB_E_STATE: return "invalid state";
  }
  return "unknown status";
}

const char* glmb_last_error(const glmb_ctx* x) { return x ? x->c.err.c_str() : "null context"; }

glmb_status glmb_create(const glmb_params* p, int device, void* stream, glmb_ctx** out) {
  if (!p || !out) return GLMB_E_ARG;
  *out = nullptr;
  if (!(p->sigma_z > 0) || !(p->clutter_density > 0) || !(p->det_rate > 0) || !(p->gate_d2 > 0) || p->h_max < 1 ||
      !(p->p_survive >= 0 && p->p_survive <= 1) || !(p->dt > 0) || !(p->q >= 0) || !(p->tau >= 0 && p->tau < 1) ||
      !(p->birth_r_max >= 0 && p->birth_r_max <= 1) || p->cap_nodes < 0 || p->cap_labels < 0)
    return GLMB_E_ARG;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) return GLMB_E_DEVICE;
  glmb_ctx* x = new glmb_ctx();
  x->c.p = *p;
  if (x->c.p.cap_labels == 0) x->c.p.cap_labels = 4096;
  x->c.device = device;
  x->c.s = (hipStream_t)stream;
  const char* tr = std::getenv("GLMB_TRACE");
  x->c.trace = tr && tr[0] && tr[0] != '0';
  // diagnostic: GLMB_SEARCH_FORM=multi runs every selection on the host-driven multi-kernel
  // levels (the form a batched scene falls back to when its search outgrows one workgroup);
  // GLMB_SEARCH_FORM=coop starts every selection on the whole GPU (one cooperative launch)
  if (const char* sf = std::getenv("GLMB_SEARCH_FORM")) {
    x->c.force_multi = std::strcmp(sf, "multi") == 0;
    x->c.force_coop = std::strcmp(sf, "coop") == 0;
  }
  // diagnostic: GLMB_SEARCH_GROUP_BITS=0|1|2 limits the one-workgroup search's item tables in LDS
  // (0: none, 1: hashed group bits only, 2: exact bits allowed, the default)
  if (const char* gb = std::getenv("GLMB_SEARCH_GROUP_BITS")) {
    const int v = std::atoi(gb);
    if (v >= 0 && v <= 2) x->c.group_bits = v;
  }
  // diagnostic: GLMB_DP_BOUND_INFLATE=x (0 < x < 1) raises the update's counting bound part of
  // the way to the best value, so that its search keeps fewer than K children and the search
  // again from the caller's bound runs (results unchanged)
  if (const char* di = std::getenv("GLMB_DP_BOUND_INFLATE")) {
    const float v = std::strtof(di, nullptr);
    if (v > 0.f && v < 1.f) x->c.dp_inflate = v;
  }
  if (const char* ss = std::getenv("GLMB_SIDE_STREAM")) x->c.fork_ok = std::strcmp(ss, "0") != 0;
  if (const char* hb = std::getenv("GLMB_REC_HASH_BITS")) {
    const int bits = std::atoi(hb);
    if (bits >= 1 && bits < 16) x->c.rec_hash_mask = (1u << bits) - 1u;
  }
  glmb_status st = guarded(x, [&](Ctx& c) {
    glmb::noalloc_setup(c.device);  // the device is current here
    c.ev_ok = true;
    for (auto& e : c.ev) GLMB_HIP(hipEventCreate(&e));
    // one hypothesis without tracks
    upload_state(c, {}, {}, {}, {0.0f}, {0}, {}, {});
  });
  if (st != GLMB_OK) {
    delete x;
    return st;
  }
  *out = x;
  return GLMB_OK;
}

glmb_status glmb_destroy(glmb_ctx* x) {
  if (!x) return GLMB_E_ARG;
  (void)hipSetDevice(x->c.device);
  (void)hipStreamSynchronize(x->c.s);
  glmb::Ctx& c = x->c;
  if (c.s2) {
    (void)hipStreamSynchronize(c.s2);
    for (auto& e : c.fork) (void)hipEventDestroy(e);
    (void)hipStreamDestroy(c.s2);
  }
  glmb::DevBuf* bufs[] = {&c.inst, &c.inst2, &c.inst_nz, &c.inst_z, &c.logw, &c.ntrk, &c.rows, &c.hparent, &c.logw2,
                          &c.ntrk2, &c.rows2, &c.births, &c.births2, &c.diag_best, &c.diag_logpi, &c.diag_ru, &c.prev_rows,
                          &c.prev_src, &c.child_par, &c.dev_off, &c.dev_i, &c.dev_slot, &c.z, &c.cmax, &c.gbits,
                          &c.phi, &c.lbits, &c.lpre, &c.llen, &c.loff, &c.lmeas, &c.inst_beg, &c.ccnt, &c.coff,
                          &c.cand, &c.best16, &c.dev1, &c.lserel, &c.tbits, &c.tpre, &c.bprime, &c.lzprime, &c.cells,
                          &c.ccount, &c.coff2, &c.it_h, &c.it_delta, &c.it_group, &c.it_opt, &c.it_off, &c.keys,
                          &c.vals32, &c.scal, &c.sel_logw, &c.hp_map, &c.first, &c.dmask, &c.exc, &c.cmod, &c.recs,
                          &c.rec_keys, &c.rec_vals, &c.ids, &c.row_mark, &c.ru_part, &c.ru, &c.bt, &c.tmp, &c.tk,
                          &c.tv, &c.flags, &c.pre, &c.pmult, &c.pvals, &c.rec_m, &c.sb.nd_parent, &c.sb.nd_item, &c.sb.nd_h, &c.sb.nd_bloom,
                          &c.sb.nd_value, &c.sb.cnt, &c.sb.pre, &c.sb.pre64, &c.sb.flags, &c.sb.map, &c.sb.tmp,
                          &c.sb.tk, &c.sb.tv, &c.sb.keys, &c.sb.vals, &c.sb.sel_node, &c.sb.sel_val, &c.sb.sel_rank, &c.sb.hist,
                          &c.sb.scal, &c.sb.dp, &c.sb.dpc, &c.sb.dpa, &c.sb.cand, &c.prop_w, &c.pcnt, &c.poff, &c.ppre, &c.pu, &c.pi, &c.plogit, &c.slot_r,
                          &c.slot_part, &c.slot_age, &c.pm_part, &c.pe_part, &c.lz_t, &c.mlp_part, &c.est_buf, &c.ref_b1, &c.ref_opts, &c.ref_top, &c.ref_rest, &c.ref_tot, &c.hopts, &c.ref_sel, &c.rec_lead,
                          &c.s_theta, &c.s_value, &c.s_keys, &c.s_vals, &c.s_flag, &c.s_pre, &c.s_rkeys, &c.s_rvals,
                          &c.s_selv, &c.j_corr, &c.j_val, &c.j_keys, &c.child_perm, &c.j_lw, &c.j_tmp, &c.rows3,
                          &c.rmass, &c.lz_r, &c.s_prow, &c.s_hash, &c.s_nt, &c.s_krank, &c.s_br};
  for (auto* b : bufs) b->release();
  c.sb.hs.release();
  if (c.age_pin) (void)hipHostFree(c.age_pin);
  if (c.ev_ok)
    for (auto& e : c.ev) (void)hipEventDestroy(e);
  delete x;
  return GLMB_OK;
}

glmb_status glmb_import_state(glmb_ctx* x, const glmb_state_host* s) {
  if (!x || !s) return GLMB_E_ARG;
  if (s->n_inst < 0 || s->n_hyp < 1 || s->n_birth < 0 || (s->n_inst > 0 && (!s->inst_lab || !s->inst_m || !s->inst_P)) ||
      !s->hyp_logw || !s->hyp_off || (s->n_birth > 0 && (!s->birth_lab || !s->birth_m || !s->birth_P || !s->birth_r)))
    return fail(x, GLMB_E_ARG, "null pointer or negative count in the state");
  const int N = s->n_inst, H = s->n_hyp;
  if (s->hyp_off[0] != 0) return fail(x, GLMB_E_ARG, "hyp_off[0] must be 0");
  for (int h = 0; h < H; ++h)
    if (s->hyp_off[h + 1] < s->hyp_off[h]) return fail(x, GLMB_E_ARG, "hyp_off must be non-decreasing");
  if (s->hyp_off[H] > 0 && !s->hyp_idx) return fail(x, GLMB_E_ARG, "null hyp_idx");
  // labels -> slots
  std::map<std::pair<int32_t, int32_t>, int32_t> slot;
  for (int u = 0; u < N; ++u) slot[{s->inst_lab[2 * u], s->inst_lab[2 * u + 1]}] = 0;
  std::vector<std::pair<int32_t, int32_t>> labs;
  for (auto& kv : slot) {
    kv.second = (int32_t)labs.size();
    labs.push_back(kv.first);
  }
  if ((int)labs.size() > x->c.p.cap_labels || (int)labs.size() > 32766)
    return fail(x, GLMB_E_CAPACITY, "more labels than cap_labels");
  std::vector<int32_t> order(N);
  for (int u = 0; u < N; ++u) order[u] = u;
  std::vector<int32_t> us(N);
  for (int u = 0; u < N; ++u) us[u] = slot[{s->inst_lab[2 * u], s->inst_lab[2 * u + 1]}];
  std::stable_sort(order.begin(), order.end(), [&](int32_t a, int32_t b) { return us[a] < us[b]; });
  std::vector<int32_t> nid(N);
  std::vector<DInst> inst(N);
  for (int k = 0; k < N; ++k) {
    const int u = order[k];
    nid[u] = k;
    DInst d{};
    for (int j = 0; j < 4; ++j) {
      d.m[j] = s->inst_m[4 * u + j];
      if (!std::isfinite(d.m[j])) return fail(x, GLMB_E_ARG, "non-finite instance mean");
    }
    const float* P = s->inst_P + 16 * u;
    const int ij[10][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 1}, {1, 2}, {1, 3}, {2, 2}, {2, 3}, {3, 3}};
    for (int t = 0; t < 10; ++t) d.P[t] = P[4 * ij[t][0] + ij[t][1]];
    d.slot = us[u];
    d.src = u;
    inst[k] = d;
  }
  const int NS = (int)labs.size();
  // the rows are kept in rank order (weight descending): an input in another order is ranked
  // here, stably (equal weights keep the input order); hparent names the input position
  std::vector<int32_t> hord(H);
  for (int h = 0; h < H; ++h) {
    const float w = s->hyp_logw[h];
    if (!(w > -INFINITY) || std::isnan(w) || std::isinf(w)) return fail(x, GLMB_E_ARG, "non-finite hypothesis weight");
    hord[h] = h;
  }
  std::stable_sort(hord.begin(), hord.end(), [&](int32_t a, int32_t b) { return s->hyp_logw[a] > s->hyp_logw[b]; });
  std::vector<int32_t> rows((size_t)H * NS, -1);
  std::vector<int32_t> ntrk(H);
  std::vector<double> lw(H);
  for (int r0 = 0; r0 < H; ++r0) {
    const int h = hord[r0];
    lw[r0] = s->hyp_logw[h];
    for (int j = s->hyp_off[h]; j < s->hyp_off[h + 1]; ++j) {
      const int u = s->hyp_idx[j];
      if (u < 0 || u >= N) return fail(x, GLMB_E_ARG, "instance index out of range");
      int32_t& r = rows[(size_t)r0 * NS + us[u]];
      if (r >= 0) return fail(x, GLMB_E_ARG, "a hypothesis holds a label twice");
      r = nid[u];
    }
    ntrk[r0] = s->hyp_off[h + 1] - s->hyp_off[h];
  }
  const float L = log_sum_exp(lw);
  std::vector<float> logw(H);
  for (int h = 0; h < H; ++h) logw[h] = (float)(lw[h] - L);
  std::vector<DBirth> births(s->n_birth);
  std::vector<std::pair<int32_t, int32_t>> blab(s->n_birth);
  for (int b = 0; b < s->n_birth; ++b) {
    blab[b] = {s->birth_lab[2 * b], s->birth_lab[2 * b + 1]};
    if ((NS > 0 && !(labs.back() < blab[b])) || (b > 0 && !(blab[b - 1] < blab[b])))
      return fail(x, GLMB_E_ARG, "birth labels must sort after all instance labels");
    const float r = s->birth_r[b];
    if (!(r >= 0.0f && r <= 1.0f)) return fail(x, GLMB_E_ARG, "birth probability outside [0, 1]");
    DBirth d{};
    for (int j = 0; j < 4; ++j) d.m[j] = s->birth_m[4 * b + j];
    const float* P = s->birth_P + 16 * b;
    const int ij[10][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 1}, {1, 2}, {1, 3}, {2, 2}, {2, 3}, {3, 3}};
    for (int t = 0; t < 10; ++t) d.P[t] = P[4 * ij[t][0] + ij[t][1]];
    d.r = r;
    births[b] = d;
  }
  return guarded(x, [&](Ctx& c) {
    upload_state(c, labs, inst, rows, logw, ntrk, births, blab, &hord);
    c.last_M = -1;
  });
}

glmb_status glmb_state_sizes(glmb_ctx* x, int32_t* n_inst, int32_t* n_hyp, int32_t* n_idx, int32_t* n_birth) {
  if (!x || !n_inst || !n_hyp || !n_idx || !n_birth) return GLMB_E_ARG;
  return guarded(x, [&](Ctx& c) {
    *n_inst = c.ninst;
    *n_hyp = c.nhyp;
    *n_birth = c.nbirth;
    std::vector<int32_t> nt(c.nhyp);
    if (c.nhyp) GLMB_HIP(hipMemcpyAsync(nt.data(), c.ntrk.p, c.nhyp * sizeof(int32_t), hipMemcpyDeviceToHost, c.s));
    GLMB_HIP(stream_sync(c.s));
    int64_t t = 0;
    for (int v : nt) t += v;
    *n_idx = (int32_t)t;
  });
}

glmb_status glmb_export_state(glmb_ctx* x, glmb_state_host* o) {
  if (!x || !o) return GLMB_E_ARG;
  return guarded(x, [&](Ctx& c) {
    hipStream_t s = c.s;
    const int U = c.ninst, H = c.nhyp, NS = c.stride, NB = c.nbirth;
    std::vector<DInst> inst(U);
    std::vector<int32_t> rows((size_t)H * NS), par(H), nz(U), zz((size_t)U * 8);
    std::vector<float> logw(H);
    std::vector<DBirth> births(NB);
    if (U) GLMB_HIP(hipMemcpyAsync(inst.data(), c.inst.p, U * sizeof(DInst), hipMemcpyDeviceToHost, s));
    if (H * NS) GLMB_HIP(hipMemcpyAsync(rows.data(), c.rows.p, rows.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (H) GLMB_HIP(hipMemcpyAsync(logw.data(), c.logw.p, H * sizeof(float), hipMemcpyDeviceToHost, s));
    if (H) GLMB_HIP(hipMemcpyAsync(par.data(), c.hparent.p, H * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (NB) GLMB_HIP(hipMemcpyAsync(births.data(), c.births.p, NB * sizeof(DBirth), hipMemcpyDeviceToHost, s));
    const bool dets = c.last_M >= 0 && c.inst_nz.bytes >= (size_t)U * sizeof(int32_t) && U > 0;
    if (dets) {
      GLMB_HIP(hipMemcpyAsync(nz.data(), c.inst_nz.p, U * sizeof(int32_t), hipMemcpyDeviceToHost, s));
      GLMB_HIP(hipMemcpyAsync(zz.data(), c.inst_z.p, zz.size() * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    }
    GLMB_HIP(stream_sync(s));
    if (o->n_inst < U || o->n_hyp < H || o->n_birth < NB) throw Error{GLMB_E_CAPACITY, "export arrays too small"};
    const int ij[10][2] = {{0, 0}, {0, 1}, {0, 2}, {0, 3}, {1, 1}, {1, 2}, {1, 3}, {2, 2}, {2, 3}, {3, 3}};
    for (int u = 0; u < U; ++u) {
      o->inst_lab[2 * u] = c.slot_lab[inst[u].slot].first;
      o->inst_lab[2 * u + 1] = c.slot_lab[inst[u].slot].second;
      for (int j = 0; j < 4; ++j) o->inst_m[4 * u + j] = inst[u].m[j];
      for (int t = 0; t < 10; ++t) {
        o->inst_P[16 * u + 4 * ij[t][0] + ij[t][1]] = inst[u].P[t];
        o->inst_P[16 * u + 4 * ij[t][1] + ij[t][0]] = inst[u].P[t];
      }
      if (o->inst_src) o->inst_src[u] = inst[u].src;
      if (o->inst_nz) o->inst_nz[u] = dets ? nz[u] : 0;
      if (o->inst_z)
        for (int j = 0; j < 8; ++j) o->inst_z[8 * u + j] = dets && j < nz[u] ? zz[(size_t)u * 8 + j] : -1;
    }
    int j = 0;
    for (int h = 0; h < H; ++h) {
      o->hyp_logw[h] = logw[h];
      o->hyp_off[h] = j;
      for (int sl = 0; sl < NS; ++sl) {
        const int u = rows[(size_t)h * NS + sl];
        if (u >= 0) {
          if (j >= o->n_idx) throw Error{GLMB_E_CAPACITY, "export index array too small"};
          o->hyp_idx[j++] = u;
        }
      }
      if (o->hyp_parent) o->hyp_parent[h] = par[h];
    }
    o->hyp_off[H] = j;
    for (int b = 0; b < NB; ++b) {
      o->birth_lab[2 * b] = c.birth_lab[b].first;
      o->birth_lab[2 * b + 1] = c.birth_lab[b].second;
      for (int k = 0; k < 4; ++k) o->birth_m[4 * b + k] = births[b].m[k];
      for (int t = 0; t < 10; ++t) {
        o->birth_P[16 * b + 4 * ij[t][0] + ij[t][1]] = births[b].P[t];
        o->birth_P[16 * b + 4 * ij[t][1] + ij[t][0]] = births[b].P[t];
      }
      o->birth_r[b] = births[b].r;
    }
    o->n_inst = U;
    o->n_hyp = H;
    o->n_idx = j;
    o->n_birth = NB;
  });
}

glmb_status glmb_predict(glmb_ctx* x, int32_t k) {
  return guarded(x, [&](Ctx& c) {
    glmb::stage_predict(c, k);
    c.last_M = -1;
  });
}

glmb_status glmb_update(glmb_ctx* x, int32_t k, const float* z, int32_t M) {
  if (!x) return GLMB_E_ARG;
  if (M < 0 || (M > 0 && !z)) return fail(x, GLMB_E_ARG, "M < 0 or null detections");
  if (M > 32768) return fail(x, GLMB_E_CAPACITY, "more than 32768 detections in one scan");
  return guarded(x, [&](Ctx& c) { glmb::stage_update(c, k, z, M); });
}

glmb_status glmb_truncate(glmb_ctx* x, int32_t h_max, float tau) {
  if (!x) return GLMB_E_ARG;
  if (h_max < 1 || !(tau >= 0.0f && tau < 1.0f)) return fail(x, GLMB_E_ARG, "h_max < 1 or tau outside [0, 1)");
  return guarded(x, [&](Ctx& c) { glmb::stage_truncate(c, h_max, tau); });
}

glmb_status glmb_estimate(glmb_ctx* x, int32_t cap, int32_t* n_out, int32_t* labels_out, float* means_out) {
  if (!x || !n_out || cap < 0 || (cap > 0 && (!labels_out || !means_out))) return GLMB_E_ARG;
  glmb_status cap_err = GLMB_OK;
  glmb_status st = guarded(x, [&](Ctx& c) {
    int32_t* scal = glmb::need<int32_t>(c.scal, 64);
    GLMB_LAUNCH(glmb::k_estimate, 1, 1024, 0, c.s, c.nhyp, c.logw.as<float>(), c.ntrk.as<int32_t>(), scal + 20);
    // one gather and one round trip: the estimated hypothesis' row and its instance means
    const int NS = c.stride;
    int32_t* present = glmb::need<int32_t>(c.est_buf, 5 * (int64_t)NS + 4);
    float4* means = (float4*)(present + ((NS + 3) & ~3));
    GLMB_LAUNCH(glmb::k_est_gather, glmb::cdiv(NS, 256), 256, 0, c.s, NS, NS, c.rows.as<int32_t>(),
                c.inst.as<DInst>(), scal + 20, present, means);
    int32_t r[2];
    std::vector<int32_t> hp(NS);
    std::vector<float> hm(4 * (size_t)NS);
    {
      const uint32_t* h = glmb::read_back(c.sb.hs, c.s, {{scal + 20, 2}, {present, NS}, {means, 4 * (int64_t)NS}});
      std::memcpy(r, h, sizeof(r));
      std::memcpy(hp.data(), h + 2, (size_t)NS * sizeof(int32_t));
      std::memcpy(hm.data(), h + 2 + NS, (size_t)NS * sizeof(float4));
    }
    const int n = r[0];
    *n_out = n;
    if (n > cap) {
      cap_err = GLMB_E_CAPACITY;
      return;
    }
    int j = 0;
    for (int sl = 0; sl < NS && j < n; ++sl) {
      if (!hp[sl]) continue;
      labels_out[2 * j] = c.slot_lab[sl].first;
      labels_out[2 * j + 1] = c.slot_lab[sl].second;
      for (int k = 0; k < 4; ++k) means_out[4 * j + k] = hm[4 * (size_t)sl + k];
      ++j;
    }
  });
  if (st == GLMB_OK && cap_err != GLMB_OK) return fail(x, cap_err, "estimate larger than cap");
  return st;
}

glmb_status glmb_stats(glmb_ctx* x, glmb_step_stats* out) {
  if (!x || !out) return GLMB_E_ARG;
  return guarded(x, [&](Ctx& c) {
    GLMB_HIP(stream_sync(c.s));
    *out = c.stats;
  });
}

glmb_status glmb_update_diag(glmb_ctx* x, int32_t H, int32_t M, float* best, float* logpi, float* ru) {
  if (!x || !best || !logpi || (M > 0 && !ru)) return GLMB_E_ARG;
  return guarded(x, [&](Ctx& c) {
    if (c.last_M < 0 || H != c.last_H || M != c.last_M) throw Error{GLMB_E_STATE, "no update with these sizes"};
    GLMB_HIP(hipMemcpyAsync(best, c.diag_best.p, H * sizeof(float), hipMemcpyDeviceToHost, c.s));
    GLMB_HIP(hipMemcpyAsync(logpi, c.diag_logpi.p, H * sizeof(float), hipMemcpyDeviceToHost, c.s));
    if (M) GLMB_HIP(hipMemcpyAsync(ru, c.diag_ru.p, M * sizeof(float), hipMemcpyDeviceToHost, c.s));
    GLMB_HIP(stream_sync(c.s));
  });
}

glmb_status glmb_update_theta(glmb_ctx* x, int32_t n_hyp, int32_t M, int32_t* theta) {
  if (!x || (n_hyp * M > 0 && !theta)) return GLMB_E_ARG;
  return guarded(x, [&](Ctx& c) {
    if (c.last_M < 0 || M != c.last_M || n_hyp != c.nhyp) throw Error{GLMB_E_STATE, "no update with these sizes"};
    hipStream_t s = c.s;
    const int H = c.last_H, SW = c.last_stride, n = c.nhyp;
    std::vector<int16_t> best((size_t)H * M);
    // the predicted rows and instances of the last update are kept in rows2 / inst2
    const int UP = c.stats.n_inst_in;
    std::vector<int32_t> prows((size_t)H * SW), psrc(std::max(1, UP)), par(n), doff(n + 1);
    std::vector<DInst> pinst(std::max(1, UP));
    // association cells: hypothesis 0 dense, the other hypotheses' touched cells (see CellView)
    const int WM = (M + 31) / 32;
    std::vector<uint32_t> tb((size_t)H * WM);
    std::vector<uint16_t> tp((size_t)H * WM);
    if (H * M) {
      GLMB_HIP(hipMemcpyAsync(best.data(), c.best16.p, best.size() * 2, hipMemcpyDeviceToHost, s));
      GLMB_HIP(hipMemcpyAsync(tb.data(), c.tbits.p, tb.size() * 4, hipMemcpyDeviceToHost, s));
      GLMB_HIP(hipMemcpyAsync(tp.data(), c.tpre.p, tp.size() * 2, hipMemcpyDeviceToHost, s));
    }
    if (H * SW) GLMB_HIP(hipMemcpyAsync(prows.data(), c.rows2.p, prows.size() * 4, hipMemcpyDeviceToHost, s));
    if (UP) GLMB_HIP(hipMemcpyAsync(pinst.data(), c.inst2.p, (size_t)UP * sizeof(DInst), hipMemcpyDeviceToHost, s));
    GLMB_HIP(hipMemcpyAsync(par.data(), c.hparent.p, n * 4, hipMemcpyDeviceToHost, s));
    // children re-ranked by the exact-joint reweighting: child_perm names each one's position
    // in the selection's order, which the deviation lists follow
    std::vector<uint32_t> perm(n);
    for (int h = 0; h < n; ++h) perm[h] = (uint32_t)h;
    if (c.last_perm && n) GLMB_HIP(hipMemcpyAsync(perm.data(), c.child_perm.p, n * 4, hipMemcpyDeviceToHost, s));
    int nsel = n;
    for (int h = 0; h < n; ++h) nsel = std::max(nsel, (int)perm[h] + 1);
    doff.resize(nsel + 1);
    GLMB_HIP(hipMemcpyAsync(doff.data(), c.dev_off.p, (nsel + 1) * 4, hipMemcpyDeviceToHost, s));
    GLMB_HIP(stream_sync(s));
    for (int u = 0; u < UP; ++u) psrc[u] = pinst[u].src;
    const int nd = doff[nsel];
    std::vector<int32_t> di(nd), dn(nd);
    if (nd) {
      GLMB_HIP(hipMemcpyAsync(di.data(), c.dev_i.p, nd * 4, hipMemcpyDeviceToHost, s));
      GLMB_HIP(hipMemcpyAsync(dn.data(), c.dev_slot.p, nd * 4, hipMemcpyDeviceToHost, s));
      GLMB_HIP(stream_sync(s));
    }
    for (int h = 0; h < n; ++h) {
      const int ph = par[h];
      std::vector<int32_t> sl(M);
      for (int i = 0; i < M; ++i) {
        size_t at = (size_t)i;
        if (ph > 0) {
          const size_t wi = (size_t)ph * WM + (i >> 5);
          const uint32_t bit = 1u << (i & 31);
          if (tb[wi] & bit) at = (size_t)ph * M + tp[wi] + __builtin_popcount(tb[wi] & (bit - 1u));
        }
        sl[i] = (int)best[at] - 1;
      }
      const int o = (int)perm[h];
      for (int q = doff[o]; q < doff[o + 1]; ++q) sl[di[q]] = dn[q];
      for (int i = 0; i < M; ++i)
        theta[(size_t)h * M + i] = sl[i] < 0 ? -1 : psrc[prows[(size_t)ph * SW + sl[i]]];
    }
  });
}

glmb_status glmb_set_proposal(glmb_ctx* x, const float* params, const float* norm, float threshold, int32_t flags) {
  if (!x) return GLMB_E_ARG;
  if (!params) {
    x->c.prop_on = false;
    x->c.prop_loaded = false;
    return GLMB_OK;
  }
  if (!norm || !(threshold > 0.0f && threshold < 1.0f) || (flags & ~3))
    return fail(x, GLMB_E_ARG, "null norm, threshold outside (0, 1) or unknown flags");
  for (int k = 0; k < 12; ++k)
    if (!std::isfinite(norm[k]) || (k >= 6 && !(norm[k] > 0.0f)))
      return fail(x, GLMB_E_ARG, "feature norm must be finite with positive standard deviations");
  return guarded(x, [&](Ctx& c) {
    float* w = glmb::need<float>(c.prop_w, glmb::kNParam);
    GLMB_HIP(hipMemcpyAsync(w, params, glmb::kNParam * sizeof(float), hipMemcpyDeviceToDevice, c.s));
    GLMB_HIP(stream_sync(c.s));
    std::memcpy(c.prop_norm, norm, sizeof(c.prop_norm));
    c.prop_thr = (float)std::log((double)threshold / (1.0 - (double)threshold));
    c.prop_t = threshold;
    c.prop_loaded = true;
    c.prop_on = (flags & GLMB_PROPOSAL_APPLY) != 0;
    c.prop_measure = (flags & GLMB_PROPOSAL_MEASURE) != 0;
  });
}

glmb_status glmb_pair_features(glmb_ctx* x, int32_t k, const float* z, int32_t M, int32_t cap, float* feat,
                               int32_t* pair, float* target, float* weight, int32_t* n_pairs) {
  if (!x || !n_pairs || cap < 0 || M < 0 || (M > 0 && !z) || (cap > 0 && (!feat || !pair || !target || !weight)))
    return GLMB_E_ARG;
  if (M > 32768) return fail(x, GLMB_E_CAPACITY, "more than 32768 detections in one scan");
  int n = 0;
  glmb_status st = guarded(x, [&](Ctx& c) { n = glmb::proposal_features(c, k, z, M, cap, feat, pair, target, weight); });
  if (st != GLMB_OK) return st;
  *n_pairs = n;
  if (n > cap) return fail(x, GLMB_E_CAPACITY, "more gated pairs than cap");
  return GLMB_OK;
}

glmb_status glmb_proposal_lost(glmb_ctx* x, int32_t k, const float* z, int32_t M, int32_t T, const float* thr,
                               double* lost) {
  if (!x || !thr || !lost || M < 0 || (M > 0 && !z)) return GLMB_E_ARG;
  if (T < 1 || T > glmb::kMaxThr) return fail(x, GLMB_E_ARG, "1 <= T <= 16 thresholds");
  for (int j = 0; j < T; ++j)
    if (!(thr[j] > 0.0f && thr[j] < 1.0f)) return fail(x, GLMB_E_ARG, "thresholds must lie in (0, 1)");
  if (M > 32768) return fail(x, GLMB_E_CAPACITY, "more than 32768 detections in one scan");
  return guarded(x, [&](Ctx& c) {
    if (!c.prop_loaded) throw Error{GLMB_E_STATE, "no proposal parameters loaded"};
    glmb::proposal_lost(c, k, z, M, thr, T, lost);
  });
}

glmb_status glmb_mlp_forward(glmb_ctx* x, const float* params, const float* norm, const float* feat, int32_t n,
                             float* logit) {
  if (!x || !params || !norm || n < 0 || (n > 0 && (!feat || !logit))) return GLMB_E_ARG;
  return guarded(x, [&](Ctx& c) { glmb::mlp_forward(c, params, norm, feat, n, logit); });
}

glmb_status glmb_mlp_grad(glmb_ctx* x, const float* params, const float* norm, const float* feat, const float* y,
                          const float* w, int32_t n, float* grad, float* loss) {
  if (!x || !params || !norm || !grad || !loss || n < 1 || !feat || !y || !w) return GLMB_E_ARG;
  return guarded(x, [&](Ctx& c) { glmb::mlp_grad(c, params, norm, feat, y, w, n, grad, loss); });
}

glmb_status glmb_set_sampling(glmb_ctx* x, int32_t h_up, uint64_t seed) {
  if (!x) return GLMB_E_ARG;
  if (h_up < 0 || h_up > 65536) return fail(x, GLMB_E_ARG, "h_up must lie in [0, 65536]");
  x->c.sample_hup = h_up;
  x->c.sample_seed = seed;
  return GLMB_OK;
}

glmb_status glmb_set_joint_reweighting(glmb_ctx* x, int32_t on) {
  if (!x) return GLMB_E_ARG;
  x->c.joint_rw = on != 0;
  return GLMB_OK;
}

glmb_status glmb_mlp_grad_noalloc(glmb_ctx* x, const float* params, const float* norm, const float* feat,
                                  const float* y, const float* w, int32_t n, float* grad, float* loss) {
  if (!x || !params || !norm || !grad || !loss || n < 1 || !feat || !y || !w) return GLMB_E_ARG;
  if (n > GLMB_MLP_NOALLOC_MAX) return fail(x, GLMB_E_CAPACITY, "more samples than GLMB_MLP_NOALLOC_MAX");
  return guarded(x, [&](Ctx& c) { glmb::mlp_grad_noalloc(c, params, norm, feat, y, w, n, grad, loss); });
}

glmb_status glmb_mlp_adam(glmb_ctx* x, float* params, float* m, float* v, const float* g, int32_t t, float lr,
                          float beta1, float beta2, float eps) {
  if (!x || !params || !m || !v || !g || t < 1 || !(lr > 0.0f) || !(beta1 >= 0.0f && beta1 < 1.0f) ||
      !(beta2 >= 0.0f && beta2 < 1.0f) || !(eps > 0.0f))
    return GLMB_E_ARG;
  return guarded(x, [&](Ctx& c) { glmb::mlp_adam(c, params, m, v, g, t, lr, beta1, beta2, eps); });
}

}  // extern "C"
