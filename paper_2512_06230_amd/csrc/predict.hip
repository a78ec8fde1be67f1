// Prediction (Sec. 3, prediction step): every track is propagated with the constant-velocity
// Kalman prediction, the pending LMB birth components join as new labels, and of all the
// survive/die x include/exclude children of every hypothesis the H_max most likely are kept
// (same exact selection engine as the update: one group per track or birth, its single
// deviation is |log p - log(1 - p)|).  Children of different parents with the same track set
// are merged (weights added, representative = smallest canonical key), the result is
// normalised, and labels and instances no hypothesis uses any more are dropped.
#include <algorithm>
#include <cmath>

#include "ctx.hpp"

namespace glmb {

__global__ void k_kpredict(DInst* inst, int U, CV cv) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= U) return;
  DInst x = inst[u];
  cv_predict(cv, x.m, x.P);
  inst[u] = x;
}

__global__ void k_births_in(const DBirth* b, int NB, int U, int NS, CV cv, DInst* inst) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= NB) return;
  DInst x;
  for (int k = 0; k < 4; ++k) x.m[k] = b[j].m[k];
  for (int k = 0; k < 10; ++k) x.P[k] = b[j].P[k];
  cv_predict(cv, x.m, x.P);
  x.slot = NS + j;
  x.src = U + j;
  inst[U + j] = x;
}

// parent values and (value, multiplicity) pairs whose K-th largest bounds the cut
__global__ void k_pvals(int H, int NB, const float* logw, const int32_t* ntrk, float tb, float dt_, const float* bd,
                        float* V, float* vals, int32_t* mult) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= H) return;
  const float v = logw[h] + (float)ntrk[h] * tb;
  V[h] = v;
  const size_t o = (size_t)h * (NB + 2);
  vals[o] = v;
  mult[o] = 1;
  vals[o + 1] = v - dt_;
  mult[o + 1] = isinf(dt_) ? 0 : ntrk[h];
  for (int b = 0; b < NB; ++b) {
    vals[o + 2 + b] = v - bd[b];
    mult[o + 2 + b] = isinf(bd[b]) ? 0 : 1;
  }
}

// Items of a parent, already in (delta, generation) order: its tracks (group = slot, delta
// dt_, in slot order) and the births (group NS + b, delta bd[b]) whose value stays above the
// cut bound.  The births come sorted by (bd, b) (bs, bg); the nlt of them with bd < dt_ go
// before the tracks, the others after (tracks are generated first, so they lead among equal
// deltas).  V - bd is non-increasing along the sorted births, so the kept ones are a prefix.
// Counting pass (ioff null): icount[h]; writing pass: items at ioff[h].
__global__ __launch_bounds__(256) void k_pitems(int H, int nbs, int nlt, int stride, const int32_t* rows,
                                                const float* V, float dt_, const float* bs, const int32_t* bg,
                                                const float* t0, const int32_t* ioff, int32_t* icount, float* it_d,
                                                int32_t* it_g) {
  __shared__ int32_t wsum[4];
  __shared__ int32_t nkb_s;
  const int h = blockIdx.x;
  const float t = *t0, v = V[h];
  const bool tracks = !isinf(dt_) && v - dt_ >= t;
  if (threadIdx.x == 0) {
    int lo = 0, hi = nbs;  // kept births: the prefix with v - bs >= t
    while (lo < hi) {
      const int m = (lo + hi) >> 1;
      if (v - bs[m] >= t) lo = m + 1;
      else hi = m;
    }
    nkb_s = lo;
  }
  __syncthreads();
  const int nkb = nkb_s;
  const int nbefore = min(nlt, nkb);
  const int q0 = ioff ? ioff[h] : 0;
  int ntr = 0;
  if (tracks) {
    // present slots in slot order: block-wide compaction over the row
    for (int s0 = 0; s0 < stride; s0 += blockDim.x) {
      const int sl = s0 + threadIdx.x;
      const bool pres = sl < stride && rows[(size_t)h * stride + sl] >= 0;
      const uint64_t bal = __ballot(pres);
      const int w = threadIdx.x / kWave;
      if (lane_id() == 0) wsum[w] = __popcll(bal);
      __syncthreads();
      int before = 0, all = 0;
      for (int j = 0; j < (int)(blockDim.x / kWave); ++j) {
        if (j < w) before += wsum[j];
        all += wsum[j];
      }
      if (pres && ioff) {
        const int q = q0 + nbefore + ntr + before + __popcll(bal & lanemask_lt());
        it_d[q] = dt_;
        it_g[q] = sl;
      }
      ntr += all;
      __syncthreads();
    }
  }
  if (ioff)
    for (int j = threadIdx.x; j < nkb; j += blockDim.x) {
      const int q = j < nlt ? q0 + j : q0 + ntr + j;
      it_d[q] = bs[j];
      it_g[q] = bg[j];
    }
  if (!ioff && threadIdx.x == 0) icount[h] = ntr + nkb;
}

// child rows (width NS + NB), their hash and track count; one wave per child
__global__ __launch_bounds__(64) void k_prows(int n, int NS, int NB, int stride, int U, int t_yes,
                                              const int32_t* byes, const int32_t* sel_node, const int32_t* nd_parent,
                                              const int32_t* nd_item, const int32_t* nd_h, const int32_t* it_g,
                                              const int32_t* rows, int32_t* out, uint64_t* hash, int32_t* nt,
                                              int32_t* par) {
  const int c = blockIdx.x;
  const int W2 = NS + NB;
  const int node = sel_node[c];
  const int h = nd_h[node];
  int32_t* o = out + (size_t)c * W2;
  // slot s of the parent's row (kept tracks, or births taken), and its value with the child's
  // deviation at s (the track dropped or the birth not taken, and the reverse)
  auto dflt = [&](int s) {
    if (s < NS) return t_yes ? rows[(size_t)h * stride + s] : -1;
    return byes[s - NS] ? U + (s - NS) : -1;
  };
  auto flip = [&](int s) {
    if (s < NS) return t_yes ? -1 : rows[(size_t)h * stride + s];
    return byes[s - NS] ? -1 : U + (s - NS);
  };
  // hash and track count of the default row, taken while it is written; the deviations' slots
  // are corrected below (the hash is a sum over the occupied slots, so a slot's term can be
  // taken out exactly)
  unsigned long long hl = 0;
  int cl = 0;
  for (int s = threadIdx.x; s < W2; s += blockDim.x) {
    const int v = dflt(s);
    o[s] = v;
    if (v >= 0) {
      hl += mix64(((uint64_t)(uint32_t)s << 32) | (uint32_t)v);
      ++cl;
    }
  }
  for (int d = kWave / 2; d > 0; d >>= 1) {
    hl += __shfl_xor(hl, d, kWave);
    cl += __shfl_xor(cl, d, kWave);
  }
  __syncthreads();  // the default row is written before the deviations overwrite their slots
  if (threadIdx.x == 0) {
    // one deviation per slot (a child picks at most one item per group)
    for (int x = node; nd_item[x] >= 0; x = nd_parent[x]) {
      const int g = it_g[nd_item[x]];
      const int ov = dflt(g), nv = flip(g);
      o[g] = nv;
      if (ov >= 0) {
        hl -= mix64(((uint64_t)(uint32_t)g << 32) | (uint32_t)ov);
        --cl;
      }
      if (nv >= 0) {
        hl += mix64(((uint64_t)(uint32_t)g << 32) | (uint32_t)nv);
        ++cl;
      }
    }
    par[c] = h;
    hash[c] = hl;
    nt[c] = cl;
  }
}

// 16 bits of the row hash: children with equal rows share them, and rows of one run are
// compared by full hash and then in full, so a shorter key only lengthens a few runs (about
// n^2 / 2^17 pairs)
__global__ void k_hash_keys(int n, const uint64_t* hash, uint64_t* keys, uint32_t* vals) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  keys[c] = hash[c] >> 48;
  vals[c] = (uint32_t)c;
}

// eight words per step, all loaded before they are compared
__device__ bool rows_equal(const int32_t* a, const int32_t* b, int W2) {
  int s = 0;
  for (; s + 8 <= W2; s += 8) {
    int d = 0;
#pragma unroll
    for (int u = 0; u < 8; ++u) d |= a[s + u] ^ b[s + u];
    if (d) return false;
  }
  for (; s < W2; ++s)
    if (a[s] != b[s]) return false;
  return true;
}

// leader of every child: first child of its hash run with an identical row.  Equal rows have
// equal 64-bit row hashes, so rows are compared in full only where those agree.
__global__ void k_leaders(int n, int W2, const uint64_t* keys, const uint32_t* vals, const uint64_t* hash,
                          const int32_t* crow, int32_t* leader) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int r0 = p;
  while (r0 > 0 && keys[r0 - 1] == keys[p]) --r0;
  const uint32_t me = vals[p];
  const uint64_t hm = hash[me];
  int lead = (int)me;
  for (int q = r0; q < p; ++q) {
    const uint32_t o = vals[q];
    if (hash[o] == hm && rows_equal(crow + (size_t)o * W2, crow + (size_t)me * W2, W2)) {
      lead = (int)o;
      break;
    }
  }
  leader[me] = lead;
}

// merged value (log-add over the members, in hash-run order) and representative (the member
// with the smallest canonical key) of each leader; members follow their leader in its hash run
__global__ void k_merge(int n, const int32_t* leader, const float* val, const int32_t* keyrank, const uint64_t* keys,
                        const uint32_t* vals, int32_t* is_lead, float* mval, int32_t* mrank, int32_t* mrep) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int c = (int)vals[p];
  if (leader[c] != c) {
    is_lead[c] = 0;
    return;
  }
  is_lead[c] = 1;
  float m = val[c];
  int r = keyrank[c], rp = c;
  for (int q = p + 1; q < n && keys[q] == keys[p]; ++q) {
    const int j = (int)vals[q];
    if (leader[j] != c) continue;
    m = fmaxf(m, val[j]);
    if (keyrank[j] < r) {
      r = keyrank[j];
      rp = j;
    }
  }
  float acc = __expf(val[c] - m);
  for (int q = p + 1; q < n && keys[q] == keys[p]; ++q) {
    const int j = (int)vals[q];
    if (leader[j] == c) acc += __expf(val[j] - m);
  }
  mval[c] = m + __logf(acc);
  mrank[c] = r;
  mrep[c] = rp;
}

// sort keys of the merged hypotheses: value descending, then rank (below 2^rb)
__global__ void k_lead_keys(int n, int rb, const int32_t* is_lead, const int32_t* lpre, const float* mval,
                            const int32_t* mrank, uint64_t* keys, uint32_t* vals) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n || !is_lead[c]) return;
  const int d = lpre[c];
  keys[d] = ((uint64_t)(~f2o(mval[c])) << rb) | (uint32_t)mrank[c];
  vals[d] = (uint32_t)c;
}

// one workgroup per final hypothesis: the slots and instances its row uses.  Many rows share
// them, so a flag is written only where it still reads clear (all writers store the same 1).
__global__ void k_used(int W2, const uint32_t* order, const int32_t* crow, int32_t* sused, int32_t* uused) {
  const int32_t* r = crow + (size_t)order[blockIdx.x] * W2;
  for (int s = threadIdx.x; s < W2; s += blockDim.x) {
    const int u = r[s];
    if (u >= 0) {
      if (!sused[s]) sused[s] = 1;
      if (!uused[u]) uused[u] = 1;
    }
  }
}

// sum over the workgroup (every thread gets it)
__device__ __forceinline__ float bsum(float v, float* sh) {
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  __syncthreads();
  if (lane_id() == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  float r = 0.0f;
  for (int j = 0; j < (int)(blockDim.x / kWave); ++j) r += sh[j];
  return r;
}

// one block: normalised log weights of the merged hypotheses in final order (up to kPnormLds
// values gathered once and kept in LDS for the second pass)
constexpr int kPnormLds = 16384;
__global__ __launch_bounds__(1024) void k_pnorm(int nh, const uint32_t* order, const float* mval, float* logw) {
  __shared__ float red[16];
  __shared__ float lv[kPnormLds];
  const bool cached = nh <= kPnormLds;
  const float mx = mval[order[0]];
  float s = 0.0f;
  for (int h = threadIdx.x; h < nh; h += blockDim.x) {
    const float v = mval[order[h]];
    if (cached) lv[h] = v;
    s += __expf(v - mx);
  }
  s = bsum(s, red);  // its barriers also make lv visible
  const float L = mx + __logf(s);
  for (int h = threadIdx.x; h < nh; h += blockDim.x) logw[h] = (cached ? lv[h] : mval[order[h]]) - L;
}

// track count and parent of every final hypothesis (also when rows have no slots)
__global__ void k_final_meta(int nh, const uint32_t* order, const int32_t* nt_c, const int32_t* par_c,
                             const int32_t* mrep, int32_t* ntrk, int32_t* hpar) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= nh) return;
  const int c = (int)order[h];
  ntrk[h] = nt_c[c];
  hpar[h] = par_c[mrep[c]];
}

// one workgroup per final hypothesis h: its row over the kept slots
__global__ void k_final_rows(int W2, int NS2, const uint32_t* order, const int32_t* crow, const int32_t* spre,
                             const int32_t* sused, const int32_t* upre, int32_t* rows) {
  const int h = blockIdx.x;
  const int32_t* r = crow + (size_t)order[h] * W2;
  int32_t* o = rows + (size_t)h * NS2;
  for (int s = threadIdx.x; s < W2; s += blockDim.x) {
    if (!sused[s]) continue;
    const int u = r[s];
    o[spre[s]] = u >= 0 ? upre[u] : -1;
  }
}

__global__ void k_compact_inst(int U2, const int32_t* uused, const int32_t* upre, const int32_t* spre, const DInst* in,
                               DInst* out) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= U2 || !uused[u]) return;
  DInst x = in[u];
  x.slot = spre[x.slot];
  out[upre[u]] = x;
}

void stage_predict(Ctx& c, int k) {
  (void)k;
  hipStream_t s = c.s;
  const int T = 256;
  const int H = c.nhyp, U = c.ninst, NS = c.nslot, SW = c.stride, NB = c.nbirth;
  const glmb_params& p = c.p;
  // birth labels must sort after every label in use, in index order
  for (int b = 0; b < NB; ++b) {
    const auto& L = c.birth_lab[b];
    if ((NS > 0 && !(c.slot_lab.back() < L)) || (b > 0 && !(c.birth_lab[b - 1] < L)))
      throw Error{GLMB_E_ARG, "birth labels must sort after all existing labels"};
  }
  if (NS + NB > 32766) throw Error{GLMB_E_CAPACITY, "too many labels"};
  const CV cv = cv_of(p);
  int32_t* scal = need<int32_t>(c.scal, 64);
  float* t0 = (float*)(scal + 9);
  int32_t* tot = scal + 12;
  trace(c, "predict.begin", H, NB);
  // ---- Kalman prediction; births become instances U.. and slots NS..
  c.inst.reserve((size_t)(U + NB + 1) * sizeof(DInst), true, s);
  GLMB_LAUNCH(k_kpredict, cdiv(U, T), T, 0, s, c.inst.as<DInst>(), U, cv);
  GLMB_LAUNCH(k_births_in, cdiv(NB, T), T, 0, s, (const DBirth*)c.births.p, NB, U, NS, cv, c.inst.as<DInst>());
  // ---- dimensions
  const double ps = p.p_survive;
  const double ly = std::log(ps), ln = std::log1p(-ps);
  const int t_yes = ly >= ln ? 1 : 0;
  const float tb = (float)std::max(ly, ln);
  const float dt_ = (float)std::fabs(ly - ln);
  static_assert(sizeof(DBirth) % 4 == 0, "whole words");
  std::vector<DBirth> hb(NB);
  if (c.birth_host_ok && (int)c.birth_host.size() == NB) {
    hb = c.birth_host;  // read back with the last update's statistics, or imported
  } else if (NB) {
    const uint32_t* h = read_back(c.sb.hs, s, {{c.births.p, (int64_t)NB * (int64_t)(sizeof(DBirth) / 4)}});
    std::memcpy(hb.data(), h, (size_t)NB * sizeof(DBirth));
  }
  std::vector<float> bd(NB + 1, 0.0f);
  std::vector<int32_t> by(NB + 1, 0);
  for (int b = 0; b < NB; ++b) {
    const double r = hb[b].r;
    const double a = std::log(r), q = std::log1p(-r);
    by[b] = a >= q ? 1 : 0;
    bd[b] = (float)std::fabs(a - q);
  }
  // births with a finite deviation sorted by (bd, b), and how many lie below the tracks' dt_
  std::vector<int32_t> bord;
  for (int b = 0; b < NB; ++b)
    if (!std::isinf(bd[b])) bord.push_back(b);
  std::stable_sort(bord.begin(), bord.end(), [&](int32_t x, int32_t y) { return bd[x] < bd[y]; });
  const int nbs = (int)bord.size();
  int nlt = 0;
  while (nlt < nbs && bd[bord[nlt]] < dt_) ++nlt;
  std::vector<float> bsv(nbs + 1, 0.0f);
  std::vector<int32_t> bgv(nbs + 1, 0);
  for (int j = 0; j < nbs; ++j) {
    bsv[j] = bd[bord[j]];
    bgv[j] = NS + bord[j];
  }
  float* dbd = need<float>(c.bt, 4 * (int64_t)NB + 4);
  int32_t* dby = (int32_t*)(dbd + NB + 1);
  float* dbs = (float*)(dby + NB + 1);
  int32_t* dbg = (int32_t*)(dbs + NB + 1);
  {
    // the four birth tables packed into one upload
    std::vector<uint32_t> up(4 * (size_t)NB + 4, 0u);
    std::memcpy(up.data(), bd.data(), (NB + 1) * sizeof(float));
    std::memcpy(up.data() + NB + 1, by.data(), (NB + 1) * sizeof(int32_t));
    std::memcpy(up.data() + 2 * (NB + 1), bsv.data(), (nbs + 1) * sizeof(float));
    std::memcpy(up.data() + 3 * (NB + 1), bgv.data(), (nbs + 1) * sizeof(int32_t));
    GLMB_HIP(hipMemcpyAsync(dbd, up.data(), up.size() * sizeof(uint32_t), hipMemcpyHostToDevice, s));
  }
  const int W2 = NS + NB;
  int n = 0, nodes = 0;
  int32_t *crow = nullptr, *ntc = nullptr, *parc = nullptr;
  uint64_t* hash = nullptr;
  const float* selval = nullptr;
  const int32_t* keyrank = nullptr;
  if (c.sample_hup > 0) {
    // ---- the paper's generator: survive/die and include/exclude drawn per hypothesis
    trace(c, "predict.sampled", H, c.sample_hup);
    std::vector<float> hr(NB + 1, 0.0f);
    for (int b = 0; b < NB; ++b) hr[b] = hb[b].r;
    float* br = need<float>(c.s_br, NB + 1);
    GLMB_HIP(hipMemcpyAsync(br, hr.data(), (NB + 1) * sizeof(float), hipMemcpyHostToDevice, s));
    PredictOut po{};
    n = sample_predict(c, k, NS, NB, U, (float)p.p_survive, br, p.h_max, po);
    if (n < 1) throw Error{GLMB_E_STATE, "sampled prediction kept no hypothesis"};
    crow = po.crow;
    hash = po.hash;
    ntc = po.ntc;
    parc = po.parc;
    selval = po.value;
    keyrank = po.keyrank;
    nodes = po.nodes;
  } else {
    // ---- lower bound of the cut
    float* V = need<float>(c.bprime, H);
    float* pv = need<float>(c.pvals, (int64_t)H * (NB + 2));
    int32_t* pm = need<int32_t>(c.pmult, (int64_t)H * (NB + 2));
    GLMB_LAUNCH(k_pvals, cdiv(H, T), T, 0, s, H, NB, c.logw.as<float>(), c.ntrk.as<int32_t>(), tb, dt_, dbd, V, pv, pm);
    kth_bound_mult(pv, pm, H * (NB + 2), p.h_max, t0, c.tmp, s);
    // ---- items
    int32_t* icount = need<int32_t>(c.ccount, H + 1);
    GLMB_LAUNCH(k_pitems, H, 256, 0, s, H, nbs, nlt, SW, c.rows.as<int32_t>(), V, dt_, dbs, dbg, t0,
                (const int32_t*)nullptr, icount, (float*)nullptr, (int32_t*)nullptr);
    int32_t* itoff = need<int32_t>(c.it_off, H + 1);
    scan_excl(icount, itoff, H, itoff + H, c.tmp, s);
    // a parent has at most one item per present track and per birth: the item lists are
    // sized for that, so their total needs no round trip
    const int64_t icap = (int64_t)H * (SW + nbs) + 1;
    float* itd = need<float>(c.it_delta, icap);
    int32_t* itg = need<int32_t>(c.it_group, icap);
    GLMB_LAUNCH(k_pitems, H, 256, 0, s, H, nbs, nlt, SW, c.rows.as<int32_t>(), V, dt_, dbs, dbg, t0,
                (const int32_t*)itoff, icount, itd, itg);
    // ---- exact selection
    trace(c, "predict.select", H);
    if (c.force_coop) c.sel_multi[0] = true;
    SelectIn si{H, V, itoff, itd, itg, p.h_max, t0, &c.sel_multi[0], c.coop_ok, c.force_multi};
    si.group_bits = c.group_bits;
    Selected sel{};
    std::string serr;
    const int cap_nodes = p.cap_nodes > 0 ? p.cap_nodes : (1 << 22);
    glmb_status st = select_topk(si, cap_nodes, c.sb, sel, s, serr, c.trace);
    if (st != GLMB_OK) throw Error{st, serr};
    n = sel.n;
    if (n < 1) throw Error{GLMB_E_STATE, "prediction kept no hypothesis (non-finite weights?)"};
    trace(c, "predict.merge", n);
    // ---- child rows, duplicate merge
    crow = need<int32_t>(c.rows2, (int64_t)n * W2 + 1);
    hash = need<uint64_t>(c.rec_keys, n + 1);
    ntc = need<int32_t>(c.ntrk2, n + 1);
    parc = need<int32_t>(c.child_par, n + 1);
    GLMB_LAUNCH(k_prows, n, kWave, 0, s, n, NS, NB, SW, U, t_yes, dby, sel.node, sel.nd_parent, sel.nd_item, sel.nd_h, itg,
                c.rows.as<int32_t>(), crow, hash, ntc, parc);
    selval = sel.value;
    keyrank = sel.keyrank;
    nodes = sel.nodes;
  }
  uint64_t* hk = need<uint64_t>(c.keys, n + 1);
  uint32_t* hv = need<uint32_t>(c.vals32, n + 1);
  GLMB_LAUNCH(k_hash_keys, cdiv(n, T), T, 0, s, n, hash, hk, hv);
  sort_pairs(hk, hv, n, 0, 16, c.tk, c.tv, c.tmp, s);  // 16 hash bits: rows of a run are compared in full
  int32_t* leader = need<int32_t>(c.first, 4 * (int64_t)n + 4);
  int32_t* islead = leader + n + 1;
  int32_t* mrank = islead + n + 1;
  int32_t* mrep = mrank + n + 1;
  float* mval = need<float>(c.sel_logw, n + 1);
  GLMB_LAUNCH(k_leaders, cdiv(n, T), T, 0, s, n, W2, hk, hv, (const uint64_t*)hash, crow, leader);
  GLMB_LAUNCH(k_merge, cdiv(n, T), T, 0, s, n, leader, selval, keyrank, hk, hv, islead, mval, mrank, mrep);
  int32_t* lpre = need<int32_t>(c.pre, n + 1);
  scan_excl(islead, lpre, n, tot, c.tmp, s);
  const int32_t nh = (int32_t)read_back(c.sb.hs, s, {{tot, 1}})[0];
  uint64_t* lk = need<uint64_t>(c.rec_keys, nh + 1);
  uint32_t* lv = need<uint32_t>(c.rec_vals, nh + 1);
  int rb = 0;  // ranks are positions among the search's candidates, below its node count
  while (((int64_t)1 << rb) < (int64_t)nodes + 1) ++rb;
  rb = std::min(32, (rb + 7) / 8 * 8);
  GLMB_LAUNCH(k_lead_keys, cdiv(n, T), T, 0, s, n, rb, islead, lpre, mval, mrank, lk, lv);
  // without merged children the leaders are every child, in rank order already
  if (nh < n) sort_pairs(lk, lv, nh, 0, 32 + rb, c.tk, c.tv, c.tmp, s);
  // ---- normalise, garbage-collect labels and instances, final rows
  trace(c, "predict.gc", nh);
  float* nlw = need<float>(c.logw2, nh + 1);
  GLMB_LAUNCH(k_pnorm, 1, 1024, 0, s, nh, lv, mval, nlw);
  const int U2 = U + NB;
  // zeroed as whole 16-byte words (one fill kernel)
  const size_t nused = ((size_t)W2 + U2 + 2 + 3) & ~(size_t)3;
  int32_t* sused = need<int32_t>(c.flags, (int64_t)nused);
  int32_t* uused = sused + W2 + 1;
  GLMB_HIP(hipMemsetAsync(sused, 0, nused * sizeof(int32_t), s));
  GLMB_LAUNCH(k_used, nh, T, 0, s, W2, lv, crow, sused, uused);
  int32_t* spre = need<int32_t>(c.lpre, (int64_t)W2 + U2 + 4);
  int32_t* upre = spre + W2 + 2;
  scan_excl(sused, spre, W2, spre + W2, c.tmp, s);
  scan_excl(uused, upre, U2, upre + U2, c.tmp, s);
  std::vector<int32_t> hsu(W2 + 1);
  int32_t cnts[2];
  {
    const uint32_t* h = read_back(c.sb.hs, s, {{sused, W2}, {spre + W2, 1}, {upre + U2, 1}});
    std::memcpy(hsu.data(), h, (size_t)W2 * sizeof(int32_t));
    std::memcpy(cnts, h + W2, sizeof(cnts));
  }
  const int NS2 = cnts[0], Unew = cnts[1];
  int32_t* frows = need<int32_t>(c.prev_rows, (int64_t)nh * NS2 + 1);
  int32_t* fnt = need<int32_t>(c.hp_map, nh + 1);
  int32_t* fpar = need<int32_t>(c.hparent, nh + 1);
  // every (hypothesis, kept slot) entry is written: a kept slot is used, absent tracks as -1
  GLMB_LAUNCH(k_final_rows, nh, T, 0, s, W2, NS2, lv, crow, spre, sused, upre, frows);
  GLMB_LAUNCH(k_final_meta, cdiv(nh, T), T, 0, s, nh, lv, ntc, parc, mrep, fnt, fpar);
  DInst* ninst = (DInst*)need<uint8_t>(c.inst2, (int64_t)(Unew + 1) * sizeof(DInst));
  GLMB_LAUNCH(k_compact_inst, cdiv(U2, T), T, 0, s, U2, uused, upre, spre, c.inst.as<DInst>(), ninst);
  // the final rows, counts and weights become the primary buffers (the old ones, scratch)
  std::swap(c.rows, c.prev_rows);
  std::swap(c.ntrk, c.hp_map);
  std::swap(c.logw, c.logw2);
  std::swap(c.inst, c.inst2);
  // host label table
  std::vector<std::pair<int32_t, int32_t>> lab;
  for (int sl = 0; sl < W2; ++sl)
    if (hsu[sl]) lab.push_back(sl < NS ? c.slot_lab[sl] : c.birth_lab[sl - NS]);
  c.slot_lab.swap(lab);
  c.nslot = NS2;
  c.stride = NS2;
  c.ninst = Unew;
  c.nhyp = nh;
  c.nbirth = 0;
  c.birth_host.clear();
  c.birth_host_ok = true;
  c.birth_lab.clear();
}

}  // namespace glmb
