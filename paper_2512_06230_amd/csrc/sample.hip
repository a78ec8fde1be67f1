// The paper's own hypothesis generator (Sec. 3, hypothesis generation) on the GPU, as an
// alternative to the exact top-H_max selection of the update:
//
//   draws     per predicted hypothesis h, h_up association maps; in every map each detection
//             independently takes clutter or one of h's gated tracks, drawn from the
//             normalised row of the compatibility matrix (Eq. 2 entries over clutter and h's
//             tracks, options in key order: clutter, then tracks by label).  One wave per
//             map, lanes over the detections; the uniform numbers come from Philox4x32-10
//             (Salmon, Moraes, Dror and Shaw, SC'11) at counter (detection, draw, hypothesis
//             rank, 16 x scan + 1) under the caller's 64-bit seed, so every map is
//             reproducible on its own and every scan draws afresh;
//   distinct  maps sorted by (parent, 64-bit fingerprint); a map is kept when no earlier draw
//             of its run holds the same map (full comparison, so that fingerprint collisions
//             cannot merge different maps);
//   weights   the exact log weight of each kept map: parent weight times the likelihood of
//             its associations (the Eq. 2 entries and the miss term), as in the exact update;
//   cut       kept maps ranked by (weight descending, parent rank, first draw) and the best
//             H_max taken; tau and the child rows follow as in the exact update.
//
// A kept map is handed to the materialisation as its parent and its deviations from the
// parent's best association map, the form the exact selection produces.
#include "ctx.hpp"

namespace glmb {

namespace {

constexpr uint32_t kStreamAssoc = 1;

// Philox4x32-10: ten rounds of two 32 x 32 -> 64-bit products (constants 0xD2511F53 and
// 0xCD9E8D57) whose halves are mixed with the other two words and the key; the key advances
// by the Weyl increments 0x9E3779B9 and 0xBB67AE85 before every round after the first.  Only
// the first output word is used.
__device__ __forceinline__ uint32_t philox_first(uint32_t x0, uint32_t x1, uint32_t x2, uint32_t x3, uint32_t k0,
                                                 uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t lo0 = 0xD2511F53u * x0, hi0 = __umulhi(0xD2511F53u, x0);
    const uint32_t lo1 = 0xCD9E8D57u * x2, hi1 = __umulhi(0xCD9E8D57u, x2);
    const uint32_t y0 = hi1 ^ x1 ^ k0, y2 = hi0 ^ x3 ^ k1;
    x0 = y0;
    x1 = lo1;
    x2 = y2;
    x3 = lo0;
  }
  return x0;
}

// 24-bit uniform in [0, 1), exact in single precision
__device__ __forceinline__ float uniform24(uint32_t w) { return (float)(w >> 8) * (1.0f / 16777216.0f); }

// one wave per draw w = h * h_up + d, lanes over the detections
__global__ __launch_bounds__(256) void k_sample_draws(int H, int M, int h_up, int stride, const int32_t* rows,
                                                      const float* logw, const int32_t* ntrk, float gamma, float lgk,
                                                      const int32_t* coff, const int32_t* cand, const float* phi,
                                                      const uint32_t* cmax, uint32_t ctr3, uint32_t seed_lo,
                                                      uint32_t seed_hi, int16_t* theta, float* value, uint64_t* keys,
                                                      uint32_t* vals) {
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (w >= (int64_t)H * h_up) return;
  const int h = (int)(w / h_up), d = (int)(w % h_up);
  const int lane = lane_id();
  const int32_t* row = rows + (size_t)h * stride;
  float acc = 0.0f;
  uint64_t fp = 0;
  for (int i = lane; i < M; i += kWave) {
    const float c = o2f(cmax[i]);
    const int e0 = coff[i], e1 = coff[i + 1];
    const float pc = expf(lgk - c);
    float tot = pc;
    for (int e = e0; e < e1; ++e) {
      const int u = row[cand[e]];
      if (u < 0) continue;
      const float v = phi[(size_t)u * M + i];
      if (v > -INFINITY) tot += expf(v - c);
    }
    const float target = uniform24(philox_first((uint32_t)i, (uint32_t)d, (uint32_t)h, ctr3, seed_lo, seed_hi)) * tot;
    int pick = -1;
    float pv = lgk;
    float cum = pc;
    if (!(target < cum)) {
      for (int e = e0; e < e1; ++e) {
        const int u = row[cand[e]];
        if (u < 0) continue;
        const float v = phi[(size_t)u * M + i];
        if (!(v > -INFINITY)) continue;
        cum += expf(v - c);
        pick = cand[e];  // the last option takes what rounding leaves above the final sum
        pv = v;
        if (target < cum) break;
      }
    }
    theta[(size_t)w * M + i] = (int16_t)pick;
    acc += pv - c;
    fp ^= mix64(((uint64_t)(uint32_t)i << 32) | (uint32_t)(pick + 1));
  }
  for (int s = kWave / 2; s > 0; s >>= 1) {
    acc += __shfl_xor(acc, s, kWave);
    fp ^= __shfl_xor(fp, s, kWave);
  }
  if (lane == 0) {
    value[w] = logw[h] - gamma * (float)ntrk[h] + acc;
    keys[w] = ((uint64_t)(uint32_t)h << 40) | (fp >> 24);
    vals[w] = (uint32_t)w;
  }
}

// one thread per sorted draw: kept when no earlier draw of its (parent, fingerprint) run holds
// the same map (the sort is stable, so earlier means a smaller draw index)
__global__ void k_sample_distinct(int n, int M, const uint64_t* keys, const uint32_t* vals, const int16_t* theta,
                                  int32_t* flag) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint64_t k = keys[p];
  const int16_t* a = theta + (size_t)vals[p] * M;
  int keep = 1;
  for (int q = p - 1; q >= 0 && keys[q] == k; --q) {
    const int16_t* b = theta + (size_t)vals[q] * M;
    int i = 0;
    while (i < M && a[i] == b[i]) ++i;
    if (i == M) {
      keep = 0;
      break;
    }
  }
  flag[p] = keep;
}

// the kept draws, keyed for the rank order (weight descending, then draw index ascending,
// i.e. parent rank then draw)
__global__ void k_sample_rank_keys(int n, const int32_t* flag, const int32_t* pre, const uint32_t* vals,
                                   const float* value, uint64_t* rkeys, uint32_t* rvals) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n || !flag[p]) return;
  const uint32_t w = vals[p];
  rkeys[pre[p]] = ((uint64_t)(~f2o(value[w])) << 32) | w;
  rvals[pre[p]] = w;
}

// kept child c (draw rw[c]): its parent, value and number of deviations from the parent's best map
__global__ void k_sample_depth(int n, int M, int h_up, const uint32_t* rw, const int16_t* theta, const float* value,
                               CellView cv, float* sel_value, int32_t* depth, int32_t* ch_h) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const uint32_t w = rw[c];
  const int h = (int)(w / (uint32_t)h_up);
  const int16_t* t = theta + (size_t)w * M;
  int nd = 0;
  for (int i = 0; i < M; ++i) nd += (t[i] != (int16_t)(cv.best16[cv.at(h, i)] - 1));
  sel_value[c] = value[w];
  depth[c] = nd;
  ch_h[c] = h;
}

__global__ void k_sample_devs(int n, int M, const uint32_t* rw, const int16_t* theta, CellView cv,
                              const int32_t* ch_h, const int32_t* doff, int32_t* dev_i, int32_t* dev_new,
                              int32_t* dev_old) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int16_t* t = theta + (size_t)rw[c] * M;
  const int h = ch_h[c];
  int q = doff[c];
  for (int i = 0; i < M; ++i) {
    const int bo = (int)cv.best16[cv.at(h, i)] - 1;
    if ((int)t[i] == bo) continue;
    dev_i[q] = i;
    dev_new[q] = t[i];
    dev_old[q] = bo;
    ++q;
  }
}

// ---- the prediction's Bernoulli stage: one wave per draw w = h * h_up + d, lanes over the
// columns of the child row (label slots, then pending births)
__global__ __launch_bounds__(256) void k_psample_draws(int H, int NS, int NB, int stride, int U, int h_up,
                                                       const int32_t* rows, const float* logw, float ps,
                                                       const float* br, uint32_t ctr3, uint32_t seed_lo,
                                                       uint32_t seed_hi, int32_t* drow, float* value, uint64_t* keys,
                                                       uint32_t* vals, uint64_t* hfull, int32_t* ntv) {
  const int64_t w = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  if (w >= (int64_t)H * h_up) return;
  const int h = (int)(w / h_up), d = (int)(w % h_up);
  const int W2 = NS + NB;
  const int lane = lane_id();
  float acc = 0.0f;
  unsigned long long hs = 0;
  int cnt = 0;
  for (int s = lane; s < W2; s += kWave) {
    int o = -1;
    if (s < NS) {
      const int u = rows[(size_t)h * stride + s];
      if (u >= 0) {
        const float x = uniform24(philox_first((uint32_t)s, (uint32_t)d, (uint32_t)h, ctr3, seed_lo, seed_hi));
        if (x < ps) {
          o = u;
          acc += logf(ps);
        } else {
          acc += log1pf(-ps);
        }
      }
    } else {
      const float r = br[s - NS];
      const float x = uniform24(philox_first((uint32_t)s, (uint32_t)d, (uint32_t)h, ctr3, seed_lo, seed_hi));
      if (x < r) {
        o = U + (s - NS);
        acc += logf(r);
      } else {
        acc += log1pf(-r);
      }
    }
    drow[(size_t)w * W2 + s] = o;
    if (o >= 0) {
      hs += mix64(((uint64_t)(uint32_t)s << 32) | (uint32_t)o);
      ++cnt;
    }
  }
  for (int t = kWave / 2; t > 0; t >>= 1) {
    acc += __shfl_xor(acc, t, kWave);
    hs += __shfl_xor(hs, t, kWave);
    cnt += __shfl_xor(cnt, t, kWave);
  }
  if (lane == 0) {
    value[w] = logw[h] + acc;
    keys[w] = ((uint64_t)(uint32_t)h << 40) | (hs >> 24);
    vals[w] = (uint32_t)w;
    hfull[w] = hs;
    ntv[w] = cnt;
  }
}

// one thread per sorted draw: kept when no earlier draw of its (parent, fingerprint) run has
// the same row
__global__ void k_psample_distinct(int n, int W2, const uint64_t* keys, const uint32_t* vals, const int32_t* drow,
                                   int32_t* flag) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint64_t k = keys[p];
  const int32_t* a = drow + (size_t)vals[p] * W2;
  int keep = 1;
  for (int q = p - 1; q >= 0 && keys[q] == k; --q) {
    const int32_t* b = drow + (size_t)vals[q] * W2;
    int s = 0;
    while (s < W2 && a[s] == b[s]) ++s;
    if (s == W2) {
      keep = 0;
      break;
    }
  }
  flag[p] = keep;
}

// the kept outcome c (draw rw[c], in rank order): hash, track count, parent, value and canonical
// rank (the draw index: parent rank, then draw); then its row
__global__ void k_psample_meta(int n, int h_up, const uint32_t* rw, const float* value, const uint64_t* hfull,
                               const int32_t* ntv, uint64_t* hash, int32_t* ntc, int32_t* parc, float* sval,
                               int32_t* krank) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const uint32_t w = rw[c];
  hash[c] = hfull[w];
  ntc[c] = ntv[w];
  parc[c] = (int)(w / (uint32_t)h_up);
  sval[c] = value[w];
  krank[c] = (int)w;
}
__global__ void k_psample_rows(int n, int W2, const uint32_t* rw, const int32_t* drow, int32_t* crow) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * W2) return;
  const int c = (int)(t / W2), s = (int)(t % W2);
  crow[t] = drow[(size_t)rw[c] * W2 + s];
}

}  // namespace

int sample_predict(Ctx& c, int k, int NS, int NB, int U, float ps, const float* br, int K, PredictOut& out) {
  hipStream_t s = c.s;
  const int T = 256;
  const int H = c.nhyp, SW = c.stride, hu = c.sample_hup, W2 = NS + NB;
  const int64_t nd = (int64_t)H * hu;
  if (nd > (int64_t)INT32_MAX / 2 || (uint64_t)H >= (1ull << 24))
    throw Error{GLMB_E_CAPACITY, "sampled prediction: more than 2^30 draws or 2^24 hypotheses"};
  if (nd * std::max(1, W2) > ((int64_t)1 << 31))
    throw Error{GLMB_E_CAPACITY, "sampled prediction: draw rows above 8 GiB"};
  const int n = (int)nd;
  int32_t* drow = need<int32_t>(c.s_prow, std::max<int64_t>(1, nd * W2));
  float* value = need<float>(c.s_value, n);
  uint64_t* keys = need<uint64_t>(c.s_keys, n);
  uint32_t* vals = need<uint32_t>(c.s_vals, n);
  uint64_t* hfull = need<uint64_t>(c.s_hash, n);
  int32_t* ntv = need<int32_t>(c.s_nt, n);
  GLMB_LAUNCH(k_psample_draws, cdiv(nd * kWave, T), T, 0, s, H, NS, NB, SW, U, hu, c.rows.as<int32_t>(),
              c.logw.as<float>(), ps, br, (uint32_t)k * 16u + 4u, (uint32_t)c.sample_seed,
              (uint32_t)(c.sample_seed >> 32), drow, value, keys, vals, hfull, ntv);
  int hb = 0;
  while ((1 << hb) < H) ++hb;
  sort_pairs(keys, vals, n, 0, 40 + ((hb + 7) / 8) * 8, c.tk, c.tv, c.tmp, s);
  int32_t* flag = need<int32_t>(c.s_flag, n + 1);
  int32_t* pre = need<int32_t>(c.s_pre, n + 1);
  GLMB_LAUNCH(k_psample_distinct, cdiv(n, T), T, 0, s, n, W2, keys, vals, drow, flag);
  scan_excl(flag, pre, n, pre + n, c.tmp, s);
  int32_t nu = 0;
  nu = (int32_t)read_back(c.sb.hs, s, {{pre + n, 1}})[0];
  c.sample_unique = nu;
  uint64_t* rkeys = need<uint64_t>(c.s_rkeys, nu);
  uint32_t* rvals = need<uint32_t>(c.s_rvals, nu);
  GLMB_LAUNCH(k_sample_rank_keys, cdiv(n, T), T, 0, s, n, flag, pre, vals, value, rkeys, rvals);
  sort_pairs(rkeys, rvals, nu, 0, 64, c.tk, c.tv, c.tmp, s);
  const int nk = std::min(nu, K);
  out.crow = need<int32_t>(c.rows2, (int64_t)nk * W2 + 1);
  out.hash = need<uint64_t>(c.rec_keys, nk + 1);
  out.ntc = need<int32_t>(c.ntrk2, nk + 1);
  out.parc = need<int32_t>(c.child_par, nk + 1);
  out.value = need<float>(c.s_selv, nk + 1);
  out.keyrank = need<int32_t>(c.s_krank, nk + 1);
  out.nodes = n;
  GLMB_LAUNCH(k_psample_meta, cdiv(nk, T), T, 0, s, nk, hu, rvals, value, hfull, ntv, out.hash, out.ntc, out.parc,
              out.value, out.keyrank);
  if (W2 > 0) GLMB_LAUNCH(k_psample_rows, cdiv((int64_t)nk * W2, T), T, 0, s, nk, W2, rvals, drow, out.crow);
  return nk;
}

int sample_children(Ctx& c, int k, int M, int K, float** sel_value, const uint32_t** kept_draw) {
  hipStream_t s = c.s;
  const int T = 256;
  const int H = c.nhyp, SW = c.stride, hu = c.sample_hup;
  const int64_t nd = (int64_t)H * hu;
  if (nd > (int64_t)INT32_MAX / 2 || (uint64_t)H >= (1ull << 24))
    throw Error{GLMB_E_CAPACITY, "sampled update: more than 2^30 draws or 2^24 hypotheses"};
  if (M > 0 && nd * M > ((int64_t)1 << 34)) throw Error{GLMB_E_CAPACITY, "sampled update: draw store above 32 GiB"};
  const int n = (int)nd;
  int16_t* theta = need<int16_t>(c.s_theta, std::max<int64_t>(1, nd * M));
  float* value = need<float>(c.s_value, n);
  uint64_t* keys = need<uint64_t>(c.s_keys, n);
  uint32_t* vals = need<uint32_t>(c.s_vals, n);
  GLMB_LAUNCH(k_sample_draws, cdiv(nd * kWave, T), T, 0, s, H, M, hu, SW, c.rows.as<int32_t>(), c.logw.as<float>(),
              c.ntrk.as<int32_t>(), c.p.det_rate, logf(c.p.clutter_density), c.coff.as<int32_t>(),
              c.cand.as<int32_t>(), c.phi.as<float>(), c.cmax.as<uint32_t>(), (uint32_t)k * 16u + kStreamAssoc,
              (uint32_t)c.sample_seed,
              (uint32_t)(c.sample_seed >> 32), theta, value, keys, vals);
  int hb = 0;
  while ((1 << hb) < H) ++hb;
  sort_pairs(keys, vals, n, 0, 40 + ((hb + 7) / 8) * 8, c.tk, c.tv, c.tmp, s);
  int32_t* flag = need<int32_t>(c.s_flag, n + 1);
  int32_t* pre = need<int32_t>(c.s_pre, n + 1);
  GLMB_LAUNCH(k_sample_distinct, cdiv(n, T), T, 0, s, n, M, keys, vals, theta, flag);
  scan_excl(flag, pre, n, pre + n, c.tmp, s);
  int32_t nu = 0;
  nu = (int32_t)read_back(c.sb.hs, s, {{pre + n, 1}})[0];
  c.sample_unique = nu;
  uint64_t* rkeys = need<uint64_t>(c.s_rkeys, nu);
  uint32_t* rvals = need<uint32_t>(c.s_rvals, nu);
  GLMB_LAUNCH(k_sample_rank_keys, cdiv(n, T), T, 0, s, n, flag, pre, vals, value, rkeys, rvals);
  sort_pairs(rkeys, rvals, nu, 0, 64, c.tk, c.tv, c.tmp, s);
  *sel_value = need<float>(c.s_selv, std::min(nu, K) + 1);
  *kept_draw = rvals;
  return std::min(nu, K);
}

void sample_children_devs(Ctx& c, int M, int nk, const uint32_t* kept_draw, float* sel_value, int32_t* depth,
                          int32_t* ch_h) {
  GLMB_LAUNCH(k_sample_depth, cdiv(nk, 256), 256, 0, c.s, nk, M, c.sample_hup, kept_draw, c.s_theta.as<int16_t>(),
              c.s_value.as<float>(), cells_of(c, M), sel_value, depth, ch_h);
}

void sample_children_list(Ctx& c, int M, int nk, const uint32_t* kept_draw, const int32_t* ch_h, const int32_t* doff,
                          int32_t* dev_i, int32_t* dev_new, int32_t* dev_old) {
  GLMB_LAUNCH(k_sample_devs, cdiv(nk, 256), 256, 0, c.s, nk, M, kept_draw, c.s_theta.as<int16_t>(),
              cells_of(c, M), ch_h, doff, dev_i, dev_new, dev_old);
}

}  // namespace glmb
