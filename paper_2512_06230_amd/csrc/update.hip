// The update of Sec. 3 (Eq. 2 through the end of the section) on the GPU.
//
//   U1  gate + score  every (track instance, detection) pair: Mahalanobis gate and the
//       log Eq. 2 entry phi = log gamma + log N(z; H m, S); per-label detection lists.
//   U2  for every (hypothesis, detection) cell: best option, first deviation and the
//       log-sum-exp over {clutter} + gated tracks of the hypothesis; per hypothesis the
//       best-child log weight B_h and the log mass of all its children (factorised).
//   U3  exact top-H_max children: per-parent deviation item lists under a lower bound
//       of the cut, then the level-synchronous selection engine; tau pruning.
//   U4  one new instance per distinct (predicted instance, detection set) with the
//       multi-detection Kalman update; child hypothesis rows.
//   births for the next scan from detections the posterior attributes to clutter.
//
// Numerics: FP32 throughout.  Per-hypothesis sums are accumulated relative to a
// per-detection reference c_i = max(log kappa, max phi_ui), so that hypotheses which agree
// on a detection contribute an exact 0 there (log weights of ~-5000 never appear); the
// common constant sum_i c_i cancels in every normalised quantity.
#include <climits>

#include "ctx.hpp"

namespace glmb {

enum : uint32_t { ERR_BIRTH = 1, ERR_DEPTH = 4, ERR_NAN = 8 };

// ------------------------------------------------------------------ U0 / U1
// detections in; with pcnt (the learned update), also the n per-instance gated counts and the
// M + 1 removed masses zeroed
__global__ void k_z_in(const float* zin, int M, float2* z, uint32_t* errf, int32_t* pcnt, int n,
                       unsigned long long* rmass) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (pcnt && i < n) pcnt[i] = 0;
  if (rmass && i <= M) rmass[i] = 0ull;
  if (i >= M) return;
  const float x = zin[2 * i], y = zin[2 * i + 1];
  if (!(x == x) || !(y == y) || isinf(x) || isinf(y)) atomicOr(errf, ERR_NAN);
  z[i] = make_float2(x, y);
}

__global__ void k_fill_u32(uint32_t* p, int n, uint32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}
__global__ void k_fill_i32(int32_t* p, int n, int32_t v) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

// one wave per (instance, chunk of 64 detections)
// One wave per (group of kGateIpw instances, 64 detections): per instance the gate test and
// score of its 64 pairs, one ballot into the gate bitmap; the running maximum of the scores
// goes to the per-detection reference c_i with one atomic per lane for the whole group.
constexpr int kGateIpw = 8;
// With pn (the learned update): every instance's gated count is added to pcnt, and the gated
// pairs are appended to (pu, pi), one reservation per wave, each wave's pairs by (instance,
// detection); the order of the waves' runs is arbitrary.
__global__ __launch_bounds__(256) void k_gate(const DInst* inst, int U, const float2* z, int M, int W, float sig2,
                                              float gate, float lgc, uint32_t* gbits, float* phi, uint32_t* cmax,
                                              unsigned long long* ngated, int32_t* pcnt, int32_t* pn, int32_t* pu,
                                              int32_t* pi) {
  const int gw = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  const int nch = (M + kWave - 1) / kWave;
  const int ug = gw / nch, ch = gw % nch;
  const int lane = lane_id();
  const int i = ch * kWave + lane;
  const float2 zi = i < M ? z[i] : make_float2(0.0f, 0.0f);
  float fmx = -INFINITY;
  int ng = 0;
  uint32_t gk = 0;  // this lane's gate decisions, one bit per instance of the group
  for (int k = 0; k < kGateIpw; ++k) {
    const int u = ug * kGateIpw + k;
    if (u >= U) break;  // the same for the whole wave
    bool g = false;
    if (i < M) {
      const DInst& x = inst[u];
      const float s00 = x.P[0] + sig2, s01 = x.P[1], s11 = x.P[4] + sig2;
      const float det = s00 * s11 - s01 * s01;
      const float n0 = zi.x - x.m[0], n1 = zi.y - x.m[1];
      const float qd = s11 * n0 * n0 - 2.0f * s01 * n0 * n1 + s00 * n1 * n1;
      const float d2 = qd / det;
      g = d2 <= gate;
      const float f = g ? lgc - 0.5f * __logf(det) - 0.5f * d2 : -INFINITY;
      phi[(size_t)u * M + i] = f;
      fmx = fmaxf(fmx, f);
    }
    const uint64_t bal = __ballot(g);
    if (lane == 0) {
      gbits[(size_t)u * W + 2 * ch] = (uint32_t)bal;
      if (2 * ch + 1 < W) gbits[(size_t)u * W + 2 * ch + 1] = (uint32_t)(bal >> 32);
      if (pn && bal) atomicAdd(&pcnt[u], (int32_t)__popcll(bal));
    }
    if (g) gk |= 1u << k;
    ng += __popcll(bal);
  }
  if (pn && ng) {
    int base = 0;
    if (lane == 0) base = atomicAdd(pn, ng);
    base = __shfl(base, 0, kWave);
    for (int k = 0; k < kGateIpw; ++k) {
      const int u = ug * kGateIpw + k;
      if (u >= U) break;
      const bool g = (gk >> k) & 1u;
      const uint64_t bal = __ballot(g);
      if (g) {
        const int at = base + __popcll(bal & lanemask_lt());
        pu[at] = u;
        pi[at] = i;
      }
      base += __popcll(bal);
    }
  }
  if (fmx > -INFINITY) atomicMax(&cmax[i], f2o(fmx));
  // one counter update per workgroup
  __shared__ int32_t wg[4];
  if (lane == 0) wg[threadIdx.x / kWave] = ng;
  __syncthreads();
  if (threadIdx.x == 0) {
    const int n = wg[0] + wg[1] + wg[2] + wg[3];
    if (n) atomicAdd(ngated, (unsigned long long)n);
  }
}

// first instance of every slot (instances are sorted by slot; a slot may hold none)
__global__ void k_inst_beg(const DInst* inst, int U, int nslot, int32_t* beg) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s > nslot) return;
  int a = 0, b = U;
  while (a < b) {
    const int m = (a + b) >> 1;
    if (inst[m].slot < s) a = m + 1;
    else b = m;
  }
  beg[s] = a;
}

// per label: union of its instances' gate bits, prefix popcounts, list length
__global__ __launch_bounds__(256) void k_label_bits(const uint32_t* gbits, const int32_t* beg, int W, uint32_t* lbits,
                                                    int32_t* lpre, int32_t* llen, uint32_t* errf, int32_t* maxlen) {
  __shared__ int32_t pc[1024];
  const int s = blockIdx.x;
  for (int w = threadIdx.x; w < W; w += blockDim.x) {
    uint32_t acc = 0;
    for (int u = beg[s]; u < beg[s + 1]; ++u) acc |= gbits[(size_t)u * W + w];
    lbits[(size_t)s * W + w] = acc;
    pc[w] = __popc(acc);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    int run = 0;
    for (int w = 0; w < W; ++w) {
      lpre[(size_t)s * W + w] = run;
      run += pc[w];
    }
    llen[s] = run;
    if (run) atomicMax(maxlen, run);
  }
}

__global__ void k_label_list(const uint32_t* lbits, const int32_t* lpre, const int32_t* loff, int nslot, int W,
                             int32_t* lmeas) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= nslot * W) return;
  const int s = t / W, w = t % W;
  uint32_t b = lbits[t];
  int pos = loff[s] + lpre[t];
  while (b) {
    const int k = __ffs(b) - 1;
    lmeas[pos++] = w * 32 + k;
    b &= b - 1;
  }
}

// per detection (one wave each): candidate label slots in ascending order
__global__ __launch_bounds__(256) void k_cand(const uint32_t* lbits, int nslot, int W, int M, const int32_t* coff,
                                              int32_t* ccnt, int32_t* cand) {
  const int i = (int)((blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  if (i >= M) return;
  const int lane = lane_id();
  int run = 0;
  for (int s0 = 0; s0 < nslot; s0 += kWave) {
    const int s = s0 + lane;
    const bool bit = s < nslot && ((lbits[(size_t)s * W + (i >> 5)] >> (i & 31)) & 1u);
    const uint64_t bal = __ballot(bit);
    if (coff && bit) cand[coff[i] + run + __popcll(bal & lanemask_lt())] = s;
    run += __popcll(bal);
  }
  if (!coff && lane == 0) ccnt[i] = run;
}

// ------------------------------------------------------------------ U2
__device__ __forceinline__ float block_sum_f(float v, float* sh) {
  // fixed-order tree: wave butterfly, then waves in order
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) sh[w] = v;
  __syncthreads();
  float r = 0.0f;
  for (int j = 0; j < (int)(blockDim.x / kWave); ++j) r += sh[j];
  return r;
}
__device__ __forceinline__ float block_max_f(float v, float* sh) {
  for (int d = kWave / 2; d > 0; d >>= 1) v = fmaxf(v, __shfl_xor(v, d, kWave));
  const int w = threadIdx.x / kWave;
  __syncthreads();
  if (lane_id() == 0) sh[w] = v;
  __syncthreads();
  float r = -INFINITY;
  for (int j = 0; j < (int)(blockDim.x / kWave); ++j) r = fmaxf(r, sh[j]);
  return r;
}

// Cell (h, i) from the hypothesis row in LDS: best option (slot + 1, 0 = clutter), first
// deviation, log-sum-exp over clutter and the gated tracks; returns the best value b1.
struct CellOut {
  float b1, l;
  unsigned opts;
};
// The first kTop options of a cell in (value descending, candidate position) order, clutter
// (slot -1) first among equals; unused entries hold -inf and slot -2.  Candidate position order
// is label-slot order (the candidate lists are built slot by slot).
constexpr int kTop = 8;
struct TopT {
  float v[kTop];
  int32_t s[kTop];
};
// a cell's listed options with their mass exp(v - c_i) (stored once by hypothesis 0's pass)
struct TopE {
  TopT t;
  float e[kTop];
};
__device__ __forceinline__ CellOut assoc_cell(int i, int M, const int32_t* row, float lgk, const int32_t* coff,
                                              const int32_t* cand, const float* phi, int16_t* best16, float* dev1,
                                              size_t cell, float c) {
  float b1 = lgk, b2 = -INFINITY, mx = lgk, sm = 1.0f;
  int k1 = -1;
  unsigned opts = 0;
  auto take = [&](int s, float f) {
    if (!(f > -INFINITY)) return;  // label absent from the hypothesis, or not gated
    ++opts;
    if (f > b1) {
      b2 = b1;
      b1 = f;
      k1 = s;
    } else if (f > b2) {
      b2 = f;
    }
    if (f > mx) {
      sm = sm * __expf(mx - f) + 1.0f;
      mx = f;
    } else {
      sm += __expf(f - mx);
    }
  };
  auto gather = [&](int u) { return u >= 0 ? phi[(size_t)u * M + i] : -INFINITY; };
  const int e1 = coff[i + 1];
  int e = coff[i];
  // eight independent gathers in flight, then the options in candidate order
  for (; e + 8 <= e1; e += 8) {
    int sv[8];
    float fv[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) sv[j] = cand[e + j];
#pragma unroll
    for (int j = 0; j < 8; ++j) fv[j] = gather(row[sv[j]]);
#pragma unroll
    for (int j = 0; j < 8; ++j) take(sv[j], fv[j]);
  }
  for (; e < e1; ++e) {
    const int s = cand[e];
    take(s, gather(row[s]));
  }
  const float l = mx + __logf(sm);
  best16[cell] = (int16_t)(k1 + 1);
  dev1[cell] = b2 > -INFINITY ? b1 - b2 : INFINITY;
  (void)c;
  return CellOut{b1, l, opts};
}

// per-hypothesis results; the option count goes to hopts[h] (summed later in a fixed order:
// one global counter updated by every workgroup would serialise ten thousand atomics)
__device__ __forceinline__ void assoc_finish(int h, float bsum, float lsum, unsigned opts, const float* logw,
                                             const int32_t* ntrk, float gamma, float* bprime, float* lzprime,
                                             int32_t* hopts, float* red) {
  bsum = block_sum_f(bsum, red);
  lsum = block_sum_f(lsum, red + 8);
  const float o = block_sum_f((float)opts, red);  // exact: counts stay far below 2^24
  if (threadIdx.x == 0) {
    // the miss terms relative to hypothesis 0's track count keep the values small
    const float base = logw[h] - gamma * (float)(ntrk[h] - ntrk[0]);
    bprime[h] = base + bsum;
    lzprime[h] = base + lsum;
    hopts[h] = (int32_t)o;
  }
}

// Hypothesis 0, one wave per cell: the lanes take the detection's candidates 64 at a time,
// each keeping its first kTop options, log-sum-exp and option count, merged across the wave
// in a fixed butterfly.  Besides the cell's own results it stores the reference values the
// other hypotheses start from (b1 - c_i, the option count, the first kTop options and the mass
// of the options after them).
__device__ __forceinline__ bool top_before(float va, int sa, float vb, int sb) {
  return va > vb || (va == vb && sa < sb);
}
// Insert an option into a list ordered by top_before; it arrives after every listed option of
// equal value (larger slot), so a strict comparison keeps the order.  Static indices only.
__device__ __forceinline__ void top_insert(TopT& t, float f, int sl) {
#pragma unroll
  for (int j = kTop - 1; j > 0; --j) {
    const bool up = f > t.v[j - 1];
    const bool here = f > t.v[j];
    t.s[j] = up ? t.s[j - 1] : (here ? sl : t.s[j]);
    t.v[j] = up ? t.v[j - 1] : (here ? f : t.v[j]);
  }
  if (f > t.v[0]) {
    t.v[0] = f;
    t.s[0] = sl;
  }
}
// The first kTop of the union of two ordered lists: the better of a[j] and b[kTop-1-j] (a
// bitonic sequence holding exactly those entries), then a bitonic sort.  Both partners of a
// butterfly get the same list.
__device__ __forceinline__ TopT top_merge(const TopT& a, const TopT& b) {
  TopT r;
#pragma unroll
  for (int j = 0; j < kTop; ++j) {
    const bool ta = top_before(a.v[j], a.s[j], b.v[kTop - 1 - j], b.s[kTop - 1 - j]);
    r.v[j] = ta ? a.v[j] : b.v[kTop - 1 - j];
    r.s[j] = ta ? a.s[j] : b.s[kTop - 1 - j];
  }
#pragma unroll
  for (int d = kTop / 2; d > 0; d >>= 1) {
#pragma unroll
    for (int j = 0; j < kTop; ++j) {
      if (j & d) continue;
      const bool sw = top_before(r.v[j + d], r.s[j + d], r.v[j], r.s[j]);
      const float v0 = r.v[j], v1 = r.v[j + d];
      const int s0 = r.s[j], s1 = r.s[j + d];
      r.v[j] = sw ? v1 : v0;
      r.s[j] = sw ? s1 : s0;
      r.v[j + d] = sw ? v0 : v1;
      r.s[j + d] = sw ? s0 : s1;
    }
  }
  return r;
}
__device__ __forceinline__ bool top_has(const TopT& t, int sl) {
  bool in = false;
#pragma unroll
  for (int j = 0; j < kTop; ++j) in |= t.s[j] == sl;
  return in;
}
__global__ __launch_bounds__(256) void k_assoc_ref(int M, const int32_t* rows, float lgk, const int32_t* coff,
                                                   const int32_t* cand, const float* phi, const uint32_t* cmax,
                                                   int16_t* best16, float* dev1, float* lserel, float* ref_b1,
                                                   int32_t* ref_opts, TopE* ref_top, float* ref_rest) {
  const int i = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kWave);
  if (i >= M) return;
  const int lane = lane_id();
  TopT t;
#pragma unroll
  for (int j = 0; j < kTop; ++j) {
    t.v[j] = -INFINITY;
    t.s[j] = -2;
  }
  float mx = -INFINITY, sm = 0.0f;
  unsigned opts = 0;
  if (lane == 0) {  // clutter, ahead of every candidate
    t.v[0] = lgk;
    t.s[0] = -1;
    mx = lgk;
    sm = 1.0f;
  }
  for (int e = coff[i] + lane; e < coff[i + 1]; e += kWave) {
    const int sl = cand[e];
    const int u = rows[sl];
    if (u < 0) continue;
    const float f = phi[(size_t)u * M + i];
    if (!(f > -INFINITY)) continue;
    ++opts;
    top_insert(t, f, sl);
    if (f > mx) {
      sm = sm * __expf(mx - f) + 1.0f;
      mx = f;
    } else {
      sm += __expf(f - mx);
    }
  }
  // not unrolled: the merge network inlined six times takes the compiler minutes
#pragma unroll 1
  for (int d = kWave / 2; d > 0; d >>= 1) {
    TopT o;
#pragma unroll
    for (int j = 0; j < kTop; ++j) {
      o.v[j] = __shfl_xor(t.v[j], d, kWave);
      o.s[j] = __shfl_xor(t.s[j], d, kWave);
    }
    const float omx = __shfl_xor(mx, d, kWave), osm = __shfl_xor(sm, d, kWave);
    opts += __shfl_xor(opts, d, kWave);
    t = top_merge(t, o);
    const float m = fmaxf(mx, omx);
    sm = m > -INFINITY ? sm * __expf(mx - m) + osm * __expf(omx - m) : 0.0f;
    mx = m;
  }
  // the mass of the options after the listed ones (clutter among them when it is not listed)
  float rx = -INFINITY, rs = 0.0f;
  if (lane == 0 && !top_has(t, -1)) {
    rx = lgk;
    rs = 1.0f;
  }
  for (int e = coff[i] + lane; e < coff[i + 1]; e += kWave) {
    const int sl = cand[e];
    const int u = rows[sl];
    if (u < 0 || top_has(t, sl)) continue;
    const float f = phi[(size_t)u * M + i];
    if (!(f > -INFINITY)) continue;
    if (f > rx) {
      rs = rs * __expf(rx - f) + 1.0f;
      rx = f;
    } else {
      rs += __expf(f - rx);
    }
  }
  for (int d = kWave / 2; d > 0; d >>= 1) {
    const float ox = __shfl_xor(rx, d, kWave), os = __shfl_xor(rs, d, kWave);
    const float m = fmaxf(rx, ox);
    rs = m > -INFINITY ? rs * __expf(rx - m) + os * __expf(ox - m) : 0.0f;
    rx = m;
  }
  if (lane == 0) {
    const float c = o2f(cmax[i]);
    const float l = mx + __logf(sm);
    best16[i] = (int16_t)(t.s[0] + 1);
    dev1[i] = t.v[1] > -INFINITY ? t.v[0] - t.v[1] : INFINITY;
    lserel[i] = l - c;
    ref_b1[i] = t.v[0] - c;
    ref_opts[i] = (int32_t)opts;
    TopE te;
    te.t = t;
#pragma unroll
    for (int j = 0; j < kTop; ++j) te.e[j] = t.v[j] > -INFINITY ? __expf(t.v[j] - c) : 0.0f;
    ref_top[i] = te;
    ref_rest[i] = rx > -INFINITY ? rs * __expf(rx - c) : 0.0f;
  }
}

// hypothesis 0's sums over its cells, in a fixed order; the same sums in FP64 (rtot: b1, log
// mass, options), from which the other hypotheses take their untouched cells' share
__global__ __launch_bounds__(256) void k_assoc_ref_sum(int M, const float* ref_b1, const float* lserel,
                                                       const int32_t* ref_opts, const float* logw,
                                                       const int32_t* ntrk, float gamma, float* bprime,
                                                       float* lzprime, int32_t* hopts, double* rtot) {
  __shared__ float red[16];
  __shared__ double dred[3][4];
  float bsum = 0.0f, lsum = 0.0f;
  double db = 0.0, dl = 0.0, dn = 0.0;
  unsigned opts = 0;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    bsum += ref_b1[i];
    lsum += lserel[i];
    opts += (unsigned)ref_opts[i];
    db += (double)ref_b1[i];
    dl += (double)lserel[i];
    dn += (double)ref_opts[i];
  }
  for (int d = kWave / 2; d > 0; d >>= 1) {
    db += __shfl_xor(db, d, kWave);
    dl += __shfl_xor(dl, d, kWave);
    dn += __shfl_xor(dn, d, kWave);
  }
  if (lane_id() == 0) {
    dred[0][threadIdx.x / kWave] = db;
    dred[1][threadIdx.x / kWave] = dl;
    dred[2][threadIdx.x / kWave] = dn;
  }
  assoc_finish(0, bsum, lsum, opts, logw, ntrk, gamma, bprime, lzprime, hopts, red);  // synchronises
  if (threadIdx.x < 3) {
    double s = 0.0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) s += dred[threadIdx.x][w];
    rtot[threadIdx.x] = s;
  }
}

// Hypotheses 1..H-1, one wave each (no workgroup barrier: the waves of a workgroup take
// different hypotheses).  A cell's options depend only on the instances of the labels gated
// with its detection, so a cell whose labels hold the same instances as in hypothesis 0 equals
// hypothesis 0's cell and is not stored again (the cell layout of CellView).  A cell that differs ("touched": gated with a label whose
// instance changed) is derived from hypothesis 0's: it loses the changed labels' old options
// and gains their new ones.  Its best option and second value follow from hypothesis 0's
// first kTop options that remain and the added options; its option mass is the sum of three
// positive parts, the remaining listed options, the unlisted mass less the unlisted options
// removed, and the added options.  It is recomputed from all its options when fewer than two
// listed options remain (and hypothesis 0 had unlisted ones), or when the removed unlisted
// options carry more than half of an unlisted mass that exceeds 64 times the cell's other
// mass (the difference, exact to a few ulps of the unlisted mass, could then lose precision
// against the cell's total).
// The wave finds the changed labels with a ballot over the row, marks their gated detections
// in an LDS bit set (all lanes on the flattened (label, detection) pairs), compacts the
// touched cells into a list, derives them one per lane into the row's sparse entries, and adds
// hypothesis 0's values of the other cells to the row's sums.  More than kAssocNd changed
// labels: every cell recomputed and stored.
constexpr int kAssocNd = 64;
constexpr int kAssocRowChunks = 8;
// LDS words of one wave: changed labels (slot, old and new instance, list offset, length
// prefix), touched bits, touched list (16-bit), gate words of the first nq changed labels
__host__ __device__ inline int assoc_wave_words(int M, int nq) {
  const int W = (M + 31) / 32;
  return 5 * kAssocNd + 1 + W + (M + 1) / 2 + nq * W;
}
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}
__global__ __launch_bounds__(256) void k_assoc(int H, int M, int stride, int nq, const int32_t* rows,
                                               const float* logw, const int32_t* ntrk, float gamma, float lgk,
                                               const int32_t* coff, const int32_t* cand, const float* phi,
                                               const uint32_t* cmax, const int32_t* loff, const int32_t* llen,
                                               const int32_t* lmeas, const uint32_t* lbits, const float* ref_b1,
                                               const int32_t* ref_opts, const TopE* ref_top,
                                               const float* ref_rest, int16_t* best16, float* dev1, float* lserel,
                                               uint32_t* tbits, uint16_t* tpre, const double* rtot,
                                               float* bprime, float* lzprime, int32_t* hopts) {
  extern __shared__ int32_t lds[];
  const int wv = (int)threadIdx.x / kWave, lane = lane_id();
  const int h = 1 + (int)blockIdx.x * ((int)blockDim.x / kWave) + wv;
  if (h >= H) return;  // whole waves only
  const int W = (M + 31) / 32;
  int32_t* ds = lds + (size_t)wv * assoc_wave_words(M, nq);  // changed label slots, ascending
  int32_t* du0 = ds + kAssocNd;                               // their instances in hypothesis 0
  int32_t* duh = du0 + kAssocNd;                              // ... and in hypothesis h
  int32_t* dof = duh + kAssocNd;                              // offsets of their detection lists
  int32_t* dpf = dof + kAssocNd;                              // prefix of the list lengths
  uint32_t* touched = (uint32_t*)(dpf + kAssocNd + 1);
  uint16_t* tl = (uint16_t*)(touched + W);
  uint32_t* stage = touched + W + (M + 1) / 2;
  const int32_t* rowh = rows + (size_t)h * stride;
  int nd = 0;
  auto changed = [&](int s, int uh, int u0) {
    const bool f = uh != u0;
    const uint64_t bal = __ballot(f);
    const int pos = nd + __popcll(bal & lanemask_lt());
    if (f && pos < kAssocNd) {
      ds[pos] = s;
      du0[pos] = u0;
      duh[pos] = uh;
    }
    nd += __popcll(bal);
  };
  // the row in chunks of kAssocRowChunks x 64 slots, every load of a chunk issued before the
  // first comparison (the row comes from HBM: one latency per chunk, not per 64 slots)
  for (int s0 = 0; s0 < stride; s0 += kAssocRowChunks * kWave) {
    int uh[kAssocRowChunks], u0[kAssocRowChunks];
#pragma unroll
    for (int j = 0; j < kAssocRowChunks; ++j) {
      const int s = s0 + j * kWave + lane;
      uh[j] = s < stride ? rowh[s] : 0;
      u0[j] = s < stride ? rows[s] : 0;
    }
#pragma unroll
    for (int j = 0; j < kAssocRowChunks; ++j) changed(s0 + j * kWave + lane, uh[j], u0[j]);
  }
  float bsum = 0.0f, lsum = 0.0f;  // over the cells derived or recomputed here
  unsigned opts = 0;
  double xb = 0.0, xl = 0.0, xo = 0.0;  // hypothesis 0's values of those cells
  if (nd > kAssocNd) {
    // every cell stored (a dense row)
    for (int w = lane; w < W; w += kWave) {
      const int nb = min(32, M - 32 * w);
      tbits[(size_t)h * W + w] = nb == 32 ? ~0u : ((1u << nb) - 1u);
      tpre[(size_t)h * W + w] = (uint16_t)(32 * w);
    }
    for (int i = lane; i < M; i += kWave) {
      const size_t cell = (size_t)h * M + i;
      const float c = o2f(cmax[i]);
      const CellOut o = assoc_cell(i, M, rowh, lgk, coff, cand, phi, best16, dev1, cell, c);
      lserel[cell] = o.l - c;
      bsum += o.b1 - c;
      lsum += o.l - c;
      opts += o.opts;
      xb += (double)ref_b1[i];
      xl += (double)lserel[i];
      xo += (double)ref_opts[i];
    }
  } else {
    const int nst = nd < nq ? nd : nq;
    for (int e = lane; e < nst * W; e += kWave) {
      const int q = e / W;
      stage[e] = lbits[(size_t)ds[q] * W + (e - q * W)];
    }
    wave_lds_sync();
    // touched detections: the union of the changed labels' gate words (a label's detection
    // list holds exactly the bits of its gate words), lanes over the words
    for (int w = lane; w < W; w += kWave) {
      uint32_t acc = 0u;
      for (int q = 0; q < nd; ++q) acc |= q < nst ? stage[q * W + w] : lbits[(size_t)ds[q] * W + w];
      touched[w] = acc;
    }
    wave_lds_sync();
    // touched list, ascending
    int nt = 0;
    for (int w0 = 0; w0 < W; w0 += kWave) {
      const int w = w0 + lane;
      uint32_t word = w < W ? touched[w] : 0u;
      const int cnt = __popc(word);
      int y = cnt;
      for (int d = 1; d < kWave; d <<= 1) {
        const int z = __shfl_up(y, d, kWave);
        if (lane >= d) y += z;
      }
      int pos = nt + y - cnt;
      if (w < W) {
        tbits[(size_t)h * W + w] = word;
        tpre[(size_t)h * W + w] = (uint16_t)pos;
      }
      while (word) {
        const int b = __ffs(word) - 1;
        word &= word - 1u;
        tl[pos++] = (uint16_t)(w * 32 + b);
      }
      nt += __shfl(y, kWave - 1, kWave);
    }
    wave_lds_sync();
    // touched cells, one per lane
    for (int t = lane; t < nt; t += kWave) {
      const int i = tl[t];
      const size_t cell = (size_t)h * M + t;  // the t-th touched cell of the row
      const float c = o2f(cmax[i]);
      const TopE TE = ref_top[i];
      const TopT& T = TE.t;
      const float restT = ref_rest[i];
      xb += (double)ref_b1[i];
      xl += (double)lserel[i];
      xo += (double)ref_opts[i];
      const uint32_t bit = 1u << (i & 31);
      float rem = 0.0f, add = 0.0f;          // removed unlisted mass, added mass
      float a1 = -INFINITY, a2 = -INFINITY;  // best two added options (best: smallest slot among equals)
      int a1s = INT_MAX, dopt = 0;
      unsigned gone = 0;  // listed entries whose option is removed
      for (int q = 0; q < nd; ++q) {
        const uint32_t g = q < nst ? stage[q * W + (i >> 5)] : lbits[(size_t)ds[q] * W + (i >> 5)];
        if (!(g & bit)) continue;
        const int s = ds[q], u0 = du0[q], uh = duh[q];
        if (u0 >= 0) {
          const float f0 = phi[(size_t)u0 * M + i];
          if (f0 > -INFINITY) {
            bool listed = false;
#pragma unroll
            for (int j = 0; j < kTop; ++j)
              if (T.s[j] == s) {
                gone |= 1u << j;
                listed = true;
              }
            if (!listed) rem += __expf(f0 - c);
            --dopt;
          }
        }
        if (uh >= 0) {
          const float fh = phi[(size_t)uh * M + i];
          if (fh > -INFINITY) {
            add += __expf(fh - c);
            ++dopt;
            if (fh > a1 || (fh == a1 && s < a1s)) {
              a2 = a1;
              a1 = fh;
              a1s = s;
            } else if (fh > a2) {
              a2 = fh;
            }
          }
        }
      }
      // hypothesis 0's listed options that remain, in order, and their mass
      float r1 = -INFINITY, r2 = -INFINITY, top = 0.0f;
      int r1s = -2, nrem = 0;
#pragma unroll
      for (int j = 0; j < kTop; ++j)
        if (T.s[j] != -2 && !((gone >> j) & 1u)) {
          if (nrem == 0) {
            r1 = T.v[j];
            r1s = T.s[j];
          } else if (nrem == 1) {
            r2 = T.v[j];
          }
          ++nrem;
          top += TE.e[j];
        }
      const bool known = ref_opts[i] + 1 <= kTop || nrem >= 2;
      // restT - rem loses at most a few ulps of restT: recomputed only when that could matter
      // against the cell's mass (rem a large part of a restT that dwarfs the rest)
      if (!known || (rem > 0.5f * restT && restT > 64.0f * (top + add))) {
        const CellOut o = assoc_cell(i, M, rowh, lgk, coff, cand, phi, best16, dev1, cell, c);
        lserel[cell] = o.l - c;
        bsum += o.b1 - c;
        lsum += o.l - c;
        opts += o.opts;
      } else {
        float nb1, nb2;
        int nk1;
        if (a1 > r1 || (a1 == r1 && a1s < r1s)) {
          nb1 = a1;
          nk1 = a1s;
          nb2 = fmaxf(r1, a2);
        } else {
          nb1 = r1;
          nk1 = r1s;
          nb2 = fmaxf(r2, a1);
        }
        const float lc = __logf(top + fmaxf(restT - rem, 0.0f) + add);
        best16[cell] = (int16_t)(nk1 + 1);
        dev1[cell] = nb2 > -INFINITY ? nb1 - nb2 : INFINITY;
        lserel[cell] = lc;
        bsum += nb1 - c;
        lsum += lc;
        opts += (unsigned)(ref_opts[i] + dopt);
      }
    }
  }
  // per-hypothesis sums, fixed butterfly; the other cells are hypothesis 0's (not stored
  // again): their share is hypothesis 0's total less its values of the cells above, in FP64
  for (int d = kWave / 2; d > 0; d >>= 1) {
    bsum += __shfl_xor(bsum, d, kWave);
    lsum += __shfl_xor(lsum, d, kWave);
    opts += __shfl_xor(opts, d, kWave);
    xb += __shfl_xor(xb, d, kWave);
    xl += __shfl_xor(xl, d, kWave);
    xo += __shfl_xor(xo, d, kWave);
  }
  if (lane == 0) {
    // the miss terms relative to hypothesis 0's track count keep the values small
    const float base = logw[h] - gamma * (float)(ntrk[h] - ntrk[0]);
    bprime[h] = base + (float)((double)bsum + (rtot[0] - xb));
    lzprime[h] = base + (float)((double)lsum + (rtot[1] - xl));
    hopts[h] = (int32_t)((double)opts + (rtot[2] - xo));
  }
}

// ------------------------------------------------------------------ U3
// one block: log of the total mass, per-parent diagnostics
__global__ __launch_bounds__(1024) void k_norm(int H, int M, const float* bprime, const float* lzprime,
                                               const int32_t* hopts, const int32_t* ntrk, float* lz,
                                               float* diag_best, float* diag_logpi, unsigned long long* nopts,
                                               unsigned long long* ndense) {
  __shared__ float red[32];
  __shared__ unsigned long long ired[32];
  {
    // statistics: options of every cell, and sum_h |J_h| * M
    unsigned long long o = 0, d = 0;
    for (int h = threadIdx.x; h < H; h += blockDim.x) {
      o += (unsigned long long)hopts[h];
      d += (unsigned long long)ntrk[h] * (unsigned long long)M;
    }
    for (int k = kWave / 2; k > 0; k >>= 1) {
      o += __shfl_xor(o, k, kWave);
      d += __shfl_xor(d, k, kWave);
    }
    if (lane_id() == 0) {
      ired[threadIdx.x / kWave] = o;
      ired[16 + threadIdx.x / kWave] = d;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      unsigned long long so = 0, sd = 0;
      for (int j = 0; j < (int)(blockDim.x / kWave); ++j) {
        so += ired[j];
        sd += ired[16 + j];
      }
      *nopts = so;
      *ndense = sd;
    }
  }
  float mx = -INFINITY;
  for (int h = threadIdx.x; h < H; h += blockDim.x) mx = fmaxf(mx, lzprime[h]);
  mx = block_max_f(mx, red);
  float sm = 0.0f;
  for (int h = threadIdx.x; h < H; h += blockDim.x) sm += __expf(lzprime[h] - mx);
  sm = block_sum_f(sm, red + 16);
  const float L = mx + __logf(sm);
  for (int h = threadIdx.x; h < H; h += blockDim.x) {
    diag_best[h] = bprime[h] - L;
    diag_logpi[h] = lzprime[h] - L;
  }
  if (threadIdx.x == 0) *lz = L;
}

// One wave per parent: its cells (h, i) with B'_h - dev1 >= t0, in ascending i.  dev1 >= 0, so
// a parent below the bound has none and its row is not read.  Counting pass (roff null):
// rcount[h]; writing pass: cell indices h * M + i at roff[h].
__global__ __launch_bounds__(256) void k_row_cells(int H, int M, const float* bprime, CellView cv,
                                                   const float* t0, const int32_t* roff, int32_t* rcount,
                                                   int32_t* cells) {
  const int h = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kWave);
  if (h >= H) return;
  const int lane = lane_id();
  const float B = bprime[h], t = *t0;
  int cnt = 0;
  if (B >= t) {
    const int q0 = roff ? roff[h] : 0;
    for (int i0 = 0; i0 < M; i0 += kWave) {
      const int i = i0 + lane;
      const bool f = i < M && B - cv.dev1[cv.at(h, i)] >= t;
      const uint64_t bal = __ballot(f);
      if (roff && f) cells[q0 + cnt + __popcll(bal & lanemask_lt())] = h * M + i;
      cnt += __popcll(bal);
    }
  }
  if (!roff && lane == 0) rcount[h] = cnt;
}

// Deviation items of cell (h, i): every option other than the cell's best whose deviation
// d = phi_best - phi keeps B'_h - d above the cut bound.  One wave per cell: the lanes take
// detection i's gated candidates 64 at a time.  The best option is the first candidate (in
// list order, i.e. ascending key) of the largest score if that beats the clutter score, else
// clutter (key -1); the items come in the order clutter first, then the candidates in list
// order, and the sort by (h, d) that follows keeps that order among equal deviations.
// Counting pass (ioff null): icount[c] = number of items; writing pass: items at ioff[c].
__global__ __launch_bounds__(256) void k_items(int ncell, const int32_t* cells, int M, int stride,
                                               const int32_t* rows, const int32_t* coff, const int32_t* cand,
                                               const float* phi, float lgk, const float* bprime, const float* t0,
                                               const int32_t* ioff, int32_t* icount, float* it_delta,
                                               int32_t* it_group, int32_t* it_opt, uint64_t* keys, uint32_t* vals) {
  const int c = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kWave);
  if (c >= ncell) return;
  const int lane = lane_id();
  const int cell = cells[c];
  const int h = cell / M, i = cell % M;
  const int32_t* row = rows + (size_t)h * stride;
  const int e0 = coff[i], e1 = coff[i + 1];
  float lv = -INFINITY;
  int le = INT_MAX;
  for (int e = e0 + lane; e < e1; e += kWave) {
    const int u = row[cand[e]];
    if (u < 0) continue;
    const float v = phi[(size_t)u * M + i];
    if (v > lv) {
      lv = v;
      le = e;
    }
  }
  for (int d = kWave / 2; d > 0; d >>= 1) {
    const float ov = __shfl_xor(lv, d, kWave);
    const int oe = __shfl_xor(le, d, kWave);
    if (ov > lv || (ov == lv && oe < le)) {
      lv = ov;
      le = oe;
    }
  }
  const bool cand_best = lv > lgk;
  const float best = cand_best ? lv : lgk;
  const int bkey = cand_best ? cand[le] : -1;
  const float B = bprime[h], t = *t0;
  int cnt = 0;
  const int q0 = ioff ? ioff[c] : 0;
  auto put = [&](int q, float d, int key) {
    it_delta[q] = d;
    it_group[q] = i;
    it_opt[q] = key;
    if (keys) {
      keys[q] = ((uint64_t)(uint32_t)h << 32) | f2o(d);
      vals[q] = (uint32_t)q;
    }
  };
  if (bkey >= 0) {
    const float d = best - lgk;
    if (B - d >= t) {
      if (ioff && lane == 0) put(q0, d, -1);
      cnt = 1;
    }
  }
  for (int eb = e0; eb < e1; eb += kWave) {
    const int e = eb + lane;
    bool emit = false;
    float d = 0.f;
    int sk = -1;
    if (e < e1) {
      sk = cand[e];
      const int u = row[sk];
      if (sk != bkey && u >= 0) {
        const float v = phi[(size_t)u * M + i];
        d = best - v;
        emit = v > -INFINITY && B - d >= t;
      }
    }
    const uint64_t bal = __ballot(emit);
    if (ioff && emit) put(q0 + cnt + __popcll(bal & lanemask_lt()), d, sk);
    cnt += __popcll(bal);
  }
  if (!ioff && lane == 0) icount[c] = cnt;
}

// first item of every parent (items are generated in cell order, so each parent's items are
// contiguous), the largest per-parent count, and the list of parents with items (any order)
__global__ void k_item_ranges(int H, int ncell, int M, const int32_t* cells, const int32_t* ioff, int32_t* itoff,
                              int32_t* maxlen, int32_t* nlist, int32_t* list) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h > H) return;
  auto first_cell = [&](int64_t key) {
    int a = 0, b = ncell;
    while (a < b) {
      const int m = (a + b) >> 1;
      if ((int64_t)cells[m] < key) a = m + 1;
      else b = m;
    }
    return a;
  };
  const int c0 = first_cell((int64_t)h * M);
  itoff[h] = ioff[c0];
  if (h < H) {
    const int len = ioff[first_cell((int64_t)(h + 1) * M)] - ioff[c0];
    if (len > 0) list[atomicAdd(nlist, 1)] = h;
    if (len > 1) atomicMax(maxlen, len);
  }
}

// Every workgroup takes listed parents in turn and sorts the parent's items by delta in LDS
// (at most kSegSort items).  Ties keep the generation order (detection, then option), as the
// stable radix sort of the general path does, through the item's position in the low bits of
// the key.
constexpr int kSegSort = 4096;
#ifndef GLMB_SEGSORT_MAX
#define GLMB_SEGSORT_MAX kSegSort  // largest per-parent item count sorted in LDS (a build may lower it)
#endif
static_assert(GLMB_SEGSORT_MAX <= kSegSort, "per-parent LDS sort holds at most kSegSort items");
template <int NT>
__global__ __launch_bounds__(NT) void k_item_segsort(const int32_t* nlist, const int32_t* list, const int32_t* itoff,
                                                     const float* d0, const int32_t* g0, const int32_t* o0,
                                                     float* d1, int32_t* g1, int32_t* o1) {
  __shared__ uint64_t key[kSegSort];
  const int nl = *nlist;
  for (int k = blockIdx.x; k < nl; k += gridDim.x) {
    const int h = list[k];
    const int b = itoff[h], n = itoff[h + 1] - b;
    int P = 1;
    while (P < n) P <<= 1;
    __syncthreads();  // the previous parent's keys are read
    for (int q = threadIdx.x; q < P; q += NT)
      key[q] = q < n ? ((uint64_t)f2o(d0[b + q]) << 32) | (uint32_t)q : ~0ull;
    __syncthreads();
    for (int kk = 2; kk <= P; kk <<= 1)
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int q = threadIdx.x; q < P; q += NT) {
          const int r = q ^ j;
          if (r > q) {
            const uint64_t x = key[q], y = key[r];
            if ((x > y) == ((q & kk) == 0)) {
              key[q] = y;
              key[r] = x;
            }
          }
        }
        __syncthreads();
      }
    for (int q = threadIdx.x; q < n; q += NT) {
      const int src = b + (int)(uint32_t)key[q];
      d1[b + q] = d0[src];
      g1[b + q] = g0[src];
      o1[b + q] = o0[src];
    }
  }
}

__global__ void k_item_perm(int n, const uint32_t* vals, const float* d0, const int32_t* g0, const int32_t* o0,
                            float* d1, int32_t* g1, int32_t* o1) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const uint32_t q = vals[p];
  d1[p] = d0[q];
  g1[p] = g0[q];
  o1[p] = o0[q];
}

// one block: normalise over the selected children, tau pruning (the first is always kept)
__global__ __launch_bounds__(1024) void k_prune(int n, const float* v, float tau, const float* lz, float* logw_out,
                                                int32_t* nkeep, float* retained) {
  __shared__ float red[32];
  __shared__ int32_t cnt;
  float mx = v[0];
  float sm = 0.0f;
  for (int j = threadIdx.x; j < n; j += blockDim.x) sm += __expf(v[j] - mx);
  sm = block_sum_f(sm, red);
  const float L = mx + __logf(sm);
  if (threadIdx.x == 0) cnt = 1;
  __syncthreads();
  int mine = 0;
  if (tau > 0.0f) {
    for (int j = 1 + threadIdx.x; j < n; j += blockDim.x)
      if (__expf(v[j] - L) >= tau) ++mine;
  } else {
    for (int j = 1 + threadIdx.x; j < n; j += blockDim.x) ++mine;
  }
  if (mine) atomicAdd(&cnt, mine);
  __syncthreads();
  const int keep = cnt;
  float s2 = 0.0f;
  for (int j = threadIdx.x; j < keep; j += blockDim.x) s2 += __expf(v[j] - mx);
  s2 = block_sum_f(s2, red + 16);
  const float L2 = mx + __logf(s2);
  for (int j = threadIdx.x; j < keep; j += blockDim.x) logw_out[j] = v[j] - L2;
  if (threadIdx.x == 0) {
    *nkeep = keep;
    *retained = L2 - *lz;  // log of the retained posterior mass
  }
}

// ------------------------------------------------------------------ U4 materialise
__global__ void k_child_depth(int n, const int32_t* sel_node, const int32_t* nd_parent, const int32_t* nd_item,
                              const int32_t* nd_h, int32_t* depth, int32_t* ch_h, uint32_t* errf) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int d = 0;
  int x = sel_node[c];
  ch_h[c] = nd_h[x];
  for (; nd_item[x] >= 0; x = nd_parent[x]) ++d;
  if (d > kMaxDepth) atomicOr(errf, ERR_DEPTH);
  depth[c] = d;
}

__global__ void k_child_devs(int n, int M, const int32_t* sel_node, const int32_t* nd_parent, const int32_t* nd_item,
                             const int32_t* ch_h, const int32_t* doff, const int32_t* it_group, const int32_t* it_opt,
                             CellView cv, int32_t* dev_i, int32_t* dev_new, int32_t* dev_old) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  int q = doff[c];
  const int h = ch_h[c];
  for (int x = sel_node[c]; nd_item[x] >= 0; x = nd_parent[x], ++q) {
    const int it = nd_item[x];
    const int i = it_group[it];
    dev_i[q] = i;
    dev_new[q] = it_opt[it];
    dev_old[q] = (int)cv.best16[cv.at(h, i)] - 1;
  }
}

__global__ void k_mark(int n, const int32_t* ch_h, int32_t* mark) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c < n) mark[ch_h[c]] = 1;
}
__global__ void k_plist(int H, const int32_t* mark, const int32_t* pre, int32_t* plist, int32_t* hp_map) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h >= H) return;
  hp_map[h] = mark[h] ? pre[h] : -1;
  if (mark[h]) plist[pre[h]] = h;
}

__global__ void k_first(int np, const int32_t* plist, int stride, const int32_t* rows, int32_t* first) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)np * stride) return;
  const int h = plist[t / stride];
  const int u = rows[(size_t)h * stride + (t % stride)];
  if (u >= 0) atomicMin(&first[u], h);
}

__device__ __forceinline__ int lpos(const int32_t* lmeas, int off, int len, int i) {
  int a = 0, b = len;
  while (a < b) {
    const int m = (a + b) >> 1;
    if (lmeas[off + m] < i) a = m + 1;
    else b = m;
  }
  return a;
}

// Detection-set masks of every slot of hypothesis h under its best association map.  A mask
// has LW 32-bit words; bit j stands for the j-th detection gated with the slot's label.
__device__ void build_masks(int h, int M, int nslot, int LW, const CellView& cv, const int32_t* loff,
                            const int32_t* llen, const int32_t* lmeas, uint32_t* mask) {
  for (int k = threadIdx.x; k < nslot * LW; k += blockDim.x) mask[k] = 0u;
  __syncthreads();
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    const int s = (int)cv.best16[cv.at(h, i)] - 1;
    if (s < 0) continue;
    const int j = lpos(lmeas, loff[s], llen[s], i);
    if (j < llen[s]) atomicOr(&mask[s * LW + (j >> 5)], 1u << (j & 31));
  }
  __syncthreads();
}

__global__ __launch_bounds__(256) void k_default_masks(const int32_t* plist, int M, int nslot, int LW, int stride,
                                                       const int32_t* rows, CellView cv,
                                                       const int32_t* loff, const int32_t* llen,
                                                       const int32_t* lmeas, const int32_t* first, uint32_t* dmask) {
  extern __shared__ uint32_t mask[];
  const int h = plist[blockIdx.x];
  build_masks(h, M, nslot, LW, cv, loff, llen, lmeas, mask);
  for (int s = threadIdx.x; s < nslot; s += blockDim.x) {
    const int u = rows[(size_t)h * stride + s];
    if (u >= 0 && first[u] == h)
      for (int w = 0; w < LW; ++w) dmask[(size_t)u * LW + w] = mask[s * LW + w];
  }
}

// (instance, slot) pairs of retained parents whose detection set differs from the default
__global__ __launch_bounds__(256) void k_exceptions(const int32_t* plist, int M, int nslot, int LW, int stride,
                                                    const int32_t* rows, CellView cv, const int32_t* loff,
                                                    const int32_t* llen, const int32_t* lmeas, const uint32_t* dmask,
                                                    int32_t* nexc, int32_t* eu, int32_t* ea, int32_t* eb,
                                                    uint32_t* em, int cap) {
  extern __shared__ uint32_t mask[];
  const int hp = blockIdx.x;
  const int h = plist[hp];
  build_masks(h, M, nslot, LW, cv, loff, llen, lmeas, mask);
  for (int s = threadIdx.x; s < nslot; s += blockDim.x) {
    const int u = rows[(size_t)h * stride + s];
    if (u < 0) continue;
    bool diff = false;
    for (int w = 0; w < LW && !diff; ++w) diff = dmask[(size_t)u * LW + w] != mask[s * LW + w];
    if (!diff) continue;
    const int k = atomicAdd(nexc, 1);
    if (k >= cap) continue;
    eu[k] = u;
    ea[k] = hp;
    eb[k] = s;
    for (int w = 0; w < LW; ++w) em[(size_t)k * LW + w] = mask[s * LW + w];
  }
}

__global__ void k_exc_keys(int n, const int32_t* ea, const int32_t* eb, uint64_t* keys, uint32_t* vals) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  keys[k] = ((uint64_t)(uint32_t)ea[k] << 32) | (uint32_t)eb[k];
  vals[k] = (uint32_t)k;
}
__global__ void k_exc_perm(int n, int LW, const uint32_t* vals, const int32_t* u0, const int32_t* a0,
                           const int32_t* b0, const uint32_t* m0, int32_t* u1, int32_t* a1, int32_t* b1,
                           uint32_t* m1) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t q = vals[k];
  u1[k] = u0[q];
  a1[k] = a0[q];
  b1[k] = b0[q];
  for (int w = 0; w < LW; ++w) m1[(size_t)k * LW + w] = m0[(size_t)q * LW + w];
}
__global__ void k_exc_off(int np, int n, const int32_t* ea, int32_t* eoff) {
  const int hp = blockIdx.x * blockDim.x + threadIdx.x;
  if (hp > np) return;
  int a = 0, b = n;
  while (a < b) {
    const int m = (a + b) >> 1;
    if (ea[m] < hp) a = m + 1;
    else b = m;
  }
  eoff[hp] = a;
}

__device__ __forceinline__ int find_exc(const int32_t* eb, const int32_t* eoff, int hp, int s) {
  int a = eoff[hp], b = eoff[hp + 1];
  const int e1 = b;
  while (a < b) {
    const int m = (a + b) >> 1;
    if (eb[m] < s) a = m + 1;
    else b = m;
  }
  return (a < e1 && eb[a] == s) ? a : -1;
}

// per child: the slots its deviations touch, each once (count pass: ma == null; writing pass:
// child and slot of every touched slot at moff[c])
__global__ void k_child_mods(int n, const int32_t* doff, const int32_t* dev_new, const int32_t* dev_old,
                             const int32_t* moff, int32_t* mcount, int32_t* ma, int32_t* mb) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  if (c >= n) return;
  const int d0 = doff[c], d1 = doff[c + 1];
  int cnt = 0;
  for (int q = d0; q < d1; ++q) {
    for (int side = 0; side < 2; ++side) {
      const int s = side ? dev_new[q] : dev_old[q];
      if (s < 0) continue;
      bool seen = side == 1 && dev_old[q] == s;
      for (int r = d0; r < q && !seen; ++r) seen = dev_old[r] == s || dev_new[r] == s;
      if (seen) continue;
      if (ma) {
        const int o = moff[c] + cnt;
        ma[o] = c;
        mb[o] = s;
      }
      ++cnt;
    }
  }
  if (!ma) mcount[c] = cnt;
}

// one thread per touched (child, slot): the slot's detection-set mask in the child, i.e. the
// parent's mask (its exception, else the instance's default) with the child's deviations on
// that slot applied
__global__ void k_mod_masks(int nm, int LW, const int32_t* ch_h, const int32_t* hp_map, const int32_t* doff,
                            const int32_t* dev_i, const int32_t* dev_new, const int32_t* dev_old, int stride,
                            const int32_t* rows, const int32_t* loff, const int32_t* llen, const int32_t* lmeas,
                            const uint32_t* dmask, const int32_t* eb, const uint32_t* em, const int32_t* eoff,
                            const int32_t* ma, const int32_t* mb, int32_t* mu, uint32_t* mm) {
  const int o = blockIdx.x * blockDim.x + threadIdx.x;
  if (o >= nm) return;
  const int c = ma[o], s = mb[o];
  const int h = ch_h[c], hp = hp_map[h];
  const int d0 = doff[c], d1 = doff[c + 1];
  const int u = rows[(size_t)h * stride + s];
  const int e = find_exc(eb, eoff, hp, s);
  const uint32_t* base = e >= 0 ? em + (size_t)e * LW : dmask + (size_t)u * LW;
  uint32_t* out = mm + (size_t)o * LW;
  for (int w = 0; w < LW; ++w) out[w] = base[w];
  for (int t = d0; t < d1; ++t) {
    if (dev_old[t] != s && dev_new[t] != s) continue;
    const int j = lpos(lmeas, loff[s], llen[s], dev_i[t]);
    if (j >= llen[s]) continue;
    if (dev_old[t] == s) out[j >> 5] &= ~(1u << (j & 31));
    if (dev_new[t] == s) out[j >> 5] |= 1u << (j & 31);
  }
  mu[o] = u;
}

__device__ __forceinline__ uint32_t mask_hash(const uint32_t* m, int LW) {
  uint64_t x = 0x51ed270b27ull;
  for (int w = 0; w < LW; ++w) x = mix64(x ^ ((uint64_t)m[w] << 17) ^ (uint64_t)w);
  return (uint32_t)(x >> 32);
}

// records (instance, mask): defaults (one per referenced instance), exceptions, child masks
__global__ void k_rec_defaults(int U, int LW, const int32_t* first, const uint32_t* dmask, const int32_t* dpre,
                               int32_t* ru, uint32_t* rm) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u >= U || first[u] == INT32_MAX) return;
  const int o = dpre[u];
  ru[o] = u;
  for (int w = 0; w < LW; ++w) rm[(size_t)o * LW + w] = dmask[(size_t)u * LW + w];
}
__global__ void k_rec_copy(int n, int LW, const int32_t* u0, const uint32_t* m0, int32_t* u1, uint32_t* m1) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  u1[k] = u0[k];
  for (int w = 0; w < LW; ++w) m1[(size_t)k * LW + w] = m0[(size_t)k * LW + w];
}
__global__ void k_rec_keys(int n, int LW, uint32_t hmask, const int32_t* ru, const uint32_t* rm, uint64_t* keys,
                           uint32_t* vals) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= n) return;
  const uint32_t hh = mask_hash(rm + (size_t)k * LW, LW);
  keys[k] = ((uint64_t)(uint32_t)ru[k] << 16) | ((hh ^ (hh >> 16)) & hmask & 0xFFFFu);
  vals[k] = (uint32_t)k;
}
__device__ __forceinline__ bool rec_equal(int LW, const int32_t* ru, const uint32_t* rm, uint32_t a, uint32_t b) {
  bool eq = ru[a] == ru[b];
  for (int w = 0; w < LW && eq; ++w) eq = rm[(size_t)a * LW + w] == rm[(size_t)b * LW + w];
  return eq;
}
// distinct records in (instance, fingerprint) order: a record starts a new id unless it equals
// its predecessor.  Two different detection sets of one instance with equal fingerprints make
// a run in which equal records need not be adjacent; such a run is flagged (*ncoll) and
// k_rec_resolve then assigns the ids by full comparison.
__global__ void k_rec_unique(int n, int LW, const uint64_t* keys, const uint32_t* vals, const int32_t* ru,
                             const uint32_t* rm, int32_t* flag, int32_t* ncoll) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  bool nw = p == 0 || keys[p] != keys[p - 1];
  if (!nw && !rec_equal(LW, ru, rm, vals[p], vals[p - 1])) {
    nw = true;
    atomicAdd(ncoll, 1);
  }
  flag[p] = nw ? 1 : 0;
}
// collision path: the leader of a record is the first record of its fingerprint run that
// equals it (full comparison); only leaders start an id
__global__ void k_rec_resolve(int n, int LW, const uint64_t* keys, const uint32_t* vals, const int32_t* ru,
                              const uint32_t* rm, int32_t* flag, int32_t* lead) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  int r0 = p;
  while (r0 > 0 && keys[r0 - 1] == keys[p]) --r0;
  int q = r0;
  while (q < p && !rec_equal(LW, ru, rm, vals[q], vals[p])) ++q;
  lead[p] = q;
  flag[p] = q == p ? 1 : 0;
}
// id of every record (pre: exclusive scan of the leader flags); lead == null: equal records
// are adjacent, so a record's leader is the last flagged one at or before it
__global__ void k_rec_ids(int n, const uint32_t* vals, const int32_t* flag, const int32_t* pre, const int32_t* lead,
                          int32_t* rec_id, int32_t* rep) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int id = lead ? pre[lead[p]] : pre[p] + flag[p] - 1;
  rec_id[vals[p]] = id;
  if (flag[p]) rep[id] = (int32_t)vals[p];
}

// Kalman update of every distinct (instance, detection set): the detections of one object are
// equivalent to their mean observed with noise R / n
// With jc non-null, also the exact-joint correction of every new instance with n >= 2
// detections: log J(S) - sum_{i in S} log l_i, where the joint likelihood of the detection set
// is J(S) = C_S N(zbar; H m, H P H^T + R/n) with
// C_S = (2 pi sigma^2)^-(n-1) n^-1 exp(-sum_i |z_i - zbar|^2 / (2 sigma^2)) (the product of the
// detections' densities around their mean, R = sigma^2 I), and log l_i = phi_i - log gamma.
__global__ void k_kalman(int nnew, int LW, const int32_t* rep, const int32_t* ru, const uint32_t* rm,
                         const DInst* pin, const int32_t* loff, const int32_t* lmeas, const float2* z, float sig2,
                         DInst* out, int32_t* onz, int32_t* oz, const float* phi, int M, float lgg, float* jc) {
  const int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id >= nnew) return;
  const int r = rep[id];
  const DInst x = pin[ru[r]];
  DInst y = x;
  int nz = 0;
  float sx = 0.0f, sy = 0.0f;
  const int off = loff[x.slot];
  const uint32_t* m = rm + (size_t)r * LW;
  for (int w = 0; w < LW; ++w) {
    uint32_t b = m[w];
    while (b) {
      const int j = w * 32 + __ffs(b) - 1;
      b &= b - 1;
      const int i = lmeas[off + j];
      const float2 zi = z[i];
      sx += zi.x;
      sy += zi.y;
      if (nz < 8) oz[(size_t)id * 8 + nz] = i;
      ++nz;
    }
  }
  onz[id] = nz;
  if (nz > 0) {
    const float inv = 1.0f / (float)nz;
    const float zb0 = sx * inv, zb1 = sy * inv;
    const float* P = x.P;
    const float rr = sig2 * inv;
    const float s00 = P[0] + rr, s01 = P[1], s11 = P[4] + rr;
    const float det = s00 * s11 - s01 * s01;
    const float i00 = s11 / det, i01 = -s01 / det, i11 = s00 / det;
    // columns of P H^T: a_k = P[k][0], b_k = P[k][1]
    const float a[4] = {P[0], P[1], P[2], P[3]};
    const float bq[4] = {P[1], P[4], P[5], P[6]};
    float K0[4], K1[4];
    for (int k = 0; k < 4; ++k) {
      K0[k] = a[k] * i00 + bq[k] * i01;
      K1[k] = a[k] * i01 + bq[k] * i11;
    }
    const float n0 = zb0 - x.m[0], n1 = zb1 - x.m[1];
    for (int k = 0; k < 4; ++k) y.m[k] = x.m[k] + K0[k] * n0 + K1[k] * n1;
    // P' = P - [a b] S^-1 [a b]^T
    int t = 0;
    for (int r0 = 0; r0 < 4; ++r0)
      for (int c0 = r0; c0 < 4; ++c0, ++t) y.P[t] = P[t] - (K0[r0] * a[c0] + K1[r0] * bq[c0]);
    if (jc && nz >= 2) {
      // second pass: the spread around the mean and the per-detection log likelihoods
      float ss = 0.0f, sl = 0.0f;
      const int u = ru[r];
      for (int w = 0; w < LW; ++w) {
        uint32_t b = m[w];
        while (b) {
          const int j = w * 32 + __ffs(b) - 1;
          b &= b - 1;
          const int i = lmeas[off + j];
          const float dx = z[i].x - zb0, dy = z[i].y - zb1;
          ss += dx * dx + dy * dy;
          sl += phi[(size_t)u * M + i] - lgg;
        }
      }
      const float l2pi = 1.8378770664093453f;  // log(2 pi)
      const float lcs = -(float)(nz - 1) * (l2pi + logf(sig2)) - logf((float)nz) - 0.5f * ss / sig2;
      const float quad = n0 * n0 * i00 + 2.0f * n0 * n1 * i01 + n1 * n1 * i11;
      const float lzb = -l2pi - 0.5f * logf(det) - 0.5f * quad;
      jc[id] = lcs + lzb - sl;
    }
  }
  if (jc && nz < 2) jc[id] = 0.0f;
  out[id] = y;
}

// exact-joint reweighting: one wave per kept child, its weight plus the corrections of the new
// instances in its row (fixed order), keyed for the rank order (weight descending, then the
// child's rank under the factorised weights)
__global__ __launch_bounds__(256) void k_joint_child(int n, int stride, const int32_t* rows, const float* jc,
                                                     const float* logw, float* val, uint64_t* keys, uint32_t* perm) {
  const int c = (int)(((size_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave);
  if (c >= n) return;
  float a = 0.0f;
  for (int s = lane_id(); s < stride; s += kWave) {
    const int id = rows[(size_t)c * stride + s];
    if (id >= 0) a += jc[id];
  }
  for (int d = kWave / 2; d > 0; d >>= 1) a += __shfl_xor(a, d, kWave);
  if (lane_id() == 0) {
    const float v = logw[c] + a;
    val[c] = v;
    keys[c] = ((uint64_t)(~f2o(v)) << 32) | (uint32_t)c;
    perm[c] = (uint32_t)c;
  }
}

// one workgroup: tau prefix of the re-ranked weights (the best is kept) and renormalisation
__global__ __launch_bounds__(1024) void k_joint_tau(int n, const uint32_t* perm, const float* val, float tau,
                                                    float* logw_out, int32_t* nkeep) {
  __shared__ float red[32];
  __shared__ int ired[32];
  float mx = -INFINITY;
  for (int j = threadIdx.x; j < n; j += blockDim.x) mx = fmaxf(mx, val[perm[j]]);
  mx = block_max_f(mx, red);
  float sm = 0.0f;
  for (int j = threadIdx.x; j < n; j += blockDim.x) sm += __expf(val[perm[j]] - mx);
  sm = block_sum_f(sm, red + 16);
  const float L = mx + __logf(sm);
  int keep = n;
  if (tau > 0.0f) {
    const float lt = __logf(tau);
    int cnt = 0;  // sorted descending: the kept ones are a prefix
    for (int j = threadIdx.x; j < n; j += blockDim.x) cnt += (val[perm[j]] - L >= lt) ? 1 : 0;
    for (int d = kWave / 2; d > 0; d >>= 1) cnt += __shfl_xor(cnt, d, kWave);
    __syncthreads();
    if (lane_id() == 0) ired[threadIdx.x / kWave] = cnt;
    __syncthreads();
    keep = 0;
    for (int w = 0; w < (int)(blockDim.x / kWave); ++w) keep += ired[w];
    keep = max(keep, 1);
  }
  float m2 = -INFINITY;
  for (int j = threadIdx.x; j < keep; j += blockDim.x) m2 = fmaxf(m2, val[perm[j]]);
  m2 = block_max_f(m2, red);
  float s2 = 0.0f;
  for (int j = threadIdx.x; j < keep; j += blockDim.x) s2 += __expf(val[perm[j]] - m2);
  s2 = block_sum_f(s2, red + 16);
  const float L2 = m2 + __logf(s2);
  for (int j = threadIdx.x; j < keep; j += blockDim.x) logw_out[j] = val[perm[j]] - L2;
  if (threadIdx.x == 0) *nkeep = keep;
}

__global__ void k_gather_rows(int n, int stride, const uint32_t* perm, const int32_t* in, int32_t* out) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)n * stride) return;
  const int j = (int)(t / stride), s = (int)(t % stride);
  out[t] = in[(size_t)perm[j] * stride + s];
}
__global__ void k_gather_u(int n, const uint32_t* perm, const int32_t* in, int32_t* out) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) out[j] = in[perm[j]];
}

// child rows: parent row with every instance replaced by its updated instance
__global__ __launch_bounds__(256) void k_child_rows(int n, int stride, const int32_t* ch_h, const int32_t* hp_map,
                                                    const int32_t* rows, const int32_t* did, const int32_t* eb,
                                                    const int32_t* eoff, const int32_t* exc_id, const int32_t* moff,
                                                    const int32_t* mod_b, const int32_t* mod_id, int32_t* out) {
  const int c = blockIdx.x;
  const int h = ch_h[c], hp = hp_map[h];
  const int m0 = moff[c], m1 = moff[c + 1];
  for (int s = threadIdx.x; s < stride; s += blockDim.x) {
    const int u = rows[(size_t)h * stride + s];
    int id = -1;
    if (u >= 0) {
      id = did[u];
      const int e = find_exc(eb, eoff, hp, s);
      if (e >= 0) id = exc_id[e];
      for (int q = m0; q < m1; ++q)
        if (mod_b[q] == s) id = mod_id[q];
    }
    out[(size_t)c * stride + s] = id;
  }
}

__global__ void k_gather_i32(int n, const int32_t* idx, const int32_t* in, int32_t* out) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < n) out[k] = in[idx[k]];
}
__global__ void k_did(int U, const int32_t* first, const int32_t* dpre, const int32_t* rec_id, int32_t* did) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < U) did[u] = first[u] == INT32_MAX ? -1 : rec_id[dpre[u]];
}
__global__ void k_def_flags(int U, const int32_t* first, int32_t* fl) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  if (u < U) fl[u] = first[u] == INT32_MAX ? 0 : 1;
}

// ------------------------------------------------------------------ births
// With a learned proposal applied, rmass[i] (fixed point) is the likelihood of the pairs it
// removed from detection i over the most likely hypothesis' instances; it is restored in every
// cell's mass (and so in every hypothesis' mass), so that the clutter probabilities behind the
// births do not count the removed pairs as clutter.
// log(e^a + e^b); the log of 1 + x with x in (0, 1] loses at most 6e-8 absolute against log1p
__device__ __forceinline__ float lse2(float a, float b) { return fmaxf(a, b) + __logf(1.0f + __expf(-fabsf(a - b))); }

// lzr[h] = lzprime[h] + sum_i (log(e^{l_hi} + R_i) - l_hi) over the detections with removed
// mass R_i.  One workgroup first: per detection lr_i = log R_i - c_i (-inf without removed
// mass; R_i from the fixed-point sums) and hypothesis 0's terms T0_i, with their FP64 total,
// which stand for every untouched cell.
__global__ __launch_bounds__(256) void k_ru_t0(int M, const uint32_t* cmax, const unsigned long long* rmass,
                                               const float* lserel0, float* lr, float* t0, double* tot) {
  __shared__ double red[4];
  double acc = 0.0;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    const float r = rmass[i] == 0ull ? -INFINITY : logf((float)((double)rmass[i] / kRemovedScale)) - o2f(cmax[i]);
    lr[i] = r;
    const float ls = lserel0[i];
    const float v = r == -INFINITY ? 0.0f : lse2(ls, r) - ls;
    t0[i] = v;
    acc += (double)v;
  }
  for (int d = kWave / 2; d > 0; d >>= 1) acc += __shfl_xor(acc, d, kWave);
  if (lane_id() == 0) red[threadIdx.x / kWave] = acc;
  __syncthreads();
  if (threadIdx.x == 0) *tot = red[0] + red[1] + red[2] + red[3];
}
// Then one wave per hypothesis exchanges T0_i for its own term on its touched cells: the
// touched cells lie at h M + j in ascending detection order, so the wave lists their detection
// indices in LDS (a chunk of 64 touched-set words at a time) and its lanes take the cells in
// turn, fixed butterfly.  (A last-workgroup normaliser here measured slower than its own
// launch: the agent-scope fences it needs write back every XCD's L2.)
constexpr int kRestoreT = 256;
__global__ __launch_bounds__(kRestoreT) void k_ru_restore(int H, int M, const float* lzprime, CellView cv,
                                                          const float* lr, const float* t0, const double* tot,
                                                          float* lzr) {
  __shared__ uint16_t list[kRestoreT / kWave][kWave * 32];
  const int w = threadIdx.x / kWave, lane = lane_id();
  const int h = blockIdx.x * (kRestoreT / kWave) + w;
  if (h < H) {
    float acc = 0.0f;
    if (h > 0) {
      int nbase = 0;  // touched cells before the chunk
      for (int x0 = 0; x0 < cv.W; x0 += kWave) {
        const int x = x0 + lane;
        const uint32_t word = x < cv.W ? cv.tbits[(size_t)h * cv.W + x] : 0u;
        const int c = __popc(word);
        int incl = c;  // inclusive scan of the counts over the lanes
        for (int d = 1; d < kWave; d <<= 1) {
          const int y = __shfl_up(incl, d, kWave);
          if (lane >= d) incl += y;
        }
        const int tot_c = __shfl(incl, kWave - 1, kWave);
        uint32_t b = word;
        for (int q = incl - c; b; ++q) {
          list[w][q] = (uint16_t)(32 * x + __ffs(b) - 1);
          b &= b - 1u;
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        for (int j = lane; j < tot_c; j += kWave) {
          const int i = list[w][j];
          const float r = lr[i];
          if (r != -INFINITY) {
            const float ls = cv.lserel[(size_t)h * M + nbase + j];
            acc += (lse2(ls, r) - ls) - t0[i];
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        __builtin_amdgcn_wave_barrier();
        nbase += tot_c;
      }
    }
    for (int d = kWave / 2; d > 0; d >>= 1) acc += __shfl_xor(acc, d, kWave);
    if (lane == 0) lzr[h] = lzprime[h] + (float)(*tot + (double)acc);
  }
}
// one workgroup: out = log sum_h exp(v[h])
__global__ __launch_bounds__(1024) void k_lse_block(int H, const float* v, float* out) {
  __shared__ float red[32];
  float mx = -INFINITY;
  for (int h = threadIdx.x; h < H; h += blockDim.x) mx = fmaxf(mx, v[h]);
  mx = block_max_f(mx, red);
  float sm = 0.0f;
  for (int h = threadIdx.x; h < H; h += blockDim.x) sm += __expf(v[h] - mx);
  sm = block_sum_f(sm, red + 16);
  if (threadIdx.x == 0) *out = mx + __logf(sm);
}
constexpr int kRuChunk = 16;  // hypotheses per partial sum of the births' clutter shares
__global__ __launch_bounds__(256) void k_ru_part(int H, int M, const float* lzprime, const float* lz,
                                                 CellView cv, const uint32_t* cmax, float lgk,
                                                 const float* lrm, float* part) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  const int ch = blockIdx.y;
  if (i >= M) return;
  const float c = o2f(cmax[i]);
  const float L = *lz;
  const bool rest = lrm && lrm[i] != -INFINITY;
  const float lr = rest ? lrm[i] : 0.0f;
  // the clutter share exp(log kappa - c_i - log mass) of a cell with log mass ls (relative to
  // c_i, with the removed mass restored when the proposal removed pairs of this detection)
  auto share = [&](float ls) { return __expf(lgk - c - (rest ? lse2(ls, lr) : ls)); };
  // sum over the chunk of pi_h * share(ls_hi): the chunk's weight times hypothesis 0's share,
  // plus pi_h * (share - hypothesis 0's) over the chunk's touched cells of detection i
  const float g0 = share(cv.lserel[i]);
  const uint32_t bit = 1u << (i & 31);
  float wsum = 0.0f, acc = 0.0f;
  // the chunk's touched words first (independent loads), then the touched cells
  uint32_t word[kRuChunk];
  float pi[kRuChunk];
#pragma unroll
  for (int j = 0; j < kRuChunk; ++j) {
    const int h = ch * kRuChunk + j;
    const bool in = h < H;
    pi[j] = in ? __expf(lzprime[h] - L) : 0.0f;
    word[j] = (in && h > 0) ? cv.tbits[(size_t)h * cv.W + (i >> 5)] : 0u;
  }
#pragma unroll
  for (int j = 0; j < kRuChunk; ++j) {
    wsum += pi[j];
    if (word[j] & bit) {
      const int h = ch * kRuChunk + j;
      const size_t wi = (size_t)h * cv.W + (i >> 5);
      acc += pi[j] * (share(cv.lserel[(size_t)h * M + cv.tpre[wi] + __popc(word[j] & (bit - 1u))]) - g0);
    }
  }
  part[(size_t)ch * M + i] = wsum * g0 + acc;
}
// one wave per detection: the chunks' partial sums, lanes over the chunks, fixed butterfly
__global__ __launch_bounds__(256) void k_ru_final(int M, int nch, const float* part, float* ru) {
  const int i = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kWave);
  if (i >= M) return;
  float s = 0.0f;
  for (int ch = lane_id(); ch < nch; ch += kWave) s += part[(size_t)ch * M + i];
  for (int d = kWave / 2; d > 0; d >>= 1) s += __shfl_xor(s, d, kWave);
  if (lane_id() == 0) ru[i] = 1.0f - s;
}

// one wave: greedy clustering of the seeds in detection order (a seed joins the first
// cluster whose first seed lies within cd), one birth per cluster.  Lane 0 keeps every
// cluster's sums while it assigns the seeds in detection order, so each sum adds its terms in
// detection order; the lanes fetch the detections of a chunk of 64 at once.
constexpr int kMaxClusters = 4096;
__global__ __launch_bounds__(64) void k_births(int M, const float2* z, const float* ru, float rumax, float cd,
                                               float sig2, float sigv2, float rmax, float brate, int32_t* member,
                                               DBirth* out, int32_t* nb_out, uint32_t* errf) {
  __shared__ float2 az[kMaxClusters];   // first seed of each cluster
  __shared__ float4 acc[kMaxClusters];  // sum x, sum y, sum (1 - r_U), count
  const int lane = lane_id();
  int ncl = 0;
  float tot = 0.0f;  // lane 0: total weight of the seeds, in detection order
  const float cd2 = cd * cd;
  for (int i0 = 0; i0 < M; i0 += kWave) {
    const int ii = i0 + lane;
    float2 zl = make_float2(0.f, 0.f);
    float rl = 1.0f;
    if (ii < M) {
      zl = z[ii];
      rl = ru[ii];
    }
    const bool seed = ii < M && rl < rumax;
    const uint64_t seeds = __ballot(seed);
    if (ii < M && !seed) member[ii] = -1;
    uint64_t b = seeds;
    while (b) {
      const int k = __ffsll((unsigned long long)b) - 1;
      b &= b - 1;
      const float2 zi = make_float2(__shfl(zl.x, k, kWave), __shfl(zl.y, k, kWave));
      const float ri = __shfl(rl, k, kWave);
      int found = -1;
      for (int c0 = 0; c0 < ncl && found < 0; c0 += kWave) {
        const int c = c0 + lane;
        bool hit = false;
        if (c < ncl) {
          const float dx = zi.x - az[c].x, dy = zi.y - az[c].y;
          hit = dx * dx + dy * dy <= cd2;
        }
        const uint64_t hb = __ballot(hit);
        if (hb) found = c0 + __ffsll((unsigned long long)hb) - 1;
      }
      if (found < 0) {
        if (ncl >= kMaxClusters) {
          if (lane == 0) atomicOr(errf, ERR_BIRTH);
          found = kMaxClusters - 1;
        } else {
          if (lane == 0) {
            az[ncl] = zi;
            acc[ncl] = make_float4(0.f, 0.f, 0.f, 0.f);
          }
          found = ncl++;
        }
      }
      if (lane == 0) {
        member[i0 + k] = found;
        float4 a4 = acc[found];
        a4.x += zi.x;
        a4.y += zi.y;
        a4.z += 1.0f - ri;
        a4.w += 1.0f;
        acc[found] = a4;
        tot += 1.0f - ri;
      }
      __syncthreads();
    }
  }
  tot = __shfl(tot, 0, kWave);
  __syncthreads();
  for (int c = lane; c < ncl; c += kWave) {
    const float4 a4 = acc[c];
    const float n = a4.w;
    DBirth bb;
    bb.m[0] = a4.x / n;
    bb.m[1] = a4.y / n;
    bb.m[2] = bb.m[3] = 0.0f;
    for (int k = 0; k < 10; ++k) bb.P[k] = 0.0f;
    bb.P[0] = bb.P[4] = sig2 / n;
    bb.P[7] = bb.P[9] = sigv2;
    bb.r = fminf(rmax, brate * a4.z / tot);
    bb.pad = 0;
    out[c] = bb;
  }
  if (lane == 0) *nb_out = ncl;
}

// ------------------------------------------------------------------ orchestration
namespace {
template <class T> T read1(Ctx& c, const T* p) {
  static_assert(sizeof(T) == 4, "one 32-bit word");
  const uint32_t* h = read_back(c.sb.hs, c.s, {{p, 1}});
  T v;
  std::memcpy(&v, h, sizeof(T));
  return v;
}
void check_err_bits(uint32_t e) {
  if (e & ERR_NAN) throw Error{GLMB_E_ARG, "detections contain NaN or infinity"};
  if (e & ERR_BIRTH) throw Error{GLMB_E_CAPACITY, "more than 4096 birth clusters in one scan"};
  if (e & ERR_DEPTH) throw Error{GLMB_E_CAPACITY, "a kept child deviates in more than 48 detections"};
}
}  // namespace

// Lists sized for every (label, detection) pair when that stays below kListsCap entries.
constexpr int64_t kListsCap = int64_t(1) << 26;
// mask width in words for a longest list of mx detections, with the LDS the mask kernels need
static int mask_width(int NS, int mx) {
  const int LW = std::max(1, (mx + 31) / 32);
  const size_t lds_need = (size_t)NS * LW * sizeof(uint32_t);
  if (lds_need > 160 * 1024)
    throw Error{GLMB_E_CAPACITY, "labels x detection-set mask width exceed the 160 KB LDS of a workgroup"};
  if (lds_need > 64 * 1024) {
    GLMB_HIP(hipFuncSetAttribute((const void*)k_default_masks, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds_need));
    GLMB_HIP(hipFuncSetAttribute((const void*)k_exceptions, hipFuncAttributeMaxDynamicSharedMemorySize,
                                 (int)lds_need));
  }
  return LW;
}

// U0 + U1 scores: detections, gate bits and Eq. 2 entries of every (instance, detection) pair.
// Scalars: see stage_update.
void gate_scores(Ctx& c, const float* zin, int M, bool pairs) {
  hipStream_t s = c.s;
  const int T = 256;
  const int U = c.ninst;
  const glmb_params& p = c.p;
  const float sig2 = p.sigma_z * p.sigma_z;
  const float lgk = logf(p.clutter_density);
  const float lgc = (float)(std::log((double)p.det_rate) - std::log(2.0 * M_PI));
  const int W = std::max(1, (M + 31) / 32);
  int32_t* scal = need<int32_t>(c.scal, 64);
  uint32_t* errf = (uint32_t*)scal;
  unsigned long long* ngated = (unsigned long long*)(scal + 2);
  GLMB_HIP(hipMemsetAsync(scal, 0, 64 * sizeof(int32_t), s));
  float2* z = need<float2>(c.z, M);
  int32_t* pcnt = pairs ? need<int32_t>(c.pcnt, U + 1) : nullptr;
  unsigned long long* rmass = pairs ? need<unsigned long long>(c.rmass, M + 1) : nullptr;
  GLMB_LAUNCH(k_z_in, cdiv(std::max(M + 1, pairs ? U + 1 : 0), T), T, 0, s, zin, M, z, errf, pcnt, U + 1, rmass);
  uint32_t* cmax = need<uint32_t>(c.cmax, M);
  {
    float fl = lgk;
    uint32_t uu;
    std::memcpy(&uu, &fl, 4);
    const uint32_t init = (uu & 0x80000000u) ? ~uu : (uu | 0x80000000u);
    GLMB_LAUNCH(k_fill_u32, cdiv(M, T), T, 0, s, cmax, M, init);
  }
  uint32_t* gbits = need<uint32_t>(c.gbits, (int64_t)U * W);
  float* phi = need<float>(c.phi, (int64_t)U * M);
  int32_t *pn = nullptr, *pu = nullptr, *pi = nullptr;
  if (pairs) {  // the learned update's pair list, in arbitrary order of the gate's waves
    pn = scal + 19;  // zeroed with the scalars above
    pu = need<int32_t>(c.pu, (int64_t)U * M);
    pi = need<int32_t>(c.pi, (int64_t)U * M);
  }
  if (U > 0 && M > 0) {
    const int64_t waves = (int64_t)cdiv(U, kGateIpw) * cdiv(M, kWave);
    GLMB_LAUNCH(k_gate, cdiv(waves * kWave, T), T, 0, s, (const DInst*)c.inst.p, U, z, M, W, sig2, p.gate_d2, lgc,
                gbits, phi, cmax, ngated, pcnt, pn, pu, pi);
  } else if (U > 0) {
    GLMB_LAUNCH(k_fill_u32, cdiv((int64_t)U * W, T), T, 0, s, gbits, U * W, 0u);  // no detections: nothing gated
  }
}

// U1 lists from the gate bits: per-label gated detection lists and per-detection candidate
// label slots.  Sets c.LW (detection-set mask width in words), or with `defer` leaves it to
// lw_from_lists (the longest list is at scal[27]) and sizes the lists for every (label,
// detection) pair instead of reading their total back; the error flags are then read with
// the update's statistics.
void gate_lists(Ctx& c, int M, bool defer) {
  hipStream_t s = c.s;
  const int T = 256;
  const int U = c.ninst, NS = c.nslot;
  const int W = std::max(1, (M + 31) / 32);
  int32_t* scal = c.scal.as<int32_t>();
  uint32_t* errf = (uint32_t*)scal;
  int32_t* tot = scal + 12;
  const uint32_t* gbits = c.gbits.as<uint32_t>();
  int32_t* beg = need<int32_t>(c.inst_beg, NS + 1);
  GLMB_LAUNCH(k_inst_beg, cdiv(NS + 1, T), T, 0, s, (const DInst*)c.inst.p, U, NS, beg);
  uint32_t* lbits = need<uint32_t>(c.lbits, (int64_t)NS * W);
  int32_t* lpre = need<int32_t>(c.lpre, (int64_t)NS * W);
  int32_t* llen = need<int32_t>(c.llen, NS + 1);
  int32_t* loff = need<int32_t>(c.loff, NS + 1);
  int32_t* maxlen = scal + 27;  // zeroed with the scalars at the start of the update
  if (M > 0) GLMB_LAUNCH(k_label_bits, NS, 256, 0, s, gbits, beg, W, lbits, lpre, llen, errf, maxlen);
  else GLMB_LAUNCH(k_fill_i32, cdiv(NS + 1, T), T, 0, s, llen, NS + 1, 0);
  scan_excl(llen, loff, NS, tot, c.tmp, s);
  int LW = 1, nl = 0;
  defer = defer && (int64_t)NS * M <= kListsCap;
  if (defer) {
    nl = NS * M;
    LW = 0;  // lw_from_lists
  } else {
    // one round trip: the list lengths, their total and the error flags (set by k_z_in and
    // k_label_bits, both queued above)
    const uint32_t* hb = read_back(c.sb.hs, s, {{llen, NS}, {tot, 1}, {errf, 1}});
    const int32_t* hl = (const int32_t*)hb;
    nl = hl[NS];
    const uint32_t e = hb[NS + 1];
    if (e & ERR_NAN) throw Error{GLMB_E_ARG, "detections contain NaN or infinity"};
    int mx = 0;
    for (int j = 0; j < NS; ++j) mx = std::max(mx, hl[j]);
    LW = mask_width(NS, mx);
  }
  c.LW = LW;
  int32_t* lmeas = need<int32_t>(c.lmeas, nl);
  if (M > 0) GLMB_LAUNCH(k_label_list, cdiv((int64_t)NS * W, T), T, 0, s, lbits, lpre, loff, NS, W, lmeas);
  int32_t* ccnt = need<int32_t>(c.ccnt, M + 1);
  int32_t* coff = need<int32_t>(c.coff, M + 1);
  GLMB_LAUNCH(k_cand, cdiv((int64_t)M * kWave, T), T, 0, s, lbits, NS, W, M, (const int32_t*)nullptr, ccnt,
              (int32_t*)nullptr);
  scan_excl(ccnt, coff, M, coff + M, c.tmp, s);
  // the candidate lists hold the same gated (label, detection) pairs as the label lists
  const int ncand = M > 0 ? nl : 0;
  int32_t* cand = need<int32_t>(c.cand, ncand);
  GLMB_LAUNCH(k_cand, cdiv((int64_t)M * kWave, T), T, 0, s, lbits, NS, W, M, (const int32_t*)coff, ccnt, cand);
  trace(c, "update.lists", ncand, NS);
}

// U2 on the current lists: per-cell normalisers, per-hypothesis B'_h and log Z'_h, log Z'.
void assoc_norm(Ctx& c, int M) {
  hipStream_t s = c.s;
  const int H = c.nhyp, SW = c.stride;
  const glmb_params& p = c.p;
  const float lgk = logf(p.clutter_density);
  int32_t* scal = c.scal.as<int32_t>();
  unsigned long long* nopts = (unsigned long long*)(scal + 4);
  float* lz = (float*)(scal + 8);
  unsigned long long* ndense = (unsigned long long*)(scal + 16);
  const int64_t HM = (int64_t)H * M;
  int16_t* best16 = need<int16_t>(c.best16, HM);
  float* dev1 = need<float>(c.dev1, HM);
  float* lserel = need<float>(c.lserel, HM);
  const int WM = (M + 31) / 32;
  uint32_t* tbits = need<uint32_t>(c.tbits, (int64_t)H * WM);
  uint16_t* tpre = need<uint16_t>(c.tpre, (int64_t)H * WM);
  float* bprime = need<float>(c.bprime, H);
  float* lzprime = need<float>(c.lzprime, H);
  float* ref_b1 = need<float>(c.ref_b1, M + 1);
  int32_t* ref_opts = need<int32_t>(c.ref_opts, M + 1);
  TopE* ref_top = need<TopE>(c.ref_top, M + 1);
  float* ref_rest = need<float>(c.ref_rest, M + 1);
  int32_t* hopts = need<int32_t>(c.hopts, H + 1);
  GLMB_LAUNCH(k_assoc_ref, cdiv((int64_t)M * kWave, 256), 256, 0, s, M, c.rows.as<int32_t>(), lgk,
              c.coff.as<int32_t>(), c.cand.as<int32_t>(), c.phi.as<float>(), c.cmax.as<uint32_t>(), best16, dev1,
              lserel, ref_b1, ref_opts, ref_top, ref_rest);
  double* rtot = need<double>(c.ref_tot, 4);
  GLMB_LAUNCH(k_assoc_ref_sum, 1, 256, 0, s, M, (const float*)ref_b1, (const float*)lserel,
              (const int32_t*)ref_opts, c.logw.as<float>(), c.ntrk.as<int32_t>(), p.det_rate, bprime, lzprime,
              hopts, rtot);
  // one wave per hypothesis; up to four waves per workgroup, as LDS allows
  const int W = std::max(1, (M + 31) / 32);
  const int nq = std::min(16, 512 / W);
  const size_t wbytes = (size_t)assoc_wave_words(M, nq) * sizeof(int32_t);
  const int wpb = (int)std::max<size_t>(1, std::min<size_t>(4, (64 * 1024) / wbytes));
  const size_t lds = wbytes * wpb;
  if (lds > 160 * 1024) throw Error{GLMB_E_CAPACITY, "association pass needs more than 160 KB of LDS"};
  if (lds > 64 * 1024)
    GLMB_HIP(hipFuncSetAttribute((const void*)k_assoc, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  c.mark(1);  // the events bracket k_assoc alone
  GLMB_LAUNCH(k_assoc, cdiv(H - 1, wpb), wpb * kWave, lds, s, H, M, SW, nq, c.rows.as<int32_t>(),
              c.logw.as<float>(), c.ntrk.as<int32_t>(), p.det_rate, lgk, c.coff.as<int32_t>(), c.cand.as<int32_t>(),
              c.phi.as<float>(), c.cmax.as<uint32_t>(), c.loff.as<int32_t>(), c.llen.as<int32_t>(),
              c.lmeas.as<int32_t>(), c.lbits.as<uint32_t>(), ref_b1, ref_opts, (const TopE*)ref_top,
              (const float*)ref_rest, best16, dev1, lserel, tbits, tpre, (const double*)rtot, bprime, lzprime,
              hopts);
  c.mark(2);
  float* dbest = need<float>(c.diag_best, H);
  float* dlogpi = need<float>(c.diag_logpi, H);
  GLMB_LAUNCH(k_norm, 1, 1024, 0, s, H, M, bprime, lzprime, hopts, c.ntrk.as<int32_t>(), lz, dbest, dlogpi, nopts,
              ndense);
}

void stage_update(Ctx& c, int k, const float* zin, int M) {
  hipStream_t s = c.s;
  const int T = 256;
  const int H = c.nhyp, U = c.ninst, NS = c.nslot, SW = c.stride;
  const glmb_params& p = c.p;
  const float sig2 = p.sigma_z * p.sigma_z;
  const float lgk = logf(p.clutter_density);
  // scalars: [0] errf, [2..3] ngated (u64), [4..5] nopts (u64), [8] logZ', [9] t0, [10] nkeep,
  // [11] retained, [12] scratch total, [13] births, [14] exceptions, [16..17] dense triples (u64),
  // [18] pairs removed by the proposal
  c.stats = glmb_step_stats{};
  const int64_t syncs0 = g_stream_syncs;
  c.stats.n_hyp_in = H;
  c.stats.n_meas = M;
  c.stats.n_inst_in = U;
  c.stats.n_labels = NS;
  double lost = 0.0;
  if (c.prop_on && c.prop_measure) {
    // posterior mass the proposal removes, measured on the full association space first
    proposal_lost(c, k, zin, M, &c.prop_t, 1, &lost);
  }

  // ---- U0 + U1: detections, gate, scores
  trace(c, "update.begin", H, M);
  c.mark(0);
  // the learned proposal's label inputs beside the gate (joined before the pairs are scored)
  bool slots_ready = false;
  if (c.prop_on && M > 0 && c.fork_ok) {
    c.side_ready();
    GLMB_HIP(hipEventRecord(c.fork[0], s));
    GLMB_HIP(hipStreamWaitEvent(c.s2, c.fork[0], 0));
    prepare_slots(c, k, c.s2);
    GLMB_HIP(hipEventRecord(c.fork[2], c.s2));
    slots_ready = true;
  }
  gate_scores(c, zin, M, c.prop_on && M > 0);
  int32_t* scal = c.scal.as<int32_t>();
  uint32_t* errf = (uint32_t*)scal;
  unsigned long long* ngated = (unsigned long long*)(scal + 2);
  unsigned long long* nopts = (unsigned long long*)(scal + 4);
  float* lz = (float*)(scal + 8);
  float* t0 = (float*)(scal + 9);
  int32_t* nkeep = scal + 10;
  float* retained = (float*)(scal + 11);
  int32_t* tot = scal + 12;
  int32_t* nb_out = scal + 13;
  unsigned long long* ndense = (unsigned long long*)(scal + 16);
  (void)ngated;
  (void)nopts;
  (void)ndense;
  float2* z = c.z.as<float2>();
  uint32_t* cmax = c.cmax.as<uint32_t>();
  float* phi = c.phi.as<float>();
  if (c.prop_on && M > 0) proposal_apply(c, k, M, slots_ready);
  gate_lists(c, M, true);
  int32_t* loff = c.loff.as<int32_t>();
  int32_t* llen = c.llen.as<int32_t>();
  int32_t* lmeas = c.lmeas.as<int32_t>();
  int32_t* coff = c.coff.as<int32_t>();
  int32_t* cand = c.cand.as<int32_t>();

  // ---- U2: per (hypothesis, detection) normalisers
  trace(c, "update.U2");
  assoc_norm(c, M);
  const CellView cv = cells_of(c, M);
  float* bprime = c.bprime.as<float>();
  float* lzprime = c.lzprime.as<float>();

  // ---- the births' clutter probabilities r_U(z_i) need only U2's results: on the side
  // stream, beside the selection and the materialisation (joined before the births)
  float* ru = need<float>(c.diag_ru, M + 1);
  auto launch_ru = [&](hipStream_t st) {
    const int nch = cdiv(H, kRuChunk);
    float* part = need<float>(c.ru_part, (int64_t)nch * M);
    const float* lzb = lzprime;
    const float* Lb = lz;
    float* lrm = nullptr;
    if (c.prop_on) {  // hypothesis masses with the removed pairs restored, and their normaliser
      // [H + 1 masses and normaliser | M removed masses | M terms of hypothesis 0 | FP64 total]
      const int64_t o_tot = ((int64_t)H + 1 + 2 * (int64_t)M + 1) & ~(int64_t)1;
      float* lzr = need<float>(c.lz_r, o_tot + 2);
      lrm = lzr + H + 1;
      float* t0r = lrm + M;
      double* tot0 = (double*)(lzr + o_tot);
      GLMB_LAUNCH(k_ru_t0, 1, 256, 0, st, M, cmax, (const unsigned long long*)c.rmass.as<unsigned long long>(),
                  cv.lserel, lrm, t0r, tot0);
      GLMB_LAUNCH(k_ru_restore, cdiv(H, kRestoreT / kWave), kRestoreT, 0, st, H, M, lzprime, cv, (const float*)lrm,
                  (const float*)t0r, (const double*)tot0, lzr);
      GLMB_LAUNCH(k_lse_block, 1, 1024, 0, st, H, lzr, lzr + H);
      lzb = lzr;
      Lb = lzr + H;
    }
    hipLaunchKernelGGL(k_ru_part, dim3(cdiv(M, T), nch), dim3(T), 0, st, H, M, lzb, Lb, cv, cmax, lgk, lrm, part);
    GLMB_HIP(hipGetLastError());
    GLMB_LAUNCH(k_ru_final, cdiv((int64_t)M * kWave, T), T, 0, st, M, nch, part, ru);
  };
  bool ru_forked = false;
  if (M > 0 && c.fork_ok) {
    c.side_ready();
    GLMB_HIP(hipEventRecord(c.fork[1], s));
    GLMB_HIP(hipStreamWaitEvent(c.s2, c.fork[1], 0));
    launch_ru(c.s2);
    GLMB_HIP(hipEventRecord(c.fork[3], c.s2));
    ru_forked = true;
  }

  const int K = p.h_max;
  const bool sampled = c.sample_hup > 0;
  Selected sel{};
  const int32_t* ito = nullptr;
  const int32_t* itg = nullptr;
  int nsel = 0;
  const uint32_t* kept_draw = nullptr;
  float* sel_value = nullptr;
  if (sampled) {
    // ---- U3 by the paper's generator: h_up maps drawn per hypothesis, distinct ones kept
    trace(c, "update.U3.sampled", H, c.sample_hup);
    nsel = sample_children(c, k, M, K, &sel_value, &kept_draw);
    if (nsel < 1) throw Error{GLMB_E_STATE, "sampled update kept no hypothesis"};
    sel.n = nsel;
    sel.nodes = c.sample_unique;
    sel.value = sel_value;
    sel.form = 3;
  } else {
  // ---- U3: lower bound of the cut, deviation items, exact selection
  trace(c, "update.U3");
  kth_bound_cells_sub(bprime, cv, H, M, K, t0, c.tmp, c.ref_sel, s);
  // counting bound, first pass (from the cells' first deviations): the items are generated
  // for the children above it only
  const float* tcut = dp_bound_rows(bprime, H, cv, M, K, t0, c.sb, s);
  struct Items {
    int ncell, nitem;
    int32_t *itoff, *itg, *ito;
    float* itd;
  };
  // cells (h, i) and their deviation items above the bound *tb, sorted per parent by delta
  auto make_items = [&](const float* tb) {
    Items r{};
    int32_t* rcount = need<int32_t>(c.flags, H + 1);
    int32_t* roff = need<int32_t>(c.pre, H + 1);
    const int row_blocks = cdiv((int64_t)H * kWave, 256);
    GLMB_LAUNCH(k_row_cells, row_blocks, 256, 0, s, H, M, bprime, cv, tb, (const int32_t*)nullptr, rcount,
                (int32_t*)nullptr);
    scan_excl(rcount, roff, H, tot, c.tmp, s);
    const int ncell = read1(c, tot);
    int32_t* cells = need<int32_t>(c.cells, ncell);
    GLMB_LAUNCH(k_row_cells, row_blocks, 256, 0, s, H, M, bprime, cv, tb, (const int32_t*)roff, rcount, cells);
    int32_t* icount = need<int32_t>(c.ccount, ncell + 1);
    int32_t* ioff = need<int32_t>(c.coff2, ncell + 1);
    const int item_blocks = cdiv((int64_t)ncell * kWave, 256);
    GLMB_LAUNCH(k_items, item_blocks, 256, 0, s, ncell, cells, M, SW, c.rows.as<int32_t>(), coff, cand, phi, lgk,
                bprime, tb, (const int32_t*)nullptr, icount, (float*)nullptr, (int32_t*)nullptr, (int32_t*)nullptr,
                (uint64_t*)nullptr, (uint32_t*)nullptr);
    scan_excl(icount, ioff, ncell, ioff + ncell, c.tmp, s);
    int32_t* itoff = need<int32_t>(c.it_off, H + 1);
    int32_t* maxlen = scal + 22;
    int32_t* nlist = scal + 23;
    int32_t* ilist = need<int32_t>(c.it_h, H);
    GLMB_LAUNCH(k_fill_i32, 1, T, 0, s, maxlen, 2, 0);
    GLMB_LAUNCH(k_item_ranges, cdiv(H + 1, T), T, 0, s, H, ncell, M, cells, ioff, itoff, maxlen, nlist, ilist);
    int32_t hv[2];
    std::memcpy(hv, read_back(c.sb.hs, s, {{ioff + ncell, 1}, {maxlen, 1}}), sizeof(hv));
    const int nitem = hv[0];
    float* itd0 = need<float>(c.it_delta, 2 * (int64_t)nitem);
    int32_t* itg0 = need<int32_t>(c.it_group, 2 * (int64_t)nitem);
    int32_t* ito0 = need<int32_t>(c.it_opt, 2 * (int64_t)nitem);
    uint64_t* ikeys = need<uint64_t>(c.keys, nitem);
    uint32_t* ivals = need<uint32_t>(c.vals32, nitem);
    const bool segsort = hv[1] <= GLMB_SEGSORT_MAX;
    GLMB_LAUNCH(k_items, item_blocks, 256, 0, s, ncell, cells, M, SW, c.rows.as<int32_t>(), coff, cand, phi, lgk,
                bprime, tb, (const int32_t*)ioff, icount, itd0, itg0, ito0, segsort ? nullptr : ikeys,
                segsort ? nullptr : ivals);
    r.ncell = ncell;
    r.nitem = nitem;
    r.itoff = itoff;
    r.itd = itd0 + nitem;
    r.itg = itg0 + nitem;
    r.ito = ito0 + nitem;
    if (segsort) {
      // per-parent lists sorted in LDS, one workgroup per parent
      if (hv[1] > 1024)
        GLMB_LAUNCH(k_item_segsort<1024>, std::min(H, 512), 1024, 0, s, nlist, ilist, itoff, itd0, itg0, ito0, r.itd,
                    r.itg, r.ito);
      else
        GLMB_LAUNCH(k_item_segsort<256>, std::min(H, 1024), 256, 0, s, nlist, ilist, itoff, itd0, itg0, ito0, r.itd,
                    r.itg, r.ito);
    } else {
      // a parent with more items than one workgroup sorts: stable radix sort by (parent, delta)
      // of the items in generation order (detection, then option key)
      int hbits = 0;
      while ((1 << hbits) < H) ++hbits;
      sort_pairs(ikeys, ivals, nitem, 0, 32 + ((hbits + 7) / 8) * 8, c.tk, c.tv, c.tmp, s);
      GLMB_LAUNCH(k_item_perm, cdiv(nitem, T), T, 0, s, nitem, ivals, itd0, itg0, ito0, r.itd, r.itg, r.ito);
    }
    return r;
  };
  Items it = make_items(tcut);
  if (c.force_coop) c.sel_multi[1] = true;
  SelectIn si{H, bprime, it.itoff, it.itd, it.itg, K, tcut, &c.sel_multi[1], c.coop_ok, c.force_multi};
  si.group_bits = c.group_bits;
  si.dp_inflate = c.dp_inflate;
  dp_bound_items(si, c.sb, s);  // second pass: raises *tcut
  if (c.trace) dp_bound_trace(c.sb, s);
  trace(c, "update.select", it.ncell, it.nitem);
  std::string serr;
  const int cap_nodes = p.cap_nodes > 0 ? p.cap_nodes : (1 << 22);
  glmb_status st = select_topk(si, cap_nodes, c.sb, sel, s, serr, c.trace);
  if (st == GLMB_OK && sel.n < K && dp_bound_refined(c.sb, s)) {
    // fewer than K children above a bound whose count promised K: search again from the
    // caller's bound, with the items above it
    trace(c, "update.refine_retry", sel.n, K);
    it = make_items(t0);
    if (c.force_coop) c.sel_multi[1] = true;
    si = SelectIn{H, bprime, it.itoff, it.itd, it.itg, K, t0, &c.sel_multi[1], c.coop_ok, c.force_multi};
    si.group_bits = c.group_bits;
    st = select_topk(si, cap_nodes, c.sb, sel, s, serr, c.trace);
  }
  if (st != GLMB_OK) throw Error{st, serr};
  ito = it.ito;
  itg = it.itg;
  nsel = sel.n;
  if (nsel < 1) throw Error{GLMB_E_STATE, "selection kept no hypothesis (non-finite weights?)"};
  }
  if (sampled) {
    // values of the taken maps in rank order, with their parents and deviation counts
    int32_t* depth0 = need<int32_t>(c.ccount, nsel + 1);
    int32_t* chh0 = need<int32_t>(c.child_par, nsel + 1);
    sample_children_devs(c, M, nsel, kept_draw, sel_value, depth0, chh0);
  }
  float* wout = need<float>(c.logw2, nsel);
  GLMB_LAUNCH(k_prune, 1, 1024, 0, s, nsel, sel.value, p.tau, lz, wout, nkeep, retained);
  const int nk = read1(c, nkeep);

  // ---- U4: children, distinct (instance, detection set), Kalman, rows
  trace(c, "update.U4", nsel, nk);
  c.mark(3);
  int32_t* depth = need<int32_t>(c.ccount, nk + 1);
  int32_t* chh = need<int32_t>(c.child_par, nk + 1);
  int32_t* doff = need<int32_t>(c.dev_off, nk + 1);
  if (!sampled)
    GLMB_LAUNCH(k_child_depth, cdiv(nk, T), T, 0, s, nk, sel.node, sel.nd_parent, sel.nd_item, sel.nd_h, depth, chh,
                errf);
  scan_excl(depth, doff, nk, doff + nk, c.tmp, s);
  // retained parents
  int32_t* mark = need<int32_t>(c.row_mark, H + 1);
  GLMB_LAUNCH(k_fill_i32, cdiv(H + 1, T), T, 0, s, mark, H + 1, 0);
  GLMB_LAUNCH(k_mark, cdiv(nk, T), T, 0, s, nk, chh, mark);
  int32_t* ppre = need<int32_t>(c.pre, H + 1);
  scan_excl(mark, ppre, H, tot, c.tmp, s);
  // deviations of the kept children, retained parents (and the longest label list, when the
  // gate left the mask width open): one round trip
  const int32_t* cnt2 = (const int32_t*)read_back(c.sb.hs, s, {{doff + nk, 1}, {tot, 1}, {scal + 27, 1}});
  const int ndev = cnt2[0], np = cnt2[1];
  if (c.LW == 0) c.LW = mask_width(NS, cnt2[2]);
  const int LW = c.LW;
  int32_t* devi = need<int32_t>(c.dev_i, ndev);
  int32_t* devn = need<int32_t>(c.dev_slot, 2 * (int64_t)ndev);
  int32_t* devo = devn + ndev;
  if (sampled)
    sample_children_list(c, M, nk, kept_draw, chh, doff, devi, devn, devo);
  else
    GLMB_LAUNCH(k_child_devs, cdiv(nk, T), T, 0, s, nk, M, sel.node, sel.nd_parent, sel.nd_item, chh, doff, itg, ito,
                cv, devi, devn, devo);
  int32_t* plist = need<int32_t>(c.cells, np + 1);
  int32_t* hpm = need<int32_t>(c.hp_map, H + 1);
  GLMB_LAUNCH(k_plist, cdiv(H, T), T, 0, s, H, mark, ppre, plist, hpm);
  int32_t* first = need<int32_t>(c.first, 2 * (int64_t)U + 2);  // [first | default ids]
  GLMB_LAUNCH(k_fill_i32, cdiv(U + 1, T), T, 0, s, first, U + 1, INT32_MAX);
  GLMB_LAUNCH(k_first, cdiv((int64_t)np * SW, T), T, 0, s, np, plist, SW, c.rows.as<int32_t>(), first);
  uint32_t* dmask = need<uint32_t>(c.dmask, (int64_t)(U + 1) * LW);
  const size_t lds = (size_t)NS * LW * sizeof(uint32_t);
  GLMB_LAUNCH(k_default_masks, np, 256, lds, s, plist, M, NS, LW, SW, c.rows.as<int32_t>(), cv, loff, llen, lmeas,
              first, dmask);
  int ecap = std::max(1024, 4 * nk);
  int32_t* nexc = scal + 14;
  auto exc_bufs = [&](int cap_) {
    int32_t* b = need<int32_t>(c.exc, 6 * (int64_t)cap_ + 6);
    uint32_t* m = need<uint32_t>(c.cmod, 2 * (int64_t)cap_ * LW + 2);
    return std::make_pair(b, m);
  };
  auto eb_ = exc_bufs(ecap);
  GLMB_LAUNCH(k_exceptions, np, 256, lds, s, plist, M, NS, LW, SW, c.rows.as<int32_t>(), cv, loff, llen, lmeas,
              dmask, nexc, eb_.first, eb_.first + ecap, eb_.first + 2 * ecap, eb_.second, ecap);
  // child masks (count) and default records (flags) before the one round trip that reads the
  // exception, child-mask and default counts
  int32_t* mcount = need<int32_t>(c.ccount, nk + 1);
  int32_t* moff = need<int32_t>(c.coff2, nk + 1);
  GLMB_LAUNCH(k_child_mods, cdiv(nk, T), T, 0, s, nk, doff, devn, devo, (const int32_t*)nullptr, mcount,
              (int32_t*)nullptr, (int32_t*)nullptr);
  scan_excl(mcount, moff, nk, moff + nk, c.tmp, s);
  int32_t* dfl = need<int32_t>(c.flags, U + 1);
  int32_t* dpre = need<int32_t>(c.pmult, U + 1);
  GLMB_LAUNCH(k_def_flags, cdiv(U, T), T, 0, s, U, first, dfl);
  scan_excl(dfl, dpre, U, tot, c.tmp, s);
  const int32_t* cnt3 = (const int32_t*)read_back(c.sb.hs, s, {{nexc, 1}, {moff + nk, 1}, {tot, 1}});
  int ne = cnt3[0];
  const int nm = cnt3[1], nd = cnt3[2];
  if (ne > ecap) {  // grow and redo
    ecap = ne;
    eb_ = exc_bufs(ecap);
    GLMB_LAUNCH(k_fill_i32, 1, T, 0, s, nexc, 1, 0);
    GLMB_LAUNCH(k_exceptions, np, 256, lds, s, plist, M, NS, LW, SW, c.rows.as<int32_t>(), cv, loff, llen,
                lmeas, dmask, nexc, eb_.first, eb_.first + ecap, eb_.first + 2 * ecap, eb_.second, ecap);
    ne = read1(c, nexc);
  }
  // exceptions sorted by (retained parent, slot)
  int32_t *eu0 = eb_.first, *ea0 = eu0 + ecap, *eb0 = ea0 + ecap, *eu = eb0 + ecap, *ea = eu + ecap, *eb = ea + ecap;
  uint32_t *em0 = eb_.second, *em = em0 + (size_t)ecap * LW;
  {
    uint64_t* ek = need<uint64_t>(c.keys, ne + 1);
    uint32_t* ev = need<uint32_t>(c.vals32, ne + 1);
    GLMB_LAUNCH(k_exc_keys, cdiv(ne, T), T, 0, s, ne, ea0, eb0, ek, ev);
    int pb = 0;
    while ((1 << pb) < np) ++pb;
    sort_pairs(ek, ev, ne, 0, 32 + ((pb + 7) / 8) * 8, c.tk, c.tv, c.tmp, s);
    GLMB_LAUNCH(k_exc_perm, cdiv(ne, T), T, 0, s, ne, LW, ev, eu0, ea0, eb0, em0, eu, ea, eb, em);
  }
  int32_t* eoff = need<int32_t>(c.ids, np + 2);
  GLMB_LAUNCH(k_exc_off, cdiv(np + 1, T), T, 0, s, np, ne, ea, eoff);
  trace(c, "update.masks", np, ne);
  // records: defaults | exceptions | child masks
  const int R = nd + ne + nm;
  int32_t* rec_u = need<int32_t>(c.recs, 3 * (int64_t)R + 3);
  int32_t* rec_a = rec_u + R + 1;
  int32_t* rec_b = rec_a + R + 1;
  uint32_t* rec_m = need<uint32_t>(c.rec_m, (int64_t)(R + 1) * LW);
  GLMB_LAUNCH(k_rec_defaults, cdiv(U, T), T, 0, s, U, LW, first, dmask, dpre, rec_u, rec_m);
  GLMB_LAUNCH(k_rec_copy, cdiv(ne, T), T, 0, s, ne, LW, eu, em, rec_u + nd, rec_m + (size_t)nd * LW);
  GLMB_LAUNCH(k_child_mods, cdiv(nk, T), T, 0, s, nk, doff, devn, devo, (const int32_t*)moff, mcount,
              rec_a + nd + ne, rec_b + nd + ne);
  GLMB_LAUNCH(k_mod_masks, cdiv(nm, T), T, 0, s, nm, LW, chh, hpm, doff, devi, devn, devo, SW, c.rows.as<int32_t>(),
              loff, llen, lmeas, dmask, eb, em, eoff, (const int32_t*)(rec_a + nd + ne),
              (const int32_t*)(rec_b + nd + ne), rec_u + nd + ne, rec_m + (size_t)(nd + ne) * LW);
  uint64_t* rk = need<uint64_t>(c.rec_keys, R + 1);
  uint32_t* rv = need<uint32_t>(c.rec_vals, R + 1);
  GLMB_LAUNCH(k_rec_keys, cdiv(R, T), T, 0, s, R, LW, c.rec_hash_mask, rec_u, rec_m, rk, rv);
  int ub = 0;
  while ((1 << ub) < U) ++ub;
  sort_pairs(rk, rv, R, 0, 16 + ((ub + 7) / 8) * 8, c.tk, c.tv, c.tmp, s);
  int32_t* rfl = need<int32_t>(c.flags, R + 1);
  int32_t* rpre = need<int32_t>(c.pre, R + 1);
  int32_t* ncoll = scal + 24;  // tot (scal + 12) and this count come back in one round trip
  GLMB_LAUNCH(k_fill_i32, 1, T, 0, s, ncoll, 1, 0);
  GLMB_LAUNCH(k_rec_unique, cdiv(R, T), T, 0, s, R, LW, rk, rv, rec_u, rec_m, rfl, ncoll);
  scan_excl(rfl, rpre, R, tot, c.tmp, s);
  int32_t* rlead = nullptr;
  int nnew = 0;
  {
    int32_t hv2[13];
    std::memcpy(hv2, read_back(c.sb.hs, s, {{tot, 13}}), sizeof(hv2));
    nnew = hv2[0];
    if (hv2[12] > 0) {  // fingerprint collisions: ids by full comparison within each run
      trace(c, "update.fingerprint_collisions", hv2[12]);
      rlead = need<int32_t>(c.rec_lead, R + 1);
      GLMB_LAUNCH(k_rec_resolve, cdiv(R, T), T, 0, s, R, LW, rk, rv, rec_u, rec_m, rfl, rlead);
      scan_excl(rfl, rpre, R, tot, c.tmp, s);
      nnew = read1(c, tot);
    }
    c.stats.rec_collisions = hv2[12];
  }
  int32_t* rec_id = need<int32_t>(c.ids, (int64_t)R + np + 2);
  int32_t* rep = need<int32_t>(c.bt, nnew + 1);
  // eoff shares c.ids with rec_id: place it behind the record ids again
  int32_t* eoff2 = rec_id + R;
  GLMB_LAUNCH(k_exc_off, cdiv(np + 1, T), T, 0, s, np, ne, ea, eoff2);
  GLMB_LAUNCH(k_rec_ids, cdiv(R, T), T, 0, s, R, rv, rfl, rpre, (const int32_t*)rlead, rec_id, rep);
  trace(c, "update.kalman", R, nnew);
  DInst* ninst = (DInst*)need<uint8_t>(c.inst2, (int64_t)(nnew + 1) * sizeof(DInst));
  int32_t* onz = need<int32_t>(c.inst_nz, nnew + 1);
  int32_t* oz = need<int32_t>(c.inst_z, 8 * (int64_t)(nnew + 1));
  float* jc = c.joint_rw ? need<float>(c.j_corr, nnew + 1) : nullptr;
  GLMB_LAUNCH(k_kalman, cdiv(nnew, T), T, 0, s, nnew, LW, rep, rec_u, rec_m, (const DInst*)c.inst.p, loff, lmeas, z,
              sig2, ninst, onz, oz, phi, M, logf(p.det_rate), jc);
  int32_t* did = first + U + 1;
  GLMB_LAUNCH(k_did, cdiv(U, T), T, 0, s, U, first, dpre, rec_id, did);
  int32_t* nrows = need<int32_t>(c.rows2, (int64_t)nk * SW);
  GLMB_LAUNCH(k_child_rows, nk, 256, 0, s, nk, SW, chh, hpm, c.rows.as<int32_t>(), did, eb, eoff2, rec_id + nd, moff,
              rec_b + nd + ne, rec_id + nd + ne, nrows);
  int32_t* nntrk = need<int32_t>(c.ntrk2, nk + 1);
  GLMB_LAUNCH(k_gather_i32, cdiv(nk, T), T, 0, s, nk, chh, c.ntrk.as<int32_t>(), nntrk);
  c.last_perm = false;
  int nkept = nk;  // children after the (optional) exact-joint reweighting
  const int32_t* hpar = chh;
  if (c.joint_rw && nk > 0) {
    // ---- exact-joint reweighting of the kept children: joint likelihood of every track's
    // detection set, re-ranked, tau on the renormalised weights, renormalised
    trace(c, "update.joint", nk);
    float* jv = need<float>(c.j_val, nk + 1);
    uint64_t* jk = need<uint64_t>(c.j_keys, nk + 1);
    uint32_t* perm = need<uint32_t>(c.child_perm, nk + 1);
    GLMB_LAUNCH(k_joint_child, cdiv((int64_t)nk * kWave, T), T, 0, s, nk, SW, nrows, jc, wout, jv, jk, perm);
    sort_pairs(jk, perm, nk, 0, 64, c.tk, c.tv, c.tmp, s);
    float* jl = need<float>(c.j_lw, nk + 1);
    GLMB_LAUNCH(k_joint_tau, 1, 1024, 0, s, nk, perm, jv, p.tau, jl, nkeep);
    nkept = read1(c, nkeep);
    int32_t* rows3 = need<int32_t>(c.rows3, (int64_t)nkept * SW + 1);
    GLMB_LAUNCH(k_gather_rows, cdiv((int64_t)nkept * SW, T), T, 0, s, nkept, SW, perm, nrows, rows3);
    int32_t* jt = need<int32_t>(c.j_tmp, 2 * (int64_t)nkept + 2);
    GLMB_LAUNCH(k_gather_u, cdiv(nkept, T), T, 0, s, nkept, perm, nntrk, jt);
    GLMB_LAUNCH(k_gather_u, cdiv(nkept, T), T, 0, s, nkept, perm, chh, jt + nkept + 1);
    GLMB_HIP(hipMemcpyAsync(nntrk, jt, (size_t)nkept * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    GLMB_HIP(hipMemcpyAsync(wout, jl, (size_t)nkept * sizeof(float), hipMemcpyDeviceToDevice, s));
    hpar = jt + nkept + 1;
    std::swap(c.rows2, c.rows3);  // the re-ranked rows become the child rows
    c.last_perm = true;
  }

  // ---- births for the next scan
  trace(c, "update.births");
  c.mark(4);
  if (M > 0) {
    if (ru_forked) GLMB_HIP(hipStreamWaitEvent(s, c.fork[3], 0));
    else launch_ru(s);
  }
  int32_t* member = need<int32_t>(c.ru, (int64_t)M + 1);
  DBirth* nb = (DBirth*)need<uint8_t>(c.births2, (int64_t)(M + 1) * sizeof(DBirth));
  GLMB_LAUNCH(k_births, 1, 64, 0, s, M, z, ru, p.birth_ru_max, p.birth_cluster_d, sig2,
              p.birth_sigma_v * p.birth_sigma_v, p.birth_r_max, p.birth_rate, member, nb, nb_out, errf);

  // ---- statistics and swap in the new state
  trace(c, "update.stats");
  c.mark(5);
  // scalars (the error flags, scal[0], among them) and the first births: one round trip; the
  // prediction then needs no read of the births when there are at most kBirthHost of them
  constexpr int kBirthHost = 64;
  const int nbh = std::min(M + 1, kBirthHost);
  int32_t hs[19];
  const uint32_t* hb = read_back(c.sb.hs, s, {{scal, 19}, {nb, (int64_t)nbh * (int64_t)(sizeof(DBirth) / 4)}});
  std::memcpy(hs, hb, sizeof(hs));
  c.birth_host_ok = hs[13] >= 0 && hs[13] <= nbh;
  c.birth_host.resize(c.birth_host_ok ? hs[13] : 0);
  if (c.birth_host_ok && hs[13] > 0) std::memcpy(c.birth_host.data(), hb + 19, (size_t)hs[13] * sizeof(DBirth));
  check_err_bits((uint32_t)hs[0]);
  uint64_t ng, no;
  std::memcpy(&ng, hs + 2, 8);
  std::memcpy(&no, hs + 4, 8);
  uint64_t dense;
  std::memcpy(&dense, hs + 16, 8);
  float ret;
  std::memcpy(&ret, hs + 11, 4);
  // the predicted rows and instances stay in rows2 / inst2 after the swap below, until the
  // next prediction: the association-map export of this update reads them there
  c.last_H = H;
  c.last_M = M;
  c.last_stride = SW;
  std::swap(c.inst, c.inst2);
  std::swap(c.rows, c.rows2);
  std::swap(c.ntrk, c.ntrk2);
  std::swap(c.logw, c.logw2);
  std::swap(c.births, c.births2);
  if (hpar == c.child_par.as<int32_t>()) {
    std::swap(c.hparent, c.child_par);  // the children's parents become the state's (no copy)
  } else {
    int32_t* hp = need<int32_t>(c.hparent, nkept + 1);
    GLMB_HIP(hipMemcpyAsync(hp, hpar, (size_t)nkept * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
  }
  c.ninst = nnew;
  c.nhyp = nkept;
  c.nbirth = hs[13];
  c.birth_lab.clear();
  for (int b = 0; b < c.nbirth; ++b) c.birth_lab.push_back({k + 1, b});
  c.stats.n_hyp_out = nkept;
  c.stats.n_inst_out = nnew;
  c.stats.gated_pairs = (int64_t)ng;
  c.stats.option_terms = (int64_t)no;
  c.stats.dense_triples = (int64_t)dense;
  c.stats.search_nodes = sel.nodes;
  c.stats.search_levels = sel.levels;
  c.stats.search_form = sel.form;
  c.stats.n_births = c.nbirth;
  c.stats.retained_mass = std::exp((double)ret);
  c.stats.lost_mass = lost;
  c.stats.pairs_removed = hs[18];
  c.stats.host_syncs = (int32_t)(g_stream_syncs - syncs0);
  if (c.ev_ok) {
    const int a[6] = {0, 1, 2, 3, 4, 0}, b[6] = {1, 2, 3, 4, 5, 5};
    for (int j = 0; j < 6; ++j) {
      float ms = 0.0f;
      GLMB_HIP(hipEventElapsedTime(&ms, c.ev[a[j]], c.ev[b[j]]));
      c.stats.stage_ms[j] = ms;
    }
  }
}

}  // namespace glmb
