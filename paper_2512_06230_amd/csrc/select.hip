// Exact top-K over implicitly defined children (the "retain the H_max most likely
// hypotheses" step at the end of Sec. 3, and the same choice in prediction).
//
// A parent h has a base value B_h and a list of items (group g, option, delta >= 0)
// sorted by (delta, group, option).  A child picks at most one item per group; its
// value is B_h minus the picked deltas subtracted in item order.  Children are
// ranked by value descending, then by the canonical key (parent rank, number of
// picks, picked item positions in lexicographic order).
//
// GPU method: level-synchronous enumeration.  Level l holds every child with l picks
// whose value is >= the current threshold t; a node is extended by the items after
// its last one whose value stays >= t (a binary search on the sorted deltas gives the
// range, so no candidate below t is ever written).  Since removing a pick never lowers
// a value, this reaches every child >= t exactly once.  t starts at a lower bound on
// the K-th best value and is raised to a lower bound on the K-th largest value found so
// far whenever the node store runs full or a level completes; nodes below the new t are
// compacted away (their descendants are below it too).  At the end every child >= t is
// present, and a stable sort by (value desc, key) of those yields the exact top-K: the
// enumeration order is (level, parent rank, positions), so a stable sort by parent rank
// gives the canonical key order.
#include <hip/hip_cooperative_groups.h>

#include <atomic>

#include "common.hpp"

namespace glmb {

// one bit per group out of 64 (a one-hash Bloom filter of the groups a node has picked): a
// clear bit proves the group is not picked yet, so the walk up the node's picks is skipped
__device__ __forceinline__ uint64_t group_bit(int g) { return 1ull << (((uint32_t)g * 0x9E3779B1u) >> 26); }

__global__ void k_root_flags(const float* base, int P, const float* t, int32_t* flags) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h < P) flags[h] = base[h] >= *t ? 1 : 0;
}

__global__ void k_root_write(const float* base, int P, const float* t, const int32_t* pre, int32_t* nd_parent,
                             int32_t* nd_item, int32_t* nd_h, float* nd_value, uint64_t* nd_b) {
  const int h = blockIdx.x * blockDim.x + threadIdx.x;
  if (h < P && base[h] >= *t) {
    const int n = pre[h];
    nd_b[n] = 0ull;
    nd_parent[n] = -1;
    nd_item[n] = -1;
    nd_h[n] = h;
    nd_value[n] = base[h];
  }
}

// first item index after node n, and the end of the items with value - delta >= t
__device__ __forceinline__ void ext_range(int n, const int32_t* nd_item, const int32_t* nd_h, const float* nd_value,
                                          const int32_t* it_off, const float* it_delta, float t, int* lo_out,
                                          int* hi_out) {
  const float v = nd_value[n];
  const int h = nd_h[n];
  const int lo = nd_item[n] < 0 ? it_off[h] : nd_item[n] + 1;
  int a = lo, b = it_off[h + 1];
  if (!(v >= t)) b = lo;
  // largest prefix of [lo, b) with v - delta >= t (monotone in delta): probes at lo + 2^k - 1
  // first, since near the threshold the prefix is short, then bisection of the last gap
  for (int step = 1; a < b; step <<= 1) {
    const int m = min(a + step - 1, b - 1);
    if (v - it_delta[m] >= t) {
      a = m + 1;
    } else {
      b = m;
      break;
    }
  }
  while (a < b) {
    const int m = (a + b) >> 1;
    if (v - it_delta[m] >= t) a = m + 1;
    else b = m;
  }
  *lo_out = lo;
  *hi_out = a;
}

__global__ void k_count(int first, int nlev, const int32_t* nd_item, const int32_t* nd_h, const float* nd_value,
                        const int32_t* it_off, const float* it_delta, const float* t, int64_t* cnt) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= nlev) return;
  int lo, hi;
  ext_range(first + j, nd_item, nd_h, nd_value, it_off, it_delta, *t, &lo, &hi);
  cnt[j] = hi - lo;
}

// largest m with (sum of the first m counts) <= room; out = {m, that sum}
__global__ void k_cut(const int64_t* pre, const int64_t* cnt, int nlev, int64_t room, int32_t* out) {
  if (threadIdx.x != 0) return;
  int a = 0, b = nlev;  // predicate(m): pre[m-1] + cnt[m-1] <= room, monotone
  while (a < b) {
    const int m = (a + b + 1) >> 1;
    if (pre[m - 1] + cnt[m - 1] <= room) a = m;
    else b = m - 1;
  }
  out[0] = a;
  out[1] = a > 0 ? (int32_t)(pre[a - 1] + cnt[a - 1]) : 0;
}

__global__ void k_expand(int first, int m, int total, int out_base, const int64_t* pre, int32_t* nd_parent,
                         int32_t* nd_item, int32_t* nd_h, float* nd_value, uint64_t* nd_b, const int32_t* it_off,
                         const float* it_delta, const int32_t* it_group, const float* t) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int a = 0, b = m - 1;  // last j with pre[j] <= e
  while (a < b) {
    const int c = (a + b + 1) >> 1;
    if (pre[c] <= e) a = c;
    else b = c - 1;
  }
  const int n = first + a;
  int lo, hi;
  ext_range(n, nd_item, nd_h, nd_value, it_off, it_delta, *t, &lo, &hi);
  const int q = lo + (int)(e - pre[a]);
  float v = nd_value[n] - it_delta[q];
  const int g = it_group[q];
  const uint64_t pb = nd_b[n], gb = group_bit(g);
  if (pb & gb)
    for (int x = n; nd_item[x] >= 0; x = nd_parent[x])
      if (it_group[nd_item[x]] == g) {
        // two picks in one group: not a child.  NaN fails every `value >= t` test, so such a
        // node is never extended nor kept, even while t is still -inf.
        v = __uint_as_float(0xffc00000u);
        break;
      }
  const int o = out_base + e;
  nd_b[o] = pb | gb;
  nd_parent[o] = n;
  nd_item[o] = q;
  nd_h[o] = nd_h[n];
  nd_value[o] = v;
}

__global__ void k_keep_flags(const float* nd_value, int n, const float* t, int32_t* flags) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) flags[i] = nd_value[i] >= *t ? 1 : 0;
}

__global__ void k_compact_nodes(int n, const float* t, const int32_t* pre, const int32_t* p0, const int32_t* i0,
                                const int32_t* h0, const float* v0, const uint64_t* b0, int32_t* p1, int32_t* i1,
                                int32_t* h1, float* v1, uint64_t* b1) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n || !(v0[i] >= *t)) return;
  const int d = pre[i];
  b1[d] = b0[i];
  p1[d] = p0[i] >= 0 ? pre[p0[i]] : -1;
  i1[d] = i0[i];
  h1[d] = h0[i];
  v1[d] = v0[i];
}

// remapped positions of the given node indices (index == n maps to the kept total)
__global__ void k_remap_pos(const int32_t* pre, const int32_t* total, int n, int a, int b, int c, int32_t* out) {
  if (threadIdx.x != 0) return;
  const int xs[3] = {a, b, c};
  for (int j = 0; j < 3; ++j) out[j] = xs[j] >= n ? *total : pre[xs[j]];
}

__global__ void k_final_keys(int nc, const uint32_t* byh_vals, const float* nd_value, uint64_t* keys, uint32_t* vals) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= nc) return;
  const uint32_t node = byh_vals[p];
  keys[p] = ((uint64_t)(~f2o(nd_value[node])) << 32) | (uint32_t)p;  // value desc, key rank asc
  vals[p] = node;
}

__global__ void k_take(int n, const uint64_t* keys, const uint32_t* vals, const float* nd_value, int32_t* sel_node,
                       float* sel_val, int32_t* sel_rank) {
  const int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  sel_node[j] = (int32_t)vals[j];
  sel_val[j] = nd_value[vals[j]];
  sel_rank[j] = (int32_t)(keys[j] & 0xffffffffu);
}

// ---------------------------------------------------------------- single-workgroup search
// The same level-synchronous search in one 1024-thread workgroup: no host round trip per
// level.  Used first; if the node store would overflow it reports it and the multi-kernel
// search below (with compaction) takes over.
constexpr int kSB = 1024;
constexpr int kBlockNodes = 1 << 18;  // node budget of the one-workgroup search
constexpr int kSearchLdsItems = 24576;  // item deltas kept in LDS (the 160 KB of a CDNA4 workgroup)
constexpr int kSmallItems = 1024;       // items whose group tables are kept in LDS too (one per thread)

// end of the largest prefix of items [lo, b) with v - delta >= t (monotone in delta): probes at
// lo + 2^k - 1 first, since near the threshold the prefix is short, then bisection of the gap
__device__ __forceinline__ int ext_end(int lo, int b, float v, const float* it_delta, float t) {
  int a = lo;
  for (int step = 1; a < b; step <<= 1) {
    const int m = min(a + step - 1, b - 1);
    if (v - it_delta[m] >= t) {
      a = m + 1;
    } else {
      b = m;
      break;
    }
  }
  while (a < b) {
    const int m = (a + b) >> 1;
    if (v - it_delta[m] >= t) a = m + 1;
    else b = m;
  }
  return a;
}

__device__ __forceinline__ int64_t sb_excl_scan(int64_t v, int64_t* sh, int64_t* total) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  int64_t x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  __syncthreads();  // sh may still be read from the previous call
  if (lane == kWave - 1) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    int64_t run = 0;
    for (int i = 0; i < kSB / kWave; ++i) {
      const int64_t t = sh[i];
      sh[i] = run;
      run += t;
    }
    sh[32] = run;
  }
  __syncthreads();
  *total = sh[32];
  return x - v + sh[w];
}

// lower edge of the 24-bit orderable bin holding the K-th largest of v[0..n) (-inf if n < K)
__device__ float sb_bound(const float* v, int n, int K, int32_t* hist, int64_t* sh, int64_t* sel) {
  if (n < K) return -INFINITY;
  uint32_t prefix = 0, bin2 = 0;
  int64_t need_k = K;
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = threadIdx.x; j < 4096; j += kSB) hist[j] = 0;
    __syncthreads();
    for (int i0 = 0; i0 < n; i0 += kSB) {
      const int i = i0 + (int)threadIdx.x;
      bool act = false;
      uint32_t bin = 0;
      if (i < n) {
        const uint32_t o = f2o(v[i]);
        if (pass == 0) {
          act = true;
          bin = o >> 20;
        } else if ((o >> 20) == prefix) {
          act = true;
          bin = (o >> 8) & 4095;
        }
      }
      // The values of a search cluster in few bins, and same-address LDS atomics serialise: the
      // lanes that share the bin of the first pending lane add once, for a few rounds; the lanes
      // left then add one each.
      uint64_t pend = __ballot(act);
      for (int r = 0; r < 4 && pend != 0ull; ++r) {
        const int lead = __ffsll((unsigned long long)pend) - 1;
        const uint32_t b = (uint32_t)__shfl((int)bin, lead, kWave);
        const bool mine = act && bin == b;
        const uint64_t same = __ballot(mine);
        if (lane_id() == lead) atomicAdd(&hist[b], (int)__popcll(same));
        if (mine) act = false;
        pend &= ~same;
      }
      if (act) atomicAdd(&hist[bin], 1);
    }
    __syncthreads();
    const int t = threadIdx.x;  // owns bins 4t .. 4t+3
    const int64_t mine = (int64_t)hist[4 * t] + hist[4 * t + 1] + hist[4 * t + 2] + hist[4 * t + 3];
    int64_t tot;
    const int64_t excl = sb_excl_scan(mine, sh, &tot);
    const int64_t above = tot - excl - mine;  // count in bins above this thread's
    if (above < need_k && above + mine >= need_k) {
      int64_t acc = above;
      int b = 4 * t + 3;
      for (; b > 4 * t; --b) {
        if (acc + hist[b] >= need_k) break;
        acc += hist[b];
      }
      sel[0] = b;
      sel[1] = need_k - acc;
    }
    __syncthreads();
    if (pass == 0) {
      prefix = (uint32_t)sel[0];
      need_k = sel[1];
    } else {
      bin2 = (uint32_t)sel[0];
    }
    __syncthreads();
  }
  const float e = o2f((prefix << 20) | (bin2 << 8));
  return e == e ? e : -INFINITY;
}

__global__ __launch_bounds__(kSB) void k_select_block(int P, const float* base, const int32_t* it_off,
                                                      const float* it_delta, const int32_t* it_group, int K,
                                                      const float* t0, int cap, int32_t* nd_p, int32_t* nd_i,
                                                      int32_t* nd_h, float* nd_v, uint64_t* nd_b, float* t_out,
                                                      int32_t* out, int32_t* cand, int gmax) {
  __shared__ int64_t sh[40];
  __shared__ int32_t hist[4096];
  __shared__ int64_t sel[4];
  __shared__ int64_t cpre[kSB];
  __shared__ int64_t ccnt[kSB];
  __shared__ int32_t clo[kSB];
  __shared__ float cv[kSB];       // value, parent and group bits of the chunk's nodes
  __shared__ int32_t chh[kSB];
  __shared__ uint64_t cbb[kSB];
  __shared__ int32_t cnn[kSB];    // node index of the chunk's nodes
  __shared__ __align__(16) float ldel[kSearchLdsItems];  // the item deltas, when they fit
  __shared__ int32_t s_ng;
  const int nitem = it_off[P];
  const float* idel = it_delta;
  if (nitem <= kSearchLdsItems) {
    for (int q = threadIdx.x; q < nitem; q += kSB) ldel[q] = it_delta[q];
    idel = ldel;
  }
  // Up to kSmallItems items also keep, behind their deltas in the same LDS array: their group
  // (lg), the bit of their group (ibit) and the end of their parent's item list (iend, set for
  // the items of the roots the first level expands).  The bit is exact when the items carry at
  // most 64 distinct groups (gm = 2: a set bit proves the group picked, so no walk up a node's
  // picks is needed), else the hashed bit of group_bit (gm = 1).  Distinct groups get their
  // numbers through a hash table in hist (keys in its first half, numbers in its second).
  static_assert(5 * kSmallItems <= kSearchLdsItems, "item tables exceed the delta array");
  int32_t* lg = (int32_t*)(ldel + kSmallItems);
  uint64_t* ibit = (uint64_t*)(ldel + 2 * kSmallItems);
  int32_t* iend = (int32_t*)(ldel + 4 * kSmallItems);
  int gm = 0;
  if (nitem <= kSmallItems && gmax > 0) {
    constexpr int32_t kEmpty = (int32_t)0x80000000;  // groups are indices (>= 0)
    for (int j = threadIdx.x; j < 2048; j += kSB) hist[j] = kEmpty;
    if (threadIdx.x == 0) s_ng = 0;
    __syncthreads();
    const int q = threadIdx.x;
    int slot = 0, g = 0;
    if (q < nitem) {
      g = it_group[q];
      lg[q] = g;
      // at most kSmallItems (1024) keys in 2048 slots: an empty or matching slot is always found
      int sl = (int)(((uint32_t)g * 0x9E3779B1u) >> 21);
      for (;;) {
        const int prev = atomicCAS(&hist[sl], kEmpty, g);
        if (prev == kEmpty) {
          hist[2048 + sl] = atomicAdd(&s_ng, 1);
          break;
        }
        if (prev == g) break;
        sl = (sl + 1) & 2047;
      }
      slot = sl;
    }
    __syncthreads();
    gm = s_ng <= 64 && gmax == 2 ? 2 : 1;
    if (q < nitem) ibit[q] = gm == 2 ? 1ull << hist[2048 + slot] : group_bit(g);
  }
  __syncthreads();
  const float nan = __uint_as_float(0xffc00000u);
  float t = *t0;
  int status = 0;  // 0 done, 1 node store full, 2 too deep
  int used = 0;
  // roots, in parent rank order; the roots with an extension above t (the items with
  // v - delta >= t are a prefix of the parent's list) are listed in cand, in the same order, so
  // that the first level looks at those only.  One scan counts both: roots in the low half of
  // the 64-bit value, listed roots in the high half.
  // Each thread takes one contiguous range of parents: it counts them, one scan places them,
  // and a second sweep writes them.
  // Ordered compaction of the roots without a scan per 1024 parents: wave w takes the parents
  // [w*span, (w+1)*span), reads them kWave at a time (kRootBatch loads in flight), counts its roots
  // and listed roots with ballots; the waves' counts give each wave its first positions, and a
  // second sweep writes the roots there, in order (consecutive lanes write consecutive nodes).
  constexpr int kRootBatch = 8;
  constexpr int kWaves = kSB / kWave;
  int nx = 0;
  {
    const int w = threadIdx.x / kWave, lane = lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;  // lanes below this one
    const int span = ((P + kWaves - 1) / kWaves + kWave - 1) / kWave * kWave;
    const int a = min(P, w * span), b = min(P, a + span);
    float bv[kRootBatch];
    int bo0[kRootBatch], bo1[kRootBatch];
    // parent i = i0 + u*kWave + lane of the batch at i0: root (bit 0), listed (bit 1)
    auto load = [&](int i0) {
#pragma unroll
      for (int u = 0; u < kRootBatch; ++u) {
        const int i = i0 + u * kWave + lane;
        const bool in = i < b;
        bv[u] = in ? base[i] : 0.f;
        bo0[u] = in ? it_off[i] : 0;
        bo1[u] = in ? it_off[i + 1] : 0;  // it_off has P + 1 entries
      }
    };
    auto flags = [&](int i0, int u) {
      const int i = i0 + u * kWave + lane;
      if (!(i < b && bv[u] >= t)) return 0;
      return 1 | (bo0[u] < bo1[u] && bv[u] - idel[bo0[u]] >= t ? 2 : 0);
    };
    int cf = 0, cx = 0;
    for (int i0 = a; i0 < b; i0 += kRootBatch * kWave) {
      load(i0);
#pragma unroll
      for (int u = 0; u < kRootBatch; ++u) {
        const int fl = flags(i0, u);
        cf += __popcll(__ballot(fl & 1));
        cx += __popcll(__ballot((fl >> 1) & 1));
      }
    }
    int32_t* ws = clo;  // per-wave counts (clo is free until the levels)
    if (lane == 0) {
      ws[w] = cf;
      ws[kWaves + w] = cx;
    }
    __syncthreads();
    int of = 0, ox = 0, tf = 0, tx = 0;
    for (int j = 0; j < kWaves; ++j) {
      const int u = ws[j], v = ws[kWaves + j];
      if (j < w) {
        of += u;
        ox += v;
      }
      tf += u;
      tx += v;
    }
    if (tf > cap) {
      status = 1;
    } else {
      for (int i0 = a; i0 < b; i0 += kRootBatch * kWave) {
        load(i0);
#pragma unroll
        for (int u = 0; u < kRootBatch; ++u) {
          const int fl = flags(i0, u);
          const uint64_t bf = __ballot(fl & 1), bx = __ballot((fl >> 1) & 1);
          if (fl & 1) {
            const int n = of + (int)__popcll(bf & lt);
            nd_p[n] = -1;
            nd_i[n] = -1;
            nd_h[n] = i0 + u * kWave + lane;
            nd_v[n] = bv[u];
            nd_b[n] = 0ull;
            if (fl & 2) {
              cand[ox + (int)__popcll(bx & lt)] = n;
              if (gm)
                for (int q = bo0[u]; q < bo1[u]; ++q) iend[q] = bo1[u];
            }
          }
          of += (int)__popcll(bf);
          ox += (int)__popcll(bx);
        }
      }
      used = tf;
      nx = tx;
    }
  }
  __syncthreads();  // the roots, the list and iend are read by other threads below
  // no root has a child above t: the candidates are the roots, in order
  const bool roots_only = status == 0 && nx == 0;
  // a level expands the nodes [first, end), through the list lst when it is set (the first level)
  const int32_t* lst = cand;
  int first = 0, end = roots_only ? 0 : nx, levels = roots_only ? 1 : 0, last_raise = used;
  while (status == 0 && first < end) {
    if (++levels > kMaxDepth + 1) {
      status = 2;
      break;
    }
    const int level_start = used;  // the nodes this level writes start here
    int c0 = first;
    while (c0 < end) {
      const int nchunk = min(kSB, end - c0);
      int lo = 0, hi = 0;
      if ((int)threadIdx.x < nchunk) {
        const int n = lst ? lst[c0 + threadIdx.x] : c0 + (int)threadIdx.x;
        const int ni = nd_i[n], h = nd_h[n];
        const float v = nd_v[n];
        // the items after the node's last pick, to the end of its parent's list
        if (ni < 0) {
          lo = it_off[h];
          hi = it_off[h + 1];
        } else {
          lo = ni + 1;
          hi = gm ? iend[ni] : it_off[h + 1];
        }
        hi = v >= t ? ext_end(lo, hi, v, idel, t) : lo;
        cv[threadIdx.x] = v;
        chh[threadIdx.x] = h;
        cbb[threadIdx.x] = nd_b[n];
        cnn[threadIdx.x] = n;
      }
      const int64_t cnt = hi - lo;
      int64_t tot;
      const int64_t excl = sb_excl_scan(cnt, sh, &tot);
      cpre[threadIdx.x] = excl;
      ccnt[threadIdx.x] = cnt;
      clo[threadIdx.x] = lo;
      if (threadIdx.x == 0) sel[2] = 0;
      __syncthreads();
      // Expand a prefix of the chunk whose extensions fit a soft room of about the store's
      // current size (at least 2K), so that the threshold is raised (below) before the store
      // grows much further; the hard room is what the store can still hold.
      const int64_t hard = (int64_t)cap - used;
      const int64_t soft = min(hard, max(2 * (int64_t)K, (int64_t)used));
      int take = nchunk;
      int64_t te = tot;
      if (tot > soft) {
        if ((int)threadIdx.x < nchunk && excl + cnt <= soft)
          atomicMax((unsigned long long*)&sel[2], (unsigned long long)(threadIdx.x + 1));
        __syncthreads();
        take = (int)sel[2];
        if (take == 0 && used >= K && used > last_raise) {
          const float b = sb_bound(nd_v, used, K, hist, sh, sel);
          last_raise = used;
          if (b > t) {
            t = b;  // recount this chunk under the raised threshold
            continue;
          }
        }
        if (take == 0 && soft < hard) {
          __syncthreads();
          if (threadIdx.x == 0) sel[2] = 0;
          __syncthreads();
          if ((int)threadIdx.x < nchunk && excl + cnt <= hard)
            atomicMax((unsigned long long*)&sel[2], (unsigned long long)(threadIdx.x + 1));
          __syncthreads();
          take = (int)sel[2];
        }
        if (take == 0) {
          status = 1;
          break;
        }
        te = cpre[take - 1] + ccnt[take - 1];
      }
      for (int64_t e = threadIdx.x; e < te; e += kSB) {
        int a = 0, b = take - 1;  // last node with cpre <= e
        while (a < b) {
          const int m = (a + b + 1) >> 1;
          if (cpre[m] <= e) a = m;
          else b = m - 1;
        }
        const int nn = cnn[a];
        const int q = clo[a] + (int)(e - cpre[a]);
        float v = cv[a] - idel[q];
        const int g = gm ? lg[q] : it_group[q];
        const uint64_t pb = cbb[a], gb = gm ? ibit[q] : group_bit(g);
        if (pb & gb) {
          if (gm == 2) {
            v = nan;  // exact bits: the group is picked already, so not a child
          } else {
            for (int x = nn; nd_i[x] >= 0; x = nd_p[x]) {
              const int ix = nd_i[x];
              if ((gm ? lg[ix] : it_group[ix]) == g) {
                v = nan;  // two picks in one group: not a child
                break;
              }
            }
          }
        }
        const int o = used + (int)e;
        nd_b[o] = pb | gb;
        nd_p[o] = nn;
        nd_i[o] = q;
        nd_h[o] = chh[a];
        nd_v[o] = v;
      }
      __syncthreads();
      used += (int)te;
      c0 += take;
      // raise the threshold whenever the store has doubled since the last raise: the rest of
      // the level is then expanded under the higher threshold
      if (used >= K && used >= 2 * last_raise) {
        const float b = sb_bound(nd_v, used, K, hist, sh, sel);
        if (b > t) t = b;
        last_raise = used;
      }
    }
    if (status != 0) break;
    first = level_start;
    end = used;
    lst = nullptr;
    // at a level's end once the store has grown by a quarter since the last raise (each raise
    // reads every node twice)
    if (first < end && used >= K && used >= last_raise + last_raise / 4) {
      const float b = sb_bound(nd_v, used, K, hist, sh, sel);
      if (b > t) t = b;
      last_raise = used;
    }
  }
  // candidates: every node >= t, in enumeration order, and the range of their value keys
  __shared__ uint32_t vlo, vhi;
  if (threadIdx.x == 0) {
    vlo = 0xffffffffu;
    vhi = 0u;
  }
  int nc = 0;
  uint32_t mlo = 0xffffffffu, mhi = 0u;
  if (roots_only) {
    for (int n = threadIdx.x; n < used; n += kSB) {
      cand[n] = n;
      const uint32_t o = f2o(nd_v[n]);
      mlo = min(mlo, o);
      mhi = max(mhi, o);
    }
    nc = used;
  } else if (status == 0) {
    // the same ordered compaction as the roots': per-wave ranges, ballots, coalesced writes
    const int w = threadIdx.x / kWave, lane = lane_id();
    const uint64_t lt = (1ull << lane) - 1ull;
    const int span = ((used + kWaves - 1) / kWaves + kWave - 1) / kWave * kWave;
    const int a = min(used, w * span), b = min(used, a + span);
    float bv[kRootBatch];
    auto load = [&](int i0) {
#pragma unroll
      for (int u = 0; u < kRootBatch; ++u) {
        const int i = i0 + u * kWave + lane;
        bv[u] = i < b ? nd_v[i] : nan;
      }
    };
    int cf = 0;
    for (int i0 = a; i0 < b; i0 += kRootBatch * kWave) {
      load(i0);
#pragma unroll
      for (int u = 0; u < kRootBatch; ++u) cf += __popcll(__ballot(bv[u] >= t));
    }
    __syncthreads();  // clo is no longer read by the levels
    if (lane == 0) clo[w] = cf;
    __syncthreads();
    int of = 0;
    for (int j = 0; j < kWaves; ++j) {
      const int u = clo[j];
      if (j < w) of += u;
      nc += u;
    }
    for (int i0 = a; i0 < b; i0 += kRootBatch * kWave) {
      load(i0);
#pragma unroll
      for (int u = 0; u < kRootBatch; ++u) {
        const bool f = bv[u] >= t;
        const uint64_t bf = __ballot(f);
        if (f) {
          cand[of + (int)__popcll(bf & lt)] = i0 + u * kWave + lane;
          const uint32_t k = f2o(bv[u]);
          mlo = min(mlo, k);
          mhi = max(mhi, k);
        }
        of += (int)__popcll(bf);
      }
    }
  }
  for (int d = kWave / 2; d > 0; d >>= 1) {
    mlo = min(mlo, (uint32_t)__shfl_xor((int)mlo, d, kWave));
    mhi = max(mhi, (uint32_t)__shfl_xor((int)mhi, d, kWave));
  }
  __syncthreads();
  if (lane_id() == 0) {
    atomicMin(&vlo, mlo);
    atomicMax(&vhi, mhi);
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = used;
    out[1] = levels;
    out[2] = status;
    out[3] = nc;
    out[4] = (int32_t)(vlo ^ vhi);  // the value-key bits that vary among the candidates
    *t_out = t;
  }
}

// candidate list of the whole-GPU searches: nodes >= t in enumeration order
__global__ void k_cand_list(int n, const float* t, const int32_t* pre, const float* nd_value, int32_t* cand) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n && nd_value[i] >= *t) cand[pre[i]] = i;
}
__global__ void k_cand_keys(int nc, const int32_t* cand, const int32_t* nd_h, uint64_t* keys, uint32_t* vals) {
  const int d = blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= nc) return;
  keys[d] = (uint64_t)(uint32_t)nd_h[cand[d]];
  vals[d] = (uint32_t)cand[d];
}

// ---------------------------------------------------------------- cooperative search
// The same level-synchronous search as one cooperative launch on the whole GPU: every
// workgroup runs the same loop, the phases (count, scan, expand, threshold raise, compaction)
// are separated by grid-wide barriers, and every control decision is computed identically by
// all workgroups from values in global memory written before the last barrier, so the
// barriers are always reached by every workgroup the same number of times.
constexpr int kCB = 256;          // threads per workgroup
constexpr int kChunk = 1 << 16;   // nodes of a level counted at once at most
constexpr int kCoopGrid = 16;     // workgroups: the phases are short, so grid barriers dominate

struct CoopArgs {
  int P;
  const float* base;
  const int32_t* it_off;
  const float* it_delta;
  const int32_t* it_group;
  int K;
  const float* t0;
  int cap;
  int32_t* np[2];
  int32_t* ni[2];
  int32_t* nh[2];
  float* nv[2];
  uint64_t* nb[2];
  int32_t* cnt;     // [kChunk] extension counts of the chunk's nodes
  int64_t* pre;     // [kChunk] their exclusive prefix
  int32_t* map;     // [cap] compaction: kept nodes before each node
  int64_t* part;    // [gridDim.x] per-workgroup partial sums
  int32_t* hist;    // [2][4096] K-th value histograms (zero on entry, zero on exit)
  int32_t* out;     // used, levels, status, which, nodes created
  float* t_out;
};

namespace {
namespace cg = cooperative_groups;

__device__ __forceinline__ void grid_barrier() {
  __threadfence();
  cg::this_grid().sync();
}

// exclusive scan of one value per thread of the workgroup (kCB threads); total in *tot
__device__ __forceinline__ int64_t cb_excl_scan(int64_t v, int64_t* lds, int64_t* tot) {
  const int lane = lane_id(), w = threadIdx.x / kWave;
  int64_t x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  __syncthreads();
  if (lane == kWave - 1) lds[w] = x;
  __syncthreads();
  int64_t before = 0, all = 0;
  for (int j = 0; j < kCB / kWave; ++j) {
    const int64_t y = lds[j];
    if (j < w) before += y;
    all += y;
  }
  *tot = all;
  return x - v + before;
}

__device__ __forceinline__ int64_t cb_sum(int64_t v, int64_t* lds) {
  int64_t tot;
  (void)cb_excl_scan(v, lds, &tot);
  return tot;
}

// exclusive scan over the grid of f(0..n-1): out(i, prefix) for every i; returns the total
// (in every thread).  Each workgroup scans one contiguous range.  The caller places a grid
// barrier before the outputs are read.
template <class F, class O>
__device__ int64_t grid_scan(int n, F f, O out, int64_t* part, int64_t* lds) {
  const int G = gridDim.x, b = blockIdx.x;
  const int per = (n + G - 1) / G;
  const int lo = min(n, b * per), hi = min(n, lo + per);
  int64_t s = 0;
  for (int i = lo + (int)threadIdx.x; i < hi; i += kCB) s += f(i);
  s = cb_sum(s, lds);
  if (threadIdx.x == 0) part[b] = s;
  grid_barrier();
  int64_t off = 0, tot = 0;
  for (int j = threadIdx.x; j < G; j += kCB) {
    const int64_t v = part[j];
    tot += v;
    if (j < b) off += v;
  }
  off = cb_sum(off, lds);
  tot = cb_sum(tot, lds);
  int64_t carry = off;
  for (int base = lo; base < hi; base += kCB) {
    const int i = base + (int)threadIdx.x;
    const int64_t v = i < hi ? f(i) : 0;
    int64_t t;
    const int64_t ex = cb_excl_scan(v, lds, &t);
    if (i < hi) out(i, carry + ex);
    carry += t;
  }
  return tot;
}

// bin (from the top) holding the K-th largest count of a 4096-bin histogram in global memory;
// every workgroup computes the same result.  *need_k: in the rank, out the rank in the bin.
__device__ int pick_bin(const int32_t* hist, int64_t* need_k, int64_t* lds, int32_t* sel) {
  constexpr int per = 4096 / kCB;
  const int t = threadIdx.x;
  int64_t mine = 0;
  for (int j = 0; j < per; ++j) mine += hist[per * t + j];
  int64_t tot;
  const int64_t excl = cb_excl_scan(mine, lds, &tot);
  const int64_t above = tot - excl - mine;
  if (t == 0) sel[0] = -1;
  __syncthreads();
  const int64_t K = *need_k;
  if (above < K && above + mine >= K) {
    int64_t acc = above;
    int bb = per * t + per - 1;
    for (; bb > per * t; --bb) {
      if (acc + hist[bb] >= K) break;
      acc += hist[bb];
    }
    sel[0] = bb;
    sel[1] = (int32_t)(K - acc);
  }
  __syncthreads();
  const int r = sel[0];
  if (r >= 0) *need_k = sel[1];
  __syncthreads();
  return r;
}

// lower edge of the 24-bit orderable bin holding the K-th largest of v[0..n) (-inf if n < K)
__device__ float grid_kth(const float* v, int n, int K, int32_t* hist, int32_t* lhist, int64_t* lds, int32_t* sel) {
  if (n < K) return -INFINITY;
  int64_t need = K;
  uint32_t prefix = 0;
  int bin2 = 0;
  for (int pass = 0; pass < 2; ++pass) {
    for (int j = threadIdx.x; j < 4096; j += kCB) lhist[j] = 0;
    __syncthreads();
    for (int i = blockIdx.x * kCB + threadIdx.x; i < n; i += gridDim.x * kCB) {
      const uint32_t o = f2o(v[i]);
      if (pass == 0) atomicAdd(&lhist[o >> 20], 1);
      else if ((o >> 20) == prefix) atomicAdd(&lhist[(o >> 8) & 4095], 1);
    }
    __syncthreads();
    int32_t* gh = hist + 4096 * pass;
    for (int j = threadIdx.x; j < 4096; j += kCB)
      if (lhist[j]) atomicAdd(&gh[j], lhist[j]);
    grid_barrier();
    const int b = pick_bin(gh, &need, lds, sel);
    if (b < 0) {
      bin2 = -1;
      break;
    }
    if (pass == 0) prefix = (uint32_t)b;
    else bin2 = b;
  }
  grid_barrier();  // every workgroup has read both histograms
  if (blockIdx.x == 0)
    for (int j = threadIdx.x; j < 2 * 4096; j += kCB) hist[j] = 0;
  if (bin2 < 0) return -INFINITY;
  const float e = o2f((prefix << 20) | ((uint32_t)bin2 << 8));
  return e == e ? e : -INFINITY;
}
}  // namespace

__global__ __launch_bounds__(kCB) void k_select_coop(CoopArgs a) {
  extern __shared__ int32_t smem[];
  int32_t* lhist = smem;                              // 4096
  int64_t* lds = (int64_t*)(smem + 4096);             // kCB / 64 partial sums
  int32_t* sel = smem + 4096 + 2 * (kCB / kWave);     // 2
  const float nan = __uint_as_float(0xffc00000u);
  float t = *a.t0;
  int which = 0, status = 0;
  // roots, in parent rank order
  int used;
  {
    int32_t *P0 = a.np[0], *I0 = a.ni[0], *H0 = a.nh[0];
    float* V0 = a.nv[0];
    uint64_t* B0 = a.nb[0];
    const float* base = a.base;
    used = (int)grid_scan(a.P, [&](int h) -> int64_t { return base[h] >= t ? 1 : 0; },
                          [&](int h, int64_t pos) {
                            if (base[h] >= t) {
                              P0[pos] = -1;
                              I0[pos] = -1;
                              H0[pos] = h;
                              V0[pos] = base[h];
                              B0[pos] = 0ull;
                            }
                          },
                          a.part, lds);
    grid_barrier();
  }
  int lfirst = 0, lend = used, cursor = 0, levels = 1, last_raise = used;

  // raise the threshold to the bin of the K-th largest node value; compact if it rose
  auto raise = [&]() {
    const float t2 = grid_kth(a.nv[which], used, a.K, a.hist, lhist, lds, sel);
    last_raise = used;
    if (!(t2 > t)) return;
    t = t2;
    const float* V = a.nv[which];
    int32_t* map = a.map;
    const int kept = (int)grid_scan(used, [&](int i) -> int64_t { return V[i] >= t ? 1 : 0; },
                                    [&](int i, int64_t pos) { map[i] = (int32_t)pos; }, a.part, lds);
    grid_barrier();
    const int o = which ^ 1;
    for (int i = blockIdx.x * kCB + threadIdx.x; i < used; i += gridDim.x * kCB) {
      if (!(V[i] >= t)) continue;
      const int d = map[i];
      const int p = a.np[which][i];
      a.np[o][d] = p >= 0 ? map[p] : -1;
      a.ni[o][d] = a.ni[which][i];
      a.nh[o][d] = a.nh[which][i];
      a.nv[o][d] = V[i];
      a.nb[o][d] = a.nb[which][i];
    }
    auto remap = [&](int x) { return x < used ? map[x] : kept; };
    lfirst = remap(lfirst);
    lend = remap(lend);
    cursor = remap(cursor);
    grid_barrier();
    which = o;
    used = kept;
    last_raise = kept;
  };

  // extension counts of the nodes [cbase, cend) under the current threshold, with their
  // exclusive prefix; valid until the threshold changes, so a level is counted once per raise
  int cbase = 0, cend = 0;
  int64_t created = used;
  for (;;) {
    if (cursor >= lend) {  // the level is complete
      lfirst = lend;
      lend = used;
      cursor = lfirst;
      cbase = cend = 0;
      if (lfirst >= lend) break;
      if (++levels > kMaxDepth + 1) {
        status = 2;
        break;
      }
      if (used >= a.K && used > last_raise) raise();
      continue;
    }
    const int32_t* NI = a.ni[which];
    const int32_t* NH = a.nh[which];
    const float* NV = a.nv[which];
    if (cursor < cbase || cursor >= cend) {
      const int nchunk = min(lend - cursor, kChunk);
      for (int j = blockIdx.x * kCB + threadIdx.x; j < nchunk; j += gridDim.x * kCB) {
        int lo, hi;
        ext_range(cursor + j, NI, NH, NV, a.it_off, a.it_delta, t, &lo, &hi);
        a.cnt[j] = hi - lo;
      }
      grid_barrier();
      const int32_t* cnt0 = a.cnt;
      int64_t* pre0 = a.pre;
      (void)grid_scan(nchunk, [&](int j) -> int64_t { return cnt0[j]; }, [&](int j, int64_t x) { pre0[j] = x; },
                      a.part, lds);
      grid_barrier();
      cbase = cursor;
      cend = cursor + nchunk;
    }
    const int off = cursor - cbase, avail = cend - cursor;
    const int32_t* cnt = a.cnt + off;
    const int64_t* pre = a.pre + off;
    const int64_t p0 = pre[0];
    // largest prefix of the counted nodes whose extensions fit the room (monotone)
    auto fit = [&](int64_t room) {
      int lo2 = 0, hi2 = avail;
      while (lo2 < hi2) {
        const int m = (lo2 + hi2 + 1) >> 1;
        if (pre[m - 1] + cnt[m - 1] - p0 <= room) lo2 = m;
        else hi2 = m - 1;
      }
      return lo2;
    };
    const int64_t hard = (int64_t)a.cap - used;
    const int64_t soft = min(hard, max(2 * (int64_t)a.K, (int64_t)used));
    int m = fit(soft);
    if (m == 0 && soft < hard) m = fit(hard);
    if (m == 0) {
      if (used >= a.K && used > last_raise) {
        raise();  // a higher threshold shrinks the counts
        cbase = cend = 0;
        continue;
      }
      status = 1;
      break;
    }
    const int64_t te = pre[m - 1] + cnt[m - 1] - p0;
    {
      int32_t *NP = a.np[which], *NIw = a.ni[which], *NHw = a.nh[which];
      float* NVw = a.nv[which];
      uint64_t* NB = a.nb[which];
      for (int64_t e = blockIdx.x * kCB + threadIdx.x; e < te; e += (int64_t)gridDim.x * kCB) {
        const int64_t ee = e + p0;
        int x0 = 0, x1 = m - 1;  // last node with pre <= ee
        while (x0 < x1) {
          const int c = (x0 + x1 + 1) >> 1;
          if (pre[c] <= ee) x0 = c;
          else x1 = c - 1;
        }
        const int nn = cursor + x0;
        const int lo = NIw[nn] < 0 ? a.it_off[NHw[nn]] : NIw[nn] + 1;
        const int q = lo + (int)(ee - pre[x0]);
        float v = NVw[nn] - a.it_delta[q];
        const int g = a.it_group[q];
        const uint64_t pb = NB[nn], gb = group_bit(g);
        if (pb & gb)
          for (int x = nn; NIw[x] >= 0; x = NP[x])
            if (a.it_group[NIw[x]] == g) {
              v = nan;  // two picks in one group: not a child
              break;
            }
        const int o = used + (int)e;
        NB[o] = pb | gb;
        NP[o] = nn;
        NIw[o] = q;
        NHw[o] = NHw[nn];
        NVw[o] = v;
      }
    }
    grid_barrier();
    used += (int)te;
    created += te;
    cursor += m;
    if (used >= a.K && used >= 2 * last_raise) {
      const float before = t;
      raise();
      if (t != before) cbase = cend = 0;
    }
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    a.out[0] = used;
    a.out[1] = levels;
    a.out[2] = status;
    a.out[3] = which;
    a.out[4] = (int32_t)min(created, (int64_t)INT32_MAX);
    *a.t_out = t;
  }
}

// ---------------------------------------------------------------- starting threshold
// The search writes every child above its running threshold, so its cost is set by how tight
// the starting bound is.  When the K best children are combinations of many near-zero
// deviations of a few parents, the K-th best root or single deviation (the caller's bound)
// lies far below the K-th best child, and the search would write many times K children on
// its way up.  A counting bound closes the gap without enumerating: with a bin width w, every
// delta is rounded up to a multiple of w, and each parent's valid pick sets (at most one item
// per group) are counted by total rounded cost with the multiple-choice knapsack recursion over
// its groups, counts saturating at K.  Rounding up only lowers a child's value and saturation
// or leaving items out only lowers a count, so if at least K counted children of all parents
// have rounded value >= v_max - j*w (v_max: the best parent), the K-th best child is at least
// v_max - j*w, less a margin for the float rounding of the sequential subtractions.  A first
// pass with coarse bins over the whole range [t0, v_max] counts each parent's smallest first
// deviations (one item per detection, read from the dense rows of the association step) and
// finds a range E, so that the items can be generated for that range only; a second pass
// with fine bins over [v_max - E, v_max] counts the items and sharpens the bound.
constexpr int kDpBins1 = 1024, kDpItems1 = 64;    // first pass
constexpr int kDpBins2 = 2048, kDpItems2 = 2048;  // second pass
constexpr int kDpThreads = 1024;      // init and pick
constexpr int kDpCountThreads = 1024;  // counting: one or a few bins per thread and step

constexpr int kDpGrid = 512;  // workgroups of a counting pass (each takes parents in turn)

struct DpState {
  float vmax, t0, tref;
  int32_t ok;       // the current pass runs (a previous one found its count)
  double E;         // range of the current pass below vmax
  int32_t refined;  // tref > t0
  int32_t nact;     // parents with base >= t0, listed in act (any order)
};

__global__ __launch_bounds__(kDpThreads) void k_dp_init(int P, const float* base, const float* t0, DpState* st,
                                                        int32_t* act) {
  __shared__ float red[kDpThreads / kWave];
  __shared__ int32_t nact;
  const float t = *t0;
  if (threadIdx.x == 0) nact = 0;
  __syncthreads();
  float m = -INFINITY;
  for (int h = threadIdx.x; h < P; h += kDpThreads) {
    const float b = base[h];
    if (b >= t) {
      act[atomicAdd(&nact, 1)] = h;
      if (b > m) m = b;
    }
  }
  for (int d = kWave / 2; d > 0; d >>= 1) m = fmaxf(m, __shfl_xor(m, d, kWave));
  if (lane_id() == 0) red[threadIdx.x / kWave] = m;
  __syncthreads();
  if (threadIdx.x == 0) {
    for (int w = 1; w < kDpThreads / kWave; ++w) m = fmaxf(m, red[w]);
    const double E = (double)m - (double)t;
    st->vmax = m;
    st->t0 = t;
    st->tref = t;
    st->E = E;
    st->ok = (m >= t && E < INFINITY) ? 1 : 0;
    st->refined = 0;
    st->nact = nact;
  }
}

// First pass.  Every workgroup takes listed parents in turn: the parent's smallest first
// deviations (dev1 of its detections, one item per detection) sorted in LDS, counted by
// rounded cost with the 0/1 knapsack recursion (two items per step), added into C at the
// parent's offset (its own rounded distance below vmax).
constexpr int kDpRowMax = 4096;  // detections of a row looked at (a subset only loosens the bound)
__global__ __launch_bounds__(kDpThreads) void k_dp_rows(const float* base, CellView cv, int M, int K,
                                                        const DpState* st, const int32_t* act,
                                                        unsigned long long* C) {
  __shared__ float sv[kDpRowMax];
  __shared__ int32_t fa[kDpBins1], fb[kDpBins1];
  __shared__ int32_t cst[kDpItems1];
  __shared__ int32_t ne_s;
  if (!st->ok) return;
  const int NB = kDpBins1;
  const double E = st->E, w = E / NB;
  const int nact = st->nact, Mr = min(M, kDpRowMax);
  int P2 = 1;
  while (P2 < Mr) P2 <<= 1;
  for (int k = blockIdx.x; k < nact; k += gridDim.x) {
    const int h = act[k];
    const double gap = (double)st->vmax - (double)base[h];
    const double dd = ceil(gap / w);
    if (!(dd < NB)) continue;
    const int dh = (int)dd;
    __syncthreads();  // the previous parent's arrays are no longer read
    if (threadIdx.x == 0) ne_s = 0;
    __syncthreads();
    // the row's first deviations, and how many lie within the range
    int mine = 0;
    for (int q = threadIdx.x; q < Mr; q += kDpThreads) {
      const float v = cv.dev1[cv.at(h, q)];
      sv[q] = v;
      mine += (double)v <= E - gap ? 1 : 0;
    }
    for (int b = threadIdx.x; b < NB; b += kDpThreads) fa[b] = b == 0 ? 1 : 0;
    if (mine) atomicAdd(&ne_s, mine);
    __syncthreads();
    const int nin = ne_s;
    __syncthreads();  // every thread has read the count before it is reused below
    if (nin <= kDpItems1) {
      // all of them are items: the counts of a 0/1 knapsack (saturated at K) do not depend on
      // the order of its items, so no sort is needed
      if (threadIdx.x == 0) ne_s = 0;
      __syncthreads();
      for (int q = threadIdx.x; q < Mr; q += kDpThreads) {
        const float v = sv[q];
        if ((double)v <= E - gap) {
          const double c = ceil((double)v / w);
          cst[atomicAdd(&ne_s, 1)] = c < NB ? (int)c : NB;
        }
      }
      __syncthreads();
    } else {
      // more than kDpItems1: the smallest kDpItems1 of them, by a bitonic sort of the row
      for (int q = Mr + threadIdx.x; q < P2; q += kDpThreads) sv[q] = INFINITY;
      __syncthreads();
      for (int kk = 2; kk <= P2; kk <<= 1)
        for (int j = kk >> 1; j > 0; j >>= 1) {
          for (int q = threadIdx.x; q < P2; q += kDpThreads) {
            const int r = q ^ j;
            if (r > q) {
              const float x = sv[q], y = sv[r];
              if ((x > y) == ((q & kk) == 0)) {
                sv[q] = y;
                sv[r] = x;
              }
            }
          }
          __syncthreads();
        }
      // the first deviations within the range (a prefix of the sorted ones), at most kDpItems1
      if (threadIdx.x < kWave) {
        const int q = threadIdx.x;
        const bool in = q < min(Mr, kDpItems1) && (double)sv[q] <= E - gap;
        const uint64_t bal = __ballot(in);
        if (in) {
          const double c = ceil((double)sv[q] / w);
          cst[q] = c < NB ? (int)c : NB;
        }
        if (q == 0) ne_s = __popcll(bal);
      }
      __syncthreads();
    }
    const int ne = ne_s;
    int32_t* f = fa;
    int32_t* g = fb;
    for (int q = 0; q < ne; q += 2) {
      const int c1 = cst[q], c2 = q + 1 < ne ? cst[q + 1] : NB;
      for (int b = threadIdx.x; b < NB; b += kDpThreads) {
        int v = f[b];
        if (c1 <= b) v = min(K, v + f[b - c1]);
        if (c2 <= b) {
          v = min(K, v + f[b - c2]);
          if (c1 + c2 <= b) v = min(K, v + f[b - c1 - c2]);
        }
        g[b] = v;
      }
      __syncthreads();
      int32_t* x = f;
      f = g;
      g = x;
    }
    for (int b = threadIdx.x; b < NB - dh; b += kDpThreads)
      if (f[b]) atomicAdd(&C[b + dh], (unsigned long long)f[b]);
  }
}

// Second pass.  Every workgroup takes listed parents in turn: the counts of the parent's valid
// pick sets of items by rounded cost, added into C at the parent's offset.
__global__ __launch_bounds__(kDpCountThreads) void k_dp_count(const float* base, const int32_t* it_off,
                                                         const float* it_delta, const int32_t* it_group, int K,
                                                         const DpState* st, const int32_t* act,
                                                         unsigned long long* C) {
  __shared__ uint64_t key[kDpItems2];
  __shared__ int32_t gs[kDpItems2 + 1];    // starts of the group runs
  __shared__ int32_t fa[kDpBins2], fb[kDpBins2];
  __shared__ int32_t wcnt[kDpCountThreads / kWave];
  __shared__ int32_t ne_s, ngs;
  if (!st->ok) return;
  const int NB = kDpBins2, ncap = kDpItems2;
  const double E = st->E, w = E / NB;
  const int nact = st->nact;
  for (int k = blockIdx.x; k < nact; k += gridDim.x) {
    const int h = act[k];
    const double gap = (double)st->vmax - (double)base[h];
    const double dd = ceil(gap / w);
    if (!(dd < NB)) continue;
    const int dh = (int)dd;
    const int a = it_off[h], n = it_off[h + 1] - a;
    __syncthreads();  // ne_s, key and fa of the previous parent are no longer read
    if (threadIdx.x == 0) {
      // items with delta <= E - gap can be picked within the range (the list is sorted by delta)
      const double Eh = E - gap;
      int lo = 0, hi = n;
      while (lo < hi) {
        const int m = (lo + hi) >> 1;
        if ((double)it_delta[a + m] <= Eh) lo = m + 1;
        else hi = m;
      }
      ne_s = min(lo, ncap);
      ngs = 0;
    }
    __syncthreads();
    const int ne = ne_s;
    if (ne == 0) {
      if (threadIdx.x == 0) atomicAdd(&C[dh], 1ull);
      continue;
    }
    // (group, rounded cost) of the items, sorted by group so that each group is one run
    int P2 = 1;
    while (P2 < ne) P2 <<= 1;
    for (int q = threadIdx.x; q < P2; q += kDpCountThreads) {
      if (q < ne) {
        const double c = ceil((double)it_delta[a + q] / w);
        const uint32_t cost = c < NB ? (uint32_t)c : (uint32_t)NB;
        key[q] = ((uint64_t)(uint32_t)it_group[a + q] << 32) | cost;
      } else {
        key[q] = ~0ull;
      }
    }
    for (int b = threadIdx.x; b < NB; b += kDpCountThreads) fa[b] = b == 0 ? 1 : 0;
    __syncthreads();
    for (int kk = 2; kk <= P2; kk <<= 1)
      for (int j = kk >> 1; j > 0; j >>= 1) {
        for (int q = threadIdx.x; q < P2; q += kDpCountThreads) {
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
    // starts of the group runs, in order (wave ballots, then the waves' counts)
    for (int c0 = 0; c0 < ne; c0 += kDpCountThreads) {
      const int q = c0 + (int)threadIdx.x;
      const bool st0 = q < ne && (q == 0 || (key[q] >> 32) != (key[q - 1] >> 32));
      const uint64_t bal = __ballot(st0);
      if (lane_id() == 0) wcnt[threadIdx.x / kWave] = __popcll(bal);
      __syncthreads();
      int before = ngs;
      for (int w2 = 0; w2 < (int)threadIdx.x / kWave; ++w2) before += wcnt[w2];
      if (st0) gs[before + __popcll(bal & lanemask_lt())] = q;
      __syncthreads();
      if (threadIdx.x == 0) {
        int tot = 0;
        for (int w2 = 0; w2 < kDpCountThreads / kWave; ++w2) tot += wcnt[w2];
        ngs += tot;
      }
      __syncthreads();
    }
    const int ng = ngs;
    if (threadIdx.x == 0) gs[ng] = ne;
    __syncthreads();
    // two groups per step: f'' = f * (1 + sum_i x^c_i) * (1 + sum_j x^c_j), counts saturating at K
    int32_t* f = fa;
    int32_t* g = fb;
    for (int k2 = 0; k2 < ng; k2 += 2) {
      const int a0 = gs[k2], a1 = gs[k2 + 1], a2 = k2 + 1 < ng ? gs[k2 + 2] : a1;
      for (int b = threadIdx.x; b < NB; b += kDpCountThreads) {
        int v = f[b];
        for (int i = a0; i < a1; ++i) {
          const int ci = (int)(uint32_t)key[i];
          if (ci > b) continue;
          v = min(K, v + f[b - ci]);
          for (int j = a1; j < a2; ++j) {
            const int cj = (int)(uint32_t)key[j];
            if (ci + cj <= b) v = min(K, v + f[b - ci - cj]);
          }
        }
        for (int j = a1; j < a2; ++j) {
          const int cj = (int)(uint32_t)key[j];
          if (cj <= b) v = min(K, v + f[b - cj]);
        }
        g[b] = v;
      }
      __syncthreads();
      int32_t* x = f;
      f = g;
      g = x;
    }
    for (int b = threadIdx.x; b < NB - dh; b += kDpCountThreads)
      if (f[b]) atomicAdd(&C[b + dh], (unsigned long long)f[b]);
  }
}

// first bin whose cumulative count reaches K; the bound it gives, and the next pass's range.
// Leaves C zeroed.
__global__ __launch_bounds__(kDpThreads) void k_dp_pick(int pass, int K, DpState* st, unsigned long long* C,
                                                        float inflate) {
  __shared__ unsigned long long part[kDpThreads];
  __shared__ int32_t first;
  const int NB = pass == 1 ? kDpBins1 : kDpBins2, per = NB / kDpThreads;
  if (!st->ok) return;
  const int t = threadIdx.x;
  unsigned long long mine = 0;
  for (int j = 0; j < per; ++j) mine += C[per * t + j];
  part[t] = mine;
  if (t == 0) first = NB;
  __syncthreads();
  // inclusive scan of the per-thread sums (Hillis-Steele in LDS)
  for (int d = 1; d < kDpThreads; d <<= 1) {
    const unsigned long long y = t >= d ? part[t - d] : 0ull;
    __syncthreads();
    part[t] += y;
    __syncthreads();
  }
  const unsigned long long before = part[t] - mine;
  if (before < (unsigned long long)K && part[t] >= (unsigned long long)K) {
    unsigned long long acc = before;
    int j = per * t;
    for (; j < per * t + per - 1; ++j) {
      acc += C[j];
      if (acc >= (unsigned long long)K) break;
    }
    first = j;
  }
  __syncthreads();
  for (int j = 0; j < per; ++j) C[per * t + j] = 0ull;
  if (t != 0) return;
  const int j = first;
  if (j >= NB) {  // not enough counted children in range: keep the bound found so far
    st->ok = 0;
    return;
  }
  const double w = st->E / NB;
  const double vmax = st->vmax;
  // rounding of up to kMaxDepth sequential float subtractions, and one bin
  const double tau = vmax - j * w - w - 1e-5 * fmax(1.0, fabs(vmax));
  float f = (float)tau;
  if ((double)f > tau) f = nextafterf(f, -INFINITY);
  if (f > st->tref) {
    st->tref = f;
    st->refined = 1;
  }
  if (pass == 1) {
    st->E = (j + 2) * w;  // the fine pass covers the coarse bin found and the next
    st->ok = j > 0 ? 1 : 0;
  }
  // diagnostic (0 < inflate < 1): a refined bound moved that part of the way up to the best
  // value, no longer a bound, so that the search keeps fewer than K children and the caller's
  // search again from its own bound is exercised
  if (inflate > 0.f && st->refined) st->tref = st->tref + inflate * (st->vmax - st->tref);
}

namespace {
struct Nodes {
  int32_t *p, *i, *h;
  float* v;
  uint64_t* b;
};
}  // namespace

// Workgroups of the cooperative search: one per compute unit when the device supports
// cooperative launches and that many fit at once (0: use the multi-kernel levels).
constexpr size_t kCoopLds = (4096 + 2 * (kCB / kWave) + 4) * sizeof(int32_t);
namespace {
std::atomic<int> g_coop_grid{-1};  // per process (one device type)
}
static int coop_grid(size_t lds) {
  const int known = g_coop_grid.load();
  if (known >= 0) return known;
  int dev = 0, ncu = 0, coop = 0, per = 0;
  g_coop_grid = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 0;
  if (hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, dev) != hipSuccess || !coop) return 0;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || ncu < 1) return 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)k_select_coop, kCB, lds) != hipSuccess ||
      per < 1)
    return 0;
  const int G = std::min(ncu, kCoopGrid);
  g_coop_grid = G;
  return G;
}
static void coop_disable() { g_coop_grid = 0; }

const float* dp_bound_rows(const float* base, int P, const CellView& cv, int M, int K, const float* t0,
                           SelectBufs& b, hipStream_t s) {
  DpState* st = need<DpState>(b.dp, 1);
  int32_t* act = need<int32_t>(b.dpa, std::max(P, 1));
  unsigned long long* C = need<unsigned long long>(b.dpc, kDpBins2);
  if (!b.dpc_ready) {
    GLMB_HIP(hipMemsetAsync(C, 0, kDpBins2 * sizeof(unsigned long long), s));  // k_dp_pick leaves it zeroed
    b.dpc_ready = true;
  }
  GLMB_LAUNCH(k_dp_init, 1, kDpThreads, 0, s, P, base, t0, st, act);
  if (K > 0 && P > 0 && M > 0) {
    GLMB_LAUNCH(k_dp_rows, std::min(P, kDpGrid), kDpThreads, 0, s, base, cv, M, K, (const DpState*)st,
                (const int32_t*)act, C);
    GLMB_LAUNCH(k_dp_pick, 1, kDpThreads, 0, s, 1, K, st, C, 0.f);
  }
  return &st->tref;
}

void dp_bound_items(const SelectIn& in, SelectBufs& b, hipStream_t s) {
  if (in.K <= 0 || in.P <= 0) return;
  DpState* st = b.dp.as<DpState>();
  unsigned long long* C = b.dpc.as<unsigned long long>();
  GLMB_LAUNCH(k_dp_count, std::min(in.P, kDpGrid), kDpCountThreads, 0, s, in.base, in.it_off, in.it_delta,
              in.it_group, in.K, (const DpState*)st, (const int32_t*)b.dpa.as<int32_t>(), C);
  GLMB_LAUNCH(k_dp_pick, 1, kDpThreads, 0, s, 2, in.K, st, C, in.dp_inflate);
}

bool dp_bound_refined(SelectBufs& b, hipStream_t s) {
  return read_back(b.hs, s, {{&b.dp.as<DpState>()->refined, 1}})[0] != 0;
}

void dp_bound_trace(SelectBufs& b, hipStream_t s) {
  DpState h{};
  GLMB_HIP(hipMemcpyAsync(&h, b.dp.p, sizeof(DpState), hipMemcpyDeviceToHost, s));
  GLMB_HIP(stream_sync(s));
  std::fprintf(stderr, "[glmb] select.refine t0 %.7g tref %.7g vmax %.7g refined %d\n", h.t0, h.tref, h.vmax,
               h.refined);
  std::fflush(stderr);
}

glmb_status select_topk(const SelectIn& in, int cap, SelectBufs& b, Selected& out, hipStream_t s, std::string& err,
                        bool trace) {
  auto tr = [&](const char* what, long long a, long long c) {
    if (trace) {
      std::fprintf(stderr, "[glmb] select.%s %lld %lld\n", what, a, c);
      std::fflush(stderr);
    }
  };
  const int T = 256;
  // node store: two copies for compaction
  auto alloc = [&](int which) {
    Nodes n;
    const int64_t c2 = 2 * (int64_t)cap;
    n.p = need<int32_t>(b.nd_parent, c2) + (which ? cap : 0);
    n.i = need<int32_t>(b.nd_item, c2) + (which ? cap : 0);
    n.h = need<int32_t>(b.nd_h, c2) + (which ? cap : 0);
    n.v = need<float>(b.nd_value, c2) + (which ? cap : 0);
    n.b = need<uint64_t>(b.nd_bloom, c2) + (which ? cap : 0);
    return n;
  };
  if (in.P > cap) {
    err = "selection: more parents than search nodes";
    return GLMB_E_CAPACITY;
  }
  Nodes A = alloc(0), B = alloc(1);
  int32_t* scal = need<int32_t>(b.scal, 32);   // [0]=total, [1..2]=cut, [4..6]=remap, [8..9] t, [16..20] coop,
                                               // [24..28] one-workgroup search
  float* t = (float*)(scal + 8);               // current threshold
  float* t2 = (float*)(scal + 9);
  // t is written by every search form (the one-workgroup and cooperative kernels at their end,
  // the host-driven levels from t0 before their roots)
  int32_t hs[8];
  auto read = [&](int n) { std::memcpy(hs, read_back(b.hs, s, {{scal, n}}), n * sizeof(int32_t)); };
  // Small searches run in one workgroup (no host round trip per level).  A search that
  // outgrows kBlockNodes continues on the whole GPU (multi-kernel levels below); the call
  // site remembers that and starts there next time, until a search is small again.
  int used = 0, levels = 0, nc_fast = 0;
  uint32_t vary = 0xffffffffu;  // value-key bits that differ among the candidates
  bool fast = false;
  if (!in.force_multi && !(in.prefer_multi && *in.prefer_multi)) {
    GLMB_LAUNCH(k_select_block, 1, kSB, 0, s, in.P, in.base, in.it_off, in.it_delta, in.it_group, in.K, in.t0,
                std::min(cap, kBlockNodes), A.p, A.i, A.h, A.v, A.b, t, scal + 24,
                need<int32_t>(b.cand, std::min(cap, kBlockNodes) + 1), in.group_bits);
    std::memcpy(hs, read_back(b.hs, s, {{scal + 24, 5}}), 5 * sizeof(int32_t));
    used = hs[0];
    levels = hs[1];
    fast = hs[2] == 0;
    nc_fast = hs[3];
    vary = (uint32_t)hs[4];
    tr("block", used, hs[2]);
    if (in.prefer_multi) *in.prefer_multi = !fast;
  }
  // On the whole GPU: one cooperative launch when the device supports it, else the
  // host-driven multi-kernel levels below.
  bool coop = false;
  if (!fast && in.allow_coop && !in.force_multi) {
    int G = coop_grid(kCoopLds);
    if (G > 0) {
      CoopArgs ca{};
      ca.P = in.P;
      ca.base = in.base;
      ca.it_off = in.it_off;
      ca.it_delta = in.it_delta;
      ca.it_group = in.it_group;
      ca.K = in.K;
      ca.t0 = in.t0;
      ca.cap = cap;
      const Nodes* nb2[2] = {&A, &B};
      for (int j = 0; j < 2; ++j) {
        ca.np[j] = nb2[j]->p;
        ca.ni[j] = nb2[j]->i;
        ca.nh[j] = nb2[j]->h;
        ca.nv[j] = nb2[j]->v;
        ca.nb[j] = nb2[j]->b;
      }
      ca.cnt = need<int32_t>(b.flags, std::max(kChunk, in.P) + 1);
      ca.pre = need<int64_t>(b.pre64, kChunk + 1);
      ca.map = need<int32_t>(b.map, (int64_t)cap + 1);
      ca.part = need<int64_t>(b.cnt, G + 1);
      if (!b.hist_ready) {
        int32_t* hz = need<int32_t>(b.hist, 2 * 4096);
        GLMB_HIP(hipMemsetAsync(hz, 0, 2 * 4096 * sizeof(int32_t), s));  // the kernel leaves it zeroed
        b.hist_ready = true;
      }
      ca.hist = b.hist.as<int32_t>();
      ca.out = scal + 16;
      ca.t_out = t;
      void* args[] = {&ca};
      const hipError_t e = hipLaunchCooperativeKernel((const void*)k_select_coop, dim3(G), dim3(kCB), args,
                                                      kCoopLds, s);
      if (e == hipSuccess) {
        std::memcpy(hs, read_back(b.hs, s, {{scal + 16, 5}}), 5 * sizeof(int32_t));
        used = hs[0];
        levels = hs[1];
        tr("coop", used, hs[4]);
        // a search that created few nodes fits one workgroup: try that first next time
        if (in.prefer_multi && !in.force_multi && hs[2] == 0 && hs[4] < kBlockNodes / 4) *in.prefer_multi = false;
        if (hs[2] == 1) {
          err = "selection: search node capacity exhausted (tie class at the cut larger than the node store?)";
          return GLMB_E_CAPACITY;
        }
        if (hs[2] == 2) {
          err = "selection: deeper than the supported number of deviations";
          return GLMB_E_CAPACITY;
        }
        if (hs[3]) std::swap(A, B);
        coop = true;
      } else {
        (void)hipGetLastError();  // not launchable here: the multi-kernel levels take over
        coop_disable();
      }
    }
  }
  if (!fast && !coop) {
    // roots
    GLMB_HIP(hipMemcpyAsync(t, in.t0, sizeof(float), hipMemcpyDeviceToDevice, s));
    int32_t* fl = need<int32_t>(b.flags, in.P + 1);
    int32_t* pre = need<int32_t>(b.pre, in.P + 1);
    GLMB_LAUNCH(k_root_flags, cdiv(in.P, T), T, 0, s, in.base, in.P, t, fl);
    scan_excl(fl, pre, in.P, scal, b.tmp, s);
    GLMB_LAUNCH(k_root_write, cdiv(in.P, T), T, 0, s, in.base, in.P, t, pre, A.p, A.i, A.h, A.v, A.b);
    read(1);
    used = hs[0];
    levels = 0;
  }
  int level_first = 0, level_end = (fast || coop) ? 0 : used;

  // raise t to a bound on the K-th largest node value and drop nodes below it
  auto raise_and_compact = [&](int* cursor) -> bool {
    if (used < in.K) return false;
    kth_bound(A.v, used, in.K, t2, b.tmp, s);
    // t = max(t, t2)
    float th[2];
    std::memcpy(th, read_back(b.hs, s, {{scal + 8, 2}}), sizeof(th));
    if (!(th[1] > th[0])) return false;
    GLMB_HIP(hipMemcpyAsync(t, t2, sizeof(float), hipMemcpyDeviceToDevice, s));
    int32_t* fl = need<int32_t>(b.flags, used + 1);
    int32_t* pre = need<int32_t>(b.pre, used + 1);
    GLMB_LAUNCH(k_keep_flags, cdiv(used, T), T, 0, s, A.v, used, t, fl);
    scan_excl(fl, pre, used, scal, b.tmp, s);
    GLMB_LAUNCH(k_compact_nodes, cdiv(used, T), T, 0, s, used, t, pre, A.p, A.i, A.h, A.v, A.b, B.p, B.i, B.h, B.v,
                B.b);
    GLMB_LAUNCH(k_remap_pos, 1, 64, 0, s, pre, scal, used, level_first, *cursor, level_end, scal + 4);
    read(8);
    used = hs[0];
    level_first = hs[4];
    *cursor = hs[5];
    level_end = hs[6];
    std::swap(A, B);
    return true;
  };

  int last_raise = used;  // node count after the last threshold raise
  int64_t created = used;  // nodes written by this search (compacted ones included)
  while (level_first < level_end) {
    ++levels;
    tr("level", levels, level_end - level_first);
    if (levels > kMaxDepth + 1) {
      err = "selection: deeper than the supported number of deviations";
      return GLMB_E_CAPACITY;
    }
    int cursor = level_first;
    while (cursor < level_end) {
      const int nlev = level_end - cursor;
      int64_t* cnt = need<int64_t>(b.cnt, nlev + 1);
      int64_t* pre = need<int64_t>(b.pre64, nlev + 1);
      int64_t* tot64 = (int64_t*)(scal + 12);
      GLMB_LAUNCH(k_count, cdiv(nlev, T), T, 0, s, cursor, nlev, A.i, A.h, A.v, in.it_off, in.it_delta, t, cnt);
      scan_excl64(cnt, pre, nlev, tot64, b.tmp, s);
      int64_t total = 0;
      std::memcpy(&total, read_back(b.hs, s, {{tot64, 2}}), sizeof(total));
      if (total == 0) break;
      // Expand at most about as many nodes as the store holds (at least 2K) before the
      // threshold is raised again: a raised threshold prunes the rest of the level.
      const int64_t hard_room = (int64_t)cap - used;
      const int64_t room = std::min(hard_room, std::max<int64_t>(2 * (int64_t)in.K, used));
      int m = nlev;
      int64_t te = total;
      auto cut = [&](int64_t r) {
        GLMB_LAUNCH(k_cut, 1, 64, 0, s, pre, cnt, nlev, r, scal + 1);
        read(3);
        m = hs[1];
        te = hs[2];
      };
      if (total > room) {
        if (used >= 2 * last_raise && raise_and_compact(&cursor)) {
          last_raise = used;
          continue;
        }
        cut(room);
        if (m == 0 && room < hard_room) cut(hard_room);
        if (m == 0 || used > cap / 2) {
          if (raise_and_compact(&cursor)) {
            last_raise = used;
            continue;
          }
          if (m == 0) {
            err = "selection: search node capacity exhausted (tie class at the cut larger than the node store?)";
            return GLMB_E_CAPACITY;
          }
        }
      }
      GLMB_LAUNCH(k_expand, cdiv(te, T), T, 0, s, cursor, m, (int)te, used, pre, A.p, A.i, A.h, A.v, A.b, in.it_off,
                  in.it_delta, in.it_group, t);
      used += (int)te;
      created += te;
      cursor += m;
    }
    const int next_first = level_end, next_end = used;
    level_first = next_first;
    level_end = next_end;
    if (level_first < level_end) {
      int c = level_first;
      if (raise_and_compact(&c)) last_raise = used;
    }
  }
  if (!fast && !coop && in.prefer_multi && !in.force_multi && created < kBlockNodes / 4) *in.prefer_multi = false;
  tr("final", used, levels);
  tr("created", created, fast ? 1 : 0);
  // candidates: every node >= t, in enumeration order
  int nc = nc_fast;
  if (!fast) {
    int32_t* fl = need<int32_t>(b.flags, used + 1);
    int32_t* pre = need<int32_t>(b.pre, used + 1);
    GLMB_LAUNCH(k_keep_flags, cdiv(used, T), T, 0, s, A.v, used, t, fl);
    scan_excl(fl, pre, used, scal, b.tmp, s);
    read(1);
    nc = hs[0];
    GLMB_LAUNCH(k_cand_list, cdiv(used, T), T, 0, s, used, t, pre, A.v, need<int32_t>(b.cand, nc + 1));
  }
  const int32_t* cand = b.cand.as<int32_t>();
  int hbits = 0;
  while ((1 << hbits) < in.P) ++hbits;
  const int n = std::min(nc, in.K);
  out.node = need<int32_t>(b.sel_node, n + 1);
  out.value = need<float>(b.sel_val, n + 1);
  out.keyrank = need<int32_t>(b.sel_rank, n + 1);
  uint64_t* keys = need<uint64_t>(b.keys, nc + 1);
  uint32_t* vals = need<uint32_t>(b.vals, nc + 1);
  GLMB_LAUNCH(k_cand_keys, cdiv(nc, T), T, 0, s, nc, cand, A.h, keys, vals);
  // canonical key order: a stable sort by parent rank of the enumeration order, unless every
  // candidate is a root (one level), whose enumeration order is the parent order
  if (!(fast && levels <= 1)) sort_pairs(keys, vals, nc, 0, ((hbits + 7) / 8) * 8, b.tk, b.tv, b.tmp, s);
  GLMB_LAUNCH(k_final_keys, cdiv(nc, T), T, 0, s, nc, vals, A.v, keys, vals);
  // stable sort on the value bits only (the input is in canonical key order already), and only
  // on the bytes below the highest one in which the candidates' values differ
  int vb = 32;
  while (vb > 0 && !((vary >> (vb - 1)) & 1u)) --vb;
  sort_pairs(keys, vals, nc, 32, 32 + ((vb + 7) / 8) * 8, b.tk, b.tv, b.tmp, s);
  GLMB_LAUNCH(k_take, cdiv(n, T), T, 0, s, n, keys, vals, A.v, out.node, out.value, out.keyrank);
  out.n = n;
  out.nd_parent = A.p;
  out.nd_item = A.i;
  out.nd_h = A.h;
  out.nd_value = A.v;
  out.levels = levels;
  out.nodes = used;
  out.form = fast ? 0 : (coop ? 1 : 2);
  return GLMB_OK;
}

}  // namespace glmb
