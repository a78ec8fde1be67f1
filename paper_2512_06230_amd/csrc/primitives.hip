// Device primitives: exclusive scan, stable LSD radix sort of (u64 key, u32 value) pairs,
// and a two-pass histogram bound on the K-th largest float.
#include "common.hpp"

#include <chrono>

namespace glmb {

// ============================================================================ read back
constexpr int kReadMax = 8;
constexpr int kReadSpinUs = 2000;  // host spin before a stream wait takes over
struct ReadList {
  const uint32_t* src[kReadMax];
  int32_t n[kReadMax];
  int32_t off[kReadMax];
  int32_t cnt;
};

// One workgroup copies the pieces to dst[1..], then every thread's stores are made visible to
// the host (system-scope fence) before thread 0 writes the sequence number to dst[0], a word that
// never holds data: the host may wait for that word instead of for the stream.
constexpr int kReadT = 1024;
__global__ __launch_bounds__(kReadT) void k_read_back(ReadList l, uint32_t* dst, uint32_t seq) {
  for (int p = 0; p < l.cnt; ++p) {
    const uint32_t* src = l.src[p];
    uint32_t* out = dst + 1 + l.off[p];
    for (int j = threadIdx.x; j < l.n[p]; j += kReadT) out[j] = src[j];
  }
  // a release at system scope (the host reads the words once it sees the sequence number); no
  // acquire, so the device's L2 is written back but not invalidated for the kernels after this
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "");
  __syncthreads();
  if (threadIdx.x == 0) __hip_atomic_store(dst, seq, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

const uint32_t* read_back(HostStage& st, hipStream_t s, std::initializer_list<ReadPiece> pieces) {
  if (pieces.size() > (size_t)kReadMax) throw Error{GLMB_E_STATE, "read_back: more than eight pieces"};
  ReadList l{};
  int64_t tot = 0;
  for (const ReadPiece& p : pieces) {
    const int64_t w = std::max<int64_t>(p.words, 0);
    l.src[l.cnt] = (const uint32_t*)p.src;
    l.n[l.cnt] = (int32_t)w;
    l.off[l.cnt] = (int32_t)tot;
    tot += w;
    ++l.cnt;
  }
  st.reserve((size_t)tot + 1);
  if (++st.seq == 0) st.seq = 1;
  const uint32_t seq = st.seq;
  GLMB_LAUNCH(k_read_back, 1, kReadT, 0, s, l, st.d, seq);
  // wait for the sequence word (a spin on pinned memory answers sooner than a stream wait);
  // after a while, or if the word does not come, wait for the stream, which also reports
  // any device error
  ++g_stream_syncs;
  const auto t0 = std::chrono::steady_clock::now();
  bool seen = false;
  while (!(seen = __atomic_load_n(st.h, __ATOMIC_ACQUIRE) == seq)) {
    if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(kReadSpinUs)) break;
  }
  if (!seen) {
    GLMB_HIP(hipStreamSynchronize(s));
    if (__atomic_load_n(st.h, __ATOMIC_ACQUIRE) != seq)
      throw Error{GLMB_E_DEVICE, "read_back: the gather kernel finished without its sequence word"};
  }
  return st.h + 1;
}

// ============================================================================ scan
constexpr int kScanT = 256;
constexpr int kScanI = 8;
constexpr int kScanTile = kScanT * kScanI;

template <class I>
__device__ __forceinline__ I block_excl_scan(I v, I* sh, I* total) {
  // wave inclusive scan via shuffles, then across the waves of the block
  const int lane = lane_id(), w = threadIdx.x / kWave;
  I x = v;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    I y = __shfl_up(x, d, kWave);
    if (lane >= d) x += y;
  }
  if (lane == kWave - 1) sh[w] = x;
  __syncthreads();
  if (threadIdx.x == 0) {
    I run = 0;
    for (int i = 0; i < (int)(blockDim.x / kWave); ++i) {
      I t = sh[i];
      sh[i] = run;
      run += t;
    }
    sh[16] = run;
  }
  __syncthreads();
  I r = x - v + sh[w];
  *total = sh[16];
  __syncthreads();
  return r;
}

template <class I>
__global__ __launch_bounds__(kScanT) void k_scan_tiles(const I* in, I* out, int n, I* tile_sums) {
  __shared__ I sh[32];
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanI;
  I v[kScanI];
  I s = 0;
#pragma unroll
  for (int j = 0; j < kScanI; ++j) {
    v[j] = (base + j < n) ? in[base + j] : 0;
    s += v[j];
  }
  I tot;
  I off = block_excl_scan<I>(s, sh, &tot);
#pragma unroll
  for (int j = 0; j < kScanI; ++j) {
    if (base + j < n) out[base + j] = off;
    off += v[j];
  }
  if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// one block: exclusive scan of the tile sums in chunks with a running carry
template <class I>
__global__ __launch_bounds__(kScanT) void k_scan_sums(I* sums, int nt, I* total) {
  __shared__ I sh[32];
  I carry = 0;
  for (int c = 0; c < nt; c += kScanT) {
    const int i = c + threadIdx.x;
    I v = i < nt ? sums[i] : 0;
    I tot;
    I r = block_excl_scan<I>(v, sh, &tot);
    if (i < nt) sums[i] = r + carry;
    carry += tot;
  }
  if (threadIdx.x == 0 && total) *total = carry;
}

template <class I>
__global__ __launch_bounds__(kScanT) void k_scan_add(I* out, int n, const I* sums) {
  const int base = blockIdx.x * kScanTile + threadIdx.x * kScanI;
  const I a = sums[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kScanI; ++j)
    if (base + j < n) out[base + j] += a;
}

// one workgroup of 1024 threads, each scanning a contiguous run of at most 16 elements:
// one launch for the small scans (radix-sort histograms, per-hypothesis counts)
constexpr int kScanSmallT = 1024, kScanSmallI = 16;
template <class I>
__global__ __launch_bounds__(kScanSmallT) void k_scan_small(const I* in, I* out, int n, I* total) {
  __shared__ I sh[32];
  const int per = (n + kScanSmallT - 1) / kScanSmallT;
  const int b = min(n, (int)threadIdx.x * per), e = min(n, b + per);
  I v[kScanSmallI];
  I sum = 0;
#pragma unroll
  for (int j = 0; j < kScanSmallI; ++j) {
    v[j] = b + j < e ? in[b + j] : (I)0;
    sum += v[j];
  }
  I tot;
  I off = block_excl_scan<I>(sum, sh, &tot);
#pragma unroll
  for (int j = 0; j < kScanSmallI; ++j) {
    if (b + j < e) out[b + j] = off;
    off += v[j];
  }
  if (threadIdx.x == 0 && total) *total = tot;
}

template <class I>
static void scan_impl(const I* in, I* out, int n, I* total, DevBuf& tmp, hipStream_t s) {
  if (n <= kScanSmallT * kScanSmallI) {
    GLMB_LAUNCH(k_scan_small<I>, 1, kScanSmallT, 0, s, in, out, n, total);
    return;
  }
  const int nt = std::max(1, cdiv(n, kScanTile));
  I* sums = need<I>(tmp, nt);
  if (n > 0) GLMB_LAUNCH(k_scan_tiles<I>, nt, kScanT, 0, s, in, out, n, sums);
  else GLMB_HIP(hipMemsetAsync(sums, 0, sizeof(I), s));
  GLMB_LAUNCH(k_scan_sums<I>, 1, kScanT, 0, s, sums, nt, total);
  if (n > 0) GLMB_LAUNCH(k_scan_add<I>, nt, kScanT, 0, s, out, n, sums);
}

void scan_excl(const int32_t* in, int32_t* out, int n, int32_t* total, DevBuf& tmp, hipStream_t s) {
  scan_impl<int32_t>(in, out, n, total, tmp, s);
}
void scan_excl64(const int64_t* in, int64_t* out, int n, int64_t* total, DevBuf& tmp, hipStream_t s) {
  scan_impl<int64_t>(in, out, n, total, tmp, s);
}

// ============================================================================ radix sort
// Stable LSD radix sort by 8-bit digits.  Per pass: per-tile digit counts, then a scatter in
// which every tile places its items at (items of smaller digits) + (items of its digit in
// earlier tiles) + (rank within the tile).  With few tiles the scatter computes those offsets
// from the counts itself; otherwise a scan of the counts runs between the two kernels.
constexpr int kSortT = 256;
constexpr int kSortRBig = 8;    // rounds of kSortT items per tile for large inputs
constexpr int kSortRSmall = 2;  // ... and for small ones (more tiles in flight)
constexpr int kSortFuseTiles = 64;

__global__ __launch_bounds__(kSortT) void k_sort_hist(const uint64_t* keys, int n, int shift, int nb, int rounds,
                                                      int32_t* hist) {
  __shared__ int32_t h[256];
  h[threadIdx.x] = 0;
  __syncthreads();
  const int base = blockIdx.x * kSortT * rounds;
  for (int r = 0; r < rounds; ++r) {
    const int i = base + r * kSortT + threadIdx.x;
    if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
  }
  __syncthreads();
  hist[threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// hist: the scanned counts, or (fused) the raw counts [digit][tile]
__global__ __launch_bounds__(kSortT) void k_sort_scatter(const uint64_t* kin, const uint32_t* vin, uint64_t* kout,
                                                         uint32_t* vout, int n, int shift, int nb, int rounds,
                                                         const int32_t* hist, int fused) {
  __shared__ int32_t base_d[256];
  __shared__ int32_t running[256];
  __shared__ int32_t wcnt[kSortT / kWave][256];
  __shared__ int32_t woff[kSortT / kWave][256];
  __shared__ int32_t rtot[256];
  __shared__ int32_t sh[32];
  const int t = threadIdx.x, w = t / kWave;
  if (fused) {
    // this digit's counts in every tile, every load issued before the first add
    int32_t v[kSortFuseTiles];
#pragma unroll
    for (int k = 0; k < kSortFuseTiles; ++k) v[k] = k < nb ? hist[t * nb + k] : 0;
    int tot = 0, before = 0;
#pragma unroll
    for (int k = 0; k < kSortFuseTiles; ++k) {
      tot += v[k];
      before += k < (int)blockIdx.x ? v[k] : 0;
    }
    int all;
    base_d[t] = block_excl_scan<int32_t>(tot, sh, &all) + before;
  } else {
    base_d[t] = hist[t * nb + blockIdx.x];
  }
  running[t] = 0;
  for (int j = 0; j < kSortT / kWave; ++j) wcnt[j][t] = 0;
  __syncthreads();
  const int tile = blockIdx.x * kSortT * rounds;
  for (int r = 0; r < rounds; ++r) {
    const int i = tile + r * kSortT + t;
    const bool valid = i < n;
    uint64_t k = valid ? kin[i] : 0;
    uint32_t v = valid ? vin[i] : 0;
    const int d = (int)((k >> shift) & 255);
    uint64_t same = __ballot(valid);
#pragma unroll
    for (int b = 0; b < 8; ++b) {
      const uint64_t bal = __ballot((d >> b) & 1);
      same &= ((d >> b) & 1) ? bal : ~bal;
    }
    const int rank = __popcll(same & lanemask_lt());
    if (valid && rank == 0) wcnt[w][d] = __popcll(same);
    __syncthreads();
    {
      int32_t run = 0;
      for (int j = 0; j < kSortT / kWave; ++j) {
        const int32_t c = wcnt[j][t];
        woff[j][t] = run;
        run += c;
      }
      rtot[t] = run;
    }
    __syncthreads();
    if (valid) {
      const int pos = base_d[d] + running[d] + woff[w][d] + rank;
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    running[t] += rtot[t];
    for (int j = 0; j < kSortT / kWave; ++j) wcnt[j][t] = 0;
    __syncthreads();
  }
}

__global__ void k_copy_pairs(int n, const uint64_t* ks, const uint32_t* vs, uint64_t* kd, uint32_t* vd) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) {
    kd[i] = ks[i];
    vd[i] = vs[i];
  }
}

void sort_pairs(uint64_t* keys, uint32_t* vals, int n, int bit0, int bit1, DevBuf& tk, DevBuf& tv, DevBuf& tmp,
                hipStream_t s) {
  if (n <= 1 || bit1 <= bit0) return;
  const int rounds = n <= kSortFuseTiles * kSortT * kSortRSmall ? kSortRSmall : kSortRBig;
  const int nb = cdiv(n, kSortT * rounds);
  const bool fused = nb <= kSortFuseTiles;
  uint64_t* k2 = need<uint64_t>(tk, n);
  uint32_t* v2 = need<uint32_t>(tv, n);
  // scan scratch: hist (256*nb) + tile sums
  tmp.reserve(((size_t)256 * nb + (size_t)cdiv(256 * nb, kScanTile) + 64) * sizeof(int32_t));
  int32_t* hist = tmp.as<int32_t>();
  int32_t* sums = hist + (size_t)256 * nb;
  uint64_t *ka = keys, *kb = k2;
  uint32_t *va = vals, *vb = v2;
  int passes = 0;
  for (int sh = bit0; sh < bit1; sh += 8, ++passes) {
    GLMB_LAUNCH(k_sort_hist, nb, kSortT, 0, s, ka, n, sh, nb, rounds, hist);
    if (!fused) {
      const int m = 256 * nb;
      if (m <= kScanSmallT * kScanSmallI) {
        GLMB_LAUNCH(k_scan_small<int32_t>, 1, kScanSmallT, 0, s, hist, hist, m, (int32_t*)nullptr);
      } else {
        const int nt = cdiv(m, kScanTile);
        GLMB_LAUNCH(k_scan_tiles<int32_t>, nt, kScanT, 0, s, hist, hist, m, sums);
        GLMB_LAUNCH(k_scan_sums<int32_t>, 1, kScanT, 0, s, sums, nt, (int32_t*)nullptr);
        GLMB_LAUNCH(k_scan_add<int32_t>, nt, kScanT, 0, s, hist, m, sums);
      }
    }
    GLMB_LAUNCH(k_sort_scatter, nb, kSortT, 0, s, ka, va, kb, vb, n, sh, nb, rounds, hist, fused ? 1 : 0);
    std::swap(ka, kb);
    std::swap(va, vb);
  }
  if (passes & 1) GLMB_LAUNCH(k_copy_pairs, cdiv(n, 256), 256, 0, s, n, ka, va, keys, vals);
}

// ============================================================================ K-th bound
constexpr int kBins = 4096;

__global__ __launch_bounds__(256) void k_bound_hist(const float* v, const int32_t* mult, int n, int pass,
                                                    const uint32_t* prefix, int32_t* hist) {
  __shared__ int32_t h[kBins];
  for (int j = threadIdx.x; j < kBins; j += blockDim.x) h[j] = 0;
  __syncthreads();
  const uint32_t pre = pass ? *prefix : 0u;
  for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) {
    const uint32_t o = f2o(v[i]);
    const int32_t c = mult ? mult[i] : 1;
    if (c <= 0) continue;
    if (pass == 0) atomicAdd(&h[o >> 20], c);
    else if ((o >> 20) == pre) atomicAdd(&h[(o >> 8) & (kBins - 1)], c);
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kBins; j += blockDim.x)
    if (h[j]) atomicAdd(&hist[j], h[j]);
}

// one workgroup of 1024 threads, four bins each: find the bin holding the K-th largest value
// (counting from the top), then clear the histogram for the next use
__global__ __launch_bounds__(1024) void k_bound_pick(int32_t* hist, int pass, uint32_t* prefix, int32_t* need_k,
                                                     float* out) {
  static_assert(kBins == 4 * 1024, "four bins per thread");
  __shared__ int64_t wsum[16];
  __shared__ int found;
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave;
  const int64_t K = *need_k;
  int32_t c[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) c[j] = hist[4 * t + j];
  const int64_t mine = (int64_t)c[0] + c[1] + c[2] + c[3];
  // inclusive scan of `mine` over threads in descending bin order (thread 1023 first)
  int64_t x = mine;
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int64_t y = __shfl_down(x, d, kWave);
    if (lane + d < kWave) x += y;
  }
  if (lane == 0) wsum[w] = x;  // total of this wave
  if (t == 0) found = 0;
  __syncthreads();
  int64_t above = x - mine;  // bins of higher threads within the wave
  for (int j = w + 1; j < 16; ++j) above += wsum[j];
  if (above < K && above + mine >= K) {
    int64_t acc = above;
    int b = 4 * t + 3;
    for (; b > 4 * t; --b) {
      if (acc + c[b - 4 * t] >= K) break;
      acc += c[b - 4 * t];
    }
    found = 1;
    if (pass == 0) {
      *prefix = (uint32_t)b;
      *need_k = (int32_t)(K - acc);
    } else {
      // lowest value of the bin; the bin of -inf starts below -inf (a NaN pattern)
      const float e = o2f(((*prefix) << 20) | ((uint32_t)b << 8));
      *out = e == e ? e : -INFINITY;
    }
  }
  __syncthreads();
  if (t == 0 && !found) {
    *out = -INFINITY;
    *prefix = 0xffffffffu;  // no second pass restriction matches
  }
#pragma unroll
  for (int j = 0; j < 4; ++j) hist[4 * t + j] = 0;
}

__global__ void k_bound_init(int32_t* hist, int32_t* need_k, int32_t K) {
  for (int j = threadIdx.x; j < kBins; j += blockDim.x) hist[j] = 0;
  if (threadIdx.x == 0) *need_k = K;
}

static void kth_bound_impl(const float* v, const int32_t* mult, int n, int K, float* out, DevBuf& tmp,
                           hipStream_t s) {
  tmp.reserve((kBins + 8) * sizeof(int32_t));
  int32_t* hist = tmp.as<int32_t>();
  uint32_t* prefix = (uint32_t*)(hist + kBins);
  int32_t* need_k = hist + kBins + 1;
  GLMB_LAUNCH(k_bound_init, 1, 256, 0, s, hist, need_k, (int32_t)K);
  const int grid = std::max(1, std::min(cdiv(n, 256 * 8), 1024));
  GLMB_LAUNCH(k_bound_hist, grid, 256, 0, s, v, mult, n, 0, prefix, hist);
  GLMB_LAUNCH(k_bound_pick, 1, 1024, 0, s, hist, 0, prefix, need_k, out);
  GLMB_LAUNCH(k_bound_hist, grid, 256, 0, s, v, mult, n, 1, prefix, hist);
  GLMB_LAUNCH(k_bound_pick, 1, 1024, 0, s, hist, 1, prefix, need_k, out);
}

// the same bound over the values B[h] - dev1 of every cell (h, i) and B[h] of every row
__global__ __launch_bounds__(256) void k_bound_hist_cells(int H, int M, const float* B, CellView cv, int pass,
                                                          const uint32_t* prefix, int32_t* hist) {
  __shared__ int32_t h[kBins];
  for (int j = threadIdx.x; j < kBins; j += blockDim.x) h[j] = 0;
  __syncthreads();
  const uint32_t pre = pass ? *prefix : 0u;
  auto bin_of = [&](float v) -> int {
    const uint32_t o = f2o(v);
    if (pass == 0) return (int)(o >> 20);
    return (o >> 20) == pre ? (int)((o >> 8) & (kBins - 1)) : -1;
  };
  // rows in turn, the threads along a row (no division per element); the values crowd into
  // few bins, so a wave whose lanes all share one bin adds 64 with one atomic.  A row counts
  // every cell with hypothesis 0's first deviation, then exchanges that count for its own on
  // its touched cells, one (word, bit) of the touched set per thread (the counts are
  // integers: the exchange is exact).
  for (int r = blockIdx.x; r < H; r += gridDim.x) {
    const float b = B[r];
    for (int i0 = 0; i0 < M; i0 += blockDim.x) {
      const int i = i0 + threadIdx.x;
      const int bin = i < M ? bin_of(b - cv.dev1[i]) : -1;
      const int b0 = __shfl(bin, 0, kWave);
      if (b0 >= 0 && __ballot(bin == b0) == ~0ull) {
        if (lane_id() == 0) atomicAdd(&h[b0], kWave);
      } else if (bin >= 0) {
        atomicAdd(&h[bin], 1);
      }
    }
    if (r > 0)
      for (int x = threadIdx.x; x < 32 * cv.W; x += blockDim.x) {
        const size_t wi = (size_t)r * cv.W + (x >> 5);
        const uint32_t word = cv.tbits[wi], bit = 1u << (x & 31);
        if (!(word & bit)) continue;
        const size_t e = (size_t)r * M + cv.tpre[wi] + __popc(word & (bit - 1u));
        const int bn = bin_of(b - cv.dev1[e]), bo = bin_of(b - cv.dev1[x]);
        if (bn != bo) {
          if (bn >= 0) atomicAdd(&h[bn], 1);
          if (bo >= 0) atomicSub(&h[bo], 1);
        }
      }
    if (threadIdx.x == 0) {
      const int br = bin_of(b);
      if (br >= 0) atomicAdd(&h[br], 1);
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kBins; j += blockDim.x)
    if (h[j]) atomicAdd(&hist[j], h[j]);
}

void kth_bound_cells(const float* B, const CellView& cv, int H, int M, int K, float* out, DevBuf& tmp,
                     hipStream_t s) {
  tmp.reserve((kBins + 8) * sizeof(int32_t));
  int32_t* hist = tmp.as<int32_t>();
  uint32_t* prefix = (uint32_t*)(hist + kBins);
  int32_t* need_k = hist + kBins + 1;
  const int64_t n = (int64_t)H * (M + 1);
  GLMB_LAUNCH(k_bound_init, 1, 256, 0, s, hist, need_k, (int32_t)K);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((n + 256 * 8 - 1) / (256 * 8), std::min(H, 1024)));
  GLMB_LAUNCH(k_bound_hist_cells, grid, 256, 0, s, H, M, B, cv, 0, prefix, hist);
  GLMB_LAUNCH(k_bound_pick, 1, 1024, 0, s, hist, 0, prefix, need_k, out);
  GLMB_LAUNCH(k_bound_hist_cells, grid, 256, 0, s, H, M, B, cv, 1, prefix, hist);
  GLMB_LAUNCH(k_bound_pick, 1, 1024, 0, s, hist, 1, prefix, need_k, out);
}

// The same bound over a subset of the children: every root B[h] and, in every row, the cells of
// the m detections whose first deviation is smallest in row 0 (sel).  The K-th largest of a
// subset of the children's values is at most the K-th largest of all, so the result is still
// a lower bound; it reads H (m + 1) cells instead of H (M + 1).
__global__ __launch_bounds__(256) void k_bound_hist_sub(int H, int m, const int32_t* sel, const int32_t* msel,
                                                        const float* B, CellView cv, int pass, const uint32_t* prefix,
                                                        int32_t* hist) {
  __shared__ int32_t h[kBins];
  for (int j = threadIdx.x; j < kBins; j += blockDim.x) h[j] = 0;
  __syncthreads();
  const uint32_t pre = pass ? *prefix : 0u;
  const int mt = min(*msel, m), lane = lane_id();
  auto bin_of = [&](float v) -> int {
    const uint32_t o = f2o(v);
    if (pass == 0) return (int)(o >> 20);
    return (o >> 20) == pre ? (int)((o >> 8) & (kBins - 1)) : -1;
  };
  // each wave takes kRB rows at a time (the loads of all of them issued before any is used):
  // the lanes over the selected detections, lane 0 also the roots; a wave whose lanes all
  // share one bin adds its count with one atomic
  constexpr int kRB = 4;
  const int nw = gridDim.x * (blockDim.x / kWave);
  const int gw = blockIdx.x * (blockDim.x / kWave) + (int)threadIdx.x / kWave;
  for (int q0 = 0; q0 < mt; q0 += kWave) {
    const int q = q0 + lane;
    const bool on = q < mt;
    const int iq = on ? sel[q] : 0;
    const uint64_t all = __ballot(on);
    for (int r0 = gw; r0 < H; r0 += kRB * nw) {
      float bv[kRB], dv[kRB];
#pragma unroll
      for (int j = 0; j < kRB; ++j) {
        const int r = r0 + j * nw;
        bv[j] = r < H ? B[r] : -INFINITY;
        dv[j] = (r < H && on) ? cv.dev1[cv.at(r, iq)] : INFINITY;
      }
#pragma unroll
      for (int j = 0; j < kRB; ++j) {
        const int r = r0 + j * nw;
        if (r >= H) break;  // uniform: r depends on the wave only
        const int bin = on ? bin_of(bv[j] - dv[j]) : -1;
        const int b0 = __shfl(bin, 0, kWave);
        if (b0 >= 0 && __ballot(bin == b0) == all) {
          if (lane == 0) atomicAdd(&h[b0], __popcll(all));
        } else if (bin >= 0) {
          atomicAdd(&h[bin], 1);
        }
        if (q0 == 0 && lane == 0) {
          const int br = bin_of(bv[j]);
          if (br >= 0) atomicAdd(&h[br], 1);
        }
      }
    }
  }
  __syncthreads();
  for (int j = threadIdx.x; j < kBins; j += blockDim.x)
    if (h[j]) atomicAdd(&hist[j], h[j]);
}

// One workgroup: about m detections with the smallest first deviations of row 0 (any subset of
// the cells gives a valid bound; the smallest ones make it tight).  A 256-bin histogram of the
// top byte of the orderable values finds the bin b in which the m-th smallest lies; every
// detection of a lower bin is taken, then those of bin b in index order, up to m in all
// (m <= M, so exactly m are taken; the count is written to *msel all the same).
__global__ __launch_bounds__(1024) void k_ref_order(int M, const float* dev1, int m, int32_t* sel, int32_t* msel) {
  __shared__ int32_t hist[256];
  __shared__ int32_t wc[16];
  __shared__ int32_t cut, taken;
  const int t = threadIdx.x, lane = lane_id(), w = t / kWave, nw = blockDim.x / kWave;
  if (t < 256) hist[t] = 0;
  __syncthreads();
  for (int i = t; i < M; i += blockDim.x) atomicAdd(&hist[f2o(dev1[i]) >> 24], 1);
  __syncthreads();
  // the bin where the running count from the smallest values reaches m: a scan over the 256
  // bins by the first four waves (bin 255 when the count stays below m)
  if (t == 0) {
    cut = 255;
    taken = 0;
  }
  int c = 0, x = 0;
  if (t < 256) {
    c = hist[t];
    x = c;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const int y = __shfl_up(x, d, kWave);
      if (lane >= d) x += y;
    }
    if (lane == kWave - 1) wc[w] = x;
  }
  __syncthreads();
  if (t < 256) {
    int before = x - c;
    for (int q = 0; q < w; ++q) before += wc[q];
    if (before < m && before + c >= m) cut = t;
  }
  __syncthreads();
  const int b = cut;
  // two sweeps in index order: the lower bins, then bin b while fewer than m are taken
  for (int sweep = 0; sweep < 2; ++sweep) {
    for (int i0 = 0; i0 < M; i0 += blockDim.x) {
      const int i = i0 + t;
      const int bi = i < M ? (int)(f2o(dev1[i]) >> 24) : 256;
      const bool on = sweep == 0 ? bi < b : bi == b;
      const uint64_t bal = __ballot(on);
      if (lane == 0) wc[w] = __popcll(bal);
      __syncthreads();
      int before = 0, tot = 0;
      for (int x = 0; x < nw; ++x) {
        if (x < w) before += wc[x];
        tot += wc[x];
      }
      const int at = taken + before + __popcll(bal & lanemask_lt());
      if (on && at < m) sel[at] = i;
      __syncthreads();
      if (t == 0) taken = min(m, taken + tot);
      __syncthreads();
      if (taken >= m) break;
    }
  }
  if (t == 0) *msel = taken;
}

void kth_bound_cells_sub(const float* B, const CellView& cv, int H, int M, int K, float* out, DevBuf& tmp,
                         DevBuf& selbuf, hipStream_t s) {
  // enough values that the subset's K-th largest stays close to the full one's
  int m = 64;
  if ((int64_t)H * (m + 1) < 4 * (int64_t)K) m = (int)std::min<int64_t>(M, cdiv(4 * (int64_t)K, H));
  if (m * 2 > M || H < 2) {
    kth_bound_cells(B, cv, H, M, K, out, tmp, s);
    return;
  }
  int32_t* sel = need<int32_t>(selbuf, m + 1);
  GLMB_LAUNCH(k_ref_order, 1, 1024, 0, s, M, cv.dev1, m, sel, sel + m);
  tmp.reserve((kBins + 8) * sizeof(int32_t));
  int32_t* hist = tmp.as<int32_t>();
  uint32_t* prefix = (uint32_t*)(hist + kBins);
  int32_t* need_k = hist + kBins + 1;
  GLMB_LAUNCH(k_bound_init, 1, 256, 0, s, hist, need_k, (int32_t)K);
  const int grid = std::max(1, std::min(cdiv(H, 4 * 4), 256));
  GLMB_LAUNCH(k_bound_hist_sub, grid, 256, 0, s, H, m, (const int32_t*)sel, (const int32_t*)(sel + m), B, cv, 0, prefix,
              hist);
  GLMB_LAUNCH(k_bound_pick, 1, 1024, 0, s, hist, 0, prefix, need_k, out);
  GLMB_LAUNCH(k_bound_hist_sub, grid, 256, 0, s, H, m, (const int32_t*)sel, (const int32_t*)(sel + m), B, cv, 1, prefix,
              hist);
  GLMB_LAUNCH(k_bound_pick, 1, 1024, 0, s, hist, 1, prefix, need_k, out);
}

void kth_bound(const float* v, int n, int K, float* out, DevBuf& tmp, hipStream_t s) {
  kth_bound_impl(v, nullptr, n, K, out, tmp, s);
}
void kth_bound_mult(const float* v, const int32_t* mult, int n, int K, float* out, DevBuf& tmp, hipStream_t s) {
  kth_bound_impl(v, mult, n, K, out, tmp, s);
}

}  // namespace glmb
