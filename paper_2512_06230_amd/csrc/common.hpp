// Internal declarations shared by the HIP translation units of libglmb.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <initializer_list>
#include <string>
#include <vector>

#include "../../include/glmb.h"

namespace glmb {

constexpr int kWave = 64;
constexpr int kMaxDepth = 48;       // deviations of one child

struct Error {
  glmb_status st;
  std::string msg;
};

#define GLMB_HIP(call)                                                                   \
  do {                                                                                   \
    hipError_t e_ = (call);                                                              \
    if (e_ != hipSuccess)                                                                \
      throw ::glmb::Error{GLMB_E_DEVICE, std::string(#call) + ": " + hipGetErrorString(e_)}; \
  } while (0)

#define GLMB_LAUNCH(kernel, grid, block, shmem, stream, ...)                             \
  do {                                                                                   \
    if ((grid) > 0) {                                                                    \
      hipLaunchKernelGGL(kernel, dim3(grid), dim3(block), shmem, stream, __VA_ARGS__);   \
      GLMB_HIP(hipGetLastError());                                                       \
    }                                                                                    \
  } while (0)

inline int cdiv(int64_t a, int64_t b) { return (int)((a + b - 1) / b); }

// Host waits on a stream, counted per host thread (the update reports how many it made).
inline thread_local int64_t g_stream_syncs = 0;
inline hipError_t stream_sync(hipStream_t s) {
  ++g_stream_syncs;
  return hipStreamSynchronize(s);
}

// Growable device buffer (contents are not preserved on growth unless asked).
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  void reserve(size_t n, bool keep = false, hipStream_t s = nullptr) {
    if (n <= bytes) return;
    // at least twice the request: sizes creep up over the first scans of a scene, and every
    // growth costs an allocation and a device-wide synchronisation
    size_t nb = bytes ? bytes : 4096;
    while (nb < 2 * n) nb *= 2;
    void* q = nullptr;
    if (hipMalloc(&q, nb) != hipSuccess) throw Error{GLMB_E_NOMEM, "hipMalloc of " + std::to_string(nb) + " bytes failed"};
    if (keep && p && bytes) {
      GLMB_HIP(hipMemcpyAsync(q, p, bytes, hipMemcpyDeviceToDevice, s));
      GLMB_HIP(stream_sync(s));
    }
    if (p) {
      (void)hipDeviceSynchronize();  // queued work may still use the old allocation
      (void)hipFree(p);
    }
    p = q;
    bytes = nb;
  }
  template <class T> T* as() const { return static_cast<T*>(p); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
};

// Pinned host memory, mapped into the device's address space and coherent, into which one
// kernel copies the small results (sizes, counts, flags) that a host round trip reads.
struct HostStage {
  uint32_t* h = nullptr;  // host address
  uint32_t* d = nullptr;  // the same memory as the device addresses it
  size_t words = 0;
  uint32_t seq = 0;       // sequence number of the last round trip (word 0, the data follow; never 0)
  void reserve(size_t n) {
    if (n <= words) return;
    size_t nw = words ? words : 1024;
    while (nw < n) nw *= 2;
    release();  // every read waits for its kernel: nothing still writes the old block
    void* q = nullptr;
    if (hipHostMalloc(&q, nw * sizeof(uint32_t), hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess)
      throw Error{GLMB_E_NOMEM, "hipHostMalloc of " + std::to_string(nw * 4) + " bytes failed"};
    void* dq = nullptr;
    if (hipHostGetDevicePointer(&dq, q, 0) != hipSuccess) {
      (void)hipHostFree(q);
      throw Error{GLMB_E_DEVICE, "hipHostGetDevicePointer failed on pinned host memory"};
    }
    h = (uint32_t*)q;
    d = (uint32_t*)dq;
    words = nw;
    std::memset(h, 0, nw * sizeof(uint32_t));  // no stale word can equal a later sequence number
  }
  void release() {
    if (h) (void)hipHostFree(h);
    h = d = nullptr;
    words = 0;
  }
};
// A piece of device memory read back: `words` 32-bit words from `src` (4-byte aligned).
struct ReadPiece {
  const void* src;
  int64_t words;
};
// One host round trip: the pieces are copied, in order and packed, into st (from word 1) by one
// kernel on s, which then writes a new sequence number to word 0; the host waits for that number
// (or for s).  Returns the host address of the first piece's first word.  At most eight pieces.
const uint32_t* read_back(HostStage& st, hipStream_t s, std::initializer_list<ReadPiece> pieces);

template <class T> inline T* need(DevBuf& b, int64_t n) {
  b.reserve((size_t)std::max<int64_t>(n, 1) * sizeof(T));
  return b.as<T>();
}

// ------------------------------------------------------------------ device helpers
// Order-preserving map of a float to uint32 (ascending floats -> ascending integers).
__device__ __forceinline__ uint32_t f2o(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ __forceinline__ float o2f(uint32_t o) {
  uint32_t u = (o & 0x80000000u) ? (o & 0x7fffffffu) : ~o;
  return __uint_as_float(u);
}
__host__ __device__ __forceinline__ uint64_t mix64(uint64_t x) {
  x += 0x9e3779b97f4a7c15ull;
  x = (x ^ (x >> 30)) * 0xbf58476d1ce4e5b9ull;
  x = (x ^ (x >> 27)) * 0x94d049bb133111ebull;
  return x ^ (x >> 31);
}
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (kWave - 1)); }
__device__ __forceinline__ uint64_t lanemask_lt() {
  const int l = lane_id();
  return l == 0 ? 0ull : (~0ull >> (64 - l));
}

// ------------------------------------------------------------------ association cells
// The per-(hypothesis, detection) results of the association pass: best option (slot + 1),
// first deviation and log option mass relative to c_i.  Hypothesis 0's cells are dense at
// [0, M); hypothesis h >= 1 stores only its cells that differ from hypothesis 0's
// ("touched"), in ascending detection order at [h * M, h * M + n_h), with one bit per
// detection in tbits (H x W words) and the touched count before each word in tpre.
struct CellView {
  const int16_t* best16;
  const float* dev1;
  const float* lserel;
  const uint32_t* tbits;
  const uint16_t* tpre;
  int M, W;
  __device__ __forceinline__ size_t at(int h, int i) const {
    if (h == 0) return (size_t)i;
    const size_t wi = (size_t)h * W + (i >> 5);
    const uint32_t word = tbits[wi], bit = 1u << (i & 31);
    if (!(word & bit)) return (size_t)i;
    return (size_t)h * M + tpre[wi] + __popc(word & (bit - 1u));
  }
};

// ------------------------------------------------------------------ primitives (primitives.hip)
// Exclusive scan of n int32 values (in may equal out); total written to *total (device).
void scan_excl(const int32_t* in, int32_t* out, int n, int32_t* total, DevBuf& tmp, hipStream_t s);
void scan_excl64(const int64_t* in, int64_t* out, int n, int64_t* total, DevBuf& tmp, hipStream_t s);
// Stable LSD radix sort of (key, value) pairs on key bits [bit0, bit1).
void sort_pairs(uint64_t* keys, uint32_t* vals, int n, int bit0, int bit1, DevBuf& tk, DevBuf& tv,
                DevBuf& tmp, hipStream_t s);
// Lower bound t on the K-th largest of n floats with count(v >= t) >= K (a value of the
// K-th largest's 24-bit orderable bin).  Writes -inf when n < K.  Result in *out (device).
void kth_bound(const float* v, int n, int K, float* out, DevBuf& tmp, hipStream_t s);
// Same, for values given as (value, multiplicity) pairs.
void kth_bound_mult(const float* v, const int32_t* mult, int n, int K, float* out, DevBuf& tmp, hipStream_t s);
// Same, over the H * (M + 1) values B[h] - dev1 of cell (h, i) (i < M) and B[h].
void kth_bound_cells(const float* B, const CellView& cv, int H, int M, int K, float* out, DevBuf& tmp,
                     hipStream_t s);
// Same, over the roots and, per row, the cells of the m detections with the smallest first
// deviations in row 0 (m chosen from H and K; all cells when that subset would be most of them).
void kth_bound_cells_sub(const float* B, const CellView& cv, int H, int M, int K, float* out, DevBuf& tmp,
                         DevBuf& selbuf, hipStream_t s);

// ------------------------------------------------------------------ selection engine (select.hip)
// Parents with base values; per-parent item lists sorted by (delta, group, option).
struct SelectIn {
  int P;                  // number of parents (rank order)
  const float* base;      // [P]
  const int32_t* it_off;  // [P+1]
  const float* it_delta;  // [n_items]
  const int32_t* it_group;
  int K;
  const float* t0;        // device scalar: a lower bound on the K-th best child value
  bool* prefer_multi;     // per call site: the previous search outgrew one workgroup (may be null)
  bool allow_coop = true; // the whole-GPU search may be one cooperative launch
  bool force_multi = false;  // always the host-driven multi-kernel levels (diagnostic setting)
  float dp_inflate = 0.f;    // diagnostic: the counting bound raised this part of the way to the best value
  int group_bits = 2;        // one-workgroup search, items' group tables in LDS: 0 never, 1 with hashed
                             // group bits only, 2 exact bits where the items carry <= 64 groups
};
struct Selected {
  int n;                  // number of selected children (<= K)
  // device arrays (owned by the engine's buffers, valid until the next select):
  int32_t* node;          // [n] node index of each selected child, in rank order
  float* value;           // [n]
  int32_t* keyrank;       // [n] position of the child in canonical-key order among the selected
  // node storage
  int32_t* nd_parent;     // parent node (-1 for roots)
  int32_t* nd_item;       // item index (-1 for roots)
  int32_t* nd_h;          // parent hypothesis
  float* nd_value;
  int levels, nodes;
  int form;               // 0: one workgroup, 1: cooperative whole-GPU launch, 2: multi-kernel levels,
                          // 3: sampled maps (no search)
};
struct SelectBufs {
  DevBuf nd_parent, nd_item, nd_h, nd_value, nd_bloom, cnt, pre, pre64, flags, map, tmp, tk, tv, keys, vals, sel_node,
      sel_val, sel_rank, scal, hist, dp, dpc, dpa, cand;
  HostStage hs;             // host round trips of the selection and of the stages that own it
  bool hist_ready = false;  // hist holds zeros (the cooperative search leaves it so)
  bool dpc_ready = false;   // dpc holds zeros (the counting bound leaves it so)
};
glmb_status select_topk(const SelectIn& in, int cap_nodes, SelectBufs& b, Selected& out, hipStream_t s,
                        std::string& err, bool trace = false);
// Counting lower bound on the K-th best child (select.hip): the first pass counts each parent's
// first deviations (dev1 of its cells) and returns a device scalar holding the bound (t0 when no
// count reaches K); dp_bound_items raises it with the items of the children above it;
// dp_bound_refined reads whether it rose above t0 (synchronises).
const float* dp_bound_rows(const float* base, int P, const CellView& cv, int M, int K, const float* t0,
                           SelectBufs& b, hipStream_t s);
void dp_bound_items(const SelectIn& in, SelectBufs& b, hipStream_t s);
bool dp_bound_refined(SelectBufs& b, hipStream_t s);
void dp_bound_trace(SelectBufs& b, hipStream_t s);

}  // namespace glmb
