// Learned pair proposal, an addition to the update of Sec. 3, on the GPU:
//
//   pairs      compaction of the gated (instance, detection) pairs from the gate bits;
//   features   [d2, nu_x, nu_y, r_label, age, n_gate] of every pair;
//   network    6 -> 64 -> 64 -> 1 with ReLU: bfloat16 weights, standardised inputs and
//              hidden activations, float32 sums; one thread per pair, weights in LDS;
//   removal    pairs whose logit is below the threshold leave the gate (gate bit cleared,
//              Eq. 2 entry set to -inf) before the per-label lists are built, so every later
//              stage of the update sees fewer options;
//   lost mass  1 - Z_kept / Z_full for up to 16 thresholds in one pass over the hypotheses;
//   training   targets from the full posterior of the plain update; forward + backward over
//              64 samples per workgroup with per-sample vectors in LDS and a fixed-order
//              gradient reduction; Adam.
#include <mutex>

#include "ctx.hpp"

namespace glmb {

namespace {

// offsets in the parameter vector W1[64][6] | b1[64] | W2[64][64] | b2[64] | w3[64] | b3
constexpr int oW1 = 0, oB1 = oW1 + kNHid * kNFeat, oW2 = oB1 + kNHid, oB2 = oW2 + kNHid * kNHid, oW3 = oB2 + kNHid,
              oB3 = oW3 + kNHid;
static_assert(oB3 + 1 == kNParam, "parameter layout");
constexpr int kPartW = kNParam + 2;  // partial gradients + [sum of weights, sum of weighted losses]
constexpr int kLS = 65;              // LDS row stride of per-sample vectors (odd: no bank conflicts)

struct Norm {
  float mu[kNFeat], sd[kNFeat];
};
struct Thr {
  float t[kMaxThr];
};

// round to the nearest bfloat16 value, ties to even
__device__ __forceinline__ float bf16r(float x) {
  uint32_t u = __float_as_uint(x);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return __uint_as_float(u & 0xFFFF0000u);
}

__device__ __forceinline__ void load_params(const float* __restrict__ w, float* sw) {
  for (int q = threadIdx.x; q < kNParam; q += blockDim.x) sw[q] = bf16r(w[q]);
  __syncthreads();
}

__device__ __forceinline__ void standardise(const float* x, const Norm& nm, float* xs) {
#pragma unroll
  for (int k = 0; k < kNFeat; ++k) xs[k] = bf16r((x[k] - nm.mu[k]) / nm.sd[k]);
}

__device__ __forceinline__ void layer1(const float* sw, const float* xs, float* h1) {
#pragma unroll
  for (int j = 0; j < kNHid; ++j) {
    float a = sw[oB1 + j];
#pragma unroll
    for (int k = 0; k < kNFeat; ++k) a = fmaf(sw[oW1 + j * kNFeat + k], xs[k], a);
    h1[j] = bf16r(fmaxf(a, 0.0f));
  }
}

// pre-activation of unit j of the second hidden layer
__device__ __forceinline__ float layer2_unit(const float* sw, const float* h1, int j) {
  float a = sw[oB2 + j];
  const float* wr = sw + oW2 + j * kNHid;
#pragma unroll
  for (int k = 0; k < kNHid; ++k) a = fmaf(wr[k], h1[k], a);
  return a;
}

// Inference form of the network: weights and activations as packed bfloat16 pairs; the first
// layer's sums of two products taken by one v_dot2 instruction into an FP32 accumulator
// (products of two bfloat16 values are exact in FP32).  LDS words: W1 [64][3] | W2 [64][32] | w3 [32] packed,
// then b1 [64] | b2 [64] | b3 as floats.
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
constexpr int qW1 = 0, qW2 = qW1 + kNHid * (kNFeat / 2), qW3 = qW2 + kNHid * (kNHid / 2), qB1 = qW3 + kNHid / 2,
              qB2 = qB1 + kNHid, qB3 = qB2 + kNHid, kNQ = qB3 + 1;
static_assert(kNFeat % 2 == 0, "inputs in pairs");

// two floats rounded to the nearest bfloat16 values (ties to even) and packed, lo in the low
// half (one v_cvt_pk_bf16_f32)
__device__ __forceinline__ uint32_t pack2(float lo, float hi) {
  const bf16x2_t v = {(__bf16)lo, (__bf16)hi};
  return __builtin_bit_cast(uint32_t, v);
}
__device__ __forceinline__ float dot2(uint32_t a, uint32_t b, float c) {
  return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), c, false);
}

__device__ __forceinline__ void load_params_q(const float* __restrict__ w, uint32_t* q) {
  for (int j = threadIdx.x; j < kNHid * (kNFeat / 2); j += blockDim.x)
    q[qW1 + j] = pack2(w[oW1 + 2 * j], w[oW1 + 2 * j + 1]);
  for (int j = threadIdx.x; j < kNHid * (kNHid / 2); j += blockDim.x)
    q[qW2 + j] = pack2(w[oW2 + 2 * j], w[oW2 + 2 * j + 1]);
  for (int j = threadIdx.x; j < kNHid / 2; j += blockDim.x) q[qW3 + j] = pack2(w[oW3 + 2 * j], w[oW3 + 2 * j + 1]);
  for (int j = threadIdx.x; j < kNHid; j += blockDim.x) {
    q[qB1 + j] = __float_as_uint(bf16r(w[oB1 + j]));
    q[qB2 + j] = __float_as_uint(bf16r(w[oB2 + j]));
  }
  if (threadIdx.x == 0) q[qB3] = __float_as_uint(bf16r(w[oB3]));
  __syncthreads();
}

// standardised inputs and the first hidden layer of one sample, packed
__device__ __forceinline__ void layer1_q(const uint32_t* q, const float* x, const Norm& nm, uint32_t* h1) {
  uint32_t xq[kNFeat / 2];
#pragma unroll
  for (int k = 0; k < kNFeat / 2; ++k)
    xq[k] = pack2((x[2 * k] - nm.mu[2 * k]) / nm.sd[2 * k], (x[2 * k + 1] - nm.mu[2 * k + 1]) / nm.sd[2 * k + 1]);
#pragma unroll
  for (int j = 0; j < kNHid; j += 2) {
    float a0 = __uint_as_float(q[qB1 + j]), a1 = __uint_as_float(q[qB1 + j + 1]);
#pragma unroll
    for (int k = 0; k < kNFeat / 2; ++k) {
      a0 = dot2(q[qW1 + j * (kNFeat / 2) + k], xq[k], a0);
      a1 = dot2(q[qW1 + (j + 1) * (kNFeat / 2) + k], xq[k], a1);
    }
    h1[j / 2] = pack2(fmaxf(a0, 0.0f), fmaxf(a1, 0.0f));
  }
}

// The same network for the 64 samples of a wave (lane l: sample l; every lane of the wave must
// call it): layer 1 per lane with v_dot2, the 64 x 64 layer on the matrix cores as
// H2^T = W2 H1^T (units as rows, samples as columns) with v_mfma_f32_32x32x16_bf16: two tiles of
// 32 units by two tiles of 32 samples, four steps of 16 inputs.  Operand layouts (lane l, half
// g = l / 32): A holds row l % 32, inputs 8g..8g+7 of the step; B holds column l % 32, the same
// inputs; the accumulator's value v holds row 8 (v / 4) + 4 g + v % 4, column l % 32.  Column c of
// sample tile t is sample 32 t + c, whose hidden values lane 32 t + c holds: a lane keeps the
// half of the step's inputs its own B needs and swaps the other half with lane l ^ 32.  The
// output layer sums each lane's 32 units and its partner's.
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
typedef float f32x16_t __attribute__((ext_vector_type(16)));
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));

__device__ __forceinline__ float mlp_logit_mfma(const uint32_t* q, const float* x, const Norm& nm) {
  uint32_t h1[kNHid / 2];
  layer1_q(q, x, nm, h1);
  const int l = lane_id(), g = l >> 5, col = l & 31;
  f32x16_t acc[2][2];  // [unit tile][sample tile]
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int v = 0; v < 16; ++v) {
      const float b = __uint_as_float(q[qB2 + mt * 32 + 8 * (v >> 2) + 4 * g + (v & 3)]);
      acc[mt][0][v] = b;
      acc[mt][1][v] = b;
    }
#pragma unroll
  for (int ks = 0; ks < 4; ++ks) {
    // this lane's inputs [16 ks, 16 ks + 8) and [16 ks + 8, 16 ks + 16), four words each
    u32x4_t lo, hi, snd, rcv;
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      lo[e] = h1[8 * ks + e];
      hi[e] = h1[8 * ks + 4 + e];
    }
    snd = g ? lo : hi;
#pragma unroll
    for (int e = 0; e < 4; ++e) rcv[e] = (uint32_t)__shfl_xor((int)snd[e], 32, kWave);
    const u32x4_t b0 = g ? rcv : lo;  // samples 0..31: sample col, inputs of half g
    const u32x4_t b1 = g ? hi : rcv;  // samples 32..63
#pragma unroll
    for (int mt = 0; mt < 2; ++mt) {
      const u32x4_t a = *(const u32x4_t*)(q + qW2 + (mt * 32 + col) * (kNHid / 2) + 8 * ks + 4 * g);
      acc[mt][0] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                          __builtin_bit_cast(bf16x8_t, b0), acc[mt][0], 0, 0, 0);
      acc[mt][1] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                          __builtin_bit_cast(bf16x8_t, b1), acc[mt][1], 0, 0, 0);
    }
  }
  // output layer: values v and v + 1 of a lane are units u and u + 1 (u even), one packed
  // weight word and one v_dot2 per pair of units
  float part[2] = {0.0f, 0.0f};
#pragma unroll
  for (int mt = 0; mt < 2; ++mt)
#pragma unroll
    for (int v = 0; v < 16; v += 2) {
      const int unit = mt * 32 + 8 * (v >> 2) + 4 * g + (v & 3);
      const uint32_t wq = q[qW3 + unit / 2];
#pragma unroll
      for (int t = 0; t < 2; ++t)
        part[t] = dot2(wq, pack2(fmaxf(acc[mt][t][v], 0.0f), fmaxf(acc[mt][t][v + 1], 0.0f)), part[t]);
    }
  const float mine = part[g];
  return __uint_as_float(q[qB3]) + (mine + __shfl_xor(part[g ^ 1], 32, kWave));
}

// features of pair (instance x, detection zi); d2 uses the gate's expression
__device__ __forceinline__ void pair_feature(const DInst& x, float2 zi, float sig2, float r, float age, float ng,
                                             float* f) {
  const float s00 = x.P[0] + sig2, s01 = x.P[1], s11 = x.P[4] + sig2;
  const float det = s00 * s11 - s01 * s01;
  const float n0 = zi.x - x.m[0], n1 = zi.y - x.m[1];
  const float qd = s11 * n0 * n0 - 2.0f * s01 * n0 * n1 + s00 * n1 * n1;
  f[0] = qd / det;
  f[1] = n0;
  f[2] = n1;
  f[3] = r;
  f[4] = age;
  f[5] = ng;
}

__device__ __forceinline__ float wsum(float v, float* sh) {
  for (int d = kWave / 2; d > 0; d >>= 1) v += __shfl_xor(v, d, kWave);
  __syncthreads();
  if (lane_id() == 0) sh[threadIdx.x / kWave] = v;
  __syncthreads();
  float r = 0.0f;
  for (int j = 0; j < (int)(blockDim.x / kWave); ++j) r += sh[j];
  return r;
}

}  // namespace

// ------------------------------------------------------------------ pairs and features
// per instance: gated detection count and per-word prefix counts of its gate bits
// one wave per instance: gated detections per word of its gate bits, their prefix and total
__global__ __launch_bounds__(256) void k_pair_count(int U, int W, const uint32_t* gbits, int32_t* cnt,
                                                    int32_t* ppre) {
  const int u = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kWave);
  if (u >= U) return;
  const int lane = lane_id();
  int run = 0;
  for (int w0 = 0; w0 < W; w0 += kWave) {
    const int w = w0 + lane;
    const int c = w < W ? __popc(gbits[(size_t)u * W + w]) : 0;
    int x = c;  // inclusive scan over the lanes
    for (int d = 1; d < kWave; d <<= 1) {
      const int y = __shfl_up(x, d, kWave);
      if (lane >= d) x += y;
    }
    if (w < W) ppre[(size_t)u * W + w] = run + x - c;
    run += __shfl(x, kWave - 1, kWave);
  }
  if (lane == 0) cnt[u] = run;
}

// one thread per (instance, word): the pairs of the word's gate bits, in detection order
__global__ void k_pair_list(int U, int W, const uint32_t* gbits, const int32_t* poff, const int32_t* ppre,
                            int32_t* pu, int32_t* pi) {
  const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (int64_t)U * W) return;
  const int u = (int)(t / W), w = (int)(t % W);
  uint32_t b = gbits[t];
  int pos = poff[u] + ppre[t];
  while (b) {
    pu[pos] = u;
    pi[pos] = w * 32 + __ffs(b) - 1;
    ++pos;
    b &= b - 1;
  }
}

// existence probability of every label slot: partial sums over chunks of kSlotChunk hypotheses
constexpr int kSlotChunk = 16;
__global__ void k_slot_part(int H, int NS, int SW, const int32_t* rows, const float* logw, float* part) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  const int ch = blockIdx.y;
  if (s >= NS) return;
  // the chunk's row entries and weights first (independent loads), then the sum in order
  int32_t id[kSlotChunk];
  float lw[kSlotChunk];
#pragma unroll
  for (int j = 0; j < kSlotChunk; ++j) {
    const int h = ch * kSlotChunk + j;
    id[j] = h < H ? rows[(size_t)h * SW + s] : -1;
    lw[j] = h < H ? logw[h] : -INFINITY;
  }
  float acc = 0.0f;
#pragma unroll
  for (int j = 0; j < kSlotChunk; ++j)
    if (id[j] >= 0) acc += __expf(lw[j]);
  part[(size_t)ch * NS + s] = acc;
}
// one wave per slot: the partial sums, lanes over the chunks, then a fixed butterfly
__global__ __launch_bounds__(256) void k_slot_final(int NS, int nch, const float* part, float* r) {
  const int s = (int)((blockIdx.x * (size_t)blockDim.x + threadIdx.x) / kWave);
  if (s >= NS) return;
  float acc = 0.0f;
  for (int ch = lane_id(); ch < nch; ch += kWave) acc += part[(size_t)ch * NS + s];
  for (int d = kWave / 2; d > 0; d >>= 1) acc += __shfl_xor(acc, d, kWave);
  if (lane_id() == 0) r[s] = acc;
}

__global__ void k_pair_feat(int n, const int32_t* pu, const int32_t* pi, const DInst* inst, const float2* z,
                            float sig2, const float* slot_r, const int32_t* slot_age, const int32_t* pcnt, float* feat,
                            int32_t* pair) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int u = pu[p], i = pi[p];
  const DInst x = inst[u];
  float f[kNFeat];
  pair_feature(x, z[i], sig2, slot_r[x.slot], (float)slot_age[x.slot], (float)pcnt[u], f);
#pragma unroll
  for (int k = 0; k < kNFeat; ++k) feat[(size_t)p * kNFeat + k] = f[k];
  pair[2 * (size_t)p] = x.src;
  pair[2 * (size_t)p + 1] = i;
}


// network score of every pair; with `remove`, pairs scoring below thr leave the gate, and the
// likelihood exp(phi) of a removed pair whose instance belongs to the most likely predicted
// hypothesis (row0) is added to its detection's removed mass (fixed point, so that the sum
// does not depend on the order of the atomic additions; zeroed with the detections)
__global__ __launch_bounds__(256) void k_prop_apply(const int32_t* np, const int32_t* pu, const int32_t* pi,
                                                    const DInst* inst,
                                                    const float2* z, float sig2, const float* slot_r,
                                                    const int32_t* slot_age, const int32_t* pcnt,
                                                    const float* params, Norm nm, float thr, int remove, int M,
                                                    int W, float* phi, uint32_t* gbits, float* logit_out,
                                                    int32_t* nremoved, const int32_t* row0,
                                                    unsigned long long* rmass) {
  __shared__ __align__(16) uint32_t sq[kNQ];
  const int n = *np;
  if ((int)(blockIdx.x * blockDim.x) >= n) return;  // the grid covers an upper bound
  load_params_q(params, sq);
  const int lane = lane_id();
  // workgroups take chunks of blockDim pairs in turn (the parameters are loaded once)
  for (int p0 = blockIdx.x * blockDim.x; p0 < n; p0 += gridDim.x * blockDim.x) {
    const int p = p0 + threadIdx.x;
    const bool valid = p < n;
    // every lane takes part in the network (a lane without a pair scores zero features)
    int u = 0, i = 0, slot = 0;
    float f[kNFeat] = {0.0f, 0.0f, 0.0f, 0.0f, 0.0f, 0.0f};
    if (valid) {
      u = pu[p];
      i = pi[p];
      const DInst x = inst[u];
      slot = x.slot;
      pair_feature(x, z[i], sig2, slot_r[x.slot], (float)slot_age[x.slot], (float)pcnt[u], f);
    }
    const float s = mlp_logit_mfma(sq, f, nm);
    bool rm = false;
    if (valid) {
      if (logit_out) logit_out[p] = s;
      if (remove && s < thr) {
        rm = true;
        if (rmass && row0[slot] == u)
          atomicAdd(&rmass[i], (unsigned long long)(expf(phi[(size_t)u * M + i]) * kRemovedScale));
        phi[(size_t)u * M + i] = -INFINITY;
      }
    }
    // the removed pairs' gate bits: the pairs are listed by (instance, detection), so the lanes
    // of one gate word are adjacent; each run's first lane clears the run's bits with one atomic
    const int key = valid ? u * W + (i >> 5) : INT32_MAX;
    uint32_t bits = rm ? (1u << (i & 31)) : 0u;
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
      const uint32_t ob = __shfl_down(bits, d, kWave);
      const int ok = __shfl_down(key, d, kWave);
      if (lane + d < kWave && ok == key) bits |= ob;
    }
    const int pk = __shfl_up(key, 1, kWave);
    if (valid && bits && (lane == 0 || pk != key)) atomicAnd(&gbits[key], ~bits);
    const uint64_t b = __ballot(rm);
    if (lane == 0 && b) atomicAdd(nremoved, (int32_t)__popcll(b));
  }
}

// ------------------------------------------------------------------ lost mass
// One block per hypothesis (as the association kernel).  Per cell: the log-sum-exp over all
// options and, for each threshold j, over the options kept at j (clutter is always kept);
// per hypothesis: lz_full = log w - gamma (n - n_0) + sum_i (l_i - c_i) and
// dlt[j] = sum_i (l_ij - l_i), the log of the kept share of the hypothesis' children.
__global__ __launch_bounds__(256) void k_assoc_lost(int M, int stride, const int32_t* rows, const float* logw,
                                                    const int32_t* ntrk, float gamma, float lgk, const int32_t* coff,
                                                    const int32_t* cand, const float* phi, const uint32_t* cmax,
                                                    int W, const uint32_t* gbits, const int32_t* ppre,
                                                    const int32_t* poff, const float* plogit, int T, Thr thr, int H,
                                                    float* lz_full, float* dlt) {
  extern __shared__ int32_t row[];
  __shared__ float red[(kMaxThr + 1) * 4];
  const int h = blockIdx.x;
  for (int s = threadIdx.x; s < stride; s += blockDim.x) row[s] = rows[(size_t)h * stride + s];
  __syncthreads();
  float lsum = 0.0f;
  float dsum[kMaxThr];
#pragma unroll
  for (int j = 0; j < kMaxThr; ++j) dsum[j] = 0.0f;
  for (int i = threadIdx.x; i < M; i += blockDim.x) {
    const float c = o2f(cmax[i]);
    float mx = lgk, mj[kMaxThr];
#pragma unroll
    for (int j = 0; j < kMaxThr; ++j) mj[j] = lgk;
    const int e1 = coff[i + 1];
    const int w = i >> 5;
    const uint32_t below = (1u << (i & 31)) - 1u;
    for (int e = coff[i]; e < e1; ++e) {
      const int u = row[cand[e]];
      if (u < 0) continue;
      const float f = phi[(size_t)u * M + i];
      if (!(f > -INFINITY)) continue;
      const float s = plogit[poff[u] + ppre[(size_t)u * W + w] + __popc(gbits[(size_t)u * W + w] & below)];
      mx = fmaxf(mx, f);
#pragma unroll
      for (int j = 0; j < kMaxThr; ++j)
        if (j < T && s >= thr.t[j]) mj[j] = fmaxf(mj[j], f);
    }
    float sm = __expf(lgk - mx), sj[kMaxThr];
#pragma unroll
    for (int j = 0; j < kMaxThr; ++j) sj[j] = __expf(lgk - mj[j]);
    for (int e = coff[i]; e < e1; ++e) {
      const int u = row[cand[e]];
      if (u < 0) continue;
      const float f = phi[(size_t)u * M + i];
      if (!(f > -INFINITY)) continue;
      const float s = plogit[poff[u] + ppre[(size_t)u * W + w] + __popc(gbits[(size_t)u * W + w] & below)];
      sm += __expf(f - mx);
#pragma unroll
      for (int j = 0; j < kMaxThr; ++j)
        if (j < T && s >= thr.t[j]) sj[j] += __expf(f - mj[j]);
    }
    const float l = mx + __logf(sm);
    lsum += l - c;
#pragma unroll
    for (int j = 0; j < kMaxThr; ++j)
      if (j < T) dsum[j] += (mj[j] + __logf(sj[j])) - l;
  }
  lsum = wsum(lsum, red);
#pragma unroll
  for (int j = 0; j < kMaxThr; ++j)
    if (j < T) dsum[j] = wsum(dsum[j], red + 4 * (j + 1));
  if (threadIdx.x == 0) {
    lz_full[h] = logw[h] - gamma * (float)(ntrk[h] - ntrk[0]) + lsum;
    for (int j = 0; j < T; ++j) dlt[(size_t)j * H + h] = fminf(dsum[j], 0.0f);
  }
}

// one block: lost[j] = sum_h pi_h (1 - exp(dlt[j][h])), pi_h = exp(lz_full[h] - LSE lz_full)
__global__ __launch_bounds__(1024) void k_lost_final(int H, int T, const float* lz_full, const float* dlt,
                                                     float* lost) {
  __shared__ float red[32];
  float mx = -INFINITY;
  for (int h = threadIdx.x; h < H; h += blockDim.x) mx = fmaxf(mx, lz_full[h]);
  for (int d = kWave / 2; d > 0; d >>= 1) mx = fmaxf(mx, __shfl_xor(mx, d, kWave));
  if (lane_id() == 0) red[threadIdx.x / kWave] = mx;
  __syncthreads();
  mx = -INFINITY;
  for (int j = 0; j < (int)(blockDim.x / kWave); ++j) mx = fmaxf(mx, red[j]);
  __syncthreads();
  float sm = 0.0f;
  for (int h = threadIdx.x; h < H; h += blockDim.x) sm += __expf(lz_full[h] - mx);
  sm = wsum(sm, red + 16);
  const float L = mx + __logf(sm);
  for (int j = 0; j < T; ++j) {
    float a = 0.0f;
    for (int h = threadIdx.x; h < H; h += blockDim.x)
      a += __expf(lz_full[h] - L) * -expm1f(dlt[(size_t)j * H + h]);
    a = wsum(a, red + 16);
    // a mass fraction: FP32 rounding of the normalised weights can take the sum just outside [0, 1]
    if (threadIdx.x == 0) lost[j] = fminf(fmaxf(a, 0.0f), 1.0f);
  }
}

// ------------------------------------------------------------------ training targets
// partial association masses over chunks of 256 hypotheses, one thread per (instance, chunk):
// pm[ch][p] = sum over h in the chunk holding u of pi_h exp(phi_ui - LSE_hi), pe[ch][u] = sum of pi_h
__global__ void k_pair_mass(int U, int H, int M, int SW, const DInst* inst, const int32_t* rows, const float* logpi,
                            CellView cv, const uint32_t* cmax, const float* phi, const int32_t* poff,
                            const int32_t* pi, int npairs, float* pm, float* pe) {
  const int u = blockIdx.x * blockDim.x + threadIdx.x;
  const int ch = blockIdx.y;
  if (u >= U) return;
  const int slot = inst[u].slot;
  const int p0 = poff[u], p1 = poff[u + 1];
  float* out = pm + (size_t)ch * npairs;
  for (int p = p0; p < p1; ++p) out[p] = 0.0f;
  float e = 0.0f;
  const int h1 = min(H, (ch + 1) * 256);
  for (int h = ch * 256; h < h1; ++h) {
    if (rows[(size_t)h * SW + slot] != u) continue;
    const float w = __expf(logpi[h]);
    e += w;
    for (int p = p0; p < p1; ++p) {
      const int i = pi[p];
      out[p] += w * __expf(phi[(size_t)u * M + i] - (cv.lserel[cv.at(h, i)] + o2f(cmax[i])));
    }
  }
  pe[(size_t)ch * U + u] = e;
}

__global__ void k_pair_target(int n, int U, int nch, const int32_t* pu, const float* pm, const float* pe, float* y,
                              float* w) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= n) return;
  const int u = pu[p];
  float m = 0.0f, e = 0.0f;
  for (int ch = 0; ch < nch; ++ch) {
    m += pm[(size_t)ch * n + p];
    e += pe[(size_t)ch * U + u];
  }
  w[p] = e;
  y[p] = e > 0.0f ? fminf(fmaxf(m / e, 0.0f), 1.0f) : 0.0f;
}

// ------------------------------------------------------------------ network kernels
__global__ __launch_bounds__(256) void k_mlp_fwd(int n, const float* feat, const float* params, Norm nm,
                                                 float* logit) {
  __shared__ __align__(16) uint32_t sq[kNQ];
  load_params_q(params, sq);
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  float f[kNFeat];
#pragma unroll
  for (int k = 0; k < kNFeat; ++k) f[k] = p < n ? feat[(size_t)p * kNFeat + k] : 0.0f;
  const float s = mlp_logit_mfma(sq, f, nm);  // every lane of the wave
  if (p < n) logit[p] = s;
}

// One wave per 64 samples: forward, loss, backward to per-sample vectors in LDS, then the
// wave's partial sums of every gradient entry in sample order.  LDS: parameters | xs[6][65] |
// h1[64][65] | h2[64][65] | da1[64][65] | da2[64][65] | ds[64] | w l[64] | w[64].
__global__ __launch_bounds__(64) void k_mlp_fb(int n, const float* feat, const float* y, const float* wt,
                                               const float* params, Norm nm, float* part) {
  extern __shared__ float lds[];
  float* sw = lds;
  float* Lxs = sw + kNParam + 3;
  float* Lh1 = Lxs + kNFeat * kLS;
  float* Lh2 = Lh1 + kNHid * kLS;
  float* Lda1 = Lh2 + kNHid * kLS;
  float* Lda2 = Lda1 + kNHid * kLS;
  float* Lds = Lda2 + kNHid * kLS;
  float* Lwl = Lds + 64;
  float* Lw = Lwl + 64;
  load_params(params, sw);
  const int s = threadIdx.x;
  const int q = blockIdx.x * 64 + s;
  const bool valid = q < n;
  float x[kNFeat], xs[kNFeat], h1[kNHid], dh1[kNHid];
#pragma unroll
  for (int k = 0; k < kNFeat; ++k) x[k] = valid ? feat[(size_t)q * kNFeat + k] : nm.mu[k];
  const float w = valid ? wt[q] : 0.0f;
  const float yy = valid ? y[q] : 0.0f;
  standardise(x, nm, xs);
#pragma unroll
  for (int k = 0; k < kNFeat; ++k) Lxs[k * kLS + s] = xs[k];
  layer1(sw, xs, h1);
#pragma unroll
  for (int k = 0; k < kNHid; ++k) Lh1[k * kLS + s] = h1[k];
  float sc = sw[oB3];
  for (int j = 0; j < kNHid; ++j) {
    const float h2 = bf16r(fmaxf(layer2_unit(sw, h1, j), 0.0f));
    Lh2[j * kLS + s] = h2;
    sc = fmaf(sw[oW3 + j], h2, sc);
  }
  const float sig = 1.0f / (1.0f + expf(-sc));
  const float ds = w * (sig - yy);
  const float loss = w * (fmaxf(sc, 0.0f) + log1pf(expf(-fabsf(sc))) - yy * sc);
#pragma unroll
  for (int k = 0; k < kNHid; ++k) dh1[k] = 0.0f;
  for (int j = 0; j < kNHid; ++j) {
    const float da2 = Lh2[j * kLS + s] > 0.0f ? ds * sw[oW3 + j] : 0.0f;
    Lda2[j * kLS + s] = da2;
    const float* wr = sw + oW2 + j * kNHid;
#pragma unroll
    for (int k = 0; k < kNHid; ++k) dh1[k] = fmaf(da2, wr[k], dh1[k]);
  }
#pragma unroll
  for (int k = 0; k < kNHid; ++k) Lda1[k * kLS + s] = h1[k] > 0.0f ? dh1[k] : 0.0f;
  Lds[s] = ds;
  Lwl[s] = loss;
  Lw[s] = w;
  __syncthreads();
  float* out = part + (size_t)blockIdx.x * kPartW;
  for (int t = s; t < kPartW; t += 64) {
    float acc = 0.0f;
    if (t < oB1) {
      const float* a = Lda1 + (t / kNFeat) * kLS;
      const float* b = Lxs + (t % kNFeat) * kLS;
      for (int r = 0; r < 64; ++r) acc = fmaf(a[r], b[r], acc);
    } else if (t < oW2) {
      const float* a = Lda1 + (t - oB1) * kLS;
      for (int r = 0; r < 64; ++r) acc += a[r];
    } else if (t < oB2) {
      const int j = (t - oW2) / kNHid, k = (t - oW2) % kNHid;
      const float* a = Lda2 + j * kLS;
      const float* b = Lh1 + k * kLS;
      for (int r = 0; r < 64; ++r) acc = fmaf(a[r], b[r], acc);
    } else if (t < oW3) {
      const float* a = Lda2 + (t - oB2) * kLS;
      for (int r = 0; r < 64; ++r) acc += a[r];
    } else if (t < oB3) {
      const float* b = Lh2 + (t - oW3) * kLS;
      for (int r = 0; r < 64; ++r) acc = fmaf(Lds[r], b[r], acc);
    } else if (t == oB3) {
      for (int r = 0; r < 64; ++r) acc += Lds[r];
    } else if (t == kNParam) {
      for (int r = 0; r < 64; ++r) acc += Lw[r];
    } else {
      for (int r = 0; r < 64; ++r) acc += Lwl[r];
    }
    out[t] = acc;
  }
}

// gradient and loss: sums of the partials in block order, divided by the sum of the weights
__global__ void k_mlp_reduce(int nblk, const float* part, float* grad, float* loss) {
  const int t = blockIdx.x * blockDim.x + threadIdx.x;
  if (t > kNParam) return;
  float W = 0.0f, a = 0.0f;
  const int col = t < kNParam ? t : kNParam + 1;
  for (int b = 0; b < nblk; ++b) {
    W += part[(size_t)b * kPartW + kNParam];
    a += part[(size_t)b * kPartW + col];
  }
  if (t < kNParam) grad[t] = a / W;
  else *loss = a / W;
}

__global__ void k_adam(int n, float* th, float* m, float* v, const float* g, float lr, float b1, float b2, float eps,
                       float c1, float c2) {
  const int q = blockIdx.x * blockDim.x + threadIdx.x;
  if (q >= n) return;
  const float gg = g[q];
  const float mm = b1 * m[q] + (1.0f - b1) * gg;
  const float vv = b2 * v[q] + (1.0f - b2) * gg * gg;
  m[q] = mm;
  v[q] = vv;
  th[q] -= lr * (mm * c1) / (sqrtf(vv * c2) + eps);
}

// ------------------------------------------------------------------ host side
namespace {

Norm norm_of(const float* nm) {
  Norm n;
  for (int k = 0; k < kNFeat; ++k) {
    n.mu[k] = nm[k];
    n.sd[k] = nm[kNFeat + k];
  }
  return n;
}

// label existence and age of every slot (the network's inputs besides the pair's own)
}  // namespace

void prepare_slots(Ctx& c, int k, hipStream_t s) {
  const int T = 256;
  const int H = c.nhyp, NS = c.nslot, SW = c.stride;
  const int nch = cdiv(H, kSlotChunk);
  float* part = need<float>(c.slot_part, (int64_t)nch * std::max(NS, 1));
  float* r = need<float>(c.slot_r, NS + 1);
  if (NS > 0) {
    hipLaunchKernelGGL(k_slot_part, dim3(cdiv(NS, T), nch), dim3(T), 0, s, H, NS, SW, c.rows.as<int32_t>(),
                       c.logw.as<float>(), part);
    GLMB_HIP(hipGetLastError());
    GLMB_LAUNCH(k_slot_final, cdiv((int64_t)NS * kWave, T), T, 0, s, NS, nch, part, r);
  }
  if (c.age_cap < NS + 1) {  // pinned, so that the upload below does not wait for the stream
    if (c.age_pin) GLMB_HIP(hipHostFree(c.age_pin));
    c.age_pin = nullptr;
    c.age_cap = 0;
    GLMB_HIP(hipHostMalloc((void**)&c.age_pin, (size_t)2 * (NS + 1) * sizeof(int32_t), hipHostMallocDefault));
    c.age_cap = 2 * (NS + 1);
  }
  // every caller synchronises the stream before it can get here again (the update reads its
  // counts back, the lost-mass and feature calls their results), so no upload still reads it
  for (int j = 0; j < NS; ++j) c.age_pin[j] = k - c.slot_lab[j].first;
  int32_t* age = need<int32_t>(c.slot_age, NS + 1);
  if (NS) GLMB_HIP(hipMemcpyAsync(age, c.age_pin, NS * sizeof(int32_t), hipMemcpyHostToDevice, s));
}

namespace {

// label existence and ages, and the gated pairs listed by (instance, detection); returns their
// count (one round trip)
int prepare_pairs(Ctx& c, int k, int M) {
  hipStream_t s = c.s;
  const int T = 256;
  const int U = c.ninst;
  const int W = std::max(1, (M + 31) / 32);
  prepare_slots(c, k, s);
  int32_t* cnt = need<int32_t>(c.pcnt, U + 1);
  int32_t* off = need<int32_t>(c.poff, U + 1);
  int32_t* ppre = need<int32_t>(c.ppre, (int64_t)U * W);
  GLMB_LAUNCH(k_pair_count, cdiv((int64_t)U * kWave, T), T, 0, s, U, W, c.gbits.as<uint32_t>(), cnt, ppre);
  scan_excl(cnt, off, U, off + U, c.tmp, s);
  const int n = U > 0 ? (int)read_back(c.sb.hs, s, {{off + U, 1}})[0] : 0;
  int32_t* pu = need<int32_t>(c.pu, n);
  int32_t* pi = need<int32_t>(c.pi, n);
  GLMB_LAUNCH(k_pair_list, cdiv((int64_t)U * W, T), T, 0, s, U, W, c.gbits.as<uint32_t>(), off, ppre, pu, pi);
  return n;
}

// network scores of the listed pairs (into c.plogit unless removing), optionally removing the
// low ones; n < 0: the gate's pair list, whose count is on the device (scal[19]), and the grid
// covers at most U x M pairs
void score_pairs(Ctx& c, int n, int M, bool remove) {
  const int W = std::max(1, (M + 31) / 32);
  const int64_t cap = n >= 0 ? n : (int64_t)c.ninst * M;
  float* logit = remove ? nullptr : need<float>(c.plogit, cap);
  int32_t* nremoved = c.scal.as<int32_t>() + 18;
  const int grid = std::min(cdiv(cap, 256), 4096);
  unsigned long long* rmass = remove ? c.rmass.as<unsigned long long>() : nullptr;
  const int32_t* np = n >= 0 ? c.poff.as<int32_t>() + c.ninst : c.scal.as<int32_t>() + 19;
  GLMB_LAUNCH(k_prop_apply, grid, 256, 0, c.s, np, c.pu.as<int32_t>(), c.pi.as<int32_t>(),
              (const DInst*)c.inst.p, c.z.as<float2>(), c.p.sigma_z * c.p.sigma_z, c.slot_r.as<float>(),
              c.slot_age.as<int32_t>(), c.pcnt.as<int32_t>(), c.prop_w.as<float>(), norm_of(c.prop_norm),
              c.prop_thr, remove ? 1 : 0, M, W, c.phi.as<float>(), c.gbits.as<uint32_t>(), logit, nremoved,
              c.rows.as<int32_t>(), rmass);
}
}  // namespace

void proposal_apply(Ctx& c, int k, int M, bool slots_ready) {
  trace(c, "update.proposal");
  // the gate listed the pairs (count at scal[19]) and the per-instance counts
  if (slots_ready) GLMB_HIP(hipStreamWaitEvent(c.s, c.fork[2], 0));
  else prepare_slots(c, k, c.s);
  score_pairs(c, -1, M, true);
}

void proposal_lost(Ctx& c, int k, const float* zin, int M, const float* thr_prob, int T, double* lost) {
  if (T < 1 || T > kMaxThr) throw Error{GLMB_E_ARG, "1 <= T <= 16 thresholds"};
  Thr thr{};
  for (int j = 0; j < T; ++j) {
    const double t = thr_prob[j];
    if (!(t > 0.0 && t < 1.0)) throw Error{GLMB_E_ARG, "thresholds must lie in (0, 1)"};
    thr.t[j] = (float)std::log(t / (1.0 - t));
  }
  hipStream_t s = c.s;
  const int H = c.nhyp, SW = c.stride;
  gate_scores(c, zin, M);
  gate_lists(c, M);
  const int n = prepare_pairs(c, k, M);
  score_pairs(c, n, M, false);
  float* lzf = need<float>(c.lz_t, (int64_t)(T + 1) * H + 32);
  float* dlt = lzf + H;
  float* out = dlt + (size_t)T * H;
  const int W = std::max(1, (M + 31) / 32);
  GLMB_LAUNCH(k_assoc_lost, H, 256, SW * sizeof(int32_t), s, M, SW, c.rows.as<int32_t>(), c.logw.as<float>(),
              c.ntrk.as<int32_t>(), c.p.det_rate, logf(c.p.clutter_density), c.coff.as<int32_t>(),
              c.cand.as<int32_t>(), c.phi.as<float>(), c.cmax.as<uint32_t>(), W, c.gbits.as<uint32_t>(),
              c.ppre.as<int32_t>(), c.poff.as<int32_t>(), c.plogit.as<float>(), T, thr, H, lzf, dlt);
  GLMB_LAUNCH(k_lost_final, 1, 1024, 0, s, H, T, lzf, dlt, out);
  float h[kMaxThr];
  std::memcpy(h, read_back(c.sb.hs, s, {{out, T}}), (size_t)T * sizeof(float));
  for (int j = 0; j < T; ++j) lost[j] = h[j];
  c.last_M = -1;  // the update diagnostics buffers no longer describe an update
}

int proposal_features(Ctx& c, int k, const float* zin, int M, int cap, float* feat, int32_t* pair, float* target,
                      float* weight) {
  hipStream_t s = c.s;
  const int T = 256;
  const int H = c.nhyp, U = c.ninst, SW = c.stride;
  gate_scores(c, zin, M);
  gate_lists(c, M);
  assoc_norm(c, M);
  c.last_M = -1;
  const int n = prepare_pairs(c, k, M);
  if (n > cap) return n;
  if (n == 0) return 0;
  GLMB_LAUNCH(k_pair_feat, cdiv(n, T), T, 0, s, n, c.pu.as<int32_t>(), c.pi.as<int32_t>(), (const DInst*)c.inst.p,
              c.z.as<float2>(), c.p.sigma_z * c.p.sigma_z, c.slot_r.as<float>(), c.slot_age.as<int32_t>(),
              c.pcnt.as<int32_t>(), feat, pair);
  const int nch = cdiv(H, 256);
  float* pm = need<float>(c.pm_part, (int64_t)nch * n);
  float* pe = need<float>(c.pe_part, (int64_t)nch * std::max(U, 1));
  hipLaunchKernelGGL(k_pair_mass, dim3(cdiv(U, T), nch), dim3(T), 0, s, U, H, M, SW, (const DInst*)c.inst.p,
                     c.rows.as<int32_t>(), c.diag_logpi.as<float>(), cells_of(c, M), c.cmax.as<uint32_t>(),
                     c.phi.as<float>(), c.poff.as<int32_t>(), c.pi.as<int32_t>(), n, pm, pe);
  GLMB_HIP(hipGetLastError());
  GLMB_LAUNCH(k_pair_target, cdiv(n, T), T, 0, s, n, U, nch, c.pu.as<int32_t>(), pm, pe, target, weight);
  GLMB_HIP(stream_sync(s));
  return n;
}

void mlp_forward(Ctx& c, const float* params, const float* norm, const float* feat, int n, float* logit) {
  GLMB_LAUNCH(k_mlp_fwd, cdiv(n, 256), 256, 0, c.s, n, feat, params, norm_of(norm), logit);
}

namespace {

// Partial sums of glmb_mlp_grad_noalloc: one row of kPartW floats per 64-sample workgroup.
// Host code never names this array: it uses the address noalloc_setup looked up per device.
constexpr int kNoAllocBlocks = GLMB_MLP_NOALLOC_MAX / 64;
static_assert(GLMB_MLP_NOALLOC_MAX % 64 == 0, "whole workgroups");
__device__ __align__(256) float scratch[(size_t)kNoAllocBlocks * kPartW];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
float* g_scratch[kMaxDevices] = {};  // device address of `scratch` on each device

void mlp_grad_launch(Ctx& c, const float* params, const float* norm, const float* feat, const float* y,
                     const float* w, int n, float* grad, float* loss, float* part) {
  const int nblk = std::max(1, cdiv(n, 64));
  const size_t lds = (size_t)(kNParam + 3 + kNFeat * kLS + 4 * kNHid * kLS + 3 * 64) * sizeof(float);
  static_assert((kNParam + 3 + kNFeat * kLS + 4 * kNHid * kLS + 3 * 64) * 4 <= 160 * 1024, "LDS of k_mlp_fb");
  GLMB_HIP(hipFuncSetAttribute((const void*)k_mlp_fb, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
  GLMB_LAUNCH(k_mlp_fb, nblk, 64, lds, c.s, n, feat, y, w, params, norm_of(norm), part);
  GLMB_LAUNCH(k_mlp_reduce, cdiv(kNParam + 1, 256), 256, 0, c.s, nblk, part, grad, loss);
}

}  // namespace

void mlp_grad(Ctx& c, const float* params, const float* norm, const float* feat, const float* y, const float* w,
              int n, float* grad, float* loss) {
  const int nblk = std::max(1, cdiv(n, 64));
  float* part = need<float>(c.mlp_part, (int64_t)nblk * kPartW);
  mlp_grad_launch(c, params, norm, feat, y, w, n, grad, loss, part);
}

void noalloc_setup(int device) {
  if (device < 0 || device >= kMaxDevices) throw Error{GLMB_E_DEVICE, "device index beyond the supported 64"};
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[device]) return;
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    throw Error{GLMB_E_DEVICE, std::string("hipGetSymbolAddress of the gradient scratch array: ") + hipGetErrorString(e)};
  g_scratch[device] = (float*)p;
}

void mlp_grad_noalloc(Ctx& c, const float* params, const float* norm, const float* feat, const float* y,
                      const float* w, int n, float* grad, float* loss) {
  float* part = (c.device >= 0 && c.device < kMaxDevices) ? g_scratch[c.device] : nullptr;
  if (!part) throw Error{GLMB_E_STATE, "gradient scratch array not set up on this device"};
  // every row the reduction reads (one per workgroup of this call) is written first by k_mlp_fb
  mlp_grad_launch(c, params, norm, feat, y, w, n, grad, loss, part);
}

void mlp_adam(Ctx& c, float* params, float* m, float* v, const float* g, int t, float lr, float b1, float b2,
              float eps) {
  const float c1 = (float)(1.0 / (1.0 - std::pow((double)b1, (double)t)));
  const float c2 = (float)(1.0 / (1.0 - std::pow((double)b2, (double)t)));
  GLMB_LAUNCH(k_adam, cdiv(kNParam, 256), 256, 0, c.s, kNParam, params, m, v, g, lr, b1, b2, eps, c1, c2);
}

}  // namespace glmb
