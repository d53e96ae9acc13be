// Radiance-cache kernels for gfx950: BF16 matrix-core inference and training.
//
// k_nrc_pack      FP32 master weights -> bf16 operand fragments (forward and
//                 transposed for the backward pass), in the chained K order;
//                 FP32 inference weights -> forward fragments of the queries.
// k_nrc_infer     encode + 6 layers per 32 queries per wave, weights in LDS.
// k_nrc_fwd_bwd   forward with kept activations, relative-L2 loss gradient,
//                 backward through the transposed fragments; writes layer
//                 inputs and layer output gradients (bf16, [feature][sample]).
// k_nrc_dw        dW_l = g_l^T a_l as a matrix-core GEMM over samples, split
//                 over sample ranges; partial tiles in FP32.
// k_nrc_adam      fixed-order sum of the partials, Adam with FP32 master weights,
//                 moving average of the weights for inference.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>

#include "pt_internal.h"
#include "pt_nrc.h"

namespace pt {

typedef __bf16 bf16x8 __attribute__((__vector_size__(8 * sizeof(__bf16))));
typedef float f32x4 __attribute__((__vector_size__(4 * sizeof(float))));

__device__ inline bf16x8 as_bf16x8(uint4 u) { return __builtin_bit_cast(bf16x8, u); }

__device__ inline f32x4 mfma(bf16x8 a, bf16x8 b, f32x4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

typedef __bf16 bf16x2 __attribute__((ext_vector_type(2)));

// Two floats to bfloat16 (round to nearest even) in one v_cvt_pk_bf16_f32;
// for finite values the same bits as bf16_bits().
__device__ inline uint32_t pack2(float a, float b) {
  bf16x2 v = {(__bf16)a, (__bf16)b};
  return __builtin_bit_cast(uint32_t, v);
}

typedef short i16x2 __attribute__((ext_vector_type(2)));

// ReLU of a packed bfloat16 pair: a bfloat16 with its sign bit set is a
// negative int16, so an int16 maximum with 0 zeroes exactly the negative
// values and -0 (v_pk_max_i16).  Equal to rounding max(x, 0) for every
// non-NaN x, since rounding to nearest is monotonic and keeps the sign.
__device__ inline uint32_t relu2(uint32_t u) {
  // An empty asm statement keeps u one 32-bit register, so that the pair is
  // converted by one v_cvt_pk_bf16_f32 (seen through, the conversion was
  // split into two and a permute).
  asm("" : "+v"(u));
  i16x2 v = __builtin_bit_cast(i16x2, u);
  v = __builtin_elementwise_max(v, i16x2{0, 0});
  return __builtin_bit_cast(uint32_t, v);
}

// B operand of a chained chunk from two result tiles, with ReLU.
__device__ inline bf16x8 chain_relu(f32x4 lo, f32x4 hi) {
  uint4 u;
  u.x = relu2(pack2(lo[0], lo[1]));
  u.y = relu2(pack2(lo[2], lo[3]));
  u.z = relu2(pack2(hi[0], hi[1]));
  u.w = relu2(pack2(hi[2], hi[3]));
  return as_bf16x8(u);
}

__device__ inline float bf16x8_get(bf16x8 v, int j) { return (float)v[j]; }

// --------------------------------------------------------------- packing
// Training fragments (forward and transposed) from the weights w, and the
// inference fragments (forward layout) from the inference weights wi.
// Also counts the Adam step just applied (t_step, when given), unless the
// batch had no records (n_records given and zero): the step then left the
// weights and moments unchanged and is not counted.
__global__ void k_nrc_pack(const float* __restrict__ w, const float* __restrict__ wi, uint4* __restrict__ fwd,
                           uint4* __restrict__ bwd, uint4* __restrict__ inf, uint32_t* __restrict__ t_step,
                           const uint32_t* __restrict__ n_records) {
  int id = blockIdx.x * blockDim.x + threadIdx.x;
  if (id == 0 && t_step && (!n_records || *n_records > 0u)) *t_step += 1u;
  int total = (2 * kNrcFwdFrags + kNrcBwdFrags) * 64;
  if (id >= total) return;
  int frag = id / 64, lane = id % 64, g = lane / 16, r = lane % 16;
  const bool to_inf = frag >= kNrcFwdFrags + kNrcBwdFrags;
  if (to_inf) {
    frag -= kNrcFwdFrags + kNrcBwdFrags;
    w = wi;
  }
  float v[8];
  if (frag < kNrcFwdFrags) {
    if (frag < 40) {
      int l = frag / 8, t = (frag % 8) / 2, c = frag % 2;
      for (int j = 0; j < 8; ++j) {
        int in = l == 0 ? nrc_k_in(c, g, j) : nrc_k_chained(c, g, j);
        v[j] = w[nrc_widx(l, 16 * t + r, in)];
      }
    } else {
      int c = frag - 40;
      for (int j = 0; j < 8; ++j) v[j] = r < 3 ? w[nrc_widx(5, r, nrc_k_chained(c, g, j))] : 0.0f;
    }
  } else {
    int f = frag - kNrcFwdFrags;
    if (f < 32) {
      int l = 1 + f / 8, t = (f % 8) / 2, c = f % 2;
      for (int j = 0; j < 8; ++j) v[j] = w[nrc_widx(l, nrc_k_chained(c, g, j), 16 * t + r)];
    } else {
      int t = f - 32;
      for (int j = 0; j < 8; ++j) {
        int k = 8 * g + j;
        v[j] = k < 3 ? w[nrc_widx(5, k, 16 * t + r)] : 0.0f;
      }
    }
  }
  uint4 u;
  u.x = pack2(v[0], v[1]);
  u.y = pack2(v[2], v[3]);
  u.z = pack2(v[4], v[5]);
  u.w = pack2(v[6], v[7]);
  if (to_inf) inf[frag * 64 + lane] = u;
  else if (frag < kNrcFwdFrags) fwd[frag * 64 + lane] = u;
  else bwd[(frag - kNrcFwdFrags) * 64 + lane] = u;
}

// Encoded input as the layer-0 B operand: lane (g, q) holds the features
// nrc_k_in(c, g, j) of query q.  Every lane runs the same instructions (no
// per-lane branch on the feature index): five sin/cos pairs, the four
// one-blob bins of one direction coordinate, one roughness bin and two
// copied values, with lane-dependent arguments chosen by selects.
// Lane-dependent choice among registers, written as a sum of selects against
// zero so the compiler keeps the inputs in registers (a select between two
// array loads would become an indexed load from a stack copy).
__device__ inline float pick3(int a, float v0, float v1, float v2) {
  return ((a == 0 ? v0 : 0.0f) + (a == 1 ? v1 : 0.0f)) + (a == 2 ? v2 : 0.0f);
}

__device__ inline float pick4(int a, float v0, float v1, float v2, float v3) {
  return ((a == 0 ? v0 : 0.0f) + (a == 1 ? v1 : 0.0f)) + ((a == 2 ? v2 : 0.0f) + (a == 3 ? v3 : 0.0f));
}

__device__ inline void encode_operand(const float* x, int g, bf16x8 B[2]) {
  // sincospif shares one argument reduction between sin and cos; its results
  // are bitwise those of sinpif and cospif (checked on 2^24 arguments of the
  // form u 2^k, k = 0..5, and quarter integers).
  float f0[8];
  // pairs 4g, 4g + 1 share an axis, and so do pairs 4g + 2, 4g + 3 (p = 6a + k)
  const float xa01 = pick3(g < 2 ? 0 : g - 1, x[0], x[1], x[2]);
  const float xa23 = pick3(g == 0 ? 0 : (g < 3 ? 1 : 2), x[0], x[1], x[2]);
#pragma unroll
  for (int m = 0; m < 4; ++m) {  // pair p = 4g + m: sin and cos of 2^k pi x_a
    const int k = (4 * g + m) % 6;
    const float w = (m < 2 ? xa01 : xa23) * (float)(1 << k);
    sincospif(w, &f0[2 * m], &f0[2 * m + 1]);
  }
  float f1[8];
  {  // feature 32 + g: sin (g even) or cos (g odd) of 16 pi x2 (g < 2) or 32 pi x2
    const float w = x[2] * (float)(16 << (g >> 1));
    float sv, cv;
    sincospif(w, &sv, &cv);
    f1[0] = (g & 1) ? cv : sv;
  }
  {  // features 36 + 4g + i: one-blob bins of direction coordinate g (x3..x6; x4 and x6 are periodic)
    const float sd = pick4(g, x[3], x[4], x[5], x[6]);
    const bool periodic = (g & 1) != 0;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      float d = sd - ((float)i + 0.5f) * 0.25f;
      if (periodic) d -= floorf(d + 0.5f);
      const float z = d * 4.0f;
      f1[1 + i] = expf(-0.5f * z * z);
    }
  }
  {  // feature 52 + g: bin g of 1 - exp(-roughness)
    const float rr = 1.0f - expf(-x[7]);
    const float z = (rr - ((float)g + 0.5f) * 0.25f) * 4.0f;
    f1[5] = expf(-0.5f * z * z);
  }
  // features 56 + 2g, 57 + 2g: albedos x8..x11, then the constants 1, 0, 0, 0
  f1[6] = pick4(g, x[8], x[10], 1.0f, 0.0f);
  f1[7] = pick4(g, x[9], x[11], 0.0f, 0.0f);
  uint4 u0, u1;
  u0.x = pack2(f0[0], f0[1]);
  u0.y = pack2(f0[2], f0[3]);
  u0.z = pack2(f0[4], f0[5]);
  u0.w = pack2(f0[6], f0[7]);
  u1.x = pack2(f1[0], f1[1]);
  u1.y = pack2(f1[2], f1[3]);
  u1.z = pack2(f1[4], f1[5]);
  u1.w = pack2(f1[6], f1[7]);
  B[0] = as_bf16x8(u0);
  B[1] = as_bf16x8(u1);
}

// Five hidden layers and the output layer; returns the output tile (rows 0..2 valid in lanes g == 0).
__device__ inline f32x4 mlp_forward(const uint4* __restrict__ sw, int lane, bf16x8 B[2], bf16x8* keep) {
  if (keep) {
    keep[0] = B[0];
    keep[1] = B[1];
  }
#pragma unroll
  for (int l = 0; l < 5; ++l) {
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
      for (int c = 0; c < 2; ++c) acc[t] = mfma(as_bf16x8(sw[((l * 4 + t) * 2 + c) * 64 + lane]), B[c], acc[t]);
    }
    B[0] = chain_relu(acc[0], acc[1]);
    B[1] = chain_relu(acc[2], acc[3]);
    if (keep) {
      keep[2 * (l + 1)] = B[0];
      keep[2 * (l + 1) + 1] = B[1];
    }
  }
  f32x4 out = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
  for (int c = 0; c < 2; ++c) out = mfma(as_bf16x8(sw[(40 + c) * 64 + lane]), B[c], out);
  return out;
}

// Reflectance factor of a query's inputs: the cache predicts radiance divided
// by (diffuse albedo + specular albedo) per channel when factorising.
__device__ inline float nrc_factor(const float* x, int c, bool on) { return on ? x[8 + c] + x[11] : 1.0f; }

// ------------------------------------------------------------- inference
// MODE 0: inputs x[n][12], outputs y[n][3].
// MODE 1: the cache queries of a sampling pass: slot = q_nrc[i] for i < counts[kCountQuery];
//         inputs nrc_q[slot][0..11], throughput nrc_q[slot][12..14]; L[slot] += beta * factor * max(y, 0).
// MODE 2: the terminal vertices of n training paths (self-training): path k's record at vertex
//         P.train_end, if it is a terminal record, gives out4[k] = beta * factor * max(y, 0); else 0.
// A wave takes 32 queries per iteration, two groups of 16, so that every
// weight fragment read from LDS feeds two matrix-core instructions.
constexpr int kInferWaves = 8;  // waves per workgroup sharing one LDS copy of the weight fragments
constexpr int kInferSub = 2;    // groups of 16 queries per wave and iteration

// The 12 inputs of query row qc (always a valid row: callers clamp), as
// float4 loads where the rows are 16-byte aligned by construction.
template <int MODE>
__device__ inline const float* infer_row(const float* xin, const PathsDev& P, int64_t qc, uint32_t& slot) {
  if (MODE == 0) return xin + qc * 12;
  if (MODE == 1) {
    slot = P.q_nrc[qc];
    return P.nrc_q + (size_t)slot * kNrcQueryFloats;
  }
  return P.rec + ((size_t)qc * P.rec_depth + P.train_end) * kNrcRecFloats;
}

template <int MODE>
__device__ inline void infer_load(const float* r, float* x) {
  if (MODE == 0) {  // caller's rows of 48 bytes: only 4-byte alignment is known
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = r[k];
  } else {
    const float4* r4 = reinterpret_cast<const float4*>(r);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const float4 v = r4[k];
      x[4 * k] = v.x;
      x[4 * k + 1] = v.y;
      x[4 * k + 2] = v.z;
      x[4 * k + 3] = v.w;
    }
  }
}

template <int MODE>
__global__ __launch_bounds__(64 * kInferWaves) void k_nrc_infer(const float* __restrict__ xin, int64_t n_arg,
                                                                PathsDev P, const uint4* __restrict__ fwd,
                                                                float* __restrict__ out) {
  __shared__ uint4 sw[kNrcFwdFrags * 64];
  const int64_t n = MODE == 1 ? (int64_t)P.counts[kCountQuery] : n_arg;
  if (MODE == 1 && blockIdx.x == 0 && threadIdx.x == 0) atomicAdd(&P.stats[kStatQueries], (unsigned long long)n);
  constexpr int kPerIter = 16 * kInferSub;
  if ((int64_t)blockIdx.x * kInferWaves * kPerIter >= n) return;  // no work: skip staging the weights
  for (int i = threadIdx.x; i < kNrcFwdFrags * 64; i += blockDim.x) sw[i] = fwd[i];
  __syncthreads();
  float4* out4 = reinterpret_cast<float4*>(out);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, g = lane / 16, q = lane % 16;
  unsigned long long nonfinite = 0;
  for (int64_t it = (int64_t)blockIdx.x * kInferWaves + wave; it * kPerIter < n;
       it += (int64_t)gridDim.x * kInferWaves) {
    // Read the weight fragments from LDS in every iteration: held in
    // registers they would take 168 VGPRs and leave one wave per SIMD.
    asm volatile("" ::: "memory");
    int64_t qi[kInferSub];
    bool valid[kInferSub];
    const float* r[kInferSub];
    uint32_t slot[kInferSub];
    float x[kInferSub][12];
    bf16x8 B[kInferSub][2];
#pragma unroll
    for (int h = 0; h < kInferSub; ++h) {
      qi[h] = it * kPerIter + 16 * h + q;
      valid[h] = qi[h] < n;
      slot[h] = 0;
      // rows past n read row n - 1 (their results are dropped), so every load is in bounds
      r[h] = infer_row<MODE>(xin, P, valid[h] ? qi[h] : n - 1, slot[h]);
      infer_load<MODE>(r[h], x[h]);
      encode_operand(x[h], g, B[h]);
    }
    f32x4 acc[kInferSub][4];
#pragma unroll
    for (int l = 0; l < 5; ++l) {
#pragma unroll
      for (int t = 0; t < 4; ++t) {
#pragma unroll
        for (int h = 0; h < kInferSub; ++h) acc[h][t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < 2; ++c) {
          const bf16x8 a = as_bf16x8(sw[((l * 4 + t) * 2 + c) * 64 + lane]);
#pragma unroll
          for (int h = 0; h < kInferSub; ++h) acc[h][t] = mfma(a, B[h][c], acc[h][t]);
        }
      }
#pragma unroll
      for (int h = 0; h < kInferSub; ++h) {
        B[h][0] = chain_relu(acc[h][0], acc[h][1]);
        B[h][1] = chain_relu(acc[h][2], acc[h][3]);
      }
    }
    f32x4 y[kInferSub];
#pragma unroll
    for (int h = 0; h < kInferSub; ++h) y[h] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
    for (int c = 0; c < 2; ++c) {
      const bf16x8 a = as_bf16x8(sw[(40 + c) * 64 + lane]);
#pragma unroll
      for (int h = 0; h < kInferSub; ++h) y[h] = mfma(a, B[h][c], y[h]);
    }
    if (g != 0) continue;  // lanes g == 0 hold output rows 0..3 of query q
#pragma unroll
    for (int h = 0; h < kInferSub; ++h) {
      if (!valid[h]) continue;
      if (MODE == 0) {
        out[qi[h] * 3 + 0] = y[h][0];
        out[qi[h] * 3 + 1] = y[h][1];
        out[qi[h] * 3 + 2] = y[h][2];
        continue;
      }
      const bool fo = P.nrc_factor != 0;
      if (MODE == 2) {  // every path below n gets an output: 0 unless its record is terminal
        float4 t = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        const float4 tail = reinterpret_cast<const float4*>(r[h])[3];  // beta at 15..17, flag at 18
        const float4 more = reinterpret_cast<const float4*>(r[h])[4];
        if (more.z == 2.0f) {
          t.x = tail.w * nrc_factor(x[h], 0, fo) * fmaxf(y[h][0], 0.0f);
          t.y = more.x * nrc_factor(x[h], 1, fo) * fmaxf(y[h][1], 0.0f);
          t.z = more.y * nrc_factor(x[h], 2, fo) * fmaxf(y[h][2], 0.0f);
          if (!(isfinite(t.x) && isfinite(t.y) && isfinite(t.z))) t = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
        }
        out4[qi[h]] = t;
        continue;
      }
      const float4 beta = reinterpret_cast<const float4*>(r[h])[3];
      const float cx = beta.x * nrc_factor(x[h], 0, fo) * fmaxf(y[h][0], 0.0f);
      const float cy = beta.y * nrc_factor(x[h], 1, fo) * fmaxf(y[h][1], 0.0f);
      const float cz = beta.z * nrc_factor(x[h], 2, fo) * fmaxf(y[h][2], 0.0f);
      if (isfinite(cx) && isfinite(cy) && isfinite(cz)) {
        const float4 l = P.L[slot[h]];
        P.L[slot[h]] = make_float4(l.x + cx, l.y + cy, l.z + cz, l.w);
      } else {
        nonfinite++;
      }
    }
  }
  if (MODE == 1 && nonfinite) atomicAdd(&P.stats[kStatNonFinite], nonfinite);
}

// -------------------------------------------------------- forward+backward
// a_store[l][f][n] (l = 0..5 layer inputs) and g_store[l][f][n] (l = 0..5
// gradients of the layer outputs), bf16, n padded to npad.  Samples at
// n >= N are written as zeros.  loss_part[block] = sum of the block's loss terms.
__global__ __launch_bounds__(256) void k_nrc_fwd_bwd(const float* __restrict__ X, const float* __restrict__ T,
                                                     int N, int npad, const uint4* __restrict__ fwd,
                                                     const uint4* __restrict__ bwd, uint16_t* __restrict__ a_store,
                                                     uint16_t* __restrict__ g_store, float* __restrict__ loss_part) {
  __shared__ uint4 sw[kNrcFwdFrags * 64];
  __shared__ uint4 swt[kNrcBwdFrags * 64];
  __shared__ float wave_loss[4];
  for (int i = threadIdx.x; i < kNrcFwdFrags * 64; i += blockDim.x) sw[i] = fwd[i];
  for (int i = threadIdx.x; i < kNrcBwdFrags * 64; i += blockDim.x) swt[i] = bwd[i];
  __syncthreads();
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, g = lane / 16, q = lane % 16;
  const float inv_count = 1.0f / (3.0f * (float)N);
  float my_loss = 0.0f;
  const size_t L = (size_t)64 * npad;  // one layer of a store
  for (int grp = blockIdx.x * 4 + wave; grp * 16 < npad; grp += gridDim.x * 4) {
    int qi = grp * 16 + q;
    bool valid = qi < N;
    float x[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) x[k] = valid ? X[(size_t)qi * 12 + k] : 0.0f;
    bf16x8 keep[12];
    bf16x8 B[2];
    encode_operand(x, g, B);
    f32x4 y = mlp_forward(sw, lane, B, keep);
    // layer inputs a_0..a_5
#pragma unroll
    for (int l = 0; l < 6; ++l)
#pragma unroll
      for (int c = 0; c < 2; ++c)
#pragma unroll
        for (int j = 0; j < 8; ++j) {
          int f = l == 0 ? nrc_k_in(c, g, j) : nrc_k_chained(c, g, j);
          float v = valid ? bf16x8_get(keep[2 * l + c], j) : 0.0f;
          a_store[l * L + (size_t)f * npad + qi] = bf16_bits(v);
        }
    // loss gradient (lanes g == 0 hold the three outputs of query q)
    float dy[3] = {0.0f, 0.0f, 0.0f};
    if (g == 0 && valid) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) {
        float t = T[(size_t)qi * 3 + ch];
        float d = y[ch] * y[ch] + 0.01f;
        float r = y[ch] - t;
        my_loss += r * r / d;
        dy[ch] = 2.0f * r / d * inv_count;
      }
    }
    uint4 gu;
    gu.x = pack2(dy[0], dy[1]);
    gu.y = pack2(dy[2], 0.0f);
    gu.z = 0u;
    gu.w = 0u;
    bf16x8 G5 = as_bf16x8(gu);
    if (g == 0) {
#pragma unroll
      for (int ch = 0; ch < 3; ++ch) g_store[5 * L + (size_t)ch * npad + qi] = bf16_bits(dy[ch]);
    }
    // g_4 = (W5^T g_5) * [a_5 > 0]
    f32x4 acc[4];
#pragma unroll
    for (int t = 0; t < 4; ++t) acc[t] = mfma(as_bf16x8(swt[(32 + t) * 64 + lane]), G5, f32x4{0.0f, 0.0f, 0.0f, 0.0f});
    bf16x8 Gc[2];
#pragma unroll
    for (int lo = 4; lo >= 0; --lo) {
      // mask with a_{lo+1} > 0, store g_lo, form the chained operand
      float gv[4][4];
#pragma unroll
      for (int t = 0; t < 4; ++t)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          float a = bf16x8_get(keep[2 * (lo + 1) + t / 2], (t % 2) * 4 + i);
          gv[t][i] = a > 0.0f ? acc[t][i] : 0.0f;
          g_store[lo * L + (size_t)(16 * t + 4 * g + i) * npad + qi] = bf16_bits(valid ? gv[t][i] : 0.0f);
        }
#pragma unroll
      for (int c = 0; c < 2; ++c) {
        uint4 u;
        u.x = pack2(gv[2 * c][0], gv[2 * c][1]);
        u.y = pack2(gv[2 * c][2], gv[2 * c][3]);
        u.z = pack2(gv[2 * c + 1][0], gv[2 * c + 1][1]);
        u.w = pack2(gv[2 * c + 1][2], gv[2 * c + 1][3]);
        Gc[c] = as_bf16x8(u);
      }
      if (lo == 0) break;
      // g_{lo-1} (pre-mask) = W_lo^T g_lo
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        acc[t] = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int c = 0; c < 2; ++c) acc[t] = mfma(as_bf16x8(swt[(((lo - 1) * 4 + t) * 2 + c) * 64 + lane]), Gc[c], acc[t]);
      }
    }
  }
  // fixed-order block reduction of the loss
  for (int off = 32; off > 0; off >>= 1) my_loss += __shfl_down(my_loss, off);
  if (lane == 0) wave_loss[wave] = my_loss;
  __syncthreads();
  if (threadIdx.x == 0) loss_part[blockIdx.x] = ((wave_loss[0] + wave_loss[1]) + wave_loss[2]) + wave_loss[3];
}

// ---------------------------------------------------------- weight grads
// One wave per (tile, split): dW_l[16 to + .][16 ti + .] over samples of the split.
__global__ __launch_bounds__(256) void k_nrc_dw(const uint16_t* __restrict__ a_store,
                                                const uint16_t* __restrict__ g_store, int npad, int n_split,
                                                float* __restrict__ dw_part) {
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64, g = lane / 16, r = lane % 16;
  const int wid = blockIdx.x * 4 + wave;
  if (wid >= 84 * n_split) return;
  const int tile = wid % 84, split = wid / 84;
  int l, to, ti;
  if (tile < 80) {
    l = tile / 16;
    to = (tile % 16) / 4;
    ti = tile % 4;
  } else {
    l = 5;
    to = 0;
    ti = tile - 80;
  }
  const size_t L = (size_t)64 * npad;
  const int per = npad / n_split;
  const int n0 = split * per, n1 = n0 + per;
  const uint16_t* ga = g_store + l * L + (size_t)(16 * to + r) * npad;
  const uint16_t* aa = a_store + l * L + (size_t)(16 * ti + r) * npad;
  const bool row_ok = l < 5 || r < 3;
  f32x4 acc = f32x4{0.0f, 0.0f, 0.0f, 0.0f};
  for (int k = n0; k < n1; k += 32) {
    uint4 au = row_ok ? *reinterpret_cast<const uint4*>(ga + k + 8 * g) : make_uint4(0u, 0u, 0u, 0u);
    uint4 bu = *reinterpret_cast<const uint4*>(aa + k + 8 * g);
    acc = mfma(as_bf16x8(au), as_bf16x8(bu), acc);
  }
  float* dst = dw_part + (size_t)split * kNrcParams;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    int o = 16 * to + 4 * g + i, in = 16 * ti + r;
    if (l < 5 || o < 3) dst[nrc_widx(l, o, in)] = acc[i];
  }
}

// ------------------------------------------------------------------ Adam
// Step t = t_step + 1 (the counter of applied steps lives on the device, so
// that a batch drawn from zero records, known only on the device, can be
// skipped without the host waiting for the record count).  Bias corrections
// 1 / (1 - beta^t) in double, rounded to float.  Then the moving average of
// the weights, e = ema e + (1 - ema) w, and the inference weights
// wi = e / (1 - ema^t) (wi = w when ema is 0).
__global__ __launch_bounds__(256) void k_nrc_adam(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                                  float* __restrict__ e, float* __restrict__ wi,
                                                  const float* __restrict__ dw_part, int n_split,
                                                  float* __restrict__ grad_out, float lr, float b1, float b2,
                                                  float eps, float ema, const uint32_t* __restrict__ t_step,
                                                  const uint32_t* __restrict__ n_records, int apply) {
  int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= kNrcParams) return;
  float gsum = 0.0f;
  for (int s = 0; s < n_split; ++s) gsum += dw_part[(size_t)s * kNrcParams + p];
  if (grad_out) grad_out[p] = gsum;
  if (!apply || (n_records && *n_records == 0u)) return;
  const double t = (double)(*t_step + 1u);
  const float c1 = (float)(1.0 / (1.0 - pow((double)b1, t)));
  const float c2 = (float)(1.0 / (1.0 - pow((double)b2, t)));
  float mm = b1 * m[p] + (1.0f - b1) * gsum;
  float vv = b2 * v[p] + (1.0f - b2) * gsum * gsum;
  m[p] = mm;
  v[p] = vv;
  const float wn = w[p] - lr * (mm * c1) / (sqrtf(vv * c2) + eps);
  w[p] = wn;
  if (ema > 0.0f) {
    const float ce = (float)(1.0 / (1.0 - pow((double)ema, t)));
    const float ee = ema * e[p] + (1.0f - ema) * wn;
    e[p] = ee;
    wi[p] = ee * ce;
  } else {
    wi[p] = wn;
  }
}

// ------------------------------------------------------- training targets
// Record r of training path k is valid (flag 1) when the path scattered at
// vertex r with r < max_depth; its target is (L_end - L_r) / beta_r, divided
// by the reflectance factor when factorising, dropped when a channel of
// beta_r or of the factor is zero or the target is not finite.  A terminal
// record (flag 2, self-training) is no sample: its cache answer is in L_end.
// Offsets come from an exclusive scan over paths, so the compacted list is in
// path-major, vertex order whatever the scheduling.
__device__ inline bool nrc_target(const float* rec, float4 Lend, bool factor, float t[3]) {
  if (rec[18] != 1.0f) return false;
  const float Lr[3] = {rec[12], rec[13], rec[14]}, be[3] = {rec[15], rec[16], rec[17]};
  const float Le[3] = {Lend.x, Lend.y, Lend.z};
  bool ok = true;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    const float f = nrc_factor(rec, c, factor);
    ok = ok && be[c] != 0.0f && f != 0.0f;
    t[c] = (Le[c] - Lr[c]) / be[c];
    if (factor) t[c] = t[c] / f;
    ok = ok && isfinite(t[c]);
  }
  return ok;
}

// L at the end of training path k: its radiance plus, with self-training, the cache at its terminal vertex.
__device__ inline float4 nrc_path_end(const PathsDev& P, const float4* tail, int k) {
  float4 Le = P.L[P.n_render + k];
  if (tail) {
    const float4 t = tail[k];
    Le.x += t.x;
    Le.y += t.y;
    Le.z += t.z;
  }
  return Le;
}

// Compaction in three kernels: per-path counts with per-workgroup sums, a
// scan of the workgroup sums, and the in-workgroup scan + copy.
__device__ inline uint32_t block_exclusive_scan(uint32_t v, uint32_t* s, uint32_t& total) {
  s[threadIdx.x] = v;
  __syncthreads();
  for (int off = 1; off < 256; off <<= 1) {  // Hillis-Steele inclusive scan
    uint32_t u = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0u;
    __syncthreads();
    s[threadIdx.x] += u;
    __syncthreads();
  }
  total = s[255];
  return s[threadIdx.x] - v;
}

__global__ __launch_bounds__(256) void k_nrc_count(PathsDev P, int n_paths, const float4* __restrict__ tail,
                                                   uint32_t* __restrict__ counts, uint32_t* __restrict__ block_sums) {
  __shared__ uint32_t s[256];
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t c = 0;
  if (k < n_paths) {
    const float4 Le = nrc_path_end(P, tail, k);
    for (int r = 0; r < P.rec_depth; ++r) {
      float t[3];
      c += nrc_target(P.rec + ((size_t)k * P.rec_depth + r) * kNrcRecFloats, Le, P.nrc_factor != 0, t) ? 1u : 0u;
    }
    counts[k] = c;
  }
  uint32_t total;
  block_exclusive_scan(c, s, total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// In-place exclusive scan of the workgroup sums (one workgroup); total to *n_out.
__global__ __launch_bounds__(1024) void k_nrc_scan(int n, uint32_t* __restrict__ sums, uint32_t* __restrict__ n_out,
                                                  unsigned long long* __restrict__ stats) {
  __shared__ uint32_t part[1024];
  const int per = (n + 1023) / 1024;
  const int k0 = min(n, (int)threadIdx.x * per), k1 = min(n, k0 + per);
  uint32_t local = 0;
  for (int k = k0; k < k1; ++k) local += sums[k];
  part[threadIdx.x] = local;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t base = part[threadIdx.x] - local;
  for (int k = k0; k < k1; ++k) {
    uint32_t c = sums[k];
    sums[k] = base;
    base += c;
  }
  if (threadIdx.x == 1023) {
    *n_out = part[1023];
    if (stats) atomicAdd(&stats[kStatRecords], (unsigned long long)part[1023]);
  }
}

__global__ __launch_bounds__(256) void k_nrc_compact(PathsDev P, int n_paths, const float4* __restrict__ tail,
                                                     uint32_t* __restrict__ offsets,
                                                     const uint32_t* __restrict__ block_base, float* __restrict__ X,
                                                     float* __restrict__ T) {
  __shared__ uint32_t s[256];
  int k = blockIdx.x * blockDim.x + threadIdx.x;
  uint32_t c = k < n_paths ? offsets[k] : 0u;
  uint32_t total;
  uint32_t o = block_base[blockIdx.x] + block_exclusive_scan(c, s, total);
  if (k >= n_paths) return;
  offsets[k] = o;
  const float4 Le = nrc_path_end(P, tail, k);
  for (int r = 0; r < P.rec_depth; ++r) {
    const float* rec = P.rec + ((size_t)k * P.rec_depth + r) * kNrcRecFloats;
    float t[3];
    if (!nrc_target(rec, Le, P.nrc_factor != 0, t)) continue;
    for (int i = 0; i < 12; ++i) X[(size_t)o * 12 + i] = rec[i];
    for (int j = 0; j < 3; ++j) T[(size_t)o * 3 + j] = t[j];
    ++o;
  }
}

// Batch of step s of a frame: sample j takes record floor(m * n / 2^24), m the
// top 24 bits of Philox word s % 4 at counter (j, 2^31 + frame, 0x4E5253, s / 4).
__global__ __launch_bounds__(256) void k_nrc_gather(const float* __restrict__ X_all, const float* __restrict__ T_all,
                                                    const uint32_t* __restrict__ n_all, int B, uint32_t frame,
                                                    int step, uint32_t k0, uint32_t k1, float* __restrict__ Xb,
                                                    float* __restrict__ Tb) {
  int j = blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= B) return;
  uint32_t n = *n_all;
  if (n == 0u) {
    for (int i = 0; i < 12; ++i) Xb[(size_t)j * 12 + i] = 0.0f;
    for (int c = 0; c < 3; ++c) Tb[(size_t)j * 3 + c] = 0.0f;
    return;
  }
  U4 r = philox((uint32_t)j, 0x80000000u + frame, 0x4E5253u, (uint32_t)step / 4u, k0, k1);
  uint32_t w = (step % 4) == 0 ? r.x : (step % 4) == 1 ? r.y : (step % 4) == 2 ? r.z : r.w;
  uint32_t idx = (uint32_t)(((uint64_t)(w >> 8) * n) >> 24);
  for (int i = 0; i < 12; ++i) Xb[(size_t)j * 12 + i] = X_all[(size_t)idx * 12 + i];
  for (int c = 0; c < 3; ++c) Tb[(size_t)j * 3 + c] = T_all[(size_t)idx * 3 + c];
}

// ------------------------------------------------------------- launchers
hipError_t nrc_launch_pack(const float* w, const float* wi, uint4* fwd, uint4* bwd, uint4* inf, uint32_t* t_step,
                           const uint32_t* n_records, hipStream_t st) {
  int total = (2 * kNrcFwdFrags + kNrcBwdFrags) * 64;
  hipLaunchKernelGGL(k_nrc_pack, dim3((total + 255) / 256), dim3(256), 0, st, w, wi, fwd, bwd, inf, t_step,
                     n_records);
  return hipGetLastError();
}

// The inference kernel stages the weight fragments in LDS once per
// workgroup: launch at most one resident set of workgroups and let each wave
// stride over the queries.
static int nrc_infer_grid() {
  static int resident = 0;
  if (!resident) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_nrc_infer<1>, 64 * kInferWaves, 0) != hipSuccess ||
        per < 1)
      per = 1;
    resident = std::max(1, cus * per);
  }
  return resident;
}

// Workgroups for n queries: enough for one iteration per wave, at most one resident set.
static int nrc_infer_groups(int64_t n) {
  const int64_t per_group = (int64_t)16 * kInferSub * kInferWaves;
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + per_group - 1) / per_group, nrc_infer_grid()));
}

hipError_t nrc_launch_forward(const float* x, int64_t n, const uint4* fwd, float* y, hipStream_t st) {
  PathsDev P;
  __builtin_memset(&P, 0, sizeof(P));
  const int grid = nrc_infer_groups(n);
  hipLaunchKernelGGL((k_nrc_infer<0>), dim3(grid), dim3(64 * kInferWaves), 0, st, x, n, P, fwd, y);
  return hipGetLastError();
}

hipError_t nrc_launch_query(const PathsDev& P, const uint4* fwd, int grid, hipStream_t st) {
  grid = std::max(1, std::min(grid, nrc_infer_grid()));
  hipLaunchKernelGGL((k_nrc_infer<1>), dim3(grid), dim3(64 * kInferWaves), 0, st, nullptr, (int64_t)0, P, fwd,
                     nullptr);
  return hipGetLastError();
}

hipError_t nrc_launch_train(const float* X, const float* T, int N, int npad, int n_split, const uint4* fwd,
                            const uint4* bwd, uint16_t* a_store, uint16_t* g_store, float* loss_part, int grid_fb,
                            float* dw_part, hipStream_t st) {
  hipLaunchKernelGGL(k_nrc_fwd_bwd, dim3(grid_fb), dim3(256), 0, st, X, T, N, npad, fwd, bwd, a_store, g_store,
                     loss_part);
  int waves = 84 * n_split;
  hipLaunchKernelGGL(k_nrc_dw, dim3((waves + 3) / 4), dim3(256), 0, st, a_store, g_store, npad, n_split, dw_part);
  return hipGetLastError();
}

hipError_t nrc_launch_adam(float* w, float* m, float* v, float* e, float* wi, const float* dw_part, int n_split,
                           float* grad_out, float lr, float b1, float b2, float eps, float ema, const uint32_t* t_step,
                           const uint32_t* n_records, int apply, hipStream_t st) {
  hipLaunchKernelGGL(k_nrc_adam, dim3((kNrcParams + 255) / 256), dim3(256), 0, st, w, m, v, e, wi, dw_part, n_split,
                     grad_out, lr, b1, b2, eps, ema, t_step, n_records, apply);
  return hipGetLastError();
}

hipError_t nrc_launch_terminal(const PathsDev& P, int n_paths, const uint4* fwd, float4* tail, hipStream_t st) {
  const int grid = nrc_infer_groups(n_paths);
  hipLaunchKernelGGL((k_nrc_infer<2>), dim3(grid), dim3(64 * kInferWaves), 0, st, nullptr, (int64_t)n_paths, P, fwd,
                     reinterpret_cast<float*>(tail));
  return hipGetLastError();
}

hipError_t nrc_launch_targets(const PathsDev& P, int n_paths, const float4* tail, uint32_t* offsets,
                              uint32_t* block_sums, float* X, float* T, uint32_t* n_out,
                              unsigned long long* record_stats, hipStream_t st) {
  const int nb = (n_paths + 255) / 256;
  hipLaunchKernelGGL(k_nrc_count, dim3(nb), dim3(256), 0, st, P, n_paths, tail, offsets, block_sums);
  hipLaunchKernelGGL(k_nrc_scan, dim3(1), dim3(1024), 0, st, nb, block_sums, n_out, record_stats);
  hipLaunchKernelGGL(k_nrc_compact, dim3(nb), dim3(256), 0, st, P, n_paths, tail, offsets, block_sums, X, T);
  return hipGetLastError();
}

hipError_t nrc_launch_gather(const float* X_all, const float* T_all, const uint32_t* n_all, int B, uint32_t frame,
                             int step, uint32_t k0, uint32_t k1, float* Xb, float* Tb, hipStream_t st) {
  hipLaunchKernelGGL(k_nrc_gather, dim3((B + 255) / 256), dim3(256), 0, st, X_all, T_all, n_all, B, frame, step, k0,
                     k1, Xb, Tb);
  return hipGetLastError();
}

}  // namespace pt
