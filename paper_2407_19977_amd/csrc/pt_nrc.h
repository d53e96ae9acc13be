// Radiance cache (neural radiance caching, named by the paper as future work
// in Sec. 6.1): device-side inputs, encoding and the matrix-core operand layout.
//
// Inputs at a vertex (12): position in the scene box (3); wo and the shading
// normal as (acos(y)/pi, atan2(x,-z)/2pi + 1/2) (2 + 2); specular roughness;
// diffuse albedo (1-metalness)(1-transmission) kd, kd the diffuse lobe's albedo (3);
// specular albedo metalness lum(bw bc) + (1-metalness) (F + transmission (1 - F)),
// F = F_dielectric(1, ior): what the metal or the dielectric interface reflects or
// transmits at normal incidence (so that a glass's reflectance factor is about 1).
// Encoding (64): sin / cos(2^k pi x_a), k = 0..5 (36); one-blob, 4 bins, of
// the four direction coordinates (16; the two azimuths periodic) and of
// 1 - exp(-roughness) (4); the four albedo values (4); constants 1, 0, 0, 0 (4).
// Network: 64 -> 5 x (64, ReLU) -> 3, no biases, bfloat16 operands, FP32 sums.
//
// Matrix-core layout (v_mfma_f32_16x16x32_bf16, wave64): the layer computes
// Z^T = W X^T with queries as columns.  Operand A (weights) lane (g, r) holds
// row r of a 16-row tile and K entries 8g..8g+7; operand B (activations) lane
// (g, q) holds query q and K entries 8g..8g+7; the result lane (g, q) holds
// rows 4g..4g+3 of query q.  For hidden layers the K entries of chunk c are
// ordered [tile 2c rows 4g..4g+3, tile 2c+1 rows 4g..4g+3], so a layer's
// result registers are the next layer's B operand without any data movement;
// the input layer's K entries follow nrc_k_in.  The weight fragments are
// stored in these orders.
#pragma once

#include <math.h>
#include <stdint.h>

#include "pt_shade.h"

namespace pt {

constexpr int kNrcParams = 5 * 64 * 64 + 3 * 64;  // 20672
constexpr int kNrcFwdFrags = 5 * 8 + 2;          // hidden: 4 tiles x 2 chunks; output: 2 chunks
constexpr int kNrcBwdFrags = 4 * 8 + 4;          // W_l^T for l = 1..4; W5^T: 4 tiles x 1 chunk
constexpr int kNrcQueryFloats = 16;              // x[12], beta[3], slot bits
constexpr int kNrcRecFloats = 20;                // x[12], L[3], beta[3], valid, pad

__host__ __device__ inline uint16_t bf16_bits(float x) {
  uint32_t u;
  __builtin_memcpy(&u, &x, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) return (uint16_t)(u >> 16);
  u += 0x7FFFu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__host__ __device__ inline float bf16_float(uint16_t b) {
  uint32_t u = (uint32_t)b << 16;
  float f;
  __builtin_memcpy(&f, &u, 4);
  return f;
}

// Input feature index of layer-0 K entry (chunk c, lane group g, element j).
// The order spreads the encoding evenly over the four lanes of a query, so
// that every lane runs the same instructions: chunk 0 holds the sin/cos
// pairs 4g..4g+3 (pair p = 6a + k: axis a, frequency 2^k); chunk 1 holds
// feature 32 + g (one value of the last two pairs), the four one-blob bins
// of direction coordinate g, bin g of the roughness, and two of the albedo
// and constant features.
__host__ __device__ inline int nrc_k_in(int c, int g, int j) {
  if (c == 0) return 8 * g + j;
  if (j == 0) return 32 + g;
  if (j <= 4) return 36 + 4 * g + (j - 1);
  if (j == 5) return 52 + g;
  return 56 + 2 * g + (j - 6);
}

// Input index of hidden-layer K entry (chunk c, lane group g, element j).
__host__ __device__ inline int nrc_k_chained(int c, int g, int j) {
  return j < 4 ? 32 * c + 4 * g + j : 32 * c + 16 + 4 * g + (j - 4);
}

// Offset of W_l[o][i] in the concatenated parameter vector.
__host__ __device__ inline int nrc_widx(int l, int o, int i) { return l * 4096 + o * 64 + i; }

__host__ __device__ inline float nrc_one_blob(float s, int i) {
  float z = (s - ((float)i + 0.5f) * 0.25f) * 4.0f;
  return expf(-0.5f * z * z);
}

// One-blob bin of an azimuth (periodic: 0 and 1 are the same direction): the
// distance to the bin centre is taken modulo 1 into [-1/2, 1/2).
__host__ __device__ inline float nrc_one_blob_periodic(float s, int i) {
  float d = s - ((float)i + 0.5f) * 0.25f;
  d -= floorf(d + 0.5f);
  float z = d * 4.0f;
  return expf(-0.5f * z * z);
}

// Feature f (0..63) of the 12 inputs.
__host__ __device__ inline float nrc_feature(int f, const float* x) {
  if (f < 36) {
    int a = f / 12, k = (f % 12) >> 1;
    float w = x[a] * (float)(1 << k);
#ifdef __HIP_DEVICE_COMPILE__
    return (f & 1) ? cospif(w) : sinpif(w);
#else
    return (f & 1) ? cosf(kPi * w) : sinf(kPi * w);
#endif
  }
  if (f < 52) {
    int c = (f - 36) >> 2, i = (f - 36) & 3;
    return (c & 1) ? nrc_one_blob_periodic(x[3 + c], i) : nrc_one_blob(x[3 + c], i);
  }
  if (f < 56) return nrc_one_blob(1.0f - expf(-x[7]), f - 52);
  if (f < 60) return x[8 + (f - 56)];
  return f == 60 ? 1.0f : 0.0f;
}

// The 12 inputs at a shading point.
__host__ __device__ inline void nrc_inputs(const float* lo, const float* inv_ext, V3 p, V3 wo, V3 n,
                                           const MatRec& m, float* x) {
  x[0] = (p.x - lo[0]) * inv_ext[0];
  x[1] = (p.y - lo[1]) * inv_ext[1];
  x[2] = (p.z - lo[2]) * inv_ext[2];
  V3 d[2] = {wo, n};
#pragma unroll
  for (int k = 0; k < 2; ++k) {
    float y = fminf(fmaxf(d[k].y, -1.0f), 1.0f);
    x[3 + 2 * k] = acosf(y) * (1.0f / kPi);
    // + 0.0f turns -0 into +0, so that a direction exactly at a pole has azimuth 0 on every side
    x[4 + 2 * k] = atan2f(d[k].x + 0.0f, -d[k].z + 0.0f) * (0.5f / kPi) + 0.5f;
  }
  x[7] = m.spec_rough;
  const float k = (1.0f - m.metalness) * (1.0f - m.trans_weight);
  x[8] = k * m.kd[0];
  x[9] = k * m.kd[1];
  x[10] = k * m.kd[2];
  x[11] = m.metalness * m.bwbc_lum + (1.0f - m.metalness) * (m.f0_diel + m.trans_weight * (1.0f - m.f0_diel));
}

}  // namespace pt
