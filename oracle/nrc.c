/*
 * Oracle of the radiance cache (test infrastructure only), FP64.
 *
 * The paper names neural radiance caching (Mueller et al. 2021) as future
 * work for needing fewer samples (Sec. 6.1).  The reading implemented here:
 *
 * Inputs at a path vertex (12): position normalised to the scene box (3);
 * the outgoing direction wo and the shading normal n, each as
 * (acos(y)/pi, atan2(x, -z)/2pi + 1/2) (2 + 2); specular roughness (1);
 * diffuse albedo (1-metalness)(1-transmission) rho, rho the diffuse lobe's
 * albedo (base_weight base_color, mixed with subsurface_color) (3);
 * specular albedo metalness lum(base_weight base_color) +
 * (1-metalness) (F + transmission_weight (1 - F)), F = F_dielectric(1, eta')
 * (1), eta' the IOR after the specular_weight modulation: what the metal or
 * the dielectric interface reflects or transmits at normal incidence.
 *
 * Encoding to 64 features: for each position axis and k = 0..5 the pair
 * sin(2^k pi x), cos(2^k pi x) (36); one-blob encodings with 4 bins of the
 * four direction coordinates (16) and of 1 - exp(-roughness) (4), bin i of s
 * being exp(-(4 d)^2 / 2) with d = s - (i + 1/2)/4; for the two azimuths
 * (inputs 4 and 6, periodic: 0 and 1 are the same direction) d is taken
 * modulo 1 into [-1/2, 1/2); the four albedo values (4); and the constants
 * 1, 0, 0, 0 (4).
 *
 * Network: 64 -> 64 x 5 hidden layers with ReLU -> 3 linear outputs, no
 * biases; weights W0..W4 (64 x 64) and W5 (3 x 64), row-major [out][in],
 * concatenated (20,672 values).  With bf16 = 1 the weights, the encoded
 * input and every hidden activation are rounded to bfloat16 (round to
 * nearest even) before use, as the GPU's tensor operands are; sums stay FP64.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

#include "oracle_internal.h"

#define NRC_IN 64
#define NRC_HIDDEN 5
#define NRC_OUT 3
#define NRC_PARAMS (NRC_HIDDEN * 64 * 64 + NRC_OUT * 64)

double oracle_bf16_round(double x) {
  float f = (float)x;
  uint32_t u;
  memcpy(&u, &f, 4);
  if ((u & 0x7F800000u) == 0x7F800000u) return (double)f; /* inf / nan unchanged */
  uint32_t lsb = (u >> 16) & 1u;
  u += 0x7FFFu + lsb;
  u &= 0xFFFF0000u;
  memcpy(&f, &u, 4);
  return (double)f;
}

static double one_blob(double s, int i, int periodic) {
  double d = s - (i + 0.5) / 4.0;
  if (periodic) d -= floor(d + 0.5);
  double z = d * 4.0;
  return exp(-0.5 * z * z);
}

void oracle_nrc_encode(const double x[12], double f[64]) {
  for (int a = 0; a < 3; ++a)
    for (int k = 0; k < 6; ++k) {
      double w = ldexp(O_PI, k) * x[a];
      f[12 * a + 2 * k] = sin(w);
      f[12 * a + 2 * k + 1] = cos(w);
    }
  for (int c = 0; c < 4; ++c)
    for (int i = 0; i < 4; ++i) f[36 + 4 * c + i] = one_blob(x[3 + c], i, c & 1);
  double rr = 1.0 - exp(-x[7]);
  for (int i = 0; i < 4; ++i) f[52 + i] = one_blob(rr, i, 0);
  for (int i = 0; i < 4; ++i) f[56 + i] = x[8 + i];
  f[60] = 1.0;
  f[61] = f[62] = f[63] = 0.0;
}

void oracle_nrc_forward(const double* W, const double x[12], int32_t bf16, double y[3]) {
  double a[64], z[64];
  oracle_nrc_encode(x, a);
  if (bf16)
    for (int i = 0; i < 64; ++i) a[i] = oracle_bf16_round(a[i]);
  const double* w = W;
  for (int l = 0; l < NRC_HIDDEN; ++l) {
    for (int o = 0; o < 64; ++o) {
      double s = 0.0;
      for (int i = 0; i < 64; ++i) s += (bf16 ? oracle_bf16_round(w[64 * o + i]) : w[64 * o + i]) * a[i];
      z[o] = s > 0.0 ? s : 0.0;
    }
    for (int o = 0; o < 64; ++o) a[o] = bf16 ? oracle_bf16_round(z[o]) : z[o];
    w += 64 * 64;
  }
  for (int o = 0; o < NRC_OUT; ++o) {
    double s = 0.0;
    for (int i = 0; i < 64; ++i) s += (bf16 ? oracle_bf16_round(w[64 * o + i]) : w[64 * o + i]) * a[i];
    y[o] = s;
  }
}

/* Inputs of the cache at a shading point (see the header comment). */
void onrc_inputs(const oracle_scene* s, v3 p, v3 wo, v3 n, const omat* m, double x[12]) {
  for (int k = 0; k < 3; ++k) {
    double e = s->hi[k] - s->lo[k];
    x[k] = e > 0.0 ? (vget(p, k) - s->lo[k]) / e : 0.0;
  }
  v3 dirs[2] = {wo, n};
  for (int d = 0; d < 2; ++d) {
    double yv = dirs[d].y < -1.0 ? -1.0 : (dirs[d].y > 1.0 ? 1.0 : dirs[d].y);
    x[3 + 2 * d] = acos(yv) / O_PI;
    /* + 0.0 turns -0 into +0: a direction exactly at a pole gets azimuth 0 whatever the signs of its zeros */
    x[4 + 2 * d] = atan2(dirs[d].x + 0.0, -dirs[d].z + 0.0) / (2.0 * O_PI) + 0.5;
  }
  x[7] = m->spec_rough;
  double k = (1.0 - m->metalness) * (1.0 - m->trans_weight);
  for (int c = 0; c < 3; ++c) x[8 + c] = k * odiffuse_albedo(m, c);
  double F0[3] = {m->base_weight * m->base_color[0], m->base_weight * m->base_color[1],
                  m->base_weight * m->base_color[2]};
  const double Fd = ofresnel_diel(1.0, omod_ior(m));
  x[11] = m->metalness * lum3(F0) + (1.0 - m->metalness) * (Fd + m->trans_weight * (1.0 - Fd));
}

/* Test hook: onrc_inputs for a scene box [lo, hi] and a material given as
 * its 35 OpenPBR floats. */
void oracle_nrc_inputs(const double lo[3], const double hi[3], const double p[3], const double wo[3],
                       const double n[3], const float* mat, double x[12]) {
  oracle_scene s;
  memset(&s, 0, sizeof s);
  for (int k = 0; k < 3; ++k) { s.lo[k] = lo[k]; s.hi[k] = hi[k]; }
  omat m;
  omat_from_floats(mat, &m);
  onrc_inputs(&s, V(p[0], p[1], p[2]), V(wo[0], wo[1], wo[2]), V(n[0], n[1], n[2]), &m, x);
}
