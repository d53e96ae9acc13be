// Shading math of the path tracer in FP32: counter-based random numbers,
// the OpenPBR-subset BSDF and light sampling.
//
// Random numbers (the paper draws from a per-pixel PCG, Sec. 5.1.2): a
// Philox4x32-10 block (Salmon et al., SC'11) with counter (pixel, sample,
// bounce, dimension / 4) and key (seed low, seed high); dimension k of a
// bounce is word k mod 4, mapped to (x >> 8) * 2^-24.  Dimensions per
// bounce: 0-1 pixel jitter, 2 lobe, 3 roulette, 4-5 direction,
// 6 reflect/refract, 7 light choice, 8-9 light point.
//
// BSDF (OpenPBR, Sec. 4; importance sampling, Sec. 5.1.3): coat C
// (dielectric GGX reflection), metal M (GGX with F82-tint Fresnel),
// dielectric interface I (GGX reflection + rough refraction after Walter et
// al. 2007, with the 1/eta^2 radiance factor), diffuse D (Lambert, or the
// energy-preserving Oren-Nayar model at base_diffuse_roughness > 0,
// attenuated by the interface Fresnel on both sides):
//   f = C + [(1-cw) + cw*coat_color*(1-Fc(|mu_i|))(1-Fc(mu_o))]
//           * [metalness*M + (1-metalness)*(I + D)]
// GGX uses alpha = roughness^2 with the OpenPBR anisotropy mapping,
// height-correlated masking-shadowing and visible-normal sampling (Heitz
// 2014, 2018); a lobe with roughness < 1e-3 is a delta lobe.  One lobe is
// chosen per bounce with probabilities proportional to
//   w_C = cw*Fc, w_M = Tc*metalness*sw*lum(F82), w_I = Tc*(1-metalness)*(Fd + tw(1-Fd)),
//   w_D = Tc*(1-metalness)*(1-tw)*(1-Fd)*lum(bw*bc),  Tc = 1-cw*Fc(mu_o), Fd = F(eta', mu_o),
// and the non-delta weight is f*|cos|/sum_k P_k pdf_k (one-sample MIS).  eta'
// is the IOR after the specular_weight modulation; with a thin film the
// interface reflectance is per channel and Fd its luminance (iface_fresnel).
#pragma once

#include <math.h>
#include <stdint.h>

#include "pt_layout.h"

namespace pt {

constexpr float kPi = 3.14159265358979323846f;

// ----------------------------------------------------------------- vectors
struct V3 {
  float x, y, z;
};
__host__ __device__ inline V3 v3(float x, float y, float z) { return V3{x, y, z}; }
__host__ __device__ inline V3 operator+(V3 a, V3 b) { return v3(a.x + b.x, a.y + b.y, a.z + b.z); }
__host__ __device__ inline V3 operator-(V3 a, V3 b) { return v3(a.x - b.x, a.y - b.y, a.z - b.z); }
__host__ __device__ inline V3 operator*(V3 a, float s) { return v3(a.x * s, a.y * s, a.z * s); }
__host__ __device__ inline float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__host__ __device__ inline V3 cross(V3 a, V3 b) {
  return v3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__host__ __device__ inline float length(V3 a) { return sqrtf(dot(a, a)); }
__host__ __device__ inline V3 normalize(V3 a) { return a * (1.0f / length(a)); }
__host__ __device__ inline float lum(float r, float g, float b) { return 0.2126f * r + 0.7152f * g + 0.0722f * b; }

// ------------------------------------------------------------------ Philox
struct U4 {
  uint32_t x, y, z, w;
};

__host__ __device__ inline uint32_t mulhi32(uint32_t a, uint32_t b) {
#ifdef __HIP_DEVICE_COMPILE__
  return __umulhi(a, b);
#else
  return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
#endif
}

__host__ __device__ inline U4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    uint32_t h0 = mulhi32(0xD2511F53u, c0), l0 = 0xD2511F53u * c0;
    uint32_t h1 = mulhi32(0xCD9E8D57u, c2), l1 = 0xCD9E8D57u * c2;
    uint32_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
    c0 = n0;
    c1 = l1;
    c2 = n2;
    c3 = l0;
    k0 += 0x9E3779B9u;
    k1 += 0xBB67AE85u;
  }
  return U4{c0, c1, c2, c3};
}

__host__ __device__ inline float u01(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

// The 12 uniforms of one bounce, computed block by block on demand.
struct Rng {
  uint32_t pixel, sample, k0, k1;
  __host__ __device__ inline U4 block(uint32_t bounce, uint32_t b) const {
    return philox(pixel, sample, bounce, b, k0, k1);
  }
};

// -------------------------------------------------------------- Fresnel
// Exact unpolarised dielectric reflectance (Walter et al. 2007, eq. 22);
// c = |cos| on the incident side, eta = n_transmitted / n_incident.
__host__ __device__ inline float fresnel_diel(float c, float eta) {
  c = fabsf(c);
  float g2 = eta * eta - 1.0f + c * c;
  if (g2 < 0.0f) return 1.0f;
  float g = sqrtf(g2);
  float a = (g - c) / (g + c);
  float b = (c * (g + c) - 1.0f) / (c * (g - c) + 1.0f);
  return 0.5f * a * a * (1.0f + b * b);
}

// Thin film on the dielectric interface: reflectance of the stack incident
// medium (index 1) | film (relative index n2) | base (relative index n3) at
// incident cosine c1 for one wavelength, by the Airy sum of the film's
// multiply reflected waves, per polarisation
// R = (r12^2 + r23^2 + 2 r12 r23 cos d) / (1 + r12^2 r23^2 + 2 r12 r23 cos d),
// r_ij = (a_i - a_j) / (a_i + a_j) with a = n cos (s) or cos / n (p), phase
// d = 2 pi (2 film_ior d_nm cos_film / lambda); unpolarised: the mean.  Total
// internal reflection at either interface reflects everything (the film's
// index is at least 1).
__host__ __device__ inline __attribute__((noinline)) float film_airy(float c1, float n2, float n3, float film_ior, float d_nm,
                                           float inv_lambda) {
  c1 = fabsf(c1);
  const float s2 = 1.0f - c1 * c1;
  const float c2sq = 1.0f - s2 / (n2 * n2), c3sq = 1.0f - s2 / (n3 * n3);
  if (c2sq < 0.0f || c3sq < 0.0f) return 1.0f;
  const float c2 = sqrtf(c2sq), c3 = sqrtf(c3sq);
  const float cyc = 2.0f * (2.0f * film_ior * d_nm * c2 * inv_lambda);  // phase / pi
#ifdef __HIP_DEVICE_COMPILE__
  const float cd = cospif(cyc);
#else
  const float cd = cosf(kPi * cyc);
#endif
  const float as[3] = {c1, n2 * c2, n3 * c3}, ap[3] = {c1, c2 / n2, c3 / n3};
  float R = 0.0f;
#pragma unroll
  for (int pol = 0; pol < 2; ++pol) {
    const float* a = pol == 0 ? as : ap;
    const float r12 = (a[0] - a[1]) / (a[0] + a[1]);
    const float r23 = (a[1] - a[2]) / (a[1] + a[2]);
    const float x = 2.0f * r12 * r23 * cd;
    R += 0.5f * (r12 * r12 + r23 * r23 + x) / (1.0f + r12 * r12 * r23 * r23 + x);
  }
  return R;
}

// OpenPBR F82-tint metal Fresnel, clamped to [0,1].
__host__ __device__ inline V3 fresnel_f82(const MatRec& m, float mu) {
  const float mb = 1.0f / 7.0f;
  float om = 1.0f - mu;
  float om5 = om * om * om * om * om;
  const float omb = 1.0f - mb;
  const float omb5 = omb * omb * omb * omb * omb;
  const float denom = mb * omb5 * omb;
  float r[3];
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    float F0 = m.base_weight * m.base_color[c];
    float S = F0 + (1.0f - F0) * om5;
    float Sb = F0 + (1.0f - F0) * omb5;
    float b = Sb * (1.0f - m.spec_color[c]) / denom;
    float v = S - mu * om5 * om * b;
    r[c] = fminf(fmaxf(v, 0.0f), 1.0f);
  }
  return v3(r[0], r[1], r[2]);
}

// ------------------------------------------------------------------- GGX
__host__ __device__ inline float ggx_D(float at, float ab, V3 m) {
  if (m.z <= 0.0f) return 0.0f;
  float x = m.x / at, y = m.y / ab;
  float k = x * x + y * y + m.z * m.z;
  return 1.0f / (kPi * at * ab * k * k);
}

__host__ __device__ inline float ggx_lambda(float at, float ab, V3 w) {
  float z2 = w.z * w.z;
  if (z2 == 0.0f) return INFINITY;
  float a2 = (at * at * w.x * w.x + ab * ab * w.y * w.y) / z2;
  return 0.5f * (-1.0f + sqrtf(1.0f + a2));
}

__host__ __device__ inline V3 ggx_vndf_sample(float at, float ab, V3 wo, float u1, float u2) {
  V3 vh = normalize(v3(at * wo.x, ab * wo.y, wo.z));
  float lensq = vh.x * vh.x + vh.y * vh.y;
  V3 T1 = lensq > 0.0f ? v3(-vh.y, vh.x, 0.0f) * (1.0f / sqrtf(lensq)) : v3(1.0f, 0.0f, 0.0f);
  V3 T2 = cross(vh, T1);
  float r = sqrtf(u1);
  float phi = 2.0f * kPi * u2;
  float s_, c_;
  sincosf(phi, &s_, &c_);
  float t1 = r * c_, t2 = r * s_;
  float s = 0.5f * (1.0f + vh.z);
  t2 = (1.0f - s) * sqrtf(fmaxf(0.0f, 1.0f - t1 * t1)) + s * t2;
  float tz = fmaxf(0.0f, 1.0f - t1 * t1 - t2 * t2);
  V3 nh = T1 * t1 + T2 * t2 + vh * sqrtf(tz);
  return normalize(v3(at * nh.x, ab * nh.y, fmaxf(0.0f, nh.z)));
}

__host__ __device__ inline float ggx_vndf_pdf(float at, float ab, V3 wo, V3 m) {
  float wm = dot(wo, m);
  if (wm <= 0.0f || wo.z <= 0.0f) return 0.0f;
  float G1 = 1.0f / (1.0f + ggx_lambda(at, ab, wo));
  return G1 * wm * ggx_D(at, ab, m) / wo.z;
}

__host__ __device__ inline float ggx_G2(float at, float ab, V3 wo, V3 wi) {
  return 1.0f / (1.0f + ggx_lambda(at, ab, wo) + ggx_lambda(at, ab, wi));
}

// ------------------------------------------------------------------ BSDF
// Compile-time lobe set of a material class (zero lobes are skipped).
template <int CLS>
struct Lobes {
  static constexpr bool C = CLS == kClsPlastic || CLS == kClsGeneral;
  static constexpr bool M = CLS == kClsMetal || CLS == kClsGeneral;
  static constexpr bool I = CLS == kClsPlastic || CLS == kClsGlass || CLS == kClsGeneral;
  static constexpr bool D = CLS == kClsDiffuse || CLS == kClsPlastic || CLS == kClsGlass || CLS == kClsGeneral;
  static constexpr bool T = CLS == kClsGlass || CLS == kClsGeneral;
  static constexpr bool F = CLS == kClsGeneral;  // thin film (materials with one are of the general class)
  static constexpr bool Z = CLS == kClsGeneral;  // fuzz (likewise)
};

struct Bsdf {
  float eta;  // relative IOR of the interface seen from wo
  float film_n2;  // thin film IOR relative to the medium wo is in
  bool entering;
  float P[5];  // lobe probabilities C, M, I, D, Z (fuzz)
  bool absorbed;
};

// Fuzz (OpenPBR fuzz_*): a sheen lobe on top of the material, the "Charlie"
// distribution (Estevez & Kulla 2017) D = (2 + 1/a) sin^(1/a)(theta_h) / (2 pi)
// with Neubelt & Pettineo's visibility 1 / (4 (mu_i + mu_o - mu_i mu_o)); the
// layers below are attenuated by (1 - w E(mu_i)) (1 - w E(mu_o)), E the lobe's
// directional albedo (a table at mu = k/64, interpolated linearly, clamped to [0, 1]).
// (not inlined, as film_airy: materials without fuzz or film never call them,
// and inlined they raise the register count of the tail kernel, which runs
// beside the next pass's traversal, from 224 to 232: one traversal wave per
// SIMD fewer beside it, 5 % slower passes)
__host__ __device__ inline __attribute__((noinline)) float fuzz_f(float a, V3 wo, V3 wi) {
  if (wo.z <= 0.0f || wi.z <= 0.0f) return 0.0f;
  V3 h = normalize(wo + wi);
  const float sn = sqrtf(fmaxf(0.0f, 1.0f - h.z * h.z));
  const float D = (2.0f + 1.0f / a) * powf(sn, 1.0f / a) * (0.5f / kPi);
  const float V = 1.0f / (4.0f * (wi.z + wo.z - wi.z * wo.z));
  return D * V;
}

__host__ __device__ inline float fuzz_albedo(const MatRec& m, float mu) {
  const float t = fminf(fmaxf(mu, 0.0f), 1.0f) * 64.0f;
  const int k = min((int)floorf(t), 63);
  const float e = m.fuzz_E[k] + (t - (float)k) * (m.fuzz_E[k + 1] - m.fuzz_E[k]);
  return fminf(fmaxf(e, 0.0f), 1.0f);
}

template <int CLS>
__host__ __device__ inline float fuzz_att(const MatRec& m, float mu_i, float mu_o) {
  if (!Lobes<CLS>::Z || !(m.fuzz_w > 0.0f)) return 1.0f;
  return (1.0f - m.fuzz_w * fuzz_albedo(m, fabsf(mu_i))) * (1.0f - m.fuzz_w * fuzz_albedo(m, mu_o));
}

// Reflectance of the specular dielectric interface at incident cosine c: per
// channel, and the scalar Fs that chooses lobes and reflection vs refraction
// (the plain Fresnel without a film, the luminance of the three with one).
// One wavelength per channel: 650, 550, 450 nm.
template <int CLS>
__host__ __device__ inline V3 iface_fresnel(const MatRec& m, const Bsdf& b, float c, float& Fs) {
  const float F0 = fresnel_diel(c, b.eta);
  const float w = m.film_w;
  if (!Lobes<CLS>::F || !(w > 0.0f)) {
    Fs = F0;
    return v3(F0, F0, F0);
  }
  const float r = film_airy(c, b.film_n2, b.eta, m.film_ior, m.film_d_nm, 1.0f / 650.0f);
  const float g = film_airy(c, b.film_n2, b.eta, m.film_ior, m.film_d_nm, 1.0f / 550.0f);
  const float bl = film_airy(c, b.film_n2, b.eta, m.film_ior, m.film_d_nm, 1.0f / 450.0f);
  V3 F = v3((1.0f - w) * F0 + w * r, (1.0f - w) * F0 + w * g, (1.0f - w) * F0 + w * bl);
  Fs = lum(F.x, F.y, F.z);
  return F;
}

template <int CLS>
__host__ __device__ inline Bsdf bsdf_setup(const MatRec& m, bool entering, float mu_o) {
  using L = Lobes<CLS>;
  Bsdf b;
  b.entering = entering;
  const bool inside = m.trans_weight > 0.0f && !entering;
  b.eta = inside ? 1.0f / m.spec_ior : m.spec_ior;
  b.film_n2 = inside ? m.film_ior / m.spec_ior : m.film_ior;
  float Fc = L::C ? fresnel_diel(mu_o, m.coat_ior) : 0.0f;
  float Tc = 1.0f - m.coat_weight * Fc;
  float Fd = 0.0f;
  if (L::I || L::D) (void)iface_fresnel<CLS>(m, b, mu_o, Fd);
  float w0 = L::C ? m.coat_weight * Fc : 0.0f;
  float w1 = 0.0f;
  if (L::M) {
    V3 F = fresnel_f82(m, mu_o);
    w1 = Tc * m.metalness * m.spec_weight * lum(F.x, F.y, F.z);
  }
  float w2 = L::I ? Tc * (1.0f - m.metalness) * (Fd + m.trans_weight * (1.0f - Fd)) : 0.0f;
  float w3 = L::D ? Tc * (1.0f - m.metalness) * (1.0f - m.trans_weight) * (1.0f - Fd) * m.kd_lum : 0.0f;
  float w4 = 0.0f;
  if (L::Z && m.fuzz_w > 0.0f) {  // the fuzz reflects w E(mu_o) and passes the rest to the layers below
    const float fz = m.fuzz_w * fuzz_albedo(m, mu_o);
    w0 *= 1.0f - fz;
    w1 *= 1.0f - fz;
    w2 *= 1.0f - fz;
    w3 *= 1.0f - fz;
    w4 = fz * lum(m.fuzz_color[0], m.fuzz_color[1], m.fuzz_color[2]);
  }
  float sum = ((w0 + w1) + (w2 + w3)) + w4;
  b.absorbed = !(sum > 0.0f);
  float inv = b.absorbed ? 0.0f : 1.0f / sum;
  b.P[0] = w0 * inv;
  b.P[1] = w1 * inv;
  b.P[2] = w2 * inv;
  b.P[3] = w3 * inv;
  b.P[4] = w4 * inv;
  return b;
}

template <int CLS>
__host__ __device__ inline bool bsdf_has_nondelta(const MatRec& m, const Bsdf& b) {
  float s = b.P[3] + b.P[4];
  if (!(m.flags & kMatCoatDelta)) s += b.P[0];
  if (!(m.flags & kMatSpecDelta)) s += b.P[1] + b.P[2];
  return s > 0.0f;
}

template <int CLS>
__host__ __device__ inline V3 coat_layer(const MatRec& m, float mu_i, float mu_o) {
  if (!Lobes<CLS>::C) return v3(1.0f, 1.0f, 1.0f);
  float cw = m.coat_weight;
  float Fi = fresnel_diel(fabsf(mu_i), m.coat_ior), Fo = fresnel_diel(mu_o, m.coat_ior);
  float k = (1.0f - Fi) * (1.0f - Fo);
  return v3((1.0f - cw) + cw * m.coat_color[0] * k, (1.0f - cw) + cw * m.coat_color[1] * k,
            (1.0f - cw) + cw * m.coat_color[2] * k);
}

// Diffuse value (1/pi included) of albedo rho: Lambert when the material's
// FON B is 0, else EON, the energy-preserving Oren-Nayar model (Portsmouth,
// Kutz, Hill 2024) over Fujii's FON: rho (A + B s/t)/pi plus the
// multiple-scattering term rho_ms (1 - E(mu_o))(1 - E(mu_i)) / (pi (1 - Eb)),
// with E the FON albedo, Eb its cosine-weighted mean and
// rho_ms = rho^2 Eb / (1 - rho (1 - Eb)); s = wi.wo - mu_i mu_o.
__host__ __device__ inline float fon_albedo(float A, float B, float mu) {
  float sn = sqrtf(fmaxf(0.0f, 1.0f - mu * mu));
  float th = acosf(mu);
  float G = sn * (th - sn * mu + (2.0f / 3.0f) * mu * (1.0f + sn + sn * sn) / (1.0f + sn) - 2.0f / 3.0f);
  return A + B * (1.0f / kPi) * G;
}

__host__ __device__ inline float eon(const MatRec& m, float rho, float mu_i, float mu_o, float s) {
  const float A = m.eon_a, B = m.eon_b;
  if (!(B > 0.0f)) return rho * (1.0f / kPi);
  float t = s > 0.0f ? fmaxf(mu_i, mu_o) : 1.0f;
  float f = rho * (A + B * s / t) * (1.0f / kPi);
  float Eb = A + B * (2.0f / 3.0f - 28.0f / (15.0f * kPi));
  float Eo = fon_albedo(A, B, mu_o), Ei = fon_albedo(A, B, mu_i);
  float rho_ms = rho * rho * Eb / (1.0f - rho * (1.0f - Eb));
  return f + rho_ms * (1.0f / kPi) * (1.0f - Eo) * (1.0f - Ei) / (1.0f - Eb);
}

// Non-delta f(wo, wi) and the mixture pdf sum_k P_k pdf_k(wi).
template <int CLS>
__host__ __device__ inline V3 bsdf_eval(const MatRec& m, const Bsdf& b, V3 wo, V3 wi, float& pdf) {
  using L = Lobes<CLS>;
  pdf = 0.0f;
  V3 f = v3(0.0f, 0.0f, 0.0f);
  float mu_o = wo.z, mu_i = wi.z;
  if (b.absorbed || mu_o <= 0.0f || mu_i == 0.0f) return f;
  const bool spec_nd = !(m.flags & kMatSpecDelta);
  const bool coat_nd = !(m.flags & kMatCoatDelta);
  float mt = m.metalness, tw = m.trans_weight, sw = m.spec_weight;
  V3 Lc = coat_layer<CLS>(m, mu_i, mu_o);
  if (mu_i > 0.0f) {
    V3 h = normalize(wo + wi);
    float oh = dot(wo, h);
    float inv4 = 1.0f / (4.0f * mu_o * mu_i);
    float fc = 0.0f, pc = 0.0f;
    if (L::C && coat_nd && m.coat_weight > 0.0f) {
      float Dc = ggx_D(m.ac, m.ac, h);
      fc = m.coat_weight * fresnel_diel(oh, m.coat_ior) * Dc * ggx_G2(m.ac, m.ac, wo, wi) * inv4;
      pc = ggx_vndf_pdf(m.ac, m.ac, wo, h) / (4.0f * oh);
    }
    V3 fm = v3(0.0f, 0.0f, 0.0f);
    V3 fi = v3(0.0f, 0.0f, 0.0f);
    float pm = 0.0f, pi = 0.0f;
    if ((L::M || L::I) && spec_nd) {
      float D = ggx_D(m.at, m.ab, h);
      float g = ggx_G2(m.at, m.ab, wo, wi);
      float pv = ggx_vndf_pdf(m.at, m.ab, wo, h) / (4.0f * oh);
      if (L::M) {
        V3 F = fresnel_f82(m, oh);
        float k = sw * D * g * inv4;
        fm = v3(F.x * k, F.y * k, F.z * k);
        pm = pv;
      }
      if (L::I) {
        float Fi;
        const V3 Fiv = iface_fresnel<CLS>(m, b, oh, Fi);
        fi = v3(Fiv.x * D * g * inv4, Fiv.y * D * g * inv4, Fiv.z * D * g * inv4);
        float dn = Fi + tw * (1.0f - Fi);
        pi = dn > 0.0f ? (Fi / dn) * pv : 0.0f;
      }
    }
    V3 fd = v3(0.0f, 0.0f, 0.0f);
    if (L::D) {
      float Fsi, Fso;
      const V3 Fdi = iface_fresnel<CLS>(m, b, mu_i, Fsi), Fdo = iface_fresnel<CLS>(m, b, mu_o, Fso);
      float s = dot(wi, wo) - mu_i * mu_o;
      fd = v3((1.0f - tw) * (1.0f - Fdi.x) * (1.0f - Fdo.x) * eon(m, m.kd[0], mu_i, mu_o, s),
              (1.0f - tw) * (1.0f - Fdi.y) * (1.0f - Fdo.y) * eon(m, m.kd[1], mu_i, mu_o, s),
              (1.0f - tw) * (1.0f - Fdi.z) * (1.0f - Fdo.z) * eon(m, m.kd[2], mu_i, mu_o, s));
    }
    float fx = fc + Lc.x * (mt * fm.x + (1.0f - mt) * (fi.x + fd.x));
    float fy = fc + Lc.y * (mt * fm.y + (1.0f - mt) * (fi.y + fd.y));
    float fz = fc + Lc.z * (mt * fm.z + (1.0f - mt) * (fi.z + fd.z));
    if (L::Z && m.fuzz_w > 0.0f) {
      const float A = fuzz_att<CLS>(m, mu_i, mu_o);
      const float zf = m.fuzz_w * fuzz_f(m.fuzz_a, wo, wi);
      fx = zf * m.fuzz_color[0] + A * fx;
      fy = zf * m.fuzz_color[1] + A * fy;
      fz = zf * m.fuzz_color[2] + A * fz;
    }
    f = v3(fx, fy, fz);
    pdf = b.P[0] * pc + b.P[1] * pm + b.P[2] * pi + b.P[3] * (mu_i * (1.0f / kPi));
    if (L::Z) pdf += b.P[4] * (mu_i * (1.0f / kPi));
    return f;
  }
  if (!L::T || !spec_nd || tw <= 0.0f) return f;
  float eta = b.eta;
  V3 h = normalize(wo + wi * eta);
  if (h.z < 0.0f) h = h * -1.0f;
  float oh = dot(wo, h), ih = dot(wi, h);
  if (oh <= 0.0f || ih >= 0.0f) return f;
  float F;
  const V3 Fv = iface_fresnel<CLS>(m, b, oh, F);
  float s = ih + oh / eta;
  float denom = s * s;
  float D = ggx_D(m.at, m.ab, h);
  float g = ggx_G2(m.at, m.ab, wo, wi);
  const float den = denom * fabsf(mu_i) * mu_o;
  const float btx = tw * (1.0f - Fv.x) * D * g * fabsf(ih) * fabsf(oh) / den / (eta * eta);
  const float bty = tw * (1.0f - Fv.y) * D * g * fabsf(ih) * fabsf(oh) / den / (eta * eta);
  const float btz = tw * (1.0f - Fv.z) * D * g * fabsf(ih) * fabsf(oh) / den / (eta * eta);
  float tr = b.entering ? m.trans_color[0] : 1.0f, tg = b.entering ? m.trans_color[1] : 1.0f,
        tb = b.entering ? m.trans_color[2] : 1.0f;
  f = v3(Lc.x * ((1.0f - mt) * btx) * tr, Lc.y * ((1.0f - mt) * bty) * tg, Lc.z * ((1.0f - mt) * btz) * tb);
  float dn = F + tw * (1.0f - F);
  float pr = dn > 0.0f ? F / dn : 0.0f;
  pdf = b.P[2] * (1.0f - pr) * ggx_vndf_pdf(m.at, m.ab, wo, h) * fabsf(ih) / denom;
  return f;
}

__host__ __device__ inline V3 reflect_about(V3 wo, V3 m) { return m * (2.0f * dot(wo, m)) - wo; }

__host__ __device__ inline bool refract_about(V3 wo, V3 m, float eta, V3& wi) {
  float c = dot(wo, m);
  float k = 1.0f - (1.0f - c * c) / (eta * eta);
  if (k < 0.0f) return false;
  wi = wo * (-1.0f / eta) + m * (c / eta - sqrtf(k));
  return true;
}

struct BsdfSample {
  V3 wi;
  V3 weight;
  float pdf;
  bool ok, delta, refract;
  int lobe;  // 0 coat, 1 metal, 2 interface reflection, 3 interface refraction, 4 diffuse, -1 none
};

template <int CLS>
__host__ __device__ inline BsdfSample bsdf_sample(const MatRec& m, const Bsdf& b, V3 wo, float u_lobe, float u1,
                                                  float u2, float u_rt) {
  using L = Lobes<CLS>;
  BsdfSample s;
  s.ok = false;
  s.delta = false;
  s.refract = false;
  s.lobe = -1;
  s.pdf = 0.0f;
  s.weight = v3(0.0f, 0.0f, 0.0f);
  s.wi = v3(0.0f, 0.0f, 1.0f);
  float mu_o = wo.z;
  if (b.absorbed || mu_o <= 0.0f) return s;
  // lobe choice against the cumulative pmf; rounding overflow picks the last nonzero lobe
  int lobe = -1, last = -1;
  float acc = 0.0f;
#pragma unroll
  for (int k = 0; k < (L::Z ? 5 : 4); ++k) {
    if (b.P[k] > 0.0f) {
      last = k;
      if (lobe < 0 && u_lobe < acc + b.P[k]) lobe = k;
    }
    acc += b.P[k];
  }
  if (lobe < 0) lobe = last;
  if (lobe < 0) return s;
  const bool spec_delta = (m.flags & kMatSpecDelta) != 0;
  const bool coat_delta = (m.flags & kMatCoatDelta) != 0;
  float mt = m.metalness, tw = m.trans_weight, sw = m.spec_weight;
  V3 d;
  if (L::C && lobe == 0) {
    s.lobe = 0;
    if (coat_delta) {
      s.wi = v3(-wo.x, -wo.y, wo.z);
      float w = fuzz_att<CLS>(m, mu_o, mu_o) * m.coat_weight * fresnel_diel(mu_o, m.coat_ior) / b.P[0];
      s.weight = v3(w, w, w);
      s.delta = true;
      s.ok = true;
      return s;
    }
    V3 h = ggx_vndf_sample(m.ac, m.ac, wo, u1, u2);
    d = reflect_about(wo, h);
    if (d.z <= 0.0f) return s;
  } else if (L::M && lobe == 1) {
    s.lobe = 1;
    if (spec_delta) {
      s.wi = v3(-wo.x, -wo.y, wo.z);
      V3 Lc = coat_layer<CLS>(m, mu_o, mu_o);
      V3 F = fresnel_f82(m, mu_o);
      float k = mt * sw / b.P[1];
      const float A = fuzz_att<CLS>(m, mu_o, mu_o);
      s.weight = v3(A * (Lc.x * F.x * k), A * (Lc.y * F.y * k), A * (Lc.z * F.z * k));
      s.delta = true;
      s.ok = true;
      return s;
    }
    V3 h = ggx_vndf_sample(m.at, m.ab, wo, u1, u2);
    d = reflect_about(wo, h);
    if (d.z <= 0.0f) return s;
  } else if (L::I && lobe == 2) {
    float eta = b.eta;
    if (spec_delta) {
      float F;
      const V3 Fv = iface_fresnel<CLS>(m, b, mu_o, F);
      float dn = F + tw * (1.0f - F);
      float pr = dn > 0.0f ? F / dn : 0.0f;
      s.delta = true;
      if (u_rt < pr) {
        s.lobe = 2;
        s.wi = v3(-wo.x, -wo.y, wo.z);
        V3 Lc = coat_layer<CLS>(m, mu_o, mu_o);
        const float q = b.P[2] * pr;
        const float A = fuzz_att<CLS>(m, mu_o, mu_o);
        s.weight = v3(A * (Lc.x * ((1.0f - mt) * Fv.x / q)), A * (Lc.y * ((1.0f - mt) * Fv.y / q)),
                      A * (Lc.z * ((1.0f - mt) * Fv.z / q)));
        s.ok = true;
        return s;
      }
      s.lobe = 3;
      V3 t;
      if (!L::T || !refract_about(wo, v3(0.0f, 0.0f, 1.0f), eta, t)) return s;
      s.wi = t;
      s.refract = true;
      V3 Lc = coat_layer<CLS>(m, t.z, mu_o);
      const float q = b.P[2] * (1.0f - pr);
      float tr = b.entering ? m.trans_color[0] : 1.0f, tg = b.entering ? m.trans_color[1] : 1.0f,
            tb = b.entering ? m.trans_color[2] : 1.0f;
      s.weight = v3(Lc.x * ((1.0f - mt) * tw * (1.0f - Fv.x) / (eta * eta) / q) * tr,
                    Lc.y * ((1.0f - mt) * tw * (1.0f - Fv.y) / (eta * eta) / q) * tg,
                    Lc.z * ((1.0f - mt) * tw * (1.0f - Fv.z) / (eta * eta) / q) * tb);
      s.ok = true;
      return s;
    }
    V3 h = ggx_vndf_sample(m.at, m.ab, wo, u1, u2);
    float F;
    (void)iface_fresnel<CLS>(m, b, dot(wo, h), F);
    float dn = F + tw * (1.0f - F);
    float pr = dn > 0.0f ? F / dn : 0.0f;
    if (u_rt < pr) {
      s.lobe = 2;
      d = reflect_about(wo, h);
      if (d.z <= 0.0f) return s;
    } else {
      s.lobe = 3;
      if (!L::T || !refract_about(wo, h, eta, d)) return s;
      if (d.z >= 0.0f) return s;
      s.refract = true;
    }
  } else if ((L::D && lobe == 3) || (L::Z && lobe == 4)) {  // diffuse or fuzz: cosine-weighted
    s.lobe = lobe == 4 ? 5 : 4;
    float r = sqrtf(u1);
    float sn, cs;
    sincosf(2.0f * kPi * u2, &sn, &cs);
    d = v3(r * cs, r * sn, sqrtf(fmaxf(0.0f, 1.0f - u1)));
    if (d.z <= 0.0f) return s;
  } else {
    return s;
  }
  float p;
  V3 f = bsdf_eval<CLS>(m, b, wo, d, p);
  if (!(p > 0.0f)) {
    s.refract = false;
    return s;
  }
  s.wi = d;
  s.pdf = p;
  float k = fabsf(d.z) / p;
  s.weight = v3(f.x * k, f.y * k, f.z * k);
  s.ok = true;
  return s;
}

// Shading frame: tangent from the object's +z axis projected on the tangent
// plane, or the Duff et al. 2017 basis when that projection is short.
__host__ __device__ inline void make_frame(V3 n, V3 a, V3& t, V3& b) {
  V3 p = a - n * dot(n, a);
  float l = length(p);
  if (l >= 1e-3f) {
    t = p * (1.0f / l);
  } else {
    float sg = n.z >= 0.0f ? 1.0f : -1.0f;
    float aa = -1.0f / (sg + n.z);
    float bb = n.x * n.y * aa;
    t = v3(1.0f + sg * n.x * n.x * aa, sg * bb, -sg * n.x);
  }
  b = cross(n, t);
}

}  // namespace pt
