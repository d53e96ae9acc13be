/*
 * Oracle BSDF: the OpenPBR subset used by the path tracer, in FP64.
 *
 * The paper adopts the OpenPBR uber-shader (Sec. 4) and supports metallic,
 * glossy and diffuse surfaces with importance sampling toward the mirror
 * direction for metals and around the normal for diffuse (Sec. 5.1.3).  It
 * gives no formulas; the ones below are this project's reading, built from
 * published models:
 *
 *   roughness r -> alpha = r^2; anisotropy a: alpha_t = alpha*sqrt(2/(1+(1-a)^2)),
 *     alpha_b = (1-a)*alpha_t, both clamped >= 1e-4 (OpenPBR mapping);
 *     a lobe with r < 1e-3 is a delta lobe.
 *   GGX D, Smith Lambda, height-correlated G2 = 1/(1+L(o)+L(i)) (Heitz 2014),
 *     visible-normal sampling (Heitz 2018).
 *   Dielectric Fresnel: exact unpolarised form (Walter et al. 2007, eq. 22).
 *   Metal Fresnel: OpenPBR F82-tint.
 *   Lobes: C coat (dielectric GGX reflection), M metal, I dielectric interface
 *   (GGX reflection + rough refraction, Walter et al. 2007 eq. 21, with the
 *   1/eta^2 radiance factor), D diffuse attenuated by the interface Fresnel:
 *   Lambert, or with base_diffuse_roughness sigma > 0 the energy-preserving
 *   Oren-Nayar model EON (Portsmouth, Kutz, Hill 2024) over Fujii's FON:
 *   f = rho (A + B s/t)/pi + rho_ms (1 - E(mu_o))(1 - E(mu_i)) / (pi (1 - Eb)),
 *   A = 1/(1 + (1/2 - 2/(3 pi)) sigma), B = sigma A, s = wi.wo - mu_i mu_o,
 *   t = max(mu_i, mu_o) if s > 0 else 1, E(mu) = A + (B/pi) G(mu) the FON
 *   albedo with G(mu) = sin(th) (th - sin(th) mu + (2/3)(1 - sin^3(th))/mu - 2/3),
 *   Eb = A + B (2/3 - 28/(15 pi)) its cosine-weighted mean,
 *   rho_ms = rho^2 Eb / (1 - rho (1 - Eb)); sampled by the cosine.  Its
 *   albedo rho mixes the glossy diffuse bw*bc and OpenPBR's subsurface in
 *   its local limit (no light moving sideways under the surface: a diffuse
 *   reflector of albedo subsurface_color): rho = (1-ssw) bw*bc + ssw*ssc.
 *   specular_weight xi modulates the dielectric IOR (OpenPBR): the interface
 *   and the cache input use eta' with F0(eta') = xi F0(eta), so reflection,
 *   refraction and the diffuse attenuation stay consistent; the metal
 *   Fresnel is scaled by xi.
 *   f = C + [(1-cw) + cw*coat_color*(1-Fc(|mu_i|))(1-Fc(mu_o))]
 *           * [metalness*M + (1-metalness)*(I + D)].
 *   Lobe choice pmf at mu_o: w_C = cw*Fc, w_M = Tc*metalness*sw*lum(F82),
 *   w_I = Tc*(1-metalness)*(Fd + tw*(1-Fd)), w_D = Tc*(1-metalness)*(1-tw)*(1-Fd)*lum(rho),
 *   Tc = 1 - cw*Fc(mu_o), Fd = F(mu_o, eta').
 *   Non-delta sampling weight: f_nd*|cos|/sum_k P_k pdf_k (one-sample MIS over lobes).
 *
 * Frame: local +z is the surface normal flipped to the side of wo, so mu_o > 0.
 */
#include <pthread.h>
#include <string.h>

#include "oracle_internal.h"

double ofresnel_diel(double c, double eta) {
  /* Walter et al. 2007 eq. 22 with c = |cos| on the incident side, eta = n_t/n_i */
  c = fabs(c);
  double g2 = eta * eta - 1.0 + c * c;
  if (g2 < 0.0) return 1.0;
  double g = sqrt(g2);
  double a = (g - c) / (g + c);
  double b = (c * (g + c) - 1.0) / (c * (g - c) + 1.0);
  return 0.5 * a * a * (1.0 + b * b);
}

/*
 * Thin film on the dielectric interface (OpenPBR thin_film_*; the paper's
 * Sec. 4 names OpenPBR): reflectance of the stack incident medium (index 1)
 * | film (relative index n2) | base (relative index n3) at incident cosine
 * c1, for one wavelength, by Airy summation of the multiply reflected waves:
 * per polarisation R = (r12^2 + r23^2 + 2 r12 r23 cos d) /
 * (1 + r12^2 r23^2 + 2 r12 r23 cos d), with the Fresnel amplitudes
 * r_ij = (a_i - a_j) / (a_i + a_j), a = n cos (s) or cos / n (p), and the
 * phase d = 2 pi (2 film_ior d_nm cos_film / lambda); unpolarised: the mean.
 * Total internal reflection at either interface gives 1 (no propagating
 * wave leaves: the film's index is at least 1, so an evanescent film also
 * means an evanescent exit).
 */
double ofilm_airy(double c1, double n2, double n3, double film_ior, double d_nm, double lambda_nm) {
  c1 = fabs(c1);
  double s2 = 1.0 - c1 * c1;
  double c2sq = 1.0 - s2 / (n2 * n2), c3sq = 1.0 - s2 / (n3 * n3);
  if (c2sq < 0.0 || c3sq < 0.0) return 1.0;
  double c2 = sqrt(c2sq), c3 = sqrt(c3sq);
  double cd = cos(2.0 * O_PI * (2.0 * film_ior * d_nm * c2 / lambda_nm));
  double a[2][3] = {{c1, n2 * c2, n3 * c3}, {c1, c2 / n2, c3 / n3}};
  double R = 0.0;
  for (int pol = 0; pol < 2; ++pol) {
    double r12 = (a[pol][0] - a[pol][1]) / (a[pol][0] + a[pol][1]);
    double r23 = (a[pol][1] - a[pol][2]) / (a[pol][1] + a[pol][2]);
    double x = 2.0 * r12 * r23 * cd;
    R += 0.5 * (r12 * r12 + r23 * r23 + x) / (1.0 + r12 * r12 * r23 * r23 + x);
  }
  return R;
}

/* one wavelength per channel (nm) */
static const double FILM_LAMBDA[3] = {650.0, 550.0, 450.0};

/* Reflectance of the specular dielectric interface at incident cosine c:
 * per channel F[k], and the scalar Fs that chooses lobes and reflection vs
 * refraction (the plain Fresnel without a film, the luminance with one). */
void oiface_fresnel(const obsdf* b, double c, double F[3], double* Fs) {
  double F0 = ofresnel_diel(c, b->eta);
  double w = b->m.film_weight;
  if (!(w > 0.0)) {
    F[0] = F[1] = F[2] = F0;
    *Fs = F0;
    return;
  }
  for (int k = 0; k < 3; ++k) {
    double Rf = ofilm_airy(c, b->film_n2, b->eta, b->m.film_ior, 1000.0 * b->m.film_thickness_um, FILM_LAMBDA[k]);
    F[k] = (1.0 - w) * F0 + w * Rf;
  }
  *Fs = lum3(F);
}

/*
 * Fuzz (OpenPBR fuzz_weight, fuzz_color, fuzz_roughness): a sheen lobe on
 * top of the material.  Reading: the "Charlie" sheen distribution of
 * Estevez & Kulla (2017), D(h) = (2 + 1/a) sin(theta_h)^(1/a) / (2 pi) with
 * a = max(roughness^2, 1e-2), and the visibility term of Neubelt & Pettineo
 * (2013), V = 1 / (4 (mu_i + mu_o - mu_i mu_o)); f = w fuzz_color D V.  The
 * layers below are attenuated by (1 - w E(mu_i)) (1 - w E(mu_o)), E the
 * lobe's directional albedo, so the fuzz takes the energy it reflects.
 */
double ofuzz_alpha(double r) {
  double a = r * r;
  return a < 1e-2 ? 1e-2 : a;
}

double ofuzz_f(double alpha, v3 wo, v3 wi) {
  if (wo.z <= 0.0 || wi.z <= 0.0) return 0.0;
  v3 h = vnorm(vadd(wo, wi));
  double s2 = 1.0 - h.z * h.z;
  double sn = s2 > 0.0 ? sqrt(s2) : 0.0;
  double D = (2.0 + 1.0 / alpha) * pow(sn, 1.0 / alpha) / (2.0 * O_PI);
  double V = 1.0 / (4.0 * (wi.z + wo.z - wi.z * wo.z));
  return D * V;
}

/* E(mu_k) for mu_k = k / 64: the midpoint rule over mu_i in [0, 1] and phi in
 * [0, 2 pi) with 256 x 256 cells of the cosine-weighted lobe (the table is
 * defined by this rule), for wo = (sqrt(1 - mu^2), 0, mu).  Tables are kept
 * per roughness: a render builds each once per material. */
#define FUZZ_CACHE 16
static pthread_mutex_t fuzz_mu = PTHREAD_MUTEX_INITIALIZER;
static double fuzz_cache_r[FUZZ_CACHE];
static double fuzz_cache_E[FUZZ_CACHE][65];
static int fuzz_cache_n = 0;

void ofuzz_table(double rough, double E[65]) {
  pthread_mutex_lock(&fuzz_mu);
  for (int i = 0; i < fuzz_cache_n; ++i)
    if (fuzz_cache_r[i] == rough) {
      memcpy(E, fuzz_cache_E[i], sizeof(double) * 65);
      pthread_mutex_unlock(&fuzz_mu);
      return;
    }
  pthread_mutex_unlock(&fuzz_mu);
  const int N = 256, M = 256;
  double alpha = ofuzz_alpha(rough);
  for (int k = 0; k <= 64; ++k) {
    double mu = k / 64.0;
    v3 wo = V(sqrt(1.0 - mu * mu), 0.0, mu);
    double acc = 0.0;
    for (int a = 0; a < N; ++a) {
      double mi = (a + 0.5) / N, si = sqrt(1.0 - mi * mi);
      for (int b = 0; b < M; ++b) {
        double phi = 2.0 * O_PI * (b + 0.5) / M;
        v3 wi = V(si * cos(phi), si * sin(phi), mi);
        /* D V written out rather than ofuzz_f, which is zero for wo on the horizon: the entry at
           mu = 0 is the integrand's value there (its limit), not zero */
        v3 h = vnorm(vadd(wo, wi));
        double s2 = 1.0 - h.z * h.z;
        double sn = s2 > 0.0 ? sqrt(s2) : 0.0;
        double D = (2.0 + 1.0 / alpha) * pow(sn, 1.0 / alpha) / (2.0 * O_PI);
        acc += D / (4.0 * (wi.z + wo.z - wi.z * wo.z)) * mi;
      }
    }
    E[k] = acc * (1.0 / N) * (2.0 * O_PI / M);
  }
  pthread_mutex_lock(&fuzz_mu);
  int slot = fuzz_cache_n < FUZZ_CACHE ? fuzz_cache_n++ : FUZZ_CACHE - 1;
  fuzz_cache_r[slot] = rough;
  memcpy(fuzz_cache_E[slot], E, sizeof(double) * 65);
  pthread_mutex_unlock(&fuzz_mu);
}

/* E at mu by linear interpolation of the table, clamped to [0, 1] */
double ofuzz_albedo(const omat* m, double mu) {
  double t = (mu < 0.0 ? 0.0 : (mu > 1.0 ? 1.0 : mu)) * 64.0;
  int k = (int)floor(t);
  if (k > 63) k = 63;
  double e = m->fuzz_E[k] + (t - k) * (m->fuzz_E[k + 1] - m->fuzz_E[k]);
  return e < 0.0 ? 0.0 : (e > 1.0 ? 1.0 : e);
}

/* attenuation of the layers under the fuzz */
static double fuzz_att(const omat* m, double mu_i, double mu_o) {
  double w = m->fuzz_weight;
  if (!(w > 0.0)) return 1.0;
  return (1.0 - w * ofuzz_albedo(m, fabs(mu_i))) * (1.0 - w * ofuzz_albedo(m, mu_o));
}

double odiffuse_albedo(const omat* m, int c) {
  return (1.0 - m->ss_weight) * m->base_weight * m->base_color[c] + m->ss_weight * m->ss_color[c];
}

double omod_ior(const omat* m) {
  /* F0(eta') = xi F0(eta): eta' = (1 + sqrt(xi F0)) / (1 - sqrt(xi F0)), inverted below 1 */
  double eta = m->spec_ior, xi = m->spec_weight;
  if (xi >= 1.0) return eta;
  double r0 = (eta - 1.0) / (eta + 1.0);
  double r = sqrt(xi * r0 * r0);
  return eta >= 1.0 ? (1.0 + r) / (1.0 - r) : (1.0 - r) / (1.0 + r);
}

/* FON albedo E(mu) for rho = 1 and its cosine-weighted mean Eb */
static double ofon_albedo(double A, double B, double mu) {
  double sn = sqrt(1.0 - mu * mu > 0.0 ? 1.0 - mu * mu : 0.0);
  double th = acos(mu);
  double G = sn * (th - sn * mu + (2.0 / 3.0) * mu * (1.0 + sn + sn * sn) / (1.0 + sn) - 2.0 / 3.0);
  return A + B / O_PI * G;
}

double oeon(double rho, double sigma, double mu_i, double mu_o, double s) {
  if (!(sigma > 0.0)) return rho / O_PI;
  double A = 1.0 / (1.0 + (0.5 - 2.0 / (3.0 * O_PI)) * sigma), B = sigma * A;
  double t = s > 0.0 ? (mu_i > mu_o ? mu_i : mu_o) : 1.0;
  double f = rho * (A + B * s / t) / O_PI;
  double Eb = A + B * (2.0 / 3.0 - 28.0 / (15.0 * O_PI));
  double Eo = ofon_albedo(A, B, mu_o), Ei = ofon_albedo(A, B, mu_i);
  double rho_ms = rho * rho * Eb / (1.0 - rho * (1.0 - Eb));
  return f + rho_ms / O_PI * (1.0 - Eo) * (1.0 - Ei) / (1.0 - Eb);
}

void of82(const omat* m, double mu, double F[3]) {
  /* OpenPBR F82-tint: Schlick S(mu) corrected so that F(1/7) = specular_color * S(1/7) */
  const double mb = 1.0 / 7.0;
  double om = 1.0 - mu;
  double om5 = om * om * om * om * om;
  double omb = 1.0 - mb;
  double omb5 = omb * omb * omb * omb * omb, omb6 = omb5 * omb;
  for (int c = 0; c < 3; ++c) {
    double F0 = m->base_weight * m->base_color[c];
    double S = F0 + (1.0 - F0) * om5;
    double Sb = F0 + (1.0 - F0) * omb5;
    double b = Sb * (1.0 - m->spec_color[c]) / (mb * omb6);
    double v = S - mu * om5 * om * b;
    F[c] = v < 0.0 ? 0.0 : (v > 1.0 ? 1.0 : v);
  }
}

double oggx_D(double at, double ab, v3 m) {
  if (m.z <= 0.0) return 0.0;
  double x = m.x / at, y = m.y / ab;
  double k = x * x + y * y + m.z * m.z;
  return 1.0 / (O_PI * at * ab * k * k);
}

double oggx_lambda(double at, double ab, v3 w) {
  double z2 = w.z * w.z;
  if (z2 == 0.0) return INFINITY;
  double a2 = (at * at * w.x * w.x + ab * ab * w.y * w.y) / z2;
  return 0.5 * (-1.0 + sqrt(1.0 + a2));
}

v3 oggx_vndf_sample(double at, double ab, v3 wo, double u1, double u2) {
  /* Heitz 2018: sample the visible hemisphere of the stretched configuration */
  v3 Vh = vnorm(V(at * wo.x, ab * wo.y, wo.z));
  double lensq = Vh.x * Vh.x + Vh.y * Vh.y;
  v3 T1 = lensq > 0.0 ? vmul(V(-Vh.y, Vh.x, 0.0), 1.0 / sqrt(lensq)) : V(1.0, 0.0, 0.0);
  v3 T2 = vcross(Vh, T1);
  double r = sqrt(u1);
  double phi = 2.0 * O_PI * u2;
  double t1 = r * cos(phi), t2 = r * sin(phi);
  double s = 0.5 * (1.0 + Vh.z);
  t2 = (1.0 - s) * sqrt(1.0 - t1 * t1) + s * t2;
  double tz = 1.0 - t1 * t1 - t2 * t2;
  v3 Nh = vadd(vadd(vmul(T1, t1), vmul(T2, t2)), vmul(Vh, sqrt(tz > 0.0 ? tz : 0.0)));
  return vnorm(V(at * Nh.x, ab * Nh.y, Nh.z > 0.0 ? Nh.z : 0.0));
}

double oggx_vndf_pdf(double at, double ab, v3 wo, v3 m) {
  /* density of m: G1(wo) max(0, wo.m) D(m) / wo.z */
  double wm = vdot(wo, m);
  if (wm <= 0.0 || wo.z <= 0.0) return 0.0;
  double G1 = 1.0 / (1.0 + oggx_lambda(at, ab, wo));
  return G1 * wm * oggx_D(at, ab, m) / wo.z;
}

static double clampa(double a) { return a < 1e-4 ? 1e-4 : a; }

void obsdf_setup(const omat* m, int entering, double mu_o, obsdf* b) {
  b->m = *m;
  b->entering = entering;
  double ior = omod_ior(m);
  b->eta = (m->trans_weight > 0.0 && !entering) ? 1.0 / ior : ior;
  double r = m->spec_rough, a = m->spec_aniso;
  double alpha = r * r;
  double at = alpha * sqrt(2.0 / (1.0 + (1.0 - a) * (1.0 - a)));
  b->at = clampa(at);
  b->ab = clampa((1.0 - a) * at);
  b->spec_delta = r < 1e-3;
  b->ac = clampa(m->coat_rough * m->coat_rough);
  b->coat_delta = m->coat_rough < 1e-3;
  double cw = m->coat_weight, mt = m->metalness, tw = m->trans_weight, sw = m->spec_weight;
  /* the film's index relative to the medium wo is in: air, or the base when leaving a transmissive one */
  b->film_n2 = (m->trans_weight > 0.0 && !entering) ? m->film_ior / ior : m->film_ior;
  double Fc = ofresnel_diel(mu_o, m->coat_ior);
  double Tc = 1.0 - cw * Fc;
  double Fdv[3], Fd;
  oiface_fresnel(b, mu_o, Fdv, &Fd);
  double F82[3];
  of82(m, mu_o, F82);
  double rho[3] = {odiffuse_albedo(m, 0), odiffuse_albedo(m, 1), odiffuse_albedo(m, 2)};
  double w[5];
  w[LOBE_C] = cw * Fc;
  w[LOBE_M] = Tc * mt * sw * lum3(F82);
  w[LOBE_I] = Tc * (1.0 - mt) * (Fd + tw * (1.0 - Fd));
  w[LOBE_D] = Tc * (1.0 - mt) * (1.0 - tw) * (1.0 - Fd) * lum3(rho);
  w[LOBE_Z] = 0.0;
  if (m->fuzz_weight > 0.0) {  /* the fuzz reflects w E(mu_o) and passes the rest to the layers below */
    double fz = m->fuzz_weight * ofuzz_albedo(m, mu_o);
    for (int k = 0; k < 4; ++k) w[k] *= 1.0 - fz;
    w[LOBE_Z] = fz * lum3(m->fuzz_color);
  }
  double sum = ((w[0] + w[1]) + (w[2] + w[3])) + w[4];
  b->absorbed = !(sum > 0.0);
  for (int k = 0; k < 5; ++k) b->P[k] = b->absorbed ? 0.0 : w[k] / sum;
}

int obsdf_has_nondelta(const obsdf* b) {
  double s = b->P[LOBE_D] + b->P[LOBE_Z];
  if (!b->coat_delta) s += b->P[LOBE_C];
  if (!b->spec_delta) s += b->P[LOBE_M] + b->P[LOBE_I];
  return s > 0.0;
}

/* (1-cw) + cw*coat_color*(1-Fc(|mu_i|))*(1-Fc(mu_o)) */
static void coat_layer(const obsdf* b, double mu_i, double mu_o, double L[3]) {
  double cw = b->m.coat_weight;
  double Fi = ofresnel_diel(fabs(mu_i), b->m.coat_ior), Fo = ofresnel_diel(mu_o, b->m.coat_ior);
  for (int c = 0; c < 3; ++c) L[c] = (1.0 - cw) + cw * b->m.coat_color[c] * (1.0 - Fi) * (1.0 - Fo);
}

static double G2(double at, double ab, v3 wo, v3 wi) {
  return 1.0 / (1.0 + oggx_lambda(at, ab, wo) + oggx_lambda(at, ab, wi));
}

/* half vector of a refraction pair: normalize(wo + eta*wi), oriented to +z */
static v3 refr_half(v3 wo, v3 wi, double eta) {
  v3 h = vnorm(vadd(wo, vmul(wi, eta)));
  if (h.z < 0.0) h = vmul(h, -1.0);
  return h;
}

/* Non-delta BSDF value f(wo, wi) and the one-sample mixture pdf sum_k P_k pdf_k(wi). */
void obsdf_eval(const obsdf* b, v3 wo, v3 wi, double f[3], double* pdf) {
  f[0] = f[1] = f[2] = 0.0;
  *pdf = 0.0;
  double mu_o = wo.z, mu_i = wi.z;
  if (b->absorbed || mu_o <= 0.0 || mu_i == 0.0) return;
  const omat* m = &b->m;
  double mt = m->metalness, tw = m->trans_weight, sw = m->spec_weight, cw = m->coat_weight;
  double L[3];
  coat_layer(b, mu_i, mu_o, L);
  if (mu_i > 0.0) {
    v3 h = vnorm(vadd(wo, wi));
    double oh = vdot(wo, h);
    double fc = 0.0, pc = 0.0;
    if (!b->coat_delta && cw > 0.0) {
      double Dc = oggx_D(b->ac, b->ac, h);
      fc = cw * ofresnel_diel(oh, m->coat_ior) * Dc * G2(b->ac, b->ac, wo, wi) / (4.0 * mu_o * mu_i);
      pc = oggx_vndf_pdf(b->ac, b->ac, wo, h) / (4.0 * oh);
    }
    double fm[3] = {0, 0, 0}, fi[3] = {0, 0, 0}, pm = 0.0, pi = 0.0;
    if (!b->spec_delta) {
      double D = oggx_D(b->at, b->ab, h);
      double g = G2(b->at, b->ab, wo, wi);
      double pv = oggx_vndf_pdf(b->at, b->ab, wo, h) / (4.0 * oh);
      double F82[3];
      of82(m, oh, F82);
      for (int c = 0; c < 3; ++c) fm[c] = sw * F82[c] * D * g / (4.0 * mu_o * mu_i);
      double Fiv[3], Fi;
      oiface_fresnel(b, oh, Fiv, &Fi);
      for (int c = 0; c < 3; ++c) fi[c] = Fiv[c] * D * g / (4.0 * mu_o * mu_i);
      pm = pv;
      double denom = Fi + tw * (1.0 - Fi);
      pi = denom > 0.0 ? (Fi / denom) * pv : 0.0;
    }
    double Fdi[3], Fdo[3], Fsi, Fso;
    oiface_fresnel(b, mu_i, Fdi, &Fsi);
    oiface_fresnel(b, mu_o, Fdo, &Fso);
    double s = vdot(wi, wo) - mu_i * mu_o;
    double A = fuzz_att(m, mu_i, mu_o);
    double fz = m->fuzz_weight > 0.0 ? m->fuzz_weight * ofuzz_f(ofuzz_alpha(m->fuzz_rough), wo, wi) : 0.0;
    for (int c = 0; c < 3; ++c) {
      double kd = (1.0 - tw) * (1.0 - Fdi[c]) * (1.0 - Fdo[c]);
      double fd = kd * oeon(odiffuse_albedo(m, c), m->diffuse_roughness, mu_i, mu_o, s);
      f[c] = fz * m->fuzz_color[c] + A * (fc + L[c] * (mt * fm[c] + (1.0 - mt) * (fi[c] + fd)));
    }
    *pdf = b->P[LOBE_C] * pc + b->P[LOBE_M] * pm + b->P[LOBE_I] * pi + b->P[LOBE_D] * (mu_i / O_PI) +
           b->P[LOBE_Z] * (mu_i / O_PI);
  } else {
    if (b->spec_delta || tw <= 0.0) return;
    double eta = b->eta;
    v3 h = refr_half(wo, wi, eta);
    double oh = vdot(wo, h), ih = vdot(wi, h);
    if (oh <= 0.0 || ih >= 0.0) return;
    double Fv[3], F;
    oiface_fresnel(b, oh, Fv, &F);
    double s = ih + oh / eta;
    double denom = s * s;
    double D = oggx_D(b->at, b->ab, h);
    double g = G2(b->at, b->ab, wo, wi);
    for (int c = 0; c < 3; ++c) {
      double bt = tw * (1.0 - Fv[c]) * D * g * fabs(ih) * fabs(oh) / (denom * fabs(mu_i) * mu_o) / (eta * eta);
      double tint = b->entering ? m->trans_color[c] : 1.0;
      f[c] = L[c] * (1.0 - mt) * bt * tint;
    }
    double dn = F + tw * (1.0 - F);
    double pr = dn > 0.0 ? F / dn : 0.0;
    *pdf = b->P[LOBE_I] * (1.0 - pr) * oggx_vndf_pdf(b->at, b->ab, wo, h) * fabs(ih) / denom;
  }
}

static v3 reflect_about(v3 wo, v3 m) { return vsub(vmul(m, 2.0 * vdot(wo, m)), wo); }

/* refraction of wo through microfacet m (wo.m > 0), eta = n_t/n_i; returns 0 on TIR */
static int refract_about(v3 wo, v3 m, double eta, v3* wi) {
  double c = vdot(wo, m);
  double k = 1.0 - (1.0 - c * c) / (eta * eta);
  if (k < 0.0) return 0;
  *wi = vadd(vmul(wo, -1.0 / eta), vmul(m, c / eta - sqrt(k)));
  return 1;
}

/*
 * Sample a direction: lobe by u_lobe against the cumulative pmf (C, M, I, D,
 * Z; if rounding leaves u_lobe past the last bucket, the last lobe with
 * nonzero probability is taken), microfacet or cosine direction from
 * (u1, u2), reflect-vs-refract from u_rt.  Lobe codes: 0 coat, 1 metal,
 * 2 interface reflection, 3 interface refraction, 4 diffuse, 5 fuzz.
 */
int obsdf_sample(const obsdf* b, v3 wo, double u_lobe, double u1, double u2, double u_rt, v3* wi,
                 double weight[3], double* pdf, int* delta, int* refract, int* lobe_code) {
  weight[0] = weight[1] = weight[2] = 0.0;
  *pdf = 0.0;
  *delta = 0;
  *refract = 0;
  *lobe_code = -1;
  double mu_o = wo.z;
  if (b->absorbed || mu_o <= 0.0) return 0;
  const omat* m = &b->m;
  int lobe = -1, last = -1;
  double acc = 0.0;
  for (int k = 0; k < 5; ++k) {
    if (b->P[k] > 0.0) {
      last = k;
      if (lobe < 0 && u_lobe < acc + b->P[k]) lobe = k;
    }
    acc += b->P[k];
  }
  if (lobe < 0) lobe = last;
  if (lobe < 0) return 0;
  double mt = m->metalness, tw = m->trans_weight, sw = m->spec_weight, cw = m->coat_weight;
  v3 d;
  if (lobe == LOBE_C) {
    *lobe_code = 0;
    if (b->coat_delta) {
      *wi = V(-wo.x, -wo.y, wo.z);
      double w = fuzz_att(m, mu_o, mu_o) * cw * ofresnel_diel(mu_o, m->coat_ior) / b->P[LOBE_C];
      weight[0] = weight[1] = weight[2] = w;
      *delta = 1;
      return 1;
    }
    v3 h = oggx_vndf_sample(b->ac, b->ac, wo, u1, u2);
    d = reflect_about(wo, h);
    if (d.z <= 0.0) return 0;
  } else if (lobe == LOBE_M) {
    *lobe_code = 1;
    if (b->spec_delta) {
      *wi = V(-wo.x, -wo.y, wo.z);
      double L[3], F[3];
      coat_layer(b, mu_o, mu_o, L);
      of82(m, mu_o, F);
      double A = fuzz_att(m, mu_o, mu_o);
      for (int c = 0; c < 3; ++c) weight[c] = A * L[c] * mt * sw * F[c] / b->P[LOBE_M];
      *delta = 1;
      return 1;
    }
    v3 h = oggx_vndf_sample(b->at, b->ab, wo, u1, u2);
    d = reflect_about(wo, h);
    if (d.z <= 0.0) return 0;
  } else if (lobe == LOBE_I) {
    double eta = b->eta;
    if (b->spec_delta) {
      double Fv[3], F;
      oiface_fresnel(b, mu_o, Fv, &F);
      double dn = F + tw * (1.0 - F);
      double pr = dn > 0.0 ? F / dn : 0.0;
      double L[3];
      *delta = 1;
      if (u_rt < pr) {
        *lobe_code = 2;
        *wi = V(-wo.x, -wo.y, wo.z);
        coat_layer(b, mu_o, mu_o, L);
        double A = fuzz_att(m, mu_o, mu_o);
        for (int c = 0; c < 3; ++c) weight[c] = A * L[c] * (1.0 - mt) * Fv[c] / (b->P[LOBE_I] * pr);
        return 1;
      }
      *lobe_code = 3;
      v3 t;
      if (!refract_about(wo, V(0, 0, 1), eta, &t)) return 0;
      *wi = t;
      *refract = 1;
      coat_layer(b, t.z, mu_o, L);
      for (int c = 0; c < 3; ++c) {
        double tint = b->entering ? m->trans_color[c] : 1.0;
        weight[c] = L[c] * (1.0 - mt) * tw * tint * (1.0 - Fv[c]) / (eta * eta) / (b->P[LOBE_I] * (1.0 - pr));
      }
      return 1;
    }
    v3 h = oggx_vndf_sample(b->at, b->ab, wo, u1, u2);
    double Fv[3], F;
    oiface_fresnel(b, vdot(wo, h), Fv, &F);
    double dn = F + tw * (1.0 - F);
    double pr = dn > 0.0 ? F / dn : 0.0;
    if (u_rt < pr) {
      *lobe_code = 2;
      d = reflect_about(wo, h);
      if (d.z <= 0.0) return 0;
    } else {
      *lobe_code = 3;
      if (!refract_about(wo, h, eta, &d)) return 0;
      if (d.z >= 0.0) return 0;
      *refract = 1;
    }
  } else {
    *lobe_code = lobe == LOBE_Z ? 5 : 4;  /* fuzz and diffuse: cosine-weighted directions */
    double r = sqrt(u1), phi = 2.0 * O_PI * u2;
    double z = 1.0 - u1;
    d = V(r * cos(phi), r * sin(phi), sqrt(z > 0.0 ? z : 0.0));
    if (d.z <= 0.0) return 0;
  }
  double f[3], p;
  obsdf_eval(b, wo, d, f, &p);
  if (!(p > 0.0)) return 0;
  *wi = d;
  *pdf = p;
  for (int c = 0; c < 3; ++c) weight[c] = f[c] * fabs(d.z) / p;
  return 1;
}

/* ------------------------------------------------------- C-ABI probes -- */

static v3 v3from(const double* a) { return V(a[0], a[1], a[2]); }

int oracle_bsdf_eval(const float* mat, int32_t entering, const double wo[3], const double wi[3],
                     double f[3], double* pdf) {
  omat m;
  omat_from_floats(mat, &m);
  obsdf b;
  obsdf_setup(&m, entering, wo[2], &b);
  obsdf_eval(&b, v3from(wo), v3from(wi), f, pdf);
  return 0;
}

int oracle_bsdf_sample(const float* mat, int32_t entering, const double wo[3], const double u[4],
                       double wi[3], double weight[3], double* pdf, int32_t* flags, int32_t* lobe) {
  omat m;
  omat_from_floats(mat, &m);
  obsdf b;
  obsdf_setup(&m, entering, wo[2], &b);
  v3 w = V(0, 0, 0);
  int dl, rf, lc;
  int ok = obsdf_sample(&b, v3from(wo), u[0], u[1], u[2], u[3], &w, weight, pdf, &dl, &rf, &lc);
  wi[0] = w.x; wi[1] = w.y; wi[2] = w.z;
  *flags = (dl ? 1 : 0) | (rf ? 2 : 0);
  *lobe = lc;
  return ok;
}

void oracle_lobe_pmf(const float* mat, int32_t entering, double mu_o, double pmf[5]) {
  omat m;
  omat_from_floats(mat, &m);
  obsdf b;
  obsdf_setup(&m, entering, mu_o, &b);
  memcpy(pmf, b.P, sizeof(double) * 5);
}

double oracle_fresnel_dielectric(double cos_i, double eta) { return ofresnel_diel(cos_i, eta); }

double oracle_fuzz_albedo(double rough, double mu) {
  omat m;
  memset(&m, 0, sizeof m);
  m.fuzz_weight = 1.0;
  m.fuzz_rough = rough;
  ofuzz_table(rough, m.fuzz_E);
  return ofuzz_albedo(&m, mu);
}

double oracle_film_reflectance(double cos_i, double n2, double n3, double film_ior, double d_nm,
                               double lambda_nm) {
  return ofilm_airy(cos_i, n2, n3, film_ior, d_nm, lambda_nm);
}

void oracle_fresnel_f82(const float* mat, double mu, double F[3]) {
  omat m;
  omat_from_floats(mat, &m);
  of82(&m, mu, F);
}

double oracle_ggx_D(double at, double ab, const double m[3]) { return oggx_D(at, ab, v3from(m)); }
double oracle_ggx_G1(double at, double ab, const double w[3]) {
  return 1.0 / (1.0 + oggx_lambda(at, ab, v3from(w)));
}
void oracle_ggx_vndf_sample(double at, double ab, const double wo[3], double u1, double u2, double m[3]) {
  v3 r = oggx_vndf_sample(at, ab, v3from(wo), u1, u2);
  m[0] = r.x; m[1] = r.y; m[2] = r.z;
}
double oracle_ggx_vndf_pdf(double at, double ab, const double wo[3], const double m[3]) {
  return oggx_vndf_pdf(at, ab, v3from(wo), v3from(m));
}
