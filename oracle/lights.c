/*
 * Oracle lights: one-sided emissive triangles and an equirectangular
 * environment, in FP64.  The paper lists emission among the OpenPBR
 * parameter families (Sec. 4); it does not describe light sampling, so the
 * following is this project's reading (next-event estimation is required by
 * the build, the paper only names importance sampling in Sec. 5.1.3):
 *
 *  Selection pmf: P_env = 1 with no emissive triangles, 0 with no
 *    environment, else 1/2; triangle k gets (1-P_env) A_k lum(Le_k) / sum_j.
 *    u_select < P_env picks the environment, otherwise the first triangle
 *    whose cumulative bound exceeds u_select (last nonzero one on rounding).
 *  Triangle point: s = sqrt(u1), b0 = 1-s, b1 = u2 s, p = b0 v0 + b1 v1 + (1-b0-b1) v2.
 *    Solid-angle pdf P_k dist^2 / (cos_l A_k); zero when the light faces away.
 *  Environment (y up): theta = acos(d_y), phi = atan2(d_x, -d_z),
 *    u = phi/2pi + 1/2, v = theta/pi, texel (min(floor(uW),W-1), min(floor(vH),H-1)),
 *    nearest lookup.  Sampling: texel pmf proportional to lum(texel) sin(theta_row_centre),
 *    marginal row CDF then conditional column CDF, each inverted with the
 *    remainder reused for the position inside the texel;
 *    pdf_omega = W H P_texel / (2 pi^2 sin theta).
 */
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

int oscene_build_env(oracle_scene* s, const float* env, int32_t w, int32_t h) {
  s->env_w = s->env_h = 0;
  if (!env) return 0;
  if (w <= 0 || h <= 0) return -1;
  s->env_w = w;
  s->env_h = h;
  size_t n = (size_t)w * (size_t)h;
  s->env = (double*)malloc(sizeof(double) * 3 * n);
  s->env_row_pmf = (double*)malloc(sizeof(double) * (size_t)h);
  s->env_row_cdf = (double*)malloc(sizeof(double) * (size_t)(h + 1));
  s->env_col_pmf = (double*)malloc(sizeof(double) * n);
  s->env_col_cdf = (double*)malloc(sizeof(double) * (size_t)h * (size_t)(w + 1));
  if (!s->env || !s->env_row_pmf || !s->env_row_cdf || !s->env_col_pmf || !s->env_col_cdf) return -2;
  for (size_t i = 0; i < 3 * n; ++i) {
    double x = env[i];
    if (!(x >= 0.0) || !isfinite(x)) return -1;
    s->env[i] = x;
  }
  double total = 0.0;
  double* row_w = (double*)malloc(sizeof(double) * (size_t)h);
  for (int32_t r = 0; r < h; ++r) {
    double st = sin(O_PI * (r + 0.5) / h);
    double rs = 0.0;
    double* cdf = &s->env_col_cdf[(size_t)r * (w + 1)];
    cdf[0] = 0.0;
    for (int32_t c = 0; c < w; ++c) {
      double wt = lum3(&s->env[3 * ((size_t)r * w + c)]) * st;
      s->env_col_pmf[(size_t)r * w + c] = wt;
      rs += wt;
      cdf[c + 1] = rs;
    }
    for (int32_t c = 0; c < w; ++c) {
      s->env_col_pmf[(size_t)r * w + c] = rs > 0.0 ? s->env_col_pmf[(size_t)r * w + c] / rs : 0.0;
      cdf[c + 1] = rs > 0.0 ? cdf[c + 1] / rs : 0.0;
    }
    if (rs > 0.0) cdf[w] = 1.0;
    row_w[r] = rs;
    total += rs;
  }
  s->env_row_cdf[0] = 0.0;
  double acc = 0.0;
  for (int32_t r = 0; r < h; ++r) {
    s->env_row_pmf[r] = total > 0.0 ? row_w[r] / total : 0.0;
    acc += row_w[r];
    s->env_row_cdf[r + 1] = total > 0.0 ? acc / total : 0.0;
  }
  if (total > 0.0) s->env_row_cdf[h] = 1.0;
  free(row_w);
  if (!(total > 0.0)) {
    /* a black environment contributes nothing and is never sampled */
    free(s->env);
    s->env = NULL;
    s->env_w = s->env_h = 0;
  }
  return 0;
}

static int mat_emissive(const omat* m) {
  double c[3] = {m->emis_color[0], m->emis_color[1], m->emis_color[2]};
  return m->emis_lum > 0.0 && lum3(c) > 0.0;
}

static v3 inst_point(const oinst* I, const double* x) {
  if (I->identity) return V(x[0], x[1], x[2]);
  double y[3];
  for (int r = 0; r < 3; ++r) y[r] = I->R[r][0] * x[0] + I->R[r][1] * x[1] + I->R[r][2] * x[2] + I->T[r];
  return V(y[0], y[1], y[2]);
}

int oscene_build_lights(oracle_scene* s) {
  int64_t cnt = 0;
  for (int32_t i = 0; i < s->n_insts; ++i) {
    const oinst* I = &s->insts[i];
    const omesh* m = &s->meshes[I->mesh];
    for (int64_t t = 0; t < m->n_tris; ++t) {
      int32_t mid = I->mat_override >= 0 ? I->mat_override : m->mat[t];
      if (mat_emissive(&s->mats[mid])) cnt++;
    }
  }
  s->n_lights = cnt;
  s->lights = (olight*)calloc((size_t)(cnt > 0 ? cnt : 1), sizeof(olight));
  s->light_cdf = (double*)malloc(sizeof(double) * (size_t)(cnt + 1));
  if (!s->lights || !s->light_cdf) return -2;
  int64_t k = 0;
  double acc = 0.0;
  s->light_cdf[0] = 0.0;
  for (int32_t i = 0; i < s->n_insts; ++i) {
    oinst* I = &s->insts[i];
    const omesh* m = &s->meshes[I->mesh];
    for (int64_t t = 0; t < m->n_tris; ++t) {
      int32_t mid = I->mat_override >= 0 ? I->mat_override : m->mat[t];
      const omat* mm = &s->mats[mid];
      if (!mat_emissive(mm)) continue;
      if (!I->light_of_tri) {
        I->light_of_tri = (int32_t*)malloc(sizeof(int32_t) * (size_t)m->n_tris);
        for (int64_t q = 0; q < m->n_tris; ++q) I->light_of_tri[q] = -1;
      }
      I->light_of_tri[t] = (int32_t)k;
      olight* L = &s->lights[k];
      L->inst = i;
      L->prim = (int32_t)t;
      L->p0 = inst_point(I, &m->v[9 * t]);
      L->p1 = inst_point(I, &m->v[9 * t + 3]);
      L->p2 = inst_point(I, &m->v[9 * t + 6]);
      v3 c = vcross(vsub(L->p1, L->p0), vsub(L->p2, L->p0));
      double len = vlen(c);
      L->area = 0.5 * len;
      L->ng = len > 0.0 ? vmul(c, 1.0 / len) : V(0, 0, 0);
      for (int q = 0; q < 3; ++q) L->Le[q] = mm->emis_lum * mm->emis_color[q];
      acc += L->area * lum3(L->Le);
      s->light_cdf[k + 1] = acc;
      k++;
    }
  }
  s->light_wsum = acc;
  for (int64_t q = 1; q <= cnt; ++q) s->light_cdf[q] = acc > 0.0 ? s->light_cdf[q] / acc : 0.0;
  int has_tri = cnt > 0 && acc > 0.0;
  int has_env = s->env != NULL;
  s->p_env = !has_env ? 0.0 : (has_tri ? 0.5 : 1.0);
  if (!has_tri) s->n_lights = 0;
  return 0;
}

/* probability of picking triangle light k */
static double tri_select_pmf(const oracle_scene* s, int64_t k) {
  if (s->n_lights == 0 || !(s->light_wsum > 0.0)) return 0.0;
  const olight* L = &s->lights[k];
  return (1.0 - s->p_env) * L->area * lum3(L->Le) / s->light_wsum;
}

double olight_tri_pdf(const oracle_scene* s, int32_t light, double t, double cos_l) {
  if (light < 0 || cos_l <= 0.0) return 0.0;
  const olight* L = &s->lights[light];
  return tri_select_pmf(s, light) * t * t / (cos_l * L->area);
}

int64_t oenv_texel(const oracle_scene* s, v3 d) {
  double y = d.y < -1.0 ? -1.0 : (d.y > 1.0 ? 1.0 : d.y);
  double th = acos(y), ph = atan2(d.x, -d.z);
  double u = ph / (2.0 * O_PI) + 0.5, v = th / O_PI;
  int64_t c = (int64_t)floor(u * s->env_w), r = (int64_t)floor(v * s->env_h);
  if (c > s->env_w - 1) c = s->env_w - 1;
  if (r > s->env_h - 1) r = s->env_h - 1;
  if (c < 0) c = 0;
  if (r < 0) r = 0;
  return r * s->env_w + c;
}

void oenv_radiance(const oracle_scene* s, v3 d, double Le[3]) {
  Le[0] = Le[1] = Le[2] = 0.0;
  if (!s->env) return;
  int64_t t = oenv_texel(s, d);
  for (int c = 0; c < 3; ++c) Le[c] = s->env[3 * t + c];
}

double oenv_pdf(const oracle_scene* s, v3 d) {
  if (!s->env) return 0.0;
  int64_t t = oenv_texel(s, d);
  int64_t r = t / s->env_w;
  double P = s->env_row_pmf[r] * s->env_col_pmf[t];
  double y = d.y < -1.0 ? -1.0 : (d.y > 1.0 ? 1.0 : d.y);
  double st = sqrt(1.0 - y * y);
  if (!(st > 0.0)) return 0.0;
  return (double)s->env_w * s->env_h * P / (2.0 * O_PI * O_PI * st);
}

/* invert a CDF of n buckets: the bucket i with cdf[i] <= u < cdf[i+1] and pmf > 0 */
static int64_t cdf_invert(const double* cdf, int64_t n, double u) {
  int64_t lo = 0, hi = n; /* find the last i with cdf[i] <= u */
  while (hi - lo > 1) {
    int64_t mid = (lo + hi) / 2;
    if (cdf[mid] <= u) lo = mid;
    else hi = mid;
  }
  /* skip empty buckets (cdf[i+1] == cdf[i]) forward, then backward */
  int64_t i = lo;
  while (i < n - 1 && !(cdf[i + 1] > cdf[i])) i++;
  while (i > 0 && !(cdf[i + 1] > cdf[i])) i--;
  return i;
}

int olight_sample(const oracle_scene* s, v3 p, double usel, double u1, double u2, v3* wl, double* dist,
                  double* pdf, double Le[3], int64_t* light_id) {
  *pdf = 0.0;
  Le[0] = Le[1] = Le[2] = 0.0;
  *light_id = -1;
  if (s->p_env <= 0.0 && s->n_lights == 0) return 0;
  if (usel < s->p_env) {
    /* environment */
    int32_t W = s->env_w, H = s->env_h;
    int64_t r = cdf_invert(s->env_row_cdf, H, u1);
    double pr = s->env_row_pmf[r];
    double du = pr > 0.0 ? (u1 - s->env_row_cdf[r]) / pr : 0.5;
    const double* ccdf = &s->env_col_cdf[(size_t)r * (W + 1)];
    int64_t c = cdf_invert(ccdf, W, u2);
    double pc = s->env_col_pmf[(size_t)r * W + c];
    double dv = pc > 0.0 ? (u2 - ccdf[c]) / pc : 0.5;
    double uu = (c + dv) / W, vv = (r + du) / H;
    double th = O_PI * vv, ph = 2.0 * O_PI * (uu - 0.5);
    double st = sin(th);
    *wl = V(st * sin(ph), cos(th), -st * cos(ph));
    *dist = INFINITY;
    *light_id = (int64_t)0x80000000LL | (r * W + c);
    if (!(st > 0.0)) return 0;
    double P = pr * pc;
    *pdf = s->p_env * (double)W * H * P / (2.0 * O_PI * O_PI * st);
    for (int q = 0; q < 3; ++q) Le[q] = s->env[3 * ((size_t)r * W + c) + q];
    return *pdf > 0.0;
  }
  /* triangle: map usel in [p_env, 1) to the triangle CDF */
  double ut = s->p_env > 0.0 ? (usel - s->p_env) / (1.0 - s->p_env) : usel;
  int64_t k = cdf_invert(s->light_cdf, s->n_lights, ut);
  *light_id = k;
  const olight* L = &s->lights[k];
  double sq = sqrt(u1);
  double b0 = 1.0 - sq, b1 = u2 * sq;
  v3 q = vadd(vadd(vmul(L->p0, b0), vmul(L->p1, b1)), vmul(L->p2, 1.0 - b0 - b1));
  v3 to = vsub(q, p);
  double d2 = vdot(to, to);
  double dd = sqrt(d2);
  if (!(dd > 0.0)) return 0;
  *wl = vmul(to, 1.0 / dd);
  *dist = dd;
  double cl = -vdot(L->ng, *wl);
  if (cl <= 0.0) return 0;
  *pdf = tri_select_pmf(s, k) * d2 / (cl * L->area);
  for (int c = 0; c < 3; ++c) Le[c] = L->Le[c];
  return *pdf > 0.0;
}

/* ------------------------------------------------------- C-ABI probes -- */

int oracle_sample_light(const oracle_scene* s, const double p[3], double usel, double u1, double u2,
                        double wl[3], double* dist, double* pdf, double Le[3], int64_t* light_id) {
  v3 w = V(0, 0, 0);
  int ok = olight_sample(s, V(p[0], p[1], p[2]), usel, u1, u2, &w, dist, pdf, Le, light_id);
  wl[0] = w.x; wl[1] = w.y; wl[2] = w.z;
  return ok;
}

double oracle_env_pdf(const oracle_scene* s, const double d[3]) { return oenv_pdf(s, V(d[0], d[1], d[2])); }

void oracle_env_radiance(const oracle_scene* s, const double d[3], double Le[3]) {
  oenv_radiance(s, V(d[0], d[1], d[2]), Le);
}
