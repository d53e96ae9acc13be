/*
 * Oracle integrator: one Monte Carlo path per (pixel, sample), FP64.
 *
 * Estimates the pixel measurement of the rendering equation (Sec. 1.1)
 * truncated at max_depth scattering events:
 *   camera ray (Sec. 5.1.2; pinhole, vertical FOV, row 0 at the top, box
 *   filter jitter from dimensions 0-1 of bounce 0);
 *   closest hit through the BVH (Sec. 5.1.1);
 *   emission with MIS weight; next-event estimation with the power
 *   heuristic (Veach 1997); BSDF sampling (Sec. 5.1.3: importance sampling);
 *   Russian roulette from the second scattering event on, continuing with
 *   probability q = max_c(beta_c) * eta_scale when q < 0.995 (Sec. 5.1.3);
 *   the pixel value is the mean of its samples (Sec. 5.1.3).
 *
 * Per bounce b the uniforms are dimensions of (pixel, sample, b):
 *   0-1 pixel jitter (b = 0), 2 lobe choice, 3 Russian roulette,
 *   4-5 BSDF direction, 6 reflect/refract, 7 light choice, 8-9 light point.
 *
 * Path signature: FNV-1a 64 over little-endian 32-bit words of the event
 * stream, so that two implementations can tell whether they followed the
 * same path:
 *   hit      1, inst, prim
 *   miss     2, environment texel (0xFFFFFFFF without environment)
 *   nee      5, light id (texel | 0x80000000 for the environment), outcome
 *            (0 unoccluded, 1 occluded, 2 not traced because the
 *             contribution is zero, 3 no light sample)
 *   lobe     3, lobe code
 *   rr       4, 0 survived / 1 terminated   (only when q < 0.995)
 *   end      6, reason (0 miss, 1 max depth, 2 absorbed, 3 roulette)
 */
#include <pthread.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

#define FNV_OFFSET 0xcbf29ce484222325ULL
#define FNV_PRIME 0x100000001b3ULL

static void sig_word(uint64_t* h, uint32_t w) {
  for (int i = 0; i < 4; ++i) {
    *h ^= (uint64_t)((w >> (8 * i)) & 0xFFu);
    *h *= FNV_PRIME;
  }
}

int oracle_camera_ray(const oracle_camera* cam, double fx, double fy, double o[3], double d[3]) {
  if (!cam || cam->width <= 0 || cam->height <= 0) return -1;
  v3 eye = V(cam->eye[0], cam->eye[1], cam->eye[2]);
  v3 look = V(cam->look_at[0], cam->look_at[1], cam->look_at[2]);
  v3 up = V(cam->up[0], cam->up[1], cam->up[2]);
  v3 F = vnorm(vsub(look, eye));
  v3 R = vnorm(vcross(F, up));
  v3 U = vcross(R, F);
  double h = tan(0.5 * cam->vfov_deg * O_PI / 180.0);
  double a = (double)cam->width / (double)cam->height;
  double x = (2.0 * fx / cam->width - 1.0) * h * a;
  double y = (1.0 - 2.0 * fy / cam->height) * h;
  v3 dir = vnorm(vadd(vadd(vmul(R, x), vmul(U, y)), F));
  o[0] = eye.x; o[1] = eye.y; o[2] = eye.z;
  d[0] = dir.x; d[1] = dir.y; d[2] = dir.z;
  return 0;
}

static double pow_heur(double a, double b) {
  double a2 = a * a, b2 = b * b;
  return a2 + b2 > 0.0 ? a2 / (a2 + b2) : 0.0;
}

/* shading frame: tangent from the instance's object +z axis, Duff et al. 2017 fallback */
static void make_frame(const oinst* I, v3 n, v3* t, v3* b) {
  v3 a = I->identity ? V(0, 0, 1) : V(I->R[0][2], I->R[1][2], I->R[2][2]);
  v3 p = vsub(a, vmul(n, vdot(n, a)));
  double l = vlen(p);
  if (l >= 1e-3) {
    *t = vmul(p, 1.0 / l);
  } else {
    double sg = n.z >= 0.0 ? 1.0 : -1.0;
    double aa = -1.0 / (sg + n.z);
    double bb = n.x * n.y * aa;
    *t = V(1.0 + sg * n.x * n.x * aa, sg * bb, -sg * n.x);
  }
  *b = vcross(n, *t);
}

/* Test hook: the shading frame of make_frame for an instance whose
 * object-to-world transform is o2w (row-major 3x4; NULL = identity) at the
 * unit normal n. */
void oracle_shading_frame(const float* o2w, const double n[3], double t[3], double b[3]) {
  oinst I;
  memset(&I, 0, sizeof I);
  I.identity = o2w == NULL;
  if (o2w)
    for (int r = 0; r < 3; ++r)
      for (int c = 0; c < 3; ++c) I.R[r][c] = o2w[4 * r + c];
  v3 tt, bb;
  make_frame(&I, V(n[0], n[1], n[2]), &tt, &bb);
  t[0] = tt.x; t[1] = tt.y; t[2] = tt.z;
  b[0] = bb.x; b[1] = bb.y; b[2] = bb.z;
}

static int add_finite(double L[3], const double c[3], oracle_stats* st) {
  if (!isfinite(c[0]) || !isfinite(c[1]) || !isfinite(c[2])) {
    if (st) st->dropped_nonfinite++;
    return 0;
  }
  L[0] += c[0]; L[1] += c[1]; L[2] += c[2];
  return 1;
}

/* One path.  With rec_x != NULL, every vertex that reaches the scattering
 * stage records its cache inputs, throughput and the radiance gathered so far
 * (emission included, next-event estimation of that vertex not yet). */
static int trace_impl(const oracle_scene* s, const oracle_camera* cam, int32_t px, int32_t py, int32_t sample,
                      int32_t max_depth, uint64_t seed, const oracle_options* opt, double rgb[3], uint64_t* sig_out,
                      oracle_stats* st, double* rec_x, double* rec_L, double* rec_beta, int32_t* rec_n) {
  int est = opt ? opt->estimator : ORACLE_MIS;
  int rr_on = opt ? opt->russian_roulette : 1;
  int verbose = opt ? opt->verbose : 0;
  uint32_t pix = (uint32_t)(py * cam->width + px);
  uint32_t smp = (uint32_t)sample;
  uint64_t sig = FNV_OFFSET;
  double L[3] = {0, 0, 0}, beta[3] = {1, 1, 1};
  double o_[3], d_[3];
  double jx = ouniform(seed, pix, smp, 0, 0), jy = ouniform(seed, pix, smp, 0, 1);
  oracle_camera_ray(cam, px + jx, py + jy, o_, d_);
  v3 o = V(o_[0], o_[1], o_[2]), d = V(d_[0], d_[1], d_[2]);
  int prev_delta = 1;
  double pdf_prev = 0.0, eta_scale = 1.0;
  /* path spread of the cited cache method: primary footprint a0 and the running sum of the
   * per-bounce spread terms */
  double spread_a0 = 0.0, spread_sum = 0.0;
  int32_t skip_inst = -1, skip_prim = -1;
  const double tmin = s->tmin;
  for (int b = 0;; ++b) {
    ohit h;
    if (st) st->extension_rays++;
    int hit = oclosest(s, o, d, tmin, INFINITY, skip_inst, skip_prim, &h);
    if (hit < 0) return hit;
    if (!hit) {
      uint32_t texel = s->env ? (uint32_t)oenv_texel(s, d) : 0xFFFFFFFFu;
      sig_word(&sig, 2);
      sig_word(&sig, texel);
      if (s->env) {
        double Le[3];
        oenv_radiance(s, d, Le);
        double w = 1.0;
        if (!prev_delta) {
          if (est == ORACLE_MIS) w = pow_heur(pdf_prev, s->p_env * oenv_pdf(s, d));
          else if (est == ORACLE_NEE_ONLY) w = 0.0;
        }
        double c[3] = {beta[0] * w * Le[0], beta[1] * w * Le[1], beta[2] * w * Le[2]};
        if (w > 0.0) add_finite(L, c, st);
      }
      sig_word(&sig, 6);
      sig_word(&sig, 0);
      break;
    }
    sig_word(&sig, 1);
    sig_word(&sig, (uint32_t)h.inst);
    sig_word(&sig, (uint32_t)h.prim);
    const oinst* I = &s->insts[h.inst];
    const omesh* M = &s->meshes[I->mesh];
    const double* tv = &M->v[9 * (int64_t)h.prim];
    /* hit point and geometric normal, object space then world */
    double b0 = 1.0 - h.b1 - h.b2;
    v3 p0 = V(tv[0], tv[1], tv[2]), p1 = V(tv[3], tv[4], tv[5]), p2 = V(tv[6], tv[7], tv[8]);
    v3 po = vadd(vadd(vmul(p0, b0), vmul(p1, h.b1)), vmul(p2, h.b2));
    v3 nc = vcross(vsub(p1, p0), vsub(p2, p0));
    v3 p, ng;
    if (I->identity) {
      p = po;
      ng = vnorm(nc);
    } else {
      double x[3] = {po.x, po.y, po.z}, y[3], nx[3] = {nc.x, nc.y, nc.z}, ny[3];
      for (int r = 0; r < 3; ++r) {
        y[r] = I->R[r][0] * x[0] + I->R[r][1] * x[1] + I->R[r][2] * x[2] + I->T[r];
        ny[r] = I->R[r][0] * nx[0] + I->R[r][1] * nx[1] + I->R[r][2] * nx[2];
      }
      p = V(y[0], y[1], y[2]);
      ng = vnorm(V(ny[0], ny[1], ny[2]));
    }
    v3 wo_w = vmul(d, -1.0);
    double cos_ng = vdot(ng, wo_w);
    if (verbose)
      fprintf(stderr, "b=%d hit inst=%d prim=%d t=%.9g p=(%.9g %.9g %.9g) ng=(%.6g %.6g %.6g) cos=%.6g beta=(%.6g %.6g %.6g)\n",
              b, h.inst, h.prim, h.t, p.x, p.y, p.z, ng.x, ng.y, ng.z, cos_ng, beta[0], beta[1], beta[2]);
    int32_t mid = I->mat_override >= 0 ? I->mat_override : M->mat[h.prim];
    const omat* mat = &s->mats[mid];
    /* emission, front face only */
    if (mat->emis_lum > 0.0 && cos_ng > 0.0) {
      double Le[3] = {mat->emis_lum * mat->emis_color[0], mat->emis_lum * mat->emis_color[1],
                      mat->emis_lum * mat->emis_color[2]};
      double w = 1.0;
      if (!prev_delta) {
        int32_t k = I->light_of_tri ? I->light_of_tri[h.prim] : -1;
        double pl = olight_tri_pdf(s, k, h.t, cos_ng);
        if (est == ORACLE_MIS) w = pow_heur(pdf_prev, pl);
        else if (est == ORACLE_NEE_ONLY) w = (k >= 0 && s->n_lights > 0) ? 0.0 : 1.0;
      }
      double c[3] = {beta[0] * w * Le[0], beta[1] * w * Le[1], beta[2] * w * Le[2]};
      if (w > 0.0) add_finite(L, c, st);
    }
    if (b == max_depth) {
      sig_word(&sig, 6);
      sig_word(&sig, 1);
      break;
    }
    /* shading frame on the side of wo */
    int entering = cos_ng > 0.0;
    v3 n = entering ? ng : vmul(ng, -1.0);
    v3 t, bt;
    make_frame(I, n, &t, &bt);
    v3 wo = V(vdot(wo_w, t), vdot(wo_w, bt), vdot(wo_w, n));
    int spread_end = 0;
    if (opt && opt->nrc_weights && !rec_x && opt->spread_c > 0.0 && b <= opt->nrc_bounce) {
      double ac = fabs(cos_ng);
      if (b == 0) {
        spread_a0 = h.t * h.t / (4.0 * O_PI * ac);
      } else {
        if (!prev_delta) spread_sum += sqrt(h.t * h.t / (pdf_prev * ac));
        spread_end = spread_sum * spread_sum > opt->spread_c * spread_a0;
      }
    }
    int to_cache = opt && opt->nrc_weights &&
                   (rec_x ? (opt->train_end >= 0 && b == opt->train_end) : (b == opt->nrc_bounce || spread_end));
    if (to_cache) {
      /* the path ends in the radiance cache: outgoing radiance without emission (a training
       * path ending so is self-training: its earlier vertices' targets include this answer) */
      double x[12], y[3];
      onrc_inputs(s, p, wo_w, n, mat, x);
      oracle_nrc_forward(opt->nrc_weights, x, opt->nrc_bf16, y);
      double c[3];
      for (int k = 0; k < 3; ++k) {
        double f = opt->nrc_factor ? x[8 + k] + x[11] : 1.0;
        c[k] = beta[k] * f * (y[k] > 0.0 ? y[k] : 0.0);
      }
      add_finite(L, c, st);
      sig_word(&sig, 6);
      sig_word(&sig, 4);
      break;
    }
    if (rec_x) {
      onrc_inputs(s, p, wo_w, n, mat, rec_x + 12 * (*rec_n));
      for (int c = 0; c < 3; ++c) {
        rec_L[3 * (*rec_n) + c] = L[c];
        rec_beta[3 * (*rec_n) + c] = beta[c];
      }
      (*rec_n)++;
    }
    obsdf B;
    obsdf_setup(mat, entering, wo.z, &B);
    if (wo.z <= 0.0) B.absorbed = 1;
    /* next-event estimation */
    if (est != ORACLE_BSDF_ONLY && !B.absorbed && obsdf_has_nondelta(&B)) {
      double usel = ouniform(seed, pix, smp, (uint32_t)b, 7);
      double u1 = ouniform(seed, pix, smp, (uint32_t)b, 8), u2 = ouniform(seed, pix, smp, (uint32_t)b, 9);
      v3 wl;
      double dist, pl, Le[3];
      int64_t lid;
      int ok = olight_sample(s, p, usel, u1, u2, &wl, &dist, &pl, Le, &lid);
      uint32_t outcome = 3;
      if (ok) {
        v3 wil = V(vdot(wl, t), vdot(wl, bt), vdot(wl, n));
        double f[3], pb;
        obsdf_eval(&B, wo, wil, f, &pb);
        double w = est == ORACLE_MIS ? pow_heur(pl, pb) : 1.0;
        double k = fabs(wil.z) * w / pl;
        if (verbose)
          fprintf(stderr, "  nee light=%lld dist=%.9g pdfL=%.9g pdfB=%.9g w=%.6g cos_i=%.6g f=(%.6g %.6g %.6g)\n",
                  (long long)lid, dist, pl, pb, w, wil.z, f[0], f[1], f[2]);
        double c[3] = {beta[0] * f[0] * Le[0] * k, beta[1] * f[1] * Le[1] * k, beta[2] * f[2] * Le[2] * k};
        if (c[0] != 0.0 || c[1] != 0.0 || c[2] != 0.0) {
          double tmax = isinf(dist) ? INFINITY : (1.0 - 1e-4) * dist;
          if (st) st->shadow_rays++;
          int occ = ooccluded(s, p, wl, tmin, tmax, h.inst, h.prim);
          outcome = occ ? 1u : 0u;
          if (!occ) add_finite(L, c, st);
        } else {
          outcome = 2;
        }
      }
      sig_word(&sig, 5);
      sig_word(&sig, (uint32_t)lid);
      sig_word(&sig, outcome);
    }
    /* BSDF sampling */
    double ul = ouniform(seed, pix, smp, (uint32_t)b, 2);
    double u4 = ouniform(seed, pix, smp, (uint32_t)b, 4), u5 = ouniform(seed, pix, smp, (uint32_t)b, 5);
    double u6 = ouniform(seed, pix, smp, (uint32_t)b, 6);
    v3 wi;
    double wgt[3], pdf;
    int dl, rf, lc;
    int ok = obsdf_sample(&B, wo, ul, u4, u5, u6, &wi, wgt, &pdf, &dl, &rf, &lc);
    if (lc >= 0) {
      sig_word(&sig, 3);
      sig_word(&sig, (uint32_t)lc);
    }
    if (!ok || (wgt[0] == 0.0 && wgt[1] == 0.0 && wgt[2] == 0.0)) {
      sig_word(&sig, 6);
      sig_word(&sig, 2);
      break;
    }
    for (int c = 0; c < 3; ++c) beta[c] *= wgt[c];
    prev_delta = dl;
    pdf_prev = pdf;
    if (rf) eta_scale *= B.eta * B.eta;
    if (b >= 1 && rr_on) {
      double q = beta[0];
      if (beta[1] > q) q = beta[1];
      if (beta[2] > q) q = beta[2];
      q *= eta_scale;
      if (q < 0.995) { /* roulette only below 0.995: q within rounding of 1 never decides an event */
        double ur = ouniform(seed, pix, smp, (uint32_t)b, 3);
        int killed = ur >= q;
        sig_word(&sig, 4);
        sig_word(&sig, killed ? 1u : 0u);
        if (killed) {
          sig_word(&sig, 6);
          sig_word(&sig, 3);
          break;
        }
        for (int c = 0; c < 3; ++c) beta[c] /= q;
      }
    }
    v3 dw = vadd(vadd(vmul(t, wi.x), vmul(bt, wi.y)), vmul(n, wi.z));
    o = p;
    d = vnorm(dw);
    skip_inst = h.inst;
    skip_prim = h.prim;
  }
  rgb[0] = L[0]; rgb[1] = L[1]; rgb[2] = L[2];
  if (sig_out) *sig_out = sig;
  return 0;
}

int oracle_trace_path(const oracle_scene* s, const oracle_camera* cam, int32_t px, int32_t py,
                      int32_t sample, int32_t max_depth, uint64_t seed, const oracle_options* opt,
                      double rgb[3], uint64_t* sig_out, oracle_stats* st) {
  return trace_impl(s, cam, px, py, sample, max_depth, seed, opt, rgb, sig_out, st, NULL, NULL, NULL, NULL);
}

int oracle_training_records(const oracle_scene* s, const oracle_camera* cam, int32_t px, int32_t py,
                            int32_t sample, int32_t max_depth, uint64_t seed, const oracle_options* opt,
                            double* inputs, double* targets, int32_t* n) {
  if (!s || !cam || !inputs || !targets || !n || max_depth < 0 || max_depth > 1024) return -1;
  double rgb[3];
  double* L = (double*)malloc(sizeof(double) * 3 * (size_t)(max_depth + 1));
  double* B = (double*)malloc(sizeof(double) * 3 * (size_t)(max_depth + 1));
  int32_t k = 0;
  /* a training path never ends at the sampling paths' query vertex */
  oracle_options o;
  memset(&o, 0, sizeof o);
  if (opt) {
    o = *opt;
  } else {
    o.estimator = ORACLE_MIS;
    o.russian_roulette = 1;
    o.n_threads = 1;
    o.train_end = -1;
  }
  o.nrc_bounce = -1;
  int factor = opt && opt->nrc_factor;
  int rc = trace_impl(s, cam, px, py, sample, max_depth, seed, &o, rgb, NULL, NULL, inputs, L, B, &k);
  int32_t m = 0;
  for (int32_t i = 0; rc == 0 && i < k; ++i) {
    if (!(B[3 * i] != 0.0 && B[3 * i + 1] != 0.0 && B[3 * i + 2] != 0.0)) continue;
    double tg[3];
    int ok = 1;
    const double* xi = inputs + 12 * i;
    for (int c = 0; c < 3; ++c) {
      double f = factor ? xi[8 + c] + xi[11] : 1.0;
      if (f == 0.0) ok = 0;
      tg[c] = (rgb[c] - L[3 * i + c]) / B[3 * i + c] / f;
      if (!isfinite(tg[c])) ok = 0;
    }
    if (!ok) continue;
    if (m != i) memmove(inputs + 12 * m, inputs + 12 * i, sizeof(double) * 12);
    for (int c = 0; c < 3; ++c) targets[3 * m + c] = tg[c];
    m++;
  }
  free(L);
  free(B);
  *n = m;
  return rc;
}

/* ------------------------------------------------------------ render -- */

typedef struct {
  const oracle_scene* s;
  const oracle_camera* cam;
  int32_t x0, y0, w, h, first, n, depth;
  uint64_t seed;
  const oracle_options* opt;
  double* sum;
  double* per_sample;
  uint64_t* sigs;
  int tid, nt;
  oracle_stats st;
  int rc;
} rjob;

static void* render_worker(void* arg) {
  rjob* J = (rjob*)arg;
  memset(&J->st, 0, sizeof(J->st));
  J->rc = 0;
  for (int32_t y = J->tid; y < J->h; y += J->nt) {
    for (int32_t x = 0; x < J->w; ++x) {
      double acc[3] = {0, 0, 0};
      for (int32_t k = 0; k < J->n; ++k) {
        double rgb[3];
        uint64_t sg;
        int rc = oracle_trace_path(J->s, J->cam, J->x0 + x, J->y0 + y, J->first + k, J->depth, J->seed,
                                   J->opt, rgb, &sg, &J->st);
        if (rc) {
          J->rc = rc;
          return NULL;
        }
        int64_t idx = ((int64_t)y * J->w + x) * J->n + k;
        if (J->per_sample) {
          J->per_sample[3 * idx] = rgb[0];
          J->per_sample[3 * idx + 1] = rgb[1];
          J->per_sample[3 * idx + 2] = rgb[2];
        }
        if (J->sigs) J->sigs[idx] = sg;
        acc[0] += rgb[0]; acc[1] += rgb[1]; acc[2] += rgb[2];
      }
      double* o = &J->sum[3 * ((int64_t)y * J->w + x)];
      o[0] += acc[0]; o[1] += acc[1]; o[2] += acc[2];
    }
  }
  return NULL;
}

int oracle_render(const oracle_scene* s, const oracle_camera* cam, int32_t x0, int32_t y0, int32_t w,
                  int32_t h, int32_t first_sample, int32_t n_samples, int32_t max_depth, uint64_t seed,
                  const oracle_options* opt, double* sum_rgb, double* per_sample, uint64_t* sigs,
                  oracle_stats* st) {
  if (!s || !cam || !sum_rgb || w <= 0 || h <= 0 || n_samples < 0 || first_sample < 0) return -1;
  if (x0 < 0 || y0 < 0 || x0 + w > cam->width || y0 + h > cam->height) return -1;
  if (max_depth < 0 || max_depth > 1024) return -1;
  int nt = opt && opt->n_threads > 0 ? opt->n_threads : 1;
  if (nt > 256) nt = 256;
  pthread_t th[256];
  rjob* jobs = (rjob*)calloc((size_t)nt, sizeof(rjob));
  for (int i = 0; i < nt; ++i) {
    rjob* J = &jobs[i];
    J->s = s; J->cam = cam; J->x0 = x0; J->y0 = y0; J->w = w; J->h = h;
    J->first = first_sample; J->n = n_samples; J->depth = max_depth; J->seed = seed; J->opt = opt;
    J->sum = sum_rgb; J->per_sample = per_sample; J->sigs = sigs; J->tid = i; J->nt = nt;
    pthread_create(&th[i], NULL, render_worker, J);
  }
  int rc = 0;
  for (int i = 0; i < nt; ++i) {
    pthread_join(th[i], NULL);
    if (jobs[i].rc) rc = jobs[i].rc;
    if (st) {
      st->extension_rays += jobs[i].st.extension_rays;
      st->shadow_rays += jobs[i].st.shadow_rays;
      st->dropped_nonfinite += jobs[i].st.dropped_nonfinite;
    }
  }
  free(jobs);
  return rc;
}
