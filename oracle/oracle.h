/*
 * FP64 CPU oracle for the path tracer's hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg load this library.  The product path (the
 * HIP library under paper_2407_19977_amd/) never links, imports or calls it.
 *
 * What it computes: a Monte Carlo estimate of the pixel measurement of the
 * rendering equation (Sec. 1.1, Kajiya's equation), with camera rays from a
 * pinhole (Sec. 5.1.2), closest hits found through an AABB BVH (Sec. 5.1.1),
 * an OpenPBR-subset BSDF with importance sampling (Sec. 4, Sec. 5.1.3),
 * next-event estimation with multiple importance sampling, Russian roulette
 * (Sec. 5.1.3) and per-pixel sample averaging (Sec. 5.1.3).  Random numbers
 * come from a counter-based Philox4x32-10 keyed by (pixel, sample, bounce,
 * dimension block).  Everything is double precision except the one routine
 * that defines the single-precision closest hit (oracle_closest_f32), which
 * is the exact definition the GPU's closest-hit search must reproduce.
 *
 * All functions return 0 on success and a negative value on invalid input.
 */
#ifndef PT_ORACLE_H
#define PT_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct oracle_scene oracle_scene;

typedef struct {
  const float* vertices;      /* [n_vertices][3] */
  int64_t n_vertices;
  const int32_t* indices;     /* [n_triangles][3] */
  int64_t n_triangles;
  const int32_t* material_ids;/* [n_triangles] */
} oracle_mesh;

typedef struct {
  float object_to_world[12];  /* row-major 3x4, rigid */
  int32_t mesh;
  int32_t material_override;  /* -1: per-triangle ids */
} oracle_instance;

typedef struct {
  float eye[3], look_at[3], up[3];
  float vfov_deg;
  int32_t width, height;
} oracle_camera;

/* estimator switches (the product always uses MIS with Russian roulette) */
enum { ORACLE_MIS = 0, ORACLE_BSDF_ONLY = 1, ORACLE_NEE_ONLY = 2 };

typedef struct {
  int32_t estimator;     /* ORACLE_MIS / ORACLE_BSDF_ONLY / ORACLE_NEE_ONLY */
  int32_t russian_roulette; /* 1 = on (default), 0 = off */
  int32_t n_threads;     /* <= 0: one */
  int32_t verbose;       /* 1: print every vertex of oracle_trace_path to stderr (debugging) */
  const double* nrc_weights; /* radiance cache weights (20,672, see nrc.c) or NULL: plain paths */
  int32_t nrc_bounce;    /* vertex index at which paths end in the cache (2) */
  int32_t nrc_bf16;      /* 1: evaluate the cache with bfloat16 operands */
  int32_t train_end;     /* training records: the path ends in the cache at this vertex (self-training; needs
                            nrc_weights), -1: plain path to max_depth */
  int32_t nrc_factor;    /* 1: the cache predicts radiance / (diffuse albedo + specular albedo) */
  double spread_c;       /* > 0: adaptive termination (path spread): a rendering path ends in the cache at
                            the first vertex b >= 1 whose spread exceeds spread_c times the primary
                            footprint, at nrc_bounce at the latest; 0: always at nrc_bounce */
} oracle_options;

typedef struct {
  int64_t extension_rays;
  int64_t shadow_rays;
  int64_t dropped_nonfinite;
} oracle_stats;

/* Philox4x32-10 block: ctr[4], key[2] -> out[4]. */
void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* Uniform in [0,1) of dimension `dim` at (pixel, sample, bounce) for a 64-bit seed. */
double oracle_uniform(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t bounce, uint32_t dim);

int oracle_scene_create(const oracle_mesh* meshes, int32_t n_meshes,
                        const oracle_instance* instances, int32_t n_instances,
                        const float* materials /* [n][39] */, int32_t n_materials,
                        const float* env /* [h][w][3] or NULL */, int32_t env_w, int32_t env_h,
                        oracle_scene** out);
void oracle_scene_destroy(oracle_scene* s);
double oracle_scene_tmin(const oracle_scene* s);
int64_t oracle_scene_n_lights(const oracle_scene* s);

/* Camera ray through the image point (px + jx, py + jy); d is unit length. */
int oracle_camera_ray(const oracle_camera* cam, double fx, double fy, double o[3], double d[3]);

/* Closest hit in FP64 via the oracle's BVH.  hit[0]=t, hit[1]=b1, hit[2]=b2;
 * ids[0]=inst, ids[1]=prim; returns 1 if hit, 0 if not. */
int oracle_closest_f64(const oracle_scene* s, const double o[3], const double d[3], double tmin,
                       double tmax, int32_t skip_inst, int32_t skip_prim, double hit[3], int32_t ids[2]);
/* Same query answered by testing every triangle (no BVH). */
int oracle_closest_f64_brute(const oracle_scene* s, const double o[3], const double d[3], double tmin,
                             double tmax, int32_t skip_inst, int32_t skip_prim, double hit[3], int32_t ids[2]);

/* Single-precision closest hit by brute force over all triangles, the exact
 * reference for the GPU search.  rays: [n][8] = ox,oy,oz,tmin,dx,dy,dz,tmax.
 * hits: [n][4] uint32 = t bits, inst, prim (0xFFFFFFFF if no hit), b1 bits... see oracle.py. */
int oracle_closest_f32_brute(const oracle_scene* s, const float* rays, int64_t n, uint32_t* hits,
                             int32_t n_threads);

/* Trace one camera path; rgb[3] is the radiance estimate and *sig the path signature. */
int oracle_trace_path(const oracle_scene* s, const oracle_camera* cam, int32_t px, int32_t py,
                      int32_t sample, int32_t max_depth, uint64_t seed, const oracle_options* opt,
                      double rgb[3], uint64_t* sig, oracle_stats* st);

/* Render samples [first, first+n) of the pixels in the crop (x0,y0,w,h).
 * sum_rgb [h][w][3] receives the per-pixel sums (added to, FP64);
 * per_sample [h][w][n][3] and sigs [h][w][n] are optional (NULL). */
int oracle_render(const oracle_scene* s, const oracle_camera* cam, int32_t x0, int32_t y0,
                  int32_t w, int32_t h, int32_t first_sample, int32_t n_samples, int32_t max_depth,
                  uint64_t seed, const oracle_options* opt, double* sum_rgb, double* per_sample,
                  uint64_t* sigs, oracle_stats* st);

/* ---- radiance cache (nrc.c) ---- */
double oracle_bf16_round(double x);
void oracle_nrc_encode(const double x[12], double f[64]);
void oracle_nrc_forward(const double* W, const double x[12], int32_t bf16, double y[3]);
/* Test hook: the 12 cache inputs at point p (scene box [lo, hi]), outgoing
 * direction wo and shading normal n (world space, unit) of a material given
 * as its 35 OpenPBR floats. */
void oracle_nrc_inputs(const double lo[3], const double hi[3], const double p[3], const double wo[3],
                       const double n[3], const float* mat, double x[12]);
/* Training records of one path: for every vertex k < max_depth that scatters
 * or absorbs, the 12 cache inputs and the target (L_end - L_k) / beta_k
 * (divided by the reflectance factor with opt->nrc_factor); vertices with a
 * zero throughput or factor channel are dropped.  With opt->train_end >= 0
 * and weights, the path ends in the cache at that vertex (self-training):
 * L_end = L_T + beta_T * cache(x_T) and no record at T.  opt may be NULL
 * (plain path).  inputs [max_depth][12], targets [max_depth][3]; *n receives
 * the count. */
int oracle_training_records(const oracle_scene* s, const oracle_camera* cam, int32_t px, int32_t py,
                            int32_t sample, int32_t max_depth, uint64_t seed, const oracle_options* opt,
                            double* inputs, double* targets, int32_t* n);

/* Test hook: the shading frame (t, b, n) at unit normal n of an instance
 * with object-to-world transform o2w (row-major 3x4; NULL = world space):
 * t is the instance's object +z axis projected onto the tangent plane, or
 * the Duff et al. 2017 basis vector when that projection is shorter than
 * 1e-3; b = n x t. */
void oracle_shading_frame(const float* o2w, const double n[3], double t[3], double b[3]);

/* ---- display path (display.c): PBR Neutral tone map, sRGB, 8-bit ---- */
void oracle_pbr_neutral(const double in[3], double out[3]);
double oracle_srgb_encode(double v);
void oracle_display(const double* sum, int64_t n_pixels, double inv_samples, double exposure, double* encoded,
                    uint8_t* rgba8);

/* ---- BSDF and light-sampling probes (local shading frame, n = +z) ---- */
/* mat: 39 floats.  entering: 1 if wo is on the front side of the geometric normal. */
int oracle_bsdf_eval(const float* mat, int32_t entering, const double wo[3], const double wi[3],
                     double f[3], double* pdf);
/* u[4] = (lobe, dir1, dir2, reflect/refract).  out: wi[3], weight[3], pdf, flags
 * (bit0 delta, bit1 refraction), lobe code; returns 1 if a direction was produced. */
int oracle_bsdf_sample(const float* mat, int32_t entering, const double wo[3], const double u[4],
                       double wi[3], double weight[3], double* pdf, int32_t* flags, int32_t* lobe);
void oracle_lobe_pmf(const float* mat, int32_t entering, double mu_o, double pmf[5]);
double oracle_fresnel_dielectric(double cos_i, double eta);
/* directional albedo of the fuzz lobe (weight 1, colour 1) at cosine mu, from its table */
double oracle_fuzz_albedo(double rough, double mu);
/* thin-film reflectance (unpolarised, one wavelength): incident index 1, film n2, base n3 (relative),
 * absolute film IOR and thickness in nm for the phase */
double oracle_film_reflectance(double cos_i, double n2, double n3, double film_ior, double d_nm,
                               double lambda_nm);
void oracle_fresnel_f82(const float* mat, double mu, double F[3]);
double oracle_ggx_D(double at, double ab, const double m[3]);
double oracle_ggx_G1(double at, double ab, const double w[3]);
void oracle_ggx_vndf_sample(double at, double ab, const double wo[3], double u1, double u2, double m[3]);
double oracle_ggx_vndf_pdf(double at, double ab, const double wo[3], const double m[3]);
/* Light sampling at point p with uniforms (u_select, u1, u2).  Returns 1 if a
 * sample with nonzero pdf was produced: wl, dist (INF for env), pdf (solid
 * angle x selection), Le[3], light id. */
int oracle_sample_light(const oracle_scene* s, const double p[3], double usel, double u1, double u2,
                        double wl[3], double* dist, double* pdf, double Le[3], int64_t* light_id);
double oracle_env_pdf(const oracle_scene* s, const double d[3]);   /* solid-angle pdf, no selection */
void oracle_env_radiance(const oracle_scene* s, const double d[3], double Le[3]);

#ifdef __cplusplus
}
#endif
#endif
