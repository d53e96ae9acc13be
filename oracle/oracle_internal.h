/* Private declarations of the FP64 oracle (test infrastructure only). */
#ifndef PT_ORACLE_INTERNAL_H
#define PT_ORACLE_INTERNAL_H

#include <math.h>
#include <stddef.h>
#include <stdint.h>

#include "oracle.h"

#define O_PI 3.14159265358979323846

typedef struct { double x, y, z; } v3;

static inline v3 V(double x, double y, double z) { v3 r = {x, y, z}; return r; }
static inline v3 vadd(v3 a, v3 b) { return V(a.x + b.x, a.y + b.y, a.z + b.z); }
static inline v3 vsub(v3 a, v3 b) { return V(a.x - b.x, a.y - b.y, a.z - b.z); }
static inline v3 vmul(v3 a, double s) { return V(a.x * s, a.y * s, a.z * s); }
static inline double vdot(v3 a, v3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
static inline v3 vcross(v3 a, v3 b) {
  return V(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
static inline double vlen(v3 a) { return sqrt(vdot(a, a)); }
static inline v3 vnorm(v3 a) { return vmul(a, 1.0 / vlen(a)); }
static inline double vget(v3 a, int k) { return k == 0 ? a.x : (k == 1 ? a.y : a.z); }
static inline double lum3(const double c[3]) { return 0.2126 * c[0] + 0.7152 * c[1] + 0.0722 * c[2]; }

/* OpenPBR parameter record, widened to double. */
typedef struct {
  double base_weight, base_color[3], metalness, diffuse_roughness;
  double spec_weight, spec_color[3], spec_rough, spec_aniso, spec_ior;
  double trans_weight, trans_color[3];
  double coat_weight, coat_color[3], coat_rough, coat_ior;
  double emis_lum, emis_color[3];
  double film_weight, film_thickness_um, film_ior;
  double fuzz_weight, fuzz_color[3], fuzz_rough;
  double ss_weight, ss_color[3];  /* subsurface (its local limit: a diffuse albedo) */
  double fuzz_E[65];   /* directional albedo of the fuzz lobe at mu = k/64 (zero without fuzz) */
} omat;

/* floats of one OpenPBR parameter record at the C ABI */
#define OMAT_FLOATS 39

void omat_from_floats(const float* f, omat* m);
/* albedo of the dielectric base's diffuse lobe, channel c: the glossy
 * diffuse (base_weight base_color) and the subsurface's local limit
 * (subsurface_color) mixed by subsurface_weight (bsdf.c) */
double odiffuse_albedo(const omat* m, int c);
/* dielectric IOR after the specular_weight modulation (bsdf.c) */
double omod_ior(const omat* m);
/* EON diffuse value (1/pi included) for albedo rho, roughness sigma, s = wi.wo - mu_i mu_o (bsdf.c) */
double oeon(double rho, double sigma, double mu_i, double mu_o, double s);

/* ---- BVH over one mesh, object space, FP64 ---- */
typedef struct {
  double lo[3], hi[3];
  int32_t left, right;     /* children (internal) */
  int32_t first, count;    /* leaf: range in the mesh's triangle order; count 0 = internal */
} obvh_node;

typedef struct {
  int64_t n_tris;
  double* v;               /* [n_tris][3][3]: triangle vertices (object space) */
  int32_t* mat;            /* [n_tris] */
  int32_t* order;          /* BVH leaf order -> triangle id */
  obvh_node* nodes;
  int32_t n_nodes;
  double lo[3], hi[3];
  float* vf;               /* [n_tris][3][3]: the same vertices in FP32 */
} omesh;

typedef struct {
  double R[3][3], T[3];     /* object -> world */
  double Ri[3][3], Ti[3];   /* world -> object (rigid inverse) */
  float Wf[12];             /* world -> object rounded to FP32 (single-precision probe) */
  int identity;
  int32_t mesh, mat_override;
  double lo[3], hi[3];      /* world bounds */
  int32_t* light_of_tri;    /* [n_tris] light index or -1, NULL if none emissive */
} oinst;

typedef struct {
  int32_t inst, prim;
  v3 p0, p1, p2, ng;        /* world space, ng unit */
  double area;
  double Le[3];
} olight;

struct oracle_scene {
  omesh* meshes;
  int32_t n_meshes;
  oinst* insts;
  int32_t n_insts;
  omat* mats;
  int32_t n_mats;
  /* environment */
  int32_t env_w, env_h;
  double* env;              /* [h][w][3] */
  double* env_row_pmf;      /* [h] */
  double* env_row_cdf;      /* [h+1] */
  double* env_col_pmf;      /* [h][w] conditional */
  double* env_col_cdf;      /* [h][w+1] */
  /* lights */
  olight* lights;
  int64_t n_lights;
  double* light_cdf;        /* [n_lights+1] over triangle weights A*lum(Le) */
  double light_wsum;
  double p_env;             /* probability of choosing the environment */
  double tmin;
  double lo[3], hi[3];
};

int oscene_build_lights(oracle_scene* s);
int oscene_build_env(oracle_scene* s, const float* env, int32_t w, int32_t h);

/* ---- BSDF ---- */
typedef struct {
  omat m;
  double eta;          /* relative IOR of the dielectric interface seen from wo */
  int entering;
  double at, ab;       /* specular GGX alphas (tangent, bitangent) */
  int spec_delta;
  double ac;           /* coat alpha */
  int coat_delta;
  double P[5];         /* lobe pmf: coat, metal, dielectric interface, diffuse, fuzz */
  int absorbed;        /* sum of lobe weights is zero */
  double film_n2;      /* thin film IOR relative to the medium wo is in */
} obsdf;

enum { LOBE_C = 0, LOBE_M = 1, LOBE_I = 2, LOBE_D = 3, LOBE_Z = 4 };

void obsdf_setup(const omat* m, int entering, double mu_o, obsdf* b);
int obsdf_has_nondelta(const obsdf* b);
void obsdf_eval(const obsdf* b, v3 wo, v3 wi, double f[3], double* pdf);
int obsdf_sample(const obsdf* b, v3 wo, double u_lobe, double u1, double u2, double u_rt,
                 v3* wi, double weight[3], double* pdf, int* delta, int* refract, int* lobe_code);
double ofresnel_diel(double c, double eta);
double ofilm_airy(double c1, double n2, double n3, double film_ior, double d_nm, double lambda_nm);
void oiface_fresnel(const obsdf* b, double c, double F[3], double* Fs);
double ofuzz_f(double alpha, v3 wo, v3 wi);
double ofuzz_alpha(double rough);
void ofuzz_table(double rough, double E[65]);
double ofuzz_albedo(const omat* m, double mu);
void of82(const omat* m, double mu, double F[3]);
double oggx_D(double at, double ab, v3 m);
double oggx_lambda(double at, double ab, v3 w);
v3 oggx_vndf_sample(double at, double ab, v3 wo, double u1, double u2);
double oggx_vndf_pdf(double at, double ab, v3 wo, v3 m);

/* ---- lights ---- */
int olight_sample(const oracle_scene* s, v3 p, double usel, double u1, double u2,
                  v3* wl, double* dist, double* pdf, double Le[3], int64_t* light_id);
double olight_tri_pdf(const oracle_scene* s, int32_t light, double t, double cos_l);
double oenv_pdf(const oracle_scene* s, v3 d);
void oenv_radiance(const oracle_scene* s, v3 d, double Le[3]);
int64_t oenv_texel(const oracle_scene* s, v3 d);

/* ---- geometry ---- */
typedef struct {
  double t, b1, b2;
  int32_t inst, prim;
} ohit;
int oclosest(const oracle_scene* s, v3 o, v3 d, double tmin, double tmax, int32_t skip_inst,
             int32_t skip_prim, ohit* h);
int ooccluded(const oracle_scene* s, v3 o, v3 d, double tmin, double tmax, int32_t skip_inst,
              int32_t skip_prim);

/* ---- radiance cache ---- */
void onrc_inputs(const oracle_scene* s, v3 p, v3 wo, v3 n, const omat* m, double x[12]);

/* ---- random numbers ---- */
double ouniform(uint64_t seed, uint32_t pixel, uint32_t sample, uint32_t bounce, uint32_t dim);

#endif
