/*
 * Oracle geometry: scene set-up, an FP64 AABB BVH per mesh (Sec. 5.1.1:
 * axis-aligned boxes grouped so every child lies inside its parent), a
 * linear loop over instances, and the watertight ray/triangle test of Woop,
 * Benthin and Wald (JCGT 2013).
 *
 * Closest hit: among triangles with t in (tmin, tmax), excluding the
 * triangle the ray leaves from, the lexicographic minimum of
 * (t, instance, primitive).  Triangles are two-sided for hits; a zero
 * determinant is a miss.
 *
 * oracle_closest_f32_brute is the single-precision definition of the same
 * query: every triangle is tested, in float, with the operation order spelt
 * out below and no fused multiply-add (this file is compiled with
 * -ffp-contract=off).  It is the exact reference for the GPU search.
 */
#include <float.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

#include "oracle_internal.h"

void omat_from_floats(const float* f, omat* m) {
  int i = 0;
  m->base_weight = f[i++];
  for (int c = 0; c < 3; ++c) m->base_color[c] = f[i++];
  m->metalness = f[i++];
  m->diffuse_roughness = f[i++];
  m->spec_weight = f[i++];
  for (int c = 0; c < 3; ++c) m->spec_color[c] = f[i++];
  m->spec_rough = f[i++];
  m->spec_aniso = f[i++];
  m->spec_ior = f[i++];
  m->trans_weight = f[i++];
  for (int c = 0; c < 3; ++c) m->trans_color[c] = f[i++];
  m->coat_weight = f[i++];
  for (int c = 0; c < 3; ++c) m->coat_color[c] = f[i++];
  m->coat_rough = f[i++];
  m->coat_ior = f[i++];
  m->emis_lum = f[i++];
  for (int c = 0; c < 3; ++c) m->emis_color[c] = f[i++];
  m->film_weight = f[i++];
  m->film_thickness_um = f[i++];
  m->film_ior = f[i++];
  m->fuzz_weight = f[i++];
  for (int c = 0; c < 3; ++c) m->fuzz_color[c] = f[i++];
  m->fuzz_rough = f[i++];
  m->ss_weight = f[i++];
  for (int c = 0; c < 3; ++c) m->ss_color[c] = f[i++];
  if (m->fuzz_weight > 0.0) ofuzz_table(m->fuzz_rough, m->fuzz_E);
  else
    for (int k = 0; k < 65; ++k) m->fuzz_E[k] = 0.0;
}

/* ------------------------------------------------------------------ BVH -- */

typedef struct {
  const omesh* m;
  double* cen;   /* [n][3] */
} obuild;

static const double* g_sort_cen;
static int g_sort_axis;
static int cmp_cen(const void* a, const void* b) {
  int32_t i = *(const int32_t*)a, j = *(const int32_t*)b;
  double ci = g_sort_cen[3 * i + g_sort_axis], cj = g_sort_cen[3 * j + g_sort_axis];
  if (ci < cj) return -1;
  if (ci > cj) return 1;
  return (i > j) - (i < j);
}

static void tri_bounds(const omesh* m, int32_t t, double lo[3], double hi[3]) {
  for (int k = 0; k < 3; ++k) {
    lo[k] = INFINITY;
    hi[k] = -INFINITY;
  }
  for (int v = 0; v < 3; ++v)
    for (int k = 0; k < 3; ++k) {
      double x = m->v[9 * t + 3 * v + k];
      if (x < lo[k]) lo[k] = x;
      if (x > hi[k]) hi[k] = x;
    }
}

/* Object-median split on the longest centroid axis; leaves hold <= 4 triangles. */
static int32_t build_rec(omesh* m, const double* cen, int32_t first, int32_t count) {
  int32_t id = m->n_nodes++;
  obvh_node* n = &m->nodes[id];
  for (int k = 0; k < 3; ++k) {
    n->lo[k] = INFINITY;
    n->hi[k] = -INFINITY;
  }
  double clo[3] = {INFINITY, INFINITY, INFINITY}, chi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int32_t i = first; i < first + count; ++i) {
    double lo[3], hi[3];
    int32_t t = m->order[i];
    tri_bounds(m, t, lo, hi);
    for (int k = 0; k < 3; ++k) {
      if (lo[k] < n->lo[k]) n->lo[k] = lo[k];
      if (hi[k] > n->hi[k]) n->hi[k] = hi[k];
      double c = cen[3 * t + k];
      if (c < clo[k]) clo[k] = c;
      if (c > chi[k]) chi[k] = c;
    }
  }
  if (count <= 4) {
    n->first = first;
    n->count = count;
    n->left = n->right = -1;
    return id;
  }
  int axis = 0;
  for (int k = 1; k < 3; ++k)
    if (chi[k] - clo[k] > chi[axis] - clo[axis]) axis = k;
  g_sort_cen = cen;
  g_sort_axis = axis;
  qsort(m->order + first, (size_t)count, sizeof(int32_t), cmp_cen);
  int32_t half = count / 2;
  n->count = 0;
  n->first = -1;
  int32_t l = build_rec(m, cen, first, half);
  int32_t r = build_rec(m, cen, first + half, count - half);
  m->nodes[id].left = l;
  m->nodes[id].right = r;
  return id;
}

static int mesh_build(omesh* m) {
  m->order = (int32_t*)malloc(sizeof(int32_t) * (size_t)(m->n_tris > 0 ? m->n_tris : 1));
  m->nodes = (obvh_node*)malloc(sizeof(obvh_node) * (size_t)(2 * m->n_tris + 1));
  double* cen = (double*)malloc(sizeof(double) * 3 * (size_t)(m->n_tris > 0 ? m->n_tris : 1));
  if (!m->order || !m->nodes || !cen) {
    free(cen);
    return -2;
  }
  for (int64_t t = 0; t < m->n_tris; ++t) {
    m->order[t] = (int32_t)t;
    for (int k = 0; k < 3; ++k)
      cen[3 * t + k] = (m->v[9 * t + k] + m->v[9 * t + 3 + k] + m->v[9 * t + 6 + k]) / 3.0;
  }
  m->n_nodes = 0;
  if (m->n_tris > 0) build_rec(m, cen, 0, (int32_t)m->n_tris);
  free(cen);
  if (m->n_tris > 0) {
    for (int k = 0; k < 3; ++k) {
      m->lo[k] = m->nodes[0].lo[k];
      m->hi[k] = m->nodes[0].hi[k];
    }
  }
  return 0;
}

/* ------------------------------------------------------- scene set-up -- */

static void mat_mul_vec(const double R[3][3], const double x[3], double y[3]) {
  for (int i = 0; i < 3; ++i) y[i] = R[i][0] * x[0] + R[i][1] * x[1] + R[i][2] * x[2];
}

int oracle_scene_create(const oracle_mesh* meshes, int32_t n_meshes, const oracle_instance* instances,
                        int32_t n_instances, const float* materials, int32_t n_materials,
                        const float* env, int32_t env_w, int32_t env_h, oracle_scene** out) {
  if (!out || !meshes || n_meshes <= 0 || n_instances < 0 || !materials || n_materials <= 0) return -1;
  oracle_scene* s = (oracle_scene*)calloc(1, sizeof(oracle_scene));
  if (!s) return -2;
  s->n_mats = n_materials;
  s->mats = (omat*)calloc((size_t)n_materials, sizeof(omat));
  for (int32_t i = 0; i < n_materials; ++i) omat_from_floats(materials + OMAT_FLOATS * i, &s->mats[i]);

  /* meshes: with no instances, all meshes are concatenated into one world-space mesh */
  int32_t n_out = n_instances == 0 ? 1 : n_meshes;
  s->n_meshes = n_out;
  s->meshes = (omesh*)calloc((size_t)n_out, sizeof(omesh));
  for (int32_t mi = 0; mi < n_out; ++mi) {
    int32_t a = n_instances == 0 ? 0 : mi, b = n_instances == 0 ? n_meshes : mi + 1;
    int64_t nt = 0;
    for (int32_t j = a; j < b; ++j) nt += meshes[j].n_triangles;
    omesh* m = &s->meshes[mi];
    m->n_tris = nt;
    m->v = (double*)malloc(sizeof(double) * 9 * (size_t)(nt > 0 ? nt : 1));
    m->vf = (float*)malloc(sizeof(float) * 9 * (size_t)(nt > 0 ? nt : 1));
    m->mat = (int32_t*)malloc(sizeof(int32_t) * (size_t)(nt > 0 ? nt : 1));
    int64_t t = 0;
    for (int32_t j = a; j < b; ++j) {
      const oracle_mesh* in = &meshes[j];
      for (int64_t k = 0; k < in->n_triangles; ++k, ++t) {
        for (int v = 0; v < 3; ++v) {
          int32_t vi = in->indices[3 * k + v];
          if (vi < 0 || vi >= in->n_vertices) return -1;
          for (int c = 0; c < 3; ++c) {
            float x = in->vertices[3 * (int64_t)vi + c];
            m->vf[9 * t + 3 * v + c] = x;
            m->v[9 * t + 3 * v + c] = (double)x;
          }
        }
        m->mat[t] = in->material_ids ? in->material_ids[k] : 0;
      }
    }
    int rc = mesh_build(m);
    if (rc) return rc;
  }

  /* instances */
  s->n_insts = n_instances == 0 ? 1 : n_instances;
  s->insts = (oinst*)calloc((size_t)s->n_insts, sizeof(oinst));
  for (int32_t i = 0; i < s->n_insts; ++i) {
    oinst* I = &s->insts[i];
    if (n_instances == 0) {
      I->identity = 1;
      I->mesh = 0;
      I->mat_override = -1;
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) I->R[r][c] = I->Ri[r][c] = (r == c);
        I->T[r] = I->Ti[r] = 0.0;
      }
      for (int k = 0; k < 12; ++k) I->Wf[k] = (k == 0 || k == 5 || k == 10) ? 1.0f : 0.0f;
    } else {
      const oracle_instance* in = &instances[i];
      I->identity = 0;
      I->mesh = in->mesh;
      I->mat_override = in->material_override;
      if (in->mesh < 0 || in->mesh >= n_meshes) return -1;
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) I->R[r][c] = in->object_to_world[4 * r + c];
        I->T[r] = in->object_to_world[4 * r + 3];
      }
      /* rigid inverse: Ri = R^T, Ti = -(R^T T) */
      for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) I->Ri[r][c] = I->R[c][r];
      for (int r = 0; r < 3; ++r)
        I->Ti[r] = -(I->R[0][r] * I->T[0] + I->R[1][r] * I->T[1] + I->R[2][r] * I->T[2]);
      for (int r = 0; r < 3; ++r) {
        for (int c = 0; c < 3; ++c) I->Wf[4 * r + c] = (float)I->Ri[r][c];
        I->Wf[4 * r + 3] = (float)I->Ti[r];
      }
    }
    const omesh* m = &s->meshes[I->mesh];
    for (int k = 0; k < 3; ++k) {
      I->lo[k] = INFINITY;
      I->hi[k] = -INFINITY;
    }
    /* world bounds from the transformed vertices */
    for (int64_t t = 0; t < m->n_tris; ++t)
      for (int v = 0; v < 3; ++v) {
        double x[3] = {m->v[9 * t + 3 * v], m->v[9 * t + 3 * v + 1], m->v[9 * t + 3 * v + 2]}, y[3];
        if (I->identity) {
          y[0] = x[0]; y[1] = x[1]; y[2] = x[2];
        } else {
          mat_mul_vec(I->R, x, y);
          for (int k = 0; k < 3; ++k) y[k] += I->T[k];
        }
        for (int k = 0; k < 3; ++k) {
          if (y[k] < I->lo[k]) I->lo[k] = y[k];
          if (y[k] > I->hi[k]) I->hi[k] = y[k];
        }
      }
  }
  for (int k = 0; k < 3; ++k) {
    s->lo[k] = INFINITY;
    s->hi[k] = -INFINITY;
    for (int32_t i = 0; i < s->n_insts; ++i) {
      if (s->insts[i].lo[k] < s->lo[k]) s->lo[k] = s->insts[i].lo[k];
      if (s->insts[i].hi[k] > s->hi[k]) s->hi[k] = s->insts[i].hi[k];
    }
  }
  {
    double dx = s->hi[0] - s->lo[0], dy = s->hi[1] - s->lo[1], dz = s->hi[2] - s->lo[2];
    s->tmin = 1e-5 * sqrt(dx * dx + dy * dy + dz * dz);
  }
  /* every material id must be valid */
  for (int32_t i = 0; i < s->n_insts; ++i) {
    const oinst* I = &s->insts[i];
    if (I->mat_override >= n_materials) return -1;
    if (I->mat_override < 0) {
      const omesh* m = &s->meshes[I->mesh];
      for (int64_t t = 0; t < m->n_tris; ++t)
        if (m->mat[t] < 0 || m->mat[t] >= n_materials) return -1;
    }
  }
  int rc = oscene_build_env(s, env, env_w, env_h);
  if (rc) return rc;
  rc = oscene_build_lights(s);
  if (rc) return rc;
  *out = s;
  return 0;
}

void oracle_scene_destroy(oracle_scene* s) {
  if (!s) return;
  for (int32_t i = 0; i < s->n_meshes; ++i) {
    free(s->meshes[i].v);
    free(s->meshes[i].vf);
    free(s->meshes[i].mat);
    free(s->meshes[i].order);
    free(s->meshes[i].nodes);
  }
  for (int32_t i = 0; i < s->n_insts; ++i) free(s->insts[i].light_of_tri);
  free(s->meshes);
  free(s->insts);
  free(s->mats);
  free(s->env);
  free(s->env_row_pmf);
  free(s->env_row_cdf);
  free(s->env_col_pmf);
  free(s->env_col_cdf);
  free(s->lights);
  free(s->light_cdf);
  free(s);
}

double oracle_scene_tmin(const oracle_scene* s) { return s->tmin; }
int64_t oracle_scene_n_lights(const oracle_scene* s) { return s->n_lights; }

/* ------------------------------------------------ FP64 intersection -- */

/* Woop-Benthin-Wald watertight test in double.  Returns 1 and (t, b1, b2)
 * for a hit with nonzero determinant; b1, b2 weight v1, v2. */
static int tri_hit_f64(const double* v, v3 o, v3 d, double* t, double* b1, double* b2) {
  double ad[3] = {fabs(d.x), fabs(d.y), fabs(d.z)};
  int kz = 0;
  if (ad[1] > ad[kz]) kz = 1;
  if (ad[2] > ad[kz]) kz = 2;
  int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
  if (vget(d, kz) < 0) {
    int tmp = kx;
    kx = ky;
    ky = tmp;
  }
  double dz = vget(d, kz);
  double Sx = vget(d, kx) / dz, Sy = vget(d, ky) / dz, Sz = 1.0 / dz;
  v3 A = vsub(V(v[0], v[1], v[2]), o), B = vsub(V(v[3], v[4], v[5]), o), C = vsub(V(v[6], v[7], v[8]), o);
  double Ax = vget(A, kx) - Sx * vget(A, kz), Ay = vget(A, ky) - Sy * vget(A, kz);
  double Bx = vget(B, kx) - Sx * vget(B, kz), By = vget(B, ky) - Sy * vget(B, kz);
  double Cx = vget(C, kx) - Sx * vget(C, kz), Cy = vget(C, ky) - Sy * vget(C, kz);
  double U = Cx * By - Cy * Bx, Vv = Ax * Cy - Ay * Cx, W = Bx * Ay - By * Ax;
  if ((U < 0 || Vv < 0 || W < 0) && (U > 0 || Vv > 0 || W > 0)) return 0;
  double det = U + Vv + W;
  if (det == 0.0) return 0;
  double T = U * (Sz * vget(A, kz)) + Vv * (Sz * vget(B, kz)) + W * (Sz * vget(C, kz));
  *t = T / det;
  *b1 = Vv / det;
  *b2 = W / det;
  return 1;
}

static int box_hit(const double lo[3], const double hi[3], v3 o, v3 inv, double tmin, double tmax) {
  double t0 = tmin, t1 = tmax;
  for (int k = 0; k < 3; ++k) {
    double a = (lo[k] - vget(o, k)) * vget(inv, k), b = (hi[k] - vget(o, k)) * vget(inv, k);
    if (a != a) a = -INFINITY; /* 0 * inf: the ray lies in the slab plane */
    if (b != b) b = INFINITY;
    double n = a < b ? a : b, f = a < b ? b : a;
    if (n > t0) t0 = n;
    if (f < t1) t1 = f;
  }
  /* generous relative slack: this box test only prunes, it never decides a hit */
  return t0 <= t1 * (1.0 + 1e-9) + 1e-300;
}

static int better(double t, int32_t inst, int32_t prim, const ohit* h) {
  if (t < h->t) return 1;
  if (t > h->t) return 0;
  if (inst != h->inst) return inst < h->inst;
  return prim < h->prim;
}

static void world_to_object(const oinst* I, v3 o, v3 d, v3* oo, v3* od) {
  if (I->identity) {
    *oo = o;
    *od = d;
    return;
  }
  double x[3] = {o.x, o.y, o.z}, y[3], dx[3] = {d.x, d.y, d.z}, dy[3];
  mat_mul_vec(I->Ri, x, y);
  mat_mul_vec(I->Ri, dx, dy);
  *oo = V(y[0] + I->Ti[0], y[1] + I->Ti[1], y[2] + I->Ti[2]);
  *od = V(dy[0], dy[1], dy[2]);
}

/* any_hit: stop at the first accepted triangle. */
static int trace_mesh(const oracle_scene* s, int32_t inst, v3 o, v3 d, double tmin, double tmax,
                      int32_t skip_inst, int32_t skip_prim, ohit* h, int any_hit) {
  const oinst* I = &s->insts[inst];
  const omesh* m = &s->meshes[I->mesh];
  if (m->n_tris == 0) return 0;
  v3 oo, od;
  world_to_object(I, o, d, &oo, &od);
  v3 inv = V(1.0 / od.x, 1.0 / od.y, 1.0 / od.z);
  int32_t stack[128];
  int sp = 0;
  stack[sp++] = 0;
  int found = 0;
  while (sp) {
    const obvh_node* n = &m->nodes[stack[--sp]];
    double tcur = h->t < tmax ? h->t : tmax;
    if (!box_hit(n->lo, n->hi, oo, inv, tmin, tcur)) continue;
    if (n->count == 0) {
      if (sp + 2 > 128) return -1;
      stack[sp++] = n->left;
      stack[sp++] = n->right;
      continue;
    }
    for (int32_t i = n->first; i < n->first + n->count; ++i) {
      int32_t prim = m->order[i];
      if (inst == skip_inst && prim == skip_prim) continue;
      double t, b1, b2;
      if (!tri_hit_f64(&m->v[9 * (int64_t)prim], oo, od, &t, &b1, &b2)) continue;
      if (!(t > tmin && t < tmax)) continue;
      if (!better(t, inst, prim, h)) continue;
      h->t = t;
      h->b1 = b1;
      h->b2 = b2;
      h->inst = inst;
      h->prim = prim;
      found = 1;
      if (any_hit) return 1;
    }
  }
  return found;
}

static int inst_box_hit(const oinst* I, v3 o, v3 d, double tmin, double tmax) {
  v3 inv = V(1.0 / d.x, 1.0 / d.y, 1.0 / d.z);
  double lo[3], hi[3];
  for (int k = 0; k < 3; ++k) {
    double pad = 1e-9 * (fabs(I->lo[k]) + fabs(I->hi[k]) + 1.0);
    lo[k] = I->lo[k] - pad;
    hi[k] = I->hi[k] + pad;
  }
  return box_hit(lo, hi, o, inv, tmin, tmax);
}

int oclosest(const oracle_scene* s, v3 o, v3 d, double tmin, double tmax, int32_t skip_inst,
             int32_t skip_prim, ohit* h) {
  h->t = INFINITY;
  h->inst = h->prim = -1;
  h->b1 = h->b2 = 0;
  int found = 0;
  for (int32_t i = 0; i < s->n_insts; ++i) {
    double tcur = h->t < tmax ? h->t : tmax;
    if (!inst_box_hit(&s->insts[i], o, d, tmin, tcur)) continue;
    int r = trace_mesh(s, i, o, d, tmin, tmax, skip_inst, skip_prim, h, 0);
    if (r < 0) return r;
    found |= r;
  }
  return found;
}

int ooccluded(const oracle_scene* s, v3 o, v3 d, double tmin, double tmax, int32_t skip_inst,
              int32_t skip_prim) {
  for (int32_t i = 0; i < s->n_insts; ++i) {
    if (!inst_box_hit(&s->insts[i], o, d, tmin, tmax)) continue;
    ohit h;
    h.t = INFINITY;
    h.inst = h.prim = -1;
    if (trace_mesh(s, i, o, d, tmin, tmax, skip_inst, skip_prim, &h, 1) > 0) return 1;
  }
  return 0;
}

int oracle_closest_f64(const oracle_scene* s, const double o[3], const double d[3], double tmin,
                       double tmax, int32_t skip_inst, int32_t skip_prim, double hit[3], int32_t ids[2]) {
  ohit h;
  int r = oclosest(s, V(o[0], o[1], o[2]), V(d[0], d[1], d[2]), tmin, tmax, skip_inst, skip_prim, &h);
  if (r < 0) return r;
  hit[0] = h.t; hit[1] = h.b1; hit[2] = h.b2;
  ids[0] = h.inst; ids[1] = h.prim;
  return r;
}

int oracle_closest_f64_brute(const oracle_scene* s, const double o[3], const double d[3], double tmin,
                             double tmax, int32_t skip_inst, int32_t skip_prim, double hit[3],
                             int32_t ids[2]) {
  ohit h;
  h.t = INFINITY;
  h.inst = h.prim = -1;
  h.b1 = h.b2 = 0;
  int found = 0;
  v3 O = V(o[0], o[1], o[2]), D = V(d[0], d[1], d[2]);
  for (int32_t i = 0; i < s->n_insts; ++i) {
    const oinst* I = &s->insts[i];
    const omesh* m = &s->meshes[I->mesh];
    v3 oo, od;
    world_to_object(I, O, D, &oo, &od);
    for (int64_t p = 0; p < m->n_tris; ++p) {
      if (i == skip_inst && p == skip_prim) continue;
      double t, b1, b2;
      if (!tri_hit_f64(&m->v[9 * p], oo, od, &t, &b1, &b2)) continue;
      if (!(t > tmin && t < tmax)) continue;
      if (!better(t, i, (int32_t)p, &h)) continue;
      h.t = t; h.b1 = b1; h.b2 = b2; h.inst = i; h.prim = (int32_t)p;
      found = 1;
    }
  }
  hit[0] = h.t; hit[1] = h.b1; hit[2] = h.b2;
  ids[0] = h.inst; ids[1] = h.prim;
  return found;
}

/* ------------------------------------------- FP32 exact definition -- */

/*
 * Single-precision watertight test, every operation in float and in this
 * order (no contraction):
 *   kz = argmax |d_k| (first axis wins ties); kx = kz+1, ky = kx+1 (mod 3);
 *   swap kx, ky if d_kz < 0;  Sx = d_kx/d_kz, Sy = d_ky/d_kz, Sz = 1/d_kz;
 *   A = v0-o, B = v1-o, C = v2-o;
 *   Ax = A_kx - Sx*A_kz, Ay = A_ky - Sy*A_kz (same for B, C);
 *   U = Cx*By - Cy*Bx, V = Ax*Cy - Ay*Cx, W = Bx*Ay - By*Ax;
 *   if any of U,V,W is 0: recompute all three as float(double products difference);
 *   miss if signs differ;  det = (U+V)+W, miss if det == 0;
 *   T = (U*(Sz*A_kz) + V*(Sz*B_kz)) + W*(Sz*C_kz);  r = 1/det;
 *   t = T*r, b1 = V*r, b2 = W*r.
 * Object-space rays of an instance: o' = ((W0*ox + W1*oy) + W2*oz) + W3 per
 * row of the float world-to-object matrix, d' likewise without W3.
 */
static int tri_hit_f32(const float* v, const float o[3], const float d[3], float* tt, float* b1,
                       float* b2) {
  float a0 = fabsf(d[0]), a1 = fabsf(d[1]), a2 = fabsf(d[2]);
  int kz = 0;
  float am = a0;
  if (a1 > am) { kz = 1; am = a1; }
  if (a2 > am) { kz = 2; }
  int kx = (kz + 1) % 3, ky = (kx + 1) % 3;
  if (d[kz] < 0.0f) {
    int tmp = kx;
    kx = ky;
    ky = tmp;
  }
  float Sx = d[kx] / d[kz];
  float Sy = d[ky] / d[kz];
  float Sz = 1.0f / d[kz];
  float A[3], B[3], C[3];
  for (int k = 0; k < 3; ++k) {
    A[k] = v[k] - o[k];
    B[k] = v[3 + k] - o[k];
    C[k] = v[6 + k] - o[k];
  }
  float Ax = A[kx] - Sx * A[kz], Ay = A[ky] - Sy * A[kz];
  float Bx = B[kx] - Sx * B[kz], By = B[ky] - Sy * B[kz];
  float Cx = C[kx] - Sx * C[kz], Cy = C[ky] - Sy * C[kz];
  float U = Cx * By - Cy * Bx;
  float Vv = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.0f || Vv == 0.0f || W == 0.0f) {
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    Vv = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
  if ((U < 0.0f || Vv < 0.0f || W < 0.0f) && (U > 0.0f || Vv > 0.0f || W > 0.0f)) return 0;
  float det = (U + Vv) + W;
  if (det == 0.0f) return 0;
  float Az = Sz * A[kz], Bz = Sz * B[kz], Cz = Sz * C[kz];
  float T = (U * Az + Vv * Bz) + W * Cz;
  float r = 1.0f / det;
  *tt = T * r;
  *b1 = Vv * r;
  *b2 = W * r;
  return 1;
}

typedef struct {
  const oracle_scene* s;
  const float* rays;
  uint32_t* hits;
  int64_t n;
  int tid, nt;
} f32job;

static uint32_t fbits(float x) {
  uint32_t u;
  memcpy(&u, &x, 4);
  return u;
}

static void* f32_worker(void* arg) {
  f32job* J = (f32job*)arg;
  const oracle_scene* s = J->s;
  for (int64_t r = J->tid; r < J->n; r += J->nt) {
    const float* R = J->rays + 8 * r;
    float best_t = INFINITY, bb1 = 0.0f, bb2 = 0.0f;
    int32_t bi = -1, bp = -1;
    for (int32_t i = 0; i < s->n_insts; ++i) {
      const oinst* I = &s->insts[i];
      const omesh* m = &s->meshes[I->mesh];
      float o[3], d[3];
      if (I->identity) {
        for (int k = 0; k < 3; ++k) {
          o[k] = R[k];
          d[k] = R[4 + k];
        }
      } else {
        for (int k = 0; k < 3; ++k) {
          const float* w = &I->Wf[4 * k];
          o[k] = ((w[0] * R[0] + w[1] * R[1]) + w[2] * R[2]) + w[3];
          d[k] = (w[0] * R[4] + w[1] * R[5]) + w[2] * R[6];
        }
      }
      for (int64_t p = 0; p < m->n_tris; ++p) {
        float t, b1, b2;
        if (!tri_hit_f32(&m->vf[9 * p], o, d, &t, &b1, &b2)) continue;
        if (!(t > R[3] && t < R[7])) continue;
        int take = 0;
        if (t < best_t) take = 1;
        else if (t == best_t && (i < bi || (i == bi && p < bp))) take = 1;
        if (!take) continue;
        best_t = t; bb1 = b1; bb2 = b2; bi = i; bp = (int32_t)p;
      }
    }
    uint32_t* H = J->hits + 6 * r;
    H[0] = fbits(best_t);
    H[1] = (uint32_t)bi;
    H[2] = (uint32_t)bp;
    H[3] = fbits(bb1);
    H[4] = fbits(bb2);
    H[5] = bi >= 0 ? 1u : 0u;
  }
  return NULL;
}

int oracle_closest_f32_brute(const oracle_scene* s, const float* rays, int64_t n, uint32_t* hits,
                             int32_t n_threads) {
  if (!s || (!rays && n) || (!hits && n) || n < 0) return -1;
  int nt = n_threads > 0 ? n_threads : 1;
  if (nt > 256) nt = 256;
  pthread_t th[256];
  f32job jobs[256];
  for (int i = 0; i < nt; ++i) {
    jobs[i].s = s; jobs[i].rays = rays; jobs[i].hits = hits; jobs[i].n = n;
    jobs[i].tid = i; jobs[i].nt = nt;
    pthread_create(&th[i], NULL, f32_worker, &jobs[i]);
  }
  for (int i = 0; i < nt; ++i) pthread_join(th[i], NULL);
  return 0;
}
