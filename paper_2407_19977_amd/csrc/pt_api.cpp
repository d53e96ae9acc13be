// C ABI of the path tracer: scene set-up on the host (paper Sec. 5.1.1) and
// sampling passes on the GPU (Sec. 5.1.2 - 5.1.3).  See include/pt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <functional>
#include <memory>
#include <string>
#include <vector>

#include "pt_internal.h"
#include "pt_nrc.h"
#include "pt_trace.h"

using namespace pt;

namespace {

thread_local std::string g_err;

pt_status fail(pt_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

#define PT_HIP(call)                                                                          \
  do {                                                                                        \
    hipError_t e_ = (call);                                                                   \
    if (e_ != hipSuccess)                                                                     \
      return fail(PT_ERR_DEVICE, "%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), __FILE__, \
                  __LINE__);                                                                  \
  } while (0)

// Owning device allocation.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void release() {
    if (p) (void)hipFree(p);
    p = nullptr;
    bytes = 0;
  }
  hipError_t alloc(size_t n) {
    if (n <= bytes && p) return hipSuccess;
    release();
    hipError_t e = hipMalloc(&p, n ? n : 16);
    if (e == hipSuccess) bytes = n;
    return e;
  }
  template <class T>
  T* as() const {
    return static_cast<T*>(p);
  }
};

hipError_t upload(DevBuf& b, const void* src, size_t n, hipStream_t st) {
  hipError_t e = b.alloc(n);
  if (e != hipSuccess) return e;
  if (n) e = hipMemcpyAsync(b.p, src, n, hipMemcpyHostToDevice, st);
  return e;
}

double lumd(double r, double g, double b) { return 0.2126 * r + 0.7152 * g + 0.0722 * b; }

bool finite_all(const float* p, size_t n) {
  for (size_t i = 0; i < n; ++i)
    if (!std::isfinite(p[i])) return false;
  return true;
}

}  // namespace

// Device buffers of one set of path slots (struct-of-arrays).
struct PathBufs {
  int64_t capacity = 0, nrc_q_cap = 0;
  DevBuf ray_o, ray_d, hit, hit_inst, cls, beta, L, flags, q_ray[2], q_cls[kNumClasses], sh_o, sh_d, sh_c, sh_inst,
      counts, sig, dbg_nee, dbg_tail, spill, nrc_q, q_nrc, spread;
};

struct pt_scene {
  int device = 0;
  hipStream_t stream = nullptr;
  // geometry
  bool has_bvh = false;
  DevBuf nodes, tris;
  uint32_t n_tris = 0;
  int bvh_depth = 0;
  int64_t n_nodes = 0;       // mesh-level BVH4 nodes in `nodes`
  int bvh_max_leaf = 0;
  double bvh_sah = 0.0;      // host builds only
  double bvh_build_ms = 0.0; // triangle soup in host memory -> BVH ready where the builder leaves it
  bool bvh_on_device = false;
  float tmin = 0.0f;
  int32_t max_mat_id = -1;
  std::vector<float> host_tri_verts;  // [n][9] world space, prim order (single level)
  std::vector<int32_t> host_tri_mat;  // [n], prim order (single level)
  // two-level hierarchy
  bool two_level = false;
  DevBuf insts, tlas, tlas_items, light_map, mesh_tri_first, mesh_tri_count;
  std::vector<InstRec> host_insts;
  std::vector<std::vector<float>> host_mesh_verts;   // per mesh [n][9], object space, prim order
  std::vector<std::vector<int32_t>> host_mesh_mat;   // per mesh [n]
  // materials
  bool has_mats = false;
  std::vector<pt_openpbr_material> host_mats;
  DevBuf mats, fuzz_tabs;
  uint32_t class_mask = 0;
  // environment
  int env_w = 0, env_h = 0;
  DevBuf env, env_row_pmf, env_row_cdf, env_col_pmf, env_col_cdf, env_row_guide, env_col_guide;
  // lights
  bool lights_dirty = true;
  DevBuf lights, light_cdf, tri_light;
  int32_t n_lights = 0;
  float p_env = 0.0f;
  // path state: two sets, so that a pass's tail can run on the second stream
  // while the next pass starts on the first
  PathBufs pb[2];
  DevBuf stats;
  unsigned long long overflow_seen = 0;  // stack overflows already reported by a failed call
  hipStream_t stream2 = nullptr;       // created on first use (default priority)
  hipStream_t shade_side[2] = {nullptr, nullptr};  // side streams of the shading kernels (default priority)
  hipEvent_t shade_fork = nullptr, shade_join[2] = {nullptr, nullptr};
  hipEvent_t ev_bulk[2] = {nullptr, nullptr}, ev_done[2] = {nullptr, nullptr};
  uint32_t* tail_counts = nullptr;     // pinned host words, one per set
  // accumulation
  DevBuf sum;
  int acc_w = 0, acc_h = 0;
  int64_t acc_samples = 0;
  // profiling
  bool timing = false, counting = false;
  double ms_extend = 0.0, ms_total = 0.0;
  int64_t launches_extend = 0;
  int64_t samples = 0;
  std::vector<hipEvent_t> events[2];  // timing events per path set
  // scene box (radiance-cache position input)
  float box_lo[3] = {0.0f, 0.0f, 0.0f}, box_inv[3] = {0.0f, 0.0f, 0.0f};
  // radiance cache
  bool nrc_on = false;     // configured
  bool nrc_ready = false;  // weights set or trained: sampling passes end paths in the cache
  pt_radiance_cache_config nrc_cfg;
  DevBuf nrc_t;            // Adam steps applied (one device word: steps with no records are skipped there)
  DevBuf nrc_w, nrc_m, nrc_v, nrc_fwd, nrc_bwd;  // FP32 master weights, Adam moments, bf16 fragments
  DevBuf nrc_e, nrc_wi, nrc_inf;  // moving average of the weights, inference weights, their bf16 fragments
  DevBuf nrc_tail[2];  // per training path: beta * cache at its terminal vertex (self-training), per path set
  DevBuf nrc_rec[2];       // training records, per path set (frames overlap on two sets)
  DevBuf nrc_off, nrc_bsum, nrc_n, nrc_X, nrc_T;  // compaction
  int64_t nrc_rec_cap = 0;
  DevBuf nrc_Xb, nrc_Tb, nrc_a, nrc_g, nrc_loss, nrc_dw;  // one training step's workspace
  int64_t nrc_ws_npad = 0;
  int nrc_ws_split = 0;
  double ms_cache_query = 0.0, ms_cache_train = 0.0;
  hipEvent_t ev_train = nullptr;  // the last enqueued training's weights are in place
  hipEvent_t ev_train_t[2][2] = {{nullptr, nullptr}, {nullptr, nullptr}};  // timing around a frame's training
  // tail hand-off
  int tail_min_bounce = 2;
  double tail_fraction = 0.15;
  int gpu_bvh_builder = kGpuBvhPloc;  // builder of pt_build_bvh_gpu
  double ms_tail = 0.0;
  int64_t launches_tail = 0;
  // display path
  double ms_display = 0.0;
  int64_t launches_display = 0;
  hipEvent_t ev_display[2] = {nullptr, nullptr};
  double ms_cache_forward = 0.0;
  int64_t cache_forward_queries = 0;
  hipEvent_t ev_forward[2] = {nullptr, nullptr};
};

namespace {

pt_status check_scene(pt_scene* s) {
  if (!s) return fail(PT_ERR_INVALID_ARG, "scene is NULL");
  return PT_OK;
}

pt_status set_device(pt_scene* s) {
  PT_HIP(hipSetDevice(s->device));
  return PT_OK;
}

// Scene box from exact vertex bounds; an axis of zero extent maps to 0.
void set_box(pt_scene* s, const double lo[3], const double hi[3]) {
  for (int k = 0; k < 3; ++k) {
    double e = hi[k] - lo[k];
    s->box_lo[k] = (float)lo[k];
    s->box_inv[k] = e > 0.0 ? (float)(1.0 / e) : 0.0f;
  }
}

bool mat_emits(const pt_openpbr_material& m) {
  return m.emission_luminance > 0.0f && lumd(m.emission_color[0], m.emission_color[1], m.emission_color[2]) > 0.0;
}

struct LightTmp {
  LightTri t;
  double w;
};

// v: world-space vertices (double) of an emissive triangle
void push_light(std::vector<LightTmp>& list, const double* v, const pt_openpbr_material& m) {
  double Le[3] = {(double)m.emission_luminance * m.emission_color[0],
                  (double)m.emission_luminance * m.emission_color[1],
                  (double)m.emission_luminance * m.emission_color[2]};
  double e1[3], e2[3];
  for (int k = 0; k < 3; ++k) {
    e1[k] = v[3 + k] - v[k];
    e2[k] = v[6 + k] - v[k];
  }
  double c[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
  double len = std::sqrt(c[0] * c[0] + c[1] * c[1] + c[2] * c[2]);
  LightTmp t;
  std::memset(&t, 0, sizeof(t));
  double area = 0.5 * len;
  t.t.p0 = make_float4((float)v[0], (float)v[1], (float)v[2], (float)area);
  t.t.p1 = make_float4((float)v[3], (float)v[4], (float)v[5], 0.0f);
  t.t.p2 = make_float4((float)v[6], (float)v[7], (float)v[8], 0.0f);
  t.t.ng = len > 0 ? make_float4((float)(c[0] / len), (float)(c[1] / len), (float)(c[2] / len), 0.0f)
                   : make_float4(0, 0, 0, 0);
  t.t.Le = make_float4((float)Le[0], (float)Le[1], (float)Le[2], 0.0f);
  t.w = area * lumd(Le[0], Le[1], Le[2]);
  list.push_back(t);
}

pt_status ensure_lights(pt_scene* s) {
  if (!s->lights_dirty) return PT_OK;
  std::vector<LightTmp> list;
  std::vector<int32_t> tri_light(1, -1), lmap(1, -1);
  if (!s->two_level) {
    const int64_t n = s->n_tris;
    tri_light.assign((size_t)std::max<int64_t>(n, 1), -1);
    for (int64_t i = 0; i < n; ++i) {
      const pt_openpbr_material& m = s->host_mats[(size_t)s->host_tri_mat[(size_t)i]];
      if (!mat_emits(m)) continue;
      const float* v = &s->host_tri_verts[9 * (size_t)i];
      double vd[9];
      for (int k = 0; k < 9; ++k) vd[k] = v[k];
      tri_light[(size_t)i] = (int32_t)list.size();
      push_light(list, vd, m);
    }
  } else {
    // lights in instance order, then primitive order; each instance with emitters gets a
    // primitive -> light table
    lmap.clear();
    for (size_t i = 0; i < s->host_insts.size(); ++i) {
      InstRec& I = s->host_insts[i];
      I.light_map = -1;
      const std::vector<float>& mv = s->host_mesh_verts[I.mesh];
      const std::vector<int32_t>& mm = s->host_mesh_mat[I.mesh];
      size_t nt = mm.size();
      for (size_t t = 0; t < nt; ++t) {
        int32_t mid = I.mat_override >= 0 ? I.mat_override : mm[t];
        const pt_openpbr_material& m = s->host_mats[(size_t)mid];
        if (!mat_emits(m)) continue;
        if (I.light_map < 0) {
          I.light_map = (int32_t)lmap.size();
          lmap.resize(lmap.size() + nt, -1);
        }
        double vd[9];
        const float* q = I.o2w;
        for (int v = 0; v < 3; ++v) {
          double x = mv[9 * t + 3 * v], y = mv[9 * t + 3 * v + 1], z = mv[9 * t + 3 * v + 2];
          for (int r = 0; r < 3; ++r)
            vd[3 * v + r] = (double)q[4 * r] * x + (double)q[4 * r + 1] * y + (double)q[4 * r + 2] * z + (double)q[4 * r + 3];
        }
        lmap[(size_t)I.light_map + t] = (int32_t)list.size();
        push_light(list, vd, m);
      }
    }
    if (lmap.empty()) lmap.push_back(-1);
  }
  double wsum = 0.0;
  for (auto& t : list) wsum += t.w;
  bool has_tri = !list.empty() && wsum > 0.0;
  bool has_env = s->env_w > 0;
  double p_env = !has_env ? 0.0 : (has_tri ? 0.5 : 1.0);
  std::vector<LightTri> lt;
  std::vector<float> cdf(list.size() + 1, 0.0f);
  double acc = 0.0;
  for (size_t k = 0; k < list.size(); ++k) {
    LightTri t = list[k].t;
    t.p1.w = has_tri ? (float)((1.0 - p_env) * list[k].w / wsum) : 0.0f;
    lt.push_back(t);
    acc += list[k].w;
    cdf[k + 1] = has_tri ? (float)(acc / wsum) : 0.0f;
  }
  if (has_tri) cdf[list.size()] = 1.0f;
  if (!has_tri) {
    lt.clear();
    std::fill(tri_light.begin(), tri_light.end(), -1);
    std::fill(lmap.begin(), lmap.end(), -1);
  }
  s->n_lights = (int32_t)lt.size();
  s->p_env = (float)p_env;
  PT_HIP(upload(s->lights, lt.data(), lt.size() * sizeof(LightTri), s->stream));
  PT_HIP(upload(s->light_cdf, cdf.data(), cdf.size() * sizeof(float), s->stream));
  PT_HIP(upload(s->tri_light, tri_light.data(), tri_light.size() * sizeof(int32_t), s->stream));
  PT_HIP(upload(s->light_map, lmap.data(), lmap.size() * sizeof(int32_t), s->stream));
  if (s->two_level)
    PT_HIP(upload(s->insts, s->host_insts.data(), s->host_insts.size() * sizeof(InstRec), s->stream));
  PT_HIP(hipStreamSynchronize(s->stream));
  s->lights_dirty = false;
  return PT_OK;
}

pt_status ensure_paths(pt_scene* s, int64_t n, int set = 0) {
  PathBufs& B = s->pb[set];
  if (n <= B.capacity) return PT_OK;
  size_t f4 = (size_t)n * sizeof(float4), u4 = (size_t)n * sizeof(uint32_t);
  PT_HIP(B.ray_o.alloc(f4));
  PT_HIP(B.ray_d.alloc(f4));
  PT_HIP(B.hit.alloc(f4));
  PT_HIP(B.hit_inst.alloc(u4));
  PT_HIP(B.cls.alloc((size_t)n));
  PT_HIP(B.sh_inst.alloc(u4));
  PT_HIP(B.beta.alloc(f4));
  PT_HIP(B.L.alloc(f4));
  PT_HIP(B.flags.alloc(u4));
  for (int i = 0; i < 2; ++i) PT_HIP(B.q_ray[i].alloc(u4));
  for (int i = 0; i < kNumClasses; ++i) PT_HIP(B.q_cls[i].alloc(u4));
  PT_HIP(B.sh_o.alloc(f4));
  PT_HIP(B.sh_d.alloc(f4));
  PT_HIP(B.sh_c.alloc(f4));
  PT_HIP(B.sig.alloc((size_t)n * sizeof(uint64_t)));
  PT_HIP(B.dbg_nee.alloc(u4));
  PT_HIP(B.dbg_tail.alloc(u4));
  PT_HIP(B.spread.alloc((size_t)n * sizeof(float2)));
  B.capacity = n;
  return PT_OK;
}

int bin_grid(int64_t n) {  // 1024 rays per workgroup iteration
  return (int)std::max<int64_t>(1, std::min<int64_t>((n + 1023) / 1024, 2048));
}

int grid_for(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(b, 2048));
}

pt_status ensure_counters(pt_scene* s, int set = 0) {
  PathBufs& B = s->pb[set];
  if (!B.counts.p) {
    PT_HIP(B.counts.alloc(kNumCounts * sizeof(uint32_t)));
    PT_HIP(hipMemsetAsync(B.counts.p, 0, kNumCounts * sizeof(uint32_t), s->stream));
  }
  if (!s->stats.p) {
    PT_HIP(s->stats.alloc(kNumStats * sizeof(unsigned long long)));
    PT_HIP(launch_zero_u64(s->stats.as<unsigned long long>(), kNumStats, s->stream));
  }
  return PT_OK;
}

pt_status ensure_spill(pt_scene* s, int grid_trace, int set = 0) {
  int cap = stack_capacity(s->bvh_depth);
  size_t per = cap > kLdsStack ? (size_t)(cap - kLdsStack) : 1;
  size_t bytes = per * (size_t)grid_trace * kBlock * sizeof(uint2);
  PT_HIP(s->pb[set].spill.alloc(bytes));
  return PT_OK;
}

SceneDev scene_dev(pt_scene* s, int grid_trace, int set = 0) {
  SceneDev S;
  std::memset(&S, 0, sizeof(S));
  S.nodes = s->nodes.as<BVHNode>();
  S.tris = s->tris.as<TriRec>();
  S.n_tris = s->n_tris;
  S.root = 0;
  S.mats = s->mats.as<MatRec>();
  S.tri_light = s->tri_light.as<int32_t>();
  S.lights = s->lights.as<LightTri>();
  S.light_cdf = s->light_cdf.as<float>();
  S.n_lights = s->n_lights;
  S.p_env = s->p_env;
  S.env = s->env.as<float4>();
  S.env_row_pmf = s->env_row_pmf.as<float>();
  S.env_row_cdf = s->env_row_cdf.as<float>();
  S.env_col_pmf = s->env_col_pmf.as<float>();
  S.env_col_cdf = s->env_col_cdf.as<float>();
  S.env_row_guide = s->env_row_guide.as<int32_t>();
  S.env_col_guide = s->env_col_guide.as<int32_t>();
  S.env_w = s->env_w;
  S.env_h = s->env_h;
  S.tmin = s->tmin;
  S.axis[0] = 0.0f;
  S.axis[1] = 0.0f;
  S.axis[2] = 1.0f;
  S.spill = s->pb[set].spill.as<uint2>();
  S.stack_cap = stack_capacity(s->bvh_depth);
  S.spill_stride = (uint32_t)grid_trace * kBlock;
  S.insts = s->insts.as<InstRec>();
  S.n_insts = (uint32_t)s->host_insts.size();
  S.tlas = s->tlas.as<BVHNode>();
  S.tlas_items = s->tlas_items.as<uint32_t>();
  S.light_map = s->light_map.as<int32_t>();
  S.mesh_tri_first = s->mesh_tri_first.as<uint32_t>();
  S.mesh_tri_count = s->mesh_tri_count.as<uint32_t>();
  for (int k = 0; k < 3; ++k) {
    S.box_lo[k] = s->box_lo[k];
    S.box_inv[k] = s->box_inv[k];
  }
  return S;
}

PathsDev paths_dev(pt_scene* s, int64_t n, int x0, int y0, int w, int set = 0) {
  PathBufs& B = s->pb[set];
  PathsDev P;
  std::memset(&P, 0, sizeof(P));
  P.ray_o = B.ray_o.as<float4>();
  P.ray_d = B.ray_d.as<float4>();
  P.hit = B.hit.as<float4>();
  P.hit_inst = B.hit_inst.as<uint32_t>();
  P.cls = B.cls.as<uint8_t>();
  P.sh_inst = B.sh_inst.as<uint32_t>();
  P.beta = B.beta.as<float4>();
  P.L = B.L.as<float4>();
  P.flags = B.flags.as<uint32_t>();
  for (int i = 0; i < 2; ++i) P.q_ray[i] = B.q_ray[i].as<uint32_t>();
  for (int i = 0; i < kNumClasses; ++i) P.q_cls[i] = B.q_cls[i].as<uint32_t>();
  P.sh_o = B.sh_o.as<float4>();
  P.sh_d = B.sh_d.as<float4>();
  P.sh_c = B.sh_c.as<float4>();
  P.counts = B.counts.as<uint32_t>();
  P.stats = s->stats.as<unsigned long long>();
  P.sig = B.sig.as<uint64_t>();
  P.dbg_nee = B.dbg_nee.as<uint32_t>();
  P.dbg_tail = B.dbg_tail.as<uint32_t>();
  P.spread = B.spread.as<float2>();
  P.spread_c = s->nrc_on ? s->nrc_cfg.spread_c : 0.0f;
  P.n = (int32_t)n;
  P.n_render = (int32_t)n;
  P.x0 = x0;
  P.y0 = y0;
  P.w = w;
  P.train_end = -1;
  P.nrc_factor = s->nrc_on && s->nrc_cfg.factorize ? 1 : 0;
  return P;
}

pt_status make_camera(const pt_camera* c, CamDev& C) {
  if (!c) return fail(PT_ERR_INVALID_ARG, "camera is NULL");
  if (c->width <= 0 || c->height <= 0) return fail(PT_ERR_INVALID_ARG, "camera width/height must be > 0");
  if ((int64_t)c->width * c->height > (int64_t)1 << 28) return fail(PT_ERR_INVALID_ARG, "image too large");
  if (!(c->vfov_deg > 0.0f && c->vfov_deg < 180.0f)) return fail(PT_ERR_INVALID_ARG, "vfov_deg must be in (0, 180)");
  if (!finite_all(c->eye, 3) || !finite_all(c->look_at, 3) || !finite_all(c->up, 3))
    return fail(PT_ERR_INVALID_ARG, "camera vectors must be finite");
  double F[3], R[3], U[3];
  for (int k = 0; k < 3; ++k) F[k] = (double)c->look_at[k] - c->eye[k];
  double fl = std::sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
  if (!(fl > 0)) return fail(PT_ERR_INVALID_ARG, "look_at equals eye");
  for (int k = 0; k < 3; ++k) F[k] /= fl;
  double up[3] = {c->up[0], c->up[1], c->up[2]};
  R[0] = F[1] * up[2] - F[2] * up[1];
  R[1] = F[2] * up[0] - F[0] * up[2];
  R[2] = F[0] * up[1] - F[1] * up[0];
  double rl = std::sqrt(R[0] * R[0] + R[1] * R[1] + R[2] * R[2]);
  if (!(rl > 0)) return fail(PT_ERR_INVALID_ARG, "up is parallel to the view direction");
  for (int k = 0; k < 3; ++k) R[k] /= rl;
  U[0] = R[1] * F[2] - R[2] * F[1];
  U[1] = R[2] * F[0] - R[0] * F[2];
  U[2] = R[0] * F[1] - R[1] * F[0];
  for (int k = 0; k < 3; ++k) {
    C.eye[k] = c->eye[k];
    C.R[k] = (float)R[k];
    C.U[k] = (float)U[k];
    C.F[k] = (float)F[k];
  }
  C.tan_half = (float)std::tan(0.5 * (double)c->vfov_deg * M_PI / 180.0);
  C.aspect = (float)((double)c->width / (double)c->height);
  C.W = c->width;
  C.H = c->height;
  return PT_OK;
}

pt_status ready_to_render(pt_scene* s) {
  if (!s->has_bvh) return fail(PT_ERR_STATE, "pt_build_bvh has not been called");
  if (!s->has_mats) return fail(PT_ERR_STATE, "pt_upload_materials has not been called");
  if (s->max_mat_id >= (int32_t)s->host_mats.size())
    return fail(PT_ERR_STATE, "material id %d >= material count %d", s->max_mat_id, (int)s->host_mats.size());
  return ensure_lights(s);
}

// Training paths of a frame appended to a pass as slots [n_render, n_render + paths):
// path k starts at pixel (k * stride + o_f) mod WH, stride = max(1, floor(WH / paths)),
// o_f = floor(m * WH / 2^24) with m the top 24 bits of Philox word 0 at counter
// (0, 2^31 + frame, 0x4F4646, 0); sample index 2^31 + frame.  Each records
// (inputs, radiance so far, throughput) at its vertices below max_depth.
pt_status setup_training(pt_scene* s, const CamDev& C, PathsDev& P, int64_t n_render, uint32_t frame, int max_depth,
                         uint64_t seed, int set = 0) {
  const int64_t n = s->nrc_cfg.train_paths;
  const int depth = std::max(1, max_depth);
  if (n * depth > s->nrc_rec_cap) {
    PT_HIP(s->nrc_rec[0].alloc((size_t)n * depth * kNrcRecFloats * sizeof(float)));
    if (s->nrc_rec[1].p) PT_HIP(s->nrc_rec[1].alloc((size_t)n * depth * kNrcRecFloats * sizeof(float)));
    PT_HIP(s->nrc_X.alloc((size_t)n * depth * 12 * sizeof(float)));
    PT_HIP(s->nrc_T.alloc((size_t)n * depth * 3 * sizeof(float)));
    s->nrc_rec_cap = n * depth;
  }
  if (set == 1 && !s->nrc_rec[1].p) PT_HIP(s->nrc_rec[1].alloc(s->nrc_rec[0].bytes));
  PT_HIP(s->nrc_off.alloc((size_t)n * sizeof(uint32_t)));
  PT_HIP(s->nrc_bsum.alloc((size_t)((n + 255) / 256) * sizeof(uint32_t)));
  if (!s->nrc_n.p) PT_HIP(s->nrc_n.alloc(sizeof(uint32_t)));
  const uint64_t WH = (uint64_t)C.W * (uint64_t)C.H;
  P.n = (int32_t)(n_render + n);
  P.n_render = (int32_t)n_render;
  P.pix_total = (uint32_t)WH;
  P.pix_stride = (uint32_t)std::max<uint64_t>(1, WH / (uint64_t)n);
  U4 u = philox(0u, 0x80000000u + frame, 0x4F4646u, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
  P.pix_off = (uint32_t)(((uint64_t)(u.x >> 8) * WH) >> 24);
  P.train_sample = 0x80000000u + frame;
  P.rec = s->nrc_rec[set].as<float>();
  P.rec_depth = max_depth;
  // self-training: once the cache has weights, training paths end in it at train_end_bounce
  const int te = s->nrc_cfg.train_end_bounce;
  P.train_end = (s->nrc_ready && te >= 0 && te < max_depth) ? te : -1;
  P.nrc_factor = s->nrc_cfg.factorize ? 1 : 0;
  return PT_OK;
}

// Targets of the training paths of the last pass, compacted path by path, on stream st; the count
// stays on the device (and is added to the record statistics) unless n_records asks for it on the host.
pt_status finish_training(pt_scene* s, const PathsDev& P, uint32_t* n_records, hipStream_t st,
                          bool count_stats = false) {
  const int n = P.n - P.n_render;
  float4* tail = nullptr;
  if (P.train_end >= 0) {  // the cache's answer at the training paths' terminal vertices
    tail = s->nrc_tail[P.rec == s->nrc_rec[1].as<float>() ? 1 : 0].as<float4>();
    PT_HIP(nrc_launch_terminal(P, n, s->nrc_inf.as<uint4>(), tail, st));
  }
  PT_HIP(nrc_launch_targets(P, n, tail, s->nrc_off.as<uint32_t>(), s->nrc_bsum.as<uint32_t>(), s->nrc_X.as<float>(),
                            s->nrc_T.as<float>(), s->nrc_n.as<uint32_t>(),
                            count_stats ? s->stats.as<unsigned long long>() : nullptr, st));
  if (n_records) {
    PT_HIP(hipMemcpyAsync(n_records, s->nrc_n.p, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    PT_HIP(hipStreamSynchronize(st));
  }
  return PT_OK;
}

pt_status nrc_train_records(pt_scene* s, const float* X_all, const float* T_all, const uint32_t* n_dev,
                            uint32_t frame, uint64_t seed, double* mean_loss, hipStream_t st);
pt_status nrc_ensure_ws(pt_scene* s, int64_t N);

// Timing events of one pass (path set `set`): [0, 1] around the pass, [2, 3]
// around the cache queries, [4, 5] around the tail kernel, then 2 per
// traversal launch.
pt_status ensure_events(pt_scene* s, int set, int nev) {
  while ((int)s->events[set].size() < nev) {
    hipEvent_t e;
    PT_HIP(hipEventCreate(&e));
    s->events[set].push_back(e);
  }
  return PT_OK;
}

// Accumulate a finished pass's timing events into the profiling totals.
pt_status read_pass_events(pt_scene* s, int set, int wavefront_bounces, int trace_launches, int max_depth,
                           bool queries) {
  hipEvent_t* ev = s->events[set].data();
  PT_HIP(hipEventSynchronize(ev[1]));
  float ms = 0.0f;
  PT_HIP(hipEventElapsedTime(&ms, ev[0], ev[1]));
  s->ms_total += ms;
  for (int i = 0; i < trace_launches; ++i) {
    PT_HIP(hipEventElapsedTime(&ms, ev[6 + 2 * i], ev[6 + 2 * i + 1]));
    s->ms_extend += ms;
    s->launches_extend++;
  }
  if (wavefront_bounces <= max_depth) {
    PT_HIP(hipEventElapsedTime(&ms, ev[4], ev[5]));
    s->ms_tail += ms;
    s->launches_tail++;
  }
  if (queries) {
    PT_HIP(hipEventElapsedTime(&ms, ev[2], ev[3]));
    s->ms_cache_query += ms;
  }
  return PT_OK;
}

// Run sampling passes over the tile (x0, y0, w, h) of the camera's image.
// With train (n == 1), the pass also carries the frame's training paths and
// the cache learns from them afterwards.  Without training, consecutive
// passes use the two path sets alternately: a pass's tail kernel and its
// accumulation run on the second stream while the next pass's dense bounces
// run on the scene's stream; the accumulations stay in pass order.
#ifndef PT_SHADE_SIDE
#define PT_SHADE_SIDE 1
#endif
// Side streams for the shading kernels of a pass (created once).
pt_status shade_streams(pt_scene* s, PassArgs& A) {
  if (!PT_SHADE_SIDE) return PT_OK;
  for (int k = 0; k < 2; ++k) {
    if (!s->shade_side[k]) PT_HIP(hipStreamCreateWithFlags(&s->shade_side[k], hipStreamNonBlocking));
    if (!s->shade_join[k]) PT_HIP(hipEventCreateWithFlags(&s->shade_join[k], hipEventDisableTiming));
    A.shade_side[k] = s->shade_side[k];
    A.shade_join[k] = s->shade_join[k];
  }
  if (!s->shade_fork) PT_HIP(hipEventCreateWithFlags(&s->shade_fork, hipEventDisableTiming));
  A.shade_fork = s->shade_fork;
  return PT_OK;
}

pt_status run_passes(pt_scene* s, const CamDev& C, int x0, int y0, int w, int h, int first, int n, int max_depth,
                     uint64_t seed, double* sum, float* per_sample, uint64_t* sigs, int spp_total,
                     bool train = false) {
  int64_t N = (int64_t)w * h;
  int64_t slots = N + (train ? s->nrc_cfg.train_paths : 0);
  const bool use_cache = s->nrc_on && s->nrc_ready;
  const bool tail = s->tail_fraction > 0.0 && s->tail_min_bounce <= max_depth;
  const bool overlap = !train && !use_cache && tail && n > 1;
  const int nsets = overlap ? 2 : 1;
  int grid = grid_for(slots), grid_trace = traversal_grid(slots);
  pt_status r = PT_OK;
  for (int set = 0; set < nsets; ++set) {
    if ((r = ensure_paths(s, slots, set))) return r;
    if ((r = ensure_counters(s, set))) return r;
    if ((r = ensure_spill(s, grid_trace, set))) return r;
  }
  if (!s->tail_counts) PT_HIP(hipHostMalloc((void**)&s->tail_counts, 2 * sizeof(uint32_t), hipHostMallocDefault));
  if (overlap) {
    if (!s->stream2) PT_HIP(hipStreamCreateWithFlags(&s->stream2, hipStreamNonBlocking));
    for (int k = 0; k < 2; ++k) {
      if (!s->ev_bulk[k]) PT_HIP(hipEventCreateWithFlags(&s->ev_bulk[k], hipEventDisableTiming));
      if (!s->ev_done[k]) PT_HIP(hipEventCreateWithFlags(&s->ev_done[k], hipEventDisableTiming));
    }
  }
  const int nev = 6 + 2 * (max_depth + 2);  // a pass makes at most max_depth + 2 traversal launches
  if (s->timing)
    for (int set = 0; set < nsets; ++set)
      if ((r = ensure_events(s, set, nev))) return r;
  int wavefront[2] = {max_depth + 1, max_depth + 1}, traces[2] = {0, 0};
  bool tail_on_2[2] = {false, false};
  int pending = -1;  // path set whose timing events are not read yet (overlap)
  for (int k = 0; k < n; ++k) {
    const int set = overlap ? (k & 1) : 0;
    SceneDev S = scene_dev(s, grid_trace, set);
    PathsDev P = paths_dev(s, N, x0, y0, w, set);
    if (train && (r = setup_training(s, C, P, N, (uint32_t)first, max_depth, seed))) return r;
    PassArgs A;
    std::memset(&A, 0, sizeof(A));
    A.sample = (uint32_t)(first + k);
    A.k0 = (uint32_t)seed;
    A.k1 = (uint32_t)(seed >> 32);
    A.max_depth = max_depth;
    A.grid = grid;
    A.grid_trace = grid_trace;
    A.grid_bin = bin_grid(slots);
    A.debug = per_sample != nullptr;
    A.count = s->counting;
    A.two_level = s->two_level;
    A.class_mask = s->class_mask | (1u << kClsMiss);
    A.nrc_bounce = -1;
    if (use_cache) {
      PathBufs& B = s->pb[set];
      if (N > B.nrc_q_cap) {
        PT_HIP(B.nrc_q.alloc((size_t)N * kNrcQueryFloats * sizeof(float)));
        PT_HIP(B.q_nrc.alloc((size_t)N * sizeof(uint32_t)));
        B.nrc_q_cap = N;
      }
      A.nrc_bounce = s->nrc_cfg.query_bounce;
      A.nrc_fwd = s->nrc_inf.as<uint4>();
      P.nrc_q = B.nrc_q.as<float>();
      P.q_nrc = B.q_nrc.as<uint32_t>();
    }
    if (tail) {
      A.tail_host_count = s->tail_counts + set;
      A.tail_min_bounce = s->tail_min_bounce;
      A.tail_fraction = s->tail_fraction;
    }
    A.wavefront_bounces = &wavefront[set];
    A.trace_launches = &traces[set];
    if ((r = shade_streams(s, A))) return r;
    tail_on_2[set] = false;
    if (overlap) {
      A.tail_stream = s->stream2;
      A.tail_ready = s->ev_bulk[set];
      A.tail_launched = &tail_on_2[set];
    }
    hipEvent_t* ev = s->timing ? s->events[set].data() : nullptr;
    if (ev) {
      A.ext_events = ev + 6;
      if (A.nrc_bounce >= 0) A.nrc_events = ev + 2;
      A.tail_events = ev + 4;
    }
    // the set's buffers are free once the pass that used them two passes ago has been accumulated
    if (overlap && k >= 2) PT_HIP(hipStreamWaitEvent(s->stream, s->ev_done[set], 0));
    if (ev) PT_HIP(hipEventRecord(ev[0], s->stream));
    PT_HIP(launch_pass(S, P, C, A, s->stream));
    hipStream_t acc = s->stream;
    if (overlap) {
      acc = s->stream2;
      if (!tail_on_2[set]) {  // the pass finished on the first stream: order the accumulation after it
        PT_HIP(hipEventRecord(s->ev_bulk[set], s->stream));
        PT_HIP(hipStreamWaitEvent(s->stream2, s->ev_bulk[set], 0));
      }
    }
    PT_HIP(launch_accumulate(P, sum, C.W, per_sample, sigs, spp_total, k, acc));
    if (ev) PT_HIP(hipEventRecord(ev[1], acc));
    if (overlap) PT_HIP(hipEventRecord(s->ev_done[set], s->stream2));
    if (ev) {
      if (overlap) {  // read the previous pass while this one runs
        if (pending >= 0 &&
            (r = read_pass_events(s, pending, wavefront[pending], traces[pending], max_depth, false)))
          return r;
        pending = set;
      } else if ((r = read_pass_events(s, set, wavefront[set], traces[set], max_depth, A.nrc_bounce >= 0))) {
        return r;
      }
    }
  }
  if (overlap) {  // the scene's stream sees every pass done
    PT_HIP(hipStreamWaitEvent(s->stream, s->ev_done[0], 0));
    PT_HIP(hipStreamWaitEvent(s->stream, s->ev_done[1], 0));
    if (pending >= 0 && (r = read_pass_events(s, pending, wavefront[pending], traces[pending], max_depth, false)))
      return r;
  }
  s->samples += (int64_t)n * N;
  if (train) {
    auto t0 = std::chrono::steady_clock::now();
    PathsDev P = paths_dev(s, N, x0, y0, w, 0);
    P.n = (int32_t)slots;
    P.n_render = (int32_t)N;
    P.rec = s->nrc_rec[0].as<float>();
    P.rec_depth = max_depth;
    if ((r = finish_training(s, P, nullptr, s->stream, true))) return r;
    if ((r = nrc_train_records(s, s->nrc_X.as<float>(), s->nrc_T.as<float>(), s->nrc_n.as<uint32_t>(),
                               (uint32_t)first, seed, nullptr, s->stream)))
      return r;
    if (s->timing) {
      PT_HIP(hipStreamSynchronize(s->stream));
      s->ms_cache_train += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    }
  }
  return PT_OK;
}

// Frames of the radiance cache once it has weights, pipelined over the two
// path sets.  A frame's sampling paths all end by the query vertex; its cache
// queries, its training paths' remaining vertices (tail kernel), its
// accumulation, the training targets and the frame's Adam steps run on the
// second stream while the next frame's dense bounces run on the scene's
// stream.  Each frame's cache queries come after the previous frame's Adam
// steps, so every frame sees the weights a frame-by-frame loop would.
pt_status run_cache_frames(pt_scene* s, const CamDev& C, int first, int n, int max_depth, uint64_t seed) {
  const int64_t N = (int64_t)C.W * C.H;
  const int64_t slots = N + s->nrc_cfg.train_paths;
  int grid = grid_for(slots), grid_trace = traversal_grid(slots);
  pt_status r = PT_OK;
  PathsDev Ps[2];
  for (int set = 0; set < 2; ++set) {  // every allocation before the first launch
    if ((r = ensure_paths(s, slots, set))) return r;
    if ((r = ensure_counters(s, set))) return r;
    if ((r = ensure_spill(s, grid_trace, set))) return r;
    PathBufs& B = s->pb[set];
    if (N > B.nrc_q_cap) {
      PT_HIP(B.nrc_q.alloc((size_t)N * kNrcQueryFloats * sizeof(float)));
      PT_HIP(B.q_nrc.alloc((size_t)N * sizeof(uint32_t)));
      B.nrc_q_cap = N;
    }
    Ps[set] = paths_dev(s, N, 0, 0, C.W, set);
    if ((r = setup_training(s, C, Ps[set], N, (uint32_t)first, max_depth, seed, set))) return r;
  }
  if ((r = nrc_ensure_ws(s, s->nrc_cfg.batch_size))) return r;
  if (!s->tail_counts) PT_HIP(hipHostMalloc((void**)&s->tail_counts, 2 * sizeof(uint32_t), hipHostMallocDefault));
  if (!s->stream2) PT_HIP(hipStreamCreateWithFlags(&s->stream2, hipStreamNonBlocking));
  for (int k = 0; k < 2; ++k) {
    if (!s->ev_bulk[k]) PT_HIP(hipEventCreateWithFlags(&s->ev_bulk[k], hipEventDisableTiming));
    if (!s->ev_done[k]) PT_HIP(hipEventCreateWithFlags(&s->ev_done[k], hipEventDisableTiming));
    for (int j = 0; j < 2; ++j)
      if (s->timing && !s->ev_train_t[k][j]) PT_HIP(hipEventCreate(&s->ev_train_t[k][j]));
  }
  if (!s->ev_train) PT_HIP(hipEventCreateWithFlags(&s->ev_train, hipEventDisableTiming));
  const int nev = 6 + 2 * (max_depth + 2);
  if (s->timing)
    for (int set = 0; set < 2; ++set)
      if ((r = ensure_events(s, set, nev))) return r;
  const bool tail = s->tail_fraction > 0.0 && s->tail_min_bounce <= max_depth;
  int wavefront[2] = {max_depth + 1, max_depth + 1}, traces[2] = {0, 0};
  bool tail_on_2[2] = {false, false};
  int pending = -1;  // path set whose timing events are not read yet
  auto read_training_time = [&](int set) -> pt_status {
    float ms = 0.0f;
    PT_HIP(hipEventSynchronize(s->ev_train_t[set][1]));
    PT_HIP(hipEventElapsedTime(&ms, s->ev_train_t[set][0], s->ev_train_t[set][1]));
    s->ms_cache_train += ms;
    return PT_OK;
  };
  for (int k = 0; k < n; ++k) {
    const int set = k & 1;
    const uint32_t frame = (uint32_t)(first + k);
    SceneDev S = scene_dev(s, grid_trace, set);
    PathsDev P = Ps[set];
    if ((r = setup_training(s, C, P, N, frame, max_depth, seed, set))) return r;  // no allocation now
    P.nrc_q = s->pb[set].nrc_q.as<float>();
    P.q_nrc = s->pb[set].q_nrc.as<uint32_t>();
    PassArgs A;
    std::memset(&A, 0, sizeof(A));
    A.sample = frame;
    A.k0 = (uint32_t)seed;
    A.k1 = (uint32_t)(seed >> 32);
    A.max_depth = max_depth;
    A.grid = grid;
    A.grid_trace = grid_trace;
    A.grid_bin = bin_grid(slots);
    A.count = s->counting;
    A.two_level = s->two_level;
    A.class_mask = s->class_mask | (1u << kClsMiss);
    A.nrc_bounce = s->nrc_cfg.query_bounce;
    A.nrc_fwd = s->nrc_inf.as<uint4>();
    A.query_wait = k > 0 ? s->ev_train : nullptr;  // the previous frame's Adam steps
    A.query_beside = true;
    if (tail) {
      A.tail_host_count = s->tail_counts + set;
      A.tail_min_bounce = s->tail_min_bounce;
      A.tail_fraction = s->tail_fraction;
      A.tail_bound = (uint32_t)s->nrc_cfg.train_paths;
    }
    A.wavefront_bounces = &wavefront[set];
    A.trace_launches = &traces[set];
    if ((r = shade_streams(s, A))) return r;
    tail_on_2[set] = false;
    A.tail_stream = s->stream2;
    A.tail_ready = s->ev_bulk[set];
    A.tail_launched = &tail_on_2[set];
    hipEvent_t* ev = s->timing ? s->events[set].data() : nullptr;
    if (ev) {
      A.ext_events = ev + 6;
      A.nrc_events = ev + 2;
      A.tail_events = ev + 4;
    }
    // the set's paths and records are free once the frame that used them two frames ago has trained
    if (k >= 2) PT_HIP(hipStreamWaitEvent(s->stream, s->ev_done[set], 0));
    if (ev) PT_HIP(hipEventRecord(ev[0], s->stream));
    PT_HIP(launch_pass(S, P, C, A, s->stream));
    if (!tail_on_2[set]) {
      // no hand-off (the tail is off, or max_depth ends the paths first): everything ran here
      PT_HIP(hipEventRecord(s->ev_bulk[set], s->stream));
      PT_HIP(hipStreamWaitEvent(s->stream2, s->ev_bulk[set], 0));
    }
    // accumulation, targets and training follow on the second stream, in frame order
    PT_HIP(launch_accumulate(P, s->sum.as<double>(), C.W, nullptr, nullptr, 1, 0, s->stream2));
    if (ev) PT_HIP(hipEventRecord(ev[1], s->stream2));
    if (s->timing) PT_HIP(hipEventRecord(s->ev_train_t[set][0], s->stream2));
    if ((r = finish_training(s, P, nullptr, s->stream2, true))) return r;
    if ((r = nrc_train_records(s, s->nrc_X.as<float>(), s->nrc_T.as<float>(), s->nrc_n.as<uint32_t>(), frame, seed,
                               nullptr, s->stream2)))
      return r;
    if (s->timing) PT_HIP(hipEventRecord(s->ev_train_t[set][1], s->stream2));
    PT_HIP(hipEventRecord(s->ev_train, s->stream2));
    PT_HIP(hipEventRecord(s->ev_done[set], s->stream2));
    if (s->timing) {  // read the previous frame while this one runs
      if (pending >= 0) {  // (the training's end event follows the tail kernel's on the second stream)
        if ((r = read_training_time(pending))) return r;
        if ((r = read_pass_events(s, pending, wavefront[pending], traces[pending], max_depth, true))) return r;
      }
      pending = set;
    }
  }
  // the scene's stream sees every frame's training done
  PT_HIP(hipStreamWaitEvent(s->stream, s->ev_done[0], 0));
  PT_HIP(hipStreamWaitEvent(s->stream, s->ev_done[1], 0));
  if (pending >= 0) {
    if ((r = read_training_time(pending))) return r;
    if ((r = read_pass_events(s, pending, wavefront[pending], traces[pending], max_depth, true))) return r;
  }
  s->samples += (int64_t)n * N;
  return PT_OK;
}

// ------------------------------------------------------------ radiance cache
// He-uniform initial weights: weight k of layer l is (2u - 1) sqrt(6 / 64),
// u the Philox uniform at counter (k, l, 0x4E5243, 0) under the key init_seed.
void nrc_init_weights(uint64_t seed, std::vector<float>& w) {
  w.assign(kNrcParams, 0.0f);
  const double scale = std::sqrt(6.0 / 64.0);
  int off = 0;
  for (int l = 0; l < 6; ++l) {
    int n = l < 5 ? 4096 : 3 * 64;
    for (int k = 0; k < n; ++k) {
      U4 r = philox((uint32_t)k, (uint32_t)l, 0x4E5243u, 0u, (uint32_t)seed, (uint32_t)(seed >> 32));
      double u = (double)(r.x >> 8) * (1.0 / 16777216.0);
      w[(size_t)(off + k)] = (float)((2.0 * u - 1.0) * scale);
    }
    off += n;
  }
}

// Split of one training step's weight-gradient GEMM over sample ranges.
void nrc_split(int64_t N, int& n_split, int64_t& npad) {
  n_split = (int)std::min<int64_t>(64, std::max<int64_t>(1, (N + 1023) / 1024));
  int64_t q = 32 * (int64_t)n_split;
  npad = (N + q - 1) / q * q;
}

// All three fragment sets from the weights and the inference weights.
hipError_t nrc_pack(pt_scene* s, uint32_t* t_step, const uint32_t* n_records, hipStream_t st) {
  return nrc_launch_pack(s->nrc_w.as<float>(), s->nrc_wi.as<float>(), s->nrc_fwd.as<uint4>(), s->nrc_bwd.as<uint4>(),
                         s->nrc_inf.as<uint4>(), t_step, n_records, st);
}

pt_status nrc_ensure_ws(pt_scene* s, int64_t N) {
  int split;
  int64_t npad;
  nrc_split(N, split, npad);
  if (npad > s->nrc_ws_npad) {
    size_t store = (size_t)6 * 64 * (size_t)npad * sizeof(uint16_t);
    PT_HIP(s->nrc_a.alloc(store));
    PT_HIP(s->nrc_g.alloc(store));
    PT_HIP(s->nrc_Xb.alloc((size_t)npad * 12 * sizeof(float)));
    PT_HIP(s->nrc_Tb.alloc((size_t)npad * 3 * sizeof(float)));
    s->nrc_ws_npad = npad;
  }
  if (split > s->nrc_ws_split) {
    PT_HIP(s->nrc_dw.alloc((size_t)split * kNrcParams * sizeof(float)));
    s->nrc_ws_split = split;
  }
  if (!s->nrc_loss.p) PT_HIP(s->nrc_loss.alloc(kNrcFbGrid * sizeof(float)));
  return PT_OK;
}

// One step on N samples X [N][12], T [N][3] (device): gradient into the
// partial buffers, then Adam (apply) or just the summed gradient (grad_out).
pt_status nrc_step(pt_scene* s, const float* X, const float* T, int64_t N, float* grad_out, bool apply,
                   int* grid_used, hipStream_t st, const uint32_t* n_records = nullptr) {
  pt_status r = nrc_ensure_ws(s, N);
  if (r) return r;
  int split;
  int64_t npad;
  nrc_split(N, split, npad);
  int64_t groups = npad / 16;
  int grid_fb = (int)std::min<int64_t>(kNrcFbGrid, (groups + 3) / 4);
  if (grid_used) *grid_used = grid_fb;
  PT_HIP(nrc_launch_train(X, T, (int)N, (int)npad, split, s->nrc_fwd.as<uint4>(), s->nrc_bwd.as<uint4>(),
                          s->nrc_a.as<uint16_t>(), s->nrc_g.as<uint16_t>(), s->nrc_loss.as<float>(), grid_fb,
                          s->nrc_dw.as<float>(), st));
  const pt_radiance_cache_config& c = s->nrc_cfg;
  PT_HIP(nrc_launch_adam(s->nrc_w.as<float>(), s->nrc_m.as<float>(), s->nrc_v.as<float>(), s->nrc_e.as<float>(),
                         s->nrc_wi.as<float>(), s->nrc_dw.as<float>(), split, grad_out, c.learning_rate, c.beta1,
                         c.beta2, c.epsilon, c.ema_decay, s->nrc_t.as<uint32_t>(), n_records, apply ? 1 : 0, st));
  if (apply) PT_HIP(nrc_pack(s, s->nrc_t.as<uint32_t>(), n_records, st));
  return PT_OK;
}

pt_status nrc_read_loss(pt_scene* s, int grid, int64_t N, double* loss, hipStream_t st) {
  std::vector<float> part((size_t)grid);
  PT_HIP(hipMemcpyAsync(part.data(), s->nrc_loss.p, (size_t)grid * sizeof(float), hipMemcpyDeviceToHost, st));
  PT_HIP(hipStreamSynchronize(st));
  double sum = 0.0;
  for (float v : part) sum += v;
  *loss = sum / (3.0 * (double)N);
  return PT_OK;
}

// Trace only the training paths of a frame (no sampling paths) and compact their records.
pt_status nrc_trace_training(pt_scene* s, const CamDev& C, uint32_t frame, int max_depth, uint64_t seed,
                             uint32_t* n_records) {
  const int64_t n = s->nrc_cfg.train_paths;
  pt_status r = ensure_paths(s, n);
  if (r) return r;
  if ((r = ensure_counters(s))) return r;
  int grid = grid_for(n), grid_trace = traversal_grid(n);
  if ((r = ensure_spill(s, grid_trace))) return r;
  SceneDev S = scene_dev(s, grid_trace);
  PathsDev P = paths_dev(s, 0, 0, 0, 1);
  if ((r = setup_training(s, C, P, 0, frame, max_depth, seed))) return r;
  PassArgs A;
  std::memset(&A, 0, sizeof(A));
  A.sample = frame;
  A.k0 = (uint32_t)seed;
  A.k1 = (uint32_t)(seed >> 32);
  A.max_depth = max_depth;
  A.grid = grid;
  A.grid_trace = grid_trace;
  A.grid_bin = bin_grid(n);
  A.two_level = s->two_level;
  A.class_mask = s->class_mask | (1u << kClsMiss);
  A.nrc_bounce = -1;
  PT_HIP(launch_pass(S, P, C, A, s->stream));
  return finish_training(s, P, n_records, s->stream);
}

// The frame's Adam steps on batches drawn with replacement from n records X_all, T_all.
// The frame's Adam steps on stream st, each on a batch drawn from the n_dev
// records (a device count: with none, the steps change nothing and are not
// counted).  mean_loss (host) waits for each step's loss.
pt_status nrc_train_records(pt_scene* s, const float* X_all, const float* T_all, const uint32_t* n_dev,
                            uint32_t frame, uint64_t seed, double* mean_loss, hipStream_t st) {
  const pt_radiance_cache_config& c = s->nrc_cfg;
  const int B = c.batch_size;
  pt_status r = nrc_ensure_ws(s, B);
  if (r) return r;
  double lsum = 0.0;
  for (int step = 0; step < c.steps_per_frame; ++step) {
    PT_HIP(nrc_launch_gather(X_all, T_all, n_dev, B, frame, step, (uint32_t)seed, (uint32_t)(seed >> 32),
                             s->nrc_Xb.as<float>(), s->nrc_Tb.as<float>(), st));
    int grid = 0;
    if ((r = nrc_step(s, s->nrc_Xb.as<float>(), s->nrc_Tb.as<float>(), B, nullptr, true, &grid, st, n_dev))) return r;
    if (mean_loss) {
      double l = 0.0;
      if ((r = nrc_read_loss(s, grid, B, &l, st))) return r;
      lsum += l;
    }
  }
  if (mean_loss) *mean_loss = c.steps_per_frame > 0 ? lsum / c.steps_per_frame : 0.0;
  if (c.steps_per_frame > 0) s->nrc_ready = true;
  return PT_OK;
}


// Sampling passes of the whole image into the FP64 sums; with the radiance
// cache on, every pass is one frame: render, then train on that frame.
pt_status render_samples(pt_scene* s, const CamDev& C, int first, int n, int max_depth, uint64_t seed) {
  if (!s->nrc_on)
    return run_passes(s, C, 0, 0, C.W, C.H, first, n, max_depth, seed, s->sum.as<double>(), nullptr, nullptr, n);
  int k = 0;
  // frames before the cache has weights (and with training off) run one by one
  for (; k < n && !(s->nrc_ready && s->nrc_cfg.steps_per_frame > 0 && max_depth > s->nrc_cfg.query_bounce); ++k) {
    pt_status r = run_passes(s, C, 0, 0, C.W, C.H, first + k, 1, max_depth, seed, s->sum.as<double>(), nullptr,
                             nullptr, 1, true);
    if (r) return r;
  }
  if (k < n) return run_cache_frames(s, C, first + k, n - k, max_depth, seed);
  return PT_OK;
}

pt_status check_render_args(int spp, int max_depth) {
  if (spp <= 0) return fail(PT_ERR_INVALID_ARG, "spp must be > 0");
  if (max_depth < 0 || max_depth > 64) return fail(PT_ERR_INVALID_ARG, "max_depth must be in [0, 64]");
  return PT_OK;
}

pt_status ensure_accum(pt_scene* s, int W, int H) {
  if (s->acc_w != W || s->acc_h != H || !s->sum.p) {
    PT_HIP(s->sum.alloc((size_t)W * H * 3 * sizeof(double)));
    PT_HIP(launch_zero_f64(s->sum.as<double>(), (int64_t)W * H * 3, s->stream));
    s->acc_w = W;
    s->acc_h = H;
    s->acc_samples = 0;
  }
  return PT_OK;
}

pt_status sync(pt_scene* s) {
  PT_HIP(hipStreamSynchronize(s->stream));
  PT_HIP(hipGetLastError());
  return PT_OK;
}

// sync(), then fail the call if a traversal ran out of stack since the last
// check: its walk dropped entries, so some closest hits or occlusion tests
// may be wrong.  One 8-byte read per call.
pt_status sync_traced(pt_scene* s) {
  pt_status r = sync(s);
  if (r || !s->stats.p) return r;
  unsigned long long v = 0;
  PT_HIP(hipMemcpyAsync(&v, s->stats.as<unsigned long long>() + kStatOverflow, sizeof(v), hipMemcpyDeviceToHost,
                        s->stream));
  PT_HIP(hipStreamSynchronize(s->stream));
  if (v > s->overflow_seen) {
    unsigned long long d = v - s->overflow_seen;
    s->overflow_seen = v;
    return fail(PT_ERR_DEVICE, "traversal stack overflow in %llu workgroups (capacity %d entries per lane)", d,
                stack_capacity(s->bvh_depth));
  }
  return PT_OK;
}

pt_status validate_material(const pt_openpbr_material& m, int i) {
  const float* f = reinterpret_cast<const float*>(&m);
  for (int k = 0; k < (int)(sizeof(pt_openpbr_material) / sizeof(float)); ++k) {
    if (!std::isfinite(f[k]) || f[k] < 0.0f) return fail(PT_ERR_INVALID_ARG, "material %d: parameter %d is negative or not finite", i, k);
  }
  const float unit[] = {m.base_weight, m.base_metalness, m.specular_weight, m.specular_roughness,
                        m.specular_roughness_anisotropy, m.transmission_weight, m.coat_weight, m.coat_roughness,
                        m.thin_film_weight, m.fuzz_weight, m.fuzz_roughness, m.subsurface_weight};
  for (float u : unit)
    if (u > 1.0f) return fail(PT_ERR_INVALID_ARG, "material %d: weights and roughness must be in [0, 1]", i);
  if (!(m.specular_ior > 0.0f) || !(m.coat_ior > 0.0f)) return fail(PT_ERR_INVALID_ARG, "material %d: IOR must be > 0", i);
  if (m.base_diffuse_roughness > 1.0f)
    return fail(PT_ERR_INVALID_ARG, "material %d: base_diffuse_roughness must be in [0, 1]", i);
  if (m.thin_film_ior < 1.0f) return fail(PT_ERR_INVALID_ARG, "material %d: thin_film_ior must be >= 1", i);
  if (m.coat_weight > 0.0f && m.transmission_weight > 0.0f)
    return fail(PT_ERR_UNSUPPORTED, "material %d: coat together with transmission is not supported", i);
  if (m.fuzz_weight > 0.0f && m.transmission_weight > 0.0f)
    return fail(PT_ERR_UNSUPPORTED, "material %d: fuzz together with transmission is not supported", i);
  return PT_OK;
}

MatRec make_matrec(const pt_openpbr_material& m) {
  MatRec r;
  std::memset(&r, 0, sizeof(r));
  for (int c = 0; c < 3; ++c) {
    r.base_color[c] = m.base_color[c];
    r.spec_color[c] = m.specular_color[c];
    r.trans_color[c] = m.transmission_color[c];
    r.coat_color[c] = m.coat_color[c];
    r.Le[c] = (float)((double)m.emission_luminance * m.emission_color[c]);
  }
  r.base_weight = m.base_weight;
  r.metalness = m.base_metalness;
  r.spec_weight = m.specular_weight;
  {  // specular_weight xi modulates the dielectric IOR: F0(eta') = xi F0(eta) (OpenPBR)
    const double eta = m.specular_ior, xi = m.specular_weight;
    double mod = eta;
    if (xi < 1.0) {
      const double r0 = (eta - 1.0) / (eta + 1.0), q = std::sqrt(xi * r0 * r0);
      mod = eta >= 1.0 ? (1.0 + q) / (1.0 - q) : (1.0 - q) / (1.0 + q);
    }
    r.spec_ior = (float)mod;
  }
  {  // EON diffuse roughness: FON's A and B (B = 0: Lambert)
    const double sg = m.base_diffuse_roughness;
    const double A = 1.0 / (1.0 + (0.5 - 2.0 / (3.0 * M_PI)) * sg);
    r.eon_a = (float)A;
    r.eon_b = (float)(sg * A);
  }
  r.fuzz_w = m.fuzz_weight;
  for (int c = 0; c < 3; ++c) r.fuzz_color[c] = m.fuzz_color[c];
  r.fuzz_a = (float)std::max((double)m.fuzz_roughness * m.fuzz_roughness, 1e-2);
  r.fuzz_E = nullptr;  // set by pt_upload_materials
  r.film_w = m.thin_film_weight;
  r.film_ior = m.thin_film_ior;
  r.film_d_nm = (float)(1000.0 * (double)m.thin_film_thickness);
  r.trans_weight = m.transmission_weight;
  r.coat_weight = m.coat_weight;
  r.coat_ior = m.coat_ior;
  r.bwbc_lum = (float)lumd((double)m.base_weight * m.base_color[0], (double)m.base_weight * m.base_color[1],
                           (double)m.base_weight * m.base_color[2]);
  {  // the diffuse lobe's albedo: glossy diffuse and the subsurface's local limit, mixed
    const double ws = m.subsurface_weight;
    double kd[3];
    for (int c = 0; c < 3; ++c) {
      kd[c] = (1.0 - ws) * ((double)m.base_weight * m.base_color[c]) + ws * (double)m.subsurface_color[c];
      r.kd[c] = (float)kd[c];
    }
    r.kd_lum = (float)lumd(kd[0], kd[1], kd[2]);
  }
  double rr = m.specular_roughness, a = m.specular_roughness_anisotropy;
  double alpha = rr * rr;
  double at = alpha * std::sqrt(2.0 / (1.0 + (1.0 - a) * (1.0 - a)));
  r.at = (float)std::max(at, 1e-4);
  r.ab = (float)std::max((1.0 - a) * at, 1e-4);
  r.ac = (float)std::max((double)m.coat_roughness * m.coat_roughness, 1e-4);
  uint32_t fl = 0;
  if (m.specular_roughness < 1e-3f) fl |= kMatSpecDelta;
  if (m.coat_roughness < 1e-3f) fl |= kMatCoatDelta;
  if (m.emission_luminance > 0.0f && lumd(m.emission_color[0], m.emission_color[1], m.emission_color[2]) > 0.0)
    fl |= kMatEmissive;
  r.flags = fl;
  // class: the smallest lobe set that contains every lobe the material can use
  bool hasC = m.coat_weight > 0.0f;
  bool hasM = m.base_metalness > 0.0f && m.specular_weight > 0.0f;
  bool hasI = m.base_metalness < 1.0f &&
              (m.specular_weight > 0.0f || m.transmission_weight > 0.0f || m.thin_film_weight > 0.0f);
  bool hasD = m.base_metalness < 1.0f && m.transmission_weight < 1.0f && r.kd_lum > 0.0f;
  bool hasT = m.base_metalness < 1.0f && m.transmission_weight > 0.0f;
  int cls;
  if (!hasC && !hasM && !hasI && !hasD) cls = kClsAbsorb;
  else if (!hasC && !hasM && !hasI) cls = kClsDiffuse;
  else if (!hasC && !hasI && !hasD) cls = kClsMetal;
  else if (m.thin_film_weight > 0.0f || m.fuzz_weight > 0.0f) cls = kClsGeneral;  // only it has films and fuzz
  else if (!hasM && !hasT) cls = kClsPlastic;
  else if (!hasC && !hasM) cls = kClsGlass;
  else cls = kClsGeneral;
  r.cls = cls;
  r.spec_rough = m.specular_roughness;
  {  // exact unpolarised dielectric reflectance at normal incidence, c = 1, of the modulated IOR
    double eta = r.spec_ior, c = 1.0;
    double g = std::sqrt(eta * eta - 1.0 + c * c);
    double a = (g - c) / (g + c), b = (c * (g + c) - 1.0) / (c * (g - c) + 1.0);
    r.f0_diel = (float)(0.5 * a * a * (1.0 + b * b));
  }
  return r;
}

// Append a mesh BVH to the shared node / triangle arrays, re-basing its refs.
uint32_t append_bvh(const Bvh4& b, std::vector<BVHNode>& nodes, std::vector<TriRec>& tris) {
  uint32_t node_off = (uint32_t)nodes.size(), tri_off = (uint32_t)tris.size();
  for (BVHNode n : b.nodes) {
    for (int c = 0; c < 4; ++c) {
      uint32_t r = n.child[c];
      if (r == kEmpty) continue;
      n.child[c] = ref_is_leaf(r) ? make_leaf(leaf_first(r) + tri_off, leaf_count(r)) : r + node_off;
    }
    nodes.push_back(n);
  }
  tris.insert(tris.end(), b.tris.begin(), b.tris.end());
  return node_off;
}

// Two-level hierarchy: one BVH4 per mesh in object space, a top-level BVH4 over
// instance world boxes (computed from the transformed vertices in double and
// widened), rigid inverses in double rounded to float.
struct TwoLevel {
  std::vector<BVHNode> nodes;
  std::vector<TriRec> tris;
  Bvh4 top;
  std::vector<uint32_t> items, tfirst, tcount;
  std::vector<InstRec> insts;
  std::vector<std::vector<float>> mverts;
  std::vector<std::vector<int32_t>> mmat;
  float tmin = 0.0f;
  int depth = 0;
  int32_t max_mat = -1;
  double box_lo[3], box_hi[3];
  int64_t mesh_nodes = 0;  // BVH4 nodes of all meshes
  double build_ms = 0.0;   // summed mesh builds
  int max_leaf = 0;
  double sah = 0.0;
};

// Builds one mesh's BVH4 into host memory: the host builder, or the device builder copied back.
using MeshBuilder = std::function<bool(const float*, const uint32_t*, const uint32_t*, int64_t, Bvh4&, std::string&)>;

pt_status build_two_level_host(const pt_mesh* meshes, int32_t n_meshes, const pt_instance* instances,
                               int32_t n_instances, TwoLevel& out, const MeshBuilder* builder = nullptr) {
  std::vector<std::vector<float>> mverts((size_t)n_meshes);
  std::vector<std::vector<int32_t>> mmat((size_t)n_meshes);
  std::vector<BVHNode> nodes;
  std::vector<TriRec> tris;
  std::vector<uint32_t> root((size_t)n_meshes), tfirst((size_t)n_meshes), tcount((size_t)n_meshes);
  int blas_depth = 0;
  for (int i = 0; i < n_meshes; ++i) {
    const pt_mesh& m = meshes[i];
    std::vector<float>& v = mverts[(size_t)i];
    v.resize((size_t)m.n_triangles * 9);
    mmat[(size_t)i].assign((size_t)m.n_triangles, 0);
    std::vector<uint32_t> prim((size_t)m.n_triangles), mat((size_t)m.n_triangles, 0u);
    for (int64_t t = 0; t < m.n_triangles; ++t) {
      for (int k = 0; k < 3; ++k) {
        int32_t vi = m.indices[3 * t + k];
        for (int c = 0; c < 3; ++c) v[9 * (size_t)t + 3 * k + c] = m.vertices[3 * (size_t)vi + c];
      }
      prim[(size_t)t] = (uint32_t)t;
      if (m.material_ids) {
        mmat[(size_t)i][(size_t)t] = m.material_ids[t];
        mat[(size_t)t] = (uint32_t)m.material_ids[t];
      }
    }
    Bvh4 b;
    std::string err;
    const bool ok = builder ? (*builder)(v.data(), prim.data(), mat.data(), m.n_triangles, b, err)
                            : build_bvh4(v.data(), prim.data(), mat.data(), m.n_triangles, b, err);
    if (!ok) return fail(builder ? PT_ERR_DEVICE : PT_ERR_INVALID_ARG, "mesh %d: %s", i, err.c_str());
    out.mesh_nodes += (int64_t)b.nodes.size();
    out.build_ms += b.build_ms;
    out.max_leaf = std::max(out.max_leaf, b.max_leaf);
    out.sah += b.sah_cost;
    tfirst[(size_t)i] = (uint32_t)tris.size();
    tcount[(size_t)i] = (uint32_t)m.n_triangles;
    root[(size_t)i] = append_bvh(b, nodes, tris);
    blas_depth = std::max(blas_depth, b.depth);
    if (tris.size() >= (size_t)kLeafFirstMask) return fail(PT_ERR_INVALID_ARG, "too many unique triangles");
  }
  std::vector<InstRec> insts((size_t)n_instances);
  std::vector<float> boxes((size_t)n_instances * 9);
  double slo[3] = {INFINITY, INFINITY, INFINITY}, shi[3] = {-INFINITY, -INFINITY, -INFINITY};
  int32_t max_mat = -1;
  for (int i = 0; i < n_instances; ++i) {
    const pt_instance& in = instances[i];
    InstRec& I = insts[(size_t)i];
    std::memset(&I, 0, sizeof(I));
    const float* M = in.object_to_world;
    double R[3][3], T[3];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) R[r][c] = M[4 * r + c];
      T[r] = M[4 * r + 3];
    }
    for (int k = 0; k < 12; ++k) I.o2w[k] = M[k];
    for (int r = 0; r < 3; ++r) {
      for (int c = 0; c < 3; ++c) I.w2o[4 * r + c] = (float)R[c][r];
      I.w2o[4 * r + 3] = (float)(-(R[0][r] * T[0] + R[1][r] * T[1] + R[2][r] * T[2]));
    }
    I.blas_root = root[(size_t)in.mesh];
    I.mat_override = in.material_override;
    I.light_map = -1;
    I.mesh = (uint32_t)in.mesh;
    if (in.material_override >= 0) {
      max_mat = std::max(max_mat, in.material_override);
    } else {
      for (int32_t id : mmat[(size_t)in.mesh]) max_mat = std::max(max_mat, id);
    }
    // world box of the transformed vertices
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    const std::vector<float>& v = mverts[(size_t)in.mesh];
    for (size_t q = 0; q < v.size(); q += 3) {
      double x = v[q], y = v[q + 1], z = v[q + 2];
      for (int r = 0; r < 3; ++r) {
        double w = R[r][0] * x + R[r][1] * y + R[r][2] * z + T[r];
        lo[r] = std::min(lo[r], w);
        hi[r] = std::max(hi[r], w);
      }
    }
    for (int r = 0; r < 3; ++r) {
      slo[r] = std::min(slo[r], lo[r]);
      shi[r] = std::max(shi[r], hi[r]);
      // widen: the triangle test runs on a single-precision object-space ray
      double pad = 1e-5 * (1.0 + std::fabs(lo[r]) + std::fabs(hi[r]) + (hi[r] - lo[r]));
      float l = (float)(lo[r] - pad), h = (float)(hi[r] + pad);
      boxes[9 * (size_t)i + r] = l;
      boxes[9 * (size_t)i + 3 + r] = h;
      boxes[9 * (size_t)i + 6 + r] = l;
    }
  }
  // top level over the instance boxes (a box is fed as the triangle (lo, hi, lo))
  std::vector<uint32_t> ids((size_t)n_instances), zero((size_t)n_instances, 0u);
  for (int i = 0; i < n_instances; ++i) ids[(size_t)i] = (uint32_t)i;
  Bvh4 top;
  std::string err;
  if (!build_bvh4(boxes.data(), ids.data(), zero.data(), n_instances, top, err))
    return fail(PT_ERR_INVALID_ARG, "top level: %s", err.c_str());
  std::vector<uint32_t> items((size_t)n_instances);
  for (int i = 0; i < n_instances; ++i) std::memcpy(&items[(size_t)i], &top.tris[(size_t)i].a.w, 4);
  double dx = shi[0] - slo[0], dy = shi[1] - slo[1], dz = shi[2] - slo[2];
  out.tmin = (float)(1e-5 * std::sqrt(dx * dx + dy * dy + dz * dz));
  for (int k = 0; k < 3; ++k) {
    out.box_lo[k] = slo[k];
    out.box_hi[k] = shi[k];
  }
  out.depth = top.depth + blas_depth;
  out.max_mat = max_mat;
  out.nodes.swap(nodes);
  out.tris.swap(tris);
  out.top = std::move(top);
  out.items.swap(items);
  out.tfirst.swap(tfirst);
  out.tcount.swap(tcount);
  out.insts.swap(insts);
  out.mverts.swap(mverts);
  out.mmat.swap(mmat);
  return PT_OK;
}

// Device build of one mesh, copied back to host memory (meshes of a two-level scene are
// concatenated and re-based on the host).  Times the soup upload, the build and the copy.
bool gpu_mesh_bvh(pt_scene* s, const float* v, const uint32_t* prim, const uint32_t* mat, int64_t n, Bvh4& b,
                  std::string& err) {
  auto t0 = std::chrono::steady_clock::now();
  DevBuf dsoup, dprim, dmat, dnodes, dtris;
  const int64_t nn = std::max<int64_t>(1, n - 1);
  hipError_t e = upload(dsoup, v, (size_t)n * 9 * sizeof(float), s->stream);
  if (e == hipSuccess) e = upload(dprim, prim, (size_t)n * sizeof(uint32_t), s->stream);
  if (e == hipSuccess) e = upload(dmat, mat, (size_t)n * sizeof(uint32_t), s->stream);
  if (e == hipSuccess) e = dnodes.alloc((size_t)nn * sizeof(BVHNode));
  if (e == hipSuccess) e = dtris.alloc((size_t)n * sizeof(TriRec));
  GpuBvhStats st{};
  if (e == hipSuccess)
    e = gpu_build_bvh4(dsoup.as<float>(), dprim.as<uint32_t>(), dmat.as<uint32_t>(), n, dnodes.as<BVHNode>(),
                       dtris.as<TriRec>(), s->stream, &st, s->gpu_bvh_builder);
  if (e == hipSuccess) {
    b.nodes.resize((size_t)st.n_nodes);
    b.tris.resize((size_t)n);
    e = hipMemcpyAsync(b.nodes.data(), dnodes.p, (size_t)st.n_nodes * sizeof(BVHNode), hipMemcpyDeviceToHost,
                       s->stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(b.tris.data(), dtris.p, (size_t)n * sizeof(TriRec), hipMemcpyDeviceToHost, s->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(s->stream);
  }
  if (e != hipSuccess) {
    err = std::string("device BVH build failed: ") + hipGetErrorString(e);
    return false;
  }
  b.depth = st.depth;
  b.max_leaf = st.max_leaf;
  b.sah_cost = 0.0;
  b.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return true;
}

pt_status build_two_level(pt_scene* s, const pt_mesh* meshes, int32_t n_meshes, const pt_instance* instances,
                          int32_t n_instances, bool on_device = false) {
  TwoLevel T;
  pt_status r = set_device(s);
  if (r) return r;
  MeshBuilder gpu = [s](const float* v, const uint32_t* prim, const uint32_t* mat, int64_t n, Bvh4& b,
                        std::string& err) { return gpu_mesh_bvh(s, v, prim, mat, n, b, err); };
  r = build_two_level_host(meshes, n_meshes, instances, n_instances, T, on_device ? &gpu : nullptr);
  if (r) return r;
  PT_HIP(upload(s->nodes, T.nodes.data(), T.nodes.size() * sizeof(BVHNode), s->stream));
  PT_HIP(upload(s->tris, T.tris.data(), T.tris.size() * sizeof(TriRec), s->stream));
  PT_HIP(upload(s->tlas, T.top.nodes.data(), T.top.nodes.size() * sizeof(BVHNode), s->stream));
  PT_HIP(upload(s->tlas_items, T.items.data(), T.items.size() * sizeof(uint32_t), s->stream));
  PT_HIP(upload(s->insts, T.insts.data(), T.insts.size() * sizeof(InstRec), s->stream));
  PT_HIP(upload(s->mesh_tri_first, T.tfirst.data(), T.tfirst.size() * sizeof(uint32_t), s->stream));
  PT_HIP(upload(s->mesh_tri_count, T.tcount.data(), T.tcount.size() * sizeof(uint32_t), s->stream));
  PT_HIP(hipStreamSynchronize(s->stream));
  s->tmin = T.tmin;
  set_box(s, T.box_lo, T.box_hi);
  s->n_tris = (uint32_t)T.tris.size();
  s->bvh_depth = T.depth;
  s->n_nodes = T.mesh_nodes;
  s->bvh_max_leaf = T.max_leaf;
  s->bvh_sah = T.sah;
  s->bvh_build_ms = T.build_ms;
  s->bvh_on_device = on_device;
  s->max_mat_id = T.max_mat;
  s->host_tri_verts.clear();
  s->host_tri_mat.clear();
  s->host_insts.swap(T.insts);
  s->host_mesh_verts.swap(T.mverts);
  s->host_mesh_mat.swap(T.mmat);
  s->two_level = true;
  s->has_bvh = true;
  s->lights_dirty = true;
  return PT_OK;
}

// Validation shared by the host and device builds (checked before any state change).
pt_status check_build_args(const pt_mesh* meshes, int32_t n_meshes, const pt_instance* instances,
                           int32_t n_instances, int64_t* total_out) {
  if (!meshes || n_meshes <= 0) return fail(PT_ERR_INVALID_ARG, "meshes must be non-NULL with n_meshes > 0");
  if (n_instances < 0 || (n_instances > 0 && !instances)) return fail(PT_ERR_INVALID_ARG, "bad instances");
  for (int i = 0; i < n_instances; ++i) {
    const pt_instance& in = instances[i];
    if (in.mesh < 0 || in.mesh >= n_meshes) return fail(PT_ERR_INVALID_ARG, "instance %d: mesh %d out of range", i, in.mesh);
    if (!finite_all(in.object_to_world, 12)) return fail(PT_ERR_INVALID_ARG, "instance %d: non-finite transform", i);
    if (in.material_override < -1) return fail(PT_ERR_INVALID_ARG, "instance %d: bad material override", i);
    if (in.material_override < 0 && !meshes[in.mesh].material_ids)
      return fail(PT_ERR_INVALID_ARG, "instance %d: mesh %d has no material ids and no override", i, in.mesh);
  }
  int64_t total = 0;
  for (int i = 0; i < n_meshes; ++i) {
    const pt_mesh& m = meshes[i];
    if (!m.vertices || !m.indices || m.n_vertices <= 0 || m.n_triangles <= 0)
      return fail(PT_ERR_INVALID_ARG, "mesh %d: NULL arrays or empty counts", i);
    if (!m.material_ids && n_instances == 0)
      return fail(PT_ERR_INVALID_ARG, "mesh %d: material_ids is NULL and nothing overrides it", i);
    if (!finite_all(m.vertices, (size_t)m.n_vertices * 3)) return fail(PT_ERR_INVALID_ARG, "mesh %d: non-finite vertex", i);
    for (int64_t t = 0; t < m.n_triangles * 3; ++t)
      if (m.indices[t] < 0 || m.indices[t] >= m.n_vertices)
        return fail(PT_ERR_INVALID_ARG, "mesh %d: index %lld out of range", i, (long long)m.indices[t]);
    if (m.material_ids)
      for (int64_t t = 0; t < m.n_triangles; ++t)
        if (m.material_ids[t] < 0) return fail(PT_ERR_INVALID_ARG, "mesh %d: negative material id", i);
    total += m.n_triangles;
  }
  if (n_instances == 0 && total >= (int64_t)kLeafFirstMask) return fail(PT_ERR_INVALID_ARG, "too many triangles");
  *total_out = total;
  return PT_OK;
}

// pt_build_bvh (on_device false: host binned-SAH builder) and pt_build_bvh_gpu (device linear BVH).
pt_status build_bvh_any(pt_scene* s, const pt_mesh* meshes, int32_t n_meshes, const pt_instance* instances,
                        int32_t n_instances, bool on_device) {
  pt_status r = check_scene(s);
  if (r) return r;
  int64_t total = 0;
  if ((r = check_build_args(meshes, n_meshes, instances, n_instances, &total))) return r;
  if (n_instances > 0) return build_two_level(s, meshes, n_meshes, instances, n_instances, on_device);
  std::vector<float> verts((size_t)total * 9);
  std::vector<int32_t> mat((size_t)total);
  std::vector<uint32_t> prim((size_t)total), matu((size_t)total);
  int64_t t = 0;
  int32_t max_mat = -1;
  for (int i = 0; i < n_meshes; ++i) {
    const pt_mesh& m = meshes[i];
    for (int64_t k = 0; k < m.n_triangles; ++k, ++t) {
      for (int v = 0; v < 3; ++v) {
        int32_t vi = m.indices[3 * k + v];
        for (int c = 0; c < 3; ++c) verts[9 * (size_t)t + 3 * v + c] = m.vertices[3 * (size_t)vi + c];
      }
      mat[(size_t)t] = m.material_ids[k];
      matu[(size_t)t] = (uint32_t)m.material_ids[k];
      prim[(size_t)t] = (uint32_t)t;
      max_mat = std::max(max_mat, m.material_ids[k]);
    }
  }
  r = set_device(s);
  if (r) return r;
  int64_t n_nodes = 0;
  int depth = 0, max_leaf = 0;
  double sah = 0.0, build_ms = 0.0;
  if (on_device) {
    // the soup goes up once; nodes and triangle records are written in place
    auto t0 = std::chrono::steady_clock::now();
    DevBuf dsoup, dprim, dmat;
    PT_HIP(upload(dsoup, verts.data(), verts.size() * sizeof(float), s->stream));
    PT_HIP(upload(dprim, prim.data(), prim.size() * sizeof(uint32_t), s->stream));
    PT_HIP(upload(dmat, matu.data(), matu.size() * sizeof(uint32_t), s->stream));
    PT_HIP(s->nodes.alloc((size_t)std::max<int64_t>(1, total - 1) * sizeof(BVHNode)));
    PT_HIP(s->tris.alloc((size_t)total * sizeof(TriRec)));
    GpuBvhStats st{};
    hipError_t e = gpu_build_bvh4(dsoup.as<float>(), dprim.as<uint32_t>(), dmat.as<uint32_t>(), total,
                                  s->nodes.as<BVHNode>(), s->tris.as<TriRec>(), s->stream, &st, s->gpu_bvh_builder);
    if (e != hipSuccess) {
      s->has_bvh = false;  // the scene's buffers were overwritten
      return fail(PT_ERR_DEVICE, "device BVH build failed: %s", hipGetErrorString(e));
    }
    n_nodes = st.n_nodes;
    depth = st.depth;
    max_leaf = st.max_leaf;
    build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  } else {
    Bvh4 bvh;
    std::string err;
    if (!build_bvh4(verts.data(), prim.data(), matu.data(), total, bvh, err)) return fail(PT_ERR_INVALID_ARG, "%s", err.c_str());
    PT_HIP(upload(s->nodes, bvh.nodes.data(), bvh.nodes.size() * sizeof(BVHNode), s->stream));
    PT_HIP(upload(s->tris, bvh.tris.data(), bvh.tris.size() * sizeof(TriRec), s->stream));
    PT_HIP(hipStreamSynchronize(s->stream));
    n_nodes = (int64_t)bvh.nodes.size();
    depth = bvh.depth;
    max_leaf = bvh.max_leaf;
    sah = bvh.sah_cost;
    build_ms = bvh.build_ms;
  }
  double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (size_t q = 0; q < verts.size(); q += 3)
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], (double)verts[q + k]);
      hi[k] = std::max(hi[k], (double)verts[q + k]);
    }
  // t_min from the float box of the triangles (as the host builder reports it)
  double dx = (double)(float)hi[0] - (float)lo[0], dy = (double)(float)hi[1] - (float)lo[1],
         dz = (double)(float)hi[2] - (float)lo[2];
  s->tmin = (float)(1e-5 * std::sqrt(dx * dx + dy * dy + dz * dz));
  set_box(s, lo, hi);
  s->n_tris = (uint32_t)total;
  s->bvh_depth = depth;
  s->n_nodes = n_nodes;
  s->bvh_max_leaf = max_leaf;
  s->bvh_sah = sah;
  s->bvh_build_ms = build_ms;
  s->bvh_on_device = on_device;
  s->max_mat_id = max_mat;
  s->host_tri_verts.swap(verts);
  s->host_tri_mat.swap(mat);
  s->host_insts.clear();
  s->host_mesh_verts.clear();
  s->host_mesh_mat.clear();
  s->two_level = false;
  s->has_bvh = true;
  s->lights_dirty = true;
  return PT_OK;
}

}  // namespace

// =============================================================== C ABI ====
extern "C" {

const char* pt_last_error(void) { return g_err.c_str(); }

const char* pt_version(void) { return "pt 0.1 (gfx950 wavefront path tracer)"; }

pt_status pt_scene_create(int32_t hip_device, void* hip_stream, pt_scene** out) {
  if (!out) return fail(PT_ERR_INVALID_ARG, "out is NULL");
  *out = nullptr;
  int n = 0;
  hipError_t e = hipGetDeviceCount(&n);
  if (e != hipSuccess) return fail(PT_ERR_DEVICE, "hipGetDeviceCount failed: %s", hipGetErrorString(e));
  if (hip_device < 0 || hip_device >= n) return fail(PT_ERR_INVALID_ARG, "device %d out of range [0, %d)", hip_device, n);
  std::unique_ptr<pt_scene> s(new (std::nothrow) pt_scene());
  if (!s) return fail(PT_ERR_OUT_OF_MEMORY, "out of host memory");
  s->device = hip_device;
  s->stream = static_cast<hipStream_t>(hip_stream);
  pt_status r = set_device(s.get());
  if (r) return r;
  // set-up of the allocation-free call: this device's scratch address, looked up once per device
  unsigned char* scratch_dev = nullptr;
  e = noalloc_scratch(hip_device, &scratch_dev);
  if (e != hipSuccess)
    return fail(PT_ERR_DEVICE, "hipGetSymbolAddress of the scratch array failed: %s", hipGetErrorString(e));
  *out = s.release();
  return PT_OK;
}

void pt_scene_destroy(pt_scene* s) {
  if (!s) return;
  (void)hipSetDevice(s->device);
  (void)hipStreamSynchronize(s->stream);
  if (s->stream2) (void)hipStreamSynchronize(s->stream2);
  for (auto& v : s->events)
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
  for (int k = 0; k < 2; ++k) {
    if (s->ev_bulk[k]) (void)hipEventDestroy(s->ev_bulk[k]);
    if (s->ev_display[k]) (void)hipEventDestroy(s->ev_display[k]);
    if (s->ev_forward[k]) (void)hipEventDestroy(s->ev_forward[k]);
    if (s->ev_done[k]) (void)hipEventDestroy(s->ev_done[k]);
    for (int j = 0; j < 2; ++j)
      if (s->ev_train_t[k][j]) (void)hipEventDestroy(s->ev_train_t[k][j]);
  }
  if (s->ev_train) (void)hipEventDestroy(s->ev_train);
  for (int k = 0; k < 2; ++k) {
    if (s->shade_side[k]) (void)hipStreamSynchronize(s->shade_side[k]);
    if (s->shade_join[k]) (void)hipEventDestroy(s->shade_join[k]);
    if (s->shade_side[k]) (void)hipStreamDestroy(s->shade_side[k]);
  }
  if (s->shade_fork) (void)hipEventDestroy(s->shade_fork);
  if (s->stream2) (void)hipStreamDestroy(s->stream2);
  if (s->tail_counts) (void)hipHostFree(s->tail_counts);
  delete s;
}

pt_status pt_build_bvh(pt_scene* s, const pt_mesh* meshes, int32_t n_meshes, const pt_instance* instances,
                       int32_t n_instances) {
  return build_bvh_any(s, meshes, n_meshes, instances, n_instances, false);
}

pt_status pt_build_bvh_gpu(pt_scene* s, const pt_mesh* meshes, int32_t n_meshes, const pt_instance* instances,
                           int32_t n_instances) {
  return build_bvh_any(s, meshes, n_meshes, instances, n_instances, true);
}

pt_status pt_scene_bvh_info(pt_scene* s, pt_bvh_info* info) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!info) return fail(PT_ERR_INVALID_ARG, "info is NULL");
  if (!s->has_bvh) return fail(PT_ERR_STATE, "pt_build_bvh has not been called");
  info->n_nodes = s->n_nodes;
  info->n_tris = s->n_tris;
  info->depth = s->bvh_depth;
  info->max_leaf_tris = s->bvh_max_leaf;
  info->sah_cost = s->bvh_sah;
  info->build_ms = s->bvh_build_ms;
  info->stack_capacity = stack_capacity(s->bvh_depth);
  return PT_OK;
}

pt_status pt_scene_copy_bvh(pt_scene* s, void* nodes, void* tris) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!s->has_bvh) return fail(PT_ERR_STATE, "pt_build_bvh has not been called");
  if ((r = set_device(s))) return r;
  if (nodes)
    PT_HIP(hipMemcpyAsync(nodes, s->nodes.p, (size_t)s->n_nodes * sizeof(BVHNode), hipMemcpyDeviceToHost, s->stream));
  if (tris) PT_HIP(hipMemcpyAsync(tris, s->tris.p, (size_t)s->n_tris * sizeof(TriRec), hipMemcpyDeviceToHost, s->stream));
  return sync(s);
}

// Directional albedo of the fuzz lobe (weight 1, colour 1) at mu = k/64,
// k = 0..64: the midpoint rule over mu_i in [0, 1] and phi in [0, 2 pi) with
// 256 x 256 cells of D V mu_i, wo = (sqrt(1 - mu^2), 0, mu).
static void fuzz_albedo_table(double a, float* out) {
  const int N = 256, Np = 256;
  for (int k = 0; k <= 64; ++k) {
    const double mu = k / 64.0, so = std::sqrt(1.0 - mu * mu);
    double acc = 0.0;
    for (int i = 0; i < N; ++i) {
      const double mi = (i + 0.5) / N, si = std::sqrt(1.0 - mi * mi);
      const double V = 1.0 / (4.0 * (mi + mu - mi * mu));
      for (int j = 0; j < Np; ++j) {
        const double ph = 2.0 * M_PI * (j + 0.5) / Np;
        const double hx = si * std::cos(ph) + so, hy = si * std::sin(ph), hz = mi + mu;
        const double hl = std::sqrt(hx * hx + hy * hy + hz * hz);
        const double c = hz / hl;
        const double sn = std::sqrt(std::max(0.0, 1.0 - c * c));
        acc += (2.0 + 1.0 / a) * std::pow(sn, 1.0 / a) / (2.0 * M_PI) * V * mi;
      }
    }
    out[k] = (float)(acc * (1.0 / N) * (2.0 * M_PI / Np));
  }
}

pt_status pt_upload_materials(pt_scene* s, const pt_openpbr_material* m, int32_t n) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!m || n <= 0) return fail(PT_ERR_INVALID_ARG, "materials must be non-NULL with n > 0");
  std::vector<MatRec> recs((size_t)n);
  uint32_t mask = 0;
  for (int i = 0; i < n; ++i) {
    r = validate_material(m[i], i);
    if (r) return r;
    recs[(size_t)i] = make_matrec(m[i]);
    mask |= 1u << recs[(size_t)i].cls;
  }
  r = set_device(s);
  if (r) return r;
  // fuzz albedo tables, one per distinct sheen alpha, 65 floats each
  std::vector<float> fuzz;
  std::vector<float> alphas;
  std::vector<int> tab_of((size_t)n, -1);
  for (int i = 0; i < n; ++i) {
    if (!(recs[(size_t)i].fuzz_w > 0.0f)) continue;
    const float a = recs[(size_t)i].fuzz_a;
    int t = -1;
    for (size_t q = 0; q < alphas.size(); ++q)
      if (alphas[q] == a) t = (int)q;
    if (t < 0) {
      t = (int)alphas.size();
      alphas.push_back(a);
      fuzz.resize(fuzz.size() + 65);
      fuzz_albedo_table((double)a, fuzz.data() + 65 * (size_t)t);
    }
    tab_of[(size_t)i] = t;
  }
  if (!fuzz.empty()) {
    PT_HIP(upload(s->fuzz_tabs, fuzz.data(), fuzz.size() * sizeof(float), s->stream));
    for (int i = 0; i < n; ++i)
      if (tab_of[(size_t)i] >= 0) recs[(size_t)i].fuzz_E = s->fuzz_tabs.as<float>() + 65 * (size_t)tab_of[(size_t)i];
  }
  PT_HIP(upload(s->mats, recs.data(), recs.size() * sizeof(MatRec), s->stream));
  PT_HIP(hipStreamSynchronize(s->stream));
  s->host_mats.assign(m, m + n);
  s->class_mask = mask;
  s->has_mats = true;
  s->lights_dirty = true;
  return PT_OK;
}

pt_status pt_set_environment(pt_scene* s, const float* rgb, int32_t w, int32_t h) {
  pt_status r = check_scene(s);
  if (r) return r;
  r = set_device(s);
  if (r) return r;
  if (!rgb) {
    s->env_w = s->env_h = 0;
    s->lights_dirty = true;
    return PT_OK;
  }
  if (w <= 0 || h <= 0) return fail(PT_ERR_INVALID_ARG, "environment size must be > 0");
  size_t n = (size_t)w * h;
  for (size_t i = 0; i < 3 * n; ++i)
    if (!std::isfinite(rgb[i]) || rgb[i] < 0.0f) return fail(PT_ERR_INVALID_ARG, "environment texel %zu is negative or not finite", i / 3);
  // piecewise-constant sampling tables: texel weight lum * sin(theta at the row centre)
  std::vector<float4> tex(n);
  std::vector<double> colw(n);
  std::vector<double> roww((size_t)h);
  double total = 0.0;
  for (int y = 0; y < h; ++y) {
    double st = std::sin(M_PI * (y + 0.5) / h);
    double rs = 0.0;
    for (int x = 0; x < w; ++x) {
      size_t i = (size_t)y * w + x;
      tex[i] = make_float4(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2], 0.0f);
      double wt = lumd(rgb[3 * i], rgb[3 * i + 1], rgb[3 * i + 2]) * st;
      colw[i] = wt;
      rs += wt;
    }
    roww[(size_t)y] = rs;
    total += rs;
  }
  if (!(total > 0.0)) {  // a black environment is the same as none
    s->env_w = s->env_h = 0;
    s->lights_dirty = true;
    return PT_OK;
  }
  std::vector<float> col_pmf(n), col_cdf((size_t)h * (w + 1)), row_pmf((size_t)h), row_cdf((size_t)h + 1);
  for (int y = 0; y < h; ++y) {
    double rs = roww[(size_t)y];
    double acc = 0.0;
    float* cdf = &col_cdf[(size_t)y * (w + 1)];
    cdf[0] = 0.0f;
    for (int x = 0; x < w; ++x) {
      size_t i = (size_t)y * w + x;
      acc += colw[i];
      col_pmf[i] = rs > 0.0 ? (float)(colw[i] / rs) : 0.0f;
      cdf[x + 1] = rs > 0.0 ? (float)(acc / rs) : 0.0f;
    }
    if (rs > 0.0) cdf[w] = 1.0f;
  }
  double acc = 0.0;
  row_cdf[0] = 0.0f;
  for (int y = 0; y < h; ++y) {
    row_pmf[(size_t)y] = (float)(roww[(size_t)y] / total);
    acc += roww[(size_t)y];
    row_cdf[(size_t)y + 1] = (float)(acc / total);
  }
  row_cdf[(size_t)h] = 1.0f;
  // guide tables: entry g = largest i < n with cdf[i] <= g / G
  auto guide = [](const float* cdf, int nb, int G, int32_t* out) {
    int i = 0;
    for (int g = 0; g < G; ++g) {
      float t = (float)g / (float)G;
      while (i + 1 < nb && cdf[i + 1] <= t) ++i;
      out[g] = i;
    }
  };
  std::vector<int32_t> row_guide(kEnvRowGuide), col_guide((size_t)h * kEnvColGuide);
  guide(row_cdf.data(), h, kEnvRowGuide, row_guide.data());
  for (int y = 0; y < h; ++y)
    guide(&col_cdf[(size_t)y * (w + 1)], w, kEnvColGuide, &col_guide[(size_t)y * kEnvColGuide]);
  PT_HIP(upload(s->env_row_guide, row_guide.data(), row_guide.size() * sizeof(int32_t), s->stream));
  PT_HIP(upload(s->env_col_guide, col_guide.data(), col_guide.size() * sizeof(int32_t), s->stream));
  PT_HIP(upload(s->env, tex.data(), n * sizeof(float4), s->stream));
  PT_HIP(upload(s->env_col_pmf, col_pmf.data(), n * sizeof(float), s->stream));
  PT_HIP(upload(s->env_col_cdf, col_cdf.data(), col_cdf.size() * sizeof(float), s->stream));
  PT_HIP(upload(s->env_row_pmf, row_pmf.data(), row_pmf.size() * sizeof(float), s->stream));
  PT_HIP(upload(s->env_row_cdf, row_cdf.data(), row_cdf.size() * sizeof(float), s->stream));
  PT_HIP(hipStreamSynchronize(s->stream));
  s->env_w = w;
  s->env_h = h;
  s->lights_dirty = true;
  return PT_OK;
}

pt_status pt_reset_accumulation(pt_scene* s) {
  pt_status r = check_scene(s);
  if (r) return r;
  r = set_device(s);
  if (r) return r;
  if (s->sum.p) PT_HIP(launch_zero_f64(s->sum.as<double>(), (int64_t)s->acc_w * s->acc_h * 3, s->stream));
  s->acc_samples = 0;
  return sync(s);
}

pt_status pt_accumulate(pt_scene* s, const pt_camera* cam, int32_t first, int32_t n, int32_t max_depth,
                        uint64_t seed) {
  pt_status r = check_scene(s);
  if (r) return r;
  CamDev C;
  if ((r = make_camera(cam, C))) return r;
  if ((r = check_render_args(n, max_depth))) return r;
  if (first < 0) return fail(PT_ERR_INVALID_ARG, "first_sample must be >= 0");
  if ((r = set_device(s))) return r;
  if ((r = ready_to_render(s))) return r;
  if ((r = ensure_accum(s, C.W, C.H))) return r;
  if ((r = render_samples(s, C, first, n, max_depth, seed))) return r;
  s->acc_samples += n;
  return sync_traced(s);
}

pt_status pt_resolve(pt_scene* s, float* out, double* out_sum) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!out) return fail(PT_ERR_INVALID_ARG, "out_rgb32f is NULL");
  if (s->acc_samples <= 0) return fail(PT_ERR_STATE, "nothing accumulated");
  if ((r = set_device(s))) return r;
  int64_t nv = (int64_t)s->acc_w * s->acc_h * 3;
  PT_HIP(launch_resolve(s->sum.as<double>(), out, nv, 1.0 / (double)s->acc_samples, s->stream));
  if (out_sum) PT_HIP(hipMemcpyAsync(out_sum, s->sum.p, (size_t)nv * sizeof(double), hipMemcpyDeviceToDevice, s->stream));
  return sync(s);
}

pt_status pt_set_accumulation(pt_scene* s, const double* sum, int32_t width, int32_t height, int64_t samples) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!sum) return fail(PT_ERR_INVALID_ARG, "sum is NULL");
  if (width <= 0 || height <= 0) return fail(PT_ERR_INVALID_ARG, "width and height must be > 0");
  if (samples <= 0) return fail(PT_ERR_INVALID_ARG, "samples must be > 0");
  if ((r = set_device(s))) return r;
  if ((r = ensure_accum(s, width, height))) return r;
  PT_HIP(hipMemcpyAsync(s->sum.p, sum, (size_t)width * height * 3 * sizeof(double), hipMemcpyDeviceToDevice,
                        s->stream));
  s->acc_samples = samples;
  return sync(s);
}

pt_status pt_display(pt_scene* s, double exposure, uint32_t* out_rgba8, float* out_encoded) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!out_rgba8 && !out_encoded) return fail(PT_ERR_INVALID_ARG, "out_rgba8 and out_encoded are both NULL");
  if (!(exposure >= 0.0) || !std::isfinite(exposure)) return fail(PT_ERR_INVALID_ARG, "exposure must be finite and >= 0");
  if (s->acc_samples <= 0) return fail(PT_ERR_STATE, "nothing accumulated");
  if ((r = set_device(s))) return r;
  const int64_t np = (int64_t)s->acc_w * s->acc_h;
  if (s->timing) {
    for (hipEvent_t& e : s->ev_display)
      if (!e) PT_HIP(hipEventCreate(&e));
    PT_HIP(hipEventRecord(s->ev_display[0], s->stream));
  }
  PT_HIP(launch_display(s->sum.as<double>(), np, 1.0 / (double)s->acc_samples, exposure, out_rgba8, out_encoded,
                        s->stream));
  if (s->timing) PT_HIP(hipEventRecord(s->ev_display[1], s->stream));
  if ((r = sync(s))) return r;
  if (s->timing) {
    float ms = 0.0f;
    PT_HIP(hipEventElapsedTime(&ms, s->ev_display[0], s->ev_display[1]));
    s->ms_display += ms;
    s->launches_display += 1;
  }
  return PT_OK;
}

pt_status pt_render(pt_scene* s, const pt_camera* cam, int32_t spp, int32_t max_depth, uint64_t seed, float* out) {
  pt_status r = check_scene(s);
  if (r) return r;
  CamDev C;
  if ((r = make_camera(cam, C))) return r;
  if ((r = check_render_args(spp, max_depth))) return r;
  if (!out) return fail(PT_ERR_INVALID_ARG, "out_rgb32f is NULL");
  if ((r = set_device(s))) return r;
  if ((r = ready_to_render(s))) return r;
  if ((r = ensure_accum(s, C.W, C.H))) return r;
  PT_HIP(launch_zero_f64(s->sum.as<double>(), (int64_t)C.W * C.H * 3, s->stream));
  s->acc_samples = 0;
  if ((r = render_samples(s, C, 0, spp, max_depth, seed))) return r;
  s->acc_samples = spp;
  PT_HIP(launch_resolve(s->sum.as<double>(), out, (int64_t)C.W * C.H * 3, 1.0 / (double)spp, s->stream));
  return sync_traced(s);
}

pt_status pt_render_debug(pt_scene* s, const pt_camera* cam, int32_t x0, int32_t y0, int32_t w, int32_t h,
                          int32_t first, int32_t spp, int32_t max_depth, uint64_t seed, float* per_sample,
                          uint64_t* sig) {
  pt_status r = check_scene(s);
  if (r) return r;
  CamDev C;
  if ((r = make_camera(cam, C))) return r;
  if ((r = check_render_args(spp, max_depth))) return r;
  if (!per_sample || !sig) return fail(PT_ERR_INVALID_ARG, "output pointers are NULL");
  if (first < 0) return fail(PT_ERR_INVALID_ARG, "first_sample must be >= 0");
  if (w <= 0 || h <= 0 || x0 < 0 || y0 < 0 || x0 + w > C.W || y0 + h > C.H)
    return fail(PT_ERR_INVALID_ARG, "crop outside the image");
  if ((r = set_device(s))) return r;
  if ((r = ready_to_render(s))) return r;
  if ((r = run_passes(s, C, x0, y0, w, h, first, spp, max_depth, seed, nullptr, per_sample, sig, spp))) return r;
  return sync_traced(s);
}

// ------------------------------------------------------------ radiance cache
pt_status pt_set_radiance_cache(pt_scene* s, const pt_radiance_cache_config* cfg) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!cfg) {
    s->nrc_on = false;
    s->nrc_ready = false;
    return PT_OK;
  }
  const pt_radiance_cache_config& c = *cfg;
  if (c.query_bounce < 0) return fail(PT_ERR_INVALID_ARG, "query_bounce must be >= 0");
  if (c.train_paths < 1 || c.train_paths > (1 << 24)) return fail(PT_ERR_INVALID_ARG, "train_paths must be in [1, 2^24]");
  if (c.batch_size < 1 || c.batch_size > (1 << 22)) return fail(PT_ERR_INVALID_ARG, "batch_size must be in [1, 2^22]");
  if (c.steps_per_frame < 0 || c.steps_per_frame > 64) return fail(PT_ERR_INVALID_ARG, "steps_per_frame must be in [0, 64]");
  if (!(c.learning_rate > 0.0f) || !std::isfinite(c.learning_rate)) return fail(PT_ERR_INVALID_ARG, "learning_rate must be > 0");
  if (!(c.beta1 >= 0.0f && c.beta1 < 1.0f) || !(c.beta2 >= 0.0f && c.beta2 < 1.0f))
    return fail(PT_ERR_INVALID_ARG, "beta1 and beta2 must be in [0, 1)");
  if (!(c.epsilon > 0.0f) || !std::isfinite(c.epsilon)) return fail(PT_ERR_INVALID_ARG, "epsilon must be > 0");
  if (!(c.ema_decay >= 0.0f && c.ema_decay < 1.0f)) return fail(PT_ERR_INVALID_ARG, "ema_decay must be in [0, 1)");
  if (c.train_end_bounce < -1) return fail(PT_ERR_INVALID_ARG, "train_end_bounce must be >= -1");
  if (c.factorize != 0 && c.factorize != 1) return fail(PT_ERR_INVALID_ARG, "factorize must be 0 or 1");
  if (!(c.spread_c >= 0.0f) || !std::isfinite(c.spread_c)) return fail(PT_ERR_INVALID_ARG, "spread_c must be >= 0");
  if ((r = set_device(s))) return r;
  std::vector<float> w;
  nrc_init_weights(c.init_seed, w);
  const size_t bytes = kNrcParams * sizeof(float);
  PT_HIP(upload(s->nrc_w, w.data(), bytes, s->stream));
  PT_HIP(upload(s->nrc_wi, w.data(), bytes, s->stream));
  std::vector<float> zero(kNrcParams, 0.0f);
  PT_HIP(upload(s->nrc_m, zero.data(), bytes, s->stream));
  PT_HIP(upload(s->nrc_v, zero.data(), bytes, s->stream));
  PT_HIP(upload(s->nrc_e, zero.data(), bytes, s->stream));
  if (!s->nrc_fwd.p) PT_HIP(s->nrc_fwd.alloc(kNrcFwdFrags * 64 * sizeof(uint4)));
  if (!s->nrc_bwd.p) PT_HIP(s->nrc_bwd.alloc(kNrcBwdFrags * 64 * sizeof(uint4)));
  if (!s->nrc_inf.p) PT_HIP(s->nrc_inf.alloc(kNrcFwdFrags * 64 * sizeof(uint4)));
  if (!s->nrc_t.p) PT_HIP(s->nrc_t.alloc(sizeof(uint32_t)));
  if (c.train_end_bounce >= 0)  // both path sets: the frame loop allocates nothing while frames overlap
    for (DevBuf& b : s->nrc_tail) PT_HIP(b.alloc((size_t)c.train_paths * sizeof(float4)));
  PT_HIP(hipMemsetAsync(s->nrc_t.p, 0, sizeof(uint32_t), s->stream));
  PT_HIP(nrc_pack(s, nullptr, nullptr, s->stream));
  s->nrc_cfg = c;
  s->nrc_on = true;
  s->nrc_ready = false;
  return sync(s);
}

pt_status pt_nrc_set_weights(pt_scene* s, const float* weights, int64_t n) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!s->nrc_on) return fail(PT_ERR_STATE, "pt_set_radiance_cache has not been called");
  if (!weights || n != kNrcParams) return fail(PT_ERR_INVALID_ARG, "weights must be %d device floats", kNrcParams);
  if ((r = set_device(s))) return r;
  PT_HIP(hipMemcpyAsync(s->nrc_w.p, weights, kNrcParams * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
  PT_HIP(hipMemcpyAsync(s->nrc_wi.p, weights, kNrcParams * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
  std::vector<float> zero(kNrcParams, 0.0f);
  PT_HIP(hipMemcpyAsync(s->nrc_m.p, zero.data(), kNrcParams * sizeof(float), hipMemcpyHostToDevice, s->stream));
  PT_HIP(hipMemcpyAsync(s->nrc_v.p, zero.data(), kNrcParams * sizeof(float), hipMemcpyHostToDevice, s->stream));
  PT_HIP(hipMemcpyAsync(s->nrc_e.p, zero.data(), kNrcParams * sizeof(float), hipMemcpyHostToDevice, s->stream));
  PT_HIP(nrc_pack(s, nullptr, nullptr, s->stream));
  PT_HIP(hipMemsetAsync(s->nrc_t.p, 0, sizeof(uint32_t), s->stream));
  s->nrc_ready = true;
  return sync(s);
}

pt_status pt_nrc_get_weights(pt_scene* s, float* weights, float* adam_m, float* adam_v, int64_t* step) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!s->nrc_on) return fail(PT_ERR_STATE, "pt_set_radiance_cache has not been called");
  if ((r = set_device(s))) return r;
  const size_t bytes = kNrcParams * sizeof(float);
  if (weights) PT_HIP(hipMemcpyAsync(weights, s->nrc_w.p, bytes, hipMemcpyDeviceToDevice, s->stream));
  if (adam_m) PT_HIP(hipMemcpyAsync(adam_m, s->nrc_m.p, bytes, hipMemcpyDeviceToDevice, s->stream));
  if (adam_v) PT_HIP(hipMemcpyAsync(adam_v, s->nrc_v.p, bytes, hipMemcpyDeviceToDevice, s->stream));
  if (step) {
    uint32_t t = 0;
    PT_HIP(hipMemcpyAsync(&t, s->nrc_t.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
    PT_HIP(hipStreamSynchronize(s->stream));
    *step = (int64_t)t;
  }
  return sync(s);
}

pt_status pt_nrc_get_inference_weights(pt_scene* s, float* weights) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!s->nrc_on) return fail(PT_ERR_STATE, "pt_set_radiance_cache has not been called");
  if (!weights) return fail(PT_ERR_INVALID_ARG, "weights is NULL");
  if ((r = set_device(s))) return r;
  PT_HIP(hipMemcpyAsync(weights, s->nrc_wi.p, kNrcParams * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
  return sync(s);
}

pt_status pt_nrc_forward(pt_scene* s, const float* inputs, int64_t n, float* outputs) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!s->nrc_on) return fail(PT_ERR_STATE, "pt_set_radiance_cache has not been called");
  if (n < 0 || n > ((int64_t)1 << 31)) return fail(PT_ERR_INVALID_ARG, "n must be in [0, 2^31]");
  if (n == 0) return PT_OK;
  if (!inputs || !outputs) return fail(PT_ERR_INVALID_ARG, "inputs and outputs must be non-NULL");
  if ((r = set_device(s))) return r;
  if (s->timing) {
    for (hipEvent_t& e : s->ev_forward)
      if (!e) PT_HIP(hipEventCreate(&e));
    PT_HIP(hipEventRecord(s->ev_forward[0], s->stream));
  }
  PT_HIP(nrc_launch_forward(inputs, n, s->nrc_inf.as<uint4>(), outputs, s->stream));
  if (s->timing) PT_HIP(hipEventRecord(s->ev_forward[1], s->stream));
  if ((r = sync(s))) return r;
  if (s->timing) {
    float ms = 0.0f;
    PT_HIP(hipEventElapsedTime(&ms, s->ev_forward[0], s->ev_forward[1]));
    s->ms_cache_forward += ms;
    s->cache_forward_queries += n;
  }
  return PT_OK;
}

pt_status pt_nrc_gradient(pt_scene* s, const float* inputs, const float* targets, int32_t n, float* grad,
                          double* loss) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!s->nrc_on) return fail(PT_ERR_STATE, "pt_set_radiance_cache has not been called");
  if (n < 1 || n > (1 << 22)) return fail(PT_ERR_INVALID_ARG, "n must be in [1, 2^22]");
  if (!inputs || !targets || !grad) return fail(PT_ERR_INVALID_ARG, "inputs, targets and grad must be non-NULL");
  if ((r = set_device(s))) return r;
  int grid = 0;
  if ((r = nrc_step(s, inputs, targets, n, grad, false, &grid, s->stream))) return r;
  if (loss) return nrc_read_loss(s, grid, n, loss, s->stream);
  return sync(s);
}

pt_status pt_nrc_train(pt_scene* s, const float* inputs, const float* targets, int32_t n, int32_t frame, uint64_t seed,
                       double* mean_loss) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!s->nrc_on) return fail(PT_ERR_STATE, "pt_set_radiance_cache has not been called");
  if (n < 1) return fail(PT_ERR_INVALID_ARG, "n must be >= 1");
  if (frame < 0) return fail(PT_ERR_INVALID_ARG, "frame must be >= 0");
  if (!inputs || !targets) return fail(PT_ERR_INVALID_ARG, "inputs and targets must be non-NULL");
  if ((r = set_device(s))) return r;
  if (!s->nrc_n.p) PT_HIP(s->nrc_n.alloc(sizeof(uint32_t)));
  uint32_t nn = (uint32_t)n;
  PT_HIP(hipMemcpyAsync(s->nrc_n.p, &nn, sizeof(uint32_t), hipMemcpyHostToDevice, s->stream));
  PT_HIP(hipStreamSynchronize(s->stream));
  if ((r = nrc_train_records(s, inputs, targets, s->nrc_n.as<uint32_t>(), (uint32_t)frame, seed, mean_loss,
                             s->stream)))
    return r;
  return sync(s);
}

pt_status pt_nrc_training_records(pt_scene* s, const pt_camera* cam, int32_t frame, int32_t max_depth, uint64_t seed,
                                  float* inputs, float* targets, uint32_t* path_offsets, int64_t capacity,
                                  int64_t* n_records) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!s->nrc_on) return fail(PT_ERR_STATE, "pt_set_radiance_cache has not been called");
  CamDev C;
  if ((r = make_camera(cam, C))) return r;
  if ((r = check_render_args(1, max_depth))) return r;
  if (frame < 0) return fail(PT_ERR_INVALID_ARG, "frame must be >= 0");
  if (capacity < 0 || (capacity > 0 && (!inputs || !targets)) || !n_records)
    return fail(PT_ERR_INVALID_ARG, "bad output buffers");
  if ((r = set_device(s))) return r;
  if ((r = ready_to_render(s))) return r;
  uint32_t n = 0;
  if ((r = nrc_trace_training(s, C, (uint32_t)frame, max_depth, seed, &n))) return r;
  int64_t m = std::min<int64_t>(n, capacity);
  if (m > 0) {
    PT_HIP(hipMemcpyAsync(inputs, s->nrc_X.p, (size_t)m * 12 * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
    PT_HIP(hipMemcpyAsync(targets, s->nrc_T.p, (size_t)m * 3 * sizeof(float), hipMemcpyDeviceToDevice, s->stream));
  }
  if (path_offsets)
    PT_HIP(hipMemcpyAsync(path_offsets, s->nrc_off.p, (size_t)s->nrc_cfg.train_paths * sizeof(uint32_t),
                          hipMemcpyDeviceToDevice, s->stream));
  *n_records = n;
  return sync(s);
}

pt_status pt_trace_closest(pt_scene* s, const float* rays, int64_t n, uint32_t* hits, int32_t brute) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (n < 0 || n > 0x7FFFFFFF || (n > 0 && (!rays || !hits))) return fail(PT_ERR_INVALID_ARG, "bad rays/hits");
  if (!s->has_bvh) return fail(PT_ERR_STATE, "pt_build_bvh has not been called");
  if (n == 0) return PT_OK;
  if ((r = set_device(s))) return r;
  int grid = brute ? trace_grid_blocks() : traversal_grid(n);
  if ((r = ensure_spill(s, grid))) return r;
  if ((r = ensure_counters(s))) return r;
  SceneDev S = scene_dev(s, grid);
  PT_HIP(launch_trace_rays(S, rays, n, hits, brute != 0, s->two_level, grid, s->stats.as<unsigned long long>(),
                           s->stream));
  return sync_traced(s);
}

pt_status pt_trace_closest_noalloc(pt_scene* s, const float* rays, int64_t n, uint32_t* hits, int32_t brute) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (n < 0 || n > 0x7FFFFFFF || (n > 0 && (!rays || !hits))) return fail(PT_ERR_INVALID_ARG, "bad rays/hits");
  if (!s->has_bvh) return fail(PT_ERR_STATE, "pt_build_bvh has not been called");
  if (n == 0) return PT_OK;
  if ((r = set_device(s))) return r;
  unsigned char* base = nullptr;
  PT_HIP(noalloc_scratch(s->device, &base));
  // the spill area holds the stack entries beyond the LDS part of every lane of the grid:
  // the grid shrinks until it fits (the lanes are persistent, so any grid traces all rays)
  const int cap = stack_capacity(s->bvh_depth);
  const size_t lane_bytes = (size_t)std::max(1, cap - kLdsStack) * sizeof(uint2);
  const int64_t fit = (int64_t)((kNoAllocScratchBytes - kNoAllocStatsBytes) / (lane_bytes * kBlock));
  if (!brute && fit < 1)
    return fail(PT_ERR_UNSUPPORTED, "BVH depth %d needs %zu bytes of stack spill per workgroup, more than the %zu-byte "
                "scratch of the allocation-free call", s->bvh_depth, lane_bytes * kBlock,
                kNoAllocScratchBytes - kNoAllocStatsBytes);
  const int grid = brute ? trace_grid_blocks() : (int)std::min<int64_t>(traversal_grid(n), fit);
  SceneDev S = scene_dev(s, grid);
  S.spill = reinterpret_cast<uint2*>(base + kNoAllocStatsBytes);
  S.spill_stride = (uint32_t)grid * kBlock;
  unsigned long long* counters = reinterpret_cast<unsigned long long*>(base);
  PT_HIP(launch_zero_u64(counters, kNumStats, s->stream));  // the previous call's counters are still there
  PT_HIP(launch_trace_rays(S, rays, n, hits, brute != 0, s->two_level, grid, counters, s->stream));
  unsigned long long overflow = 0;
  PT_HIP(hipMemcpyAsync(&overflow, counters + kStatOverflow, sizeof(overflow), hipMemcpyDeviceToHost, s->stream));
  if ((r = sync(s))) return r;
  if (overflow)
    return fail(PT_ERR_DEVICE, "traversal stack overflow in %llu workgroups (capacity %d entries per lane)", overflow,
                cap);
  return PT_OK;
}

pt_status pt_get_stats(pt_scene* s, pt_stats* o) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (!o) return fail(PT_ERR_INVALID_ARG, "out is NULL");
  std::memset(o, 0, sizeof(*o));
  if (s->stats.p) {
    if ((r = set_device(s))) return r;
    unsigned long long v[kNumStats];
    PT_HIP(hipMemcpyAsync(v, s->stats.p, sizeof(v), hipMemcpyDeviceToHost, s->stream));
    PT_HIP(hipStreamSynchronize(s->stream));
    o->extension_rays = (int64_t)v[kStatExt];
    o->shadow_rays = (int64_t)v[kStatShadow];
    o->nonfinite_dropped = (int64_t)v[kStatNonFinite];
    o->node_visits = (int64_t)v[kStatNodes];
    o->tri_tests = (int64_t)v[kStatTris];
    o->shadow_node_visits = (int64_t)v[kStatShadowNodes];
    o->shadow_tri_tests = (int64_t)v[kStatShadowTris];
    o->cache_queries = (int64_t)v[kStatQueries];
    o->cache_records = (int64_t)v[kStatRecords];
    o->tail_extension_rays = (int64_t)v[kStatTailExt];
    o->tail_node_visits = (int64_t)v[kStatTailNodes];
    o->tail_tri_tests = (int64_t)v[kStatTailTris];
    o->tail_shadow_rays = (int64_t)v[kStatTailShadow];
    o->tail_shadow_node_visits = (int64_t)v[kStatTailShadowNodes];
    o->tail_shadow_tri_tests = (int64_t)v[kStatTailShadowTris];
    o->instances_entered = (int64_t)v[kStatInstances];
    o->tail_instances_entered = (int64_t)v[kStatTailInstances];
    if (v[kStatOverflow]) return fail(PT_ERR_DEVICE, "traversal stack overflow in %llu workgroups", v[kStatOverflow]);
  }
  o->samples = s->samples;
  o->ms_extend = s->ms_extend;
  o->launches_extend = s->launches_extend;
  o->ms_total = s->ms_total;
  o->cache_adam_steps = 0;
  if (s->nrc_t.p) {
    uint32_t t = 0;
    PT_HIP(hipMemcpyAsync(&t, s->nrc_t.p, sizeof(uint32_t), hipMemcpyDeviceToHost, s->stream));
    PT_HIP(hipStreamSynchronize(s->stream));
    o->cache_adam_steps = (int64_t)t;
  }
  o->ms_cache_query = s->ms_cache_query;
  o->ms_cache_train = s->ms_cache_train;
  o->ms_tail = s->ms_tail;
  o->launches_tail = s->launches_tail;
  o->ms_display = s->ms_display;
  o->launches_display = s->launches_display;
  o->ms_cache_forward = s->ms_cache_forward;
  o->cache_forward_queries = s->cache_forward_queries;
  return PT_OK;
}

pt_status pt_reset_stats(pt_scene* s) {
  pt_status r = check_scene(s);
  if (r) return r;
  if ((r = set_device(s))) return r;
  if ((r = ensure_counters(s))) return r;
  PT_HIP(launch_zero_u64(s->stats.as<unsigned long long>(), kNumStats, s->stream));
  s->overflow_seen = 0;
  s->ms_extend = s->ms_total = 0.0;
  s->launches_extend = 0;
  s->samples = 0;
  s->ms_cache_query = s->ms_cache_train = 0.0;
  s->ms_tail = 0.0;
  s->launches_tail = 0;
  s->ms_display = 0.0;
  s->launches_display = 0;
  s->ms_cache_forward = 0.0;
  s->cache_forward_queries = 0;
  return sync(s);
}

pt_status pt_set_tail(pt_scene* s, int32_t min_bounce, double max_fraction) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (min_bounce < 0) return fail(PT_ERR_INVALID_ARG, "min_bounce must be >= 0");
  if (!(max_fraction >= 0.0 && max_fraction <= 1.0)) return fail(PT_ERR_INVALID_ARG, "max_fraction must be in [0, 1]");
  s->tail_min_bounce = min_bounce;
  s->tail_fraction = max_fraction;
  return PT_OK;
}

pt_status pt_set_gpu_bvh_builder(pt_scene* s, int32_t builder) {
  pt_status r = check_scene(s);
  if (r) return r;
  if (builder != PT_GPU_BVH_PLOC && builder != PT_GPU_BVH_LBVH)
    return fail(PT_ERR_INVALID_ARG, "builder must be PT_GPU_BVH_PLOC or PT_GPU_BVH_LBVH");
  s->gpu_bvh_builder = builder == PT_GPU_BVH_PLOC ? kGpuBvhPloc : kGpuBvhLbvh;
  return PT_OK;
}

pt_status pt_set_profiling(pt_scene* s, int32_t timing, int32_t counting) {
  pt_status r = check_scene(s);
  if (r) return r;
  s->timing = timing != 0;
  s->counting = counting != 0;
  return PT_OK;
}

// ------------------------------------------------------- host-only BVH
struct pt_bvh_host {
  Bvh4 b;
  bool two = false;
  TwoLevel T;
};

pt_status pt_bvh_host_build_instanced(const pt_mesh* meshes, int32_t n_meshes, const pt_instance* instances,
                                      int32_t n_instances, pt_bvh_host** out) {
  if (!meshes || !instances || !out || n_meshes <= 0 || n_instances <= 0) return fail(PT_ERR_INVALID_ARG, "bad arguments");
  *out = nullptr;
  for (int i = 0; i < n_meshes; ++i) {
    const pt_mesh& m = meshes[i];
    if (!m.vertices || !m.indices || m.n_vertices <= 0 || m.n_triangles <= 0)
      return fail(PT_ERR_INVALID_ARG, "mesh %d: NULL arrays or empty counts", i);
    for (int64_t t = 0; t < m.n_triangles * 3; ++t)
      if (m.indices[t] < 0 || m.indices[t] >= m.n_vertices) return fail(PT_ERR_INVALID_ARG, "mesh %d: index out of range", i);
  }
  for (int i = 0; i < n_instances; ++i) {
    if (instances[i].mesh < 0 || instances[i].mesh >= n_meshes) return fail(PT_ERR_INVALID_ARG, "instance %d: bad mesh", i);
    if (!finite_all(instances[i].object_to_world, 12)) return fail(PT_ERR_INVALID_ARG, "instance %d: non-finite", i);
  }
  std::unique_ptr<pt_bvh_host> h(new (std::nothrow) pt_bvh_host());
  if (!h) return fail(PT_ERR_OUT_OF_MEMORY, "out of host memory");
  pt_status r = build_two_level_host(meshes, n_meshes, instances, n_instances, h->T);
  if (r) return r;
  h->two = true;
  *out = h.release();
  return PT_OK;
}

pt_status pt_bvh_host_build(const pt_mesh* m, pt_bvh_host** out) {
  if (!m || !out) return fail(PT_ERR_INVALID_ARG, "NULL argument");
  *out = nullptr;
  if (!m->vertices || !m->indices || m->n_vertices <= 0 || m->n_triangles <= 0)
    return fail(PT_ERR_INVALID_ARG, "NULL arrays or empty counts");
  int64_t n = m->n_triangles;
  std::vector<float> verts((size_t)n * 9);
  std::vector<uint32_t> prim((size_t)n), mat((size_t)n);
  for (int64_t t = 0; t < n; ++t) {
    for (int v = 0; v < 3; ++v) {
      int32_t vi = m->indices[3 * t + v];
      if (vi < 0 || vi >= m->n_vertices) return fail(PT_ERR_INVALID_ARG, "index out of range");
      for (int c = 0; c < 3; ++c) verts[9 * (size_t)t + 3 * v + c] = m->vertices[3 * (size_t)vi + c];
    }
    prim[(size_t)t] = (uint32_t)t;
    mat[(size_t)t] = m->material_ids ? (uint32_t)m->material_ids[t] : 0u;
  }
  std::unique_ptr<pt_bvh_host> h(new (std::nothrow) pt_bvh_host());
  if (!h) return fail(PT_ERR_OUT_OF_MEMORY, "out of host memory");
  std::string err;
  if (!build_bvh4(verts.data(), prim.data(), mat.data(), n, h->b, err)) return fail(PT_ERR_INVALID_ARG, "%s", err.c_str());
  *out = h.release();
  return PT_OK;
}

pt_status pt_bvh_host_info(const pt_bvh_host* h, pt_bvh_info* info) {
  if (!h || !info) return fail(PT_ERR_INVALID_ARG, "NULL argument");
  if (h->two) {
    info->n_nodes = (int64_t)h->T.nodes.size();
    info->n_tris = (int64_t)h->T.tris.size();
    info->depth = h->T.depth;
    info->max_leaf_tris = kMaxLeafTris;
    info->sah_cost = 0.0;
    info->build_ms = 0.0;
    info->stack_capacity = stack_capacity(h->T.depth);
    return PT_OK;
  }
  info->n_nodes = (int64_t)h->b.nodes.size();
  info->n_tris = (int64_t)h->b.tris.size();
  info->depth = h->b.depth;
  info->max_leaf_tris = h->b.max_leaf;
  info->sah_cost = h->b.sah_cost;
  info->build_ms = h->b.build_ms;
  info->stack_capacity = stack_capacity(h->b.depth);
  return PT_OK;
}

pt_status pt_bvh_host_copy(const pt_bvh_host* h, void* nodes, void* tris) {
  if (!h || !nodes || !tris) return fail(PT_ERR_INVALID_ARG, "NULL argument");
  const std::vector<BVHNode>& n = h->two ? h->T.nodes : h->b.nodes;
  const std::vector<TriRec>& t = h->two ? h->T.tris : h->b.tris;
  std::memcpy(nodes, n.data(), n.size() * sizeof(BVHNode));
  std::memcpy(tris, t.data(), t.size() * sizeof(TriRec));
  return PT_OK;
}

pt_status pt_bvh_host_trace_stack(const pt_bvh_host* h, const float* rays, int64_t n, uint32_t* hits,
                                  int32_t capacity, int32_t* high_water) {
  if (!h || n < 0 || (n > 0 && (!rays || !hits))) return fail(PT_ERR_INVALID_ARG, "bad arguments");
  const int bound = stack_capacity(h->two ? h->T.depth : h->b.depth);
  const int cap = capacity > 0 ? capacity : bound;
  if (cap > HostStack::kMax) return fail(PT_ERR_INVALID_ARG, "stack capacity above %d", HostStack::kMax);
  int high = 0;
  int64_t dropped = 0;
  for (int64_t i = 0; i < n; ++i) {
    const float* R = rays + 8 * i;
    RayPre r = ray_prepare(R[0], R[1], R[2], R[4], R[5], R[6]);
    Hit best;
    hit_clear(best);
    HostStack st;
    st.cap = cap;
    uint32_t nv = 0, nt = 0;
    if (h->two)
      traverse_two_level<false, false>(h->T.top.nodes.data(), h->T.items.data(), h->T.insts.data(),
                                       h->T.nodes.data(), h->T.tris.data(), r, R[3], R[7], 0xFFFFFFFFu, 0xFFFFFFFFu,
                                       best, st, nv, nt);
    else
      traverse_bvh<false, false>(h->b.nodes.data(), h->b.tris.data(), 0u, r, R[3], R[7], 0u, 0xFFFFFFFFu,
                                 0xFFFFFFFFu, best, st, nv, nt);
    high = std::max(high, st.high);
    if (st.overflow) dropped++;
    uint32_t* H = hits + 6 * i;
    bool hit = best.tri != 0xFFFFFFFFu;
    H[0] = f2u(best.t);
    H[1] = hit ? best.inst : 0xFFFFFFFFu;
    H[2] = hit ? best.prim : 0xFFFFFFFFu;
    H[3] = hit ? f2u(best.b1) : 0u;
    H[4] = hit ? f2u(best.b2) : 0u;
    H[5] = hit ? 1u : 0u;
  }
  if (high_water) *high_water = high;
  if (dropped) return fail(PT_ERR_DEVICE, "traversal stack overflow on %lld rays (capacity %d)", (long long)dropped, cap);
  return PT_OK;
}

pt_status pt_bvh_host_trace(const pt_bvh_host* h, const float* rays, int64_t n, uint32_t* hits) {
  return pt_bvh_host_trace_stack(h, rays, n, hits, 0, nullptr);
}

void pt_bvh_host_destroy(pt_bvh_host* h) { delete h; }

}  // extern "C"
