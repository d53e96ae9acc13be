// Internal declarations of the path-tracer library: device parameter blocks,
// the scene object behind the C ABI, and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/pt.h"
#include "bvh_build.h"
#include "pt_layout.h"

namespace pt {

constexpr int kBlock = 256;     // threads per workgroup (4 waves of 64)
#ifndef PT_LDS_STACK
#define PT_LDS_STACK 10
#endif
constexpr int kLdsStack = PT_LDS_STACK;  // traversal stack entries per lane kept in LDS
constexpr int kEnvRowGuide = 1024;      // guide-table sizes of the environment CDFs (powers of two)
constexpr int kEnvColGuide = 256;

// Scene data the kernels read (all device pointers).
struct SceneDev {
  const BVHNode* nodes;
  const TriRec* tris;
  uint32_t n_tris;
  uint32_t root;
  const MatRec* mats;
  const int32_t* tri_light;  // light index by primitive id, -1 if not emissive
  const LightTri* lights;
  const float* light_cdf;    // [n_lights + 1]
  int32_t n_lights;
  float p_env;               // probability of sampling the environment
  const float4* env;         // [h][w] rgb + unused
  const float* env_row_pmf;  // [h]
  const float* env_row_cdf;  // [h + 1]
  const float* env_col_pmf;  // [h][w]
  const float* env_col_cdf;  // [h][w + 1]
  const int32_t* env_row_guide;  // [kEnvRowGuide]: start of the search for u in [g/G, (g+1)/G)
  const int32_t* env_col_guide;  // [h][kEnvColGuide]
  int32_t env_w, env_h;
  float tmin;                // self-intersection offset: 1e-5 x scene diagonal
  float axis[3];             // object +z axis in world space (shading tangent, single level)
  // two-level hierarchy (instances); unused for a single world-space mesh
  const InstRec* insts;
  uint32_t n_insts;
  const BVHNode* tlas;
  const uint32_t* tlas_items;     // instance ids in top-level leaf order
  const int32_t* light_map;       // per instance with emitters: primitive -> light index
  const uint32_t* mesh_tri_first; // first triangle record of each mesh (brute force)
  const uint32_t* mesh_tri_count;
  uint2* spill;              // traversal stack spill, [cap - kLdsStack][grid threads]
  int32_t stack_cap;         // total stack entries per lane
  uint32_t spill_stride;     // grid threads of the traversal kernels
  float box_lo[3];           // scene box (radiance-cache position input)
  float box_inv[3];          // 1 / box extent per axis (0 for a flat axis)
};

// Camera basis computed on the host in double and rounded to float.
struct CamDev {
  float eye[3], R[3], U[3], F[3];
  float tan_half, aspect;
  int32_t W, H;
};

// Wavefront path state, structure-of-arrays, indexed by path slot.
struct PathsDev {
  float4* ray_o;       // o.xyz, skip primitive (bits)
  float4* ray_d;       // d.xyz, skip instance (bits)
  float4* hit;         // t, b1, b2, triangle record index (bits; 0xFFFFFFFF = miss)
  uint32_t* hit_inst;  // instance of the hit (two-level scenes)
  uint8_t* cls;        // material class of the hit (binning)
  float4* beta;        // throughput rgb, pdf of the last BSDF sample
  float4* L;           // radiance rgb, eta scale (product of eta^2 over refractions)
  uint32_t* flags;     // bit 0: last bounce was a delta lobe
  uint32_t* q_ray[2];  // extension queues (double-buffered)
  uint32_t* q_cls[kNumClasses];
  float4* sh_o;        // shadow ray o.xyz, tmax
  float4* sh_d;        // d.xyz, path slot (bits)
  float4* sh_c;        // contribution rgb, skip primitive (bits)
  uint32_t* sh_inst;   // skip instance
  uint32_t* counts;    // [0..1] ray queues, [2..2+kNumClasses) classes, [2+kNumClasses] shadow
  unsigned long long* stats;  // see kStat*
  uint64_t* sig;       // path signatures (debug)
  uint32_t* dbg_nee;   // pending next-event light id (debug)
  uint32_t* dbg_tail;  // pending lobe / roulette / end events (debug)
  int32_t n;           // number of path slots: n_render sampling paths, then training paths
  int32_t n_render;
  int32_t x0, y0, w;   // sampling path slot -> pixel (x0 + slot % w, y0 + slot / w)
  // training path k = slot - n_render: pixel index (k * pix_stride + pix_off) mod pix_total,
  // sample index train_sample
  uint32_t pix_stride, pix_off, pix_total, train_sample;
  // radiance cache
  float* nrc_q;        // query record per slot [n][16]: inputs x[12], beta rgb, unused
  uint32_t* q_nrc;     // slots that queried the cache (count in counts[kCountQuery])
  float* rec;          // training records [n][rec_depth][20] (nullptr: not a training pass)
  int32_t rec_depth;
  int32_t train_end;   // training paths end in the cache at this vertex (terminal record), -1: plain
  int32_t nrc_factor;  // 1: the cache predicts radiance / (diffuse albedo + specular albedo)
  // adaptive termination: per sampling path the primary footprint a0 and the running sum of the
  // spread terms; with spread_c > 0 a path ends in the cache at the first vertex b >= 1 where
  // sum^2 > spread_c * a0 (and at the query vertex at the latest)
  float2* spread;
  float spread_c;
};

enum {
  kStatExt = 0,
  kStatShadow = 1,
  kStatNonFinite = 2,
  kStatNodes = 3,
  kStatTris = 4,
  kStatOverflow = 5,
  kStatShadowNodes = 6,
  kStatShadowTris = 7,
  kStatQueries = 8,
  kStatTailExt = 9,     // closest-hit rays traced by the tail kernel (also in kStatExt)
  kStatTailNodes = 10,  // their node visits and triangle tests (not in kStatNodes / kStatTris)
  kStatTailTris = 11,
  kStatTailShadow = 12,       // shadow rays traced by the tail kernel (also in kStatShadow)
  kStatTailShadowNodes = 13,  // their node visits and triangle tests (not in kStatShadowNodes / kStatShadowTris)
  kStatTailShadowTris = 14,
  kStatRecords = 15,          // radiance-cache training records of the frame loop
  kStatInstances = 16,        // instances entered by the traversal kernel's walks (two-level; counting on)
  kStatTailInstances = 17,    // instances entered by the tail kernel's walks (two-level; counting on)
  kNumStats = 18
};
constexpr int kCountShadow = 2 + kNumClasses;
constexpr int kCountQuery = kCountShadow + 1;
constexpr int kCountTail = kCountQuery + 1;  // paths the tail kernel has taken so far
constexpr int kNumCounts = 16;

// ---- kernel launchers (pt_kernels.hip) ----
struct PassArgs {
  uint32_t sample;
  uint32_t k0, k1;  // Philox key
  int max_depth;
  int grid;         // workgroups of the persistent kernels
  int grid_trace;   // workgroups of the traversal kernels
  int grid_bin;     // workgroups of the binning kernel
  bool debug;
  bool count;
  bool two_level;
  uint32_t class_mask;  // material classes present (bit per class)
  hipEvent_t* ext_events;  // 2 per traversal launch (at most max_depth + 2) when timing, else nullptr
  int nrc_bounce;          // vertex at which paths end in the radiance cache, -1: no cache
  const uint4* nrc_fwd;    // packed forward weight fragments (when nrc_bounce >= 0)
  hipEvent_t* nrc_events;  // 2 events around the cache-query kernel when timing, else nullptr
  // tail hand-off: from bounce tail_min_bounce on, when at most tail_fraction of the slots are
  // still alive, one persistent kernel finishes the paths (tail_host_count: pinned host word)
  uint32_t* tail_host_count;
  int tail_min_bounce;
  double tail_fraction;
  hipEvent_t* tail_events;  // 2 events around the tail kernel when timing, else nullptr
  int* wavefront_bounces;   // out: bounces run by the wavefront kernels (host)
  hipStream_t tail_stream;  // if set, the tail kernel runs there after tail_ready (recorded here)
  hipEvent_t tail_ready;
  bool* tail_launched;      // out: the tail kernel was launched on tail_stream
  int* trace_launches;      // out: traversal launches of the pass (timed by ext_events)
  // radiance-cache frames: the stream waits for this event (if set) before the cache queries, and,
  // past the query vertex, at most tail_bound paths (the training paths) can be alive: when that
  // is at most tail_fraction of the slots, the tail kernel takes over without reading the count
  hipEvent_t query_wait;
  uint32_t tail_bound;
  bool query_beside;  // launch the cache queries on tail_stream at the hand-off, before the tail kernel
  // two side streams (both or neither) on which shading kernels of different material classes run
  // beside the pass's stream, with a fork event and one join event per side stream
  hipStream_t shade_side[2];
  hipEvent_t shade_fork, shade_join[2];
};

hipError_t launch_pass(const SceneDev& S, const PathsDev& P, const CamDev& C, const PassArgs& A,
                       hipStream_t st);
hipError_t launch_accumulate(const PathsDev& P, double* sum, int W, float* per_sample, uint64_t* sig_out,
                             int spp_total, int sample_index, hipStream_t st);
hipError_t launch_resolve(const double* sum, float* out, int64_t n_values, double inv_spp, hipStream_t st);
hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st);
// display image of the running mean (pt_display.hip): rgba8 and encoded are nullable
hipError_t launch_display(const double* sum, int64_t n_pixels, double inv_samples, double exposure, uint32_t* rgba8,
                          float* encoded, hipStream_t st);
hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t st);
hipError_t launch_trace_rays(const SceneDev& S, const float* rays, int64_t n, uint32_t* hits, bool brute,
                             bool two_level, int grid, unsigned long long* stats, hipStream_t st);
int trace_grid_blocks();
// Allocation-free closest hits: the library's static device scratch (one copy
// per GPU).  The first kNoAllocStatsBytes hold a launch's statistics counters,
// the rest the traversal stack spill area.
constexpr size_t kNoAllocScratchBytes = size_t(32) << 20;
constexpr size_t kNoAllocStatsBytes = 256;
static_assert(kNumStats * sizeof(unsigned long long) <= kNoAllocStatsBytes, "counters fit the scratch header");
// Device address of `dev`'s scratch; call with `dev` current.  The symbol is
// looked up once per device and the address kept.
hipError_t noalloc_scratch(int dev, unsigned char** out);
int traversal_grid(int64_t rays);  // workgroups of the traversal kernel for a pass of `rays` paths
int tail_grid(int grid_trace, uint32_t paths, bool beside);  // workgroups of the tail kernel

// ---- GPU BVH construction (pt_bvh_gpu.hip) ----
struct GpuBvhStats {
  int64_t n_nodes;  // BVH4 nodes written (at most max(1, n - 1))
  int depth;        // nodes on the longest root-to-leaf path, counting the leaf level
  int max_leaf;     // largest leaf (triangles)
};
// soup [n][9] floats, prim / mat [n] (device); nodes (device, room for max(1, n - 1) nodes; node 0 is
// the root) and tris (device, [n], leaf order) are written; synchronises the stream.
// builder: kGpuBvhPloc (locally-ordered clustering) or kGpuBvhLbvh (linear BVH)
constexpr int kGpuBvhPloc = 0, kGpuBvhLbvh = 1;
hipError_t gpu_build_bvh4(const float* soup, const uint32_t* prim, const uint32_t* mat, int64_t n, BVHNode* nodes,
                          TriRec* tris, hipStream_t st, GpuBvhStats* stats, int builder);

// ---- radiance cache (pt_nrc.hip) ----
// t_step / n_records (nullable): count the applied Adam step on the device unless the batch had no records
hipError_t nrc_launch_pack(const float* w, const float* wi, uint4* fwd, uint4* bwd, uint4* inf, uint32_t* t_step,
                           const uint32_t* n_records, hipStream_t st);
hipError_t nrc_launch_forward(const float* x, int64_t n, const uint4* fwd, float* y, hipStream_t st);
hipError_t nrc_launch_query(const PathsDev& P, const uint4* fwd, int grid, hipStream_t st);
hipError_t nrc_launch_train(const float* X, const float* T, int N, int npad, int n_split, const uint4* fwd,
                            const uint4* bwd, uint16_t* a_store, uint16_t* g_store, float* loss_part, int grid_fb,
                            float* dw_part, hipStream_t st);
hipError_t nrc_launch_adam(float* w, float* m, float* v, float* e, float* wi, const float* dw_part, int n_split,
                           float* grad_out, float lr, float b1, float b2, float eps, float ema, const uint32_t* t_step,
                           const uint32_t* n_records, int apply, hipStream_t st);
// self-training: tail[k] = beta_T * cache(x_T) for training paths with a terminal record at vertex P.train_end, else 0
hipError_t nrc_launch_terminal(const PathsDev& P, int n_paths, const uint4* fwd, float4* tail, hipStream_t st);
hipError_t nrc_launch_targets(const PathsDev& P, int n_paths, const float4* tail, uint32_t* offsets, uint32_t* block_sums, float* X,
                              float* T, uint32_t* n_out, unsigned long long* record_stats, hipStream_t st);
hipError_t nrc_launch_gather(const float* X_all, const float* T_all, const uint32_t* n_all, int B, uint32_t frame,
                             int step, uint32_t k0, uint32_t k1, float* Xb, float* Tb, hipStream_t st);
constexpr int kNrcFbGrid = 256;  // workgroups of the forward+backward kernel

}  // namespace pt
