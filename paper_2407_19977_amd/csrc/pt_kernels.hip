// Wavefront path-tracing kernels for gfx950 (wave64).
//
// One sampling pass traces one path per slot (one sample of every pixel of
// the tile) through the loop
//   generate -> [reset -> traverse -> bin -> shade<class>...] x (max_depth+1) -> traverse -> accumulate
// where traverse finds the closest hits of a bounce's rays together with the
// shadow rays of the previous bounce's shading.  From bounce 2 on, once few
// paths are alive, one persistent kernel (k_tail) finishes every remaining
// vertex instead.  Queues live in HBM and are compacted per workgroup: a
// ballot of the lanes that append, wave counts gathered in LDS, one atomic
// per workgroup on the queue tail and a lane prefix (mbcnt) for the slot.
// Queue lengths never leave the device, except the one count read to decide
// the tail hand-off: every kernel is launched over a fixed grid and strides
// over the length it reads from the counter array.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "pt_internal.h"
#include "pt_nrc.h"
#include "pt_shade.h"
#include "pt_trace.h"

namespace pt {

// ------------------------------------------------------------ wave helpers
__device__ inline uint32_t lane_id() { return __lane_id(); }

__device__ inline uint32_t lane_prefix(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

// A workgroup's share of a queue of n items in a grid of G workgroups:
// chunks of kShareChunk consecutive items dealt round-robin (chunk c to
// workgroup c mod G), so every workgroup gets items from all over the queue
// (regions of the image differ widely in cost) while a wave's refill still
// takes neighbouring items.  kShareChunk 0: one contiguous share each.
#ifndef PT_SHARE_CHUNK
#define PT_SHARE_CHUNK 256
#endif
constexpr uint32_t kShareChunk = PT_SHARE_CHUNK;
__device__ inline uint32_t share_size(uint32_t n, uint32_t wg, uint32_t G) {
  if (!kShareChunk) {
    const uint32_t per = (n + G - 1) / G, a = min(n, wg * per);
    return min(n, a + per) - a;
  }
  const uint32_t nc = (n + kShareChunk - 1) / kShareChunk;  // chunks, the last one possibly partial
  if (nc <= wg) return 0u;
  const uint32_t mine = (nc - 1 - wg) / G + 1;
  uint32_t items = mine * kShareChunk;
  if ((nc - 1) % G == wg) items -= nc * kShareChunk - n;  // this workgroup holds the partial chunk
  return items;
}
// queue index of item v (< share_size) of workgroup wg
__device__ inline uint32_t share_item(uint32_t v, uint32_t n, uint32_t wg, uint32_t G) {
  if (!kShareChunk) return min(n, wg * ((n + G - 1) / G)) + v;
  return ((v / kShareChunk) * G + wg) * kShareChunk + v % kShareChunk;
}

// Sum of a value over the wave's 64 lanes (every lane gets the sum).
__device__ inline uint32_t wave_sum(uint32_t v) {
  for (int d = 32; d >= 1; d >>= 1) v += (uint32_t)__shfl_xor((int)v, d);
  return v;
}

// ------------------------------------------------------------- signatures
constexpr uint64_t kFnvOffset = 0xcbf29ce484222325ull;
constexpr uint64_t kFnvPrime = 0x100000001b3ull;

__device__ inline uint64_t sig_word(uint64_t h, uint32_t w) {
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    h ^= (uint64_t)((w >> (8 * i)) & 0xFFu);
    h *= kFnvPrime;
  }
  return h;
}

// Tail events of a vertex, kept until the shadow ray of that vertex is
// resolved: lobe code (8 bits, 0xFF none), roulette (2 bits: 0 none,
// 1 survived, 2 killed), end reason (3 bits, 7 none).
__device__ inline uint32_t tail_pack(int lobe, int rr, int end) {
  return ((uint32_t)(lobe & 0xFF)) | ((uint32_t)rr << 8) | ((uint32_t)(end & 7) << 10);
}
__device__ inline uint64_t sig_tail(uint64_t h, uint32_t tail) {
  uint32_t lobe = tail & 0xFFu, rr = (tail >> 8) & 3u, end = (tail >> 10) & 7u;
  if (lobe != 0xFFu) { h = sig_word(h, 3); h = sig_word(h, lobe); }
  if (rr != 0u) { h = sig_word(h, 4); h = sig_word(h, rr == 2u ? 1u : 0u); }
  if (end != 7u) { h = sig_word(h, 6); h = sig_word(h, end); }
  return h;
}

// ----------------------------------------------------------------- stacks
// Traversal stack: the first kLdsStack entries of each lane in LDS as
// (ref, key) pairs, entry e of lane l at [e][l] (one 8-byte access per push
// or pop, conflict-free), deeper entries in a global spill area.  The LDS
// pointer keeps its address space so pops are LDS reads, not flat loads.
// The capacity (3 x BVH depth + 4) bounds a depth-first walk that pushes at
// most three siblings per level.
typedef __attribute__((address_space(3))) unsigned long long lds_u64;
__device__ inline unsigned long long stack_entry(uint32_t r, float k) {
  return (unsigned long long)r | ((unsigned long long)f2u(k) << 32);
}
struct DevStack {
  lds_u64* lds;
  uint2* spill;
  uint32_t sstride;
  int sp, cap;
  bool overflow;
  __device__ inline void push(uint32_t r, float k) {
    if (sp < kLdsStack) {
      lds[sp * kBlock] = stack_entry(r, k);
    } else if (sp < cap) {
      spill[(size_t)(sp - kLdsStack) * sstride] = make_uint2(r, f2u(k));
    } else {
      overflow = true;
      return;
    }
    sp++;
  }
  __device__ inline uint32_t pop(float& k) {
    --sp;
    // the LDS read is unconditional (clamped index) so it stays an LDS access;
    // the rare spill read replaces it
    unsigned long long w = lds[(sp < kLdsStack ? sp : kLdsStack - 1) * kBlock];
    if (sp >= kLdsStack)  // a relaxed atomic load is never merged with the LDS read into a flat load
      w = __hip_atomic_load(reinterpret_cast<unsigned long long*>(spill + (size_t)(sp - kLdsStack) * sstride),
                            __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WAVEFRONT);
    k = u2f((uint32_t)(w >> 32));
    return (uint32_t)w;
  }
  __device__ inline int size() const { return sp; }
};
__device__ inline lds_u64* lds_stack_base(unsigned long long* shared_stack) {
  return (lds_u64*)(shared_stack + threadIdx.x);
}

// ------------------------------------------------------------------ lights
// sin(theta) as |(x, z)| and theta = atan2(|(x, z)|, y): near the poles
// acos(y) and sqrt(1 - y^2) lose most of their FP32 digits to cancellation
// (at 0.4 degrees from the zenith sqrt(1 - y^2) is off by ~1e-3 relative,
// which moves the environment's pdf and every MIS weight that uses it).
__device__ inline int env_texel(const SceneDev& S, V3 d, float& sin_t) {
  const float sxz = sqrtf(d.x * d.x + d.z * d.z);
  float th = atan2f(sxz, d.y), ph = atan2f(d.x, -d.z);
  float u = ph * (0.5f / kPi) + 0.5f, v = th * (1.0f / kPi);
  int c = (int)floorf(u * (float)S.env_w), r = (int)floorf(v * (float)S.env_h);
  c = min(max(c, 0), S.env_w - 1);
  r = min(max(r, 0), S.env_h - 1);
  sin_t = sxz;
  return r * S.env_w + c;
}

__device__ inline float env_pdf_texel(const SceneDev& S, int texel, float sin_t) {
  int r = texel / S.env_w;
  float P = S.env_row_pmf[r] * S.env_col_pmf[texel];
  if (!(sin_t > 0.0f)) return 0.0f;
  return (float)S.env_w * (float)S.env_h * P / (2.0f * kPi * kPi * sin_t);
}

// bucket i with cdf[i] <= u < cdf[i+1], skipping empty buckets
__device__ inline int cdf_invert(const float* cdf, int n, float u) {
  int lo = 0, hi = n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (cdf[mid] <= u) lo = mid;
    else hi = mid;
  }
  int i = lo;
  while (i < n - 1 && !(cdf[i + 1] > cdf[i])) i++;
  while (i > 0 && !(cdf[i + 1] > cdf[i])) i--;
  return i;
}

// The same bucket through a guide table: guide[g] is the largest i with
// cdf[i] <= g/G, so for u in [g/G, (g+1)/G) the answer lies in
// [guide[g], guide[g+1]] and the binary search starts there (u * G is exact:
// u has 24 bits and G is a power of two).
__device__ inline int cdf_invert_guided(const float* cdf, int n, float u, const int32_t* guide, int G) {
  int g = min(G - 1, (int)(u * (float)G));
  int lo = guide[g], hi = g + 1 < G ? min(n, guide[g + 1] + 1) : n;
  while (hi - lo > 1) {
    int mid = (lo + hi) >> 1;
    if (cdf[mid] <= u) lo = mid;
    else hi = mid;
  }
  int i = lo;
  while (i < n - 1 && !(cdf[i + 1] > cdf[i])) i++;
  while (i > 0 && !(cdf[i + 1] > cdf[i])) i--;
  return i;
}

struct LightSample {
  V3 wl;
  float dist, pdf;
  V3 Le;
  uint32_t id;
  bool ok;
};

__device__ inline LightSample sample_light(const SceneDev& S, V3 p, float usel, float u1, float u2) {
  LightSample ls;
  ls.ok = false;
  ls.pdf = 0.0f;
  ls.dist = 0.0f;
  ls.Le = v3(0.0f, 0.0f, 0.0f);
  ls.wl = v3(0.0f, 0.0f, 1.0f);
  ls.id = 0xFFFFFFFFu;
  if (S.p_env <= 0.0f && S.n_lights == 0) return ls;
  if (usel < S.p_env) {
    int W = S.env_w, H = S.env_h;
    int r = cdf_invert_guided(S.env_row_cdf, H, u1, S.env_row_guide, kEnvRowGuide);
    float pr = S.env_row_pmf[r];
    float du = pr > 0.0f ? (u1 - S.env_row_cdf[r]) / pr : 0.5f;
    const float* ccdf = S.env_col_cdf + (size_t)r * (W + 1);
    int c = cdf_invert_guided(ccdf, W, u2, S.env_col_guide + (size_t)r * kEnvColGuide, kEnvColGuide);
    float pc = S.env_col_pmf[(size_t)r * W + c];
    float dv = pc > 0.0f ? (u2 - ccdf[c]) / pc : 0.5f;
    float uu = ((float)c + dv) / (float)W, vv = ((float)r + du) / (float)H;
    float th = kPi * vv, ph = 2.0f * kPi * (uu - 0.5f);
    float st, ct, sp, cp;
    sincosf(th, &st, &ct);
    sincosf(ph, &sp, &cp);
    ls.wl = v3(st * sp, ct, -st * cp);
    ls.dist = INFINITY;
    ls.id = 0x80000000u | (uint32_t)(r * W + c);
    if (!(st > 0.0f)) return ls;
    float P = pr * pc;
    ls.pdf = S.p_env * (float)W * (float)H * P / (2.0f * kPi * kPi * st);
    float4 e = S.env[(size_t)r * W + c];
    ls.Le = v3(e.x, e.y, e.z);
    ls.ok = ls.pdf > 0.0f;
    return ls;
  }
  float ut = S.p_env > 0.0f ? (usel - S.p_env) / (1.0f - S.p_env) : usel;
  int k = cdf_invert(S.light_cdf, S.n_lights, ut);
  ls.id = (uint32_t)k;
  const LightTri& L = S.lights[k];
  float sq = sqrtf(u1);
  float b0 = 1.0f - sq, b1 = u2 * sq;
  V3 q = v3(L.p0.x, L.p0.y, L.p0.z) * b0 + v3(L.p1.x, L.p1.y, L.p1.z) * b1 +
         v3(L.p2.x, L.p2.y, L.p2.z) * (1.0f - b0 - b1);
  V3 to = q - p;
  float d2 = dot(to, to);
  float dd = sqrtf(d2);
  if (!(dd > 0.0f)) return ls;
  ls.wl = to * (1.0f / dd);
  ls.dist = dd;
  float cl = -dot(v3(L.ng.x, L.ng.y, L.ng.z), ls.wl);
  if (cl <= 0.0f) return ls;
  ls.pdf = L.p1.w * d2 / (cl * L.p0.w);
  ls.Le = v3(L.Le.x, L.Le.y, L.Le.z);
  ls.ok = ls.pdf > 0.0f;
  return ls;
}

__device__ inline float pow_heuristic(float a, float b) {
  float a2 = a * a, b2 = b * b;
  return a2 + b2 > 0.0f ? a2 / (a2 + b2) : 0.0f;
}

__device__ inline bool finite3(V3 c) { return isfinite(c.x) && isfinite(c.y) && isfinite(c.z); }

// Pixel index (row-major) and sample index of a path slot: a tile of the
// image for sampling paths, the strided pixel set of the radiance cache's
// training paths after them.
__device__ inline uint32_t slot_pixel(const PathsDev& P, uint32_t slot, uint32_t img_w) {
  if (slot >= (uint32_t)P.n_render)
    return (uint32_t)(((uint64_t)(slot - (uint32_t)P.n_render) * P.pix_stride + P.pix_off) % P.pix_total);
  return (uint32_t)(P.y0 + slot / P.w) * img_w + (uint32_t)(P.x0 + slot % P.w);
}
__device__ inline uint32_t slot_sample(const PathsDev& P, uint32_t slot, uint32_t sample) {
  return slot >= (uint32_t)P.n_render ? P.train_sample : sample;
}

// ---------------------------------------------------------------- generate
template <bool DEBUG>
__global__ __launch_bounds__(kBlock) void k_generate(PathsDev P, CamDev C, uint32_t sample, uint32_t k0,
                                                     uint32_t k1) {
  int n = P.n;
  for (int slot = blockIdx.x * kBlock + threadIdx.x; slot < n; slot += gridDim.x * kBlock) {
    uint32_t pix = slot_pixel(P, (uint32_t)slot, (uint32_t)C.W);
    int px = (int)(pix % (uint32_t)C.W), py = (int)(pix / (uint32_t)C.W);
    U4 r = philox(pix, slot_sample(P, (uint32_t)slot, sample), 0u, 0u, k0, k1);
    float fx = (float)px + u01(r.x), fy = (float)py + u01(r.y);
    float x = (2.0f * fx / (float)C.W - 1.0f) * C.tan_half * C.aspect;
    float y = (1.0f - 2.0f * fy / (float)C.H) * C.tan_half;
    V3 d = normalize(v3(C.R[0], C.R[1], C.R[2]) * x + v3(C.U[0], C.U[1], C.U[2]) * y + v3(C.F[0], C.F[1], C.F[2]));
    P.ray_o[slot] = make_float4(C.eye[0], C.eye[1], C.eye[2], u2f(0xFFFFFFFFu));
    P.ray_d[slot] = make_float4(d.x, d.y, d.z, u2f(0xFFFFFFFFu));
    P.beta[slot] = make_float4(1.0f, 1.0f, 1.0f, 0.0f);
    P.L[slot] = make_float4(0.0f, 0.0f, 0.0f, 1.0f);
    P.flags[slot] = 1u;
    P.q_ray[0][slot] = (uint32_t)slot;
    if (DEBUG) P.sig[slot] = kFnvOffset;
    if (P.rec && slot >= P.n_render)
      for (int r = 0; r < P.rec_depth; ++r)
        P.rec[((size_t)(slot - P.n_render) * P.rec_depth + r) * kNrcRecFloats + 18] = 0.0f;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    P.counts[0] = (uint32_t)n;
    P.counts[kCountShadow] = 0u;
    P.counts[kCountQuery] = 0u;
  }
}

// Empty the next ray queue and the class queues (the shadow queue is still
// being traced; k_bin empties it).
__global__ void k_zero_u32(uint32_t* p) { *p = 0u; }

__global__ void k_reset_counts(uint32_t* counts, int next_queue) {
  int i = threadIdx.x;
  if (i >= 2 && i < kCountShadow) counts[i] = 0u;
  if (i == next_queue) counts[i] = 0u;
}

// ------------------------------------------------------------------ extend
// Persistent lanes: each workgroup owns a contiguous share of the ray queue
// and its lanes take rays from that share through an LDS counter.  A lane
// advances its own walk one node or one leaf per loop iteration; when half
// the wave is idle, the idle lanes take new rays, so the wave's SIMD lanes
// stay busy instead of waiting for the longest ray of a fixed batch.  The
// walk visits exactly what the recursive definition would (same culling and
// child order), so the closest hit is unchanged bit for bit.
constexpr uint32_t kNoInst = 0xFFFFFFFFu;
#ifndef PT_REFILL
#define PT_REFILL 16
#endif
constexpr uint32_t kRefill = PT_REFILL;  // idle lanes that trigger a refill
#ifndef PT_LEAF_WAIT
#define PT_LEAF_WAIT 1
#endif
#ifndef PT_LEAF_WAIT_DEN
#define PT_LEAF_WAIT_DEN 1
#endif
// traversal kernels: lanes at a leaf wait until kLeafWait x their number
// reaches kLeafWaitDen x the number of lanes at inner nodes (0: no waiting)
constexpr uint32_t kLeafWait = PT_LEAF_WAIT, kLeafWaitDen = PT_LEAF_WAIT_DEN;
#ifndef PT_SHADE_GRID_DIV
#define PT_SHADE_GRID_DIV 3
#endif
// with side streams each class kernel gets 1/PT_SHADE_GRID_DIV of the grid, so
// that the concurrent class kernels can be resident together
#ifndef PT_SHADE_BLOCK
#define PT_SHADE_BLOCK 256
#endif
constexpr int kShadeBlock = PT_SHADE_BLOCK;  // threads per workgroup of the shading kernels
#ifndef PT_TAIL_SHADE_WAIT
#define PT_TAIL_SHADE_WAIT 1
#endif
#ifndef PT_TAIL_DYNAMIC
#define PT_TAIL_DYNAMIC 1  // tail kernel: paths from a device-wide counter (0: a static share per workgroup)
#endif
// tail kernel: lanes waiting to shade go ahead once kTailShadeWait x their
// number reaches the number of lanes still walking (a large value shades at
// once, as soon as a walk ends)
constexpr uint32_t kTailShadeWait = PT_TAIL_SHADE_WAIT;
#ifndef PT_TAIL_PATHS_PER_GROUP
#define PT_TAIL_PATHS_PER_GROUP 512
#endif
// tail kernel beside the next pass: paths per workgroup (two per lane)
constexpr uint64_t kTailPathsPerGroup = PT_TAIL_PATHS_PER_GROUP;
#ifndef PT_TRACE_WAVES
#define PT_TRACE_WAVES 7
#endif
// minimum waves per SIMD the traversal kernel is compiled for
constexpr int kTraceWaves = PT_TRACE_WAVES;

struct LaneRay {
  RayPre r;   // ray in the space of the current level
  RayPre rw;  // world-space ray (two-level scenes)
  float tmin, tmax;
  uint32_t skip_inst, skip_prim;
  uint32_t cur;    // next reference to process, kEmpty: pop
  float cur_key;   // its entry distance
  uint32_t inst;   // instance of the current mesh walk, kNoInst at the top level
  int base;        // stack size when that mesh walk started
  bool any;        // shadow ray: stop at the first accepted triangle (kWalkPerLane walks)
  Hit best;
};

template <bool TWO>
__device__ inline void lane_start(LaneRay& L, float ox, float oy, float oz, float dx, float dy, float dz, float tmin,
                                  float tmax, uint32_t skip_inst, uint32_t skip_prim, uint32_t root) {
  L.r = ray_prepare(ox, oy, oz, dx, dy, dz);
  if (TWO) L.rw = L.r;
  L.tmin = tmin;
  L.tmax = tmax;
  L.skip_inst = skip_inst;
  L.skip_prim = skip_prim;
  L.cur = root;
  L.cur_key = -INFINITY;
  L.inst = kNoInst;
  L.base = 0;
  hit_clear(L.best);
}

// Walk kinds of lane_step: closest hit, any hit (shadow rays), or the kind
// the lane's own `any` flag names.
enum { kWalkClosest = 0, kWalkAny = 1, kWalkPerLane = 2 };

// One step of a lane's walk: visit one node, or test one leaf, then pop the
// next entry that can still hold a closer hit.  In two-level scenes a
// top-level leaf pushes its instances as entries (leaf bit, count 0,
// instance id) that start a mesh walk on top of the stack.  Returns true when
// the walk is over (any-hit walks: also at the first accepted triangle).
template <int KIND, bool COUNT, bool TWO>
__device__ inline bool lane_step(const SceneDev& S, LaneRay& L, DevStack& st, uint32_t& nvis, uint32_t& ntri,
                                 uint32_t& ninst) {
  const bool any = KIND == kWalkAny || (KIND == kWalkPerLane && L.any);
  const uint32_t cur = L.cur;
  if (cur != kEmpty) {
    if (!ref_is_leaf(cur)) {
      const BVHNode* nodes = (TWO && L.inst == kNoInst) ? S.tlas : S.nodes;
      const BVHNode n = nodes[cur];
      if (COUNT) nvis++;
      float tn[4];
      float tcur = fminf(L.best.t, L.tmax);
      uint32_t m = node_slabs(n, L.r, L.tmin, tcur, tn);
      float k0 = (m & 1u) ? tn[0] : INFINITY, k1 = (m & 2u) ? tn[1] : INFINITY;
      float k2 = (m & 4u) ? tn[2] : INFINITY, k3 = (m & 8u) ? tn[3] : INFINITY;
      uint32_t r0 = (m & 1u) ? n.child[0] : kEmpty, r1 = (m & 2u) ? n.child[1] : kEmpty;
      uint32_t r2 = (m & 4u) ? n.child[2] : kEmpty, r3 = (m & 8u) ? n.child[3] : kEmpty;
      cswap(k0, r0, k1, r1);
      cswap(k2, r2, k3, r3);
      cswap(k0, r0, k2, r2);
      cswap(k1, r1, k3, r3);
      cswap(k1, r1, k2, r2);
      if (r3 != kEmpty) st.push(r3, k3);
      if (r2 != kEmpty) st.push(r2, k2);
      if (r1 != kEmpty) st.push(r1, k1);
      L.cur = r0;
      L.cur_key = k0;
      if (r0 != kEmpty) return false;
    } else if (TWO && L.inst == kNoInst) {
      const uint32_t first = leaf_first(cur), cnt = leaf_count(cur);
      if (cnt == 0) {  // an instance entry: walk its mesh in object space
        const InstRec& I = S.insts[first];
        if (COUNT) ninst++;
        L.r = ray_to_object(I.w2o, L.rw.ox, L.rw.oy, L.rw.oz, L.rw.dx, L.rw.dy, L.rw.dz);
        L.inst = first;
        L.base = st.size();
        L.cur = I.blas_root;
        return false;
      }
      for (int j = (int)cnt - 1; j >= 0; --j) st.push(kLeafBit | S.tlas_items[first + j], L.cur_key);
    } else {
      if (leaf_test<KIND == kWalkAny, COUNT>(S.tris, cur, L.r, L.tmin, L.tmax, TWO ? L.inst : 0u, L.skip_inst,
                                             L.skip_prim, L.best, ntri, any) &&
          any)
        return true;
    }
    L.cur = kEmpty;
  }
  while (true) {
    if (TWO && L.inst != kNoInst && st.size() == L.base) {  // mesh walk over: back to the top level
      L.inst = kNoInst;
      L.r = L.rw;
    }
    if (st.size() == 0) return true;
    float k;
    uint32_t q = st.pop(k);
    if (k <= fminf(L.best.t, L.tmax)) {
      L.cur = q;
      L.cur_key = k;
      return false;
    }
  }
}

// The persistent-lane loop shared by the traversal kernels.  Src supplies
// start(i, L) (load item i into the lane) and finish(i, L, found).
template <int KIND, bool COUNT, bool TWO, class Src>
__device__ inline void persistent_trace(const SceneDev& S, Src& src, uint32_t count, unsigned long long* s_stack,
                                        uint32_t* s_next, uint32_t& nvis, uint32_t& ntri, bool& overflow) {
  const uint32_t per = (count + gridDim.x - 1) / gridDim.x;
  const uint32_t b0 = min(count, blockIdx.x * per), b1 = min(count, b0 + per);
  if (threadIdx.x == 0) *s_next = b0;
  __syncthreads();
  const uint32_t gtid = blockIdx.x * kBlock + threadIdx.x;
  DevStack st{lds_stack_base(s_stack), S.spill + gtid, S.spill_stride, 0, S.stack_cap, false};
  LaneRay L;
  bool busy = false, drained = false;
  uint32_t item = 0;
  while (true) {
    const uint64_t idle = __ballot(!busy);
    const uint32_t n_idle = (uint32_t)__popcll((unsigned long long)idle);
    if (!drained && (n_idle >= kRefill || n_idle == 64u)) {
      uint32_t base = 0;
      if (lane_id() == 0) base = atomicAdd(s_next, n_idle);
      base = __shfl(base, 0);
      if (base + n_idle >= b1) drained = true;
      const uint32_t i = base + lane_prefix(idle);
      if (!busy && i < b1) {
        item = i;
        st.sp = 0;
        src.start(i, L);
        busy = true;
      }
    }
    if (__ballot(busy) == 0) break;
    bool go = busy;
    if (kLeafWait) {
      // a lane at a leaf waits while there are many more lanes at inner
      // nodes, so that fewer iterations run both the node and the triangle
      // code
      const bool at_leaf = busy && L.cur != kEmpty && ref_is_leaf(L.cur);
      const uint32_t n_leaf = (uint32_t)__popcll((unsigned long long)__ballot(at_leaf));
      const uint32_t n_node = (uint32_t)__popcll((unsigned long long)__ballot(busy && !at_leaf));
      go = busy && (!at_leaf || kLeafWait * n_leaf >= kLeafWaitDen * n_node);
    }
    uint32_t ninst = 0;
    if (go && lane_step<KIND, COUNT, TWO>(S, L, st, nvis, ntri, ninst)) {
      src.finish(item, L, L.best.tri != 0xFFFFFFFFu);
      busy = false;
    }
  }
  overflow |= st.overflow;
}

template <bool TWO>
struct ExtendSrc {
  const SceneDev& S;
  const PathsDev& P;
  int cur;
  __device__ inline void start(uint32_t i, LaneRay& L) {
    uint32_t slot = P.q_ray[cur][i];
    float4 o = P.ray_o[slot], d = P.ray_d[slot];
    lane_start<TWO>(L, o.x, o.y, o.z, d.x, d.y, d.z, S.tmin, INFINITY, f2u(d.w), f2u(o.w), TWO ? 0u : S.root);
  }
  __device__ inline void finish(uint32_t i, const LaneRay& L, bool found) {
    uint32_t slot = P.q_ray[cur][i];
    int cls = kClsMiss;
    if (found) {
      P.hit[slot] = make_float4(L.best.t, L.best.b1, L.best.b2, u2f(L.best.tri));
      uint32_t mid = L.best.mat;
      if (TWO) {
        P.hit_inst[slot] = L.best.inst;
        int32_t ov = S.insts[L.best.inst].mat_override;
        if (ov >= 0) mid = (uint32_t)ov;
      }
      cls = S.mats[mid].cls;
    } else {
      P.hit[slot] = make_float4(INFINITY, 0.0f, 0.0f, u2f(0xFFFFFFFFu));
    }
    P.cls[slot] = (uint8_t)cls;
  }
};

// Material binning of the rays just traced: a counting sort by class with
// one atomic per class per workgroup (1024 rays).
__global__ __launch_bounds__(kBlock) void k_bin(PathsDev P, int cur) {
  __shared__ uint32_t s_cnt[kNumClasses], s_base[kNumClasses];
  const uint32_t count = P.counts[cur];
  // the traversal launch before this one has traced the shadow queue: empty it for the shading
  if (blockIdx.x == 0 && threadIdx.x == 0) P.counts[kCountShadow] = 0u;
  for (uint32_t blk = blockIdx.x * (4u * kBlock); blk < count; blk += gridDim.x * (4u * kBlock)) {
    if (threadIdx.x < kNumClasses) s_cnt[threadIdx.x] = 0u;
    __syncthreads();
    uint32_t slot[4], pos[4];
    int cls[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      uint32_t i = blk + k * kBlock + threadIdx.x;
      cls[k] = -1;
      if (i < count) {
        slot[k] = P.q_ray[cur][i];
        cls[k] = P.cls[slot[k]];
        pos[k] = atomicAdd(&s_cnt[cls[k]], 1u);  // LDS
      }
    }
    __syncthreads();
    if (threadIdx.x < kNumClasses) {
      uint32_t c = s_cnt[threadIdx.x];
      s_base[threadIdx.x] = c ? atomicAdd(&P.counts[2 + threadIdx.x], c) : 0u;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 4; ++k)
      if (cls[k] >= 0) P.q_cls[cls[k]][s_base[cls[k]] + pos[k]] = slot[k];
    __syncthreads();
  }
}

// ------------------------------------------------------------------- shade
struct ShadeOut {
  bool cont, shadow, query;  // next ray written / shadow ray below / path ended in the cache
  float4 sh_o, sh_d, sh_c;   // shadow ray: o, tmax; d, path slot; contribution, skip primitive
  uint32_t sh_inst;          // skip instance of the shadow ray
};

// Shade the hit (or miss) of path `slot` at vertex b: emission with MIS; at
// the last vertex stop; at the cache vertex write a query and stop;
// otherwise next-event estimation (a pre-weighted shadow ray), BSDF
// sampling, Russian roulette and the next ray.
template <int CLS, bool DEBUG, bool TWO>
__device__ inline void shade_one(const SceneDev& S, const PathsDev& P, uint32_t slot, int b, int max_depth,
                                 uint32_t sample, uint32_t k0, uint32_t k1, uint32_t img_w, int nrc_bounce,
                                 ShadeOut& o, unsigned long long& nonfinite) {
  o.cont = o.shadow = o.query = false;
  float4 rd = P.ray_d[slot];
  float4 be = P.beta[slot];
  float4 Lr = P.L[slot];
  uint32_t flags = P.flags[slot];
  V3 beta = v3(be.x, be.y, be.z);
  V3 L = v3(Lr.x, Lr.y, Lr.z);
  float pdf_prev = be.w, eta_scale = Lr.w;
  bool prev_delta = (flags & 1u) != 0u;
  V3 d = v3(rd.x, rd.y, rd.z);
  uint64_t sig = DEBUG ? P.sig[slot] : 0ull;
  if (CLS == kClsMiss) {
    if (S.env_w > 0) {
      float st;
      int texel = env_texel(S, d, st);
      if (DEBUG) { sig = sig_word(sig, 2); sig = sig_word(sig, (uint32_t)texel); }
      float4 e = S.env[texel];
      float w = 1.0f;
      if (!prev_delta) w = pow_heuristic(pdf_prev, S.p_env * env_pdf_texel(S, texel, st));
      if (w > 0.0f) {
        V3 c = v3(beta.x * w * e.x, beta.y * w * e.y, beta.z * w * e.z);
        if (finite3(c)) L = L + c;
        else nonfinite++;
      }
    } else if (DEBUG) {
      sig = sig_word(sig, 2);
      sig = sig_word(sig, 0xFFFFFFFFu);
    }
    if (DEBUG) { sig = sig_word(sig, 6); sig = sig_word(sig, 0); }
    P.L[slot] = make_float4(L.x, L.y, L.z, eta_scale);
    if (DEBUG) P.sig[slot] = sig;
  } else {
    float4 hv = P.hit[slot];
    const TriRec tr = S.tris[f2u(hv.w)];
    uint32_t prim = f2u(tr.a.w), mid = f2u(tr.b.w);
    uint32_t inst = 0;
    V3 p0 = v3(tr.a.x, tr.a.y, tr.a.z), p1 = v3(tr.b.x, tr.b.y, tr.b.z), p2 = v3(tr.c.x, tr.c.y, tr.c.z);
    float b1 = hv.y, b2 = hv.z;
    V3 p = p0 * (1.0f - b1 - b2) + p1 * b1 + p2 * b2;
    V3 nc = cross(p1 - p0, p2 - p0);
    V3 axis = v3(S.axis[0], S.axis[1], S.axis[2]);
    int light_of_prim = -1;
    if (TWO) {
      inst = P.hit_inst[slot];
      const InstRec& I = S.insts[inst];
      if (I.mat_override >= 0) mid = (uint32_t)I.mat_override;
      const float* q = I.o2w;
      p = v3(q[0] * p.x + q[1] * p.y + q[2] * p.z + q[3], q[4] * p.x + q[5] * p.y + q[6] * p.z + q[7],
             q[8] * p.x + q[9] * p.y + q[10] * p.z + q[11]);
      nc = v3(q[0] * nc.x + q[1] * nc.y + q[2] * nc.z, q[4] * nc.x + q[5] * nc.y + q[6] * nc.z,
              q[8] * nc.x + q[9] * nc.y + q[10] * nc.z);
      axis = v3(q[2], q[6], q[10]);
      if (I.light_map >= 0) light_of_prim = S.light_map[I.light_map + (int)prim];
    } else {
      light_of_prim = S.tri_light[prim];
    }
    const MatRec& m = S.mats[mid];
    if (DEBUG) { sig = sig_word(sig, 1); sig = sig_word(sig, inst); sig = sig_word(sig, prim); }
    V3 ng = normalize(nc);
    V3 wo_w = d * -1.0f;
    float cos_ng = dot(ng, wo_w);
    // emission (front face only), MIS-weighted against light sampling
    if ((m.flags & kMatEmissive) && cos_ng > 0.0f) {
      float w = 1.0f;
      if (!prev_delta) {
        int k = light_of_prim;
        float pl = 0.0f;
        if (k >= 0 && S.n_lights > 0) {
          const LightTri& Lt = S.lights[k];
          pl = Lt.p1.w * hv.x * hv.x / (cos_ng * Lt.p0.w);
        }
        w = pow_heuristic(pdf_prev, pl);
      }
      if (w > 0.0f) {
        V3 c = v3(beta.x * w * m.Le[0], beta.y * w * m.Le[1], beta.z * w * m.Le[2]);
        if (finite3(c)) L = L + c;
        else nonfinite++;
      }
    }
    int lobe_ev = -1, rr_ev = 0, end_ev = 7;
    bool pending = false;
    uint32_t nee_id = 0xFFFFFFFFu, nee_out = 3u;
    bool nee_done = false;
    bool entering = cos_ng > 0.0f;
    V3 n = entering ? ng : ng * -1.0f;
    // adaptive termination (path spread): a0 = t^2 / (4 pi |cos|) at the primary vertex, then the
    // sum of sqrt(t^2 / (pdf |cos|)) over the non-delta bounces that led to each later vertex
    bool spread_end = false;
    if (P.spread_c > 0.0f && slot < (uint32_t)P.n_render && nrc_bounce >= 0 && b <= nrc_bounce) {
      const float t = hv.x, ac = fabsf(cos_ng);
      float2 sp = b == 0 ? make_float2(t * t / (4.0f * kPi * ac), 0.0f) : P.spread[slot];
      if (b >= 1) {
        if (!prev_delta) sp.y += sqrtf(t * t / (pdf_prev * ac));
        spread_end = sp.y * sp.y > P.spread_c * sp.x;
      }
      P.spread[slot] = sp;
    }
    if (b == max_depth) {
      end_ev = 1;
    } else if ((b == nrc_bounce || spread_end) && slot < (uint32_t)P.n_render) {
      // the path ends in the radiance cache: the query adds beta * cache(x) after the pass
      float* qr = P.nrc_q + (size_t)slot * kNrcQueryFloats;
      nrc_inputs(S.box_lo, S.box_inv, p, wo_w, n, m, qr);
      qr[12] = beta.x;
      qr[13] = beta.y;
      qr[14] = beta.z;
      o.query = true;
      end_ev = 4;
    } else if (b == P.train_end && slot >= (uint32_t)P.n_render) {
      // self-training: the training path ends in the cache; its terminal record (flag 2) is
      // answered by the cache before the targets of its earlier vertices are formed
      float* rr = P.rec + ((size_t)(slot - P.n_render) * P.rec_depth + b) * kNrcRecFloats;
      nrc_inputs(S.box_lo, S.box_inv, p, wo_w, n, m, rr);
      rr[12] = L.x;
      rr[13] = L.y;
      rr[14] = L.z;
      rr[15] = beta.x;
      rr[16] = beta.y;
      rr[17] = beta.z;
      rr[18] = 2.0f;
      end_ev = 4;
    } else {
      if (P.rec && slot >= (uint32_t)P.n_render) {  // training record: inputs, radiance so far, throughput
        float* rr = P.rec + ((size_t)(slot - P.n_render) * P.rec_depth + b) * kNrcRecFloats;
        nrc_inputs(S.box_lo, S.box_inv, p, wo_w, n, m, rr);
        rr[12] = L.x;
        rr[13] = L.y;
        rr[14] = L.z;
        rr[15] = beta.x;
        rr[16] = beta.y;
        rr[17] = beta.z;
        rr[18] = 1.0f;
      }
      V3 t, bt;
      make_frame(n, axis, t, bt);
      V3 wo = v3(dot(wo_w, t), dot(wo_w, bt), dot(wo_w, n));
      Bsdf B = bsdf_setup<CLS>(m, entering, wo.z);
      if (wo.z <= 0.0f) B.absorbed = true;
      Rng rng{slot_pixel(P, slot, img_w), slot_sample(P, slot, sample), k0, k1};
      U4 r0 = rng.block((uint32_t)b, 0u), r1 = rng.block((uint32_t)b, 1u);
      // next-event estimation
      if (!B.absorbed && bsdf_has_nondelta<CLS>(m, B)) {
        nee_done = true;
        U4 r2 = rng.block((uint32_t)b, 2u);
        LightSample ls = sample_light(S, p, u01(r1.w), u01(r2.x), u01(r2.y));
        nee_id = ls.id;
        if (ls.ok) {
          V3 wil = v3(dot(ls.wl, t), dot(ls.wl, bt), dot(ls.wl, n));
          float pb;
          V3 f = bsdf_eval<CLS>(m, B, wo, wil, pb);
          float w = pow_heuristic(ls.pdf, pb);
          float k = fabsf(wil.z) * w / ls.pdf;
          V3 c = v3(beta.x * f.x * ls.Le.x * k, beta.y * f.y * ls.Le.y * k, beta.z * f.z * ls.Le.z * k);
          if (c.x != 0.0f || c.y != 0.0f || c.z != 0.0f) {
            o.shadow = true;
            pending = true;
            float tmax = isinf(ls.dist) ? INFINITY : (1.0f - 1e-4f) * ls.dist;
            o.sh_o = make_float4(p.x, p.y, p.z, tmax);
            o.sh_d = make_float4(ls.wl.x, ls.wl.y, ls.wl.z, u2f(slot));
            o.sh_c = make_float4(c.x, c.y, c.z, u2f(prim));
            o.sh_inst = inst;
          } else {
            nee_out = 2u;
          }
        }
      }
      // BSDF sampling
      BsdfSample bs = bsdf_sample<CLS>(m, B, wo, u01(r0.z), u01(r1.x), u01(r1.y), u01(r1.z));
      lobe_ev = bs.lobe;
      if (!bs.ok || (bs.weight.x == 0.0f && bs.weight.y == 0.0f && bs.weight.z == 0.0f)) {
        end_ev = 2;
      } else {
        beta = v3(beta.x * bs.weight.x, beta.y * bs.weight.y, beta.z * bs.weight.z);
        prev_delta = bs.delta;
        pdf_prev = bs.pdf;
        if (bs.refract) eta_scale *= B.eta * B.eta;
        bool killed = false;
        if (b >= 1) {
          float q = fmaxf(fmaxf(beta.x, beta.y), beta.z) * eta_scale;
          if (q < 0.995f) {  // no roulette within rounding of q = 1
            killed = u01(r0.w) >= q;
            rr_ev = killed ? 2 : 1;
            if (!killed) beta = beta * (1.0f / q);
          }
        }
        if (killed) {
          end_ev = 3;
        } else {
          V3 dn = normalize(t * bs.wi.x + bt * bs.wi.y + n * bs.wi.z);
          P.ray_o[slot] = make_float4(p.x, p.y, p.z, u2f(prim));
          P.ray_d[slot] = make_float4(dn.x, dn.y, dn.z, u2f(inst));
          P.beta[slot] = make_float4(beta.x, beta.y, beta.z, pdf_prev);
          P.flags[slot] = prev_delta ? 1u : 0u;
          o.cont = true;
        }
      }
    }
    P.L[slot] = make_float4(L.x, L.y, L.z, eta_scale);
    if (DEBUG) {
      uint32_t tail = tail_pack(lobe_ev, rr_ev, end_ev);
      if (pending) {
        P.dbg_nee[slot] = nee_id;
        P.dbg_tail[slot] = tail;
      } else {
        if (nee_done) {
          sig = sig_word(sig, 5);
          sig = sig_word(sig, nee_id);
          sig = sig_word(sig, nee_out);
        }
        sig = sig_tail(sig, tail);
      }
      P.sig[slot] = sig;
    }
  }
}

template <int CLS, bool DEBUG, bool TWO>
__global__ __launch_bounds__(kShadeBlock) void k_shade(SceneDev S, PathsDev P, int b, int max_depth, int next,
                                                  uint32_t sample, uint32_t k0, uint32_t k1, uint32_t img_w,
                                                  int nrc_bounce) {
  // per queue (next rays, shadow rays, cache queries): wave counts, then the workgroup's base
  __shared__ uint32_t s_app[3][kShadeBlock / 64 + 1];
  const uint32_t count = P.counts[2 + CLS];
  unsigned long long nonfinite = 0;
  for (uint32_t base = blockIdx.x * kShadeBlock; base < count; base += gridDim.x * kShadeBlock) {
    uint32_t i = base + threadIdx.x;
    bool active = i < count;
    uint32_t slot = 0;
    ShadeOut o;
    o.cont = o.shadow = o.query = false;
    if (active) {
      slot = P.q_cls[CLS][i];
      shade_one<CLS, DEBUG, TWO>(S, P, slot, b, max_depth, sample, k0, k1, img_w, nrc_bounce, o, nonfinite);
    }
    // One atomic per queue per workgroup iteration: the queue counters are
    // single words that every workgroup of the launch appends to.
    const uint64_t m_cont = __ballot(o.cont), m_sh = __ballot(o.shadow), m_q = __ballot(o.query);
    const int w = (int)(threadIdx.x >> 6);
    if (lane_id() == 0) {
      s_app[0][w] = (uint32_t)__popcll(m_cont);
      s_app[1][w] = (uint32_t)__popcll(m_sh);
      s_app[2][w] = (uint32_t)__popcll(m_q);
    }
    __syncthreads();
    if (threadIdx.x < 3) {
      uint32_t tot = 0;
      for (int k = 0; k < kShadeBlock / 64; ++k) tot += s_app[threadIdx.x][k];
      uint32_t* ctr = threadIdx.x == 0 ? &P.counts[next] : threadIdx.x == 1 ? &P.counts[kCountShadow]
                                                                              : &P.counts[kCountQuery];
      s_app[threadIdx.x][kShadeBlock / 64] = tot ? atomicAdd(ctr, tot) : 0u;
    }
    __syncthreads();
    uint32_t off[3];
    for (int q = 0; q < 3; ++q) {
      uint32_t acc = s_app[q][kShadeBlock / 64];
      for (int k = 0; k < w; ++k) acc += s_app[q][k];
      off[q] = acc;
    }
    __syncthreads();  // s_app is rewritten by the next iteration
    if (o.cont) P.q_ray[next][off[0] + lane_prefix(m_cont)] = slot;
    if (o.query) P.q_nrc[off[2] + lane_prefix(m_q)] = slot;
    if (o.shadow) {
      const uint32_t spos = off[1] + lane_prefix(m_sh);
      P.sh_o[spos] = o.sh_o;
      P.sh_d[spos] = o.sh_d;
      P.sh_c[spos] = o.sh_c;
      if (TWO) P.sh_inst[spos] = o.sh_inst;
    }
  }
  if (nonfinite) atomicAdd(&P.stats[kStatNonFinite], nonfinite);
}

// ----------------------------------------------------------------- connect
template <bool DEBUG, bool TWO>
struct ConnectSrc {
  const SceneDev& S;
  const PathsDev& P;
  unsigned long long& nonfinite;
  __device__ inline void start(uint32_t i, LaneRay& L) {
    float4 o = P.sh_o[i], d = P.sh_d[i];
    uint32_t skip_prim = f2u(P.sh_c[i].w);
    if (TWO) lane_start<true>(L, o.x, o.y, o.z, d.x, d.y, d.z, S.tmin, o.w, P.sh_inst[i], skip_prim, 0u);
    else lane_start<false>(L, o.x, o.y, o.z, d.x, d.y, d.z, S.tmin, o.w, 0u, skip_prim, S.root);
  }
  __device__ inline void finish(uint32_t i, const LaneRay& L, bool occ) {
    uint32_t slot = f2u(P.sh_d[i].w);
    if (!occ) {
      float4 c = P.sh_c[i];
      V3 cc = v3(c.x, c.y, c.z);
      if (finite3(cc)) {
        float4 Lr = P.L[slot];
        P.L[slot] = make_float4(Lr.x + cc.x, Lr.y + cc.y, Lr.z + cc.z, Lr.w);
      } else {
        nonfinite++;
      }
    }
    if (DEBUG) {
      uint64_t sig = P.sig[slot];
      sig = sig_word(sig, 5);
      sig = sig_word(sig, P.dbg_nee[slot]);
      sig = sig_word(sig, occ ? 1u : 0u);
      sig = sig_tail(sig, P.dbg_tail[slot]);
      P.sig[slot] = sig;
    }
  }
};

// One traversal launch per bounce: the closest hits of the bounce's rays
// (queue `cur`, none if cur < 0) and the shadow rays of the previous bounce's
// shading.  A lane's walk kind is a per-lane flag, so lanes of both kinds can
// share a wave without running the walk code twice: the node step is the same
// and the leaf step differs only in stopping at the first accepted triangle.
// Each workgroup owns a share of both queues and takes its closest-hit rays
// first; its shadow rays fill the lanes that the last closest-hit walks leave
// idle, instead of every workgroup of the GPU draining at a kernel boundary.
template <bool DEBUG, bool COUNT, bool TWO>
__global__ __launch_bounds__(kBlock, kTraceWaves) void k_traverse(SceneDev S, PathsDev P, int cur) {
  __shared__ unsigned long long s_stack[kLdsStack * kBlock];
  __shared__ uint32_t s_next;
  const uint32_t ne = cur >= 0 ? P.counts[cur] : 0u, ns = P.counts[kCountShadow];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (ne) atomicAdd(&P.stats[kStatExt], (unsigned long long)ne);
    if (ns) atomicAdd(&P.stats[kStatShadow], (unsigned long long)ns);
  }
  const uint32_t G = gridDim.x, wg = blockIdx.x;
  const uint32_t n_e = share_size(ne, wg, G), n_all = n_e + share_size(ns, wg, G);
  if (threadIdx.x == 0) s_next = 0u;
  __syncthreads();
  const uint32_t gtid = blockIdx.x * kBlock + threadIdx.x;
  DevStack st{lds_stack_base(s_stack), S.spill + gtid, S.spill_stride, 0, S.stack_cap, false};
  unsigned long long nonfinite = 0;
  ExtendSrc<TWO> es{S, P, cur < 0 ? 0 : cur};
  ConnectSrc<DEBUG, TWO> cs{S, P, nonfinite};
  LaneRay L;
  L.any = false;
  bool busy = false, drained = false, shadow = false;
  uint32_t item = 0;
  uint32_t rv = 0, rt = 0, nvis = 0, ntri = 0, svis = 0, stri = 0;  // node visits / triangle tests
  uint32_t ri = 0, ninst = 0;  // instances entered (both walk kinds)
  while (true) {
    const uint64_t idle = __ballot(!busy);
    const uint32_t n_idle = (uint32_t)__popcll((unsigned long long)idle);
    if (!drained && (n_idle >= kRefill || n_idle == 64u)) {
      uint32_t base = 0;
      if (lane_id() == 0) base = atomicAdd(&s_next, n_idle);
      base = __shfl(base, 0);
      if (base + n_idle >= n_all) drained = true;
      const uint32_t v = base + lane_prefix(idle);
      if (!busy && v < n_all) {
        shadow = v >= n_e;
        item = shadow ? share_item(v - n_e, ns, wg, G) : share_item(v, ne, wg, G);
        st.sp = 0;
        if (shadow) cs.start(item, L);
        else es.start(item, L);
        L.any = shadow;
        busy = true;
        rv = rt = ri = 0;
      }
    }
    if (__ballot(busy) == 0) break;
    bool go = busy;
    if (kLeafWait) {
      // a lane at a leaf waits while there are many more lanes at inner
      // nodes, so that fewer iterations run both the node and the triangle
      // code
      const bool at_leaf = busy && L.cur != kEmpty && ref_is_leaf(L.cur);
      const uint32_t n_leaf = (uint32_t)__popcll((unsigned long long)__ballot(at_leaf));
      const uint32_t n_node = (uint32_t)__popcll((unsigned long long)__ballot(busy && !at_leaf));
      go = busy && (!at_leaf || kLeafWait * n_leaf >= kLeafWaitDen * n_node);
    }
    if (go && lane_step<kWalkPerLane, COUNT, TWO>(S, L, st, rv, rt, ri)) {
      const bool found = L.best.tri != 0xFFFFFFFFu;
      if (shadow) cs.finish(item, L, found);
      else es.finish(item, L, found);
      if (COUNT) {
        ninst += ri;
        if (shadow) {
          svis += rv;
          stri += rt;
        } else {
          nvis += rv;
          ntri += rt;
        }
      }
      busy = false;
    }
  }
  if (COUNT) {
    atomicAdd(&P.stats[kStatNodes], (unsigned long long)nvis);
    atomicAdd(&P.stats[kStatTris], (unsigned long long)ntri);
    atomicAdd(&P.stats[kStatShadowNodes], (unsigned long long)svis);
    atomicAdd(&P.stats[kStatShadowTris], (unsigned long long)stri);
    if (TWO) atomicAdd(&P.stats[kStatInstances], (unsigned long long)ninst);
  }
  if (nonfinite) atomicAdd(&P.stats[kStatNonFinite], nonfinite);
  if (st.overflow) atomicAdd(&P.stats[kStatOverflow], 1ull);
}

// -------------------------------------------------------------------- tail
// Once few paths remain, one persistent-lane kernel finishes them: a lane
// takes a path and runs all its remaining vertices (closest hit, shading,
// shadow ray, next ray) with no kernel boundary between vertices, so short
// paths do not wait for the slowest ray of every later bounce.  Shading,
// walks and signatures are the same code as the wavefront kernels'.
template <bool DEBUG, bool TWO>
__device__ inline void shade_any(int cls, const SceneDev& S, const PathsDev& P, uint32_t slot, int b, int max_depth,
                                 uint32_t sample, uint32_t k0, uint32_t k1, uint32_t img_w, int nrc_bounce,
                                 ShadeOut& o, unsigned long long& nf) {
  const int q = nrc_bounce;
  switch (cls) {
    case kClsMiss: shade_one<kClsMiss, DEBUG, TWO>(S, P, slot, b, max_depth, sample, k0, k1, img_w, q, o, nf); break;
    case kClsAbsorb: shade_one<kClsAbsorb, DEBUG, TWO>(S, P, slot, b, max_depth, sample, k0, k1, img_w, q, o, nf); break;
    case kClsDiffuse: shade_one<kClsDiffuse, DEBUG, TWO>(S, P, slot, b, max_depth, sample, k0, k1, img_w, q, o, nf); break;
    case kClsMetal: shade_one<kClsMetal, DEBUG, TWO>(S, P, slot, b, max_depth, sample, k0, k1, img_w, q, o, nf); break;
    case kClsPlastic: shade_one<kClsPlastic, DEBUG, TWO>(S, P, slot, b, max_depth, sample, k0, k1, img_w, q, o, nf); break;
    case kClsGlass: shade_one<kClsGlass, DEBUG, TWO>(S, P, slot, b, max_depth, sample, k0, k1, img_w, q, o, nf); break;
    default: shade_one<kClsGeneral, DEBUG, TWO>(S, P, slot, b, max_depth, sample, k0, k1, img_w, q, o, nf); break;
  }
}

template <bool DEBUG, bool COUNT, bool TWO>
__global__ __launch_bounds__(kBlock) void k_tail(SceneDev S, PathsDev P, int cur, int b_first, int max_depth,
                                                 uint32_t sample, uint32_t k0, uint32_t k1, uint32_t img_w,
                                                 int nrc_bounce) {
  __shared__ unsigned long long s_stack[kLdsStack * kBlock];
  const uint32_t count = P.counts[cur];
#if PT_TAIL_DYNAMIC
  // every wave takes paths from one device-wide counter (zeroed before the
  // launch), so the longest paths do not pile up in one workgroup's share
  uint32_t* next_path = &P.counts[kCountTail];
  const uint32_t q1 = count;
#else
  __shared__ uint32_t s_next;
  const uint32_t per = (count + gridDim.x - 1) / gridDim.x;
  const uint32_t q0 = min(count, blockIdx.x * per), q1 = min(count, q0 + per);
  if (threadIdx.x == 0) s_next = q0;
  __syncthreads();
  uint32_t* next_path = &s_next;
#endif
  const uint32_t gtid = blockIdx.x * kBlock + threadIdx.x;
  DevStack st{lds_stack_base(s_stack), S.spill + gtid, S.spill_stride, 0, S.stack_cap, false};
  LaneRay L;
  // 0 idle, 1 closest-hit walk, 2 shadow-ray walk, 3 hit found and waiting to be shaded
  int phase = 0;
  bool drained = false, cont = false;
  uint32_t slot = 0;
  int b = b_first, cls = kClsMiss;
  float4 sh_c = make_float4(0, 0, 0, 0);
  uint32_t n_ext = 0, n_sh = 0, nvis = 0, ntri = 0, svis = 0, stri = 0;
  unsigned long long nonfinite = 0;
  bool overflow = false;
  uint32_t rv = 0, rt = 0, ri = 0;  // node visits / triangle tests / instances entered of the current walk
  uint32_t ninst = 0;
  auto start_closest = [&](void) {
    float4 o = P.ray_o[slot], d = P.ray_d[slot];
    st.sp = 0;
    lane_start<TWO>(L, o.x, o.y, o.z, d.x, d.y, d.z, S.tmin, INFINITY, f2u(d.w), f2u(o.w), TWO ? 0u : S.root);
    L.any = false;
    rv = rt = ri = 0;
    phase = 1;
    n_ext++;
  };
  while (true) {
    const uint64_t idle = __ballot(phase == 0);
    const uint32_t n_idle = (uint32_t)__popcll((unsigned long long)idle);
    if (!drained && (n_idle >= kRefill || n_idle == 64u)) {
      uint32_t base = 0;
      if (lane_id() == 0) base = atomicAdd(next_path, n_idle);
      base = __shfl(base, 0);
      if (base + n_idle >= q1) drained = true;
      const uint32_t i = base + lane_prefix(idle);
      if (phase == 0 && i < q1) {
        slot = P.q_ray[cur][i];
        b = b_first;
        start_closest();
      }
    }
    if (__ballot(phase != 0) == 0) break;
    // closest-hit and shadow walks share one walk step (kind per lane); a
    // lane at a leaf waits while lanes at inner nodes outnumber it
    const bool walking = phase == 1 || phase == 2;
    bool go = walking;
    if (kLeafWait) {
      const bool at_leaf = walking && L.cur != kEmpty && ref_is_leaf(L.cur);
      const uint32_t n_leaf = (uint32_t)__popcll((unsigned long long)__ballot(at_leaf));
      const uint32_t n_node = (uint32_t)__popcll((unsigned long long)__ballot(walking && !at_leaf));
      go = walking && (!at_leaf || kLeafWait * n_leaf >= kLeafWaitDen * n_node);
    }
    const bool done = go && lane_step<kWalkPerLane, COUNT, TWO>(S, L, st, rv, rt, ri);
    if (done && COUNT) {
      ninst += ri;
      if (phase == 1) {
        nvis += rv;
        ntri += rt;
      } else {
        svis += rv;
        stri += rt;
      }
    }
    if (phase == 1) {
      if (done) {
        overflow |= st.overflow;
        cls = kClsMiss;
        if (L.best.tri != 0xFFFFFFFFu) {
          P.hit[slot] = make_float4(L.best.t, L.best.b1, L.best.b2, u2f(L.best.tri));
          uint32_t mid = L.best.mat;
          if (TWO) {
            P.hit_inst[slot] = L.best.inst;
            int32_t ov = S.insts[L.best.inst].mat_override;
            if (ov >= 0) mid = (uint32_t)ov;
          }
          cls = S.mats[mid].cls;
        } else {
          P.hit[slot] = make_float4(INFINITY, 0.0f, 0.0f, u2f(0xFFFFFFFFu));
        }
        phase = 3;
      }
    } else if (phase == 2) {
      if (done) {
        overflow |= st.overflow;
        const bool occ = L.best.tri != 0xFFFFFFFFu;
        if (!occ) {
          V3 cc = v3(sh_c.x, sh_c.y, sh_c.z);
          if (finite3(cc)) {
            float4 Lr = P.L[slot];
            P.L[slot] = make_float4(Lr.x + cc.x, Lr.y + cc.y, Lr.z + cc.z, Lr.w);
          } else {
            nonfinite++;
          }
        }
        if (DEBUG) {
          uint64_t sig = P.sig[slot];
          sig = sig_word(sig, 5);
          sig = sig_word(sig, P.dbg_nee[slot]);
          sig = sig_word(sig, occ ? 1u : 0u);
          sig = sig_tail(sig, P.dbg_tail[slot]);
          P.sig[slot] = sig;
        }
        if (cont) {
          b++;
          start_closest();
        } else {
          phase = 0;
        }
      }
    }
    // Shading is a long stretch of code per material class.  Lanes that found
    // their hit wait until they are at least as many as the lanes still
    // walking (or until no lane walks), so that one pass over the shading code
    // serves many lanes instead of one pass per walk that ends.
    const uint32_t n_ready = (uint32_t)__popcll((unsigned long long)__ballot(phase == 3));
    const uint32_t n_walk = (uint32_t)__popcll((unsigned long long)__ballot(phase == 1 || phase == 2));
    if (n_ready && kTailShadeWait * n_ready >= n_walk && phase == 3) {
      ShadeOut o;
      shade_any<DEBUG, TWO>(cls, S, P, slot, b, max_depth, sample, k0, k1, img_w, nrc_bounce, o, nonfinite);
      // paths that ended in the radiance cache join its query queue (one atomic per wave)
      const uint64_t m_q = __ballot(o.query);
      if (m_q) {
        const int leader = __ffsll((long long)m_q) - 1;
        uint32_t qbase = 0;
        if ((int)lane_id() == leader) qbase = atomicAdd(&P.counts[kCountQuery], (uint32_t)__popcll(m_q));
        qbase = __shfl(qbase, leader);
        if (o.query) P.q_nrc[qbase + lane_prefix(m_q)] = slot;
      }
      if (o.shadow) {
        st.sp = 0;
        lane_start<TWO>(L, o.sh_o.x, o.sh_o.y, o.sh_o.z, o.sh_d.x, o.sh_d.y, o.sh_d.z, S.tmin, o.sh_o.w,
                        TWO ? o.sh_inst : 0u, f2u(o.sh_c.w), TWO ? 0u : S.root);
        L.any = true;
        rv = rt = ri = 0;
        sh_c = o.sh_c;
        cont = o.cont;
        phase = 2;
        n_sh++;
      } else if (o.cont) {
        b++;
        start_closest();
      } else {
        phase = 0;
      }
    }
  }
  // statistics: one atomic per wave and counter
  n_ext = wave_sum(n_ext);
  n_sh = wave_sum(n_sh);
  if (lane_id() == 0) {
    atomicAdd(&P.stats[kStatExt], (unsigned long long)n_ext);
    atomicAdd(&P.stats[kStatTailExt], (unsigned long long)n_ext);
    atomicAdd(&P.stats[kStatShadow], (unsigned long long)n_sh);
    atomicAdd(&P.stats[kStatTailShadow], (unsigned long long)n_sh);
  }
  if (COUNT) {
    atomicAdd(&P.stats[kStatTailNodes], (unsigned long long)nvis);
    atomicAdd(&P.stats[kStatTailTris], (unsigned long long)ntri);
    atomicAdd(&P.stats[kStatTailShadowNodes], (unsigned long long)svis);
    atomicAdd(&P.stats[kStatTailShadowTris], (unsigned long long)stri);
    if (TWO) atomicAdd(&P.stats[kStatTailInstances], (unsigned long long)ninst);
  }
  if (nonfinite) atomicAdd(&P.stats[kStatNonFinite], nonfinite);
  if (overflow) atomicAdd(&P.stats[kStatOverflow], 1ull);
}

// -------------------------------------------------------------- accumulate
// FP64 per-pixel running sums: one writer per pixel per pass, no atomics.
__global__ __launch_bounds__(kBlock) void k_accumulate(PathsDev P, double* sum, int W, float* per_sample,
                                                       uint64_t* sig_out, int spp_total, int sample_index) {
  for (int slot = blockIdx.x * kBlock + threadIdx.x; slot < P.n_render; slot += gridDim.x * kBlock) {
    float4 L = P.L[slot];
    if (sum) {
      int px = P.x0 + slot % P.w, py = P.y0 + slot / P.w;
      double* s = sum + 3 * ((size_t)py * W + px);
      s[0] += (double)L.x;
      s[1] += (double)L.y;
      s[2] += (double)L.z;
    }
    if (per_sample) {
      size_t o = (size_t)slot * spp_total + sample_index;
      per_sample[3 * o] = L.x;
      per_sample[3 * o + 1] = L.y;
      per_sample[3 * o + 2] = L.z;
      sig_out[o] = P.sig[slot];
    }
  }
}

__global__ __launch_bounds__(kBlock) void k_resolve(const double* sum, float* out, int64_t n, double inv) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock)
    out[i] = (float)(sum[i] * inv);
}

__global__ __launch_bounds__(kBlock) void k_zero_f64(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0.0;
}

__global__ __launch_bounds__(kBlock) void k_zero_u64(unsigned long long* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)kBlock + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBlock) p[i] = 0ull;
}

// ------------------------------------------------------- ray query kernels
// Closest hits of a ray array ([n][8]: o, tmin, d, tmax) -> [n][6] words.
__device__ inline void write_hit(uint32_t* H, const Hit& h) {
  bool hit = h.tri != 0xFFFFFFFFu;
  H[0] = f2u(h.t);
  H[1] = hit ? h.inst : 0xFFFFFFFFu;
  H[2] = hit ? h.prim : 0xFFFFFFFFu;
  H[3] = hit ? f2u(h.b1) : 0u;
  H[4] = hit ? f2u(h.b2) : 0u;
  H[5] = hit ? 1u : 0u;
}

template <bool TWO>
struct RaysSrc {
  const SceneDev& S;
  const float* rays;
  uint32_t* hits;
  __device__ inline void start(uint32_t i, LaneRay& L) {
    const float* R = rays + 8 * (size_t)i;
    lane_start<TWO>(L, R[0], R[1], R[2], R[4], R[5], R[6], R[3], R[7], 0xFFFFFFFFu, 0xFFFFFFFFu, TWO ? 0u : S.root);
  }
  __device__ inline void finish(uint32_t i, const LaneRay& L, bool) { write_hit(hits + 6 * (size_t)i, L.best); }
};

template <bool TWO>
__global__ __launch_bounds__(kBlock) void k_trace_rays(SceneDev S, const float* rays, uint32_t n, uint32_t* hits,
                                                       unsigned long long* stats) {
  __shared__ unsigned long long s_stack[kLdsStack * kBlock];
  __shared__ uint32_t s_next;
  uint32_t nvis = 0, ntri = 0;
  bool overflow = false;
  RaysSrc<TWO> src{S, rays, hits};
  persistent_trace<kWalkClosest, false, TWO>(S, src, n, s_stack, &s_next, nvis, ntri, overflow);
  if (overflow) atomicAdd(&stats[kStatOverflow], 1ull);
}

// The same definition by testing every triangle (and every instance).
template <bool TWO>
__global__ __launch_bounds__(kBlock) void k_trace_rays_brute(SceneDev S, const float* rays, uint32_t n,
                                                             uint32_t* hits) {
  for (uint32_t i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
    const float* R = rays + 8 * (size_t)i;
    Hit h;
    hit_clear(h);
    uint32_t nt = 0;
    RayPre r = ray_prepare(R[0], R[1], R[2], R[4], R[5], R[6]);
    if (TWO) brute_force_two_level(S.insts, S.n_insts, S.tris, S.mesh_tri_first, S.mesh_tri_count, r, R[3], R[7], h);
    else brute_force<false>(S.tris, S.n_tris, r, R[3], R[7], 0u, h, nt);
    write_hit(hits + 6 * (size_t)i, h);
  }
}

// --------------------------------------------------------------- launchers
int trace_grid_blocks() { return 2048; }

// Workgroups of the tail kernel.  Alone, every resident workgroup (about one
// path per lane: the tail ends with its longest path).  Beside the next
// pass's dense bounces (second stream), about three paths per lane and at
// most one workgroup per CU, which leaves most of each CU to them.
int tail_grid(int grid_trace, uint32_t paths, bool beside) {
  static int cus = 0, resident = 0;
  if (!cus) {
    int dev = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_tail<true, true, true>, kBlock, 0) != hipSuccess ||
        per < 1)
      per = 1;
    resident = cus * per;
  }
  if (!beside) return std::max(1, std::min(grid_trace, resident));
  int want = (int)std::min<uint64_t>((uint64_t)cus, std::max<uint64_t>(8, ((uint64_t)paths + kTailPathsPerGroup - 1) /
                                                                                 kTailPathsPerGroup));
  return std::max(1, std::min(grid_trace, want));
}

// The traversal kernels keep one resident set of workgroups (persistent
// lanes); more would only queue behind them.
int traversal_grid(int64_t rays) {
  int64_t need = std::max<int64_t>(1, (rays + kBlock - 1) / kBlock);
  static int resident = 0;
  if (!resident) {
    int dev = 0, cus = 0, per = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
      cus = 256;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k_traverse<true, true, true>, kBlock, 0) != hipSuccess ||
        per < 1)
      per = 1;
    resident = std::max(1, cus * per);
  }
  return (int)std::min<int64_t>(need, resident);
}

template <bool DEBUG, bool TWO>
static hipError_t shade_all(const SceneDev& S, const PathsDev& P, const PassArgs& A, int b, int next, uint32_t W,
                            hipStream_t st) {
  // The class kernels touch disjoint path slots and append through atomics,
  // so with side streams they run concurrently (each is bound by the
  // latency of its own dependent loads): class i of those present goes to
  // stream i mod 3 (0: the pass's stream), which then waits for the others.
  hipStream_t lane[3] = {st, A.shade_side[0], A.shade_side[1]};
  int n_streams = A.shade_side[0] && A.shade_side[1] ? 3 : 1, used = 0;
  dim3 g(std::max(1, A.grid * kBlock / kShadeBlock / (n_streams > 1 ? PT_SHADE_GRID_DIV : 1))), blk(kShadeBlock);
  bool forked = false;
  for (int c = 0; c < kNumClasses; ++c) {
    if (!(A.class_mask & (1u << c))) continue;
    hipStream_t q = lane[used % n_streams];
    if (q != st && !forked) {
      hipError_t e = hipEventRecord(A.shade_fork, st);
      if (e == hipSuccess) e = hipStreamWaitEvent(A.shade_side[0], A.shade_fork, 0);
      if (e == hipSuccess) e = hipStreamWaitEvent(A.shade_side[1], A.shade_fork, 0);
      if (e != hipSuccess) return e;
      forked = true;
    }
    ++used;
    switch (c) {
#define PT_SHADE(C)                                                                                      \
  case C:                                                                                                \
    hipLaunchKernelGGL((k_shade<C, DEBUG, TWO>), g, blk, 0, q, S, P, b, A.max_depth, next, A.sample, A.k0, \
                       A.k1, W, A.nrc_bounce);                                                           \
    break;
      PT_SHADE(kClsMiss)
      PT_SHADE(kClsAbsorb)
      PT_SHADE(kClsDiffuse)
      PT_SHADE(kClsMetal)
      PT_SHADE(kClsPlastic)
      PT_SHADE(kClsGlass)
      PT_SHADE(kClsGeneral)
#undef PT_SHADE
    }
  }
  if (forked) {
    for (int k = 0; k < 2; ++k) {
      hipError_t e = hipEventRecord(A.shade_join[k], A.shade_side[k]);
      if (e == hipSuccess) e = hipStreamWaitEvent(st, A.shade_join[k], 0);
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

template <bool DEBUG, bool COUNT, bool TWO>
static hipError_t bounce_loop(const SceneDev& S, const PathsDev& P, const CamDev& C, const PassArgs& A,
                              hipStream_t st) {
  dim3 blk(kBlock);
  if (A.wavefront_bounces) *A.wavefront_bounces = A.max_depth + 1;
  int n_trace = 0;
  // closest hits of queue q (none if q < 0) and the shadow rays of the last shading, on stream on
  auto traverse = [&](int q, hipStream_t on) {
    if (A.ext_events) hipEventRecord(A.ext_events[2 * n_trace], on);
    hipLaunchKernelGGL((k_traverse<DEBUG, COUNT, TWO>), dim3(A.grid_trace), blk, 0, on, S, P, q);
    if (A.ext_events) hipEventRecord(A.ext_events[2 * n_trace + 1], on);
    n_trace++;
  };
  bool shadow_pending = false;  // the last shading queued shadow rays that no launch has traced yet
  bool query_pending = false;   // the cache queries wait for the tail kernel's stream
  auto query = [&](hipStream_t q) -> hipError_t {
    if (A.query_wait) {  // the weights of the last training must be in place
      hipError_t e1 = hipStreamWaitEvent(q, A.query_wait, 0);
      if (e1 != hipSuccess) return e1;
    }
    if (A.nrc_events) hipEventRecord(A.nrc_events[0], q);
    hipError_t e2 = nrc_launch_query(P, A.nrc_fwd, std::min(A.grid, 1024), q);
    if (A.nrc_events) hipEventRecord(A.nrc_events[1], q);
    return e2;
  };
  for (int b = 0; b <= A.max_depth; ++b) {
    int cur = b & 1, next = cur ^ 1;
    if (A.tail_host_count && b >= A.tail_min_bounce) {
      // hand the remaining vertices to one persistent kernel once few paths are left
      if (A.tail_bound && A.nrc_bounce >= 0 && b > A.nrc_bounce &&
          (double)A.tail_bound <= A.tail_fraction * (double)P.n) {
        *A.tail_host_count = A.tail_bound;  // a bound known on the host: no need to read the count
      } else {
        hipError_t e0 = hipMemcpyAsync(A.tail_host_count, &P.counts[cur], sizeof(uint32_t), hipMemcpyDeviceToHost, st);
        if (e0 == hipSuccess) e0 = hipStreamSynchronize(st);
        if (e0 != hipSuccess) return e0;
      }
      if ((double)*A.tail_host_count <= A.tail_fraction * (double)P.n) {
        if (A.wavefront_bounces) *A.wavefront_bounces = b;
        hipStream_t ts = st;
        if (A.tail_stream) {  // continue on the second stream; the caller's stream is free for the next pass
          hipError_t e1 = hipEventRecord(A.tail_ready, st);
          if (e1 == hipSuccess) e1 = hipStreamWaitEvent(A.tail_stream, A.tail_ready, 0);
          if (e1 != hipSuccess) return e1;
          ts = A.tail_stream;
          if (A.tail_launched) *A.tail_launched = true;
        }
        if (shadow_pending) {  // the previous vertex's shadow rays come before the tail's next vertex
          traverse(-1, ts);
          shadow_pending = false;
        }
        if (query_pending) {  // the queries run on the tail kernel's stream, before it
          hipError_t e2 = query(ts);
          if (e2 != hipSuccess) return e2;
          query_pending = false;
        }
        if (PT_TAIL_DYNAMIC) hipLaunchKernelGGL(k_zero_u32, dim3(1), dim3(1), 0, ts, P.counts + kCountTail);
        if (A.tail_events) hipEventRecord(A.tail_events[0], ts);
        hipLaunchKernelGGL((k_tail<DEBUG, COUNT, TWO>),
                           dim3(tail_grid(A.grid_trace, *A.tail_host_count, A.tail_stream != nullptr)), blk, 0, ts,
                           S, P, cur, b, A.max_depth, A.sample, A.k0, A.k1, (uint32_t)C.W, A.nrc_bounce);
        if (A.tail_events) hipEventRecord(A.tail_events[1], ts);
        if (A.nrc_bounce >= 0 && b <= A.nrc_bounce) {
          // the tail kernel took over at or before the query vertex: the paths it ends in the
          // cache join the query queue, so the queries run after it, on its stream
          hipError_t e2 = query(ts);
          if (e2 != hipSuccess) return e2;
        }
        break;
      }
    }
    hipLaunchKernelGGL(k_reset_counts, dim3(1), dim3(64), 0, st, P.counts, next);
    traverse(cur, st);  // this bounce's closest hits and the previous bounce's shadow rays
    shadow_pending = false;
    hipLaunchKernelGGL(k_bin, dim3(A.grid_bin), blk, 0, st, P, cur);  // also empties the shadow queue
    hipError_t e = shade_all<DEBUG, TWO>(S, P, A, b, next, (uint32_t)C.W, st);
    if (e != hipSuccess) return e;
    shadow_pending = b < A.max_depth;
    if (b == A.nrc_bounce) {  // every path still alive ended in the cache at this vertex
      // (a path that ends in the cache casts no shadow ray at that vertex, so
      // the pending shadow rays touch other paths; the queries touch only the
      // paths that ended here, so they can wait for the tail kernel's stream)
      if (A.query_beside && A.tail_stream && P.n > P.n_render) {
        query_pending = true;
      } else {
        hipError_t e2 = query(st);
        if (e2 != hipSuccess) return e2;
      }
      if (P.n == P.n_render) break;  // no training paths: nothing continues
    }
  }
  if (shadow_pending) traverse(-1, st);
  if (query_pending) {  // no hand-off: the queries run here after all
    hipError_t e2 = query(st);
    if (e2 != hipSuccess) return e2;
  }
  if (A.trace_launches) *A.trace_launches = n_trace;
  return hipGetLastError();
}

hipError_t launch_pass(const SceneDev& S, const PathsDev& P, const CamDev& C, const PassArgs& A, hipStream_t st) {
  dim3 blk(kBlock);
  if (A.debug) hipLaunchKernelGGL((k_generate<true>), dim3(A.grid), blk, 0, st, P, C, A.sample, A.k0, A.k1);
  else hipLaunchKernelGGL((k_generate<false>), dim3(A.grid), blk, 0, st, P, C, A.sample, A.k0, A.k1);
  const int sel = (A.debug ? 4 : 0) | (A.count ? 2 : 0) | (A.two_level ? 1 : 0);
  switch (sel) {
    case 0: return bounce_loop<false, false, false>(S, P, C, A, st);
    case 1: return bounce_loop<false, false, true>(S, P, C, A, st);
    case 2: return bounce_loop<false, true, false>(S, P, C, A, st);
    case 3: return bounce_loop<false, true, true>(S, P, C, A, st);
    case 4: return bounce_loop<true, false, false>(S, P, C, A, st);
    case 5: return bounce_loop<true, false, true>(S, P, C, A, st);
    case 6: return bounce_loop<true, true, false>(S, P, C, A, st);
    default: return bounce_loop<true, true, true>(S, P, C, A, st);
  }
}

static int blocks_for(int64_t n) {
  int64_t b = (n + kBlock - 1) / kBlock;
  if (b < 1) b = 1;
  if (b > 4096) b = 4096;
  return (int)b;
}

hipError_t launch_accumulate(const PathsDev& P, double* sum, int W, float* per_sample, uint64_t* sig_out,
                             int spp_total, int sample_index, hipStream_t st) {
  hipLaunchKernelGGL(k_accumulate, dim3(blocks_for(P.n_render)), dim3(kBlock), 0, st, P, sum, W, per_sample, sig_out,
                     spp_total, sample_index);
  return hipGetLastError();
}

hipError_t launch_resolve(const double* sum, float* out, int64_t n, double inv, hipStream_t st) {
  hipLaunchKernelGGL(k_resolve, dim3(blocks_for(n)), dim3(kBlock), 0, st, sum, out, n, inv);
  return hipGetLastError();
}

hipError_t launch_zero_f64(double* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_f64, dim3(blocks_for(n)), dim3(kBlock), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_zero_u64(unsigned long long* p, int64_t n, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_u64, dim3(blocks_for(n)), dim3(kBlock), 0, st, p, n);
  return hipGetLastError();
}

hipError_t launch_trace_rays(const SceneDev& S, const float* rays, int64_t n, uint32_t* hits, bool brute,
                             bool two_level, int grid, unsigned long long* stats, hipStream_t st) {
  dim3 g(grid), blk(kBlock);
  const uint32_t nn = (uint32_t)n;
  if (brute && two_level) hipLaunchKernelGGL((k_trace_rays_brute<true>), g, blk, 0, st, S, rays, nn, hits);
  else if (brute) hipLaunchKernelGGL((k_trace_rays_brute<false>), g, blk, 0, st, S, rays, nn, hits);
  else if (two_level) hipLaunchKernelGGL((k_trace_rays<true>), g, blk, 0, st, S, rays, nn, hits, stats);
  else hipLaunchKernelGGL((k_trace_rays<false>), g, blk, 0, st, S, rays, nn, hits, stats);
  return hipGetLastError();
}

// ------------------------------------------------ allocation-free scratch
// Device memory of the allocation-free closest-hit call: a file-scope array,
// one copy per GPU, held until the process ends and shared by every call on
// that GPU.  In host code its name is not a device address: kernels receive
// the address hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
unsigned char* g_scratch_ptr[kMaxScratchDevices];
}  // namespace

hipError_t noalloc_scratch(int dev, unsigned char** out) {
  *out = nullptr;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    if (!p) return hipErrorInvalidSymbol;
    g_scratch_ptr[dev] = static_cast<unsigned char*>(p);
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

}  // namespace pt
