// GPU construction of the BVH4 for gfx950 (the paper builds its BVH on the
// CPU once per scene and times that set-up separately, Sec. 5.1.1, Table 1).
//
// Two builders share the first and last steps:
//   1. triangle boxes, and the centroid bounds by a block reduction;
//   2. 30-bit Morton codes (10 bits per axis) of the centroids in cubic
//      cells (one scale, that of the centroid box's longest side, for all
//      three axes, so that neighbours along the curve are near in space);
//   3. an LSD radix sort of (code, index): four 8-bit passes, each a tile
//      histogram, one scan over (digit, tile) and a stable scatter that ranks
//      equal digits with wave ballots;
//   then a binary tree over the sorted triangles, either
//   4a. linear BVH (Karras 2012): the binary radix tree over the sorted codes,
//      every internal node in parallel (ties between equal codes broken by
//      the index), and node boxes bottom-up (each leaf walks towards the root
//      and the second thread to reach a node merges its children's boxes); or
//   4b. locally-ordered clustering (PLOC, Meister & Bittner 2018): clusters
//      in Morton order, each finds the neighbour within kPlocRadius places
//      whose merged box has the least surface area, mutual nearest
//      neighbours merge into a new node, the rest are compacted in order,
//      until one cluster is left (a greedy bottom-up SAH tree);
//   5. a top-down collapse to 128-byte BVH4 nodes, one launch per level, by
//      least SAH cost (the dynamic program of Ylitie, Karras and Laine 2017,
//      its costs computed where the binary nodes are made): a 4-wide node
//      takes the roots of the best split of its four slots; leaf subtrees
//      place their triangles in depth-first order;
//   6. the 48-byte triangle records in that (leaf) order.
// The result has the layout of the host builder's (root at node 0, empty
// child slots kEmpty with zero boxes, meta[0] = child count); only the tree
// differs.  Every closest hit is the same, since the hit is defined by the
// triangle test alone.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "pt_internal.h"

namespace pt {
namespace {

constexpr int kBB = 256;               // threads per block
constexpr int kItems = 8;              // keys per thread and radix pass
constexpr int kTile = kBB * kItems;    // keys per radix tile
constexpr uint32_t kLeafRef = 0x80000000u;  // binary-tree child reference: leaf flag
constexpr int kMaxTreeLevels = 128;          // bound on any walk or level loop over the binary tree
#ifndef PT_PLOC_RADIUS
#define PT_PLOC_RADIUS 16
#endif
constexpr int kPlocRadius = PT_PLOC_RADIUS;  // clusters searched on either side
#ifndef PT_MORTON_CUBE
#define PT_MORTON_CUBE 1  // 1: Morton cells are cubes (one scale for the three axes), 0: one scale per axis
#endif
constexpr int kPlocMaxRounds = 4096;         // bound on the clustering rounds
constexpr int kPlocBatch = 8;                // rounds enqueued between two reads of the cluster count
constexpr int kCollapseBatch = 8;            // collapse levels enqueued between two reads of the job count
#ifndef PT_GPU_COLLAPSE_DP
#define PT_GPU_COLLAPSE_DP 1
#endif
// 1: BVH4 nodes by least SAH cost over the binary tree; 0: each node opens its largest-area children
constexpr bool kGpuCollapseDp = PT_GPU_COLLAPSE_DP != 0;
#ifndef PT_SAH_TRAVERSAL
#define PT_SAH_TRAVERSAL 1.0
#endif
constexpr float kSahNode = (float)PT_SAH_TRAVERSAL;  // a node step, in triangle tests
// binary-node triangle counts carry this bit when the subtree becomes one BVH4 leaf
constexpr uint32_t kLeafBitCnt = 0x80000000u;

// Float <-> order-preserving unsigned, for atomic min / max of floats.
__device__ inline uint32_t f2ord(float f) {
  uint32_t u = __float_as_uint(f);
  return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
__device__ inline float ord2f(uint32_t u) { return __uint_as_float((u & 0x80000000u) ? (u & 0x7FFFFFFFu) : ~u); }

__device__ inline uint32_t spread10(uint32_t v) {  // the 10 low bits of v to every third bit
  v &= 0x3FFu;
  v = (v | (v << 16)) & 0x030000FFu;
  v = (v | (v << 8)) & 0x0300F00Fu;
  v = (v | (v << 4)) & 0x030C30C3u;
  v = (v | (v << 2)) & 0x09249249u;
  return v;
}

// 1. boxes [n][6] (lo xyz, hi xyz) and centroid bounds cb[6] (ordered min xyz, max xyz)
__global__ __launch_bounds__(kBB) void k_tri_boxes(const float* __restrict__ soup, int64_t n, float* __restrict__ box,
                                                   uint32_t* __restrict__ cb) {
  __shared__ float red[6][kBB];
  float cmin[3] = {INFINITY, INFINITY, INFINITY}, cmax[3] = {-INFINITY, -INFINITY, -INFINITY};
  for (int64_t i = blockIdx.x * (int64_t)kBB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBB) {
    const float* p = soup + 9 * i;
    float lo[3], hi[3];
    for (int k = 0; k < 3; ++k) {
      lo[k] = fminf(fminf(p[k], p[3 + k]), p[6 + k]);
      hi[k] = fmaxf(fmaxf(p[k], p[3 + k]), p[6 + k]);
      box[6 * i + k] = lo[k];
      box[6 * i + 3 + k] = hi[k];
      const float c = 0.5f * (lo[k] + hi[k]);
      cmin[k] = fminf(cmin[k], c);
      cmax[k] = fmaxf(cmax[k], c);
    }
  }
  for (int k = 0; k < 3; ++k) {
    red[k][threadIdx.x] = cmin[k];
    red[3 + k][threadIdx.x] = cmax[k];
  }
  __syncthreads();
  for (int off = kBB / 2; off > 0; off >>= 1) {
    if ((int)threadIdx.x < off)
      for (int k = 0; k < 3; ++k) {
        red[k][threadIdx.x] = fminf(red[k][threadIdx.x], red[k][threadIdx.x + off]);
        red[3 + k][threadIdx.x] = fmaxf(red[3 + k][threadIdx.x], red[3 + k][threadIdx.x + off]);
      }
    __syncthreads();
  }
  if (threadIdx.x < 3) {
    atomicMin(&cb[threadIdx.x], f2ord(red[threadIdx.x][0]));
    atomicMax(&cb[3 + threadIdx.x], f2ord(red[3 + threadIdx.x][0]));
  }
}

__global__ void k_init_bounds(uint32_t* cb) {
  if (threadIdx.x < 3) cb[threadIdx.x] = 0xFFFFFFFFu;        // min: +inf of the order
  else if (threadIdx.x < 6) cb[threadIdx.x] = 0u;            // max: -inf of the order
}

// 2. Morton code of the centroid normalised to the centroid bounds; value = triangle index
__global__ __launch_bounds__(kBB) void k_morton(const float* __restrict__ box, int64_t n,
                                                const uint32_t* __restrict__ cb, uint32_t* __restrict__ key,
                                                uint32_t* __restrict__ val) {
  float lo[3], sc[3], ext[3], emax = 0.0f;
  for (int k = 0; k < 3; ++k) {
    lo[k] = ord2f(cb[k]);
    ext[k] = ord2f(cb[3 + k]) - lo[k];
    emax = fmaxf(emax, ext[k]);
  }
  for (int k = 0; k < 3; ++k) {
    const float e = PT_MORTON_CUBE ? emax : ext[k];
    sc[k] = e > 0.0f ? 1024.0f / e : 0.0f;
  }
  for (int64_t i = blockIdx.x * (int64_t)kBB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBB) {
    uint32_t q[3];
    for (int k = 0; k < 3; ++k) {
      const float c = 0.5f * (box[6 * i + k] + box[6 * i + 3 + k]);
      const float t = (c - lo[k]) * sc[k];
      q[k] = (uint32_t)fminf(fmaxf(t, 0.0f), 1023.0f);
    }
    key[i] = (spread10(q[0]) << 2) | (spread10(q[1]) << 1) | spread10(q[2]);
    val[i] = (uint32_t)i;
  }
}

// 3. radix sort passes over tiles of kTile keys (block b: keys [b kTile, (b + 1) kTile))
__global__ __launch_bounds__(kBB) void k_radix_hist(const uint32_t* __restrict__ key, int64_t n, int shift,
                                                    uint32_t* __restrict__ hist, int nb) {
  __shared__ uint32_t h[256];
  h[threadIdx.x] = 0u;
  __syncthreads();
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + r * kBB + threadIdx.x;
    if (i < n) atomicAdd(&h[(key[i] >> shift) & 0xFFu], 1u);
  }
  __syncthreads();
  hist[(size_t)threadIdx.x * nb + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of m counts in place (one workgroup of 1024 threads)
__global__ __launch_bounds__(1024) void k_scan_excl(uint32_t* __restrict__ a, int64_t m) {
  __shared__ uint32_t part[1024];
  const int64_t per = (m + 1023) / 1024;
  const int64_t k0 = std::min<int64_t>(m, (int64_t)threadIdx.x * per), k1 = std::min<int64_t>(m, k0 + per);
  uint32_t local = 0;
  for (int64_t k = k0; k < k1; ++k) local += a[k];
  part[threadIdx.x] = local;
  __syncthreads();
  for (int off = 1; off < 1024; off <<= 1) {
    const uint32_t v = threadIdx.x >= (unsigned)off ? part[threadIdx.x - off] : 0u;
    __syncthreads();
    part[threadIdx.x] += v;
    __syncthreads();
  }
  uint32_t run = part[threadIdx.x] - local;
  for (int64_t k = k0; k < k1; ++k) {
    const uint32_t c = a[k];
    a[k] = run;
    run += c;
  }
}

// Stable scatter: within each round of 256 keys a key's rank among equal
// digits comes from its wave's ballots (lane order) and the counts of the
// waves before it; rounds run in order and carry a per-digit running offset.
__global__ __launch_bounds__(kBB) void k_radix_scatter(const uint32_t* __restrict__ kin,
                                                       const uint32_t* __restrict__ vin, uint32_t* __restrict__ kout,
                                                       uint32_t* __restrict__ vout, int64_t n, int shift,
                                                       const uint32_t* __restrict__ offs, int nb) {
  __shared__ uint32_t run[256];
  __shared__ uint32_t wcnt[kBB / 64][256];
  const int tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
  run[tid] = offs[(size_t)tid * nb + blockIdx.x];
  for (int w = 0; w < kBB / 64; ++w) wcnt[w][tid] = 0u;
  __syncthreads();
  const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
  const int64_t base = (int64_t)blockIdx.x * kTile;
  for (int r = 0; r < kItems; ++r) {
    const int64_t i = base + r * kBB + tid;
    const bool valid = i < n;
    const uint32_t k = valid ? kin[i] : 0u, v = valid ? vin[i] : 0u;
    const uint32_t d = (k >> shift) & 0xFFu;
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
      const bool bit = ((d >> b) & 1u) != 0u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = (uint32_t)__popcll(peers & lt);
    if (valid && rank == 0u) wcnt[wave][d] = (uint32_t)__popcll(peers);
    __syncthreads();
    if (valid) {
      uint32_t pos = run[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcnt[w][d];
      kout[pos] = k;
      vout[pos] = v;
    }
    __syncthreads();
    uint32_t tot = 0u;
    for (int w = 0; w < kBB / 64; ++w) {
      tot += wcnt[w][tid];
      wcnt[w][tid] = 0u;
    }
    run[tid] += tot;
    __syncthreads();
  }
}

// 4a. binary radix tree (n - 1 internal nodes).  Child references: leaf
// (kLeafRef | sorted index) or internal node index; parents of leaves and of
// internal nodes (-1 for the root); the number of triangles under each node.
__device__ inline int delta(const uint32_t* key, int64_t n, int64_t i, int64_t j) {
  if (j < 0 || j >= n) return -1;
  const uint32_t a = key[i], b = key[j];
  if (a == b) return 32 + __clz((uint32_t)i ^ (uint32_t)j);
  return __clz(a ^ b);
}

__global__ __launch_bounds__(kBB) void k_radix_tree(const uint32_t* __restrict__ key, int64_t n,
                                                    uint2* __restrict__ child, int32_t* __restrict__ parent_leaf,
                                                    int32_t* __restrict__ parent_int, uint32_t* __restrict__ cnt,
                                                    uint32_t* __restrict__ err) {
  for (int64_t i = blockIdx.x * (int64_t)kBB + threadIdx.x; i < n - 1; i += (int64_t)gridDim.x * kBB) {
    const int d = delta(key, n, i, i + 1) - delta(key, n, i, i - 1) >= 0 ? 1 : -1;
    const int dmin = delta(key, n, i, i - d);
    int64_t lmax = 2;
    while (delta(key, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int64_t l = 0;
    for (int64_t t = lmax >> 1; t >= 1; t >>= 1)
      if (delta(key, n, i, i + (l + t) * d) > dmin) l += t;
    const int64_t j = i + l * d;
    const int dnode = delta(key, n, i, j);
    int64_t s = 0, t = l;
    do {
      t = (t + 1) >> 1;
      if (delta(key, n, i, i + (s + t) * d) > dnode) s += t;
    } while (t > 1);
    const int64_t gamma = i + s * d + (d < 0 ? -1 : 0);
    const int64_t lo = i < j ? i : j, hi = i < j ? j : i;
    if (gamma < lo || gamma + 1 > hi) {  // only unsorted codes could get here: report, write nothing
      atomicOr(err, 1u);
      continue;
    }
    uint32_t cl, cr;
    if (lo == gamma) {
      cl = kLeafRef | (uint32_t)gamma;
      parent_leaf[gamma] = (int32_t)i;
    } else {
      cl = (uint32_t)gamma;
      parent_int[gamma] = (int32_t)i;
    }
    if (hi == gamma + 1) {
      cr = kLeafRef | (uint32_t)(gamma + 1);
      parent_leaf[gamma + 1] = (int32_t)i;
    } else {
      cr = (uint32_t)(gamma + 1);
      parent_int[gamma + 1] = (int32_t)i;
    }
    child[i] = make_uint2(cl, cr);
    const uint32_t c = (uint32_t)(hi - lo + 1);
    cnt[i] = c <= (uint32_t)kMaxLeafTris ? (c | kLeafBitCnt) : c;
  }
}

// box of a binary-tree reference: a leaf's triangle box (sorted index -> triangle) or a node box
__device__ inline void ref_box(uint32_t ref, const uint32_t* val, const float* tbox, const float* nbox, float b[6]) {
  const float* src = (ref & kLeafRef) ? tbox + 6 * (size_t)val[ref & ~kLeafRef] : nbox + 6 * (size_t)ref;
  for (int k = 0; k < 6; ++k) b[k] = src[k];
}

__device__ inline uint32_t ref_count(uint32_t ref, const uint32_t* cnt) {
  return (ref & kLeafRef) ? 1u : (cnt[ref] & ~kLeafBitCnt);
}

// the subtree of `ref` becomes one BVH4 leaf
__device__ inline bool ref_is_leaf_subtree(uint32_t ref, const uint32_t* cnt) {
  return (ref & kLeafRef) || (cnt[ref] & kLeafBitCnt);
}

// Collapse by least SAH cost (as the host builder's): per binary node o,
// dp[4 o + j - 1] is the least cost of covering its subtree with at most
// j = 1..4 roots (a root costs its area times one node step plus its
// children's costs, a leaf its area times its triangles), and dsp[o] holds,
// for j = 2..4 in bits 4 (j - 1) .. 4 (j - 1) + 3, the split of those slots
// (left count in the low two bits, right count in the high two; 0: the node
// is the one root), and in bits 16..19 the split of its own four slots when
// it is a 4-wide node.
__device__ inline void dp_of_ref(uint32_t ref, const float* dp, float tri_area, float D[4]) {
  for (int j = 0; j < 4; ++j) D[j] = (ref & kLeafRef) ? tri_area : dp[4 * (size_t)ref + j];
}

__device__ inline void dp_node(uint32_t o, bool as_leaf, uint32_t c, float area, const float Da[4], const float Db[4],
                               float* __restrict__ dp, uint32_t* __restrict__ dsp) {
  if (as_leaf) {
    for (int j = 0; j < 4; ++j) dp[4 * (size_t)o + j] = (float)c * area;
    dsp[o] = 0u;
    return;
  }
  float Ds[5];
  uint32_t ks[5] = {0u, 0u, 0u, 0u, 0u};
  for (int j = 2; j <= 4; ++j) {
    Ds[j] = INFINITY;
    for (int kl = 1; kl < j; ++kl) {
      const float v = Da[kl - 1] + Db[j - kl - 1];
      if (v < Ds[j]) {
        Ds[j] = v;
        ks[j] = (uint32_t)kl;
      }
    }
  }
  float best = kSahNode * area + Ds[4];
  uint32_t dec = 0u, bits = 0u;
  dp[4 * (size_t)o] = best;
  for (int j = 2; j <= 4; ++j) {
    if (Ds[j] < best) {
      best = Ds[j];
      dec = ks[j] | ((uint32_t)(j - (int)ks[j]) << 2);
    }
    dp[4 * (size_t)o + j - 1] = best;
    bits |= dec << (4 * (j - 1));
  }
  bits |= (ks[4] | ((4u - ks[4]) << 2)) << 16;
  dsp[o] = bits;
}

__device__ inline float half_area(const float b[6]) {
  const float dx = b[3] - b[0], dy = b[4] - b[1], dz = b[5] - b[2];
  return dx * dy + dy * dz + dz * dx;
}

// boxes bottom-up: the second arrival at a node merges both children's boxes
__global__ __launch_bounds__(kBB) void k_boxes_up(int64_t n, const uint32_t* __restrict__ val,
                                                  const float* __restrict__ tbox, const uint2* __restrict__ child,
                                                  const int32_t* __restrict__ parent_leaf,
                                                  const int32_t* __restrict__ parent_int, float* nbox,
                                                  uint32_t* flag, const uint32_t* __restrict__ cnt, float* dp,
                                                  uint32_t* dsp) {
  for (int64_t i = blockIdx.x * (int64_t)kBB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBB) {
    int32_t p = n > 1 ? parent_leaf[i] : -1;
    // a radix tree over 30-bit codes and 32-bit indices is at most 63 levels deep; the bound only
    // guards the walk against a malformed tree
    for (int level = 0; p >= 0 && level < kMaxTreeLevels; ++level) {
      // release this subtree's box, acquire the sibling's
      if (__hip_atomic_fetch_add(&flag[p], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 0u) break;
      const uint2 c = child[p];
      float a[6], b[6];
      ref_box(c.x, val, tbox, nbox, a);
      ref_box(c.y, val, tbox, nbox, b);
      float u[6];
      for (int k = 0; k < 3; ++k) {
        u[k] = fminf(a[k], b[k]);
        u[3 + k] = fmaxf(a[3 + k], b[3 + k]);
        nbox[6 * (size_t)p + k] = u[k];
        nbox[6 * (size_t)p + 3 + k] = u[3 + k];
      }
      float Da[4], Db[4];
      dp_of_ref(c.x, dp, half_area(a), Da);
      dp_of_ref(c.y, dp, half_area(b), Db);
      const uint32_t cp = cnt[p];
      dp_node((uint32_t)p, (cp & kLeafBitCnt) != 0u, cp & ~kLeafBitCnt, half_area(u), Da, Db, dp, dsp);
      p = parent_int[p];
    }
  }
}

// ---- 4b. locally-ordered clustering.  Cluster i of a round: a binary-tree
// reference cid[i] and its box cbox[i][6]; m clusters in Morton order.

__global__ __launch_bounds__(kBB) void k_ploc_init(const uint32_t* __restrict__ val, const float* __restrict__ tbox,
                                                   int64_t n, uint32_t* __restrict__ cid, float* __restrict__ cbox) {
  for (int64_t i = blockIdx.x * (int64_t)kBB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBB) {
    cid[i] = kLeafRef | (uint32_t)i;
    const float* b = tbox + 6 * (size_t)val[i];
    for (int k = 0; k < 6; ++k) cbox[6 * i + k] = b[k];
  }
}

// Nearest neighbour of every cluster: the least surface area of the merged
// box; among equal areas the nearer place, then an even lower index of the
// pair, then the lower index (one rank per pair, so mutual nearest neighbours
// always exist, and equal boxes pair up as (2k, 2k + 1)).  With `forced` the
// neighbour is the adjacent cluster of the pair (2k, 2k + 1) outright (a
// round after one that merged too few).  One block per kBB clusters, whose
// boxes and their neighbours' are staged in LDS; grid >= ceil(m / kBB).  The
// round's cluster count is mc[0] (set by the round before), and that round's
// own count mc[1]: a round that kept over 99 % pairs neighbours outright.
__global__ __launch_bounds__(kBB) void k_ploc_nn(const float* __restrict__ cbox, const uint32_t* __restrict__ mc,
                                                 int32_t* __restrict__ nn) {
  constexpr int kSpan = kBB + 2 * kPlocRadius;
  __shared__ float sb[kSpan * 6];
  const uint32_t m = mc[0];
  const bool forced = (uint64_t)m * 100u > (uint64_t)mc[1] * 99u;
  const int64_t b0 = (int64_t)blockIdx.x * kBB, s0 = b0 - kPlocRadius;
  if (b0 >= (int64_t)m) return;
  for (int t = threadIdx.x; t < kSpan * 6; t += kBB) {
    const int64_t g = s0 * 6 + t;  // float index of the staged window
    sb[t] = (g >= 0 && g < (int64_t)m * 6) ? cbox[g] : 0.0f;
  }
  __syncthreads();
  const int64_t i = b0 + threadIdx.x;
  if (i >= (int64_t)m) return;
  if (forced) {
    const int64_t j = i ^ 1;
    nn[i] = (int32_t)(j < (int64_t)m ? j : i);
    return;
  }
  const float* bi = sb + 6 * (threadIdx.x + kPlocRadius);
  float best = INFINITY;
  uint32_t bd = 0xFFFFFFFFu, blo = 0xFFFFFFFFu;
  int32_t bj = (int32_t)i;
  for (int d = -kPlocRadius; d <= kPlocRadius; ++d) {
    const int64_t j = i + d;
    if (d == 0 || j < 0 || j >= (int64_t)m) continue;
    const float* bb = sb + 6 * (threadIdx.x + kPlocRadius + d);
    float u[6];
    for (int k = 0; k < 3; ++k) {
      u[k] = fminf(bi[k], bb[k]);
      u[3 + k] = fmaxf(bi[3 + k], bb[3 + k]);
    }
    const float a = half_area(u);
    const uint32_t ad = (uint32_t)(d < 0 ? -d : d), lo = (uint32_t)(d < 0 ? j : i);
    const bool better =
        a < best || (a == best && (ad < bd || (ad == bd && ((lo & 1u) < (blo & 1u) ||
                                                            ((lo & 1u) == (blo & 1u) && lo < blo)))));
    if (better) {
      best = a;
      bd = ad;
      blo = lo;
      bj = (int32_t)j;
    }
  }
  nn[i] = bj;
}

// Mutual nearest neighbours i < j merge: a new node (children cid[i], cid[j])
// takes place i; place j is dropped (keep[j] = 0).  Only thread i reads place
// j and writes place i, so the update is in place.  The new node's SAH cost
// (surface area x (kSahNode + the children's costs), a single triangle costing
// its area) decides whether its subtree becomes one BVH4 leaf: when it holds
// at most kMaxLeafTris triangles and testing them all costs no more.
__global__ __launch_bounds__(kBB) void k_ploc_merge(uint32_t* __restrict__ cid, float* __restrict__ cbox,
                                                    const uint32_t* __restrict__ mc, const int32_t* __restrict__ nn,
                                                    uint2* __restrict__ child, float* __restrict__ nbox,
                                                    uint32_t* __restrict__ cnt, float* __restrict__ ncost,
                                                    float* __restrict__ dp, uint32_t* __restrict__ dsp,
                                                    uint32_t* __restrict__ n_int, uint32_t cap,
                                                    uint32_t* __restrict__ keep, uint32_t* __restrict__ err) {
  const uint32_t m = mc[0];
  for (int64_t i = blockIdx.x * (int64_t)kBB + threadIdx.x; i < (int64_t)m; i += (int64_t)gridDim.x * kBB) {
    const int32_t j = nn[i];
    const bool mutual = j != (int32_t)i && j >= 0 && j < (int32_t)m && nn[j] == (int32_t)i;
    if (mutual && j < (int32_t)i) {
      keep[i] = 0u;
      continue;
    }
    keep[i] = 1u;
    if (!mutual) continue;
    const uint32_t o = atomicAdd(n_int, 1u);
    if (o >= cap) {  // more merges than a binary tree of this size has nodes: report
      atomicOr(err, 4u);
      continue;
    }
    const uint32_t a = cid[i], b = cid[j];
    float u[6], ba[6], bb[6];
    for (int k = 0; k < 6; ++k) {
      ba[k] = cbox[6 * i + k];
      bb[k] = cbox[6 * (size_t)j + k];
    }
    for (int k = 0; k < 3; ++k) {
      u[k] = fminf(ba[k], bb[k]);
      u[3 + k] = fmaxf(ba[3 + k], bb[3 + k]);
    }
    for (int k = 0; k < 6; ++k) {
      nbox[6 * (size_t)o + k] = u[k];
      cbox[6 * i + k] = u[k];
    }
    const uint32_t c = ref_count(a, cnt) + ref_count(b, cnt);
    const float area = half_area(u);
    const float ca = (a & kLeafRef) ? half_area(ba) : ncost[a], cb = (b & kLeafRef) ? half_area(bb) : ncost[b];
    const float split = kSahNode * area + ca + cb, leaf = (float)c * area;
    const bool as_leaf = c <= (uint32_t)kMaxLeafTris && leaf <= split;
    ncost[o] = as_leaf ? leaf : split;
    float Da[4], Db[4];
    dp_of_ref(a, dp, half_area(ba), Da);
    dp_of_ref(b, dp, half_area(bb), Db);
    dp_node(o, as_leaf, c, area, Da, Db, dp, dsp);
    child[o] = make_uint2(a, b);
    cnt[o] = as_leaf ? (c | kLeafBitCnt) : c;
    cid[i] = o;
  }
}

// Kept clusters per block of kBB places (every block of the grid writes its count).
__global__ __launch_bounds__(kBB) void k_ploc_count(const uint32_t* __restrict__ keep, const uint32_t* __restrict__ mc,
                                                    uint32_t* __restrict__ bc) {
  __shared__ uint32_t w[kBB / 64];
  const uint32_t m = mc[0];
  const int64_t i = (int64_t)blockIdx.x * kBB + threadIdx.x;
  const uint64_t bal = __ballot(i < (int64_t)m && keep[i] != 0u);
  if (threadIdx.x % 64 == 0) w[threadIdx.x / 64] = (uint32_t)__popcll(bal);
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t = 0;
    for (int k = 0; k < kBB / 64; ++k) t += w[k];
    bc[blockIdx.x] = t;
  }
}

// Kept clusters to their places in the next round's arrays, in order (off:
// exclusive scan of the block counts); the last block writes the new count
// to mc_out[0] and this round's to mc_out[1] (the next round's mc).
__global__ __launch_bounds__(kBB) void k_ploc_scatter(const uint32_t* __restrict__ cid, const float* __restrict__ cbox,
                                                      const uint32_t* __restrict__ keep, const uint32_t* __restrict__ mc,
                                                      const uint32_t* __restrict__ off, uint32_t* __restrict__ cid2,
                                                      float* __restrict__ cbox2, uint32_t* __restrict__ mc_out) {
  __shared__ uint32_t w[kBB / 64];
  const uint32_t m = mc[0];
  const int64_t i = (int64_t)blockIdx.x * kBB + threadIdx.x;
  const bool k = i < (int64_t)m && keep[i] != 0u;
  const uint64_t bal = __ballot(k);
  const int wave = threadIdx.x / 64, lane = threadIdx.x % 64;
  if (lane == 0) w[wave] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t pos = off[blockIdx.x];
  for (int q = 0; q < wave; ++q) pos += w[q];
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  pos += (uint32_t)__popcll(bal & lt);
  if (k) {
    cid2[pos] = cid[i];
    for (int q = 0; q < 6; ++q) cbox2[6 * (size_t)pos + q] = cbox[6 * i + q];
  }
  if (blockIdx.x == gridDim.x - 1 && threadIdx.x == 0) {
    uint32_t t = off[blockIdx.x];
    for (int q = 0; q < kBB / 64; ++q) t += w[q];
    mc_out[0] = t;
    mc_out[1] = m;
  }
}

// The last rounds of the clustering in one workgroup, once at most
// kFinishMax clusters are left: the same rounds as k_ploc_nn .. k_ploc_scatter
// (same ranks, same merges, same forced rounds) with the clusters in LDS and
// barriers between the steps instead of launches.  Then the root's job.
constexpr int kFinishThreads = 1024;
constexpr int kFinishMax = 2048;
constexpr int kFinishPer = kFinishMax / kFinishThreads;

__device__ inline uint32_t block_excl_scan_1024(bool flag, uint32_t* s_w, uint32_t& total) {
  const int lane = threadIdx.x % 64, wave = threadIdx.x / 64;
  const uint64_t bal = __ballot(flag);
  const uint64_t lt = lane == 0 ? 0ull : (~0ull >> (64 - lane));
  if (lane == 0) s_w[wave] = (uint32_t)__popcll(bal);
  __syncthreads();
  uint32_t before = 0, t = 0;
  for (int w = 0; w < kFinishThreads / 64; ++w) {
    if (w < wave) before += s_w[w];
    t += s_w[w];
  }
  __syncthreads();  // s_w is reused by the next scan
  total = t;
  return before + (uint32_t)__popcll(bal & lt);
}

__global__ __launch_bounds__(kFinishThreads) void k_ploc_finish(const uint32_t* __restrict__ cid_in,
                                                                const float* __restrict__ cbox_in,
                                                                const uint32_t* __restrict__ mc,
                                                                uint2* __restrict__ child, float* __restrict__ nbox,
                                                                uint32_t* __restrict__ cnt, float* __restrict__ ncost,
                                                                float* __restrict__ dp, uint32_t* __restrict__ dsp,
                                                                uint32_t* __restrict__ n_int, uint32_t cap,
                                                                uint4* __restrict__ jobs, uint32_t* __restrict__ err) {
  __shared__ float sb[kFinishMax * 6];
  __shared__ uint32_t sid[kFinishMax];
  __shared__ int32_t snn[kFinishMax];
  __shared__ uint32_t s_w[kFinishThreads / 64];
  uint32_t m = mc[0], prev = mc[1];
  if (m > (uint32_t)kFinishMax) {  // the host launches this only at or below kFinishMax clusters
    if (threadIdx.x == 0) atomicOr(err, 16u);
    return;
  }
  for (int e = 0; e < kFinishPer; ++e) {
    const uint32_t i = threadIdx.x + e * kFinishThreads;
    if (i < m) {
      sid[i] = cid_in[i];
      for (int k = 0; k < 6; ++k) sb[6 * i + k] = cbox_in[6 * (size_t)i + k];
    }
  }
  __syncthreads();
  for (int round = 0; m > 1; ++round) {
    if (round >= kPlocMaxRounds) {
      if (threadIdx.x == 0) atomicOr(err, 16u);
      return;
    }
    const bool forced = (uint64_t)m * 100u > (uint64_t)prev * 99u;
    for (int e = 0; e < kFinishPer; ++e) {  // nearest neighbours
      const int64_t i = threadIdx.x + e * kFinishThreads;
      if (i >= (int64_t)m) continue;
      if (forced) {
        const int64_t j = i ^ 1;
        snn[i] = (int32_t)(j < (int64_t)m ? j : i);
        continue;
      }
      const float* bi = sb + 6 * i;
      float best = INFINITY;
      uint32_t bd = 0xFFFFFFFFu, blo = 0xFFFFFFFFu;
      int32_t bj = (int32_t)i;
      for (int d = -kPlocRadius; d <= kPlocRadius; ++d) {
        const int64_t j = i + d;
        if (d == 0 || j < 0 || j >= (int64_t)m) continue;
        const float* bb = sb + 6 * j;
        float u[6];
        for (int k = 0; k < 3; ++k) {
          u[k] = fminf(bi[k], bb[k]);
          u[3 + k] = fmaxf(bi[3 + k], bb[3 + k]);
        }
        const float a = half_area(u);
        const uint32_t ad = (uint32_t)(d < 0 ? -d : d), lo = (uint32_t)(d < 0 ? j : i);
        const bool better =
            a < best || (a == best && (ad < bd || (ad == bd && ((lo & 1u) < (blo & 1u) ||
                                                                ((lo & 1u) == (blo & 1u) && lo < blo)))));
        if (better) {
          best = a;
          bd = ad;
          blo = lo;
          bj = (int32_t)j;
        }
      }
      snn[i] = bj;
    }
    __syncthreads();
    bool keep[kFinishPer];
    for (int e = 0; e < kFinishPer; ++e) {  // merges (in place, as in k_ploc_merge)
      const int64_t i = threadIdx.x + e * kFinishThreads;
      keep[e] = false;
      if (i >= (int64_t)m) continue;
      const int32_t j = snn[i];
      const bool mutual = j != (int32_t)i && j >= 0 && j < (int32_t)m && snn[j] == (int32_t)i;
      keep[e] = !(mutual && j < (int32_t)i);
      if (!mutual || j < (int32_t)i) continue;
      const uint32_t o = atomicAdd(n_int, 1u);
      if (o >= cap) {
        atomicOr(err, 4u);
        continue;
      }
      const uint32_t a = sid[i], b = sid[j];
      float u[6], ba[6], bb[6];
      for (int k = 0; k < 6; ++k) {
        ba[k] = sb[6 * i + k];
        bb[k] = sb[6 * j + k];
      }
      for (int k = 0; k < 3; ++k) {
        u[k] = fminf(ba[k], bb[k]);
        u[3 + k] = fmaxf(ba[3 + k], bb[3 + k]);
      }
      for (int k = 0; k < 6; ++k) {
        nbox[6 * (size_t)o + k] = u[k];
        sb[6 * i + k] = u[k];
      }
      const uint32_t c = ref_count(a, cnt) + ref_count(b, cnt);
      const float area = half_area(u);
      const float ca = (a & kLeafRef) ? half_area(ba) : ncost[a], cb = (b & kLeafRef) ? half_area(bb) : ncost[b];
      const float split = kSahNode * area + ca + cb, leaf = (float)c * area;
      const bool as_leaf = c <= (uint32_t)kMaxLeafTris && leaf <= split;
      ncost[o] = as_leaf ? leaf : split;
      float Da[4], Db[4];
      dp_of_ref(a, dp, half_area(ba), Da);
      dp_of_ref(b, dp, half_area(bb), Db);
      dp_node(o, as_leaf, c, area, Da, Db, dp, dsp);
      child[o] = make_uint2(a, b);
      cnt[o] = as_leaf ? (c | kLeafBitCnt) : c;
      sid[i] = o;
    }
    __syncthreads();
    // compaction in order: places tid (first) then tid + kFinishThreads (second)
    uint32_t pos[kFinishPer], tot[kFinishPer];
    for (int e = 0; e < kFinishPer; ++e) pos[e] = block_excl_scan_1024(keep[e], s_w, tot[e]);
    uint32_t id_r[kFinishPer];
    float box_r[kFinishPer][6];
    for (int e = 0; e < kFinishPer; ++e) {
      const uint32_t i = threadIdx.x + e * kFinishThreads;
      if (!keep[e]) continue;
      id_r[e] = sid[i];
      for (int k = 0; k < 6; ++k) box_r[e][k] = sb[6 * i + k];
    }
    __syncthreads();
    uint32_t base = 0;
    for (int e = 0; e < kFinishPer; ++e) {
      if (keep[e]) {
        const uint32_t q = base + pos[e];
        sid[q] = id_r[e];
        for (int k = 0; k < 6; ++k) sb[6 * q + k] = box_r[e][k];
      }
      base += tot[e];
    }
    __syncthreads();
    prev = m;
    m = base;
  }
  if (threadIdx.x == 0) jobs[0] = make_uint4(sid[0], 0u, 0u, 0u);
}

// Cluster counts of the first round: n clusters, and no round before it.
__global__ void k_ploc_start(uint32_t* __restrict__ mc, uint32_t n) {
  mc[0] = n;
  mc[1] = 0xFFFFFFFFu;
}

// 5. one level of the collapse: job (binary reference, BVH4 node index, place
// of its first triangle in leaf order).  A leaf's triangles take consecutive
// places in depth-first order of its subtree: order[place] = sorted index.
__device__ inline void collapse_one(const uint4 job, uint4* __restrict__ next_jobs, uint32_t* __restrict__ n_next,
                                    uint32_t* __restrict__ n_nodes, uint32_t* __restrict__ max_leaf,
                                    const uint32_t* __restrict__ val, const float* __restrict__ tbox,
                                    const float* __restrict__ nbox, const uint2* __restrict__ child,
                                    const uint32_t* __restrict__ cnt, const uint32_t* __restrict__ dsp,
                                    BVHNode* __restrict__ out, uint32_t cap, uint32_t n_tris,
                                    uint32_t* __restrict__ order, uint32_t* __restrict__ err) {
  uint32_t kids[4];
  int nk = 0;
  if (ref_is_leaf_subtree(job.x, cnt)) {
    kids[nk++] = job.x;  // the whole tree is one leaf under a one-child root
  } else if (kGpuCollapseDp) {
    // the roots of the best split of the node's four slots, left before right
    // (the slots of the entries on the stack never add up to more than four)
    const uint2 c = child[job.x];
    const uint32_t s4 = dsp[job.x] >> 16;
    uint32_t stk_ref[4], stk_j[4];
    int sp = 0;
    stk_ref[sp] = c.y;
    stk_j[sp++] = s4 >> 2;
    stk_ref[sp] = c.x;
    stk_j[sp++] = s4 & 3u;
    while (sp > 0 && nk < 4) {
      --sp;
      const uint32_t y = stk_ref[sp], j = stk_j[sp];
      if (ref_is_leaf_subtree(y, cnt) || j <= 1u || j > 4u) {
        kids[nk++] = y;
        continue;
      }
      const uint32_t d = (dsp[y] >> (4u * (j - 1u))) & 15u;
      if ((d & 3u) == 0u || sp + 2 > 4) {
        kids[nk++] = y;
        continue;
      }
      const uint2 cc = child[y];
      stk_ref[sp] = cc.y;
      stk_j[sp++] = d >> 2;
      stk_ref[sp] = cc.x;
      stk_j[sp++] = d & 3u;
    }
    if (sp > 0) atomicOr(err, 32u);  // more roots than four slots: a malformed split
  } else {
    const uint2 c = child[job.x];
    kids[nk++] = c.x;
    kids[nk++] = c.y;
    while (nk < 4) {
      int pick = -1;
      float pa = -1.0f;
      for (int q = 0; q < nk; ++q) {
        if (!ref_is_leaf_subtree(kids[q], cnt)) {
          float b[6];
          ref_box(kids[q], val, tbox, nbox, b);
          const float a = half_area(b);
          if (a > pa) {
            pa = a;
            pick = q;
          }
        }
      }
      if (pick < 0) break;
      const uint2 cc = child[kids[pick]];
      for (int q = nk; q > pick + 1; --q) kids[q] = kids[q - 1];  // open in place: siblings keep their order
      kids[pick] = cc.x;
      kids[pick + 1] = cc.y;
      nk++;
    }
  }
  BVHNode node;
  for (int q = 0; q < 4; ++q) {
    node.lo_x[q] = node.hi_x[q] = node.lo_y[q] = node.hi_y[q] = node.lo_z[q] = node.hi_z[q] = 0.0f;
    node.child[q] = kEmpty;
    node.meta[q] = 0u;
  }
  node.meta[0] = (uint32_t)nk;
  uint32_t leaf_max = 0, place = job.z;
  // the node's inner children take consecutive node indices (siblings share lines of the cache)
  int n_inner = 0;
  for (int q = 0; q < nk; ++q) n_inner += ref_is_leaf_subtree(kids[q], cnt) ? 0 : 1;
  uint32_t o_next = 0, slot_next = 0;
  if (n_inner) {
    o_next = atomicAdd(n_nodes, (uint32_t)n_inner);
    slot_next = atomicAdd(n_next, (uint32_t)n_inner);
  }
  for (int q = 0; q < nk; ++q) {
    float b[6];
    ref_box(kids[q], val, tbox, nbox, b);
    node.lo_x[q] = b[0];
    node.lo_y[q] = b[1];
    node.lo_z[q] = b[2];
    node.hi_x[q] = b[3];
    node.hi_y[q] = b[4];
    node.hi_z[q] = b[5];
    const uint32_t c = ref_count(kids[q], cnt);
    if (place + c > n_tris) {  // counts that do not add up: report
      atomicOr(err, 8u);
      break;
    }
    if (ref_is_leaf_subtree(kids[q], cnt)) {
      node.child[q] = make_leaf(place, c);
      leaf_max = c > leaf_max ? c : leaf_max;
      // the subtree's leaves, left before right (at most kMaxLeafTris of them,
      // so the stack never holds more than that many entries)
      uint32_t stk[kMaxLeafTris];
      int sp = 0;
      uint32_t w = place;
      stk[sp++] = kids[q];
      while (sp > 0) {
        const uint32_t r = stk[--sp];
        if (r & kLeafRef) {
          if (w < place + c) order[w] = r & ~kLeafRef;
          w++;
        } else if (sp + 2 <= kMaxLeafTris) {
          const uint2 cc = child[r];
          stk[sp++] = cc.y;
          stk[sp++] = cc.x;
        } else {
          atomicOr(err, 8u);
          break;
        }
      }
      if (w != place + c) atomicOr(err, 8u);
    } else {
      const uint32_t o = o_next++, slot = slot_next++;
      if (o >= cap || slot >= cap) {  // more nodes than a tree of this size can have: report
        atomicOr(err, 2u);
        continue;
      }
      node.child[q] = o;
      next_jobs[slot] = make_uint4(kids[q], o, place, 0u);
    }
    place += c;
  }
  if (job.y < cap) out[job.y] = node;
  if (leaf_max) atomicMax(max_leaf, leaf_max);
}

// Level `level` of the collapse: its job count is jc[level % 3] (written by the
// level before), its jobs append to jc[(level + 1) % 3], and it zeroes
// jc[(level + 2) % 3] for the level after next; jc[3] counts the levels that
// had jobs.  Any grid (a grid-stride loop), so that levels are enqueued
// without the host reading the counts in between.
__global__ __launch_bounds__(kBB) void k_collapse(const uint4* __restrict__ jobs, uint32_t* __restrict__ jc, int level,
                                                  uint4* __restrict__ next_jobs, uint32_t* __restrict__ n_nodes,
                                                  uint32_t* __restrict__ max_leaf, const uint32_t* __restrict__ val,
                                                  const float* __restrict__ tbox, const float* __restrict__ nbox,
                                                  const uint2* __restrict__ child, const uint32_t* __restrict__ cnt,
                                                  const uint32_t* __restrict__ dsp, BVHNode* __restrict__ out,
                                                  uint32_t cap, uint32_t n_tris, uint32_t* __restrict__ order,
                                                  uint32_t* __restrict__ err) {
  const uint32_t n_jobs = min(jc[level % 3], cap);
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    jc[(level + 2) % 3] = 0u;
    if (n_jobs) atomicMax(jc + 3, (uint32_t)(level + 1));
  }
  for (uint32_t j = blockIdx.x * kBB + threadIdx.x; j < n_jobs; j += gridDim.x * kBB)
    collapse_one(jobs[j], next_jobs, jc + (level + 1) % 3, n_nodes, max_leaf, val, tbox, nbox, child, cnt, dsp, out,
                 cap, n_tris, order, err);
}

// 6. triangle records in leaf order
__global__ __launch_bounds__(kBB) void k_sorted_tris(const float* __restrict__ soup, const uint32_t* __restrict__ prim,
                                                     const uint32_t* __restrict__ mat, const uint32_t* __restrict__ val,
                                                     const uint32_t* __restrict__ order, int64_t n,
                                                     TriRec* __restrict__ tris) {
  for (int64_t i = blockIdx.x * (int64_t)kBB + threadIdx.x; i < n; i += (int64_t)gridDim.x * kBB) {
    const uint32_t t = val[order[i]];
    const float* p = soup + 9 * (size_t)t;
    TriRec r;
    r.a = make_float4(p[0], p[1], p[2], __uint_as_float(prim[t]));
    r.b = make_float4(p[3], p[4], p[5], __uint_as_float(mat[t]));
    r.c = make_float4(p[6], p[7], p[8], 0.0f);
    tris[i] = r;
  }
}

int grid_of(int64_t n) { return (int)std::max<int64_t>(1, std::min<int64_t>((n + kBB - 1) / kBB, 8192)); }

// device workspace of one build, freed when it goes out of scope
// (one allocation sized for the whole build, carved in 256-byte aligned
// pieces; a piece that does not fit gets an allocation of its own)
struct Scratch {
  void* arena = nullptr;
  size_t cap = 0, used = 0;
  std::vector<void*> extra;
  explicit Scratch(size_t bytes) {
    if (hipMalloc(&arena, bytes) == hipSuccess) cap = bytes;
    else arena = nullptr;
  }
  ~Scratch() {
    for (void* p : extra) (void)hipFree(p);
    if (arena) (void)hipFree(arena);
  }
  template <class T>
  hipError_t get(T** out, size_t count) {
    const size_t b = (std::max<size_t>(count * sizeof(T), 16) + 255) & ~size_t(255);
    if (arena && used + b <= cap) {
      *out = reinterpret_cast<T*>(static_cast<char*>(arena) + used);
      used += b;
      return hipSuccess;
    }
    void* p = nullptr;
    hipError_t e = hipMalloc(&p, b);
    if (e == hipSuccess) extra.push_back(p);
    *out = static_cast<T*>(p);
    return e;
  }
};

// workspace bytes per triangle of one build: boxes, keys, tree, jobs, clusters (an upper bound)
constexpr size_t kBuildBytesPerTri = 232;

}  // namespace

#define PT_TRY(x)                         \
  do {                                    \
    hipError_t e_ = (x);                  \
    if (e_ != hipSuccess) return e_;      \
  } while (0)

hipError_t gpu_build_bvh4(const float* soup, const uint32_t* prim, const uint32_t* mat, int64_t n, BVHNode* nodes,
                          TriRec* tris, hipStream_t st, GpuBvhStats* stats, int builder) {
  if (n <= 0 || n >= (int64_t)kLeafFirstMask) return hipErrorInvalidValue;
  if (builder != kGpuBvhPloc && builder != kGpuBvhLbvh) return hipErrorInvalidValue;
  Scratch S((size_t)n * kBuildBytesPerTri + (size_t)256 * 4 * (size_t)((n + kTile - 1) / kTile) + (64u << 10));
  float *tbox = nullptr, *nbox = nullptr;
  uint32_t *cb = nullptr, *keyA = nullptr, *valA = nullptr, *keyB = nullptr, *valB = nullptr, *hist = nullptr;
  uint32_t *counters = nullptr, *cnt = nullptr, *order = nullptr;
  uint2* child = nullptr;
  uint4* jobs[2] = {nullptr, nullptr};
  const int nb = (int)((n + kTile - 1) / kTile);
  const int64_t ni = std::max<int64_t>(1, n - 1);
  PT_TRY(S.get(&tbox, (size_t)n * 6));
  PT_TRY(S.get(&nbox, (size_t)ni * 6));
  PT_TRY(S.get(&cb, 6));
  PT_TRY(S.get(&keyA, (size_t)n));
  PT_TRY(S.get(&valA, (size_t)n));
  PT_TRY(S.get(&keyB, (size_t)n));
  PT_TRY(S.get(&valB, (size_t)n));
  PT_TRY(S.get(&hist, (size_t)256 * nb));
  // [0] BVH4 nodes, [1] jobs of the next level, [2] largest leaf, [3] error bits, [4] binary nodes,
  // [5] clusters after a round
  PT_TRY(S.get(&counters, 8));
  PT_TRY(S.get(&child, (size_t)ni));
  PT_TRY(S.get(&cnt, (size_t)ni));
  float* dp = nullptr;
  uint32_t* dsp = nullptr;
  PT_TRY(S.get(&dp, (size_t)ni * 4));
  PT_TRY(S.get(&dsp, (size_t)ni));
  PT_TRY(S.get(&order, (size_t)n));
  PT_TRY(S.get(&jobs[0], (size_t)n));
  PT_TRY(S.get(&jobs[1], (size_t)n));

  hipLaunchKernelGGL(k_init_bounds, dim3(1), dim3(64), 0, st, cb);
  hipLaunchKernelGGL(k_tri_boxes, dim3(grid_of(n)), dim3(kBB), 0, st, soup, n, tbox, cb);
  hipLaunchKernelGGL(k_morton, dim3(grid_of(n)), dim3(kBB), 0, st, tbox, n, cb, keyA, valA);
  for (int pass = 0; pass < 4; ++pass) {  // codes have 30 bits
    const int shift = 8 * pass;
    hipLaunchKernelGGL(k_radix_hist, dim3(nb), dim3(kBB), 0, st, keyA, n, shift, hist, nb);
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, hist, (int64_t)256 * nb);
    hipLaunchKernelGGL(k_radix_scatter, dim3(nb), dim3(kBB), 0, st, keyA, valA, keyB, valB, n, shift, hist, nb);
    std::swap(keyA, keyB);
    std::swap(valA, valB);
  }
  PT_TRY(hipMemsetAsync(counters, 0, 8 * sizeof(uint32_t), st));
  if (n > 1 && builder == kGpuBvhLbvh) {
    uint32_t* flag = nullptr;
    int32_t *parent_leaf = nullptr, *parent_int = nullptr;
    PT_TRY(S.get(&flag, (size_t)ni));
    PT_TRY(S.get(&parent_leaf, (size_t)n));
    PT_TRY(S.get(&parent_int, (size_t)ni));
    PT_TRY(hipMemsetAsync(flag, 0, (size_t)ni * sizeof(uint32_t), st));
    PT_TRY(hipMemsetAsync(parent_int, 0xFF, (size_t)ni * sizeof(int32_t), st));  // root: -1
    hipLaunchKernelGGL(k_radix_tree, dim3(grid_of(n - 1)), dim3(kBB), 0, st, keyA, n, child, parent_leaf, parent_int,
                       cnt, counters + 3);
    hipLaunchKernelGGL(k_boxes_up, dim3(grid_of(n)), dim3(kBB), 0, st, n, valA, tbox, child, parent_leaf, parent_int,
                       nbox, flag, cnt, dp, dsp);
    const uint4 root = make_uint4(0u, 0u, 0u, 0u);
    PT_TRY(hipMemcpyAsync(jobs[0], &root, sizeof(root), hipMemcpyHostToDevice, st));
  } else if (n > 1) {
    uint32_t *cid[2] = {nullptr, nullptr}, *keep = nullptr, *bc = nullptr, *mc = nullptr;
    float* cbox[2] = {nullptr, nullptr};
    float* ncost = nullptr;
    int32_t* nn = nullptr;
    const int64_t nblk = (n + kBB - 1) / kBB;
    for (int k = 0; k < 2; ++k) {
      PT_TRY(S.get(&cid[k], (size_t)n));
      PT_TRY(S.get(&cbox[k], (size_t)n * 6));
    }
    PT_TRY(S.get(&keep, (size_t)n));
    PT_TRY(S.get(&bc, (size_t)nblk));
    PT_TRY(S.get(&nn, (size_t)n));
    PT_TRY(S.get(&ncost, (size_t)ni));
    PT_TRY(S.get(&mc, 4));  // cluster counts: [0..1] read by even rounds, [2..3] by odd rounds
    hipLaunchKernelGGL(k_ploc_init, dim3(grid_of(n)), dim3(kBB), 0, st, valA, tbox, n, cid[0], cbox[0]);
    hipLaunchKernelGGL(k_ploc_start, dim3(1), dim3(1), 0, st, mc, (uint32_t)n);
    // the counts stay on the device; the host reads them once per batch of rounds and sizes the
    // batch's grids by the count at its start (kernels skip the places past the current count; a
    // round with one cluster left copies it unchanged)
    uint32_t m = (uint32_t)n, m_host[2] = {0u, 0u};
    int cur = 0, rounds = 0;
    while (m > (uint32_t)kFinishMax) {
      if (rounds >= kPlocMaxRounds) return hipErrorUnknown;
      const int blocks = (int)((m + kBB - 1) / kBB);
      for (int r = 0; r < kPlocBatch; ++r, ++rounds) {
        const uint32_t* mc_in = mc + 2 * (rounds & 1);
        uint32_t* mc_out = mc + 2 * ((rounds & 1) ^ 1);
        hipLaunchKernelGGL(k_ploc_nn, dim3(blocks), dim3(kBB), 0, st, cbox[cur], mc_in, nn);
        hipLaunchKernelGGL(k_ploc_merge, dim3(grid_of(m)), dim3(kBB), 0, st, cid[cur], cbox[cur], mc_in, nn, child,
                           nbox, cnt, ncost, dp, dsp, counters + 4, (uint32_t)ni, keep, counters + 3);
        hipLaunchKernelGGL(k_ploc_count, dim3(blocks), dim3(kBB), 0, st, keep, mc_in, bc);
        hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(1024), 0, st, bc, (int64_t)blocks);
        hipLaunchKernelGGL(k_ploc_scatter, dim3(blocks), dim3(kBB), 0, st, cid[cur], cbox[cur], keep, mc_in, bc,
                           cid[cur ^ 1], cbox[cur ^ 1], mc_out);
        cur ^= 1;
      }
      PT_TRY(hipGetLastError());
      PT_TRY(hipMemcpyAsync(m_host, mc + 2 * (rounds & 1), sizeof(m_host), hipMemcpyDeviceToHost, st));
      PT_TRY(hipStreamSynchronize(st));
      if (m_host[0] == 0u || m_host[0] > m) return hipErrorUnknown;  // a round never loses every cluster
      m = m_host[0];
    }
    // the last rounds (at most kFinishMax clusters) in one workgroup; it also writes the root's job
    hipLaunchKernelGGL(k_ploc_finish, dim3(1), dim3(kFinishThreads), 0, st, cid[cur], cbox[cur],
                       mc + 2 * (rounds & 1), child, nbox, cnt, ncost, dp, dsp, counters + 4, (uint32_t)ni, jobs[0],
                       counters + 3);
  } else {
    const uint4 root = make_uint4(kLeafRef, 0u, 0u, 0u);
    PT_TRY(hipMemcpyAsync(jobs[0], &root, sizeof(root), hipMemcpyHostToDevice, st));
  }
  // collapse, level by level, from the root; the levels' job counts stay on the device and the host
  // reads the next one once per batch of levels
  const uint32_t cap = (uint32_t)ni;  // nodes of the output (and jobs of a level) at most
  uint32_t* jc = nullptr;  // job counts of three consecutive levels, [3]: levels that had jobs
  PT_TRY(S.get(&jc, 4));
  const uint32_t one = 1u, jc0[4] = {1u, 0u, 0u, 0u};
  PT_TRY(hipMemcpyAsync(counters, &one, sizeof(one), hipMemcpyHostToDevice, st));
  PT_TRY(hipMemcpyAsync(jc, jc0, sizeof(jc0), hipMemcpyHostToDevice, st));
  const int cgrid = grid_of(cap);
  int level = 0;
  uint32_t pending[2] = {1u, 0u};
  while (pending[0] > 0) {
    for (int r = 0; r < kCollapseBatch; ++r, ++level) {
      if (level >= kMaxTreeLevels) return hipErrorUnknown;
      hipLaunchKernelGGL(k_collapse, dim3(cgrid), dim3(kBB), 0, st, jobs[level & 1], jc, level, jobs[(level + 1) & 1],
                         counters, counters + 2, valA, tbox, nbox, child, cnt, dsp, nodes, cap, (uint32_t)n, order,
                         counters + 3);
    }
    PT_TRY(hipGetLastError());
    PT_TRY(hipMemcpyAsync(&pending[0], jc + level % 3, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    PT_TRY(hipMemcpyAsync(&pending[1], jc + 3, sizeof(uint32_t), hipMemcpyDeviceToHost, st));
    PT_TRY(hipStreamSynchronize(st));
  }
  const int levels = (int)pending[1];
  hipLaunchKernelGGL(k_sorted_tris, dim3(grid_of(n)), dim3(kBB), 0, st, soup, prim, mat, valA, order, n, tris);
  uint32_t fin[4];
  PT_TRY(hipMemcpyAsync(fin, counters, sizeof(fin), hipMemcpyDeviceToHost, st));
  PT_TRY(hipStreamSynchronize(st));
  if (fin[3] != 0u || fin[0] > cap) return hipErrorUnknown;  // malformed tree: no result
  stats->n_nodes = fin[0];
  stats->max_leaf = (int)fin[2];
  stats->depth = levels + 1;  // node levels, plus the leaves under the deepest nodes
  return hipGetLastError();
}

}  // namespace pt
