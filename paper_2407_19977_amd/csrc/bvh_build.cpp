// Host BVH builder (paper Sec. 5.1.1: the CPU groups adjacent primitives in
// axis-aligned boxes so that every child lies inside its parent; Table 1
// times this set-up stage).
//
// 1. Binned SAH (32 bins per axis on centroid bounds, traversal cost 1,
//    triangle cost 1) builds a binary tree with at most 4 triangles per leaf;
//    large subtrees are built on parallel threads.
// 2. The binary tree is collapsed into a 4-wide tree by the least SAH cost
//    (the dynamic program of Ylitie, Karras and Laine 2017 for wide BVHs):
//    bottom-up, D(n, j) is the least cost of covering node n's subtree with
//    at most j roots, a root costing its area times (one node step plus its
//    children's costs) or, for a leaf, times its triangle count; top-down,
//    each 4-wide node takes the roots of the best split of its four slots.
//    (PT_COLLAPSE_DP 0: a node repeatedly opens its largest-area internal
//    child until it has four children.)
// 3. Nodes are written in depth-first order as 128-byte records with the four
//    child boxes stored structure-of-arrays; triangles are written in leaf
//    order as 48-byte records.
// Boxes are the exact float min/max of the triangle vertices, so every
// triangle lies inside each box on its path.
#include "bvh_build.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstring>
#include <future>
#include <limits>
#include <memory>
#include <mutex>
#include <utility>

namespace pt {
namespace {

struct Box {
  float lo[3], hi[3];
  void clear() {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::numeric_limits<float>::infinity();
      hi[k] = -std::numeric_limits<float>::infinity();
    }
  }
  void grow(const Box& b) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], b.lo[k]);
      hi[k] = std::max(hi[k], b.hi[k]);
    }
  }
  void grow(const float* p) {
    for (int k = 0; k < 3; ++k) {
      lo[k] = std::min(lo[k], p[k]);
      hi[k] = std::max(hi[k], p[k]);
    }
  }
  double area() const {
    double dx = (double)hi[0] - lo[0], dy = (double)hi[1] - lo[1], dz = (double)hi[2] - lo[2];
    if (!(dx >= 0) || !(dy >= 0) || !(dz >= 0)) return 0.0;
    return 2.0 * (dx * dy + dy * dz + dz * dx);
  }
};

struct BNode {  // trivial, so that its storage is not initialised before the build writes it
  Box box;
  int32_t left, right;
  int32_t first, count;  // count > 0: leaf
};

// vector storage whose resize leaves trivial elements uninitialised
template <class T>
struct DefaultInitAlloc : std::allocator<T> {
  template <class U>
  struct rebind {
    using other = DefaultInitAlloc<U>;
  };
  DefaultInitAlloc() = default;
  template <class U>
  DefaultInitAlloc(const DefaultInitAlloc<U>&) noexcept {}
  template <class U>
  void construct(U* p) noexcept {
    ::new ((void*)p) U;
  }
  template <class U, class... A>
  void construct(U* p, A&&... a) {
    ::new ((void*)p) U(std::forward<A>(a)...);
  }
};
using BNodeVec = std::vector<BNode, DefaultInitAlloc<BNode>>;

// Run f(begin, end) over [0, n) in up to 16 chunks on parallel threads.
template <class F>
void parallel_chunks(int64_t n, F&& f) {
  const int64_t chunks = std::min<int64_t>(16, std::max<int64_t>(1, n / 65536));
  std::vector<std::future<void>> fs;
  for (int64_t c = 1; c < chunks; ++c)
    fs.push_back(std::async(std::launch::async, [&, c] { f(n * c / chunks, n * (c + 1) / chunks); }));
  f(0, n / chunks);
  for (auto& x : fs) x.get();
}

constexpr int kBins = 32;
#ifndef PT_SAH_TRAVERSAL
#define PT_SAH_TRAVERSAL 1.0
#endif
constexpr double kSahTraversal = PT_SAH_TRAVERSAL;  // cost of a node step relative to one triangle test

// A triangle's box, centroid and index, moved with the partitions so that a
// node's passes read its triangles in sequence (the partitions swap the same
// positions as partitions of the bare indices would: the tree is the same).
struct PrimRef {
  Box box;
  float c[3];
  int32_t t;
};

struct Builder {
  std::vector<PrimRef> pr;
  std::vector<int32_t> idx;  // the triangles in leaf order, filled after the build
  BNodeVec nodes;
  std::atomic<int32_t> next{0};

  int32_t alloc() { return next.fetch_add(1); }

  int32_t build(int32_t first, int32_t count, int level) {
    int32_t id = alloc();
    BNode nd;
    nd.left = nd.right = -1;
    nd.first = nd.count = 0;
    Box cb;
    nd.box.clear();
    cb.clear();
    for (int32_t i = first; i < first + count; ++i) {
      nd.box.grow(pr[(size_t)i].box);
      cb.grow(pr[(size_t)i].c);
    }
    int best_axis = -1, best_bin = -1;
    double best_cost = std::numeric_limits<double>::infinity();
    double parent_area = nd.box.area();
    for (int ax = 0; ax < 3 && count > 1; ++ax) {
      float ext = cb.hi[ax] - cb.lo[ax];
      if (!(ext > 0.0f)) continue;
      Box bb[kBins];
      int32_t bc[kBins];
      for (int b = 0; b < kBins; ++b) {
        bb[b].clear();
        bc[b] = 0;
      }
      double scale = kBins / (double)ext;
      for (int32_t i = first; i < first + count; ++i) {
        const PrimRef& q = pr[(size_t)i];
        int b = (int)(((double)q.c[ax] - cb.lo[ax]) * scale);
        b = std::min(std::max(b, 0), kBins - 1);
        bb[b].grow(q.box);
        bc[b]++;
      }
      double ra[kBins];
      int32_t rc[kBins];
      Box acc;
      acc.clear();
      int32_t n = 0;
      for (int b = kBins - 1; b > 0; --b) {
        acc.grow(bb[b]);
        n += bc[b];
        ra[b] = acc.area();
        rc[b] = n;
      }
      acc.clear();
      n = 0;
      for (int b = 0; b < kBins - 1; ++b) {
        acc.grow(bb[b]);
        n += bc[b];
        if (n == 0 || rc[b + 1] == 0) continue;
        double cost = acc.area() * n + ra[b + 1] * rc[b + 1];
        if (cost < best_cost) {
          best_cost = cost;
          best_axis = ax;
          best_bin = b;
        }
      }
    }
    // leaf if small and splitting does not pay (SAH: traversal cost kSahTraversal, triangle cost 1)
    double leaf_cost = (double)count;
    double split_cost = parent_area > 0 ? kSahTraversal + best_cost / parent_area : kSahTraversal + count;
    bool make_leaf = count <= 1 || (count <= kMaxLeafTris && (best_axis < 0 || leaf_cost <= split_cost));
    if (make_leaf) {
      nd.first = first;
      nd.count = count;
      nodes[id] = nd;
      return id;
    }
    int32_t mid;
    if (best_axis >= 0) {
      float ext = cb.hi[best_axis] - cb.lo[best_axis];
      double scale = kBins / (double)ext;
      int ax = best_axis, sb = best_bin;
      auto it = std::partition(pr.begin() + first, pr.begin() + first + count, [&](const PrimRef& q) {
        int b = (int)(((double)q.c[ax] - cb.lo[ax]) * scale);
        b = std::min(std::max(b, 0), kBins - 1);
        return b <= sb;
      });
      mid = (int32_t)(it - pr.begin());
      if (mid == first || mid == first + count) mid = first + count / 2;
    } else {
      // all centroids coincide: split the range in half
      mid = first + count / 2;
    }
    int32_t l, r;
    if (count > 50000 && level < 6) {
      auto fl = std::async(std::launch::async, [&] { return build(first, mid - first, level + 1); });
      r = build(mid, first + count - mid, level + 1);
      l = fl.get();
    } else {
      l = build(first, mid - first, level + 1);
      r = build(mid, first + count - mid, level + 1);
    }
    nd.left = l;
    nd.right = r;
    nd.count = 0;
    nodes[id] = nd;
    return id;
  }
};

#ifndef PT_COLLAPSE_DP
#define PT_COLLAPSE_DP 1
#endif
// cost of a 4-wide node step relative to one triangle test, for the collapse
#ifndef PT_COLLAPSE_NODE_COST
#define PT_COLLAPSE_NODE_COST 1.0
#endif

struct Collapser {
  const BNodeVec* bn;
  const std::vector<int32_t>* idx;
  std::vector<BVHNode> out;
  int max_depth = 0;
  int max_leaf = 0;
  double sah = 0.0;
  double root_area = 1.0;
  // optimal collapse: D[4 n + j - 1] the least SAH cost of covering binary
  // node n's subtree with at most j roots (j = 1..4); dec[n] packs, for
  // j = 2..4 in bits 4 (j - 1) .. 4 (j - 1) + 3, the split of the j slots
  // between n's children (left count in the low two bits, right count in the
  // high two; 0: n itself is the one root), and in bits 16..19 the split of
  // n's four slots when n is a 4-wide node (uninitialised storage: every
  // planned node is written once)
  std::unique_ptr<float[]> D;
  std::unique_ptr<uint32_t[]> dec;

  // the top levels' subtrees are planned on parallel threads (as they were built)
  void plan(int32_t b, int level = 0) {
    const BNodeVec& B = *bn;
    const BNode& x = B[b];
    const double a = x.box.area();
    if (x.count > 0) {
      for (int j = 0; j < 4; ++j) D[4 * (size_t)b + j] = (float)(a * x.count);
      dec[b] = 0u;
      return;
    }
    if (level < 4) {
      auto fl = std::async(std::launch::async, [&] { plan(x.left, level + 1); });
      plan(x.right, level + 1);
      fl.get();
    } else {
      plan(x.left, level + 1);
      plan(x.right, level + 1);
    }
    const float* Dl = &D[4 * (size_t)x.left];
    const float* Dr = &D[4 * (size_t)x.right];
    float Ds[5] = {0, 0, 0, 0, 0};
    uint32_t ks[5] = {0, 0, 0, 0, 0};
    for (int j = 2; j <= 4; ++j) {
      Ds[j] = std::numeric_limits<float>::infinity();
      for (int kl = 1; kl < j; ++kl) {
        const float c = Dl[kl - 1] + Dr[j - kl - 1];
        if (c < Ds[j]) {
          Ds[j] = c;
          ks[j] = (uint32_t)kl | ((uint32_t)(j - kl) << 2);
        }
      }
    }
    float best = (float)(a * PT_COLLAPSE_NODE_COST) + Ds[4];
    uint32_t d = 0u, bits = ks[4] << 16;
    D[4 * (size_t)b] = best;
    for (int j = 2; j <= 4; ++j) {
      if (Ds[j] < best) {
        best = Ds[j];
        d = ks[j];
      }
      D[4 * (size_t)b + j - 1] = best;
      bits |= d << (4 * (j - 1));
    }
    dec[b] = bits;
  }

  // the roots that cover binary node b's subtree with at most j of them
  void roots(int32_t b, int j, int32_t* kids, int& nk) const {
    const BNodeVec& B = *bn;
    const uint32_t d = j >= 2 ? (dec[b] >> (4 * (j - 1))) & 15u : 0u;
    if (B[b].count > 0 || (d & 3u) == 0u) {
      kids[nk++] = b;
      return;
    }
    roots(B[b].left, (int)(d & 3u), kids, nk);
    roots(B[b].right, (int)(d >> 2), kids, nk);
  }

  static void set_box(BVHNode& n, int c, const Box& b) {
    n.lo_x[c] = b.lo[0]; n.hi_x[c] = b.hi[0];
    n.lo_y[c] = b.lo[1]; n.hi_y[c] = b.hi[1];
    n.lo_z[c] = b.lo[2]; n.hi_z[c] = b.hi[2];
  }

  uint32_t emit(int32_t b, int depth) {
    const BNodeVec& B = *bn;
    int32_t kids[4];
    int nk = 0;
    if (B[b].count > 0) {
      kids[nk++] = b;  // a lone leaf under a single-child root
    } else if (PT_COLLAPSE_DP) {
      const uint32_t s4 = dec[b] >> 16;
      roots(B[b].left, (int)(s4 & 3u), kids, nk);
      roots(B[b].right, (int)(s4 >> 2), kids, nk);
    } else {
      kids[nk++] = B[b].left;
      kids[nk++] = B[b].right;
      while (nk < 4) {
        int pick = -1;
        double pa = -1.0;
        for (int i = 0; i < nk; ++i) {
          if (B[kids[i]].count == 0 && B[kids[i]].box.area() > pa) {
            pa = B[kids[i]].box.area();
            pick = i;
          }
        }
        if (pick < 0) break;
        int32_t c = kids[pick];
        // open the child in place so siblings keep their spatial order
        for (int i = nk; i > pick + 1; --i) kids[i] = kids[i - 1];
        kids[pick] = B[c].left;
        kids[pick + 1] = B[c].right;
        nk++;
      }
    }
    uint32_t id = (uint32_t)out.size();
    out.emplace_back();
    max_depth = std::max(max_depth, depth);
    sah += B[b].box.area() / root_area;
    BVHNode n;
    std::memset(&n, 0, sizeof(n));
    for (int c = 0; c < 4; ++c) {
      n.lo_x[c] = n.lo_y[c] = n.lo_z[c] = 0.0f;
      n.hi_x[c] = n.hi_y[c] = n.hi_z[c] = 0.0f;
      n.child[c] = kEmpty;
    }
    n.meta[0] = (uint32_t)nk;
    for (int c = 0; c < nk; ++c) {
      const BNode& k = B[kids[c]];
      set_box(n, c, k.box);
      if (k.count > 0) {
        n.child[c] = make_leaf((uint32_t)k.first, (uint32_t)k.count);
        max_leaf = std::max(max_leaf, (int)k.count);
        max_depth = std::max(max_depth, depth + 1);
        sah += k.box.area() / root_area * k.count;
      } else {
        n.child[c] = 0;  // patched below (emit appends to `out`)
      }
    }
    for (int c = 0; c < nk; ++c) {
      const BNode& k = B[kids[c]];
      if (k.count == 0) n.child[c] = emit(kids[c], depth + 1);
    }
    out[id] = n;
    return id;
  }
};

}  // namespace

bool build_bvh4(const float* verts, const uint32_t* prim_ids, const uint32_t* mat_ids, int64_t n, Bvh4& out,
                std::string& err) {
  auto t0 = std::chrono::steady_clock::now();
  if (n <= 0) {
    err = "a BVH needs at least one triangle";
    return false;
  }
  if (n >= (int64_t)kLeafFirstMask) {
    err = "too many triangles for one BVH (limit 2^27 - 1)";
    return false;
  }
  Builder B;
  B.pr.resize((size_t)n);
  Box all;
  all.clear();
  std::mutex mu;
  bool finite = true;
  parallel_chunks(n, [&](int64_t t0c, int64_t t1c) {
    Box part;
    part.clear();
    bool ok = true;
    for (int64_t t = t0c; t < t1c; ++t) {
      Box b;
      b.clear();
      for (int v = 0; v < 3; ++v) {
        const float* p = verts + 9 * t + 3 * v;
        for (int k = 0; k < 3; ++k) ok = ok && std::isfinite(p[k]);
        b.grow(p);
      }
      PrimRef& q = B.pr[(size_t)t];
      q.box = b;
      for (int k = 0; k < 3; ++k) q.c[k] = 0.5f * (b.lo[k] + b.hi[k]);
      q.t = (int32_t)t;
      part.grow(b);
    }
    std::lock_guard<std::mutex> g(mu);
    finite = finite && ok;
    all.grow(part);
  });
  if (!finite) {
    err = "non-finite vertex";
    return false;
  }
  B.nodes.resize(2 * (size_t)n + 1);
  int32_t root = B.build(0, (int32_t)n, 0);
  B.nodes.resize((size_t)B.next.load());
  B.idx.resize((size_t)n);
  for (int64_t i = 0; i < n; ++i) B.idx[(size_t)i] = B.pr[(size_t)i].t;
  std::vector<PrimRef>().swap(B.pr);

  Collapser C;
  C.bn = &B.nodes;
  C.idx = &B.idx;
  C.root_area = std::max(B.nodes[root].box.area(), 1e-30);
  C.out.reserve((size_t)n / 2 + 16);
  if (PT_COLLAPSE_DP) {
    C.D.reset(new float[4 * B.nodes.size()]);
    C.dec.reset(new uint32_t[B.nodes.size()]);
    C.plan(root);
  }
  C.emit(root, 1);
  out.nodes = std::move(C.out);
  out.depth = C.max_depth;
  out.max_leaf = C.max_leaf;
  out.sah_cost = C.sah;
  out.tris.resize((size_t)n);
  parallel_chunks(n, [&](int64_t i0, int64_t i1) {
    for (int64_t i = i0; i < i1; ++i) {
      int32_t t = B.idx[(size_t)i];
      const float* p = verts + 9 * (size_t)t;
      TriRec r;
      r.a = make_float4(p[0], p[1], p[2], 0.0f);
      r.b = make_float4(p[3], p[4], p[5], 0.0f);
      r.c = make_float4(p[6], p[7], p[8], 0.0f);
      uint32_t pid = prim_ids[t], mid = mat_ids[t];
      std::memcpy(&r.a.w, &pid, 4);
      std::memcpy(&r.b.w, &mid, 4);
      out.tris[(size_t)i] = r;
    }
  });
  for (int k = 0; k < 3; ++k) {
    out.lo[k] = all.lo[k];
    out.hi[k] = all.hi[k];
  }
  out.build_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  return true;
}

}  // namespace pt
