// Ray/triangle intersection and BVH4 traversal, compiled for the GPU and
// (for host-side checks) for the CPU.
//
// Closest hit (Sec. 5.1.1: the BVH rejects boxes the ray misses, so each ray
// tests O(log n) triangles): among triangles with t in (tmin, tmax), other
// than the one the ray leaves from, the lexicographic minimum of
// (t, instance, primitive).  Every triangle test is the single-precision
// watertight algorithm of Woop, Benthin and Wald (JCGT 2013) in a fixed
// operation order without fused multiply-adds, so the BVH walk, a brute
// force over all triangles and a CPU build of the same definition agree bit
// for bit.  The box test only prunes: its bounds are widened by 2^-20
// relative so it never rejects a box the exact slab test would accept.
#pragma once

#include <math.h>
#include <stdint.h>

#include "pt_layout.h"

namespace pt {

struct Hit {
  float t, b1, b2;
  uint32_t inst, prim;  // prim: primitive id as given by the user
  uint32_t tri;         // index of the triangle record (leaf order)
  uint32_t mat;         // material id
};

__host__ __device__ inline void hit_clear(Hit& h) {
  h.t = INFINITY;
  h.b1 = h.b2 = 0.0f;
  h.inst = h.prim = h.tri = h.mat = 0xFFFFFFFFu;
}

__host__ __device__ inline uint32_t f2u(float x) {
  union { float f; uint32_t u; } c;
  c.f = x;
  return c.u;
}
__host__ __device__ inline float u2f(uint32_t x) {
  union { float f; uint32_t u; } c;
  c.u = x;
  return c.f;
}

__host__ __device__ inline float sel3(float x, float y, float z, int k) {
  return k == 0 ? x : (k == 1 ? y : z);
}

// Per-ray constants of the watertight test and the slab test.
struct RayPre {
  float ox, oy, oz, dx, dy, dz;
  float ix, iy, iz;  // 1/d (IEEE, +-inf for zero components)
  int kx, ky, kz;
  float Sx, Sy, Sz;
};

__host__ __device__ inline RayPre ray_prepare(float ox, float oy, float oz, float dx, float dy, float dz) {
#pragma clang fp contract(off)
  RayPre r;
  r.ox = ox; r.oy = oy; r.oz = oz; r.dx = dx; r.dy = dy; r.dz = dz;
  r.ix = 1.0f / dx;
  r.iy = 1.0f / dy;
  r.iz = 1.0f / dz;
  float a0 = fabsf(dx), a1 = fabsf(dy), a2 = fabsf(dz);
  int kz = 0;
  float am = a0;
  if (a1 > am) { kz = 1; am = a1; }
  if (a2 > am) { kz = 2; }
  int kx = kz == 2 ? 0 : kz + 1;
  int ky = kx == 2 ? 0 : kx + 1;
  float dkz = sel3(dx, dy, dz, kz);
  if (dkz < 0.0f) { int t = kx; kx = ky; ky = t; }
  r.kx = kx; r.ky = ky; r.kz = kz;
  r.Sx = sel3(dx, dy, dz, kx) / dkz;
  r.Sy = sel3(dx, dy, dz, ky) / dkz;
  r.Sz = 1.0f / dkz;
  return r;
}

// Watertight test; returns true with t = T/det (as T * (1/det)) and the
// barycentric weights of v1 and v2.
__host__ __device__ inline bool tri_intersect(const RayPre& r, const float4& A4, const float4& B4,
                                              const float4& C4, float& t, float& b1, float& b2) {
#pragma clang fp contract(off)
  float Ax0 = A4.x - r.ox, Ay0 = A4.y - r.oy, Az0 = A4.z - r.oz;
  float Bx0 = B4.x - r.ox, By0 = B4.y - r.oy, Bz0 = B4.z - r.oz;
  float Cx0 = C4.x - r.ox, Cy0 = C4.y - r.oy, Cz0 = C4.z - r.oz;
  float Akx = sel3(Ax0, Ay0, Az0, r.kx), Aky = sel3(Ax0, Ay0, Az0, r.ky), Akz = sel3(Ax0, Ay0, Az0, r.kz);
  float Bkx = sel3(Bx0, By0, Bz0, r.kx), Bky = sel3(Bx0, By0, Bz0, r.ky), Bkz = sel3(Bx0, By0, Bz0, r.kz);
  float Ckx = sel3(Cx0, Cy0, Cz0, r.kx), Cky = sel3(Cx0, Cy0, Cz0, r.ky), Ckz = sel3(Cx0, Cy0, Cz0, r.kz);
  float Ax = Akx - r.Sx * Akz, Ay = Aky - r.Sy * Akz;
  float Bx = Bkx - r.Sx * Bkz, By = Bky - r.Sy * Bkz;
  float Cx = Ckx - r.Sx * Ckz, Cy = Cky - r.Sy * Ckz;
  float U = Cx * By - Cy * Bx;
  float V = Ax * Cy - Ay * Cx;
  float W = Bx * Ay - By * Ax;
  if (U == 0.0f || V == 0.0f || W == 0.0f) {
    U = (float)((double)Cx * (double)By - (double)Cy * (double)Bx);
    V = (float)((double)Ax * (double)Cy - (double)Ay * (double)Cx);
    W = (float)((double)Bx * (double)Ay - (double)By * (double)Ax);
  }
  if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
  float det = (U + V) + W;
  if (det == 0.0f) return false;
  float Az = r.Sz * Akz, Bz = r.Sz * Bkz, Cz = r.Sz * Ckz;
  float T = (U * Az + V * Bz) + W * Cz;
  float rc = 1.0f / det;
  t = T * rc;
  b1 = V * rc;
  b2 = W * rc;
  return true;
}

__host__ __device__ inline bool hit_better(float t, uint32_t inst, uint32_t prim, const Hit& h) {
  if (t < h.t) return true;
  if (t > h.t) return false;
  if (inst != h.inst) return inst < h.inst;
  return prim < h.prim;
}

// Slab test of the four children of a node.  Returns a 4-bit hit mask and
// the (conservatively lowered) entry distances.
__host__ __device__ inline uint32_t node_slabs(const BVHNode& n, const RayPre& r, float tmin, float tcur,
                                               float tn_out[4]) {
#pragma clang fp contract(off)
  const float lo_eps = 1.0f - 9.5367431640625e-07f;  // 1 - 2^-20
  const float hi_eps = 1.0f + 9.5367431640625e-07f;  // 1 + 2^-20
  uint32_t mask = 0;
#pragma unroll
  for (int c = 0; c < 4; ++c) {
    float x0 = (n.lo_x[c] - r.ox) * r.ix, x1 = (n.hi_x[c] - r.ox) * r.ix;
    float y0 = (n.lo_y[c] - r.oy) * r.iy, y1 = (n.hi_y[c] - r.oy) * r.iy;
    float z0 = (n.lo_z[c] - r.oz) * r.iz, z1 = (n.hi_z[c] - r.oz) * r.iz;
    float tn = fmaxf(fmaxf(fminf(x0, x1), fminf(y0, y1)), fminf(z0, z1));
    float tf = fminf(fminf(fmaxf(x0, x1), fmaxf(y0, y1)), fmaxf(z0, z1));
    tn = tn * (tn > 0.0f ? lo_eps : hi_eps);
    tf = tf * (tf > 0.0f ? hi_eps : lo_eps);
    float a = fmaxf(tn, tmin), b = fminf(tf, tcur);
    bool h = (n.child[c] != kEmpty) && (a <= b);
    tn_out[c] = a;
    mask |= h ? (1u << c) : 0u;
  }
  return mask;
}

// Test the triangles of a leaf; true if one was accepted.  ANY (or any_rt,
// the same choice made per lane at run time) stops at the first accepted
// triangle, as a shadow ray may.
template <bool ANY, bool COUNT>
__host__ __device__ inline bool leaf_test(const TriRec* __restrict__ tris, uint32_t ref, const RayPre& r,
                                          float tmin, float tmax, uint32_t inst, uint32_t skip_inst,
                                          uint32_t skip_prim, Hit& best, uint32_t& ntri, bool any_rt = false) {
  uint32_t first = leaf_first(ref), cnt = leaf_count(ref);
  bool found = false;
  for (uint32_t j = 0; j < cnt; ++j) {
    const TriRec tr = tris[first + j];
    if (COUNT) ntri++;
    uint32_t prim = f2u(tr.a.w);
    // intersect before the origin-triangle check so the record's three loads
    // issue together instead of waiting on the primitive id first
    float t, b1, b2;
    bool hit = tri_intersect(r, tr.a, tr.b, tr.c, t, b1, b2);
    if (!hit || (inst == skip_inst && prim == skip_prim)) continue;
    if (!(t > tmin && t < tmax)) continue;
    if (!hit_better(t, inst, prim, best)) continue;
    best.t = t;
    best.b1 = b1;
    best.b2 = b2;
    best.inst = inst;
    best.prim = prim;
    best.tri = first + j;
    best.mat = f2u(tr.b.w);
    found = true;
    if (ANY || any_rt) return true;
  }
  return found;
}

// compare-swap of (key, ref) pairs for the child sorting network
__host__ __device__ inline void cswap(float& ka, uint32_t& ra, float& kb, uint32_t& rb) {
  bool s = kb < ka;
  float k = s ? kb : ka;
  kb = s ? ka : kb;
  ka = k;
  uint32_t q = s ? rb : ra;
  rb = s ? ra : rb;
  ra = q;
}

// Walk one BVH4 from `root`.  Stack: push(ref, tnear), pop(ref, tnear),
// size().  Entries below `base` belong to an enclosing walk and are left
// alone.  ANY: return at the first accepted triangle (shadow rays).
template <bool ANY, bool COUNT, class Stack>
__host__ __device__ inline bool traverse_bvh(const BVHNode* __restrict__ nodes, const TriRec* __restrict__ tris,
                                             uint32_t root, const RayPre& r, float tmin, float tmax,
                                             uint32_t inst, uint32_t skip_inst, uint32_t skip_prim, Hit& best,
                                             Stack& st, uint32_t& nvis, uint32_t& ntri, int base = 0) {
  uint32_t cur = root;
  bool found = false;
  while (true) {
    if (cur != kEmpty && !ref_is_leaf(cur)) {
      const BVHNode n = nodes[cur];
      if (COUNT) nvis++;
      float tn[4];
      float tcur = fminf(best.t, tmax);
      uint32_t m = node_slabs(n, r, tmin, tcur, tn);
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
      cur = r0;
      continue;
    }
    if (cur != kEmpty) {
      if (leaf_test<ANY, COUNT>(tris, cur, r, tmin, tmax, inst, skip_inst, skip_prim, best, ntri)) {
        found = true;
        if (ANY) return true;
      }
    }
    // pop the next entry that can still hold a closer hit
    cur = kEmpty;
    while (st.size() > base) {
      float k;
      uint32_t q = st.pop(k);
      if (k <= fminf(best.t, tmax)) {
        cur = q;
        break;
      }
    }
    if (cur == kEmpty) break;
  }
  return found;
}

// World -> object transform of a ray, in the fixed FP32 order
// o'_r = ((w_r0 ox + w_r1 oy) + w_r2 oz) + w_r3,  d'_r = (w_r0 dx + w_r1 dy) + w_r2 dz.
__host__ __device__ inline RayPre ray_to_object(const float* w, float ox, float oy, float oz, float dx, float dy,
                                                float dz) {
#pragma clang fp contract(off)
  float o[3], d[3];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float* q = w + 4 * k;
    o[k] = ((q[0] * ox + q[1] * oy) + q[2] * oz) + q[3];
    d[k] = (q[0] * dx + q[1] * dy) + q[2] * dz;
  }
  return ray_prepare(o[0], o[1], o[2], d[0], d[1], d[2]);
}

// Two-level walk: a top-level BVH4 over instance world boxes whose leaves
// list instance ids; a top-level leaf pushes its instances as entries (leaf
// bit, count 0, instance id) with the leaf's key, and a popped instance entry
// moves the ray to object space and walks the mesh's BVH on top of the same
// stack — the stack discipline of the GPU's per-lane walk, so the two need
// the same stack depth.  t values are compared in each instance's object
// space, as the single-precision definition does.
template <bool ANY, bool COUNT, class Stack>
__host__ __device__ inline bool traverse_two_level(const BVHNode* __restrict__ tlas,
                                                   const uint32_t* __restrict__ tlas_items,
                                                   const InstRec* __restrict__ insts,
                                                   const BVHNode* __restrict__ nodes,
                                                   const TriRec* __restrict__ tris, const RayPre& rw, float tmin,
                                                   float tmax, uint32_t skip_inst, uint32_t skip_prim, Hit& best,
                                                   Stack& st, uint32_t& nvis, uint32_t& ntri) {
  uint32_t cur = 0;
  float cur_key = 0.0f;
  bool found = false;
  const int base = st.size();
  while (true) {
    if (cur != kEmpty && !ref_is_leaf(cur)) {
      const BVHNode n = tlas[cur];
      if (COUNT) nvis++;
      float tn[4];
      float tcur = fminf(best.t, tmax);
      uint32_t m = node_slabs(n, rw, tmin, tcur, tn);
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
      cur = r0;
      cur_key = k0;
      continue;
    }
    if (cur != kEmpty) {
      uint32_t first = leaf_first(cur), cnt = leaf_count(cur);
      if (cnt == 0) {  // an instance entry: walk its mesh in object space on top of the stack
        const InstRec& I = insts[first];
        RayPre ro = ray_to_object(I.w2o, rw.ox, rw.oy, rw.oz, rw.dx, rw.dy, rw.dz);
        if (traverse_bvh<ANY, COUNT>(nodes, tris, I.blas_root, ro, tmin, tmax, first, skip_inst, skip_prim, best,
                                     st, nvis, ntri, st.size())) {
          found = true;
          if (ANY) return true;
        }
      } else {
        for (int j = (int)cnt - 1; j >= 0; --j) st.push(kLeafBit | tlas_items[first + j], cur_key);
      }
    }
    cur = kEmpty;
    while (st.size() > base) {
      float k;
      uint32_t q = st.pop(k);
      if (k <= fminf(best.t, tmax)) {
        cur = q;
        cur_key = k;
        break;
      }
    }
    if (cur == kEmpty) break;
  }
  return found;
}

// Brute force over every instance and every triangle of its mesh.
__host__ __device__ inline bool brute_force_two_level(const InstRec* __restrict__ insts, uint32_t n_insts,
                                                      const TriRec* __restrict__ tris,
                                                      const uint32_t* __restrict__ mesh_tri_first,
                                                      const uint32_t* __restrict__ mesh_tri_count, const RayPre& rw,
                                                      float tmin, float tmax, Hit& best) {
  bool found = false;
  for (uint32_t i = 0; i < n_insts; ++i) {
    const InstRec& I = insts[i];
    RayPre ro = ray_to_object(I.w2o, rw.ox, rw.oy, rw.oz, rw.dx, rw.dy, rw.dz);
    uint32_t first = mesh_tri_first[I.mesh], cnt = mesh_tri_count[I.mesh];
    for (uint32_t k = 0; k < cnt; ++k) {
      const TriRec tr = tris[first + k];
      float t, b1, b2;
      if (!tri_intersect(ro, tr.a, tr.b, tr.c, t, b1, b2)) continue;
      if (!(t > tmin && t < tmax)) continue;
      uint32_t prim = f2u(tr.a.w);
      if (!hit_better(t, i, prim, best)) continue;
      best.t = t; best.b1 = b1; best.b2 = b2; best.inst = i; best.prim = prim; best.tri = first + k;
      best.mat = f2u(tr.b.w);
      found = true;
    }
  }
  return found;
}

// Brute force over every triangle record: the same definition without the BVH.
template <bool COUNT>
__host__ __device__ inline bool brute_force(const TriRec* __restrict__ tris, uint32_t n_tris, const RayPre& r,
                                            float tmin, float tmax, uint32_t inst, Hit& best, uint32_t& ntri) {
  bool found = false;
  for (uint32_t i = 0; i < n_tris; ++i) {
    const TriRec tr = tris[i];
    if (COUNT) ntri++;
    float t, b1, b2;
    if (!tri_intersect(r, tr.a, tr.b, tr.c, t, b1, b2)) continue;
    if (!(t > tmin && t < tmax)) continue;
    uint32_t prim = f2u(tr.a.w);
    if (!hit_better(t, inst, prim, best)) continue;
    best.t = t; best.b1 = b1; best.b2 = b2; best.inst = inst; best.prim = prim; best.tri = i;
    best.mat = f2u(tr.b.w);
    found = true;
  }
  return found;
}

// Host-side stack for CPU checks of the traversal: a push beyond `cap`
// entries is dropped and flagged, as on the GPU; `high` records the deepest
// the stack has been.
struct HostStack {
  static constexpr int kMax = 512;
  uint32_t ref[kMax];
  float key[kMax];
  int sp = 0, cap = kMax, high = 0;
  bool overflow = false;
  void push(uint32_t r, float k) {
    if (sp >= cap) { overflow = true; return; }
    ref[sp] = r; key[sp] = k; sp++;
    if (sp > high) high = sp;
  }
  uint32_t pop(float& k) { --sp; k = key[sp]; return ref[sp]; }
  int size() const { return sp; }
};

}  // namespace pt
