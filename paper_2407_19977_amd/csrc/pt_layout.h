// Device data layouts of the path tracer (HBM resident), shared by the host
// library and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pt {

// ---------------------------------------------------------------------------
// BVH4 node: 128 bytes = one cache line per visit.  Child boxes are stored
// structure-of-arrays so the four slab tests run on float4 lanes; a child
// reference is a node index (bit 31 clear), a leaf (bit 31 set: triangle
// count in bits 27..29, first triangle in bits 0..26), or kEmpty.
// ---------------------------------------------------------------------------
struct alignas(128) BVHNode {
  float lo_x[4], hi_x[4], lo_y[4], hi_y[4], lo_z[4], hi_z[4];
  uint32_t child[4];
  uint32_t meta[4];  // meta[0]: number of valid children
};
static_assert(sizeof(BVHNode) == 128, "BVH node must be one 128-byte line");

constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kLeafBit = 0x80000000u;
constexpr int kLeafCountShift = 27;
constexpr uint32_t kLeafFirstMask = (1u << kLeafCountShift) - 1u;
#ifndef PT_MAX_LEAF_TRIS
#define PT_MAX_LEAF_TRIS 4
#endif
constexpr int kMaxLeafTris = PT_MAX_LEAF_TRIS;  // at most 7 (3-bit count in a leaf reference)
static_assert(kMaxLeafTris >= 1 && kMaxLeafTris <= 7, "leaf references hold 3-bit triangle counts");

// Traversal stack entries a walk can need.  A depth-first walk that pushes
// the (at most three) siblings it does not descend into keeps at most three
// entries per inner level on the stack; a top-level leaf adds its instances
// (at most kMaxLeafTris) as entries, one of which is popped at once, before
// a mesh walk starts on top.  `depth` counts the levels of nodes and leaves
// on the longest path (top-level plus mesh levels for two-level scenes).
__host__ __device__ constexpr int stack_capacity(int depth) {
  return 3 * (depth > 1 ? depth : 1) + kMaxLeafTris;
}

__host__ __device__ inline bool ref_is_leaf(uint32_t r) { return (r & kLeafBit) != 0u; }
__host__ __device__ inline uint32_t leaf_count(uint32_t r) { return (r >> kLeafCountShift) & 7u; }
__host__ __device__ inline uint32_t leaf_first(uint32_t r) { return r & kLeafFirstMask; }
__host__ __device__ inline uint32_t make_leaf(uint32_t first, uint32_t count) {
  return kLeafBit | (count << kLeafCountShift) | first;
}

// Triangle record, 48 bytes, in BVH leaf order:
//   a = (v0.xyz, primitive id bits), b = (v1.xyz, material id bits), c = (v2.xyz, unused)
struct alignas(16) TriRec {
  float4 a, b, c;
};
static_assert(sizeof(TriRec) == 48, "triangle record is 48 bytes");

// Material classes: each has its own shading kernel so a wave shades one
// kind of surface (material-sorted shading).
enum MatClass : int {
  kClsMiss = 0,     // ray left the scene: environment lookup
  kClsAbsorb = 1,   // no scattering lobe (e.g. a pure emitter)
  kClsDiffuse = 2,  // Lambert only
  kClsMetal = 3,    // metalness 1, no coat / transmission
  kClsPlastic = 4,  // dielectric over diffuse, optional coat
  kClsGlass = 5,    // transmission (no coat)
  kClsGeneral = 6,  // anything else
  kNumClasses = 7
};

// Device material record, 192 bytes, derived on the host from the OpenPBR parameters.
struct alignas(32) MatRec {
  float base_color[3];  float base_weight;
  float metalness;      float spec_weight;  float spec_ior;     float trans_weight;
  float spec_color[3];  float coat_weight;
  float trans_color[3]; float coat_ior;
  float coat_color[3];  float bwbc_lum;     // lum(base_weight * base_color)
  float Le[3];          uint32_t flags;     // emission radiance; flags below
  float at, ab, ac;     int32_t cls;        // GGX alphas (specular t/b, coat), class
  float spec_rough;     float f0_diel;      // specular roughness; F_dielectric(1, eta')
  float eon_a, eon_b;   // diffuse roughness sigma as FON's A = 1/(1 + (1/2 - 2/(3 pi)) sigma), B = sigma A
  float film_w;         float film_ior;     // thin film on the dielectric interface: weight (0: none), IOR
  float film_d_nm;                          // its thickness in nm
  float fuzz_w;         float fuzz_color[3]; float fuzz_a;  // fuzz: weight (0: none), colour, sheen alpha
  const float* fuzz_E;  // its directional albedo at mu = k/64, k = 0..64 (device memory; null without fuzz)
  float kd[3];          float kd_lum;       // diffuse lobe albedo: (1 - ssw) bw bc + ssw subsurface_color; its lum
  float pad[2];
};
static_assert(sizeof(MatRec) == 192, "material record is 192 bytes");
constexpr uint32_t kMatSpecDelta = 1u, kMatCoatDelta = 2u, kMatEmissive = 4u;

// Instance of a mesh in the two-level hierarchy, 128 bytes.  w2o is the
// rigid inverse of o2w computed in double and rounded to float; rays enter
// object space as o' = ((w0 ox + w1 oy) + w2 oz) + w3 per row (no FMA).
struct alignas(128) InstRec {
  float w2o[12];         // world -> object, row-major 3x4
  float o2w[12];         // object -> world, row-major 3x4
  uint32_t blas_root;    // node index of the mesh's BVH root
  int32_t mat_override;  // -1: per-triangle material ids
  int32_t light_map;     // offset of this instance's primitive -> light table, -1 if none
  uint32_t mesh;
  uint32_t pad[4];
};
static_assert(sizeof(InstRec) == 128, "instance record is 128 bytes");

// Emissive triangle in world space (for next-event estimation).
struct alignas(16) LightTri {
  float4 p0;   // xyz, area
  float4 p1;   // xyz, selection probability
  float4 p2;   // xyz, unused
  float4 ng;   // unit normal xyz, lum-weighted power (unused)
  float4 Le;   // radiance rgb, unused
};

}  // namespace pt
