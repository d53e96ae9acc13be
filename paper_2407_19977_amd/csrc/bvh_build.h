// Host BVH builder: binned-SAH binary BVH, collapsed to 128-byte BVH4 nodes.
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

#include "pt_layout.h"

namespace pt {

struct Bvh4 {
  std::vector<BVHNode> nodes;  // nodes[0] is the root
  std::vector<TriRec> tris;    // leaf order
  int depth = 0;               // nodes on the longest root-to-leaf path
  int max_leaf = 0;
  double sah_cost = 0.0;
  double build_ms = 0.0;
  float lo[3] = {0, 0, 0}, hi[3] = {0, 0, 0};
};

// verts: [n][3][3] triangle vertices; prim_ids / mat_ids: [n].
// Returns false (and sets err) on invalid input.
bool build_bvh4(const float* verts, const uint32_t* prim_ids, const uint32_t* mat_ids, int64_t n,
                Bvh4& out, std::string& err);

}  // namespace pt
