// Bounding volume hierarchy over a triangle mesh: the memory layout the
// traversal kernels read, and the host builder (binned surface-area
// heuristic).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace jso {

// Node (64 bytes, four 16-byte words): the boxes of its two children and their
// links, in the order
//   lo0.xyz hi0.x | hi0.yz lo1.xy | lo1.z hi1.xyz | link0 link1 - -
// A link >= 0 names an inner node.  A leaf is stored in its parent's link as
// ~(first << kLeafBits | count): `count` triangles from `first` in the
// reordered triangle array.  The root is node 0.
constexpr int kLeafBits = 5;
constexpr int kLeafMax = (1 << kLeafBits) - 1;  // triangles per leaf at most
// Traversal keeps at most one deferred child per inner level on its stack, so
// a tree of inner depth D (root alone = 1) needs D stack entries.
constexpr int kBvhMaxStack = 32;

struct BvhNode {
  float lo0[3], hi0[3], lo1[3], hi1[3];
  int32_t link0, link1;
  int32_t pad[2];
};
static_assert(sizeof(BvhNode) == 64, "node layout");

// Reordered triangle (48 bytes, three 16-byte words): (v0, i0), (e1, i1),
// (e2, i2) with e1 = v1 - v0, e2 = v2 - v0 and the vertex indices i0..i2 as
// the bits of the fourth components.
constexpr int kTriWords = 12;

struct BvhBuild {
  std::vector<BvhNode> nodes;
  std::vector<float> tris;     // kTriWords floats per triangle, leaf order
  std::vector<int32_t> order;  // original index of each reordered triangle
  int depth = 0;               // inner depth (stack entries the traversal needs)
};

// Build the hierarchy of n_tris triangles (vertex indices `tris`, 3 per
// triangle) over n_verts vertices (`verts`, xyz).  Returns "" on success, else
// a description of what is wrong with the mesh.
std::string build_bvh(const float* verts, int n_verts, const int* tris, int n_tris,
                      BvhBuild& out);

}  // namespace jso
