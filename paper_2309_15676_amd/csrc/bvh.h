// Bounding volume hierarchy over a triangle mesh: the memory layout the
// traversal kernels read, and the host builder (binned surface-area
// heuristic).
#pragma once

#include <stdint.h>

#include <string>
#include <vector>

namespace jso {

// The builder first makes a binary hierarchy (BvhNode: the boxes of both
// children and their links) and then collapses it into four-wide nodes
// (Bvh4Node), which the kernels traverse.
//
// Links: a link >= 0 names an inner node.  A leaf is stored in its parent's
// link as ~(first << kLeafBits | count): `count` triangles from `first` in the
// reordered triangle array (count 0: an empty slot).  The root is node 0.
constexpr int kLeafBits = 5;
constexpr int kLeafMax = (1 << kLeafBits) - 1;  // triangles per leaf at most
// Inner depth cap of the binary hierarchy (the last levels before it split at
// the centroid median).
constexpr int kBvh2MaxDepth = 48;
// Traversal-stack entries per lane the kernels allow.  A four-wide node defers
// up to 3 children, so the stack a tree needs is the largest sum of
// (children - 1) over the nodes of a root-to-node path (BvhBuild::stack4).
constexpr int kBvhMaxStack = 64;

struct BvhNode {
  float lo0[3], hi0[3], lo1[3], hi1[3];
  int32_t link0, link1;
  int32_t pad[2];
};
static_assert(sizeof(BvhNode) == 64, "node layout");

// Four-wide node (128 bytes, eight 16-byte words), children's boxes as
// structure of arrays:
//   lo.x[4] | hi.x[4] | lo.y[4] | hi.y[4] | lo.z[4] | hi.z[4] | link[4] | -
// Unused slots hold an empty leaf (link ~0) with a point box.
struct Bvh4Node {
  float lo_x[4], hi_x[4], lo_y[4], hi_y[4], lo_z[4], hi_z[4];
  int32_t link[4];
  int32_t pad[4];
};
static_assert(sizeof(Bvh4Node) == 128, "node layout");

// Reordered triangle (48 bytes, three 16-byte words): (v0, i0), (e1, i1),
// (e2, i2) with e1 = v1 - v0, e2 = v2 - v0 and the vertex indices i0..i2 as
// the bits of the fourth components.
constexpr int kTriWords = 12;

struct BvhBuild {
  std::vector<BvhNode> nodes;  // binary hierarchy (depth-first order)
  std::vector<float> tris;     // kTriWords floats per triangle, leaf order
  std::vector<int32_t> order;  // original index of each reordered triangle
  int depth = 0;               // inner depth of the binary hierarchy
  // four-wide hierarchy over the same leaves, nodes in breadth-first order
  std::vector<Bvh4Node> nodes4;
  int depth4 = 0;              // its inner depth
  int stack4 = 0;              // traversal-stack entries it needs
};

// Build the hierarchy of n_tris triangles (vertex indices `tris`, 3 per
// triangle) over n_verts vertices (`verts`, xyz).  Returns "" on success, else
// a description of what is wrong with the mesh.
std::string build_bvh(const float* verts, int n_verts, const int* tris, int n_tris,
                      BvhBuild& out);

}  // namespace jso
