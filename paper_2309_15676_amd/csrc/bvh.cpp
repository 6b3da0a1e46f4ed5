// Host builder of the triangle BVH: top-down, binned surface-area heuristic
// (Wald, "On fast construction of SAH-based bounding volume hierarchies",
// 2007), two children per node, nodes in depth-first order.
#include "bvh.h"

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <limits>

namespace jso {
namespace {

constexpr float kBig = std::numeric_limits<float>::max();

struct Box {
  float lo[3] = {kBig, kBig, kBig}, hi[3] = {-kBig, -kBig, -kBig};
  void grow(const float* p) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], p[a]);
      hi[a] = std::max(hi[a], p[a]);
    }
  }
  void grow(const Box& b) {
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], b.lo[a]);
      hi[a] = std::max(hi[a], b.hi[a]);
    }
  }
  bool empty() const { return lo[0] > hi[0]; }
  double area() const {
    if (empty()) return 0.0;
    const double x = hi[0] - lo[0], y = hi[1] - lo[1], z = hi[2] - lo[2];
    return 2.0 * (x * y + y * z + z * x);
  }
};

constexpr int kBins = 16;
constexpr double kCostTrav = 1.0;  // cost of one node visit, in triangle tests
constexpr int kLeafTarget = 4;     // the heuristic makes leaves of at most this many
// The last inner levels before the stack limit split at the centroid median,
// which halves the count per level whatever the geometry.
constexpr int kMedianLevels = 8;

struct Builder {
  const float* V = nullptr;
  const int* T = nullptr;
  std::vector<Box> pbox;     // per triangle
  std::vector<float> cen;    // per triangle centroid, xyz
  std::vector<int> idx;      // triangle ids, partitioned in place
  BvhBuild* out = nullptr;
  std::string err;

  Box range_box(int b, int e) const {
    Box r;
    for (int i = b; i < e; ++i) r.grow(pbox[idx[i]]);
    return r;
  }

  int32_t leaf(int b, int e) {
    const int first = (int)out->order.size();
    for (int i = b; i < e; ++i) {
      const int t = idx[i];
      const int* tv = T + 3 * (size_t)t;
      float w[kTriWords];
      for (int a = 0; a < 3; ++a) {
        const double v0 = V[3 * (size_t)tv[0] + a];
        w[a] = (float)v0;
        w[4 + a] = (float)((double)V[3 * (size_t)tv[1] + a] - v0);
        w[8 + a] = (float)((double)V[3 * (size_t)tv[2] + a] - v0);
      }
      std::memcpy(&w[3], &tv[0], 4);
      std::memcpy(&w[7], &tv[1], 4);
      std::memcpy(&w[11], &tv[2], 4);
      out->tris.insert(out->tris.end(), w, w + kTriWords);
      out->order.push_back(t);
    }
    return ~(int32_t)(((uint32_t)first << kLeafBits) | (uint32_t)(e - b));
  }

  // Split [b, e) in two non-empty parts; returns the split position.
  int split(int b, int e, int level, double* cost) {
    const int n = e - b;
    Box cb;
    for (int i = b; i < e; ++i) cb.grow(&cen[3 * (size_t)idx[i]]);
    int axis = 0;
    for (int a = 1; a < 3; ++a)
      if (cb.hi[a] - cb.lo[a] > cb.hi[axis] - cb.lo[axis]) axis = a;
    *cost = std::numeric_limits<double>::infinity();
    if (!(cb.hi[axis] > cb.lo[axis])) {
      // every centroid coincides: halve the range
      return b + n / 2;
    }
    if (level > kBvh2MaxDepth - kMedianLevels) {
      const int mid = b + n / 2;
      std::nth_element(idx.begin() + b, idx.begin() + mid, idx.begin() + e, [&](int x, int y) {
        return cen[3 * (size_t)x + axis] < cen[3 * (size_t)y + axis];
      });
      return mid;
    }
    const double parent = range_box(b, e).area();
    int best_axis = -1, best_plane = -1;
    double best = std::numeric_limits<double>::infinity();
    for (int a = 0; a < 3; ++a) {
      const double ext = (double)cb.hi[a] - (double)cb.lo[a];
      if (!(ext > 0.0)) continue;
      Box bb[kBins];
      int cnt[kBins] = {0};
      const double scale = kBins / ext;
      for (int i = b; i < e; ++i) {
        const int t = idx[i];
        int k = (int)(((double)cen[3 * (size_t)t + a] - cb.lo[a]) * scale);
        k = std::min(std::max(k, 0), kBins - 1);
        ++cnt[k];
        bb[k].grow(pbox[t]);
      }
      double right_area[kBins];
      int right_cnt[kBins];
      Box acc;
      int c = 0;
      for (int k = kBins - 1; k > 0; --k) {
        acc.grow(bb[k]);
        c += cnt[k];
        right_area[k] = acc.area();
        right_cnt[k] = c;
      }
      acc = Box();
      c = 0;
      for (int k = 0; k < kBins - 1; ++k) {
        acc.grow(bb[k]);
        c += cnt[k];
        const int nr = right_cnt[k + 1];
        if (c == 0 || nr == 0) continue;
        const double sah = acc.area() * c + right_area[k + 1] * nr;
        if (sah < best) {
          best = sah;
          best_axis = a;
          best_plane = k;
        }
      }
    }
    if (best_axis < 0) return b + n / 2;
    *cost = kCostTrav + (parent > 0.0 ? best / parent : (double)n);
    const int a = best_axis;
    const double ext = (double)cb.hi[a] - (double)cb.lo[a];
    const double scale = kBins / ext;
    int* mid = std::partition(idx.data() + b, idx.data() + e, [&](int t) {
      int k = (int)(((double)cen[3 * (size_t)t + a] - cb.lo[a]) * scale);
      k = std::min(std::max(k, 0), kBins - 1);
      return k <= best_plane;
    });
    return (int)(mid - idx.data());
  }

  // Subtree over [b, e) whose root, if inner, sits at inner level `level`
  // (root = 1).  Returns its link and its bounds.
  int32_t build(int b, int e, int level, Box& box) {
    box = range_box(b, e);
    const int n = e - b;
    if (level > kBvh2MaxDepth) {
      if (n > kLeafMax) {
        char msg[160];
        std::snprintf(msg, sizeof(msg),
                      "BVH: %d triangles share one leaf at the depth limit %d "
                      "(degenerate mesh)", n, kBvh2MaxDepth);
        err = msg;
        return 0;
      }
      return leaf(b, e);
    }
    // the root is always an inner node
    if (level > 1 && n == 1) return leaf(b, e);
    double split_cost = 0.0;
    const int m = n > 1 ? split(b, e, level, &split_cost) : b;
    // leaf cost: one test per triangle
    if (level > 1 && n <= kLeafTarget && (double)n <= split_cost) return leaf(b, e);
    const int node = (int)out->nodes.size();
    out->nodes.push_back(BvhNode{});
    out->depth = std::max(out->depth, level);
    Box bl, br;
    int32_t l0, l1;
    if (n == 1) {
      // a one-triangle mesh: the second child is an empty leaf
      l0 = leaf(b, e);
      bl = box;
      l1 = ~(int32_t)(0u);
      br = Box();
      for (int a = 0; a < 3; ++a) br.lo[a] = br.hi[a] = box.lo[a];
    } else {
      l0 = build(b, m, level + 1, bl);
      if (!err.empty()) return 0;
      l1 = build(m, e, level + 1, br);
      if (!err.empty()) return 0;
    }
    BvhNode& N = out->nodes[node];
    for (int a = 0; a < 3; ++a) {
      N.lo0[a] = bl.lo[a];
      N.hi0[a] = bl.hi[a];
      N.lo1[a] = br.lo[a];
      N.hi1[a] = br.hi[a];
    }
    N.link0 = l0;
    N.link1 = l1;
    return node;
  }
};

// Collapse the binary hierarchy into four-wide nodes: a node's children start
// as the binary node's two, and the inner child with the largest box surface
// is replaced by its own two children until there are four or only leaves
// are left.  Nodes are numbered breadth-first (the top levels come first).
struct Child {
  float lo[3], hi[3];
  int32_t link;  // binary-hierarchy link
};

double child_area(const Child& c) {
  const double x = c.hi[0] - c.lo[0], y = c.hi[1] - c.lo[1], z = c.hi[2] - c.lo[2];
  return 2.0 * (x * y + y * z + z * x);
}

void collapse(BvhBuild& b) {
  const std::vector<BvhNode>& N = b.nodes;
  auto kids = [&](int32_t node, std::vector<Child>& out) {
    const BvhNode& n = N[node];
    Child a, c;
    for (int k = 0; k < 3; ++k) {
      a.lo[k] = n.lo0[k];
      a.hi[k] = n.hi0[k];
      c.lo[k] = n.lo1[k];
      c.hi[k] = n.hi1[k];
    }
    a.link = n.link0;
    c.link = n.link1;
    out.push_back(a);
    out.push_back(c);
  };
  struct Item {
    int32_t bin;   // binary node this four-wide node stands for
    int level;     // inner level (root = 1)
    int stack;     // pushes on the path above it
  };
  std::vector<Item> queue{{0, 1, 0}};
  b.nodes4.clear();
  b.nodes4.push_back(Bvh4Node{});
  b.depth4 = 0;
  b.stack4 = 0;
  for (size_t q = 0; q < queue.size(); ++q) {
    const Item it = queue[q];
    std::vector<Child> ch;
    kids(it.bin, ch);
    while (ch.size() < 4) {
      int best = -1;
      double area = -1.0;
      for (int i = 0; i < (int)ch.size(); ++i)
        if (ch[i].link >= 0 && child_area(ch[i]) > area) {
          area = child_area(ch[i]);
          best = i;
        }
      if (best < 0) break;
      const int32_t inner = ch[best].link;
      ch.erase(ch.begin() + best);
      kids(inner, ch);
    }
    const int pushes = it.stack + (int)ch.size() - 1;
    b.stack4 = std::max(b.stack4, pushes);
    b.depth4 = std::max(b.depth4, it.level);
    Bvh4Node nd{};
    for (int k = 0; k < 4; ++k) {
      if (k < (int)ch.size()) {
        const Child& c = ch[k];
        nd.lo_x[k] = c.lo[0];
        nd.hi_x[k] = c.hi[0];
        nd.lo_y[k] = c.lo[1];
        nd.hi_y[k] = c.hi[1];
        nd.lo_z[k] = c.lo[2];
        nd.hi_z[k] = c.hi[2];
        if (c.link >= 0) {
          nd.link[k] = (int32_t)b.nodes4.size();
          b.nodes4.push_back(Bvh4Node{});
          queue.push_back({c.link, it.level + 1, pushes});
        } else {
          nd.link[k] = c.link;
        }
      } else {  // unused slot: an empty leaf with a point box
        nd.lo_x[k] = nd.hi_x[k] = ch[0].lo[0];
        nd.lo_y[k] = nd.hi_y[k] = ch[0].lo[1];
        nd.lo_z[k] = nd.hi_z[k] = ch[0].lo[2];
        nd.link[k] = ~(int32_t)0;
      }
    }
    b.nodes4[q] = nd;
  }
}

}  // namespace

std::string build_bvh(const float* verts, int n_verts, const int* tris, int n_tris,
                      BvhBuild& out) {
  out = BvhBuild();
  if (n_tris <= 0) return "BVH: no triangles";
  if ((int64_t)n_tris > ((int64_t)1 << (31 - kLeafBits)))
    return "BVH: too many triangles";
  Builder B;
  B.V = verts;
  B.T = tris;
  B.out = &out;
  B.pbox.resize(n_tris);
  B.cen.resize(3 * (size_t)n_tris);
  B.idx.resize(n_tris);
  Box all;
  for (int t = 0; t < n_tris; ++t) {
    const int* tv = tris + 3 * (size_t)t;
    for (int k = 0; k < 3; ++k)
      if (tv[k] < 0 || tv[k] >= n_verts) return "BVH: vertex index out of range";
    Box b;
    for (int k = 0; k < 3; ++k) {
      const float* p = verts + 3 * (size_t)tv[k];
      for (int a = 0; a < 3; ++a)
        if (!std::isfinite(p[a])) return "BVH: non-finite vertex";
      b.grow(p);
    }
    B.pbox[t] = b;
    for (int a = 0; a < 3; ++a) B.cen[3 * (size_t)t + a] = 0.5f * (b.lo[a] + b.hi[a]);
    B.idx[t] = t;
    all.grow(b);
  }
  out.nodes.reserve(2 * (size_t)n_tris / kLeafTarget + 1);
  out.tris.reserve(kTriWords * (size_t)n_tris);
  out.order.reserve(n_tris);
  Box root;
  B.build(0, n_tris, 1, root);
  if (!B.err.empty()) return B.err;
  // Widen every box a little so the FP32 slab test (about one rounding per
  // operation) never rejects a box whose triangle the ray meets, including
  // flat boxes of axis-aligned geometry.
  float ext = 0.0f;
  for (int a = 0; a < 3; ++a) ext = std::max(ext, all.hi[a] - all.lo[a]);
  const float pad = 1e-5f * std::max(ext, 1.0f);
  auto widen = [&](float* lo, float* hi) {
    for (int a = 0; a < 3; ++a) {
      lo[a] -= pad + std::fabs(lo[a]) * 0x1p-18f;
      hi[a] += pad + std::fabs(hi[a]) * 0x1p-18f;
    }
  };
  for (BvhNode& N : out.nodes) {
    widen(N.lo0, N.hi0);
    widen(N.lo1, N.hi1);
  }
  collapse(out);
  if (out.stack4 > kBvhMaxStack) {
    char msg[160];
    std::snprintf(msg, sizeof(msg), "BVH: traversal needs %d stack entries (limit %d)",
                  out.stack4, kBvhMaxStack);
    return msg;
  }
  return "";
}

}  // namespace jso
