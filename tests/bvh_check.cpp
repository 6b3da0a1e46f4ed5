// Structural check of the host BVH builder (CPU only): reads a mesh
// (int32 n_verts, n_tris; float verts[n_verts][3]; int32 tris[n_tris][3]) from
// the file named by argv[1], builds the hierarchy and verifies
//   - every triangle sits in exactly one leaf, with its own vertices,
//   - every child box contains the triangles of its subtree,
//   - every inner node is reachable once and the inner depth is within the
//     traversal stack,
//   - a closest-hit search through the boxes finds the same triangle as a
//     brute-force search over all triangles, for random rays.
// The same for the four-wide hierarchy the kernels traverse, whose stack use
// in a nearest-first traversal must stay within the bound the builder reports.
// Prints "ok <depth> <nodes> <hits>" or the first violation.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <random>
#include <vector>

#include "bvh.h"

using namespace jso;

static int fail(const char* m) {
  std::printf("FAIL %s\n", m);
  return 1;
}

struct Ctx {
  const BvhBuild* b;
  std::vector<int> seen_node, seen_tri;
  int max_level = 0;
};

static bool inside(const float* lo, const float* hi, const float* p) {
  for (int a = 0; a < 3; ++a)
    if (p[a] < lo[a] || p[a] > hi[a]) return false;
  return true;
}

// walk a link; check boxes against triangles
static bool walk(Ctx& c, int32_t link, const float* lo, const float* hi, int level) {
  if (link >= 0) {
    if (link >= (int)c.b->nodes.size() || c.seen_node[link]++) return false;
    c.max_level = std::max(c.max_level, level);
    const BvhNode& N = c.b->nodes[link];
    return walk(c, N.link0, N.lo0, N.hi0, level + 1) && walk(c, N.link1, N.lo1, N.hi1, level + 1);
  }
  const uint32_t v = ~(uint32_t)link;
  const int first = (int)(v >> kLeafBits), cnt = (int)(v & kLeafMax);
  for (int i = first; i < first + cnt; ++i) {
    if (i >= (int)c.b->order.size() || c.seen_tri[i]++) return false;
    const float* w = &c.b->tris[(size_t)kTriWords * i];
    float p[3][3];
    for (int a = 0; a < 3; ++a) {
      p[0][a] = w[a];
      p[1][a] = w[a] + w[4 + a];
      p[2][a] = w[a] + w[8 + a];
    }
    for (int k = 0; k < 3; ++k)
      if (!inside(lo, hi, p[k])) return false;
  }
  return true;
}

// FP64 Moller-Trumbore on original vertices
static double tri_t(const float* V, const int* T, int k, const double* o, const double* d) {
  const int* tv = T + 3 * (size_t)k;
  double v0[3], e1[3], e2[3];
  for (int a = 0; a < 3; ++a) {
    v0[a] = V[3 * tv[0] + a];
    e1[a] = V[3 * tv[1] + a] - v0[a];
    e2[a] = V[3 * tv[2] + a] - v0[a];
  }
  auto cross = [](const double* x, const double* y, double* r) {
    r[0] = x[1] * y[2] - x[2] * y[1];
    r[1] = x[2] * y[0] - x[0] * y[2];
    r[2] = x[0] * y[1] - x[1] * y[0];
  };
  auto dot = [](const double* x, const double* y) { return x[0] * y[0] + x[1] * y[1] + x[2] * y[2]; };
  double pv[3], qv[3], sv[3];
  cross(d, e2, pv);
  const double det = dot(e1, pv);
  if (det == 0) return INFINITY;
  for (int a = 0; a < 3; ++a) sv[a] = o[a] - v0[a];
  const double u = dot(sv, pv) / det;
  cross(sv, e1, qv);
  const double v = dot(d, qv) / det;
  const double t = dot(e2, qv) / det;
  if (u < 0 || v < 0 || u + v > 1 || !(t > 0)) return INFINITY;
  return t;
}

static bool box_hit(const float* lo, const float* hi, const double* o, const double* d, double tmax) {
  double t0 = 0, t1 = tmax;
  for (int a = 0; a < 3; ++a) {
    if (d[a] == 0) {
      if (o[a] < lo[a] || o[a] > hi[a]) return false;
      continue;
    }
    double ta = (lo[a] - o[a]) / d[a], tb = (hi[a] - o[a]) / d[a];
    if (ta > tb) std::swap(ta, tb);
    t0 = std::max(t0, ta);
    t1 = std::min(t1, tb);
  }
  return t0 <= t1;
}

static bool walk4(const BvhBuild& b, std::vector<int>& seen_node, std::vector<int>& seen_tri,
                  int32_t link, const float* lo, const float* hi, int level, int& max_level) {
  if (link >= 0) {
    if (link >= (int)b.nodes4.size() || seen_node[link]++) return false;
    max_level = std::max(max_level, level);
    const Bvh4Node& N = b.nodes4[link];
    for (int k = 0; k < 4; ++k) {
      const float clo[3] = {N.lo_x[k], N.lo_y[k], N.lo_z[k]};
      const float chi[3] = {N.hi_x[k], N.hi_y[k], N.hi_z[k]};
      if (!walk4(b, seen_node, seen_tri, N.link[k], clo, chi, level + 1, max_level)) return false;
    }
    return true;
  }
  const uint32_t v = ~(uint32_t)link;
  const int first = (int)(v >> kLeafBits), cnt = (int)(v & kLeafMax);
  for (int i = first; i < first + cnt; ++i) {
    if (i >= (int)b.order.size() || seen_tri[i]++) return false;
    const float* w = &b.tris[(size_t)kTriWords * i];
    for (int k = 0; k < 3; ++k) {
      float p[3];
      for (int a = 0; a < 3; ++a) p[a] = w[a] + (k == 1 ? w[4 + a] : k == 2 ? w[8 + a] : 0.0f);
      if (!inside(lo, hi, p)) return false;
    }
  }
  return true;
}

// nearest-first traversal of the four-wide hierarchy (FP64 box tests);
// returns the largest stack depth it used
static int closest4(const BvhBuild& b, const float* V, const int* T, const double* o,
                    const double* d, double& best, int& best_tri) {
  std::vector<int32_t> st;
  int max_sp = 0;
  int32_t link = 0;
  for (;;) {
    if (link >= 0) {
      const Bvh4Node& N = b.nodes4[link];
      std::vector<std::pair<double, int32_t>> hit;
      for (int k = 0; k < 4; ++k) {
        const float lo[3] = {N.lo_x[k], N.lo_y[k], N.lo_z[k]};
        const float hi[3] = {N.hi_x[k], N.hi_y[k], N.hi_z[k]};
        if (box_hit(lo, hi, o, d, best)) {
          double t0 = 0;
          for (int a = 0; a < 3; ++a)
            if (d[a] != 0) t0 = std::max(t0, std::min((lo[a] - o[a]) / d[a], (hi[a] - o[a]) / d[a]));
          hit.push_back({t0, N.link[k]});
        }
      }
      if (!hit.empty()) {
        std::sort(hit.begin(), hit.end(),
                  [](const std::pair<double, int32_t>& x, const std::pair<double, int32_t>& y) {
                    return x.first < y.first;
                  });
        for (size_t k = hit.size() - 1; k >= 1; --k) st.push_back(hit[k].second);
        max_sp = std::max(max_sp, (int)st.size());
        link = hit[0].second;
        continue;
      }
    } else {
      const uint32_t v = ~(uint32_t)link;
      const int first = (int)(v >> kLeafBits), cnt = (int)(v & kLeafMax);
      for (int i = first; i < first + cnt; ++i) {
        const int t = b.order[i];
        const double x = tri_t(V, T, t, o, d);
        if (x < best || (x == best && t < best_tri)) {
          best = x;
          best_tri = t;
        }
      }
    }
    if (st.empty()) break;
    link = st.back();
    st.pop_back();
  }
  return max_sp;
}

static void closest(const BvhBuild& b, const float* V, const int* T, int32_t link, const double* o,
                    const double* d, double& best, int& best_tri) {
  if (link >= 0) {
    const BvhNode& N = b.nodes[link];
    if (box_hit(N.lo0, N.hi0, o, d, best)) closest(b, V, T, N.link0, o, d, best, best_tri);
    if (box_hit(N.lo1, N.hi1, o, d, best)) closest(b, V, T, N.link1, o, d, best, best_tri);
    return;
  }
  const uint32_t v = ~(uint32_t)link;
  const int first = (int)(v >> kLeafBits), cnt = (int)(v & kLeafMax);
  for (int i = first; i < first + cnt; ++i) {
    const int t = b.order[i];
    const double x = tri_t(V, T, t, o, d);
    if (x < best || (x == best && t < best_tri)) {
      best = x;
      best_tri = t;
    }
  }
}

int main(int argc, char** argv) {
  if (argc < 2) return fail("usage");
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return fail("open");
  int32_t nv = 0, nt = 0;
  if (std::fread(&nv, 4, 1, f) != 1 || std::fread(&nt, 4, 1, f) != 1) return fail("read");
  std::vector<float> V(3 * (size_t)nv);
  std::vector<int> T(3 * (size_t)nt);
  if (std::fread(V.data(), 4, V.size(), f) != V.size() ||
      std::fread(T.data(), 4, T.size(), f) != T.size())
    return fail("read");
  std::fclose(f);
  BvhBuild b;
  const std::string err = build_bvh(V.data(), nv, T.data(), nt, b);
  if (!err.empty()) {
    std::printf("ERROR %s\n", err.c_str());
    return 0;
  }
  if ((int)b.order.size() != nt || b.tris.size() != (size_t)kTriWords * nt)
    return fail("triangle count");
  // vertex data of each reordered triangle
  for (int i = 0; i < nt; ++i) {
    const int t = b.order[i];
    const float* w = &b.tris[(size_t)kTriWords * i];
    int idx[3];
    std::memcpy(&idx[0], &w[3], 4);
    std::memcpy(&idx[1], &w[7], 4);
    std::memcpy(&idx[2], &w[11], 4);
    for (int k = 0; k < 3; ++k)
      if (idx[k] != T[3 * (size_t)t + k]) return fail("vertex indices");
    for (int a = 0; a < 3; ++a)
      if (w[a] != V[3 * (size_t)idx[0] + a]) return fail("v0");
  }
  Ctx c;
  c.b = &b;
  c.seen_node.assign(b.nodes.size(), 0);
  c.seen_tri.assign(nt, 0);
  // the root (node 0) has no box of its own; its children carry theirs
  if (!walk(c, 0, nullptr, nullptr, 1)) return fail("box containment or duplicate");
  for (int x : c.seen_node)
    if (x != 1) return fail("unreachable node");
  for (int x : c.seen_tri)
    if (x != 1) return fail("triangle not in exactly one leaf");
  if (c.max_level != b.depth) return fail("depth");
  if (b.depth > kBvh2MaxDepth) return fail("depth limit");
  // four-wide hierarchy
  {
    std::vector<int> sn(b.nodes4.size(), 0), stt(nt, 0);
    int ml = 0;
    if (!walk4(b, sn, stt, 0, nullptr, nullptr, 1, ml)) return fail("4-wide containment");
    for (int x : sn)
      if (x != 1) return fail("4-wide unreachable node");
    for (int x : stt)
      if (x != 1) return fail("4-wide triangle not in exactly one leaf");
    if (ml != b.depth4) return fail("4-wide depth");
    if (b.stack4 > kBvhMaxStack) return fail("4-wide stack limit");
  }
  // random rays from a box around the mesh towards random mesh points
  float lo[3] = {1e30f, 1e30f, 1e30f}, hi[3] = {-1e30f, -1e30f, -1e30f};
  for (int i = 0; i < nv; ++i)
    for (int a = 0; a < 3; ++a) {
      lo[a] = std::min(lo[a], V[3 * (size_t)i + a]);
      hi[a] = std::max(hi[a], V[3 * (size_t)i + a]);
    }
  std::mt19937_64 g(7);
  std::uniform_real_distribution<double> U(0.0, 1.0);
  int hits = 0;
  const int n_rays = 2000;
  for (int r = 0; r < n_rays; ++r) {
    double o[3], d[3], tgt[3];
    for (int a = 0; a < 3; ++a) {
      const double c0 = 0.5 * (lo[a] + hi[a]), h = 0.5 * (hi[a] - lo[a]) + 1.0;
      o[a] = c0 + (2 * U(g) - 1) * 2 * h;
      tgt[a] = lo[a] + U(g) * (hi[a] - lo[a]);
    }
    double n = 0;
    for (int a = 0; a < 3; ++a) {
      d[a] = tgt[a] - o[a];
      n += d[a] * d[a];
    }
    n = std::sqrt(n);
    for (int a = 0; a < 3; ++a) d[a] /= n;
    double bf = INFINITY;
    int bft = -1;
    for (int t = 0; t < nt; ++t) {
      const double x = tri_t(V.data(), T.data(), t, o, d);
      if (x < bf) {
        bf = x;
        bft = t;
      }
    }
    double bt = INFINITY;
    int btt = -1;
    closest(b, V.data(), T.data(), 0, o, d, bt, btt);
    if (bft != btt || !(bf == bt || (std::isinf(bf) && std::isinf(bt)))) {
      std::printf("FAIL ray %d: brute %d %.17g bvh %d %.17g\n", r, bft, bf, btt, bt);
      return 1;
    }
    double b4 = INFINITY;
    int b4t = -1;
    const int sp = closest4(b, V.data(), T.data(), o, d, b4, b4t);
    if (bft != b4t || !(bf == b4 || (std::isinf(bf) && std::isinf(b4)))) {
      std::printf("FAIL ray %d: brute %d %.17g 4-wide %d %.17g\n", r, bft, bf, b4t, b4);
      return 1;
    }
    if (sp > b.stack4) return fail("4-wide stack bound exceeded");
    hits += bft >= 0;
  }
  std::printf("ok %d %zu %d\n", b.depth, b.nodes.size(), hits);
  return 0;
}
