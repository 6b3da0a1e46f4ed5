// FP64 CPU oracle -- test infrastructure only (see oracle.h).
//
// Plain C++17.  Every quantity is double precision.  Intersections are brute
// force over all primitives, and the derivative of each path is taken from an
// explicit tape swept backward; the GPU library does neither of these, so the
// two implementations share no algorithm beyond the estimator they both define.
#include "oracle.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

namespace {

constexpr double PI = 3.14159265358979323846;
constexpr double INF = std::numeric_limits<double>::infinity();
constexpr double RAY_EPS = 1e-4;      // origin offset along the normal
constexpr double REL_EPS = 0.01;  // relative loss: (I - T)^2 / (T^2 + REL_EPS)
constexpr double SHADOW_EPS = 1e-4;   // shadow rays stop this short of the light
constexpr double ROUGH_MIN = 0.05;    // roughness floor of the material model
constexpr double P_SPEC = 0.5;        // probability of sampling the specular lobe

enum { T_PRIMAL = 0 };

// --------------------------------------------------------------------------
// vectors
// --------------------------------------------------------------------------
struct V3 {
  double x, y, z;
};
inline V3 operator+(V3 a, V3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
inline V3 operator-(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
inline V3 operator*(V3 a, double s) { return {a.x * s, a.y * s, a.z * s}; }
inline V3 operator*(double s, V3 a) { return {a.x * s, a.y * s, a.z * s}; }
inline double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
inline V3 cross(V3 a, V3 b) {
  return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
inline double length(V3 a) { return std::sqrt(dot(a, a)); }
inline V3 normalize(V3 a) { return a * (1.0 / length(a)); }
inline V3 from(const double* p) { return {p[0], p[1], p[2]}; }

// --------------------------------------------------------------------------
// random numbers
// --------------------------------------------------------------------------
// SplitMix64 (Steele, Lea, Flood 2014): one step of the generator started at x.
uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

// Philox4x32 with 10 rounds (Salmon, Moraes, Dror, Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11).  Each round multiplies counter words 0
// and 2 by the two round multipliers (64-bit products), and the new counter is
// (hi(c2*M1) ^ c1 ^ k0, lo(c2*M1), hi(c0*M0) ^ c3 ^ k1, lo(c0*M0)); the key is
// advanced by the two Weyl increments before every round after the first.
void philox(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
  const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
  uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
  uint32_t k0 = key[0], k1 = key[1];
  for (int round = 0; round < 10; ++round) {
    if (round > 0) {
      k0 += W0;
      k1 += W1;
    }
    uint64_t p0 = (uint64_t)M0 * (uint64_t)c0;
    uint64_t p1 = (uint64_t)M1 * (uint64_t)c2;
    uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
    uint32_t n1 = (uint32_t)p1;
    uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
    uint32_t n3 = (uint32_t)p0;
    c0 = n0; c1 = n1; c2 = n2; c3 = n3;
  }
  out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

uint64_t stream_key(uint64_t seed, uint32_t iteration, uint32_t tag) {
  return splitmix64(seed ^ splitmix64(((uint64_t)iteration << 8) | (uint64_t)tag));
}

// The random numbers of one path: counter = (pixel, sample, bounce, block).
struct PathRng {
  uint32_t key[2];
  uint32_t pixel, sample;
  void draw(uint32_t bounce, uint32_t block, double u[4]) const {
    uint32_t ctr[4] = {pixel, sample, bounce, block}, r[4];
    philox(ctr, key, r);
    for (int i = 0; i < 4; ++i) u[i] = (double)(r[i] >> 8) * (1.0 / 16777216.0);
  }
};

// --------------------------------------------------------------------------
// scene
// --------------------------------------------------------------------------
struct Ray {
  V3 o, d;
};

enum Kind { K_NONE = 0, K_PLANE, K_SPHERE, K_LIGHT, K_MESH };

struct Hit {
  Kind kind = K_NONE;
  int obj = -1;             // sphere or triangle index
  double t = INF;
  double bu = 0, bv = 0;    // triangle: barycentrics of vertices 1 and 2
  V3 p{0, 0, 0}, n{0, 0, 0};
};

struct Margin {
  double m = INF;
  void add(double v) { m = std::min(m, std::fabs(v)); }
};

struct Scene {
  const orc_scene* s;
  V3 eye, cw, cu, cv;
  double tan_half, aspect;
  int n_ch;
  int ch_slot[5];  // slot of channel bit b in a texel, -1 if not a parameter
  int view_h;      // rows per view (volume scenes stack several views)

  explicit Scene(const orc_scene* sc) : s(sc) {
    eye = from(sc->cam_eye);
    cw = normalize(from(sc->cam_target) - eye);
    cu = normalize(cross(cw, from(sc->cam_up)));
    cv = cross(cu, cw);
    tan_half = std::tan(sc->vfov_deg * PI / 360.0);
    view_h = volume() ? sc->height / sc->vol_views : sc->height;
    aspect = (double)sc->width / (double)view_h;
    n_ch = 0;
    for (int b = 0; b < 5; ++b) ch_slot[b] = (sc->ch_mask >> b & 1) ? n_ch++ : -1;
  }

  bool volume() const { return s->param_layout == 2; }

  Ray camera_ray(int x, int y, double jx, double jy) const {
    if (volume()) {
      // view v: the eye turned by 2 pi v / V about the vertical line through
      // the target
      const int v = y / view_h;
      const double ang = 2.0 * PI * v / s->vol_views;
      const V3 tg = from(s->cam_target), r = eye - tg;
      const V3 e{tg.x + r.x * std::cos(ang) + r.z * std::sin(ang), eye.y,
                 tg.z - r.x * std::sin(ang) + r.z * std::cos(ang)};
      const V3 w = normalize(tg - e);
      const V3 u = normalize(cross(w, from(s->cam_up)));
      const V3 vv = cross(u, w);
      double sx = (2.0 * (x + jx) / s->width - 1.0) * tan_half * aspect;
      double sy = (1.0 - 2.0 * (y - v * view_h + jy) / view_h) * tan_half;
      return {e, normalize(w + u * sx + vv * sy)};
    }
    double sx = (2.0 * (x + jx) / s->width - 1.0) * tan_half * aspect;
    double sy = (1.0 - 2.0 * (y + jy) / s->height) * tan_half;
    return {eye, normalize(cw + cu * sx + cv * sy)};
  }

  // Candidate distances.  Each returns the hit distance (or INF) and, through
  // `near`, the distance at which a flipped hit/miss decision would place the
  // primitive together with that decision's relative margin.
  struct Cand {
    double t = INF;        // hit distance, INF = miss
    double t_near = INF;   // where the primitive would be hit if the decision flipped
    double margin = INF;   // relative distance of the decision from its threshold
  };

  Cand sphere(int k, const Ray& r) const {
    Cand c;
    const double* sp = s->spheres + 4 * k;
    V3 oc = r.o - V3{sp[0], sp[1], sp[2]};
    double rad = sp[3];
    double b = dot(oc, r.d);
    double cc = dot(oc, oc) - rad * rad;
    double disc = b * b - cc;
    c.margin = std::fabs(disc) / (rad * rad);
    if (disc < 0) {
      c.t_near = -b > 0 ? -b : INF;  // closest approach
      return c;
    }
    double sq = std::sqrt(disc);
    double t0 = -b - sq, t1 = -b + sq;
    c.t = t0 > 0 ? t0 : (t1 > 0 ? t1 : INF);
    c.t_near = c.t;
    return c;
  }

  Cand plane(const Ray& r) const {
    Cand c;
    if (!s->plane_enabled) return c;
    if (!(r.o.y > 0)) {
      // origins just below y = 0 (offset from a sphere's underside) skip the plane
      if (r.d.y < 0) {
        c.margin = std::fabs(r.o.y) / RAY_EPS;
        c.t_near = -r.o.y / r.d.y;
      }
      return c;
    }
    c.margin = std::fabs(r.d.y);
    if (r.d.y < 0) c.t = -r.o.y / r.d.y;
    c.t_near = c.t;  // a flip to d.y > 0 moves the hit to infinity
    return c;
  }

  V3 vert(int i) const { return from(s->verts + 3 * (size_t)i); }

  // Moller-Trumbore.  Margin of the inside/outside decision in barycentric
  // units: for a hit, the distance to the nearest edge, min(u, v, 1 - u - v);
  // for a miss, how far outside the point lies, max(-u, -v, u + v - 1) (every
  // violated edge would have to flip).  A triangle behind the origin that the
  // ray's line crosses inside counts how far behind it lies, in units of the
  // ray offset.
  Cand triangle(int k, const Ray& r, double* bu, double* bv) const {
    Cand c;
    const int* tr = s->tris + 3 * (size_t)k;
    const V3 v0 = vert(tr[0]), e1 = vert(tr[1]) - v0, e2 = vert(tr[2]) - v0;
    const V3 pv = cross(r.d, e2);
    const double det = dot(e1, pv);
    if (det == 0.0) return c;
    const double inv = 1.0 / det;
    const V3 sv = r.o - v0;
    const double u = dot(sv, pv) * inv;
    const V3 qv = cross(sv, e1);
    const double v = dot(r.d, qv) * inv;
    const double t = dot(e2, qv) * inv;
    const bool inside = u >= 0 && v >= 0 && u + v <= 1;
    if (!(t > 0.0)) {
      if (inside) {
        c.margin = std::fabs(t) / RAY_EPS;
        c.t_near = 0.0;
      }
      return c;
    }
    c.margin = inside ? std::min(std::min(u, v), 1.0 - u - v)
                      : std::max(std::max(-u, -v), u + v - 1.0);
    c.t_near = t;
    if (!inside) return c;
    c.t = t;
    *bu = u;
    *bv = v;
    return c;
  }

  Cand light(const Ray& r) const {
    Cand c;
    if (!s->light_enabled) return c;
    double ly = s->light_center[1];
    if (!(r.d.y > 0) || !(r.o.y < ly)) return c;
    double t = (ly - r.o.y) / r.d.y;
    double h = 0.5 * s->light_side;
    double dx = r.o.x + t * r.d.x - s->light_center[0];
    double dz = r.o.z + t * r.d.z - s->light_center[2];
    c.margin = std::min(std::fabs(h - std::fabs(dx)), std::fabs(h - std::fabs(dz))) / s->light_side;
    c.t_near = t;
    if (std::fabs(dx) <= h && std::fabs(dz) <= h) c.t = t;
    return c;
  }

  // Closest hit; primitive order plane < spheres < light, and a strictly
  // smaller t is needed to replace the current best (equal t: lower id wins).
  // Margins: the winner's own decision, every near miss that would land in
  // front of the winner, and the gap to the runner-up.
  Hit intersect(const Ray& r, Margin& mg) const {
    const Margin mg_in = mg;
    Hit h;
    const int n = s->n_spheres;
    std::vector<Cand> cs;
    cs.reserve(n + 2);
    cs.push_back(plane(r));
    for (int k = 0; k < n; ++k) cs.push_back(sphere(k, r));
    cs.push_back(light(r));
    int best = -1;
    for (int i = 0; i < (int)cs.size(); ++i)
      if (cs[i].t < h.t) {
        h.t = cs[i].t;
        best = i;
      }
    double second = INF;
    for (int i = 0; i < (int)cs.size(); ++i) {
      if (i == best) {
        mg.add(cs[i].margin);
        continue;
      }
      if (cs[i].t < second) second = cs[i].t;
      if (cs[i].t == INF && cs[i].t_near < h.t) mg.add(cs[i].margin);
    }
    // mesh triangles rank after the spheres and before the light
    int best_tri = -1;
    double tri_t = INF, tbu = 0, tbv = 0;
    if (s->n_tris > 0) {
      const double t_analytic = best >= 0 && best < (int)cs.size() - 1 ? h.t : INF;
      for (int k = 0; k < s->n_tris; ++k) {
        double bu, bv;
        const Cand c = triangle(k, r, &bu, &bv);
        if (c.t < tri_t) {
          tri_t = c.t;
          best_tri = k;
          tbu = bu;
          tbv = bv;
        }
      }
      const double t_light = best == (int)cs.size() - 1 ? h.t : INF;
      if (best_tri >= 0 && tri_t < t_analytic && !(t_light < tri_t)) {
        // the mesh wins: redo the margins of the analytic candidates
        mg = Margin{mg_in.m};
        h.t = tri_t;
        second = INF;
        for (int i = 0; i < (int)cs.size(); ++i) {
          if (cs[i].t < second) second = cs[i].t;
          if (cs[i].t == INF && cs[i].t_near < h.t) mg.add(cs[i].margin);
        }
        best = -2;
      }
      for (int k = 0; k < s->n_tris; ++k) {
        double bu, bv;
        const Cand c = triangle(k, r, &bu, &bv);
        if (best == -2 && k == best_tri) {
          mg.add(c.margin);
          continue;
        }
        if (c.t < second) second = c.t;
        if (c.t == INF && c.t_near < h.t) mg.add(c.margin);
      }
    }
    if (best == -1) return h;
    if (second < INF) mg.add((second - h.t) / h.t);
    if (best == -2) {
      h.kind = K_MESH;
      h.obj = best_tri;
      h.bu = tbu;
      h.bv = tbv;
      h.p = r.o + r.d * h.t;
      const int* tr = s->tris + 3 * (size_t)best_tri;
      const V3 v0 = vert(tr[0]);
      const V3 ng = normalize(cross(vert(tr[1]) - v0, vert(tr[2]) - v0));
      const double dn = dot(ng, r.d);
      mg.add(dn);  // which side faces the ray
      h.n = dn < 0 ? ng : ng * -1.0;
      return h;
    }
    if (best == 0) {
      h.kind = K_PLANE;
      h.obj = 0;
    } else if (best == (int)cs.size() - 1) {
      h.kind = K_LIGHT;
      h.obj = 0;
    } else {
      h.kind = K_SPHERE;
      h.obj = best - 1;
    }
    h.p = r.o + r.d * h.t;
    if (h.kind == K_PLANE) {
      h.n = {0, 1, 0};
      h.p.y = 0.0;
    } else if (h.kind == K_SPHERE) {
      const double* sp = s->spheres + 4 * h.obj;
      h.n = (h.p - V3{sp[0], sp[1], sp[2]}) * (1.0 / sp[3]);
    } else {
      h.n = {0, -1, 0};
    }
    return h;
  }

  // any occluder (plane, spheres) with 0 < t < tmax; margins of every decision
  // that could change the answer
  bool occluded(const Ray& r, double tmax, Margin& mg) const {
    bool occ = false;
    auto one = [&](const Cand& c) {
      if (c.t < INF) {
        mg.add((tmax - c.t) / tmax);
        mg.add(c.margin);
        if (c.t < tmax) occ = true;
      } else if (c.t_near < tmax) {
        mg.add(c.margin);
      }
    };
    one(plane(r));
    for (int k = 0; k < s->n_spheres; ++k) one(sphere(k, r));
    for (int k = 0; k < s->n_tris; ++k) {
      double bu, bv;
      one(triangle(k, r, &bu, &bv));
    }
    return occ;
  }
};

// --------------------------------------------------------------------------
// material and footprint
// --------------------------------------------------------------------------
struct Footprint {
  int n = 0;
  int texel[4];
  double w[4];
};

struct Material {
  double c[3], metal, rough;
  bool param = false;
  Footprint fp;
};

// Bilinear texture footprint, clamp-to-edge, texel centres at (i + 0.5) / size.
// Margin: distance (in texels) of the texel coordinates from an integer --
// the value is continuous there, but which neighbour texel receives a
// vanishing weight is a discrete choice.
Footprint bilinear(const orc_scene* s, double u, double v, Margin& mg) {
  Footprint fp;
  if (s->tex_w == 1 && s->tex_h == 1) {
    fp.n = 1;
    fp.texel[0] = 0;
    fp.w[0] = 1.0;
    return fp;
  }
  double x = u * s->tex_w - 0.5, y = v * s->tex_h - 0.5;
  double x0 = std::floor(x), y0 = std::floor(y);
  if (x > 0 && x < s->tex_w - 1) mg.add(x - std::nearbyint(x));
  if (y > 0 && y < s->tex_h - 1) mg.add(y - std::nearbyint(y));
  double fx = x - x0, fy = y - y0;
  auto cl = [](double a, int n) { return (int)std::min(std::max(a, 0.0), (double)(n - 1)); };
  int xi0 = cl(x0, s->tex_w), xi1 = cl(x0 + 1, s->tex_w);
  int yi0 = cl(y0, s->tex_h), yi1 = cl(y0 + 1, s->tex_h);
  fp.n = 4;
  fp.texel[0] = yi0 * s->tex_w + xi0; fp.w[0] = (1 - fx) * (1 - fy);
  fp.texel[1] = yi0 * s->tex_w + xi1; fp.w[1] = fx * (1 - fy);
  fp.texel[2] = yi1 * s->tex_w + xi0; fp.w[2] = (1 - fx) * fy;
  fp.texel[3] = yi1 * s->tex_w + xi1; fp.w[3] = fx * fy;
  return fp;
}

Material material_at(const Scene& sc, const Hit& h, const double* params, Margin& mg) {
  const orc_scene* s = sc.s;
  int mat = h.kind == K_PLANE ? s->plane_mat : (h.kind == K_MESH ? s->mesh_mat : s->sphere_mat[h.obj]);
  Material m;
  if (mat >= 0) {
    const double* f = s->fixed_mats + 5 * mat;
    m.c[0] = f[0]; m.c[1] = f[1]; m.c[2] = f[2];
    m.metal = f[3];
    m.rough = f[4];
    return m;
  }
  double u, v;
  if (h.kind == K_MESH && s->param_layout == 1) {
    // per-vertex parameters, interpolated barycentrically
    const int* tr = s->tris + 3 * (size_t)h.obj;
    m.param = true;
    m.fp.n = 3;
    m.fp.texel[0] = tr[0];
    m.fp.w[0] = 1.0 - h.bu - h.bv;
    m.fp.texel[1] = tr[1];
    m.fp.w[1] = h.bu;
    m.fp.texel[2] = tr[2];
    m.fp.w[2] = h.bv;
  } else if (h.kind == K_PLANE || h.kind == K_MESH) {
    u = (h.p.x - s->plane_extent[0]) / (s->plane_extent[1] - s->plane_extent[0]);
    v = (h.p.z - s->plane_extent[2]) / (s->plane_extent[3] - s->plane_extent[2]);
  } else {
    // latitude-longitude map; the seam sits at atan2 = +-pi (n.x < 0, n.z = 0)
    V3 n = h.n;
    if (n.x < 0 && s->tex_w > 1) mg.add(n.z);
    u = 0.5 + std::atan2(n.z, n.x) / (2 * PI);
    v = std::atan2(std::sqrt(n.x * n.x + n.z * n.z), n.y) / PI;
  }
  if (!m.param) {
    m.param = true;
    m.fp = bilinear(s, u, v, mg);
  }
  double val[5];
  for (int b = 0; b < 5; ++b) {
    if (sc.ch_slot[b] < 0) {
      val[b] = s->fixed_default[b];
      continue;
    }
    double acc = 0;
    for (int k = 0; k < m.fp.n; ++k) acc += m.fp.w[k] * params[m.fp.texel[k] * sc.n_ch + sc.ch_slot[b]];
    val[b] = acc;
  }
  m.c[0] = val[0]; m.c[1] = val[1]; m.c[2] = val[2];
  m.metal = val[3];
  m.rough = val[4];
  return m;
}

// --------------------------------------------------------------------------
// BSDF: metallic-roughness.  f = (1-m) c / pi + D G F / (4 cos_o cos_i) with
// GGX D (alpha = rough^2), separable Smith G1, Schlick F with
// F0 = 0.04 (1-m) + m c.  Partials w.r.t. c (per channel), m and rough.
// --------------------------------------------------------------------------
struct Bsdf {
  double f[3] = {0, 0, 0};
  double dc[3] = {0, 0, 0};  // df^k / dc^k
  double dm[3] = {0, 0, 0};  // df^k / dm
  double dr[3] = {0, 0, 0};  // df^k / drough
  double pdf = 0;            // solid-angle density of the sampler for wi
};

double sin2(V3 n, V3 v) {
  V3 c = cross(n, v);
  return dot(c, c);
}

Bsdf eval_bsdf(const Material& m, V3 n, V3 wo, V3 wi, int flags) {
  Bsdf b;
  double co = dot(n, wo), ci = dot(n, wi);
  if (!(co > 0) || !(ci > 0)) return b;
  if (flags & ORC_LAMBERT_ONLY) {
    for (int k = 0; k < 3; ++k) {
      b.f[k] = m.c[k] / PI;
      b.dc[k] = 1.0 / PI;
    }
    b.pdf = ci / PI;
    return b;
  }
  double r = std::max(m.rough, ROUGH_MIN);
  double drough = m.rough >= ROUGH_MIN ? 1.0 : 0.0;
  double a = r * r;
  double a2 = a * a;
  V3 h = normalize(wo + wi);
  double ch = dot(n, h), sh2 = sin2(n, h);
  double Q = ch * ch * a2 + sh2;
  double D = a2 / (PI * Q * Q);
  auto g1 = [&](double c, double s2, double& dlog) {
    double q = std::sqrt(a2 * s2 + c * c);
    dlog = -(a * s2 / q) / (c + q);
    return 2 * c / (c + q);
  };
  double dlgo, dlgi;
  double Go = g1(co, sin2(n, wo), dlgo);
  double Gi = g1(ci, sin2(n, wi), dlgi);
  double S = D * Go * Gi / (4 * co * ci);
  double dlogS_da = 2.0 / a - 4.0 * ch * ch * a / Q + dlgo + dlgi;
  double dS_dr = S * dlogS_da * 2.0 * r * drough;
  double dh = std::min(1.0, dot(wi, h));
  double w5 = std::pow(1.0 - dh, 5);
  for (int k = 0; k < 3; ++k) {
    double F0 = 0.04 * (1 - m.metal) + m.metal * m.c[k];
    double F = F0 + (1 - F0) * w5;
    b.f[k] = (1 - m.metal) * m.c[k] / PI + S * F;
    b.dc[k] = (1 - m.metal) / PI + S * (1 - w5) * m.metal;
    b.dm[k] = -m.c[k] / PI + S * (1 - w5) * (m.c[k] - 0.04);
    b.dr[k] = dS_dr * F;
  }
  if (flags & ORC_PARAM_INDEP) {
    b.pdf = ci / PI;
  } else {
    double pdf_s = D * ch / (4 * dh);
    b.pdf = P_SPEC * pdf_s + (1 - P_SPEC) * ci / PI;
  }
  return b;
}

// Orthonormal basis around n (Duff et al., "Building an Orthonormal Basis,
// Revisited", JCGT 2017).
void basis(V3 n, V3& b1, V3& b2) {
  double sign = std::copysign(1.0, n.z);
  double a = -1.0 / (sign + n.z);
  double b = n.x * n.y * a;
  b1 = {1.0 + sign * n.x * n.x * a, sign * b, -sign * n.x};
  b2 = {b, sign + n.y * n.y * a, -n.y};
}

// Direction sampling: u[0] picks the lobe (specular if u[0] < P_SPEC), u[1],
// u[2] place the direction.  GGX half-vectors follow Walter et al. 2007.
// The basis flips with the sign of n.z; that is a decision unless the normal
// is exactly axis-aligned by construction (exact_normal: the plane's).
V3 sample_dir(const Material& m, V3 n, V3 wo, const double u[4], int flags, Margin& mg,
              bool exact_normal) {
  V3 b1, b2;
  if (!(exact_normal && n.z == 0.0)) mg.add(n.z);
  basis(n, b1, b2);
  double phi = 2 * PI * u[2];
  bool spec = !(flags & (ORC_LAMBERT_ONLY | ORC_PARAM_INDEP)) && u[0] < P_SPEC;
  if (!spec) {
    double rr = std::sqrt(u[1]);
    double z = std::sqrt(std::max(0.0, 1.0 - u[1]));
    return b1 * (rr * std::cos(phi)) + b2 * (rr * std::sin(phi)) + n * z;
  }
  double r = std::max(m.rough, ROUGH_MIN);
  double a = r * r;
  double t2 = a * a * u[1] / (1.0 - u[1]);
  double ct = 1.0 / std::sqrt(1.0 + t2);
  double st = std::sqrt(t2) * ct;
  V3 h = b1 * (st * std::cos(phi)) + b2 * (st * std::sin(phi)) + n * ct;
  return h * (2 * dot(wo, h)) - wo;
}

// --------------------------------------------------------------------------
// path tracing with an optional tape
// --------------------------------------------------------------------------
struct TapeVertex {
  double beta[3];           // throughput arriving at the vertex (beta_{j-1})
  bool param;
  Footprint fp;
  bool nee = false;
  double K[3];              // NEE factor: cos Le w_mis / p_light (per unit f)
  Bsdf nb;                  // BSDF (and partials) towards the light sample
  bool cont = false;
  double cw;                // cos_i / (pdf q)
  Bsdf cb;                  // BSDF (and partials) along the continuation
  double E[3] = {0, 0, 0};  // emission picked up by the continuation, per unit beta_j
};

// One sample of an emission-absorption ray march (volume scenes).
struct VolSample {
  double T;        // transmittance before the sample
  double alpha;    // 1 - exp(-sigma dt)
  double e[3];     // emission
  double sigma;    // density per unit length (vol_sigma x the density parameter)
  double dt;       // segment length
  size_t vox[8];   // trilinear corners (voxel indices) and weights
  double w[8];
};

struct PathResult {
  double L[3] = {0, 0, 0};
  double margin = INF;
  std::vector<TapeVertex> tape;
  std::vector<VolSample> vtape;  // volume scenes
};

// Test hook: a fixed offset (in pixels) added to every primary sample
// position.  Tracing the same random numbers with the primary ray turned by
// about the size of single-precision rounding measures how strongly a path
// amplifies such rounding (its conditioning).  Zero in normal use.
double g_jitter_dx = 0.0, g_jitter_dy = 0.0;

// Workload statistics: paths traced, surface vertices, vertices on the
// parameterised material.
std::atomic<uint64_t> g_paths{0}, g_vertices{0}, g_param_vertices{0};

// Emission-absorption volume (the volume experiment of the Experiments
// section): the camera ray's chord through the cube is split into
// N = ceil(chord / voxel) equal segments of length dt, sampled at
// t0 + (k + u) dt with one jitter u per ray (0.5 under ORC_PIXEL_CENTER);
// each sample reads the trilinearly interpolated voxel values (centres at
// (i + 0.5) / R of the cube, clamp-to-edge) and the radiance is the
// quadrature sum_k T_k alpha_k e_k + T_N env, alpha_k = 1 - exp(-sigma_k dt),
// T_{k+1} = T_k (1 - alpha_k).  Margins: the hit/miss of the cube and the
// rounding of chord / voxel to N.  A sample's cell is no decision for the
// radiance (trilinear values are continuous across cells); only which corner
// takes a vanishing weight changes there, which a gradient comparison must
// allow for between neighbouring voxels.
void trace_volume(const Scene& sc, const double* params, const PathRng& rng, int px, int py,
                  int flags, bool record, PathResult& out) {
  const orc_scene* s = sc.s;
  Margin mg;
  double u[4];
  g_paths.fetch_add(1, std::memory_order_relaxed);
  rng.draw(0, 0, u);
  const bool center = (flags & ORC_PIXEL_CENTER) != 0;
  const double jx = center ? 0.5 : u[0], jy = center ? 0.5 : u[1], us = center ? 0.5 : u[2];
  const Ray ray = sc.camera_ray(px, py, jx + g_jitter_dx, jy + g_jitter_dy);
  const double R = s->vol_res, side = s->vol_box[3];
  // slab test against the cube
  double t0 = 0.0, t1 = INF;
  const double o[3] = {ray.o.x, ray.o.y, ray.o.z}, d[3] = {ray.d.x, ray.d.y, ray.d.z};
  for (int a = 0; a < 3; ++a) {
    const double lo = s->vol_box[a], hi = s->vol_box[a] + side;
    if (d[a] == 0.0) {
      if (o[a] < lo || o[a] > hi) t1 = -INF;
      continue;
    }
    double ta = (lo - o[a]) / d[a], tb = (hi - o[a]) / d[a];
    if (ta > tb) std::swap(ta, tb);
    t0 = std::max(t0, ta);
    t1 = std::min(t1, tb);
  }
  double* L = out.L;
  const double vox = side / R;
  mg.add((t1 - t0) / vox);  // grazing the cube: hit or miss
  if (!(t1 > t0)) {
    for (int k = 0; k < 3; ++k) L[k] = s->env[k];
    out.margin = mg.m;
    return;
  }
  const double q = (t1 - t0) / vox;
  const int N = std::max(1, (int)std::ceil(q));
  mg.add((q - std::floor(q)) / std::max(q, 1.0));
  mg.add((std::ceil(q) - q) / std::max(q, 1.0));
  const double dt = (t1 - t0) / N;
  double T = 1.0;
  for (int k = 0; k < N; ++k) {
    const double t = t0 + (k + us) * dt;
    const double x[3] = {o[0] + t * d[0], o[1] + t * d[1], o[2] + t * d[2]};
    int i0[3], i1[3];
    double f[3];
    for (int a = 0; a < 3; ++a) {
      const double g = (x[a] - s->vol_box[a]) / vox - 0.5;
      const double fl = std::floor(g);
      f[a] = g - fl;
      i0[a] = (int)std::min(std::max(fl, 0.0), R - 1);
      i1[a] = (int)std::min(std::max(fl + 1.0, 0.0), R - 1);
    }
    VolSample vs;
    double val[4] = {0, 0, 0, 0};
    for (int c = 0; c < 8; ++c) {
      const int ix = (c & 1) ? i1[0] : i0[0], iy = (c & 2) ? i1[1] : i0[1],
                iz = (c & 4) ? i1[2] : i0[2];
      const double w = ((c & 1) ? f[0] : 1 - f[0]) * ((c & 2) ? f[1] : 1 - f[1]) *
                       ((c & 4) ? f[2] : 1 - f[2]);
      vs.vox[c] = ((size_t)iz * s->vol_res + iy) * s->vol_res + ix;
      vs.w[c] = w;
      for (int ch = 0; ch < 4; ++ch) val[ch] += w * params[4 * vs.vox[c] + ch];
    }
    vs.T = T;
    vs.sigma = s->vol_sigma * val[3];
    vs.dt = dt;
    vs.alpha = 1.0 - std::exp(-vs.sigma * dt);
    for (int ch = 0; ch < 3; ++ch) {
      vs.e[ch] = val[ch];
      L[ch] += T * vs.alpha * val[ch];
    }
    T *= std::exp(-vs.sigma * dt);
    if (record) out.vtape.push_back(vs);
  }
  g_vertices.fetch_add((uint64_t)N, std::memory_order_relaxed);
  g_param_vertices.fetch_add((uint64_t)N, std::memory_order_relaxed);
  for (int k = 0; k < 3; ++k) L[k] += T * s->env[k];
  out.margin = mg.m;
}

// Reverse sweep over a volume tape.  D = radiance behind the sample per unit
// transmittance in front of it: D_N = env, D_k = alpha_k e_k + (1 - alpha_k) D_{k+1},
// C = D_0.  Hence dC/de_k = T_k alpha_k and
// dC/dsigma_k = T_k dt exp(-sigma_k dt) (e_k - D_{k+1}); the density parameter
// adds the factor vol_sigma, and trilinear weights spread both over 8 voxels.
void backprop_volume(const Scene& sc, const std::vector<VolSample>& tape, const double adj[3],
                     double* grad, double* gabs) {
  double D[3] = {sc.s->env[0], sc.s->env[1], sc.s->env[2]};
  for (int k = (int)tape.size() - 1; k >= 0; --k) {
    const VolSample& v = tape[k];
    double g[4] = {0, 0, 0, 0}, ga[4] = {0, 0, 0, 0};
    const double et = std::exp(-v.sigma * v.dt);
    for (int ch = 0; ch < 3; ++ch) {
      const double ge = adj[ch] * v.T * v.alpha;
      const double gs = adj[ch] * v.T * v.dt * et * (v.e[ch] - D[ch]) * sc.s->vol_sigma;
      g[ch] += ge;
      ga[ch] += std::fabs(ge);
      g[3] += gs;
      ga[3] += std::fabs(gs);
    }
    for (int c = 0; c < 8; ++c)
      for (int ch = 0; ch < 4; ++ch) {
        grad[4 * v.vox[c] + ch] += v.w[c] * g[ch];
        gabs[4 * v.vox[c] + ch] += v.w[c] * ga[ch];
      }
    for (int ch = 0; ch < 3; ++ch) D[ch] = v.alpha * v.e[ch] + (1.0 - v.alpha) * D[ch];
  }
}

// sample_params (nullable, else = params): the parameters whose BSDF
// densities choose the directions.  The path is then drawn at sample_params
// and weighted by f(x; params) / p(x; sample_params) -- every density (the
// continuation's, and those in both MIS weights) is taken at sample_params --
// which is the finite-difference sample of Eq. 5 when params = pi_{i-1} and
// sample_params = pi_i: one path, the integrand evaluated at both parameter
// vectors over the density of the current ones.
void trace(const Scene& sc, const double* params, const double* sample_params,
           const PathRng& rng, int px, int py, int flags, bool record, PathResult& out) {
  if (sc.volume()) {
    // the march does not sample anything from the parameters: the path is
    // the same at every parameter vector
    trace_volume(sc, params, rng, px, py, flags, record, out);
    return;
  }
  const orc_scene* s = sc.s;
  Margin mg;
  double u[4];
  g_paths.fetch_add(1, std::memory_order_relaxed);
  double jx = 0.5, jy = 0.5;
  if (!(flags & ORC_PIXEL_CENTER)) {
    rng.draw(0, 0, u);
    jx = u[0];
    jy = u[1];
  }
  Ray ray = sc.camera_ray(px, py, jx + g_jitter_dx, jy + g_jitter_dy);
  Hit hit = sc.intersect(ray, mg);
  double* L = out.L;
  if (hit.kind == K_NONE) {
    for (int k = 0; k < 3; ++k) L[k] += s->env[k];
    out.margin = mg.m;
    return;
  }
  if (hit.kind == K_LIGHT) {
    for (int k = 0; k < 3; ++k) L[k] += s->light_Le[k];
    out.margin = mg.m;
    return;
  }
  double beta[3] = {1, 1, 1};
  const double area = s->light_side * s->light_side;
  for (int j = 1; j <= s->depth; ++j) {
    V3 p = hit.p, n = hit.n, wo = ray.d * -1.0;
    Material mat = material_at(sc, hit, params, mg);
    Material smat = sample_params ? material_at(sc, hit, sample_params, mg) : mat;
    g_vertices.fetch_add(1, std::memory_order_relaxed);
    if (mat.param) g_param_vertices.fetch_add(1, std::memory_order_relaxed);
    TapeVertex tv;
    for (int k = 0; k < 3; ++k) tv.beta[k] = beta[k];
    tv.param = mat.param;
    tv.fp = mat.fp;
    V3 p_off = p + n * RAY_EPS;

    // next-event estimation towards the square light
    if (s->light_enabled && !(flags & ORC_NO_NEE)) {
      rng.draw(j, 1, u);
      double h = 0.5 * s->light_side;
      V3 lp{s->light_center[0] + (2 * u[0] - 1) * h, s->light_center[1],
            s->light_center[2] + (2 * u[1] - 1) * h};
      V3 dl = lp - p;
      double dist2 = dot(dl, dl), dist = std::sqrt(dist2);
      V3 wl = dl * (1.0 / dist);
      double cos_l = wl.y, cos_s = dot(n, wl);
      // the light term vanishes continuously at zero cosines, but which
      // parameters receive (tiny) derivatives still depends on the sign
      mg.add(cos_l);
      mg.add(cos_s);
      if (cos_l > 0 && cos_s > 0 && !sc.occluded({p_off, wl}, dist - SHADOW_EPS, mg)) {
        Bsdf nb = eval_bsdf(mat, n, wo, wl, flags);
        if (sample_params) nb.pdf = eval_bsdf(smat, n, wo, wl, flags).pdf;
        double pl = dist2 / (cos_l * area);
        double wmis = pl / (pl + nb.pdf);
        tv.nee = true;
        tv.nb = nb;
        for (int k = 0; k < 3; ++k) {
          tv.K[k] = cos_s * s->light_Le[k] * wmis / pl;
          L[k] += beta[k] * nb.f[k] * tv.K[k];
        }
      }
    }

    // continuation
    rng.draw(j, 0, u);
    V3 wi = sample_dir(smat, n, wo, u, flags, mg, hit.kind == K_PLANE);
    double ci = dot(n, wi);
    mg.add(ci);  // continuous in value, not in which vertices follow
    bool go = ci > 0;
    Bsdf cb;
    double q = 1.0;
    if (go) {
      cb = eval_bsdf(mat, n, wo, wi, flags);
      if (sample_params) cb.pdf = eval_bsdf(smat, n, wo, wi, flags).pdf;
      go = cb.pdf > 0;
    }
    if (go && s->rr_start > 0 && j >= s->rr_start) {
      if (u[3] >= s->rr_q) go = false;
      q = s->rr_q;
    }
    if (!go) {
      if (record) out.tape.push_back(tv);
      break;
    }
    tv.cont = true;
    tv.cb = cb;
    tv.cw = ci / (cb.pdf * q);
    for (int k = 0; k < 3; ++k) beta[k] *= cb.f[k] * tv.cw;
    ray = {p_off, wi};
    hit = sc.intersect(ray, mg);
    bool end = true;
    if (hit.kind == K_NONE) {
      for (int k = 0; k < 3; ++k) tv.E[k] = s->env[k];
    } else if (hit.kind == K_LIGHT) {
      double pl = hit.t * hit.t / (wi.y * area);
      double wb = (flags & ORC_NO_NEE) ? 1.0 : cb.pdf / (cb.pdf + pl);
      for (int k = 0; k < 3; ++k) tv.E[k] = s->light_Le[k] * wb;
    } else {
      end = j == s->depth;
    }
    for (int k = 0; k < 3; ++k) L[k] += beta[k] * tv.E[k];
    if (record) out.tape.push_back(tv);
    if (end) break;
  }
  out.margin = mg.m;
}

// Reverse sweep over the tape: adjoint dL/dparams += sum_k adj^k dC^k/dparams,
// where adj is the RGB weight of this path's radiance in the loss.
//   T_j = N'_j + w_j (E'_j + T_{j+1})   downstream radiance per unit beta_{j-1}
//   S_j = E'_j + T_{j+1}                downstream per unit beta_j
// NEE term:          adj beta_{j-1} K df(w_l)/dtheta
// continuation term: adj beta_{j-1} (cos/(pdf q)) S_j df(w_i)/dtheta
void backprop(const Scene& sc, const std::vector<TapeVertex>& tape, const double adj[3],
              double* grad, double* gabs) {
  if (sc.volume()) return;  // volume tapes: backprop_volume
  const int nv = (int)tape.size();
  double T_next[3] = {0, 0, 0};
  for (int j = nv - 1; j >= 0; --j) {
    const TapeVertex& v = tape[j];
    double S[3] = {0, 0, 0}, T[3] = {0, 0, 0};
    for (int k = 0; k < 3; ++k) {
      S[k] = v.E[k] + T_next[k];
      double nee = v.nee ? v.nb.f[k] * v.K[k] : 0.0;
      double cont = v.cont ? v.cb.f[k] * v.cw * S[k] : 0.0;
      T[k] = nee + cont;
    }
    if (v.param) {
      // material-attribute gradients (R, G, B, metal, rough) for this vertex
      double g[5] = {0, 0, 0, 0, 0}, ga[5] = {0, 0, 0, 0, 0};
      for (int k = 0; k < 3; ++k) {
        double cn = v.nee ? adj[k] * v.beta[k] * v.K[k] : 0.0;
        double cc = v.cont ? adj[k] * v.beta[k] * v.cw * S[k] : 0.0;
        double t;
        t = cn * v.nb.dc[k]; g[k] += t; ga[k] += std::fabs(t);
        t = cc * v.cb.dc[k]; g[k] += t; ga[k] += std::fabs(t);
        t = cn * v.nb.dm[k]; g[3] += t; ga[3] += std::fabs(t);
        t = cc * v.cb.dm[k]; g[3] += t; ga[3] += std::fabs(t);
        t = cn * v.nb.dr[k]; g[4] += t; ga[4] += std::fabs(t);
        t = cc * v.cb.dr[k]; g[4] += t; ga[4] += std::fabs(t);
      }
      for (int b = 0; b < 5; ++b) {
        int slot = sc.ch_slot[b];
        if (slot < 0) continue;
        for (int f = 0; f < v.fp.n; ++f) {
          size_t idx = (size_t)v.fp.texel[f] * sc.n_ch + slot;
          grad[idx] += v.fp.w[f] * g[b];
          gabs[idx] += v.fp.w[f] * ga[b];
        }
      }
    }
    for (int k = 0; k < 3; ++k) T_next[k] = T[k];
  }
}

struct Crop {
  int x0, y0, x1, y1;
};

Crop get_crop(const orc_scene* s, const int* crop) {
  if (!crop) return {0, 0, s->width, s->height};
  return {std::max(0, crop[0]), std::max(0, crop[1]), std::min(s->width, crop[2]),
          std::min(s->height, crop[3])};
}

PathRng make_rng(uint64_t key, uint32_t pixel, uint32_t sample) {
  PathRng r;
  r.key[0] = (uint32_t)key;
  r.key[1] = (uint32_t)(key >> 32);
  r.pixel = pixel;
  r.sample = sample;
  return r;
}

size_t n_params(const Scene& sc) {
  if (sc.volume()) return 4 * (size_t)sc.s->vol_res * sc.s->vol_res * sc.s->vol_res;
  const size_t elems = sc.s->param_layout == 1 ? (size_t)sc.s->n_verts
                                               : (size_t)sc.s->tex_w * sc.s->tex_h;
  return elems * sc.n_ch;
}

// Run fn(row, thread) over crop rows, one contiguous band of rows per thread.
template <class Fn>
void parallel_rows(const Crop& c, int nthreads, Fn fn) {
  int rows = c.y1 - c.y0;
  if (rows <= 0) return;
  nthreads = std::max(1, std::min(nthreads, rows));
  std::vector<std::thread> pool;
  for (int t = 0; t < nthreads; ++t) {
    int r0 = c.y0 + rows * t / nthreads, r1 = c.y0 + rows * (t + 1) / nthreads;
    pool.emplace_back([=]() {
      for (int y = r0; y < r1; ++y) fn(y, t);
    });
  }
  for (auto& th : pool) th.join();
}

int check(const orc_scene* s) {
  if (!s || s->width <= 0 || s->height <= 0 || s->depth < 1 || s->tex_w < 1 || s->tex_h < 1)
    return -1;
  if ((s->ch_mask & ~31) != 0 || s->ch_mask == 0) return -1;
  if (s->n_tris < 0 || s->n_verts < 0 || (s->n_tris > 0 && (!s->tris || !s->verts))) return -1;
  for (long k = 0; k < 3L * s->n_tris; ++k)
    if (s->tris[k] < 0 || s->tris[k] >= s->n_verts) return -1;
  if (s->param_layout == 1) {
    // only the mesh may carry per-vertex parameters
    if (s->n_tris == 0 || s->mesh_mat != -1) return -1;
    if (s->plane_enabled && s->plane_mat < 0) return -1;
    for (int k = 0; k < s->n_spheres; ++k)
      if (s->sphere_mat[k] < 0) return -1;
  } else if (s->param_layout == 2) {
    // a volume alone: no surfaces, no light
    if (s->vol_res < 1 || s->vol_views < 1 || s->height % s->vol_views != 0) return -1;
    if (!(s->vol_box[3] > 0) || !(s->vol_sigma >= 0) || s->ch_mask != 15) return -1;
    if (s->plane_enabled || s->n_spheres > 0 || s->n_tris > 0 || s->light_enabled) return -1;
  } else if (s->param_layout != 0) {
    return -1;
  }
  return 0;
}

}  // namespace

// --------------------------------------------------------------------------
// C API
// --------------------------------------------------------------------------
extern "C" {

uint64_t orc_splitmix64(uint64_t x) { return splitmix64(x); }

void orc_reset_stats(void) {
  g_paths = 0;
  g_vertices = 0;
  g_param_vertices = 0;
}

void orc_get_stats(uint64_t out[3]) {
  out[0] = g_paths.load();
  out[1] = g_vertices.load();
  out[2] = g_param_vertices.load();
}

void orc_set_jitter_offset(double dx, double dy) {
  g_jitter_dx = dx;
  g_jitter_dy = dy;
}

void orc_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]) {
  philox(ctr, key, out);
}

uint64_t orc_stream_key(uint64_t seed, uint32_t iteration, uint32_t tag) {
  return stream_key(seed, iteration, tag);
}

void orc_bsdf(const double mat[5], const double n[3], const double wo[3], const double wi[3],
              int flags, double out[13]) {
  Material m;
  m.c[0] = mat[0]; m.c[1] = mat[1]; m.c[2] = mat[2];
  m.metal = mat[3];
  m.rough = mat[4];
  Bsdf b = eval_bsdf(m, from(n), from(wo), from(wi), flags);
  for (int k = 0; k < 3; ++k) {
    out[k] = b.f[k];
    out[3 + k] = b.dc[k];
    out[6 + k] = b.dm[k];
    out[9 + k] = b.dr[k];
  }
  out[12] = b.pdf;
}

void orc_bsdf_many(int count, const double mat[5], const double n[3], const double wo[3],
                   const double* wi, int flags, double* out) {
  for (int i = 0; i < count; ++i) orc_bsdf(mat, n, wo, wi + 3 * i, flags, out + 13 * i);
}

int orc_render(const orc_scene* s, const double* params, uint64_t seed, uint32_t iteration,
               uint32_t tag, int spp, int flags, const int* crop, double* img, double* margin,
               int nthreads) {
  return orc_render_sampled(s, params, nullptr, seed, iteration, tag, spp, flags, crop, img,
                            margin, nthreads);
}

int orc_render_sampled(const orc_scene* s, const double* params, const double* sample_params,
                       uint64_t seed, uint32_t iteration, uint32_t tag, int spp, int flags,
                       const int* crop, double* img, double* margin, int nthreads) {
  if (check(s) || spp < 1 || !img) return -1;
  Scene sc(s);
  Crop c = get_crop(s, crop);
  uint64_t key = stream_key(seed, iteration, tag);
  parallel_rows(c, nthreads, [&](int y, int) {
    for (int x = c.x0; x < c.x1; ++x) {
      uint32_t pix = (uint32_t)(y * s->width + x);
      double acc[3] = {0, 0, 0}, mg = INF;
      for (int smp = 0; smp < spp; ++smp) {
        PathResult r;
        trace(sc, params, sample_params, make_rng(key, pix, smp), x, y, flags, false, r);
        for (int k = 0; k < 3; ++k) acc[k] += r.L[k];
        mg = std::min(mg, r.margin);
      }
      for (int k = 0; k < 3; ++k) img[3 * (size_t)pix + k] = acc[k] / spp;
      if (margin) margin[pix] = mg;
    }
  });
  return 0;
}

static int grad_common(const orc_scene* s, const double* params, const double* sample_params,
                       uint64_t key_adj, int spp,
                       const double* dimg, int flags, const Crop& c, const unsigned char* mask,
                       double* grad, double* gabs, double* margin, double* adj_img,
                       int nthreads) {
  Scene sc(s);
  size_t np = n_params(sc);
  int rows = c.y1 - c.y0;
  int nt = std::max(1, std::min(nthreads, std::max(rows, 1)));
  std::vector<std::vector<double>> g(nt, std::vector<double>(np, 0.0));
  std::vector<std::vector<double>> ga(nt, std::vector<double>(np, 0.0));
  parallel_rows(c, nt, [&](int y, int t) {
    for (int x = c.x0; x < c.x1; ++x) {
      uint32_t pix = (uint32_t)(y * s->width + x);
      if (mask && mask[pix]) continue;
      double adj[3];
      for (int k = 0; k < 3; ++k) adj[k] = dimg[3 * (size_t)pix + k] / spp;
      double mg = margin ? margin[pix] : INF;
      double acc[3] = {0, 0, 0};
      for (int smp = 0; smp < spp; ++smp) {
        PathResult r;
        trace(sc, params, sample_params, make_rng(key_adj, pix, smp), x, y, flags, true, r);
        if (sc.volume())
          backprop_volume(sc, r.vtape, adj, g[t].data(), ga[t].data());
        else
          backprop(sc, r.tape, adj, g[t].data(), ga[t].data());
        mg = std::min(mg, r.margin);
        for (int k = 0; k < 3; ++k) acc[k] += r.L[k];
      }
      if (margin) margin[pix] = mg;
      if (adj_img)
        for (int k = 0; k < 3; ++k) adj_img[3 * (size_t)pix + k] = acc[k] / spp;
    }
  });
  for (size_t i = 0; i < np; ++i) {
    double a = 0, b = 0;
    for (int t = 0; t < nt; ++t) {
      a += g[t][i];
      b += ga[t][i];
    }
    grad[i] = a;
    if (gabs) gabs[i] = b;
  }
  return 0;
}

int orc_grad(const orc_scene* s, const double* params, uint64_t seed, uint32_t iteration,
             uint32_t tag_primal, uint32_t tag_adj, int spp, const double* target, int flags,
             const int* crop, const unsigned char* mask, double* grad, double* gabs, double* img,
             double* margin, double* adj_img, int nthreads) {
  return orc_grad_sampled(s, params, nullptr, seed, iteration, tag_primal, tag_adj, spp, target,
                          flags, crop, mask, grad, gabs, img, margin, adj_img, nthreads);
}

int orc_grad_sampled(const orc_scene* s, const double* params, const double* sample_params,
                     uint64_t seed, uint32_t iteration, uint32_t tag_primal, uint32_t tag_adj,
                     int spp, const double* target, int flags, const int* crop,
                     const unsigned char* mask, double* grad, double* gabs, double* img,
                     double* margin, double* adj_img, int nthreads) {
  if (check(s) || spp < 1 || !grad || !target) return -1;
  Crop c = get_crop(s, crop);
  size_t npix = (size_t)s->width * s->height;
  std::vector<double> I(3 * npix, 0.0), mg(npix, INF), dimg(3 * npix, 0.0);
  orc_render_sampled(s, params, sample_params, seed, iteration, tag_primal, spp, flags, crop,
                     I.data(), mg.data(), nthreads);
  // L = sum (I - T)^2 / (3 W H)  ->  dL/dI = 2 (I - T) / (3 W H); the relative
  // form divides each term by T^2 + REL_EPS (a constant per pixel, so the
  // primal from its own stream keeps the gradient sample unbiased)
  const double norm = 2.0 / (3.0 * (double)npix);
  const bool relative = (flags & ORC_RELATIVE_LOSS) != 0;
  for (int y = c.y0; y < c.y1; ++y)
    for (int x = c.x0; x < c.x1; ++x)
      for (int k = 0; k < 3; ++k) {
        size_t i = 3 * ((size_t)y * s->width + x) + k;
        const double w = relative ? 1.0 / (target[i] * target[i] + REL_EPS) : 1.0;
        dimg[i] = norm * (I[i] - target[i]) * w;
      }
  int rc = grad_common(s, params, sample_params, stream_key(seed, iteration, tag_adj), spp,
                       dimg.data(), flags, c, mask, grad, gabs, mg.data(), adj_img, nthreads);
  if (img)
    for (int y = c.y0; y < c.y1; ++y)
      for (int x = c.x0; x < c.x1; ++x)
        for (int k = 0; k < 3; ++k) {
          size_t i = 3 * ((size_t)y * s->width + x) + k;
          img[i] = I[i];
        }
  if (margin)
    for (int y = c.y0; y < c.y1; ++y)
      for (int x = c.x0; x < c.x1; ++x) margin[(size_t)y * s->width + x] = mg[(size_t)y * s->width + x];
  return rc;
}

int orc_render_bwd(const orc_scene* s, const double* params, uint64_t seed, uint32_t iteration,
                   uint32_t tag, int spp, const double* dimg, int flags, const int* crop,
                   const unsigned char* mask, double* grad, double* gabs, double* margin,
                   double* adj_img, int nthreads) {
  return orc_render_bwd_sampled(s, params, nullptr, seed, iteration, tag, spp, dimg, flags, crop,
                                mask, grad, gabs, margin, adj_img, nthreads);
}

int orc_render_bwd_sampled(const orc_scene* s, const double* params,
                           const double* sample_params, uint64_t seed, uint32_t iteration,
                           uint32_t tag, int spp, const double* dimg, int flags, const int* crop,
                           const unsigned char* mask, double* grad, double* gabs, double* margin,
                           double* adj_img, int nthreads) {
  if (check(s) || spp < 1 || !grad || !dimg) return -1;
  Crop c = get_crop(s, crop);
  if (margin)
    for (int y = c.y0; y < c.y1; ++y)
      for (int x = c.x0; x < c.x1; ++x) margin[(size_t)y * s->width + x] = INF;
  return grad_common(s, params, sample_params, stream_key(seed, iteration, tag), spp, dimg, flags,
                     c, mask, grad, gabs, margin, adj_img, nthreads);
}

}  // extern "C"
