// Device-side building blocks of the jso path tracer (gfx950, wave64).
//
// FP32 radiance arithmetic; each path's radiance ledger is kept in FP64 so
// that the replayed adjoint can recover the radiance still to come after a
// vertex (total minus collected) without cancellation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "bvh.h"
#include "jso.h"
#include "kernels.h"

namespace jso {

constexpr float kPi = 3.14159265358979323846f;
constexpr float kInvPi = 0.318309886183790671538f;
constexpr float kTwoPi = 6.28318530717958647692f;
constexpr float kRayEps = 1e-4f;     // ray origins move this far along the normal
constexpr float kShadowEps = 1e-4f;  // shadow rays stop this short of the light
constexpr float kRoughMin = 0.05f;   // roughness floor of the material model
constexpr float kPSpec = 0.5f;       // probability of the specular lobe
constexpr float kInf = __builtin_huge_valf();

// ---------------------------------------------------------------------------
// scene as seen by the kernels (passed by value as a kernel argument, so all
// of it lives in the scalar-loaded kernarg segment)
// ---------------------------------------------------------------------------
struct DevScene {
  int width, height;
  float eye[3], cw[3], cu[3], cv[3];
  float tan_half, aspect;
  int plane_enabled, plane_mat;
  float plane_x0, plane_x1, plane_z0, plane_z1;
  int n_spheres;
  float sph[JSO_MAX_SPHERES][4];
  int sph_mat[JSO_MAX_SPHERES];
  int light_enabled;
  float lc[3], lside, lhalf, larea, Le[3];
  float env[3];
  int depth, rr_start;
  float rr_q;
  int tex_w, tex_h, n_ch;
  int slot[5];          // slot of channel b inside a texel, -1 if fixed
  float defaults[5];
  int n_fixed;
  float fixed[JSO_MAX_FIXED_MATS][5];
  // triangle mesh (n_tris = 0: none), indexed by a BVH in the layout of bvh.h
  int n_tris, mesh_mat, layout, bvh_depth;
  JSO_GMEM const float4* bvh_nodes;  // four-wide nodes, 8 words each
  JSO_GMEM const float4* bvh_tris;   // 3 words per triangle, leaf order
  JSO_GMEM const int* bvh_tri_id;    // original index of each reordered triangle
  // emission-absorption volume (layout JSO_LAYOUT_VOLUME); vol_rb: bricks of
  // 4x4x4 voxels per side of the kernels' bricked copy of the parameters
  int vol_res, vol_rb, vol_views, view_h;
  float vol_lo[3], vol_side, vol_inv_vox, vol_sigma;
  float view_eye[JSO_MAX_VIEWS][3], view_cw[JSO_MAX_VIEWS][3], view_cu[JSO_MAX_VIEWS][3],
      view_cv[JSO_MAX_VIEWS][3];
};

// ---------------------------------------------------------------------------
// small vector type
// ---------------------------------------------------------------------------
struct V3 {
  float x, y, z;
};
__device__ __forceinline__ V3 mk(float x, float y, float z) { return V3{x, y, z}; }
__device__ __forceinline__ V3 operator+(V3 a, V3 b) { return mk(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ V3 operator-(V3 a, V3 b) { return mk(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ V3 operator*(V3 a, float s) { return mk(a.x * s, a.y * s, a.z * s); }
__device__ __forceinline__ float dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
  return mk(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ V3 normalize(V3 a) { return a * (1.0f / sqrtf(dot(a, a))); }
__device__ __forceinline__ V3 ld3(const float* p) { return mk(p[0], p[1], p[2]); }

// ---------------------------------------------------------------------------
// counter-based random numbers
// ---------------------------------------------------------------------------
// Philox4x32-10, Salmon, Moraes, Dror, Shaw (SC'11): ten rounds of two
// 32x32->64 multiplies with xor mixing; the key advances by the Weyl
// constants between rounds.
__host__ __device__ __forceinline__ uint32_t mulhi32(uint32_t a, uint32_t b) {
  return (uint32_t)(((uint64_t)a * (uint64_t)b) >> 32);
}

__host__ __device__ __forceinline__ uint4 philox10(uint4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r != 0) {
      k0 += 0x9E3779B9u;
      k1 += 0xBB67AE85u;
    }
    const uint32_t a = c.x, b = c.z;
    const uint32_t lo_a = 0xD2511F53u * a, hi_a = mulhi32(0xD2511F53u, a);
    const uint32_t lo_b = 0xCD9E8D57u * b, hi_b = mulhi32(0xCD9E8D57u, b);
    c = make_uint4(hi_b ^ c.y ^ k0, lo_b, hi_a ^ c.w ^ k1, lo_a);
  }
  return c;
}

// SplitMix64 output function for state x (Steele, Lea, Flood 2014).
__host__ __device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
  uint64_t z = x + 0x9E3779B97F4A7C15ull;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}

__host__ __device__ __forceinline__ uint64_t stream_key(uint64_t seed, uint32_t it, uint32_t tag) {
  return splitmix64(seed ^ splitmix64(((uint64_t)it << 8) | (uint64_t)tag));
}

// 24 high bits of a word as a float in [0, 1); exact in FP32 and FP64.
__device__ __forceinline__ float u01(uint32_t x) { return (float)(x >> 8) * (1.0f / 16777216.0f); }

struct Rng {
  uint32_t k0, k1, pixel, sample;
  __device__ __forceinline__ void draw(uint32_t bounce, uint32_t block, float u[4]) const {
    uint4 r = philox10(make_uint4(pixel, sample, bounce, block), k0, k1);
    u[0] = u01(r.x);
    u[1] = u01(r.y);
    u[2] = u01(r.z);
    u[3] = u01(r.w);
  }
};

// ---------------------------------------------------------------------------
// intersection
// ---------------------------------------------------------------------------
enum : int { HIT_NONE = 0, HIT_PLANE = 1, HIT_SPHERE = 2, HIT_LIGHT = 3, HIT_MESH = 4 };

// Ray-sphere distance in FP32: discriminant from the squared distance of the
// centre to the ray (no b^2 - c cancellation), roots via q and c/q.
__device__ __forceinline__ float hit_sphere(const float* sp, V3 o, V3 d) {
  const V3 oc = o - mk(sp[0], sp[1], sp[2]);
  const float r2 = sp[3] * sp[3];
  const float b = dot(oc, d);
  const V3 f = oc - d * b;
  const float disc = r2 - dot(f, f);
  if (!(disc >= 0.0f)) return kInf;
  const float s = sqrtf(disc);
  const float q = -(b + copysignf(s, b));
  if (q == 0.0f) return kInf;
  const float c = dot(oc, oc) - r2;
  const float t0 = c / q;
  const float lo = fminf(t0, q), hi = fmaxf(t0, q);
  if (lo > 0.0f) return lo;
  if (hi > 0.0f) return hi;
  return kInf;
}

struct Hit {
  float t;
  int kind, obj;  // obj: sphere index, or triangle index in BVH leaf order
};

// Per-lane BVH traversal stack: the first `cap` entries in LDS, entry k of
// this lane at base[k * stride] (base already offset by the lane, stride =
// lanes of the block, so the lanes of a wave touch consecutive words); deeper
// entries, which few rays reach, spill to a private array.
constexpr int kLdsStack = 16;  // LDS entries per lane at most

struct TravStack {
  uint32_t* base;
  int stride;
  int cap;  // LDS entries per lane (<= kLdsStack)
};

struct StackSpill {
  uint32_t v[kBvhMaxStack - kLdsStack];
};

// A ray prepared for slab tests: o * (1/d) precomputed so each slab bound is
// one fma.  Zero direction components are nudged to +-1e-20 (finite inverse).
struct RayQ {
  V3 o, d, inv, oinv;
};

__device__ __forceinline__ float safe_inv(float x) {
  return 1.0f / (fabsf(x) > 1e-20f ? x : copysignf(1e-20f, x));
}

__device__ __forceinline__ RayQ make_rayq(V3 o, V3 d) {
  RayQ r;
  r.o = o;
  r.d = d;
  r.inv = mk(safe_inv(d.x), safe_inv(d.y), safe_inv(d.z));
  r.oinv = mk(o.x * r.inv.x, o.y * r.inv.y, o.z * r.inv.z);
  return r;
}

// Distance at which the ray enters the box within [0, tmax], or kInf.
__device__ __forceinline__ float box_entry(const RayQ& r, float lx, float ly, float lz, float hx,
                                           float hy, float hz, float tmax) {
  const float ax = fmaf(lx, r.inv.x, -r.oinv.x), bx = fmaf(hx, r.inv.x, -r.oinv.x);
  const float ay = fmaf(ly, r.inv.y, -r.oinv.y), by = fmaf(hy, r.inv.y, -r.oinv.y);
  const float az = fmaf(lz, r.inv.z, -r.oinv.z), bz = fmaf(hz, r.inv.z, -r.oinv.z);
  const float t0 = fmaxf(fmaxf(fminf(ax, bx), fminf(ay, by)), fmaxf(fminf(az, bz), 0.0f));
  const float t1 = fminf(fminf(fmaxf(ax, bx), fmaxf(ay, by)), fminf(fmaxf(az, bz), tmax));
  return t0 <= t1 ? t0 : kInf;
}

// Moller-Trumbore (J. Graphics Tools 1997) in FP32: distance of the hit in
// (0, tmax], or kInf.  Edges count as inside (u, v >= 0, u + v <= 1).
__device__ __forceinline__ float tri_hit(const RayQ& r, V3 v0, V3 e1, V3 e2, float tmax) {
  const V3 pv = cross(r.d, e2);
  const float det = dot(e1, pv);
  if (det == 0.0f) return kInf;
  const float inv = 1.0f / det;
  const V3 sv = r.o - v0;
  const float u = dot(sv, pv) * inv;
  const V3 qv = cross(sv, e1);
  const float v = dot(r.d, qv) * inv;
  const float t = dot(e2, qv) * inv;
  return (u >= 0.0f && v >= 0.0f && u + v <= 1.0f && t > 0.0f && t <= tmax) ? t : kInf;
}

// 16-byte load from global memory (the cast back to a generic pointer keeps the
// access global once inlined).
__device__ __forceinline__ float4 ldg4(JSO_GMEM const float4* p) { return *(const float4*)p; }

// Four-wide node: the entry distances of its four child boxes (kInf = missed)
// and their links.
struct Node4 {
  float t[4];
  int32_t l[4];
};

__device__ __forceinline__ Node4 load_node4(const DevScene& S, const RayQ& r, int32_t link,
                                            float tmax) {
  JSO_GMEM const float4* nd = S.bvh_nodes + 8 * (size_t)link;
  const float4 lx = ldg4(nd), hx = ldg4(nd + 1), ly = ldg4(nd + 2), hy = ldg4(nd + 3);
  const float4 lz = ldg4(nd + 4), hz = ldg4(nd + 5), ln = ldg4(nd + 6);
  Node4 n;
  n.t[0] = box_entry(r, lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, tmax);
  n.t[1] = box_entry(r, lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, tmax);
  n.t[2] = box_entry(r, lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, tmax);
  n.t[3] = box_entry(r, lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, tmax);
  n.l[0] = __float_as_int(ln.x);
  n.l[1] = __float_as_int(ln.y);
  n.l[2] = __float_as_int(ln.z);
  n.l[3] = __float_as_int(ln.w);
  return n;
}

__device__ __forceinline__ void order2(float& ta, int32_t& la, float& tb, int32_t& lb) {
  const bool sw = tb < ta;
  const float t = sw ? tb : ta;
  const int32_t l = sw ? lb : la;
  tb = sw ? ta : tb;
  lb = sw ? la : lb;
  ta = t;
  la = l;
}

__device__ __forceinline__ void push(const TravStack& st, StackSpill& sv, int& sp, int32_t link) {
  if (sp < st.cap)
    st.base[sp * st.stride] = (uint32_t)link;
  else
    sv.v[sp - st.cap] = (uint32_t)link;
  ++sp;
}

__device__ __forceinline__ int32_t pop(const TravStack& st, const StackSpill& sv, int& sp) {
  --sp;
  return (int32_t)(sp < st.cap ? st.base[sp * st.stride] : sv.v[sp - st.cap]);
}

// Closest triangle strictly nearer than `best_t` (or at best_t with a lower
// original index than the triangle already held).  At each node the hit
// children are sorted by entry distance (a 5-exchange network); the nearest is
// visited next and the others are deferred on the stack, nearest on top.
__device__ __forceinline__ void bvh_closest(const DevScene& S, const TravStack& st, V3 o, V3 d,
                                            float& best_t, int& best_tri) {
  const RayQ r = make_rayq(o, d);
  StackSpill sv;
  int sp = 0;
  int32_t link = 0;
  for (;;) {
    if (link >= 0) {
      Node4 n = load_node4(S, r, link, best_t);
      order2(n.t[0], n.l[0], n.t[1], n.l[1]);
      order2(n.t[2], n.l[2], n.t[3], n.l[3]);
      order2(n.t[0], n.l[0], n.t[2], n.l[2]);
      order2(n.t[1], n.l[1], n.t[3], n.l[3]);
      order2(n.t[1], n.l[1], n.t[2], n.l[2]);
      if (n.t[0] != kInf) {
        if (n.t[3] != kInf) push(st, sv, sp, n.l[3]);
        if (n.t[2] != kInf) push(st, sv, sp, n.l[2]);
        if (n.t[1] != kInf) push(st, sv, sp, n.l[1]);
        link = n.l[0];
        continue;
      }
    } else {
      const uint32_t v = ~(uint32_t)link;
      const int first = (int)(v >> kLeafBits), end = first + (int)(v & (uint32_t)kLeafMax);
      for (int i = first; i < end; ++i) {
        JSO_GMEM const float4* tp = S.bvh_tris + 3 * (size_t)i;
        const float4 a = ldg4(tp), b = ldg4(tp + 1), c = ldg4(tp + 2);
        const float t = tri_hit(r, mk(a.x, a.y, a.z), mk(b.x, b.y, b.z), mk(c.x, c.y, c.z), best_t);
        if (t < best_t ||
            (t == best_t && best_tri >= 0 && S.bvh_tri_id[i] < S.bvh_tri_id[best_tri])) {
          best_t = t;
          best_tri = i;
        }
      }
    }
    if (sp == 0) break;
    link = pop(st, sv, sp);
  }
}

// Closest hit for the rays of one wave's neighbouring pixels (camera rays),
// traversed by the wave together: one node sequence for the wave, each lane
// testing the node's children against its own ray and nearest hit so far.  A
// child is visited when any lane meets it, by the lanes that meet it (their
// mask travels with it on the wave's stack), nearest first by the distances of
// the first such lane.  Node and triangle words are wave-uniform, read through
// the scalar cache.  The stack (link and 64-bit lane mask per entry, 3 words)
// lives in the wave's per-lane LDS stack words, which hold it: it defers the
// same children per node as bvh_closest, and 3 x the tree's stack bound fits
// in 64 lanes x min(bound, kLdsStack) words.  The hit is bvh_closest's: every
// lane tests every leaf whose box it meets within its nearest hit so far.
__device__ __forceinline__ bool dist_less(float a, float b) {
  // both >= 0 or +inf: the IEEE bit patterns order as unsigned integers
  return __float_as_uint(a) < __float_as_uint(b);
}

// A 16-byte word of read-only data at a wave-uniform address, through the
// scalar cache.
__device__ __forceinline__ float4 ldc4(const JSO_CMEM float* p) {
  return make_float4(p[0], p[1], p[2], p[3]);
}

__device__ __forceinline__ void bvh_closest_wave(const DevScene& S, const TravStack& st, V3 o,
                                                 V3 d, float& best_t, int& best_tri) {
  const RayQ r = make_rayq(o, d);
  const int lane = (int)__lane_id();
  uint32_t* wbase = st.base - lane;  // stack word 0 of the wave's first lane
  auto word = [&](int q) -> uint32_t* { return wbase + (q & 63) + (q >> 6) * st.stride; };
  const JSO_CMEM float* nodes = (const JSO_CMEM float*)S.bvh_nodes;
  const JSO_CMEM float* tris = (const JSO_CMEM float*)S.bvh_tris;
  uint64_t m = __ballot(1);  // lanes of the current node
  int32_t link = 0;
  int sp = 0;
  for (;;) {
    const bool me = (m >> lane) & 1ull;
    bool pop_next = true;
    if (link >= 0) {
      const JSO_CMEM float* nd = nodes + 32 * (size_t)link;
      const float4 lx = ldc4(nd), hx = ldc4(nd + 4), ly = ldc4(nd + 8), hy = ldc4(nd + 12);
      const float4 lz = ldc4(nd + 16), hz = ldc4(nd + 20), ln = ldc4(nd + 24);
      float t[4] = {kInf, kInf, kInf, kInf};
      if (me) {
        t[0] = box_entry(r, lx.x, ly.x, lz.x, hx.x, hy.x, hz.x, best_t);
        t[1] = box_entry(r, lx.y, ly.y, lz.y, hx.y, hy.y, hz.y, best_t);
        t[2] = box_entry(r, lx.z, ly.z, lz.z, hx.z, hy.z, hz.z, best_t);
        t[3] = box_entry(r, lx.w, ly.w, lz.w, hx.w, hy.w, hz.w, best_t);
      }
      uint64_t hk[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) hk[k] = __ballot(t[k] != kInf);
      const uint64_t any = hk[0] | hk[1] | hk[2] | hk[3];
      if (any != 0) {
        const int lead = __ffsll((unsigned long long)any) - 1;
        float lt[4];
        int32_t ll[4] = {__float_as_int(ln.x), __float_as_int(ln.y), __float_as_int(ln.z),
                         __float_as_int(ln.w)};
#pragma unroll
        for (int k = 0; k < 4; ++k)
          lt[k] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(t[k]), lead));
        // sort the 4 children by the first lane's entry distance
        auto cswap = [&](int a, int b) {
          if (dist_less(lt[b], lt[a])) {
            const float tf = lt[a];
            lt[a] = lt[b];
            lt[b] = tf;
            const int32_t tl = ll[a];
            ll[a] = ll[b];
            ll[b] = tl;
            const uint64_t tm = hk[a];
            hk[a] = hk[b];
            hk[b] = tm;
          }
        };
        cswap(0, 1);
        cswap(2, 3);
        cswap(0, 2);
        cswap(1, 3);
        cswap(1, 2);
        int f = 3;
#pragma unroll
        for (int k = 3; k >= 0; --k)
          if (hk[k] != 0) f = k;
#pragma unroll
        for (int k = 3; k >= 1; --k) {
          if (k <= f || hk[k] == 0) continue;
          *word(3 * sp) = (uint32_t)ll[k];
          *word(3 * sp + 1) = (uint32_t)hk[k];
          *word(3 * sp + 2) = (uint32_t)(hk[k] >> 32);
          ++sp;
        }
        link = ll[f];
        m = hk[f];
        pop_next = false;
      }
    } else {
      const uint32_t v = ~(uint32_t)link;
      const int first = (int)(v >> kLeafBits), end = first + (int)(v & (uint32_t)kLeafMax);
      for (int i = first; i < end; ++i) {
        const JSO_CMEM float* tp = tris + 12 * (size_t)i;
        const float4 a = ldc4(tp), b = ldc4(tp + 4), c = ldc4(tp + 8);
        if (me) {
          const float t = tri_hit(r, mk(a.x, a.y, a.z), mk(b.x, b.y, b.z), mk(c.x, c.y, c.z),
                                  best_t);
          if (t < best_t ||
              (t == best_t && best_tri >= 0 && S.bvh_tri_id[i] < S.bvh_tri_id[best_tri])) {
            best_t = t;
            best_tri = i;
          }
        }
      }
    }
    if (pop_next) {
      if (sp == 0) break;
      --sp;
      link = (int32_t)__builtin_amdgcn_readfirstlane(*word(3 * sp));
      const uint32_t lo = __builtin_amdgcn_readfirstlane(*word(3 * sp + 1));
      const uint32_t hi = __builtin_amdgcn_readfirstlane(*word(3 * sp + 2));
      m = (uint64_t)lo | ((uint64_t)hi << 32);
    }
  }
}

// Whether any triangle lies at a distance in (0, tmax).  Children in slot
// order, the first hit one visited next.  Each lane may hold one postponed
// leaf (speculative traversal, Aila and Laine, "Understanding the efficiency
// of ray traversal on GPUs", HPG 2009): a lane that reaches a leaf sets it
// aside and goes on down inner nodes, and the wave tests triangles once every
// lane holds a leaf or is finished, so node visits and triangle tests each run
// on more lanes at once.  Postponing changes only when a hit is found, not
// whether.  (The closest-hit traversal measured slower this way: a postponed
// leaf's hit would have culled the nodes visited meanwhile.)
__device__ __forceinline__ bool bvh_any(const DevScene& S, const TravStack& st, V3 o, V3 d,
                                        float tmax) {
  const RayQ r = make_rayq(o, d);
  StackSpill sv;
  int sp = 0;
  int32_t link = 0;
  bool go = true, hit = false;
  int32_t leaf = 0;
  bool has = false;
  for (;;) {
    while (!__all(has || !go)) {
      if (!go || (has && link < 0)) continue;
      if (link >= 0) {
        const Node4 n = load_node4(S, r, link, tmax);
        int32_t next = 0;
        bool any = false;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          if (n.t[k] == kInf) continue;
          if (any) push(st, sv, sp, n.l[k]);
          else next = n.l[k];
          any = true;
        }
        if (any) link = next;
        else if (sp == 0) go = false;
        else link = pop(st, sv, sp);
      } else {
        leaf = link;
        has = true;
        if (sp == 0) go = false;
        else link = pop(st, sv, sp);
      }
    }
    if (has) {
      const uint32_t v = ~(uint32_t)leaf;
      const int first = (int)(v >> kLeafBits), end = first + (int)(v & (uint32_t)kLeafMax);
      for (int i = first; i < end; ++i) {
        JSO_GMEM const float4* tp = S.bvh_tris + 3 * (size_t)i;
        const float4 a = ldg4(tp), b = ldg4(tp + 1), c = ldg4(tp + 2);
        if (tri_hit(r, mk(a.x, a.y, a.z), mk(b.x, b.y, b.z), mk(c.x, c.y, c.z), tmax) < tmax) {
          hit = true;
          break;
        }
      }
      has = false;
      if (hit) go = false;
    }
    if (!__any(go)) break;
  }
  return hit;
}

// Closest hit; candidates in the order plane < spheres < mesh < light, each
// replacing the current one only at a strictly smaller distance, so equal
// distances keep the earlier kind.
// kCoherent: the rays of the calling lanes come from neighbouring pixels of
// one wave (bvh_closest_wave); the hit is the same either way.
template <bool kMesh, bool kCoherent = false>
__device__ __forceinline__ Hit intersect(const DevScene& S, const TravStack& st, V3 o, V3 d) {
  Hit h{kInf, HIT_NONE, -1};
  if (S.plane_enabled && d.y < 0.0f && o.y > 0.0f) {
    h.t = -o.y / d.y;
    h.kind = HIT_PLANE;
    h.obj = 0;
  }
  for (int k = 0; k < S.n_spheres; ++k) {
    const float t = hit_sphere(S.sph[k], o, d);
    if (t < h.t) {
      h.t = t;
      h.kind = HIT_SPHERE;
      h.obj = k;
    }
  }
  if (kMesh && S.n_tris > 0) {
    int tri = -1;
    float t = h.t;
    if (kCoherent) bvh_closest_wave(S, st, o, d, t, tri);
    else bvh_closest(S, st, o, d, t, tri);
    if (tri >= 0) {
      h.t = t;
      h.kind = HIT_MESH;
      h.obj = tri;
    }
  }
  if (S.light_enabled && d.y > 0.0f && o.y < S.lc[1]) {
    const float t = (S.lc[1] - o.y) / d.y;
    const float dx = o.x + t * d.x - S.lc[0], dz = o.z + t * d.z - S.lc[2];
    if (fabsf(dx) <= S.lhalf && fabsf(dz) <= S.lhalf && t < h.t) {
      h.t = t;
      h.kind = HIT_LIGHT;
      h.obj = 0;
    }
  }
  return h;
}

template <bool kMesh>
__device__ __forceinline__ bool occluded(const DevScene& S, const TravStack& st, V3 o, V3 d,
                                         float tmax) {
  if (S.plane_enabled && d.y < 0.0f && o.y > 0.0f && -o.y / d.y < tmax) return true;
  for (int k = 0; k < S.n_spheres; ++k)
    if (hit_sphere(S.sph[k], o, d) < tmax) return true;
  if (kMesh && S.n_tris > 0) return bvh_any(S, st, o, d, tmax);
  return false;
}

// ---------------------------------------------------------------------------
// hit records
//
// The forward pass of a path that a replay will read back writes, for its
// first kHitRecs rays (the camera ray, then the continuation rays), what the
// ray hit and whether the shadow ray of the vertex it reached is blocked, so
// the replay need not trace those rays again.  Record k, kRecWords words:
//   w0: hit kind | blocked << 3 | object << 10 (the object bits of the path's
//       hit word),
//   w1: the hit distance's bits,
//   w2: the ray's tag: a hash of its origin and direction bits, its index k,
//       the path's random stream (key, pixel, sample) and the plan's epoch.
// The replay takes a record only when its tag equals the tag of the replay's
// own ray and its object index is in range, and only while it took every
// earlier record of the path; otherwise it traces.  A record left by another
// launch or another plan, or one of a path the replay does not reproduce bit
// for bit, is never used, so the replay finds exactly the hits the forward
// pass found for the same rays.
// kRec: REC_NONE (no records: the plain tracing code), REC_WRITE (forward
// pass), REC_READ (replay); with a null base the calls trace.
// ---------------------------------------------------------------------------
enum : int { REC_NONE = 0, REC_WRITE = 1, REC_READ = 2 };

struct HitRecs {
  JSO_GMEM uint32_t* base;  // record 0 of the path, or null
  uint32_t stride;          // words from record k to record k + 1
  uint32_t epoch;
};

// One step of the tag hash: a bijection of h for each word w (xor, a
// multiplication by an odd constant, an xor-shift), so two inputs that differ
// in a single word always hash apart.
__device__ __forceinline__ uint32_t tag_step(uint32_t h, uint32_t w) {
  h = (h ^ w) * 0x9E3779B1u;
  return h ^ (h >> 16);
}

__device__ __forceinline__ uint32_t ray_tag(const Rng& rng, uint32_t epoch, int k, V3 o, V3 d) {
  uint32_t h = tag_step(epoch, rng.k0);
  h = tag_step(h, rng.k1);
  h = tag_step(h, rng.pixel);
  h = tag_step(h, rng.sample ^ ((uint32_t)k << 24));
  h = tag_step(h, __float_as_uint(o.x));
  h = tag_step(h, __float_as_uint(o.y));
  h = tag_step(h, __float_as_uint(o.z));
  h = tag_step(h, __float_as_uint(d.x));
  h = tag_step(h, __float_as_uint(d.y));
  return tag_step(h, __float_as_uint(d.z));
}

// The closest hit of ray k of the path (k = 0: the camera ray).
template <bool kMesh, bool kCoherent, int kRec>
__device__ __forceinline__ Hit traced_hit(const DevScene& S, const TravStack& st, V3 o, V3 d,
                                          const HitRecs& hr, const Rng& rng, int k,
                                          bool& rec_ok) {
  if constexpr (kRec != REC_NONE) {
    if (hr.base != nullptr && k < kHitRecs) {
      JSO_GMEM uint32_t* r = hr.base + (size_t)k * hr.stride;
      const uint32_t tag = ray_tag(rng, hr.epoch, k, o, d);
      if constexpr (kRec == REC_READ) {
        if (rec_ok) {
          const uint32_t w0 = r[0], w1 = r[1], w2 = r[2];
          const int kind = (int)(w0 & 7u);
          const int obj = (int)(w0 >> 10);
          const bool in_range = kind <= HIT_MESH &&
                                (kind != HIT_SPHERE || obj < S.n_spheres) &&
                                (kind != HIT_MESH || (kMesh && obj < S.n_tris));
          if (w2 == tag && in_range) return Hit{__uint_as_float(w1), kind, obj};
          rec_ok = false;
        }
      } else {
        const Hit h = intersect<kMesh, kCoherent>(S, st, o, d);
        r[0] = (uint32_t)h.kind | ((uint32_t)h.obj << 10);
        r[1] = __float_as_uint(h.t);
        r[2] = tag;
        return h;
      }
    }
  }
  return intersect<kMesh, kCoherent>(S, st, o, d);
}

// Whether the shadow ray of the vertex that ray k reached is blocked; hit is
// that vertex's hit word.  The replay reads the bit only while rec_ok, that
// is when it took record k, so the vertex and the shadow ray are the forward
// pass's.
template <bool kMesh, int kRec>
__device__ __forceinline__ bool traced_occluded(const DevScene& S, const TravStack& st, V3 o,
                                                V3 d, float tmax, const HitRecs& hr, int k,
                                                uint32_t hit, const bool& rec_ok) {
  if constexpr (kRec != REC_NONE) {
    if (hr.base != nullptr && k < kHitRecs) {
      JSO_GMEM uint32_t* r = hr.base + (size_t)k * hr.stride;
      if constexpr (kRec == REC_READ) {
        if (rec_ok) return (r[0] & 8u) != 0u;
      } else {
        const bool occ = occluded<kMesh>(S, st, o, d, tmax);
        if (occ) r[0] = (hit & ~(127u << 3)) | 8u;  // w0 as written, with the bit
        return occ;
      }
    }
  }
  return occluded<kMesh>(S, st, o, d, tmax);
}

// ---------------------------------------------------------------------------
// materials
// ---------------------------------------------------------------------------
struct Mat {
  float c[3], m, r;
};

// Footprint of a parameterised-material lookup: the (up to four) parameter
// elements the material at a point interpolates, and their weights.
//   bilinear texture: texels t00, t01 (x + 1), t10 (y + 1) and t01 + t10 - t00,
//     weights from the fractions (fx, fy);
//   global (1x1 texture): element 0, weight 1;
//   triangle (per-vertex layout): vertices t00, t01, t10 with the barycentric
//     weights 1 - fx - fy, fx, fy (fourth weight 0).
struct Footprint {
  int global;
  int tri;
  int t00, t01, t10;
  float fx, fy;
};

// Weight of element q (0..3) of the footprint.  kMesh = false: the scene has
// no mesh, so no footprint is a triangle's.
template <bool kMesh>
__device__ __forceinline__ float footprint_weight(const Footprint& fp, int q) {
  if (kMesh && fp.tri)
    return q == 0 ? (1.0f - fp.fx) - fp.fy : (q == 1 ? fp.fx : (q == 2 ? fp.fy : 0.0f));
  return ((q & 1) ? fp.fx : 1.0f - fp.fx) * ((q & 2) ? fp.fy : 1.0f - fp.fy);
}

template <bool kMesh>
__device__ __forceinline__ void texel_weights(const Footprint& fp, float w[4]) {
#pragma unroll
  for (int q = 0; q < 4; ++q) w[q] = footprint_weight<kMesh>(fp, q);
}

// Bilinear, clamp-to-edge; texel centres at (i + 0.5) / size.
__device__ __forceinline__ Footprint footprint_uv(const DevScene& S, float u, float v) {
  Footprint fp;
  fp.global = 0;
  fp.tri = 0;
  const float x = u * (float)S.tex_w - 0.5f, y = v * (float)S.tex_h - 0.5f;
  const float x0 = floorf(x), y0 = floorf(y);
  fp.fx = x - x0;
  fp.fy = y - y0;
  const int xi0 = (int)fminf(fmaxf(x0, 0.0f), (float)(S.tex_w - 1));
  const int xi1 = (int)fminf(fmaxf(x0 + 1.0f, 0.0f), (float)(S.tex_w - 1));
  const int yi0 = (int)fminf(fmaxf(y0, 0.0f), (float)(S.tex_h - 1));
  const int yi1 = (int)fminf(fmaxf(y0 + 1.0f, 0.0f), (float)(S.tex_h - 1));
  fp.t00 = yi0 * S.tex_w + xi0;
  fp.t01 = yi0 * S.tex_w + xi1;
  fp.t10 = yi1 * S.tex_w + xi0;
  return fp;
}

// A surface point being shaded.  Mesh points also carry the triangle's vertex
// indices and the barycentric weights (bu, bv) of vertices 1 and 2.
struct Surf {
  int kind, obj;
  V3 p, n;
  int vid[3];
  float bu, bv;
};

// Material at a surface point.  Returns true for the parameterised material
// (then fp is its footprint); fixed materials return false.
template <bool kMesh>
__device__ __forceinline__ bool material_at(const DevScene& S, const float* __restrict__ params,
                                            const Surf& x, Mat& M, Footprint& fp) {
  const int mat = x.kind == HIT_PLANE ? S.plane_mat
                                      : (x.kind == HIT_MESH ? S.mesh_mat : S.sph_mat[x.obj]);
  if (mat >= 0) {
    M.c[0] = S.fixed[mat][0];
    M.c[1] = S.fixed[mat][1];
    M.c[2] = S.fixed[mat][2];
    M.m = S.fixed[mat][3];
    M.r = S.fixed[mat][4];
    return false;
  }
  float val[5];
  if (S.layout == JSO_LAYOUT_TEXTURE && S.tex_w == 1 && S.tex_h == 1) {
    fp.global = 1;
    fp.tri = 0;
    fp.t00 = fp.t01 = fp.t10 = 0;
    fp.fx = fp.fy = 0.0f;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      // load both and select the value (a select of the two addresses would
      // mix address spaces)
      const float pv = params[S.slot[b] >= 0 ? S.slot[b] : 0];
      val[b] = S.slot[b] >= 0 ? pv : S.defaults[b];
    }
  } else {
    if (kMesh && x.kind == HIT_MESH && S.layout == JSO_LAYOUT_VERTEX) {
      fp.global = 0;
      fp.tri = 1;
      fp.t00 = x.vid[0];
      fp.t01 = x.vid[1];
      fp.t10 = x.vid[2];
      fp.fx = x.bu;
      fp.fy = x.bv;
    } else {
      float u, v;
      if (x.kind == HIT_PLANE || (kMesh && x.kind == HIT_MESH)) {
        u = (x.p.x - S.plane_x0) / (S.plane_x1 - S.plane_x0);
        v = (x.p.z - S.plane_z0) / (S.plane_z1 - S.plane_z0);
      } else {
        const V3 n = x.n;
        u = 0.5f + atan2f(n.z, n.x) / kTwoPi;
        v = atan2f(sqrtf(n.x * n.x + n.z * n.z), n.y) * kInvPi;
      }
      fp = footprint_uv(S, u, v);
    }
    float w[4];
    texel_weights<kMesh>(fp, w);
    const int nc = S.n_ch;
    // the fourth element of a triangle footprint has weight 0 and is not read
    const int t11 = (kMesh && fp.tri) ? fp.t00 : fp.t01 + fp.t10 - fp.t00;
#pragma unroll
    for (int b = 0; b < 5; ++b) {
      const int s = S.slot[b];
      if (s < 0) {
        val[b] = S.defaults[b];
      } else {
        val[b] = w[0] * params[fp.t00 * nc + s] + w[1] * params[fp.t01 * nc + s] +
                 w[2] * params[fp.t10 * nc + s] + w[3] * params[t11 * nc + s];
      }
    }
  }
  M.c[0] = val[0];
  M.c[1] = val[1];
  M.c[2] = val[2];
  M.m = val[3];
  M.r = val[4];
  return true;
}

// ---------------------------------------------------------------------------
// BSDF: (1-m) c/pi + D G F / (4 cos_o cos_i), GGX D with alpha = r^2 (via
// sin^2 of the half-vector from a cross product), separable Smith G1,
// Schlick F with F0 = 0.04 (1-m) + m c.  With kGrad, the partials of f w.r.t.
// c (per channel), m and r.  pdf = density of sample_dir for wi.
// ---------------------------------------------------------------------------
struct Bsdf {
  float f[3];
  float pdf;
  float dc[3], dm[3], dr[3];
};

__device__ __forceinline__ float sin2(V3 n, V3 v) {
  const V3 c = cross(n, v);
  return dot(c, c);
}

template <bool kGrad>
__device__ __forceinline__ void eval_bsdf(const Mat& M, V3 n, V3 wo, V3 wi, uint32_t flags,
                                          Bsdf& b) {
  const float co = dot(n, wo), ci = dot(n, wi);
  b.pdf = 0.0f;
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    b.f[k] = 0.0f;
    if (kGrad) b.dc[k] = b.dm[k] = b.dr[k] = 0.0f;
  }
  if (!(co > 0.0f) || !(ci > 0.0f)) return;
  if (flags & JSO_F_LAMBERT_ONLY) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      b.f[k] = M.c[k] / kPi;
      if (kGrad) b.dc[k] = 1.0f / kPi;
    }
    b.pdf = ci / kPi;
    return;
  }
  const float r = fmaxf(M.r, kRoughMin);
  const float a = r * r, a2 = a * a;
  const V3 h = normalize(wo + wi);
  const float ch = dot(n, h), sh2 = sin2(n, h);
  const float Q = ch * ch * a2 + sh2;
  const float D = a2 / (kPi * Q * Q);
  const float so2 = sin2(n, wo), si2 = sin2(n, wi);
  const float qo = sqrtf(a2 * so2 + co * co), qi = sqrtf(a2 * si2 + ci * ci);
  const float Go = 2.0f * co / (co + qo), Gi = 2.0f * ci / (ci + qi);
  const float S = D * Go * Gi / (4.0f * co * ci);
  const float dh = fminf(1.0f, dot(wi, h));
  const float om = 1.0f - dh;
  const float om2 = om * om;
  const float w5 = om2 * om2 * om;
  float dS_dr = 0.0f;
  if (kGrad && M.r >= kRoughMin) {
    const float dlog = 2.0f / a - 4.0f * ch * ch * a / Q - (a * so2 / qo) / (co + qo) -
                       (a * si2 / qi) / (ci + qi);
    dS_dr = S * dlog * 2.0f * r;
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const float F0 = 0.04f * (1.0f - M.m) + M.m * M.c[k];
    const float F = F0 + (1.0f - F0) * w5;
    b.f[k] = (1.0f - M.m) * M.c[k] / kPi + S * F;
    if (kGrad) {
      b.dc[k] = (1.0f - M.m) / kPi + S * (1.0f - w5) * M.m;
      b.dm[k] = -M.c[k] / kPi + S * (1.0f - w5) * (M.c[k] - 0.04f);
      b.dr[k] = dS_dr * F;
    }
  }
  if (flags & JSO_F_PARAM_INDEP) {
    b.pdf = ci / kPi;
  } else {
    b.pdf = kPSpec * (D * ch / (4.0f * dh)) + (1.0f - kPSpec) * (ci / kPi);
  }
}

// Orthonormal basis around n (Duff et al., JCGT 2017).
__device__ __forceinline__ void onb(V3 n, V3& b1, V3& b2) {
  const float sign = copysignf(1.0f, n.z);
  const float a = -1.0f / (sign + n.z);
  const float b = n.x * n.y * a;
  b1 = mk(1.0f + sign * n.x * n.x * a, sign * b, -sign * n.x);
  b2 = mk(b, sign + n.y * n.y * a, -n.y);
}

// u[0] < kPSpec picks the GGX lobe (half-vector after Walter et al. 2007,
// reflected about it); otherwise a cosine-distributed direction.
__device__ __forceinline__ V3 sample_dir(const Mat& M, V3 n, V3 wo, const float u[4],
                                         uint32_t flags) {
  V3 b1, b2;
  onb(n, b1, b2);
  const float phi = kTwoPi * u[2];
  float sp, cp;
  sincosf(phi, &sp, &cp);
  const bool spec = !(flags & (JSO_F_LAMBERT_ONLY | JSO_F_PARAM_INDEP)) && u[0] < kPSpec;
  if (!spec) {
    const float rr = sqrtf(u[1]);
    const float z = sqrtf(fmaxf(0.0f, 1.0f - u[1]));
    return b1 * (rr * cp) + b2 * (rr * sp) + n * z;
  }
  const float r = fmaxf(M.r, kRoughMin);
  const float a = r * r;
  const float t2 = a * a * u[1] / (1.0f - u[1]);
  const float ct = 1.0f / sqrtf(1.0f + t2);
  const float st = sqrtf(t2) * ct;
  const V3 h = b1 * (st * cp) + b2 * (st * sp) + n * ct;
  return h * (2.0f * dot(wo, h)) - wo;
}

// ---------------------------------------------------------------------------
// path state and one vertex of a path (forward, or replay with derivatives)
// ---------------------------------------------------------------------------
struct Path {
  double led[3];  // FP64 ledger: radiance collected so far (replay: still to come)
  V3 o;           // pending hit point
  V3 d;           // direction of the ray that reached it
  float beta[3];
  uint32_t hit;   // pending hit: kind | vertex index j << 3 | object << 10
  bool alive;
  bool rec_ok;    // replay with hit records: every record of the path so far was taken
  __device__ __forceinline__ int kind() const { return (int)(hit & 7u); }
  __device__ __forceinline__ int j() const { return (int)((hit >> 3) & 127u); }
  __device__ __forceinline__ int obj() const { return (int)(hit >> 10); }
  __device__ __forceinline__ void set_hit(int kind, int obj, int j) {
    hit = (uint32_t)kind | ((uint32_t)j << 3) | ((uint32_t)obj << 10);
  }
};

// Material-attribute gradient of one vertex: g = d(adj . C)/d(R, G, B, metal, rough)
// restricted to this vertex's BSDF evaluations.
struct VertexGrad {
  bool valid;
  int j;  // vertex index along the path (1 = first surface hit)
  Footprint fp;
  float g[5];
};

// Second ledger of a shared-path finite-difference pair (Eq. 5): the path
// drawn at the first parameter vector, weighted by the BSDF of the second one
// over the first one's densities (continuation divisions and both MIS weights
// keep the first vector's pdf).  Forward: radiance collected so far; replay:
// radiance still to come.
struct Ledger2 {
  double led[3];
  float beta[3];
};

template <bool kMesh, int kRec = REC_NONE>
__device__ __forceinline__ void path_begin(const DevScene& S, const TravStack& st, const Rng& rng,
                                           int px, int py, uint32_t flags, Path& P,
                                           const HitRecs& hr = HitRecs{nullptr, 0, 0}) {
  float jx = 0.5f, jy = 0.5f;
  if (!(flags & JSO_F_PIXEL_CENTER)) {
    float u[4];
    rng.draw(0, 0, u);
    jx = u[0];
    jy = u[1];
  }
  const float sx = (2.0f * ((float)px + jx) / (float)S.width - 1.0f) * S.tan_half * S.aspect;
  const float sy = (1.0f - 2.0f * ((float)py + jy) / (float)S.height) * S.tan_half;
  const V3 eye = ld3(S.eye);
  P.d = normalize(ld3(S.cw) + ld3(S.cu) * sx + ld3(S.cv) * sy);
  P.beta[0] = P.beta[1] = P.beta[2] = 1.0f;
  P.led[0] = P.led[1] = P.led[2] = 0.0;
  if constexpr (kRec == REC_READ) P.rec_ok = true;
  const Hit h = traced_hit<kMesh, true, kRec>(S, st, eye, P.d, hr, rng, 0, P.rec_ok);
  P.o = eye + P.d * h.t;
  P.set_hit(h.kind, h.obj, 1);
  P.alive = false;
  if (h.kind == HIT_NONE) {
#pragma unroll
    for (int k = 0; k < 3; ++k) P.led[k] += (double)S.env[k];
  } else if (h.kind == HIT_LIGHT) {
#pragma unroll
    for (int k = 0; k < 3; ++k) P.led[k] += (double)S.Le[k];
  } else {
    P.alive = true;
  }
}

// Process the pending surface vertex of P.  Forward (kGrad = false): adds its
// NEE and continuation-emission terms to the ledger P.led and moves to the next
// vertex.  Replay (kGrad = true): P.led holds the radiance still to come
// (the path's total from the forward pass minus what the replay has
// reproduced so far); the same terms are recomputed and subtracted, and with
// R = that remainder after this vertex's NEE the vertex contributes
//   NEE:           adj . beta K df(w_l)
//   continuation:  adj . (R / f) df(w_i)
// which is the derivative of adj . C w.r.t. this vertex's material.
// kTwo: P also carries the second ledger L2 of a shared-path pair, evaluated
// with the material of params_b at the same point and directions; with kGrad
// vg.g is then (gradient of ledger 1) - (gradient of ledger 2, adjoint adj_b)
// over the one footprint both share.
// kRec, hr: the path's hit records (written by the forward pass, read by the
// replay) for the shadow ray of this vertex and the continuation ray.
template <bool kGrad, bool kMesh, bool kTwo, int kRec = REC_NONE>
__device__ __forceinline__ void path_vertex2(const DevScene& S, const TravStack& st,
                                             const float* __restrict__ params,
                                             const float* __restrict__ params_b, const Rng& rng,
                                             uint32_t flags, Path& P, Ledger2& L2,
                                             const float adj[3], const float adj_b[3],
                                             VertexGrad& vg,
                                             const HitRecs& hr = HitRecs{nullptr, 0, 0}) {
  Surf x;
  x.p = P.o;
  x.kind = P.kind();
  x.obj = P.obj();
  const int j = P.j();
  if (x.kind == HIT_PLANE) {
    x.p.y = 0.0f;
    x.n = mk(0.0f, 1.0f, 0.0f);
  } else if (kMesh && x.kind == HIT_MESH) {
    // two-sided: the geometric normal turned towards the incoming ray
    JSO_GMEM const float4* tp = S.bvh_tris + 3 * (size_t)x.obj;
    const float4 a = ldg4(tp), b = ldg4(tp + 1), c = ldg4(tp + 2);
    const V3 e1 = mk(b.x, b.y, b.z), e2 = mk(c.x, c.y, c.z);
    const V3 ng = normalize(cross(e1, e2));
    x.n = dot(ng, P.d) < 0.0f ? ng : ng * -1.0f;
    x.vid[0] = __float_as_int(a.w);
    x.vid[1] = __float_as_int(b.w);
    x.vid[2] = __float_as_int(c.w);
    x.bu = x.bv = 0.0f;
    if (S.layout == JSO_LAYOUT_VERTEX) {
      // barycentrics of the hit point: Moller-Trumbore's (u, v) from the point
      // itself along the ray direction, clamped into the triangle
      const V3 pv = cross(P.d, e2);
      const float inv = 1.0f / dot(e1, pv);
      const V3 sv = x.p - mk(a.x, a.y, a.z);
      float bu = fmaxf(dot(sv, pv) * inv, 0.0f);
      float bv = fmaxf(dot(P.d, cross(sv, e1)) * inv, 0.0f);
      const float sum = bu + bv;
      if (sum > 1.0f) {
        bu /= sum;
        bv /= sum;
      }
      x.bu = bu;
      x.bv = bv;
    }
  } else {
    x.n = normalize(x.p - ld3(S.sph[x.obj]));
  }
  const V3 p = x.p, n = x.n;
  const V3 wo = mk(-P.d.x, -P.d.y, -P.d.z);
  Mat M, Mb;
  vg.valid = material_at<kMesh>(S, params, x, M, vg.fp);
  if constexpr (kTwo) {
    Footprint fpb;
    material_at<kMesh>(S, params_b, x, Mb, fpb);
  }
  vg.j = j;
  // kTwo: the second ledger's gradient is summed apart and subtracted at the
  // end, so equal parameter vectors give an exactly zero difference
  float gb[5];
  if (kGrad) {
#pragma unroll
    for (int b = 0; b < 5; ++b) vg.g[b] = gb[b] = 0.0f;
  }
  const V3 po = p + n * kRayEps;
  float u[4];

  // next-event estimation towards the square light
  if (S.light_enabled && !(flags & JSO_F_NO_NEE)) {
    rng.draw((uint32_t)j, 1, u);
    const V3 lp = mk(S.lc[0] + (2.0f * u[0] - 1.0f) * S.lhalf, S.lc[1],
                     S.lc[2] + (2.0f * u[1] - 1.0f) * S.lhalf);
    const V3 dl = lp - p;
    const float dist2 = dot(dl, dl), dist = sqrtf(dist2);
    const V3 wl = dl * (1.0f / dist);
    const float cos_l = wl.y, cos_s = dot(n, wl);
    if (cos_l > 0.0f && cos_s > 0.0f &&
        !traced_occluded<kMesh, kRec>(S, st, po, wl, dist - kShadowEps, hr, j - 1, P.hit,
                                      P.rec_ok)) {
      Bsdf nb;
      eval_bsdf<kGrad>(M, n, wo, wl, flags, nb);
      const float pl = dist2 / (cos_l * S.larea);
      const float wmis = pl / (pl + nb.pdf);
      Bsdf nbb;
      if constexpr (kTwo) eval_bsdf<kGrad>(Mb, n, wo, wl, flags, nbb);
#pragma unroll
      for (int k = 0; k < 3; ++k) {
        const float K = cos_s * S.Le[k] * wmis / pl;
        const float term = P.beta[k] * nb.f[k] * K;
        P.led[k] += kGrad ? -(double)term : (double)term;
        if (kGrad) {
          const float coef = adj[k] * P.beta[k] * K;
          vg.g[k] += coef * nb.dc[k];
          vg.g[3] += coef * nb.dm[k];
          vg.g[4] += coef * nb.dr[k];
        }
        if constexpr (kTwo) {
          const float tb = L2.beta[k] * nbb.f[k] * K;
          L2.led[k] += kGrad ? -(double)tb : (double)tb;
          if (kGrad) {
            const float coef = adj_b[k] * L2.beta[k] * K;
            gb[k] += coef * nbb.dc[k];
            gb[3] += coef * nbb.dm[k];
            gb[4] += coef * nbb.dr[k];
          }
        }
      }
    }
  }

  // continuation
  rng.draw((uint32_t)j, 0, u);
  const V3 wi = sample_dir(M, n, wo, u, flags);
  const float ci = dot(n, wi);
  bool go = ci > 0.0f;
  Bsdf cb;
  float q = 1.0f;
  if (go) {
    eval_bsdf<kGrad>(M, n, wo, wi, flags, cb);
    go = cb.pdf > 0.0f;
  }
  if (go && S.rr_start > 0 && j >= S.rr_start) {
    if (u[3] >= S.rr_q) go = false;
    q = S.rr_q;
  }
  if (!go) {
    if constexpr (kTwo && kGrad) {
#pragma unroll
      for (int b = 0; b < 5; ++b) vg.g[b] -= gb[b];
    }
    P.alive = false;
    return;
  }
  const float cw = ci / (cb.pdf * q);
  Bsdf cbb;
  if constexpr (kTwo) eval_bsdf<kGrad>(Mb, n, wo, wi, flags, cbb);
  if (kGrad) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      if (cb.f[k] > 0.0f) {
        const float R = (float)P.led[k];
        const float coef = adj[k] * R / cb.f[k];
        vg.g[k] += coef * cb.dc[k];
        vg.g[3] += coef * cb.dm[k];
        vg.g[4] += coef * cb.dr[k];
      }
      if constexpr (kTwo) {
        if (cbb.f[k] > 0.0f) {
          const float R = (float)L2.led[k];
          const float coef = adj_b[k] * R / cbb.f[k];
          gb[k] += coef * cbb.dc[k];
          gb[3] += coef * cbb.dm[k];
          gb[4] += coef * cbb.dr[k];
        }
      }
    }
    if constexpr (kTwo) {
#pragma unroll
      for (int b = 0; b < 5; ++b) vg.g[b] -= gb[b];
    }
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    P.beta[k] *= cb.f[k] * cw;
    if constexpr (kTwo) L2.beta[k] *= cbb.f[k] * cw;
  }
  P.d = wi;
  const Hit h = traced_hit<kMesh, false, kRec>(S, st, po, wi, hr, rng, j, P.rec_ok);
  P.o = po + wi * h.t;
  if (h.kind == HIT_NONE) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double e = (double)(P.beta[k] * S.env[k]);
      P.led[k] += kGrad ? -e : e;
      if constexpr (kTwo) {
        const double eb = (double)(L2.beta[k] * S.env[k]);
        L2.led[k] += kGrad ? -eb : eb;
      }
    }
    P.alive = false;
  } else if (h.kind == HIT_LIGHT) {
    const float pl = h.t * h.t / (wi.y * S.larea);
    const float wb = (flags & JSO_F_NO_NEE) ? 1.0f : cb.pdf / (cb.pdf + pl);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      const double e = (double)(P.beta[k] * (S.Le[k] * wb));
      P.led[k] += kGrad ? -e : e;
      if constexpr (kTwo) {
        const double eb = (double)(L2.beta[k] * (S.Le[k] * wb));
        L2.led[k] += kGrad ? -eb : eb;
      }
    }
    P.alive = false;
  } else {
    P.alive = j < S.depth;
    P.set_hit(h.kind, h.obj, j + 1);
  }
}

template <bool kGrad, bool kMesh, int kRec = REC_NONE>
__device__ __forceinline__ void path_vertex(const DevScene& S, const TravStack& st,
                                            const float* __restrict__ params, const Rng& rng,
                                            uint32_t flags, Path& P, const float adj[3],
                                            VertexGrad& vg,
                                            const HitRecs& hr = HitRecs{nullptr, 0, 0}) {
  Ledger2 unused;
  path_vertex2<kGrad, kMesh, false, kRec>(S, st, params, nullptr, rng, flags, P, unused, adj,
                                          nullptr, vg, hr);
}

}  // namespace jso
