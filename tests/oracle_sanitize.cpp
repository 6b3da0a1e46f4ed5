// Drives every entry point of the FP64 oracle on small scenes of each kind
// (analytic, textured, triangle mesh in both parameter layouts, volume), for a
// build with AddressSanitizer and UndefinedBehaviorSanitizer.  Prints "ok" and
// a checksum; any out-of-bounds access, use of freed memory or undefined
// arithmetic aborts with the sanitizer's report.
#include <cmath>
#include <cstdio>
#include <cstring>
#include <vector>

#include "oracle.h"

namespace {

orc_scene base_scene(int w, int h) {
  orc_scene s;
  std::memset(&s, 0, sizeof(s));
  s.width = w;
  s.height = h;
  const double eye[3] = {0.0, 2.0, 6.0}, tgt[3] = {0.0, 0.8, 0.0}, up[3] = {0.0, 1.0, 0.0};
  std::memcpy(s.cam_eye, eye, sizeof(eye));
  std::memcpy(s.cam_target, tgt, sizeof(tgt));
  std::memcpy(s.cam_up, up, sizeof(up));
  s.vfov_deg = 40.0;
  s.plane_enabled = 1;
  s.plane_mat = -1;
  const double ext[4] = {-5.0, 5.0, -5.0, 5.0};
  std::memcpy(s.plane_extent, ext, sizeof(ext));
  s.light_enabled = 1;
  const double lc[3] = {1.5, 5.0, 1.5}, le[3] = {10.0, 10.0, 10.0}, env[3] = {1.0, 1.0, 1.0};
  std::memcpy(s.light_center, lc, sizeof(lc));
  s.light_side = 1.0;
  std::memcpy(s.light_Le, le, sizeof(le));
  std::memcpy(s.env, env, sizeof(env));
  s.depth = 5;
  s.rr_start = 2;
  s.rr_q = 0.8;
  s.tex_w = s.tex_h = 1;
  s.ch_mask = 31;
  const double fd[5] = {0.5, 0.5, 0.5, 0.0, 0.5};
  std::memcpy(s.fixed_default, fd, sizeof(fd));
  s.vol_views = 1;
  return s;
}

int n_params(const orc_scene& s) {
  int nch = 0;
  for (int b = 0; b < 5; ++b) nch += (s.ch_mask >> b) & 1;
  if (s.param_layout == 2) return s.vol_res * s.vol_res * s.vol_res * nch;
  if (s.param_layout == 1) return s.n_verts * nch;
  return s.tex_w * s.tex_h * nch;
}

double run_all(const orc_scene& s, int flags) {
  const int P = n_params(s), npix = s.width * s.height;
  std::vector<double> p(P), p2(P), img(3 * npix), mg(npix), tgt(3 * npix), g(P), ga(P),
      aimg(3 * npix), dimg(3 * npix);
  for (int i = 0; i < P; ++i) {
    p[i] = 0.2 + 0.6 * std::fmod(0.618 * (i + 1), 1.0);
    p2[i] = std::fmin(p[i] + 0.03, 1.0);
  }
  for (int i = 0; i < 3 * npix; ++i) {
    tgt[i] = 0.7 * std::fmod(0.37 * (i + 3), 1.0);
    dimg[i] = tgt[i] - 0.35;
  }
  std::vector<unsigned char> mask(npix, 0);
  mask[0] = 1;
  const int crop[4] = {1, 1, s.width - 1, s.height - 1};
  double sum = 0.0;
  if (orc_render(&s, p.data(), 7, 2, 8, 2, flags, nullptr, img.data(), mg.data(), 2)) return NAN;
  for (double v : img) sum += v;
  if (orc_render_sampled(&s, p.data(), p2.data(), 7, 2, 8, 1, flags, crop, img.data(),
                         mg.data(), 1))
    return NAN;
  if (orc_grad(&s, p.data(), 7, 2, 2, 3, 2, tgt.data(), flags, nullptr, mask.data(), g.data(),
               ga.data(), img.data(), mg.data(), aimg.data(), 2))
    return NAN;
  for (double v : g) sum += v;
  if (orc_grad_sampled(&s, p.data(), p2.data(), 7, 3, 4, 5, 1, tgt.data(), flags | 16, crop,
                       nullptr, g.data(), ga.data(), nullptr, nullptr, nullptr, 1))
    return NAN;
  for (double v : ga) sum += v;
  if (orc_render_bwd(&s, p.data(), 7, 2, 8, 1, dimg.data(), flags, crop, nullptr, g.data(),
                     ga.data(), mg.data(), aimg.data(), 2))
    return NAN;
  if (orc_render_bwd_sampled(&s, p2.data(), p.data(), 7, 2, 8, 1, dimg.data(), flags, nullptr,
                             mask.data(), g.data(), ga.data(), nullptr, nullptr, 1))
    return NAN;
  for (double v : g) sum += v;
  return sum;
}

}  // namespace

int main() {
  double total = 0.0;
  // random numbers and the BSDF
  const uint32_t ctr[4] = {1, 2, 3, 4}, key[2] = {5, 6};
  uint32_t out[4];
  orc_philox4x32_10(ctr, key, out);
  total += out[0] * 1e-9 + (double)(orc_stream_key(3, 4, 5) >> 40);
  const double mat[5] = {0.3, 0.6, 0.9, 0.4, 0.2}, n[3] = {0, 1, 0}, wo[3] = {0.6, 0.8, 0.0};
  const double wis[6] = {0.0, 1.0, 0.0, -0.6, 0.8, 0.0};
  double bs[26];
  orc_bsdf_many(2, mat, n, wo, wis, 0, bs);
  orc_bsdf(mat, n, wo, wis, 2, bs);
  total += bs[0];
  orc_reset_stats();
  // analytic: unit sphere with the global material on a fixed plane
  orc_scene s = base_scene(9, 7);
  const double sph[4] = {0.0, 1.0, 0.0, 1.0};
  const int sphm[1] = {-1};
  const double fixed[5] = {0.6, 0.6, 0.6, 0.0, 0.8};
  s.n_spheres = 1;
  s.spheres = sph;
  s.sphere_mat = sphm;
  s.plane_mat = 0;
  s.n_fixed = 1;
  s.fixed_mats = fixed;
  for (int flags : {0, 1, 2, 4, 8}) total += run_all(s, flags);
  // textured: plane + two spheres sharing a 5 x 4 texture of all channels
  const double sph2[8] = {-1.0, 0.5, 0.0, 0.5, 1.0, 0.7, -0.5, 0.7};
  const int sphm2[2] = {-1, -1};
  s = base_scene(11, 6);
  s.n_spheres = 2;
  s.spheres = sph2;
  s.sphere_mat = sphm2;
  s.tex_w = 5;
  s.tex_h = 4;
  total += run_all(s, 0);
  s.ch_mask = 1 | 2 | 4 | 16;
  total += run_all(s, 0);
  // triangle mesh: a tetrahedron floating over the plane, texture and per-vertex layouts
  const double verts[12] = {0, 1.5, 0, 1, 0.5, 0, -0.5, 0.5, 0.8, -0.5, 0.5, -0.8};
  const int tris[12] = {0, 1, 2, 0, 2, 3, 0, 3, 1, 1, 3, 2};
  s = base_scene(8, 8);
  s.n_verts = 4;
  s.n_tris = 4;
  s.verts = verts;
  s.tris = tris;
  s.mesh_mat = -1;
  s.tex_w = s.tex_h = 3;
  total += run_all(s, 0);
  s.param_layout = 1;
  s.plane_mat = 0;
  s.n_fixed = 1;
  s.fixed_mats = fixed;
  s.ch_mask = 1 | 2 | 4 | 16;
  total += run_all(s, 0);
  // emission-absorption volume, two views
  s = base_scene(6, 10);
  s.plane_enabled = 0;
  s.light_enabled = 0;
  s.param_layout = 2;
  s.ch_mask = 15;
  s.vol_res = 5;
  s.vol_views = 2;
  const double box[4] = {-1.0, 0.0, -1.0, 2.0};
  std::memcpy(s.vol_box, box, sizeof(box));
  s.vol_sigma = 8.0;
  s.depth = 1;
  s.rr_start = 0;
  total += run_all(s, 0);
  uint64_t st[3];
  orc_get_stats(st);
  if (!std::isfinite(total) || st[0] == 0) {
    std::printf("failed %g\n", total);
    return 1;
  }
  std::printf("ok %.6e %llu\n", total, (unsigned long long)st[0]);
  return 0;
}
