"""Seeded synthetic inputs shared by the HIP path and the FP64 oracle.

This module only *describes* scenes and draws the random numbers that define
them (sphere placement, texture values, ground-truth and initial parameters,
synthetic target images for parity cases). It holds none of the method's
arithmetic: no ray tracing, no shading, no gradients, no optimiser. Both the
product binding and the oracle's binding marshal a ``SceneSpec`` into their
own native structs.

The paper's scenes (Banner, Potted Plant, Veach Ajar, ...) are not available;
these synthetic scenes stand in for its multivariate-material experiment
(base colour, metalness, roughness; teaser figure and the "Multivariate
optimisation" paragraph of the Experiments section) and its texture
optimisation experiment ("Texture optimisation" paragraph).

Parameter layout (shared contract): a parameterised material is a texture of
``tex_h x tex_w`` texels, texel-interleaved, each texel holding the enabled
channels of (R, G, B, metalness, roughness) in that order, so parameter
``(y * tex_w + x) * n_ch + c``.  A 1x1 texture is a "global" material.  The
plane and a triangle mesh map the texture by planar UV over the plane's
extent; spheres by latitude-longitude.  With ``param_layout = LAYOUT_VERTEX``
the parameters belong to the mesh vertices instead (``v * n_ch + c``),
interpolated barycentrically; only the mesh may then be parameterised.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Tuple

import numpy as np

# channel bits of the parameterised material
CH_R, CH_G, CH_B, CH_M, CH_ROUGH = 1, 2, 4, 8, 16
CH_ALL = CH_R | CH_G | CH_B | CH_M | CH_ROUGH
CH_RGB_ROUGH = CH_R | CH_G | CH_B | CH_ROUGH

# lower/upper box of each channel (projection after every step)
ROUGH_MIN = 0.05
CHANNEL_BOUNDS = {CH_R: (0.0, 1.0), CH_G: (0.0, 1.0), CH_B: (0.0, 1.0),
                  CH_M: (0.0, 1.0), CH_ROUGH: (ROUGH_MIN, 1.0)}

MAT_PARAM = -1  # object uses the parameterised (textured / global) material

LAYOUT_TEXTURE, LAYOUT_VERTEX, LAYOUT_VOLUME = 0, 1, 2
# a volume's four channels per voxel: emission R, G, B and density (the bits of
# R, G, B and metalness; all in [0, 1])
CH_VOLUME = CH_R | CH_G | CH_B | CH_M


@dataclasses.dataclass
class SceneSpec:
    width: int
    height: int
    cam_eye: Tuple[float, float, float] = (0.0, 2.0, 6.0)
    cam_target: Tuple[float, float, float] = (0.0, 0.8, 0.0)
    cam_up: Tuple[float, float, float] = (0.0, 1.0, 0.0)
    vfov_deg: float = 40.0
    plane_enabled: bool = True
    plane_mat: int = MAT_PARAM
    plane_extent: Tuple[float, float, float, float] = (-5.0, 5.0, -5.0, 5.0)  # x0,x1,z0,z1 (UV)
    spheres: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 4)))  # cx,cy,cz,r
    sphere_mat: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0,), np.int32))
    light_enabled: bool = True
    light_center: Tuple[float, float, float] = (1.5, 5.0, 1.5)
    light_side: float = 1.0
    light_Le: Tuple[float, float, float] = (10.0, 10.0, 10.0)
    env: Tuple[float, float, float] = (1.0, 1.0, 1.0)
    depth: int = 3
    rr_start: int = 0          # 0 = no Russian roulette; else first vertex whose continuation is rouletted
    rr_q: float = 0.8          # survival probability (stored as float32 on both sides)
    tex_w: int = 1
    tex_h: int = 1
    ch_mask: int = CH_ALL
    # values of the parameterised material's channels that are not parameters
    fixed_default: Tuple[float, float, float, float, float] = (0.5, 0.5, 0.5, 0.0, 0.5)
    # fixed materials: rows of (R, G, B, metalness, roughness)
    fixed_mats: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 5)))
    # triangle mesh (optional)
    verts: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3)))
    tris: np.ndarray = dataclasses.field(default_factory=lambda: np.zeros((0, 3), np.int32))
    mesh_mat: int = MAT_PARAM
    param_layout: int = LAYOUT_TEXTURE
    # emission-absorption volume (param_layout LAYOUT_VOLUME): vol_res^3 voxels
    # in the cube of side vol_box[3] from corner vol_box[:3]; density scale
    # vol_sigma per unit length; the image stacks vol_views views (rows
    # height / vol_views each), view v's eye turned by 2 pi v / vol_views about
    # the vertical axis through cam_target
    vol_res: int = 0
    vol_views: int = 1
    vol_box: Tuple[float, float, float, float] = (-1.0, 0.0, -1.0, 2.0)
    vol_sigma: float = 8.0

    @property
    def n_ch(self) -> int:
        return bin(self.ch_mask).count("1")

    @property
    def n_elems(self) -> int:
        """Texels, mesh vertices in the per-vertex layout, or voxels."""
        if self.param_layout == LAYOUT_VOLUME:
            return self.vol_res ** 3
        if self.param_layout == LAYOUT_VERTEX:
            return int(np.asarray(self.verts).reshape(-1, 3).shape[0])
        return self.tex_w * self.tex_h

    @property
    def n_params(self) -> int:
        return self.n_elems * self.n_ch

    @property
    def n_pixels(self) -> int:
        return self.width * self.height

    def channel_bits(self) -> List[int]:
        return [b for b in (CH_R, CH_G, CH_B, CH_M, CH_ROUGH) if self.ch_mask & b]

    def param_bounds(self) -> Tuple[np.ndarray, np.ndarray]:
        """Per-parameter (lo, hi) boxes in the texel-interleaved layout."""
        bits = self.channel_bits()
        lo = np.array([CHANNEL_BOUNDS[b][0] for b in bits], np.float32)
        hi = np.array([CHANNEL_BOUNDS[b][1] for b in bits], np.float32)
        n = self.n_elems
        return np.tile(lo, n), np.tile(hi, n)


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(seed))


# ----------------------------------------------------------------------------
# texture family: smooth random-Fourier fields
# ----------------------------------------------------------------------------
def random_fourier_field(h: int, w: int, g: np.random.Generator, n_terms: int = 8,
                         lo: float = 0.1, hi: float = 0.9) -> np.ndarray:
    """T(u,v) = mid + half * tanh(sum_k a_k sin(2 pi (f_k . (u, v)) + phi_k)).

    a_k ~ N(0, 0.5^2), integer frequencies f_k in {1..4}^2, phi_k ~ U[0, 2 pi).
    Sampled at texel centres; values lie strictly inside (lo, hi).
    """
    a = g.normal(0.0, 0.5, n_terms)
    f = g.integers(1, 5, size=(n_terms, 2))
    phi = g.uniform(0.0, 2 * math.pi, n_terms)
    u = (np.arange(w) + 0.5) / w
    v = (np.arange(h) + 0.5) / h
    U, V = np.meshgrid(u, v)
    s = np.zeros((h, w))
    for k in range(n_terms):
        s += a[k] * np.sin(2 * math.pi * (f[k, 0] * U + f[k, 1] * V) + phi[k])
    mid, half = 0.5 * (lo + hi), 0.5 * (hi - lo)
    return (mid + half * np.tanh(s)).astype(np.float32)


def fourier_params(spec: SceneSpec, seed: int, lo: float = 0.1, hi: float = 0.9) -> np.ndarray:
    """A texel-interleaved parameter vector with one random-Fourier field per channel."""
    g = rng(seed)
    chans = [random_fourier_field(spec.tex_h, spec.tex_w, g, lo=lo, hi=hi)
             for _ in range(spec.n_ch)]
    return np.stack(chans, axis=-1).reshape(-1).astype(np.float32)


def uniform_params(spec: SceneSpec, seed: int, lo: float, hi: float) -> np.ndarray:
    g = rng(seed)
    return g.uniform(lo, hi, spec.n_params).astype(np.float32)


# ----------------------------------------------------------------------------
# scenes
# ----------------------------------------------------------------------------
PLANE_GREY = np.array([[0.6, 0.6, 0.6, 0.0, 0.8]])


def scene_tiny(width: int = 64, height: int = 64) -> SceneSpec:
    """Unit sphere at (0,1,0) on the plane y=0; uniform environment 1.0 and the
    square area light; depth 3, no roulette; 5 global material parameters on
    the sphere (R, G, B, metalness, roughness); fixed grey plane."""
    return SceneSpec(width=width, height=height,
                     spheres=np.array([[0.0, 1.0, 0.0, 1.0]]),
                     sphere_mat=np.array([MAT_PARAM], np.int32),
                     plane_mat=0, fixed_mats=PLANE_GREY.copy(),
                     depth=3, rr_start=0, tex_w=1, tex_h=1, ch_mask=CH_ALL)


def place_spheres(n: int, g: np.random.Generator, rmin=0.3, rmax=1.0,
                  xr=(-3.0, 3.0), zr=(-3.0, 2.0), gap=0.05) -> np.ndarray:
    """n spheres resting on y=0 with radii U[rmin,rmax], non-overlapping (rejection)."""
    out = []
    tries = 0
    while len(out) < n:
        tries += 1
        if tries > 100000:
            raise RuntimeError("sphere placement failed")
        r = g.uniform(rmin, rmax)
        x = g.uniform(*xr)
        z = g.uniform(*zr)
        ok = all((x - s[0]) ** 2 + (z - s[2]) ** 2 > (r + s[3] + gap) ** 2 for s in out)
        if ok:
            out.append((x, r, z, r))
    return np.array(out, np.float64)


def scene_textured(width: int = 512, height: int = 512, tex: int = 256, seed: int = 0,
                   n_spheres: int = 8, depth: int = 6, rr_start: int = 3,
                   rmin: float = 0.3, rmax: float = 1.0) -> SceneSpec:
    """Plane + n spheres (radii U[0.3,1], seeded non-overlapping positions); all
    objects share one texture of base colour RGB + roughness (metalness fixed 0)."""
    g = rng(seed)
    sph = place_spheres(n_spheres, g, rmin, rmax)
    return SceneSpec(width=width, height=height, spheres=sph,
                     sphere_mat=np.full((n_spheres,), MAT_PARAM, np.int32),
                     plane_mat=MAT_PARAM, depth=depth, rr_start=rr_start,
                     tex_w=tex, tex_h=tex, ch_mask=CH_RGB_ROUGH,
                     fixed_default=(0.5, 0.5, 0.5, 0.0, 0.5))


def scene_white_furnace(width: int = 16, height: int = 16) -> SceneSpec:
    """Unit sphere alone in a uniform environment of radiance 1 (no plane, no light).
    With an albedo-1 Lambertian sphere every path returns exactly 1."""
    return SceneSpec(width=width, height=height, plane_enabled=False, light_enabled=False,
                     spheres=np.array([[0.0, 1.0, 0.0, 1.0]]),
                     sphere_mat=np.array([MAT_PARAM], np.int32),
                     depth=4, tex_w=1, tex_h=1, ch_mask=CH_ALL)


def target_image_synthetic(spec: SceneSpec, seed: int) -> np.ndarray:
    """A seeded stand-in target image (H, W, 3) for parity cases: values U[0, 1.5]."""
    g = rng(seed)
    return g.uniform(0.0, 1.5, (spec.height, spec.width, 3)).astype(np.float32)


def config_tiny(seed_gt: int = 1, seed_init: int = 2):
    """64x64 tiny problem: scene, ground-truth and initial global parameters ~U[0.1,0.9]."""
    s = scene_tiny()
    return s, uniform_params(s, seed_gt, 0.1, 0.9), uniform_params(s, seed_init, 0.1, 0.9)


def config_textured(seed_scene: int = 0, seed_gt: int = 1, seed_init: int = 2,
                    width: int = 512, height: int = 512, tex: int = 256):
    """512x512 textured problem: 256x256 base-colour + roughness texture (262,144 params);
    ground truth = random-Fourier textures; initial texels ~U[0.2,0.8]."""
    s = scene_textured(width, height, tex, seed_scene)
    return s, fourier_params(s, seed_gt), uniform_params(s, seed_init, 0.2, 0.8)


# ----------------------------------------------------------------------------
# triangle meshes
# ----------------------------------------------------------------------------
def smooth_field_3d(p: np.ndarray, g: np.random.Generator, n_terms: int = 8) -> np.ndarray:
    """The random-Fourier family in 3-D: tanh(sum_k a_k sin(2 pi f_k . p + phi_k)),
    a_k ~ N(0, 0.5^2), integer f_k in {1..3}^3, phi_k ~ U[0, 2 pi); values in (-1, 1)."""
    a = g.normal(0.0, 0.5, n_terms)
    f = g.integers(1, 4, size=(n_terms, 3))
    phi = g.uniform(0.0, 2 * math.pi, n_terms)
    s = np.zeros(p.shape[0])
    for k in range(n_terms):
        s += a[k] * np.sin(2 * math.pi * (p @ f[k]) + phi[k])
    return np.tanh(s)


def icosphere(freq: int, center=(0.0, 1.2, 0.0), radius: float = 1.0, disp: float = 0.1,
              seed: int = 0):
    """Geodesic sphere: each icosahedron face split into freq^2 triangles
    (20 freq^2 triangles, 10 freq^2 + 2 vertices), projected to the sphere and
    displaced radially by radius * disp * (smooth field of the direction).
    Triangles wind counter-clockwise seen from outside."""
    t = (1.0 + math.sqrt(5.0)) / 2.0
    ico_v = np.array([[-1, t, 0], [1, t, 0], [-1, -t, 0], [1, -t, 0], [0, -1, t], [0, 1, t],
                      [0, -1, -t], [0, 1, -t], [t, 0, -1], [t, 0, 1], [-t, 0, -1], [-t, 0, 1]],
                     np.float64)
    ico_f = [(0, 11, 5), (0, 5, 1), (0, 1, 7), (0, 7, 10), (0, 10, 11), (1, 5, 9), (5, 11, 4),
             (11, 10, 2), (10, 7, 6), (7, 1, 8), (3, 9, 4), (3, 4, 2), (3, 2, 6), (3, 6, 8),
             (3, 8, 9), (4, 9, 5), (2, 4, 11), (6, 2, 10), (8, 6, 7), (9, 8, 1)]
    index = {}
    verts = []

    def vid(face, a, b):
        # point a/f along edge (0->1) and b/f along (0->2) of the face; keyed by
        # its corner weights so points on shared edges are shared
        c = freq - a - b
        key = tuple(sorted((ci, w) for ci, w in zip(face, (c, a, b)) if w > 0))
        if key not in index:
            index[key] = len(verts)
            p = sum(w * ico_v[ci] for ci, w in key) / freq
            verts.append(p / np.linalg.norm(p))
        return index[key]

    tris = []
    for face in ico_f:
        for a in range(freq):
            for b in range(freq - a):
                v00, v10, v01 = vid(face, a, b), vid(face, a + 1, b), vid(face, a, b + 1)
                tris.append((v00, v10, v01))
                if a + b < freq - 1:
                    tris.append((v10, vid(face, a + 1, b + 1), v01))
    d = np.array(verts)
    r = radius * (1.0 + disp * smooth_field_3d(d, rng(seed)))
    v = np.asarray(center) + d * r[:, None]
    return v, np.array(tris, np.int32)


def heightfield(n: int, extent=(-5.0, 5.0, -5.0, 5.0), amp: float = 0.4, seed: int = 0,
                octaves: int = 1):
    """n x n quads (2 n^2 triangles) over the plane extent.  Height
    amp * (1 + f(x, z)) >= 0 with f the smooth field of the normalised (x, z);
    with octaves > 1, a fractal sum: octave o adds 0.5^o f_o(2^o (x, z)) of
    its own random field, and the sum is rescaled into (-1, 1)."""
    x0, x1, z0, z1 = extent
    xs, zs = np.linspace(x0, x1, n + 1), np.linspace(z0, z1, n + 1)
    X, Z = np.meshgrid(xs, zs)
    pts = np.stack([(X - x0) / (x1 - x0), np.zeros_like(X), (Z - z0) / (z1 - z0)], -1).reshape(-1, 3)
    Y = amp * (1.0 + fbm_field(pts, seed, octaves))
    v = np.stack([X.reshape(-1), Y, Z.reshape(-1)], -1)
    idx = np.arange((n + 1) * (n + 1)).reshape(n + 1, n + 1)
    a, b, c, d = idx[:-1, :-1], idx[:-1, 1:], idx[1:, :-1], idx[1:, 1:]
    tris = np.concatenate([np.stack([a, c, b], -1).reshape(-1, 3),
                           np.stack([b, c, d], -1).reshape(-1, 3)])
    return v, tris.astype(np.int32)


def fbm_field(p: np.ndarray, seed: int, octaves: int = 1) -> np.ndarray:
    """Fractal sum of smooth fields (octave o: weight 0.5^o, frequency 2^o),
    in (-1, 1); one octave is the smooth field itself."""
    g = rng(seed)
    if octaves == 1:
        return smooth_field_3d(p, g)
    s = np.zeros(p.shape[0])
    w = 0.0
    for o in range(octaves):
        s += 0.5 ** o * smooth_field_3d(p * 2.0 ** o, g)
        w += 0.5 ** o
    return s / w


def terrain_height(spec_extent, amp: float, seed: int, octaves: int, x, z):
    """Height of the heightfield surface (before triangulation) at (x, z)."""
    x0, x1, z0, z1 = spec_extent
    pts = np.stack([(np.asarray(x) - x0) / (x1 - x0), np.zeros_like(np.asarray(x, float)),
                    (np.asarray(z) - z0) / (z1 - z0)], -1).reshape(-1, 3)
    return amp * (1.0 + fbm_field(pts, seed, octaves))


def vertex_fourier_params(spec: SceneSpec, seed: int, lo: float = 0.1, hi: float = 0.9):
    """Per-vertex parameters: one smooth field of the vertex position per channel."""
    g = rng(seed)
    v = np.asarray(spec.verts).reshape(-1, 3)
    chans = [lo + (hi - lo) * 0.5 * (1.0 + smooth_field_3d(v * 0.5, g)) for _ in range(spec.n_ch)]
    return np.stack(chans, -1).reshape(-1).astype(np.float32)


def scene_mesh_sphere(width: int = 1024, height: int = 1024, freq: int = 100, seed: int = 0,
                      depth: int = 8, rr_start: int = 3) -> SceneSpec:
    """A displaced geodesic sphere (20 freq^2 triangles) on a fixed grey plane,
    with per-vertex base colour RGB + roughness parameters (metalness 0)."""
    v, t = icosphere(freq, seed=seed)
    return SceneSpec(width=width, height=height, plane_mat=0, fixed_mats=PLANE_GREY.copy(),
                     verts=v, tris=t, mesh_mat=MAT_PARAM, param_layout=LAYOUT_VERTEX,
                     depth=depth, rr_start=rr_start, ch_mask=CH_RGB_ROUGH,
                     fixed_default=(0.5, 0.5, 0.5, 0.0, 0.5))


def scene_terrain(width: int = 2048, height: int = 2048, n: int = 707, n_spheres: int = 32,
                  tex: int = 512, seed: int = 0, depth: int = 12, rr_start: int = 3,
                  amp: float = 0.4, octaves: int = 5) -> SceneSpec:
    """Large scene: a fractal heightfield terrain of 2 n^2 triangles over the
    plane extent (the plane itself disabled) and n_spheres spheres (radii
    U[0.15, 0.45], non-overlapping, resting on the terrain); all share one
    tex x tex texture of all five channels (RGB, metalness, roughness), mapped
    to the terrain by planar UV and to the spheres by latitude-longitude."""
    v, t = heightfield(n, amp=amp, seed=seed, octaves=octaves)
    g = rng(seed + 1)
    sph = place_spheres(n_spheres, g, 0.15, 0.45, xr=(-4.0, 4.0), zr=(-4.0, 3.0))
    ext = SceneSpec(width=1, height=1).plane_extent
    sph[:, 1] = terrain_height(ext, amp, seed, octaves, sph[:, 0], sph[:, 2]) + sph[:, 3]
    return SceneSpec(width=width, height=height, plane_enabled=False, verts=v, tris=t,
                     mesh_mat=MAT_PARAM, spheres=sph,
                     sphere_mat=np.full((n_spheres,), MAT_PARAM, np.int32), depth=depth,
                     rr_start=rr_start, tex_w=tex, tex_h=tex, ch_mask=CH_ALL)


def config_large(seed_scene: int = 0, seed_gt: int = 1, seed_init: int = 2, **kw):
    """2048 x 2048 terrain problem: 1.0M-triangle terrain + 32 spheres, a
    512 x 512 texture of 5 channels (1,310,720 parameters); ground truth =
    random-Fourier textures, initial texels ~U[0.2, 0.8]."""
    s = scene_terrain(seed=seed_scene, **kw)
    return s, fourier_params(s, seed_gt), uniform_params(s, seed_init, 0.2, 0.8)


def config_batched(n: int = 64, seed: int = 0):
    """Many independent problems of uneven size: image side = multiple of 8
    nearest 64 * 8^U (64..512), parameter count P = round(5 * 13107^U)
    (5..65,536): P <= 5 is the global material (5 parameters, unit sphere on a
    grey plane, depth 3), otherwise a plane + spheres scene sharing one square
    texture of RGB + roughness with side ceil(sqrt(P / 4)) (depth 6, roulette
    from vertex 3).  Iteration budget ~ U{200..1000}; each problem has its own
    scene, ground truth, initial parameters and optimisation seed.
    Returns a list of dicts (spec, gt, init, max_iter, seed)."""
    g = rng(seed)
    out = []
    for k in range(n):
        side = int(round(64 * 8 ** g.uniform() / 8.0)) * 8
        side = min(max(side, 64), 512)
        P = int(round(5 * 13107 ** g.uniform()))
        max_iter = int(g.integers(200, 1001))
        sub = int(g.integers(0, 2 ** 31))
        if P <= 5:
            s = scene_tiny()
            s.width = s.height = side
            gt, init = uniform_params(s, sub + 1, 0.1, 0.9), uniform_params(s, sub + 2, 0.1, 0.9)
        else:
            tex = int(np.ceil(np.sqrt(P / 4.0)))
            s = scene_textured(side, side, tex, seed=sub, n_spheres=int(g.integers(1, 9)))
            gt, init = fourier_params(s, sub + 1), uniform_params(s, sub + 2, 0.2, 0.8)
        out.append(dict(spec=s, gt=gt, init=init, max_iter=max_iter, seed=sub))
    return out


# ----------------------------------------------------------------------------
# emission-absorption volume (the volume experiment of the paper)
# ----------------------------------------------------------------------------
def scene_volume(res: int = 256, views: int = 8, view_w: int = 256, view_h: int = 256,
                 sigma: float = 8.0) -> SceneSpec:
    """A res^3 emission-absorption volume in the cube [-1, 1] x [0, 2] x [-1, 1]
    seen by `views` cameras on a circle around it (eye 4.5 from the axis,
    slightly above the centre, vFOV 40 degrees); environment radiance 0.2;
    no surfaces or lights."""
    return SceneSpec(width=view_w, height=view_h * views, cam_eye=(0.0, 1.9, 4.5),
                     cam_target=(0.0, 1.0, 0.0), vfov_deg=40.0, plane_enabled=False,
                     light_enabled=False, env=(0.2, 0.2, 0.2), depth=1, ch_mask=CH_VOLUME,
                     param_layout=LAYOUT_VOLUME, vol_res=res, vol_views=views,
                     vol_box=(-1.0, 0.0, -1.0, 2.0), vol_sigma=sigma)


def volume_blobs(spec: SceneSpec, seed: int, n_blobs: int = 12) -> np.ndarray:
    """Ground-truth volume: the sum of seeded Gaussian blobs (centres in the
    inner 70% of the cube, radii 6-20% of its side) carrying the density and,
    weighted by it, each blob's colour; clipped to [0, 1].  Layout
    ((z R + y) R + x) * 4 + (R, G, B, density), float32."""
    g = rng(seed)
    R = spec.vol_res
    c = (np.arange(R) + 0.5) / R
    z, y, x = np.meshgrid(c, c, c, indexing="ij")
    dens = np.zeros((R, R, R))
    col = np.zeros((R, R, R, 3))
    for _ in range(n_blobs):
        ctr = g.uniform(0.15, 0.85, 3)
        rad = g.uniform(0.06, 0.2)
        amp = g.uniform(0.4, 1.0)
        rgb = g.uniform(0.1, 1.0, 3)
        b = amp * np.exp(-((x - ctr[0]) ** 2 + (y - ctr[1]) ** 2 + (z - ctr[2]) ** 2) /
                         (2 * rad * rad))
        dens += b
        col += b[..., None] * rgb
    col = col / np.maximum(dens[..., None], 1e-6)
    out = np.concatenate([np.clip(col, 0, 1), np.clip(dens, 0, 1)[..., None]], axis=-1)
    return out.reshape(-1).astype(np.float32)


def volume_uniform(spec: SceneSpec, emission: float = 0.5, density: float = 0.05) -> np.ndarray:
    """A constant volume (the usual starting point of a volume fit)."""
    v = np.empty((spec.vol_res ** 3, 4), np.float32)
    v[:, :3] = emission
    v[:, 3] = density
    return v.reshape(-1)


def config_volume(res: int = 256, views: int = 8, view_w: int = 256, view_h: int = 256,
                  seed_gt: int = 1):
    """The volume workload: (spec, ground truth, initial parameters)."""
    spec = scene_volume(res, views, view_w, view_h)
    return spec, volume_blobs(spec, seed_gt), volume_uniform(spec)
