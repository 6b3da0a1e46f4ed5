"""Pins of the oracle's triangle meshes (CPU only).

The oracle intersects every triangle by brute force (Moller-Trumbore, two-sided
geometric normal).  Each pin compares it with something it shares no code
with:

* a flat triangle fan standing in for the analytic plane gives the same image
  and gradient, for either winding (two-sidedness);
* per-vertex parameters that are constant equal a 1x1 (global) material, and
  their gradients sum to the global one (barycentric weights sum to one);
* per-vertex parameters that are a linear function of position equal a 2x2
  bilinear texture holding the same function (barycentric weights reproduce
  linear fields, so a swapped weight fails);
* shadow rays are blocked by a floating mesh square: direct light on the plane
  matches 2-D quadrature of the light with the square's shadow written here;
* the adjoint of per-vertex parameters equals central differences at fixed
  random numbers (parameter-independent sampling).
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2309_15676_amd import inputs as I


def _fan(half: float, clockwise: bool = False, y: float = 0.0, cx: float = 0.0,
         cz: float = 0.0):
    """Four triangles sharing the centre (first vertex of each) of a square of
    side 2*half in the plane y; counter-clockwise seen from above unless
    clockwise."""
    v = np.array([[cx, y, cz], [cx - half, y, cz - half], [cx + half, y, cz - half],
                  [cx + half, y, cz + half], [cx - half, y, cz + half]])
    t = np.array([[0, 2, 1], [0, 3, 2], [0, 4, 3], [0, 1, 4]], np.int32)
    if clockwise:
        t = t[:, [0, 2, 1]]
    return v, t


def _plane_as_mesh(spec, clockwise=False):
    s = I.SceneSpec(**{f: getattr(spec, f) for f in spec.__dataclass_fields__})
    s.verts, s.tris = _fan(1e6, clockwise)
    s.mesh_mat = spec.plane_mat
    s.plane_enabled = False
    return s


def _scenes():
    tiny, gt, _ = I.config_tiny(seed_gt=1)
    tiny.width, tiny.height = 24, 20
    tex = I.scene_textured(24, 20, 4, seed=0, n_spheres=3, depth=5, rr_start=3)
    return [("global", tiny, np.asarray(gt, np.float64)),
            ("textured", tex, I.fourier_params(tex, 5).astype(np.float64))]


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("clockwise", [False, True])
def test_triangle_fan_replaces_the_plane(which, clockwise):
    name, spec, p = _scenes()[which]
    mesh = _plane_as_mesh(spec, clockwise)
    for flags in (0, O.NO_NEE):
        a, ma = O.render(spec, p, 4, 2, O.TAG_EVAL, 2, flags)
        b, mb = O.render(mesh, p, 4, 2, O.TAG_EVAL, 2, flags)
        # both sides are FP64: only decisions within rounding of a boundary may
        # differ.  (The fan's margins also count the basis sign at n.z = 0,
        # which both sides take identically here, so the plane's are used.)
        ok = ma > 1e-11
        assert ok.mean() > 0.95, (name, ok.mean())
        np.testing.assert_allclose(b[ok], a[ok], rtol=1e-9, atol=1e-12)
    dimg = I.target_image_synthetic(spec, 6).astype(np.float64) - 0.7
    ga_, _, mga, _ = O.render_bwd(spec, p, dimg, 4, 2, O.TAG_EVAL, 2)
    gb_, _, mgb, _ = O.render_bwd(mesh, p, dimg, 4, 2, O.TAG_EVAL, 2)
    assert np.min(mga) > 1e-11, "a decision near its boundary: pick another seed"
    scale = np.abs(ga_).max()
    assert scale > 0
    np.testing.assert_allclose(gb_, ga_, rtol=0, atol=1e-9 * scale)


def _sphere_mesh_scene(layout, width=20, height=16, freq=2):
    v, t = I.icosphere(freq, center=(0.0, 1.1, 0.0), radius=1.0, disp=0.15, seed=3)
    s = I.SceneSpec(width=width, height=height, plane_mat=0, fixed_mats=I.PLANE_GREY.copy(),
                    verts=v, tris=t, mesh_mat=I.MAT_PARAM, param_layout=layout, depth=4,
                    rr_start=0, ch_mask=I.CH_RGB_ROUGH, fixed_default=(0.5, 0.5, 0.5, 0.0, 0.5))
    return s


def test_constant_vertex_values_equal_a_global_material():
    sv = _sphere_mesh_scene(I.LAYOUT_VERTEX)
    sg = _sphere_mesh_scene(I.LAYOUT_TEXTURE)
    c = np.array([0.7, 0.4, 0.2, 0.35])
    pv = np.tile(c, sv.n_elems)
    assert sg.n_params == 4 and sv.n_params == 4 * len(sv.verts)
    a, _ = O.render(sg, c, 8, 1, O.TAG_EVAL, 2)
    b, _ = O.render(sv, pv, 8, 1, O.TAG_EVAL, 2)
    np.testing.assert_allclose(b, a, rtol=1e-12, atol=1e-15)
    T = I.target_image_synthetic(sg, 3)
    g, _, _, _, _ = O.grad(sg, c, T, 8, 1, O.TAG_EVAL, O.TAG_ADJ_PROP, 2)
    gv, _, _, _, _ = O.grad(sv, pv, T, 8, 1, O.TAG_EVAL, O.TAG_ADJ_PROP, 2)
    assert np.all(g != 0)
    np.testing.assert_allclose(gv.reshape(-1, 4).sum(0), g, rtol=1e-10)
    # many vertices take part, so the weights are spread, not all on one corner
    assert np.count_nonzero(np.abs(gv.reshape(-1, 4)).sum(1)) > 10


def test_linear_vertex_field_equals_bilinear_texture():
    # flat square mesh over [-2.5, 2.5]^2, i.e. planar UV in [0.25, 0.75]^2: the
    # region between the centres of a 2x2 texture, where bilinear interpolation
    # of a linear field is that field
    a0, au, av = np.array([0.2, 0.3, 0.5, 0.3]), np.array([0.9, -0.4, 0.2, 0.6]), \
        np.array([-0.3, 0.8, 0.5, 0.2])
    v, t = I.heightfield(3, extent=(-2.5, 2.5, -2.5, 2.5), amp=0.0)
    assert np.all(v[:, 1] == 0)
    v = v.astype(np.float32).astype(np.float64)  # scene geometry crosses the ABI as float32
    base = dict(width=24, height=18, plane_enabled=False, verts=v, tris=t,
                spheres=np.array([[0.6, 0.7, 0.2, 0.7]]), sphere_mat=np.array([0], np.int32),
                fixed_mats=np.array([[0.8, 0.8, 0.8, 0.0, 0.3]]), mesh_mat=I.MAT_PARAM,
                depth=4, ch_mask=I.CH_RGB_ROUGH)
    st = I.SceneSpec(tex_w=2, tex_h=2, param_layout=I.LAYOUT_TEXTURE, **base)
    sv = I.SceneSpec(param_layout=I.LAYOUT_VERTEX, **base)

    def field(u, w):
        return a0 + au * u + av * w

    tex = np.array([field((x + 0.5) / 2, (y + 0.5) / 2) for y in range(2) for x in range(2)])
    ex = st.plane_extent
    vert = np.array([field((p[0] - ex[0]) / (ex[1] - ex[0]), (p[2] - ex[2]) / (ex[3] - ex[2]))
                     for p in v])
    a, _ = O.render(st, tex.reshape(-1), 2, 0, O.TAG_EVAL, 2)
    b, _ = O.render(sv, vert.reshape(-1), 2, 0, O.TAG_EVAL, 2)
    # most pixels see the mesh
    blank, _ = O.render(sv, np.zeros(sv.n_params) + 0.5, 2, 0, O.TAG_EVAL, 2)
    assert np.mean(np.any(np.abs(b - blank) > 1e-6, -1)) > 0.3
    # same geometry on both sides: the paths only see material values that
    # agree to rounding, so every pixel is compared
    np.testing.assert_allclose(b, a, rtol=1e-10, atol=1e-13)


def test_mesh_shadow_matches_quadrature():
    # Lambertian plane, square light (side 2) at y=5, a fixed black mesh square
    # (side 2) floating at y=2.5 under it; direct light at each pixel centre is
    # rho/pi * integral over the light of Le cos cos / d^2 * V, with V = 0 where
    # the segment crosses the square (midpoint rule, 600 x 600)
    occ_y, occ_h, occ_x, occ_z = 2.5, 1.0, 0.5, -0.5
    v, t = _fan(occ_h, y=occ_y, cx=occ_x, cz=occ_z)
    s = I.SceneSpec(width=10, height=6, spheres=np.zeros((0, 4)),
                    sphere_mat=np.zeros((0,), np.int32), plane_mat=I.MAT_PARAM, depth=1,
                    light_center=(0.0, 5.0, 0.0), light_side=2.0, light_Le=(3.0, 3.0, 3.0),
                    verts=v, tris=t, mesh_mat=0, fixed_mats=np.array([[0.0, 0.0, 0.0, 0.0, 1.0]]),
                    env=(0.0, 0.0, 0.0), ch_mask=I.CH_ALL)
    rho = np.array([0.8, 0.5, 0.3])
    p = np.array(list(rho) + [0.0, 0.5])
    batches = np.stack([O.render(s, p, 1, b, O.TAG_EVAL, 64,
                                 flags=O.LAMBERT_ONLY | O.PIXEL_CENTER)[0] for b in range(32)])
    mean = batches.mean(0)
    se = batches.std(0, ddof=1) / np.sqrt(batches.shape[0])
    eye = np.array(s.cam_eye)
    w = np.array(s.cam_target) - eye
    w /= np.linalg.norm(w)
    u = np.cross(w, s.cam_up)
    u /= np.linalg.norm(u)
    vv = np.cross(u, w)
    th = math.tan(math.radians(s.vfov_deg) / 2)
    cx, cy, cz = s.light_center
    h = s.light_side / 2
    n = 600
    LX, LZ = np.meshgrid(cx - h + (np.arange(n) + 0.5) * (2 * h / n),
                         cz - h + (np.arange(n) + 0.5) * (2 * h / n))
    dA = (2 * h / n) ** 2
    checked = shadowed = 0
    for py in range(s.height):
        for px in range(s.width):
            sx = (2 * (px + 0.5) / s.width - 1) * th * s.width / s.height
            sy = (1 - 2 * (py + 0.5) / s.height) * th
            d = w + sx * u + sy * vv
            d /= np.linalg.norm(d)
            if d[1] >= 0:
                continue
            # the camera (y = 2) sits below the square: a ray going down never meets it
            x = eye + (-eye[1] / d[1]) * d
            dx, dz = LX - x[0], LZ - x[2]
            d2 = dx * dx + cy * cy + dz * dz
            f = occ_y / cy  # where the segment crosses y = occ_y
            mx, mz = x[0] + f * dx, x[2] + f * dz
            vis = ~((np.abs(mx - occ_x) < occ_h) & (np.abs(mz - occ_z) < occ_h))
            E = float(np.sum(vis * (cy * cy) / (d2 * d2)) * dA)
            E0 = float(np.sum((cy * cy) / (d2 * d2)) * dA)
            ref = rho / math.pi * s.light_Le[0] * E
            assert np.all(np.abs(mean[py, px] - ref) <= 4 * se[py, px] + 2e-3 * E0), \
                (px, py, mean[py, px], ref, se[py, px])
            checked += 1
            shadowed += E < 0.9 * E0
    assert checked >= 30 and shadowed >= 5, (checked, shadowed)


def _J(spec, p, dimg, flags, seed=7, it=3, spp=2):
    img, _ = O.render(spec, p, seed, it, O.TAG_ADJ_PROP, spp, flags)
    return float(np.sum(img * dimg))


@pytest.mark.parametrize("flags", [O.PARAM_INDEP, O.PARAM_INDEP | O.NO_NEE])
def test_vertex_adjoint_matches_central_differences(flags):
    spec = _sphere_mesh_scene(I.LAYOUT_VERTEX, 24, 20)
    p = I.vertex_fourier_params(spec, 4).astype(np.float64)
    dimg = I.target_image_synthetic(spec, 11).astype(np.float64) - 0.7
    g, ga, _, _ = O.render_bwd(spec, p, dimg, 7, 3, O.TAG_ADJ_PROP, 2, flags)
    live = np.flatnonzero(g)
    assert len(live) > 40
    gen = np.random.Generator(np.random.PCG64(0))
    idx = np.concatenate([gen.choice(live, 20, replace=False),
                          gen.choice(len(p), 4, replace=False)])
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        cd = (_J(spec, pp, dimg, flags) - _J(spec, pm, dimg, flags)) / (2 * h)
        assert abs(cd - g[i]) <= 1e-6 * ga[i] + 1e-13, (i, cd, g[i], ga[i])


def test_mesh_scene_validation():
    spec = _sphere_mesh_scene(I.LAYOUT_VERTEX)
    bad = _sphere_mesh_scene(I.LAYOUT_VERTEX)
    bad.tris = bad.tris.copy()
    bad.tris[3, 1] = len(bad.verts)
    with pytest.raises(ValueError):
        O.render(bad, np.zeros(spec.n_params) + 0.5, 0, 0, O.TAG_EVAL, 1)
    # per-vertex parameters with a parameterised plane are refused
    bad = _sphere_mesh_scene(I.LAYOUT_VERTEX)
    bad.plane_mat = I.MAT_PARAM
    with pytest.raises(ValueError):
        O.render(bad, np.zeros(spec.n_params) + 0.5, 0, 0, O.TAG_EVAL, 1)
