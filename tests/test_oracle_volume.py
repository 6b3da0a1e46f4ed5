"""Pins of the oracle's emission-absorption volume (the volume experiment of
the Experiments section) (CPU only).

* A homogeneous volume's quadrature is exact for any segment count and
  jitter: C = e (1 - exp(-sigma l)) + env exp(-sigma l) over the chord l of
  each pixel's ray through the cube (distinct emission per channel: a channel
  mix-up fails).
* Horizontal rays through a density layered in y read the interpolation of
  the two middle layers, and central rays through a density layered in x
  read the two middle x-layers from the front and all of them from the side:
  a transposed voxel layout, a missing half-voxel centre offset or a wrong
  trilinear weight fails.
* The views are the base camera turned about the vertical axis.
* The adjoint equals the derivative of J(pi) = sum delta . C(pi; u) at fixed
  random numbers (the march does not depend on the parameters, so J is
  smooth): central differences pin density and emission gradients to O(h^2).
* The march samples nothing from the parameters, so the shared-path and the
  replay finite-difference samples are the same, and both vanish for equal
  parameters.
"""
import math

import numpy as np
import pytest

import oracle as O
from paper_2309_15676_amd import inputs as I


def _spec(res=4, views=2, w=16, h=12, sigma=3.0):
    s = I.scene_volume(res, views, w, h, sigma=sigma)
    return s


def _rays(spec, view, rows=None):
    """Pixel-centre rays of one view (independent camera construction: the
    eye turned about the vertical axis through the target)."""
    vh = spec.height // spec.vol_views
    ang = 2 * math.pi * view / spec.vol_views
    f32 = lambda v: np.asarray(v, np.float32).astype(np.float64)  # noqa: E731
    tg, eye0, up = f32(spec.cam_target), f32(spec.cam_eye), f32(spec.cam_up)
    rot = np.array([[math.cos(ang), 0, math.sin(ang)], [0, 1, 0],
                    [-math.sin(ang), 0, math.cos(ang)]])
    eye = tg + rot @ (eye0 - tg)
    w = (tg - eye) / np.linalg.norm(tg - eye)
    u = np.cross(w, up)
    u /= np.linalg.norm(u)
    v = np.cross(u, w)
    th = math.tan(math.radians(float(np.float32(spec.vfov_deg))) / 2)
    out = []
    for y in (range(vh) if rows is None else rows):
        for x in range(spec.width):
            sx = (2 * (x + 0.5) / spec.width - 1) * th * spec.width / vh
            sy = (1 - 2 * (y + 0.5) / vh) * th
            d = w + u * sx + v * sy
            out.append((x, y + view * vh, eye, d / np.linalg.norm(d)))
    return out


def _chord(spec, o, d):
    lo = np.asarray(spec.vol_box[:3], np.float32).astype(np.float64)
    hi = lo + float(np.float32(spec.vol_box[3]))
    with np.errstate(divide="ignore", invalid="ignore"):
        ta, tb = (lo - o) / d, (hi - o) / d
    t0 = max(0.0, np.max(np.minimum(ta, tb)))
    t1 = np.min(np.maximum(ta, tb))
    return max(t1 - t0, 0.0)


@pytest.mark.parametrize("jitter", [False, True])
def test_homogeneous_volume_closed_form(jitter):
    spec = _spec()
    e = np.array([0.3, 0.6, 0.9])
    dens = 0.4
    p = np.tile(np.r_[e, dens], spec.vol_res ** 3)
    flags = 0 if jitter else O.PIXEL_CENTER
    img, _ = O.render(spec, p, 5, 1, O.TAG_EVAL, 1, flags)
    sig = float(np.float32(spec.vol_sigma)) * dens
    env = float(np.float32(spec.env[0]))
    hits = 0
    for view in range(spec.vol_views):
        for x, y, o, d in _rays(spec, view):
            if jitter:
                continue
            l = _chord(spec, o, d)
            hits += l > 0
            want = e * (1 - math.exp(-sig * l)) + env * math.exp(-sig * l)
            np.testing.assert_allclose(img[y, x], want, rtol=1e-12, atol=1e-14)
    if jitter:
        # the same for jittered rays: every pixel is e (1 - a) + env a with a common
        # a per pixel (the quadrature of a constant field is exact)
        a = (img - e) / (env - e)
        assert np.allclose(a, a[..., :1], rtol=1e-10, atol=1e-12)
    else:
        assert 0 < hits < spec.n_pixels


def test_layered_density_horizontal_rays():
    # eye at the cube's mid-height, odd rows: the middle row's rays are
    # horizontal at y = 1, the boundary of layers 1 and 2 (of 4)
    spec = _spec(res=4, views=3, w=15, h=13)
    spec.cam_eye = (0.0, 1.0, 4.5)
    layers = np.array([0.1, 0.3, 0.6, 0.8])
    R = spec.vol_res
    p = np.zeros((R, R, R, 4))
    p[..., 3] = layers[None, :, None]  # index (z, y, x): density by y
    img, _ = O.render(spec, p.reshape(-1), 5, 1, O.TAG_EVAL, 1, O.PIXEL_CENTER)
    sig = float(np.float32(spec.vol_sigma)) * 0.5 * (layers[1] + layers[2])
    env = float(np.float32(spec.env[0]))
    n = 0
    for view in range(spec.vol_views):
        for x, y, o, d in _rays(spec, view, rows=[6]):
            assert abs(d[1]) < 1e-7
            l = _chord(spec, o, d)
            np.testing.assert_allclose(img[y, x], env * math.exp(-sig * l), rtol=1e-9)
            n += l > 0
    assert n > 20


def test_density_layered_in_x_seen_from_front_and_side():
    # central rays (odd sizes, pixel centres) at mid-height: view 0 looks along
    # -z through x = 0 (the interpolation of the two middle x-layers along a
    # chord of 2), view 1 (turned 90 degrees) along -x through every x-layer,
    # sampled at the voxel centres (4 segments of 0.5).  A layout with x and z
    # exchanged swaps the two.
    spec = _spec(res=4, views=4, w=9, h=9)
    spec.cam_eye = (0.0, 1.0, 4.5)
    layers = np.array([0.1, 0.3, 0.6, 0.2])
    R = spec.vol_res
    p = np.zeros((R, R, R, 4))
    p[..., 3] = layers[None, None, :]  # index (z, y, x): density by x
    img, _ = O.render(spec, p.reshape(-1), 5, 1, O.TAG_EVAL, 1, O.PIXEL_CENTER)
    k = float(np.float32(spec.vol_sigma))
    env = float(np.float32(spec.env[0]))
    front = env * math.exp(-k * 0.5 * (layers[1] + layers[2]) * 2.0)
    side = env * math.exp(-k * 0.5 * layers.sum())
    np.testing.assert_allclose(img[4, 4], front, rtol=1e-12)
    np.testing.assert_allclose(img[9 + 4, 4], side, rtol=1e-12)
    assert abs(front - side) > 1e-3 * front


def test_views_are_the_base_camera_turned():
    spec = _spec(res=5, views=4, w=10, h=8)
    p = I.volume_blobs(spec, 3).astype(np.float64)
    img, _ = O.render(spec, p, 5, 1, O.TAG_EVAL, 1, O.PIXEL_CENTER)
    for view in range(spec.vol_views):
        one = _spec(res=5, views=1, w=10, h=8)
        ang = 2 * math.pi * view / spec.vol_views
        e = np.asarray(spec.cam_eye, np.float64) - np.asarray(spec.cam_target)
        one.cam_eye = tuple(np.asarray(spec.cam_target) + np.array(
            [e[0] * math.cos(ang) + e[2] * math.sin(ang), e[1],
             -e[0] * math.sin(ang) + e[2] * math.cos(ang)]))
        single, _ = O.render(one, p, 5, 1, O.TAG_EVAL, 1, O.PIXEL_CENTER)
        np.testing.assert_allclose(img[8 * view:8 * (view + 1)], single, rtol=0, atol=2e-6)


def _J(spec, p, dimg, seed=7, it=3, spp=2):
    img, _ = O.render(spec, p, seed, it, O.TAG_ADJ_PROP, spp)
    return float(np.sum(img * dimg))


def test_volume_adjoint_matches_central_differences():
    spec = _spec(res=5, views=2, w=10, h=16, sigma=4.0)
    g0 = np.random.Generator(np.random.PCG64(2))
    p = g0.uniform(0.1, 0.9, spec.n_params)
    dimg = g0.normal(size=(spec.height, spec.width, 3))
    g, ga, _, _ = O.render_bwd(spec, p, dimg, 7, 3, O.TAG_ADJ_PROP, 2)
    assert np.count_nonzero(g) > 0.5 * spec.n_params
    idx = g0.choice(spec.n_params, 40, replace=False)
    assert np.any(idx % 4 == 3) and np.any(idx % 4 != 3)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        cd = (_J(spec, pp, dimg) - _J(spec, pm, dimg)) / (2 * h)
        assert abs(cd - g[i]) <= 1e-6 * ga[i] + 1e-12, (i, cd, g[i], ga[i])


def test_volume_fd_samples():
    spec = _spec(res=4, views=2, w=8, h=12)
    p = I.volume_blobs(spec, 1).astype(np.float64)
    pp = np.clip(p + np.random.Generator(np.random.PCG64(3)).normal(0, 0.05, p.shape), 0, 1)
    T = np.full((spec.height, spec.width, 3), 0.3)
    a = O.gradient_pair(spec, p, pp, T, 9, 4)
    b = O.gradient_pair(spec, p, pp, T, 9, 4, fd_shared=True)
    np.testing.assert_array_equal(a["dF"], b["dF"])
    assert np.count_nonzero(a["dF"]) > 0
    z = O.gradient_pair(spec, p, p.copy(), T, 9, 4, fd_shared=True)
    assert np.all(z["dF"] == 0.0)


def test_volume_scene_validation():
    spec = _spec()
    spec.light_enabled = True
    with pytest.raises(ValueError):
        O.render(spec, np.zeros(spec.n_params), 1, 0, O.TAG_EVAL, 1)
    spec = _spec()
    spec.height = 25  # not a multiple of the view count
    with pytest.raises(ValueError):
        O.render(spec, np.zeros(spec.n_params), 1, 0, O.TAG_EVAL, 1)
