"""Pins of the oracle's path tracer and BSDF against closed forms, quadrature
and textbook identities (CPU only)."""
import math

import numpy as np
import pytest

import oracle as O
from paper_2309_15676_amd import inputs as I


def test_white_furnace_every_sample_is_one():
    # albedo-1 Lambertian sphere in a uniform unit environment: each path
    # returns the environment radiance (up to the rounding of f cos / p)
    s = I.scene_white_furnace(16, 16)
    img, _ = O.render(s, [1, 1, 1, 0, 0.5], seed=3, iteration=0, tag=O.TAG_EVAL, spp=1,
                      flags=O.LAMBERT_ONLY | O.NO_NEE)
    np.testing.assert_allclose(img, 1.0, rtol=1e-14)
    # some pixels see the sphere (otherwise the check is vacuous)
    img2, _ = O.render(s, [0.5, 0.5, 0.5, 0, 0.5], 3, 0, O.TAG_EVAL, 1,
                       flags=O.LAMBERT_ONLY | O.NO_NEE)
    assert np.sum(np.abs(img2 - 0.5) < 1e-12) > 30


@pytest.mark.parametrize("rho", [(0.2, 0.5, 0.9), (1.0, 0.0, 0.35)])
def test_lambert_sphere_radiance_and_gradient_closed_form(rho):
    # a convex Lambertian object alone in a uniform environment L: one bounce,
    # weight f cos / p = rho, so I = rho * L on the sphere and L off it; the
    # L2-loss gradient w.r.t. rho is sum_{p on sphere} 2 (rho - T_p) L / (3 N)
    s = I.scene_white_furnace(20, 16)
    s.env = (0.75, 0.75, 0.75)
    p = np.array(list(rho) + [0.0, 0.5])
    img, _ = O.render(s, p, 5, 0, O.TAG_EVAL, 1, flags=O.LAMBERT_ONLY | O.NO_NEE)
    on = np.any(img != 0.75, axis=-1)
    assert on.sum() > 20
    np.testing.assert_allclose(img[on], np.tile(0.75 * np.array(rho), (on.sum(), 1)), rtol=1e-14)
    T = I.target_image_synthetic(s, 9).astype(np.float64)
    g, _, _, _, _ = O.grad(s, p, T, 5, 0, O.TAG_EVAL, O.TAG_EVAL, 1,
                           flags=O.LAMBERT_ONLY | O.NO_NEE)
    N = s.n_pixels
    expect = [np.sum(2 * (0.75 * rho[k] - T[on][:, k]) * 0.75 / (3 * N)) for k in range(3)]
    np.testing.assert_allclose(g[:3], expect, rtol=1e-12, atol=1e-15)
    assert g[3] == 0 and g[4] == 0


def _gauss_legendre_2d(f, a0, a1, b0, b1, n=64):
    x, w = np.polynomial.legendre.leggauss(n)
    xs = 0.5 * (a1 - a0) * x + 0.5 * (a1 + a0)
    ys = 0.5 * (b1 - b0) * x + 0.5 * (b1 + b0)
    X, Y = np.meshgrid(xs, ys)
    W = np.outer(w, w) * 0.25 * (a1 - a0) * (b1 - b0)
    return float(np.sum(W * f(X, Y)))


def _plane_only(width=4, height=4):
    s = I.SceneSpec(width=width, height=height, spheres=np.zeros((0, 4)),
                    sphere_mat=np.zeros((0,), np.int32), plane_mat=I.MAT_PARAM,
                    depth=1, tex_w=1, tex_h=1, ch_mask=I.CH_ALL, env=(0.0, 0.0, 0.0))
    return s


def test_direct_light_matches_quadrature():
    # Lambertian plane lit by the square emitter only: the pixel-centre value is
    # rho/pi * integral_light Le cos_s cos_l / d^2 dA (2-D Gauss-Legendre);
    # the MC mean of NEE + BSDF sampling with MIS must agree within 4 standard
    # errors (estimated from 32 independent batches)
    s = _plane_only(6, 4)
    rho = np.array([0.8, 0.5, 0.3])
    p = np.array(list(rho) + [0.0, 0.5])
    batches = np.stack([O.render(s, p, 1, b, O.TAG_EVAL, 128,
                                 flags=O.LAMBERT_ONLY | O.PIXEL_CENTER)[0] for b in range(32)])
    mean = batches.mean(0)
    se = batches.std(0, ddof=1) / np.sqrt(batches.shape[0])
    # per-pixel hit point from the camera model (written here, not taken from the oracle)
    eye = np.array(s.cam_eye)
    w = np.array(s.cam_target) - eye
    w /= np.linalg.norm(w)
    u = np.cross(w, s.cam_up)
    u /= np.linalg.norm(u)
    v = np.cross(u, w)
    th = math.tan(math.radians(s.vfov_deg) / 2)
    cx, cy, cz = s.light_center
    h = s.light_side / 2
    checked = 0
    for py in range(s.height):
        for px in range(s.width):
            sx = (2 * (px + 0.5) / s.width - 1) * th * s.width / s.height
            sy = (1 - 2 * (py + 0.5) / s.height) * th
            d = w + sx * u + sy * v
            d /= np.linalg.norm(d)
            if d[1] >= 0:
                continue
            x = eye + (-eye[1] / d[1]) * d

            def integrand(X, Z):
                dx, dy, dz = X - x[0], cy, Z - x[2]
                d2 = dx * dx + dy * dy + dz * dz
                cos = dy / np.sqrt(d2)
                return cos * cos / d2

            E = _gauss_legendre_2d(integrand, cx - h, cx + h, cz - h, cz + h)
            ref = rho / math.pi * s.light_Le[0] * E
            assert np.all(np.abs(mean[py, px] - ref) <= 4 * se[py, px] + 1e-12), \
                (px, py, mean[py, px], ref, se[py, px])
            assert np.all(se[py, px] < 0.02 * ref)
            checked += 1
    assert checked >= 8


def _hemisphere_quadrature(fn, n_theta=400, n_phi=800):
    """Midpoint rule in (cos theta, phi) over the upper hemisphere around +z.
    fn maps an (m, 3) array of unit directions to (m, k) values."""
    ct = (np.arange(n_theta) + 0.5) / n_theta
    ph = (np.arange(n_phi) + 0.5) / n_phi * 2 * math.pi
    C, P = np.meshgrid(ct, ph, indexing="ij")
    S = np.sqrt(1 - C * C)
    dirs = np.stack([S * np.cos(P), S * np.sin(P), C], -1).reshape(-1, 3)
    return fn(dirs).sum(0) * (1.0 / n_theta) * (2 * math.pi / n_phi)


@pytest.mark.parametrize("mat,theta", [((0.9, 0.6, 0.2, 0.0, 0.6), 0.3),
                                       ((0.8, 0.8, 0.8, 1.0, 0.35), 0.9),
                                       ((0.3, 0.5, 0.75, 0.5, 0.8), 1.2)])
def test_directional_albedo_sampling_matches_quadrature(mat, theta):
    # environment 1 above a plane of this material, depth 1, no light: the pixel
    # value is the directional albedo integral f(wo, wi) cos dwi, which the
    # quadrature evaluates from the BSDF alone; the MC estimate uses the
    # renderer's lobe sampling and mixture density, so a density that does not
    # match the sampler fails here
    s = _plane_only(1, 1)
    s.env = (1.0, 1.0, 1.0)
    s.light_enabled = False
    # aim the camera so the single pixel-centre ray reaches the plane at angle theta
    s.cam_eye = (0.0, math.cos(theta), math.sin(theta))
    s.cam_target = (0.0, 0.0, 0.0)
    s.cam_up = (0.0, 1.0, 0.0) if theta > 0.05 else (0.0, 0.0, -1.0)
    p = np.array(mat, np.float64)
    img, _ = O.render(s, p, 11, 0, O.TAG_EVAL, 200000, flags=O.PIXEL_CENTER)
    n = np.array([0.0, 1.0, 0.0])
    wo = np.array(s.cam_eye) / np.linalg.norm(s.cam_eye)

    def f_cos(wl):  # wl around +z; rotate so +z -> +y
        wi = np.stack([wl[:, 0], wl[:, 2], -wl[:, 1]], -1)
        return O.bsdf_many(p, n, wo, wi)[:, :3] * wl[:, 2:3]

    ref = _hemisphere_quadrature(f_cos)
    np.testing.assert_allclose(img[0, 0], ref, rtol=0.02)


def test_bsdf_reciprocity_and_lambert_part():
    g = np.random.Generator(np.random.PCG64(4))
    n = np.array([0.0, 0.0, 1.0])
    for _ in range(50):
        a, b = g.normal(size=3), g.normal(size=3)
        a[2], b[2] = abs(a[2]), abs(b[2])
        wo, wi = a / np.linalg.norm(a), b / np.linalg.norm(b)
        mat = g.uniform(0.06, 1.0, 5)
        f1 = O.bsdf(mat, n, wo, wi)
        f2 = O.bsdf(mat, n, wi, wo)
        np.testing.assert_allclose(f1[:12], f2[:12], rtol=1e-12, atol=1e-14)
        lam = O.bsdf(mat, n, wo, wi, O.LAMBERT_ONLY)
        np.testing.assert_allclose(lam[:3], mat[:3] / math.pi, rtol=1e-15)
        # below the surface the BSDF is zero
        wb = wi * np.array([1, 1, -1])
        assert np.all(O.bsdf(mat, n, wo, wb)[:3] == 0)


def test_bsdf_partials_match_central_differences():
    g = np.random.Generator(np.random.PCG64(5))
    n = np.array([0.0, 0.0, 1.0])
    h = 1e-6
    for _ in range(40):
        a, b = g.normal(size=3), g.normal(size=3)
        a[2], b[2] = abs(a[2]) + 0.05, abs(b[2]) + 0.05
        wo, wi = a / np.linalg.norm(a), b / np.linalg.norm(b)
        mat = g.uniform(0.1, 0.95, 5)
        out = O.bsdf(mat, n, wo, wi)
        for attr in range(5):
            mp, mm = mat.copy(), mat.copy()
            mp[attr] += h
            mm[attr] -= h
            fd = (O.bsdf(mp, n, wo, wi)[:3] - O.bsdf(mm, n, wo, wi)[:3]) / (2 * h)
            if attr < 3:
                an = np.zeros(3)
                an[attr] = out[3 + attr]
            elif attr == 3:
                an = out[6:9]
            else:
                an = out[9:12]
            np.testing.assert_allclose(an, fd, rtol=1e-5, atol=1e-7 * (1 + np.abs(out[:3]).max()))


def test_roughness_floor_has_zero_derivative():
    n = np.array([0.0, 0.0, 1.0])
    wo = np.array([0.3, 0.0, 0.95]); wo /= np.linalg.norm(wo)
    wi = np.array([-0.2, 0.1, 0.97]); wi /= np.linalg.norm(wi)
    out_lo = O.bsdf([0.5, 0.5, 0.5, 0.5, 0.01], n, wo, wi)
    out_fl = O.bsdf([0.5, 0.5, 0.5, 0.5, I.ROUGH_MIN], n, wo, wi)
    np.testing.assert_array_equal(out_lo[:3], out_fl[:3])
    assert np.all(out_lo[9:12] == 0)


def test_sampling_density_integral_closed_form():
    # the mixture density over the upper hemisphere: the cosine half integrates
    # to 1/2; at normal incidence the reflected GGX half-vector stays above the
    # surface iff theta_h < 45 deg, whose probability under the GGX density of
    # half-vectors is 1 / (1 + alpha^2); so the integral is 1/2 + 1/2 / (1 + alpha^2)
    n = np.array([0.0, 0.0, 1.0])
    for rough in (0.45, 0.6, 0.9):  # lobes wide enough for a midpoint rule
        wo = np.array([0.0, 0.0, 1.0])
        tot = _hemisphere_quadrature(
            lambda wi: O.bsdf_many([0.5] * 3 + [0.0, rough], n, wo, wi)[:, 12:13], 2000, 64)[0]
        a2 = rough ** 4
        np.testing.assert_allclose(tot, 0.5 + 0.5 / (1 + a2), rtol=2e-4)
    # oblique incidence: still a sub-probability density
    wo = np.array([math.sin(1.2), 0, math.cos(1.2)])
    tot = _hemisphere_quadrature(lambda wi: O.bsdf_many([0.5] * 3 + [0.0, 0.5], n, wo, wi)[:, 12:13])[0]
    assert 0.5 < tot <= 1.0 + 1e-3
