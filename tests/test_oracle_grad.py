"""Pins of the oracle's gradient samples (CPU only).

* With parameter-independent sampling the adjoint must equal the derivative of
  J(pi) = sum_p delta_p . I_p(pi; u) at fixed random numbers u, so central
  differences pin it to O(h^2).
* With the renderer's importance sampling (roughness-dependent GGX lobe) the
  detached adjoint is an unbiased estimator of grad E[J]; central differences
  of E[J] (common random numbers, many seeds) pin it statistically.
* The finite-difference sample of Eq. 5 vanishes identically when the two
  parameter vectors are equal, and has the mean F(pi_i) - F(pi_{i-1}).
"""
import numpy as np
import pytest

import oracle as O
from paper_2309_15676_amd import inputs as I


def _J(spec, p, dimg, flags, seed=7, it=3, spp=2):
    img, _ = O.render(spec, p, seed, it, O.TAG_ADJ_PROP, spp, flags)
    return float(np.sum(img * dimg))


def _scenes():
    tiny, gt, _ = I.config_tiny(seed_gt=1)
    tiny.width = tiny.height = 24
    tex = I.scene_textured(24, 20, 4, seed=0, n_spheres=3, depth=5, rr_start=3)
    return [("global", tiny, np.asarray(gt, np.float64)),
            ("textured", tex, I.fourier_params(tex, 5).astype(np.float64))]


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("flags", [O.PARAM_INDEP, O.PARAM_INDEP | O.NO_NEE, O.LAMBERT_ONLY])
def test_adjoint_matches_central_differences(which, flags):
    name, spec, p = _scenes()[which]
    dimg = I.target_image_synthetic(spec, 11).astype(np.float64) - 0.7
    g, ga, _, _ = O.render_bwd(spec, p, dimg, 7, 3, O.TAG_ADJ_PROP, 2, flags)
    assert np.count_nonzero(g) > 0
    idx = np.arange(len(p)) if len(p) <= 16 else \
        np.random.Generator(np.random.PCG64(0)).choice(len(p), 24, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        cd = (_J(spec, pp, dimg, flags) - _J(spec, pm, dimg, flags)) / (2 * h)
        assert abs(cd - g[i]) <= 1e-6 * ga[i] + 1e-13, (name, i, cd, g[i], ga[i])


def test_adjoint_unbiased_under_importance_sampling():
    # E[adjoint] = d/dpi E[J]; E[J(pi+h)] - E[J(pi-h)] estimated with common
    # random numbers over K independent keys
    spec, gt, _ = I.config_tiny(seed_gt=3)
    spec.width = spec.height = 16
    p = np.asarray(gt, np.float64)
    dimg = I.target_image_synthetic(spec, 2).astype(np.float64) - 0.5
    K, spp, h = 48, 8, 2e-3
    adj, fd = [], []
    for k in range(K):
        g, _, _, _ = O.render_bwd(spec, p, dimg, 100 + k, 0, O.TAG_EVAL, spp)
        adj.append(g)
        row = []
        for i in range(len(p)):
            pp, pm = p.copy(), p.copy()
            pp[i] += h
            pm[i] -= h
            row.append((_J(spec, pp, dimg, 0, 100 + k, 0, spp) -
                        _J(spec, pm, dimg, 0, 100 + k, 0, spp)) / (2 * h))
        fd.append(row)
    adj, fd = np.array(adj), np.array(fd)
    ma, mf = adj.mean(0), fd.mean(0)
    se = np.sqrt(adj.var(0, ddof=1) / K + fd.var(0, ddof=1) / K)
    assert np.all(np.abs(ma - mf) <= 4.5 * se + 1e-3 * np.abs(mf)), (ma, mf, se)


def test_fd_sample_is_exactly_zero_for_equal_parameters():
    spec = I.scene_textured(20, 16, 4, seed=1, n_spheres=3, depth=4, rr_start=2)
    p = I.fourier_params(spec, 3)
    T = I.target_image_synthetic(spec, 4)
    r = O.gradient_pair(spec, p, p.copy(), T, seed=9, iteration=5)
    assert np.all(r["dF"] == 0.0)
    assert np.count_nonzero(r["F"]) > 0


def test_fd_sample_mean_is_gradient_change():
    # Eq. 5-6: E[<dF_i>] = F_i - F_{i-1}, and E[<F_{i-1}> + <dF_i>] = F_i.
    spec, gt, init = I.config_tiny()
    spec.width = spec.height = 16
    T = I.target_image_synthetic(spec, 1)
    p0 = np.asarray(init, np.float64)
    p1 = p0 + np.array([0.05, -0.04, 0.03, -0.05, 0.04])
    K = 48
    dF, F0, F1 = [], [], []
    for k in range(K):
        r = O.gradient_pair(spec, p1, p0, T, seed=1000 + k, iteration=1, spp_prop=4, spp_fd=4)
        dF.append(r["dF"])
        F1.append(r["F"])
        F0.append(O.gradient_pair(spec, p0, None, T, seed=5000 + k, iteration=0, spp_prop=4)["F"])
    dF, F0, F1 = map(np.array, (dF, F0, F1))
    lhs = F0.mean(0) + dF.mean(0)
    se = np.sqrt(F0.var(0, ddof=1) / K + dF.var(0, ddof=1) / K + F1.var(0, ddof=1) / K)
    assert np.all(np.abs(lhs - F1.mean(0)) <= 4.5 * se), (lhs, F1.mean(0), se)
    # and the finite-difference sample is far less noisy than the proportional one
    assert np.all(dF.std(0) < F1.std(0))


@pytest.mark.parametrize("which", [0, 1])
def test_adjoint_at_base_colour_zero_lambert_only(which):
    """At a base colour of exactly 0 (the lower bound of its domain) the
    Lambert-only BSDF value of that channel vanishes, but its derivative
    (1/pi times the incident radiance) does not: the adjoint must equal the
    one-sided derivative of J there.  In Lambert-only mode J is a polynomial
    in each base-colour parameter, so the second-order one-sided difference
    (-3 J(0) + 4 J(h) - J(2h)) / 2h is exact up to O(h^2)."""
    name, spec, p = _scenes()[which]
    p = p.copy()
    n_ch = spec.n_ch
    if name == "global":
        zero = [0, 2]
    else:
        zero = list(range(0, len(p), n_ch))[::2]  # every other texel's red channel
    p[zero] = 0.0
    dimg = I.target_image_synthetic(spec, 11).astype(np.float64) - 0.7
    flags = O.LAMBERT_ONLY
    g, ga, _, _ = O.render_bwd(spec, p, dimg, 7, 3, O.TAG_ADJ_PROP, 2, flags)
    checked = 0
    h = 1e-5
    for i in zero[:12]:
        js = []
        for k in (0, 1, 2):
            q = p.copy()
            q[i] = k * h
            js.append(_J(spec, q, dimg, flags))
        fd = (-3 * js[0] + 4 * js[1] - js[2]) / (2 * h)
        assert abs(fd - g[i]) <= 1e-6 * ga[i] + 1e-12, (name, i, fd, g[i], ga[i])
        checked += g[i] != 0.0
    assert checked > 0  # the derivative at the bound is not zero
