"""Pins of the oracle's shared-path finite-difference sample (CPU only).

Eq. 5 as written draws one path x at the current parameters pi_i and
evaluates the integrand at both parameter vectors over the density of pi_i:
  <dF_i> = (f(x, pi_i) - f(x, pi_{i-1})) / p(x, pi_i).
The oracle's pi_{i-1} half is its ordinary estimator with the directions
chosen (and every BSDF density taken) at pi_i.  Pinned here:
* sampled at its own parameters it is the plain estimator, bit for bit;
* with parameter-independent sampling it is the primary-sample-space replay
  (the two forms then trace the same paths with the same densities);
* at fixed random numbers the path does not move with the evaluated
  parameters, so its adjoint is the derivative of its radiance estimate:
  central differences pin it to O(h^2) under the renderer's own importance
  sampling (no parameter-independent mode needed);
* the radiance and gradient estimates are unbiased for those of the
  evaluated parameters (statistically, common seeds), which a density taken
  at the wrong parameters would break;
* the finite-difference sample vanishes for equal parameters and has the mean
  F_i - F_{i-1} (Eq. 5-6).
"""
import numpy as np
import pytest

import oracle as O
from paper_2309_15676_amd import inputs as I


def _scenes():
    tiny, gt, _ = I.config_tiny(seed_gt=1)
    tiny.width = tiny.height = 24
    tex = I.scene_textured(24, 20, 4, seed=0, n_spheres=3, depth=5, rr_start=3)
    g = np.random.Generator(np.random.PCG64(4))
    pa_t = I.fourier_params(tex, 5).astype(np.float64)
    pb_t = np.clip(pa_t + g.normal(0, 0.08, pa_t.shape), 0.1, 0.95)
    pa = np.asarray(gt, np.float64)
    pb = np.clip(pa + np.array([0.06, -0.05, 0.04, -0.07, 0.09]), 0.1, 0.95)
    return [("global", tiny, pa, pb), ("textured", tex, pa_t, pb_t)]


def _glossy():
    spec, _, _ = I.config_tiny()
    spec.width = spec.height = 12
    pa = np.array([0.6, 0.5, 0.4, 0.85, 0.6])
    pb = np.array([0.5, 0.55, 0.45, 0.8, 0.25])  # much sharper lobe than the sampling one
    return spec, pa, pb


@pytest.mark.parametrize("which", [0, 1])
def test_sampled_at_own_parameters_is_the_plain_estimator(which):
    name, spec, p, _ = _scenes()[which]
    a, ma = O.render(spec, p, 3, 2, O.TAG_PRIMAL_FD, 2)
    b, mb = O.render(spec, p, 3, 2, O.TAG_PRIMAL_FD, 2, sample_params=p)
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(ma, mb)
    dimg = I.target_image_synthetic(spec, 11).astype(np.float64) - 0.6
    g1 = O.render_bwd(spec, p, dimg, 3, 2, O.TAG_ADJ_FD, 2)
    g2 = O.render_bwd(spec, p, dimg, 3, 2, O.TAG_ADJ_FD, 2, sample_params=p)
    for x, y in zip(g1, g2):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("which", [0, 1])
def test_shared_fd_is_the_replay_when_sampling_is_parameter_independent(which):
    name, spec, pa, pb = _scenes()[which]
    T = I.target_image_synthetic(spec, 4)
    for flags in (O.PARAM_INDEP, O.PARAM_INDEP | O.NO_NEE, O.LAMBERT_ONLY):
        r = O.gradient_pair(spec, pa, pb, T, 9, 5, flags=flags)
        s = O.gradient_pair(spec, pa, pb, T, 9, 5, flags=flags, fd_shared=True)
        assert np.count_nonzero(r["dF"]) > 0
        for k in ("dF", "I_fd0", "A_fd0", "F"):
            np.testing.assert_array_equal(r[k], s[k], err_msg="%s %s %d" % (name, k, flags))
    # under importance sampling the two forms are different estimators
    r = O.gradient_pair(spec, pa, pb, T, 9, 5)
    s = O.gradient_pair(spec, pa, pb, T, 9, 5, fd_shared=True)
    np.testing.assert_array_equal(r["I_fd1"], s["I_fd1"])  # the pi_i half is shared
    assert np.max(np.abs(r["I_fd0"] - s["I_fd0"])) > 1e-3


def _J(spec, p, p_sample, dimg, flags, seed=7, it=3, spp=2):
    img, _ = O.render(spec, p, seed, it, O.TAG_ADJ_FD, spp, flags, sample_params=p_sample)
    return float(np.sum(img * dimg))


@pytest.mark.parametrize("which", [0, 1])
@pytest.mark.parametrize("flags", [0, O.NO_NEE])
def test_shared_adjoint_matches_central_differences(which, flags):
    # the path is drawn at pa whatever the evaluated parameters are, so
    # J(pi) = sum delta . I(pi; paths of pa) is smooth in pi and its derivative
    # at pb is the adjoint of the shared estimator
    name, spec, pa, pb = _scenes()[which]
    dimg = I.target_image_synthetic(spec, 11).astype(np.float64) - 0.7
    g, ga, _, _ = O.render_bwd(spec, pb, dimg, 7, 3, O.TAG_ADJ_FD, 2, flags, sample_params=pa)
    assert np.count_nonzero(g) > 0
    idx = np.arange(len(pb)) if len(pb) <= 16 else \
        np.random.Generator(np.random.PCG64(0)).choice(len(pb), 24, replace=False)
    h = 1e-6
    for i in idx:
        pp, pm = pb.copy(), pb.copy()
        pp[i] += h
        pm[i] -= h
        cd = (_J(spec, pp, pa, dimg, flags) - _J(spec, pm, pa, dimg, flags)) / (2 * h)
        assert abs(cd - g[i]) <= 1e-6 * ga[i] + 1e-13, (name, i, cd, g[i], ga[i])


def test_shared_estimators_are_unbiased():
    # E[render(pb; paths of pa)] = E[render(pb)] and the same for the fixed-
    # adjoint gradient, with a glossy material whose lobe sharpens from pa to
    # pb (the densities differ by up to ~16x near the peak)
    spec, pa, pb = _glossy()
    dimg = I.target_image_synthetic(spec, 2).astype(np.float64) - 0.5
    K, spp = 40, 16
    sh_i, pl_i, sh_g, pl_g = [], [], [], []
    for k in range(K):
        sh_i.append(O.render(spec, pb, 100 + k, 0, O.TAG_EVAL, spp, sample_params=pa)[0].mean((0, 1)))
        pl_i.append(O.render(spec, pb, 500 + k, 0, O.TAG_EVAL, spp)[0].mean((0, 1)))
        sh_g.append(O.render_bwd(spec, pb, dimg, 100 + k, 0, O.TAG_ADJ_FD, spp,
                                 sample_params=pa)[0])
        pl_g.append(O.render_bwd(spec, pb, dimg, 500 + k, 0, O.TAG_ADJ_FD, spp)[0])
    for a, b, what in ((sh_i, pl_i, "radiance"), (sh_g, pl_g, "gradient")):
        a, b = np.array(a), np.array(b)
        se = np.sqrt(a.var(0, ddof=1) / K + b.var(0, ddof=1) / K)
        assert np.all(np.abs(a.mean(0) - b.mean(0)) <= 4.5 * se), (what, a.mean(0), b.mean(0), se)
    # the pin has power: the sampling density matters for these parameters
    img_pa_density = O.render(spec, pb, 100, 0, O.TAG_EVAL, spp, sample_params=pa)[0]
    img_own = O.render(spec, pb, 100, 0, O.TAG_EVAL, spp)[0]
    assert np.max(np.abs(img_pa_density - img_own)) > 1e-2


def test_shared_fd_sample_is_exactly_zero_for_equal_parameters():
    spec = I.scene_textured(20, 16, 4, seed=1, n_spheres=3, depth=4, rr_start=2)
    p = I.fourier_params(spec, 3)
    T = I.target_image_synthetic(spec, 4)
    r = O.gradient_pair(spec, p, p.copy(), T, seed=9, iteration=5, fd_shared=True)
    assert np.all(r["dF"] == 0.0)
    assert np.count_nonzero(r["F"]) > 0


def test_shared_fd_sample_mean_is_gradient_change():
    # Eq. 5-6 with the shared path: E[<dF_i>] = F_i - F_{i-1}
    spec, gt, init = I.config_tiny()
    spec.width = spec.height = 16
    T = I.target_image_synthetic(spec, 1)
    p0 = np.asarray(init, np.float64)
    p1 = p0 + np.array([0.05, -0.04, 0.03, -0.05, 0.04])
    K = 48
    dF, F0, F1 = [], [], []
    for k in range(K):
        r = O.gradient_pair(spec, p1, p0, T, seed=1000 + k, iteration=1, spp_prop=4, spp_fd=4,
                            fd_shared=True)
        dF.append(r["dF"])
        F1.append(r["F"])
        F0.append(O.gradient_pair(spec, p0, None, T, seed=5000 + k, iteration=0, spp_prop=4)["F"])
    dF, F0, F1 = map(np.array, (dF, F0, F1))
    lhs = F0.mean(0) + dF.mean(0)
    se = np.sqrt(F0.var(0, ddof=1) / K + dF.var(0, ddof=1) / K + F1.var(0, ddof=1) / K)
    assert np.all(np.abs(lhs - F1.mean(0)) <= 4.5 * se), (lhs, F1.mean(0), se)
    assert np.all(dF.std(0) < F1.std(0))
