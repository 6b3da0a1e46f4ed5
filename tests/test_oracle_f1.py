"""Pins of the oracle's relative loss and of the meta-estimator ablations of
the Experiments section (zero-centred EMAs, alpha clipping, sample reuse)
(CPU only)."""
import numpy as np
import pytest

import oracle as O
from oracle import meta as OM
from paper_2309_15676_amd import inputs as I

REL_EPS = 0.01


def _tiny():
    spec, gt, _ = I.config_tiny(seed_gt=1)
    spec.width, spec.height = 20, 16
    return spec, np.asarray(gt, np.float64)


def test_relative_loss_with_constant_target_is_a_scaled_l2_gradient():
    # with T = c everywhere the relative loss is the L2 loss / (c^2 + eps)
    spec, p = _tiny()
    c = 0.4
    T = np.full((spec.height, spec.width, 3), c)
    g2, a2, _, _, _ = O.grad(spec, p, T, 5, 1, O.TAG_PRIMAL_PROP, O.TAG_ADJ_PROP, 2)
    gr, ar, _, _, _ = O.grad(spec, p, T, 5, 1, O.TAG_PRIMAL_PROP, O.TAG_ADJ_PROP, 2,
                             flags=O.RELATIVE_LOSS)
    assert np.count_nonzero(g2) == 5
    np.testing.assert_allclose(gr, g2 / (c * c + REL_EPS), rtol=1e-12)
    np.testing.assert_allclose(ar, a2 / (c * c + REL_EPS), rtol=1e-12)


def test_relative_loss_weights_each_pixel_by_its_target():
    # per-pixel weights: the relative gradient equals the fixed-adjoint
    # backward pass of 2 (I - T) / (3 N (T^2 + eps)) with I the returned primal
    spec, p = _tiny()
    T = I.target_image_synthetic(spec, 4).astype(np.float64)
    T[:, : spec.width // 2] *= 0.1  # uneven weights across the image
    gr, _, img, _, _ = O.grad(spec, p, T, 5, 1, O.TAG_PRIMAL_PROP, O.TAG_ADJ_PROP, 2,
                              flags=O.RELATIVE_LOSS)
    dimg = 2.0 * (img - T) / (3.0 * spec.n_pixels * (T * T + REL_EPS))
    gb, _, _, _ = O.render_bwd(spec, p, dimg, 5, 1, O.TAG_ADJ_PROP, 2)
    np.testing.assert_allclose(gr, gb, rtol=1e-10, atol=1e-15)
    # and differs from the L2 gradient
    g2, _, _, _, _ = O.grad(spec, p, T, 5, 1, O.TAG_PRIMAL_PROP, O.TAG_ADJ_PROP, 2)
    assert np.max(np.abs(gr - g2)) > 0.1 * np.max(np.abs(g2))


def test_centred_moment_closed_forms():
    m = OM.DecayedMoment((2,), 0.9, centred=True)
    m.push(np.array([3.0, -0.25]))
    np.testing.assert_allclose(m.estimate, [0.0, 0.0], atol=1e-15)  # one sample: no spread
    for _ in range(5):
        m.push(np.array([3.0, -0.25]))
    np.testing.assert_allclose(m.estimate, [0.0, 0.0], atol=1e-12)  # constant samples
    # two samples +a, -a with start-up-corrected weights beta/(1+beta), 1/(1+beta)
    b, a = 0.8, 1.5
    m = OM.DecayedMoment((1,), b, centred=True)
    m.push(np.array([a]))
    m.push(np.array([-a]))
    mean = (b * a - a) / (1 + b)
    np.testing.assert_allclose(m.estimate, [a * a - mean * mean], rtol=1e-13)
    z = OM.DecayedMoment((1,), b)  # zero-centred: the plain second moment
    z.push(np.array([a]))
    z.push(np.array([-a]))
    np.testing.assert_allclose(z.estimate, [a * a], rtol=1e-13)


def test_no_alpha_clip_keeps_the_unclipped_weight():
    F = np.array([1.0, -2.0, 0.5])
    clipped = OM.MetaEstimate((3,))
    free = OM.MetaEstimate((3,), clip=False)
    vF = F * F
    for m in (clipped, free):
        m.update(F, np.zeros(3), vF, np.zeros(3))
        # Eq. 7's initialisation holds with or without the clip: alpha_0 = 0
        np.testing.assert_array_equal(m.alpha_last, 0.0)
        np.testing.assert_allclose(m.F_M, F, rtol=1e-15)
    # second step with a small carried variance: Eq. 8 gives
    # Var[F] / (Var[F] + Var_M + Var[dF]); the clip of Eq. 17 caps it at
    # 1 / (2 - alpha_0) = 1/2
    vF2 = 4.0 * vF
    dF, vdF = np.zeros(3), 0.01 * vF
    clipped.update(F, dF, vF2, vdF)
    free.update(F, dF, vF2, vdF)
    want = vF2 / (vF2 + vF + vdF)
    np.testing.assert_allclose(free.alpha_last, want, rtol=1e-12)
    np.testing.assert_allclose(clipped.alpha_last, np.minimum(want, 0.5), rtol=1e-12)
    assert np.all(free.alpha_last > 0.5)


def test_sample_reuse_ablation_plumbing():
    g = np.random.Generator(np.random.PCG64(3))
    lo, hi = np.zeros(4), np.ones(4)
    p0 = np.full(4, 0.5)
    a = OM.MetaOptimizer(p0, lo, hi, 0.01)
    b = OM.MetaOptimizer(p0, lo, hi, 0.01)
    for _ in range(4):
        F, dF = g.normal(size=4), 0.1 * g.normal(size=4)
        a.step(F, dF)
        b.step(F, dF, F_var=F, dF_var=dF)  # the same samples: identical
    np.testing.assert_array_equal(a.params, b.params)
    np.testing.assert_array_equal(a.meta.F_M, b.meta.F_M)
    # variance samples of zero: Var[F] = 0, so alpha = 0 and the estimate is <F_i>
    c = OM.MetaOptimizer(p0, lo, hi, 0.01)
    for _ in range(3):
        F, dF = g.normal(size=4), 0.1 * g.normal(size=4)
        c.step(F, dF, F_var=np.zeros(4), dF_var=np.zeros(4))
        np.testing.assert_allclose(c.meta.F_M, F, rtol=1e-12)
