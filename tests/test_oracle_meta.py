"""Pins of the meta-estimator / optimiser oracle (oracle/meta.py), CPU only.

Each check is a property the paper states or a closed form that follows from
it by a different route than the recurrence:
  * Eq. 7 initialisation: <F_0>_M = <F_0>, alpha_0 = 0.
  * Eq. 16 follows from Eq. 17 with alpha_{-1} = -inf: alpha_i <= i / (i + 1).
  * With no parameter change (<dF> = 0) and samples of constant magnitude the
    meta-estimate is the running mean of all proportional samples.
  * Supplement, start-up bias: <F_i>_M is the explicit weighted sum of all
    <F_j> and <dF_j> with products of alphas; Eq. 15 is the variance of that
    sum for independent samples with the approximated variances.
  * Moment2 equals the normalised exponentially weighted average of x^2.
  * Eq. 21 is invariant to rescaling all gradient samples (up to epsilon).
  * Adam agrees with torch.optim.Adam (float64, CPU).
  * Figure 2 toy: the meta-estimator reaches the ground-truth rate 0.5.
"""
import math

import numpy as np
import pytest

from oracle import meta as M


def _run(F_seq, dF_seq, n2_seq, eta=1e-3, bF=0.99, bD=0.9):
    """Drive Moment2/Meta directly (no parameters), recording alphas."""
    n = F_seq[0].shape
    vf, vd, mt = M.Moment2(n, bF), M.Moment2(n, bD), M.Meta(n, eta)
    alphas, means, vars_, steps, varF, varD = [], [], [], [], [], []
    for i, (F, dF, n2) in enumerate(zip(F_seq, dF_seq, n2_seq)):
        vf.step(F)
        if i >= 1 and n2 > 0:
            vd.step(dF / math.sqrt(n2))
            vdf = vd.m2 * n2
        else:
            dF = np.zeros_like(F)
            vdf = np.zeros_like(F)
        steps.append(mt.step(F, dF, vf.m2, vdf))
        alphas.append(mt.alpha.copy())
        means.append(mt.mean.copy())
        vars_.append(mt.var.copy())
        varF.append(vf.m2.copy())
        varD.append(np.array(vdf, copy=True))
    return alphas, means, vars_, steps, varF, varD


def test_first_iteration_is_the_proportional_sample():
    F0 = np.array([0.3, -2.0, 1e-3, 0.0])
    a, m, v, s, _, _ = _run([F0], [np.zeros(4)], [0.0], eta=0.01)
    assert np.all(a[0] == 0.0)
    np.testing.assert_array_equal(m[0], F0)
    np.testing.assert_array_equal(v[0], F0 ** 2)
    np.testing.assert_allclose(s[0], -0.01 * F0 / (np.abs(F0) + 1e-8), rtol=1e-15)


def test_alpha_bound_from_clipping():
    g = np.random.Generator(np.random.PCG64(1))
    n = 64
    F = [g.normal(size=n) * g.uniform(0.1, 10, n) for _ in range(60)]
    dF = [g.normal(size=n) * 1e-3 for _ in range(60)]
    a, *_ = _run(F, dF, [1e-4] * 60)
    for i, ai in enumerate(a):
        assert np.all(ai <= i / (i + 1) + 1e-15)


def test_no_change_constant_magnitude_gives_running_mean():
    g = np.random.Generator(np.random.PCG64(2))
    c = np.array([0.5, 2.0, 3e-2])
    F = [c * g.choice([-1.0, 1.0], size=3) for _ in range(40)]
    zeros = [np.zeros(3)] * 40
    a, m, *_ = _run(F, zeros, [0.0] * 40)
    for i in range(40):
        np.testing.assert_allclose(a[i], i / (i + 1), rtol=1e-13)
        np.testing.assert_allclose(m[i], np.mean(F[: i + 1], axis=0), rtol=1e-12, atol=1e-15)


def test_startup_expansion_and_variance_of_the_sum():
    # supplement, start-up bias: <F_i>_M = sum_j [prod_{k>j} a_k] (1 - a_j) F_j
    #   + [prod_{k>=1} a_k] F_0 + sum_j [prod_{k>=j} a_k] dF_j ; and with
    # independent terms the variance of that sum is what Eq. 15 accumulates
    g = np.random.Generator(np.random.PCG64(3))
    n, T = 8, 25
    F = [g.normal(size=n) for _ in range(T)]
    dF = [g.normal(size=n) * 0.1 for _ in range(T)]
    n2 = [0.0] + list(g.uniform(1e-4, 1e-2, T - 1))
    a, m, v, _, varF, varD = _run(F, dF, n2)
    for i in range(T):
        expl = np.zeros(n)
        var = np.zeros(n)
        for j in range(i + 1):
            prod_after = np.prod([a[k] for k in range(j + 1, i + 1)], axis=0) if j < i else np.ones(n)
            wF = prod_after * (1 - a[j])  # a_0 = 0 makes this prod_{k>=1} a_k for j = 0
            expl += wF * F[j]
            var += wF ** 2 * varF[j]
            if j >= 1:
                wD = prod_after * a[j]
                expl += wD * dF[j]
                var += wD ** 2 * varD[j]
        np.testing.assert_allclose(m[i], expl, rtol=1e-10, atol=1e-13)
        np.testing.assert_allclose(v[i], var, rtol=1e-10, atol=1e-15)


def test_moment2_is_normalised_ewma_and_exact_on_constants():
    g = np.random.Generator(np.random.PCG64(4))
    b = 0.93
    mo = M.Moment2((3,), b)
    xs = []
    for t in range(1, 30):
        x = g.normal(size=3)
        xs.append(x)
        mo.step(x)
        w = np.array([b ** (t - 1 - k) for k in range(t)])
        ref = (w[:, None] * np.array(xs) ** 2).sum(0) / w.sum()
        np.testing.assert_allclose(mo.m2, ref, rtol=1e-12)
    mc = M.Moment2((2,), 0.99)
    for _ in range(50):
        mc.step(np.array([3.0, -0.25]))
        np.testing.assert_allclose(mc.m2, [9.0, 0.0625], rtol=1e-13)


def test_step_is_scale_invariant():
    g = np.random.Generator(np.random.PCG64(5))
    n, T = 16, 20
    F = [g.normal(size=n) for _ in range(T)]
    dF = [g.normal(size=n) * 0.1 for _ in range(T)]
    n2 = [0.0] + [1e-3] * (T - 1)
    _, _, _, s1, _, _ = _run(F, dF, n2)
    _, _, _, s2, _, _ = _run([f * 37.0 for f in F], [d * 37.0 for d in dF], n2)
    for x, y in zip(s1, s2):
        np.testing.assert_allclose(x, y, rtol=1e-6)


def test_optimizer_readings_zero_step_and_projection():
    lo, hi = np.zeros(3, np.float32), np.ones(3, np.float32)
    opt = M.MetaOptimizer(np.array([0.5, 0.999, 0.2], np.float32), lo, hi, eta=0.01)
    opt.step(np.array([1.0, -1.0, 0.0]), None)
    # projection onto the box, ||dpi|| of the applied step
    assert opt.params[1] == np.float32(1.0)
    applied = opt.params.astype(np.float64) - np.array([0.5, 0.999, 0.2], np.float32)
    np.testing.assert_allclose(opt.step_norm2, np.sum(applied ** 2), rtol=1e-15)
    # a zero step: the next finite-difference sample is ignored, Var_D does not step
    opt2 = M.MetaOptimizer(np.array([0.5], np.float32), lo[:1], hi[:1], eta=0.0)
    opt2.step(np.array([1.0]), None)
    assert opt2.step_norm2 == 0.0
    opt2.step(np.array([1.0]), np.array([123.0]))
    assert opt2.var_D.count == 0
    np.testing.assert_allclose(opt2.meta.mean, [1.0])


def test_adam_matches_torch():
    torch = pytest.importorskip("torch")
    g = np.random.Generator(np.random.PCG64(6))
    p0 = g.uniform(0.2, 0.8, 10).astype(np.float32)
    lo, hi = np.full(10, -10, np.float32), np.full(10, 10, np.float32)
    ref = M.Adam(p0, lo, hi, eta=0.01)
    tp2 = torch.tensor(p0.astype(np.float64), requires_grad=True)
    topt2 = torch.optim.Adam([tp2], lr=0.01)
    g2 = np.random.Generator(np.random.PCG64(7))
    for _ in range(25):
        gr = g2.normal(size=10)
        ref.step(gr)
        tp2.grad = torch.tensor(gr)
        topt2.step()
    np.testing.assert_allclose(ref.params, tp2.detach().numpy(), rtol=0, atol=2e-6)


def test_toy_exponential_rate_converges():
    # Figure 2: fit Exp(lambda) so its mean is 2.0 -> lambda = 0.5
    finals = [M.toy_run("meta", 400, seed=s, lam0=1.0, eta=0.02)[-50:].mean() for s in range(6)]
    assert abs(np.mean(finals) - 0.5) < 0.02
    adam = [M.toy_run("adam", 400, seed=s, lam0=1.0, eta=0.02)[-50:] for s in range(6)]
    meta = [M.toy_run("meta", 400, seed=s, lam0=1.0, eta=0.02)[-50:] for s in range(6)]
    # the meta-estimator's iterates fluctuate less around the optimum than Adam's
    assert np.mean([m.std() for m in meta]) < np.mean([a.std() for a in adam])
