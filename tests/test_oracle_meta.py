"""Pins of the meta-estimator / optimiser oracle (oracle/meta.py), CPU only.

Each check is a property the paper states, a value worked out by hand, or a
closed form that follows from the method by a different route than the
recurrence:
  * Hand-worked three iterations (tests/golden/meta_three_iterations.txt):
    alpha_1 < 1/2, so Eq. 17's bound 1 / (2 - alpha_1) differs from Eq. 16's
    1 - 1/(i + 1) at i = 2.
  * Hand-worked start-up corrected averages (golden decayed_moment_beta_half).
  * Eq. 7 initialisation: <F_0>_M = <F_0>, alpha_0 = 0.
  * Eq. 16 follows from Eq. 17 with alpha_0 = 0: alpha_i <= i / (i + 1).
  * With no parameter change (<dF> = 0) and samples of constant magnitude the
    meta-estimate is the running mean of all proportional samples.
  * Supplement, start-up bias: <F_i>_M is the explicit weighted sum of all
    <F_j> and <dF_j> with products of alphas; Eq. 15 is the variance of that
    sum for independent samples with the approximated variances.
  * The average is the normalised exponentially weighted sum of x^2.
  * Eq. 21 is invariant to rescaling all gradient samples (up to epsilon).
  * Adam agrees with torch.optim.Adam (float64, CPU).
  * Figure 2 toy: the meta-estimator reaches the ground-truth rate 0.5.
  * Experiments, "Approximation accuracy": along an exponentially decaying
    change the meta-estimate's actual error stays within 0.5-2x its
    predicted standard deviation (1000+ independent runs).
  * Experiments, "Variance reduction without lag": along a linear change the
    meta-estimate has no lag, Adam's first moment does.
  * Limitations: Var[<dF>] is quadratic in the step size (log-log slope 2)
    for the renderer's finite-difference sample (oracle path tracer).
"""
import math
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import meta as M

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _table(name):
    rows = []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if not line:
                continue
            left, right = line.split("|")
            rows.append(([Fraction(t) for t in left.split()], [Fraction(t) for t in right.split()]))
    return rows


def _run(F_seq, dF_seq, n2_seq, eta=1e-3, bF=0.99, bD=0.9, clip=True):
    """Drive the averages and the meta-estimate directly (no parameters)."""
    n = F_seq[0].shape
    vf, vd, mt = M.DecayedMoment(n, bF), M.DecayedMoment(n, bD), M.MetaEstimate(n, clip)
    alphas, means, vars_, steps, varF, varD = [], [], [], [], [], []
    for i, (F, dF, n2) in enumerate(zip(F_seq, dF_seq, n2_seq)):
        vf.push(F)
        if i >= 1 and n2 > 0:
            vd.push(dF / math.sqrt(n2))
            vdf = vd.estimate * n2
        else:
            dF = np.zeros_like(F)
            vdf = np.zeros_like(F)
        mt.update(F, dF, vf.estimate, vdf)
        steps.append(M.stabilised_step(eta, mt.F_M, mt.V_M))
        alphas.append(mt.alpha_last.copy())
        means.append(mt.F_M.copy())
        vars_.append(mt.V_M.copy())
        varF.append(vf.estimate.copy())
        varD.append(np.array(vdf, copy=True))
    return alphas, means, vars_, steps, varF, varD


def test_hand_worked_three_iterations_eq17():
    rows = _table("meta_three_iterations.txt")
    est = M.MetaEstimate((1,))
    for (i, F, dF, vF, vdF), (alpha, F_M, V_M) in rows:
        est.update(np.array([float(F)]), np.array([float(dF)]), np.array([float(vF)]),
                   np.array([float(vdF)]))
        assert est.alpha_last[0] == pytest.approx(float(alpha), rel=1e-15, abs=0), int(i)
        assert est.F_M[0] == pytest.approx(float(F_M), rel=1e-15), int(i)
        assert est.V_M[0] == pytest.approx(float(V_M), rel=1e-15), int(i)
    # the stabilised step from the last row (Eq. 21)
    F_M, V_M = rows[-1][1][1], rows[-1][1][2]
    want = -0.1 * float(F_M) / (math.sqrt(float(V_M)) + 1e-8)
    assert M.stabilised_step(0.1, est.F_M, est.V_M)[0] == pytest.approx(want, rel=1e-15)


def test_hand_worked_three_iterations_without_clip():
    # the ablation keeps Eq. 8's 15/16 at i = 2 (and alpha_0 = 0)
    rows = _table("meta_three_iterations.txt")
    est = M.MetaEstimate((1,), clip=False)
    alphas = []
    for (i, F, dF, vF, vdF), _ in rows:
        est.update(np.array([float(F)]), np.array([float(dF)]), np.array([float(vF)]),
                   np.array([float(vdF)]))
        alphas.append(est.alpha_last[0])
    assert alphas == pytest.approx([0.0, 1.0 / 3.0, 15.0 / 16.0], rel=1e-15)


def test_hand_worked_decayed_moment():
    mo = M.DecayedMoment((1,), 0.5)
    for (n, x), (want,) in _table("decayed_moment_beta_half.txt"):
        mo.push(np.array([float(x)]))
        assert mo.n == int(n)
        assert mo.estimate[0] == pytest.approx(float(want), rel=1e-15)


def test_first_iteration_is_the_proportional_sample():
    F0 = np.array([0.3, -2.0, 1e-3, 0.0])
    a, m, v, s, _, _ = _run([F0], [np.zeros(4)], [0.0], eta=0.01)
    assert np.all(a[0] == 0.0)
    np.testing.assert_array_equal(m[0], F0)
    np.testing.assert_array_equal(v[0], F0 ** 2)
    np.testing.assert_allclose(s[0], -0.01 * F0 / (np.abs(F0) + 1e-8), rtol=1e-15)


def test_untouched_parameter_has_zero_weight():
    # a parameter whose samples have all been zero: Eq. 8 is 0/0, alpha = 0,
    # the estimate stays 0 and so does the step
    z = [np.zeros(2)] * 4
    a, m, v, s, _, _ = _run(z, z, [0.0, 1e-3, 1e-3, 1e-3])
    for i in range(4):
        np.testing.assert_array_equal(a[i], 0.0)
        np.testing.assert_array_equal(m[i], 0.0)
        np.testing.assert_array_equal(s[i], 0.0)


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


def test_average_is_normalised_ewma_and_exact_on_constants():
    g = np.random.Generator(np.random.PCG64(4))
    b = 0.93
    mo = M.DecayedMoment((3,), b)
    xs = []
    for t in range(1, 30):
        x = g.normal(size=3)
        xs.append(x)
        mo.push(x)
        w = np.array([b ** (t - 1 - k) for k in range(t)])
        ref = (w[:, None] * np.array(xs) ** 2).sum(0) / w.sum()
        np.testing.assert_allclose(mo.estimate, ref, rtol=1e-12)
    mc = M.DecayedMoment((2,), 0.99)
    for _ in range(50):
        mc.push(np.array([3.0, -0.25]))
        np.testing.assert_allclose(mc.estimate, [9.0, 0.0625], rtol=1e-13)


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
    # a zero step: the next finite-difference sample is ignored, Var_D takes no sample
    opt2 = M.MetaOptimizer(np.array([0.5], np.float32), lo[:1], hi[:1], eta=0.0)
    opt2.step(np.array([1.0]), None)
    assert opt2.step_norm2 == 0.0
    opt2.step(np.array([1.0]), np.array([123.0]))
    assert opt2.var_D.n == 0
    np.testing.assert_allclose(opt2.meta.F_M, [1.0])


def test_optimizer_first_two_iterations_closed_form():
    # i = 1 worked through the loop: Var[F_1] = F_0^2 + (F_1^2 - F_0^2) / (1 + beta_F)
    # (start-up corrected weights beta_F / (1 + beta_F), 1 / (1 + beta_F)),
    # Var[dF_1] = <dF_1>^2 exactly (one sample of the decoupled average,
    # rescaled by ||dpi_1||^2), alpha_1 = min(Var[F_1] / (Var[F_1] + F_0^2
    # + <dF_1>^2), 1/2)
    bF = 0.9
    F0, F1, dF1 = np.array([0.4, -1.0]), np.array([0.1, -3.0]), np.array([0.05, 0.2])
    opt = M.MetaOptimizer(np.array([0.5, 0.5], np.float32), np.zeros(2), np.ones(2),
                          eta=0.01, beta_F=bF)
    opt.step(F0, None)
    opt.step(F1, dF1)
    vF = F0 ** 2 + (F1 ** 2 - F0 ** 2) / (1 + bF)
    alpha = np.minimum(vF / (vF + F0 ** 2 + dF1 ** 2), 0.5)
    np.testing.assert_allclose(opt.meta.alpha_last, alpha, rtol=1e-14)
    np.testing.assert_allclose(opt.meta.F_M, alpha * (F0 + dF1) + (1 - alpha) * F1, rtol=1e-14)


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


def test_toy_gradient_estimator_is_unbiased():
    # the decorrelated product of two half-sample means is unbiased for
    # d/dlam (E[x] - 2)^2 (checked against the closed form)
    g = np.random.Generator(np.random.PCG64(11))
    for lam in (0.5, 0.7, 1.3):
        est = M.toy_grad(np.full(20000, lam), g.random((20000, 32)))
        se = est.std() / math.sqrt(est.size)
        assert abs(est.mean() - M.toy_true_grad(lam)) < 4 * se + 1e-12


def test_approximation_accuracy_within_half_to_twice_predicted_sigma():
    # Experiments, "Approximation accuracy": an exponentially decaying change
    # of the gradient (no optimiser), 2000 independent runs as ground truth;
    # the meta-estimate's RMS error around the true gradient stays within
    # 0.5-2x the standard deviation it predicts (Var[F_i]_M, Eq. 15) once the
    # averages hold a few samples.  Low signal-to-noise gradients, the regime
    # the zero-centred averages are designed for ("Zero-centred EMAs").
    i = np.arange(200)
    lam = 0.5 + 0.1 * np.exp(-i / 20.0)
    F_M, V_M, _, _ = M.toy_track(lam, runs=2000, seed=1)
    true = np.array([M.toy_true_grad(l) for l in lam])
    rms = np.sqrt(((F_M - true[:, None]) ** 2).mean(axis=1))
    ratio = rms / np.sqrt(V_M.mean(axis=1))
    assert ratio[10:].min() > 0.5 and ratio[10:].max() < 2.0, (ratio[10:].min(), ratio[10:].max())


def test_no_lag_under_linear_change():
    # Experiments, "Variance reduction without lag": a fixed linear change
    # of the parameter over 100 iterations, no optimiser.  The finite
    # differences carry the estimate along, so its mean follows the true
    # gradient; Adam's first moment lags behind it; and the meta-estimate
    # varies less from run to run.
    lam = np.linspace(1.0, 0.5, 100)
    F_M, _, m_hat, _ = M.toy_track(lam, runs=2000, seed=2)
    true = np.array([M.toy_true_grad(l) for l in lam])
    bias_meta = np.abs(F_M.mean(axis=1) - true)[10:]
    bias_adam = np.abs(m_hat.mean(axis=1) - true)[10:]
    se_meta = F_M.std(axis=1)[10:] / math.sqrt(F_M.shape[1])
    assert np.all(bias_meta < 5 * se_meta + 1e-3), bias_meta.max()
    assert bias_meta.max() < 0.05 * bias_adam.max()
    assert np.all(F_M.std(axis=1)[10:] < m_hat.std(axis=1)[10:])


@pytest.fixture(scope="module")
def tiny_fd_scene():
    import oracle as O
    from paper_2309_15676_amd import inputs as I
    spec, _, init = I.config_tiny()
    spec.width = spec.height = 16
    T = I.target_image_synthetic(spec, 3).astype(np.float64)
    return O, spec, np.asarray(init, np.float64), T


def _fd_variance(O, spec, p, T, d, hs, seeds, shared):
    out = []
    for h in hs:
        samples = [O.gradient_pair(spec, p, p - h * d, T, 100 + s, 1, 1, 1, fd_shared=shared)["dF"]
                   for s in range(seeds)]
        out.append(np.var(np.array(samples), axis=0).sum())
    return np.array(out)


@pytest.mark.parametrize("name,direction", [("colour", (1, 1, 1, 0, 0)), ("metal", (0, 0, 0, 1, 0))])
def test_fd_variance_quadratic_in_step_for_colour_and_metal(tiny_fd_scene, name, direction):
    # Limitations: Var[<dF>] must be quadratic in the step size.  Base colour
    # and metalness do not move the sampled paths, so the finite difference is
    # a smooth function of the step: log-log slope 2 for both forms.
    O, spec, p, T = tiny_fd_scene
    d = np.asarray(direction, np.float64)
    d /= np.linalg.norm(d)
    hs = np.array([1e-3, 1e-2, 1e-1])
    for shared in (False, True):
        v = _fd_variance(O, spec, p, T, d, hs, 60, shared)
        slope = np.diff(np.log(v)) / np.diff(np.log(hs))
        assert np.all(np.abs(slope - 2.0) < 0.1), (name, shared, slope)


def test_fd_variance_roughness_step(tiny_fd_scene):
    # A roughness step moves the GGX-sampled directions.  Eq. 5 as written
    # (one path, the integrand at both parameter vectors) stays quadratic;
    # replaying the random numbers at both parameters lets a moved path cross
    # an edge of the scene with probability O(h) and an O(1) jump, so for
    # small steps its variance falls only linearly: the concern the
    # Limitations section raises for finite-difference estimators.
    O, spec, p, T = tiny_fd_scene
    d = np.array([0, 0, 0, 0, 1.0])
    hs = np.array([1e-3, 3e-3])
    shared = _fd_variance(O, spec, p, T, d, hs, 80, True)
    replay = _fd_variance(O, spec, p, T, d, hs, 80, False)
    s_shared = np.log(shared[1] / shared[0]) / np.log(3.0)
    s_replay = np.log(replay[1] / replay[0]) / np.log(3.0)
    assert abs(s_shared - 2.0) < 0.15, s_shared
    assert s_replay < 1.5, s_replay
