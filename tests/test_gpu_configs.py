"""GPU parity of configurations the other parity tests do not reach, against
the FP64 oracle on the same seeded inputs and random streams (tolerances and
masking as in test_gpu_parity):

  * a texture of all five channels (RGB, metalness, roughness: the large
    scene's layout, with its own scatter mapping of 20 lanes per vertex), with
    both forms of the finite-difference sample;
  * a crop of the 2048x2048 terrain scene itself (999,698 triangles, 512x512
    texture of five channels, depth 12);
  * a base colour at its lower bound 0 (the GGX + Lambert material; the
    Lambert-only test mode, whose BSDF value vanishes there, is an expected
    failure of the replay);
  * three uneven problems stepped together by one batched launch (captured
    graph and direct), each checked against the oracle's gradient samples and
    meta-estimator step.
"""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import meta as OM
from paper_2309_15676_amd import inputs as I
from test_gpu_parity import (RTOL, TAU, _check_grad, _check_radiance, _gradient_mask,
                             _neighbour_allowance, _oracle_pair, _set_pair)

pytestmark = pytest.mark.gpu


def _say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2309_15676_amd.problem import Context
    c = Context(0)
    yield c
    c.close()


def _problem(ctx, spec):
    from paper_2309_15676_amd.problem import Problem
    return Problem(spec, context=ctx)


def _five_channel(w=48, h=40, tex=16, seed=5):
    """Plane + spheres sharing one texture of RGB + metalness + roughness."""
    s = I.scene_textured(w, h, tex, seed=seed, depth=6, rr_start=3)
    s.ch_mask = I.CH_ALL
    assert s.n_ch == 5
    return s, I.fourier_params(s, 1), I.uniform_params(s, 2, 0.2, 0.8)


# ---------------------------------------------------------------------------
@pytest.mark.parametrize("flags", [0, O.NO_NEE])
def test_five_channel_texture_radiance(ctx, flags):
    _say("five-channel radiance", flags)
    spec, gt, init = _five_channel()
    prob = _problem(ctx, spec)
    img = prob.render(init, seed=21, iteration=4, tag=O.TAG_EVAL, spp=2,
                      flags=flags).cpu().numpy()
    pd = init.astype(np.float64)
    (ref, mg), floor = O.rounding_sensitivity(
        spec, lambda: O.render(spec, pd, 21, 4, O.TAG_EVAL, 2, flags)[0:2])
    _check_radiance(img, ref, mg, floor[0], max_unstable=0.01)


@pytest.mark.parametrize("fd_shared", [False, True])
@pytest.mark.parametrize("params", ["gt", "init"])
def test_five_channel_texture_gradients(ctx, fd_shared, params):
    import torch
    from paper_2309_15676_amd import _lib as L
    _say("five-channel gradients", "shared" if fd_shared else "replay", params)
    spec, gt, init = _five_channel()
    p = {"gt": gt, "init": init}[params]
    g = np.random.Generator(np.random.PCG64(8))
    lo, hi = spec.param_bounds()
    p_prev = np.clip(p + g.normal(0, 0.02, p.shape).astype(np.float32), lo, hi)
    T = I.target_image_synthetic(spec, 5)
    seed, it = 33, 6
    pd, ppd, Td = p.astype(np.float64), p_prev.astype(np.float64), T.astype(np.float64)
    oracle_pair = lambda m: O.rounding_sensitivity(  # noqa: E731
        spec, lambda: O.gradient_pair(spec, pd, ppd, Td, seed, it, mask=m, fd_shared=fd_shared))
    r0, f0 = oracle_pair(None)
    bad = (r0["margin"] <= TAU) | O.ill_conditioned(r0, f0)
    print("masked %.2f%% of pixels" % (100 * bad.mean()), flush=True)
    assert bad.mean() <= 0.06
    mask = bad.astype(np.uint8)
    ref, floor = oracle_pair(mask)
    prob = _problem(ctx, spec)
    prob.set_target(T)
    _set_pair(prob, p, p_prev, it)
    r = prob.estimate_gradients(seed, it, 2, 1, mask=torch.from_numpy(mask.reshape(-1)).cuda(),
                                fd_mode=L.JSO_FD_SHARED if fd_shared else L.JSO_FD_REPLAY)
    for key in ("F", "dF"):
        got = r[key].cpu().numpy().astype(np.float64)
        _check_grad(got, ref[key], ref[key + "_abs"], floor[key], key, spec)
        # every channel (RGB, metalness, roughness) receives gradients
        per_ch = np.abs(ref[key]).reshape(-1, 5).sum(0)
        assert (per_ch > 0).all(), per_ch


def test_five_channel_texture_fd_zero_for_equal_params(ctx):
    from paper_2309_15676_amd import _lib as L
    _say("five-channel fd zero")
    spec, gt, init = _five_channel()
    prob = _problem(ctx, spec)
    prob.set_target(I.target_image_synthetic(spec, 1))
    for mode in (L.JSO_FD_REPLAY, L.JSO_FD_SHARED):
        _set_pair(prob, init, init, 9)
        r = prob.estimate_gradients(seed=4, iteration=9, fd_mode=mode)
        assert np.all(r["dF"].cpu().numpy() == 0.0), mode
        assert np.count_nonzero(r["F"].cpu().numpy()) > 0


# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def terrain(ctx):
    spec, gt, init = I.config_large()
    assert len(spec.tris) == 999698 and spec.width == 2048 and spec.depth == 12
    assert spec.n_params == 512 * 512 * 5
    return spec, gt, init, _problem(ctx, spec)


def test_terrain_crop_radiance(ctx, terrain):
    """A 16x16 crop of the 2048x2048 terrain scene in its own launch
    configuration, against the oracle's brute force over every triangle."""
    spec, gt, init, prob = terrain
    _say("terrain crop radiance")
    crop = (1016, 1100, 1032, 1116)
    img = prob.render(init, seed=5, iteration=3, tag=O.TAG_EVAL, spp=1, crop=crop).cpu().numpy()
    pd = init.astype(np.float64)
    (ref, mg), floor = O.rounding_sensitivity(
        spec, lambda: O.render(spec, pd, 5, 3, O.TAG_EVAL, 1, crop=crop)[0:2])
    sl = (slice(crop[1], crop[3]), slice(crop[0], crop[2]))
    assert (img[sl] > 0).any(-1).all()
    # depth-12 paths over a 1M-triangle mesh: FP32 hit positions drift by
    # many epsilons, so a sixth of the stable pixels (16.8% measured) need
    # the measured rounding floor beyond the plain 1e-4 (the worst at 0.15 of
    # the bound)
    _check_radiance(img[sl], ref[sl], mg[sl], floor[0][sl], max_unstable=0.05, max_strict=0.25)
    out = np.ones(img.shape[:2], bool)
    out[sl] = False
    assert np.all(img[out] == 0)


def test_terrain_crop_gradient(ctx, terrain):
    """The replayed adjoint on an 8x8 crop of the terrain scene (five-channel
    texels, depth 12) against the oracle's tape over brute-force hits."""
    import torch
    spec, gt, init, prob = terrain
    _say("terrain crop gradient")
    crop = (1020, 1104, 1028, 1112)
    pd = init.astype(np.float64)
    dimg = (I.target_image_synthetic(spec, 12) - 0.75).astype(np.float32)
    dd = dimg.astype(np.float64)
    (_, _, mg, A), fl = O.rounding_sensitivity(
        spec, lambda: (None, None) + O.render_bwd(spec, pd, dd, 5, 3, O.TAG_EVAL, 1,
                                                  crop=crop)[2:4])
    mask = ((mg <= TAU) | O.ill_conditioned({"A": A}, {"A": fl[3]})).astype(np.uint8)
    sl = (slice(crop[1], crop[3]), slice(crop[0], crop[2]))
    assert mask[sl].mean() <= 0.1, mask[sl].mean()
    (gref, gabs, _, _), gfl = O.rounding_sensitivity(
        spec, lambda: O.render_bwd(spec, pd, dd, 5, 3, O.TAG_EVAL, 1, crop=crop,
                                   mask=mask)[0:2] + (None, None))
    gg = prob.render_bwd(init, torch.from_numpy(dimg).cuda(), 5, 3, O.TAG_EVAL, 1, crop=crop,
                         mask=torch.from_numpy(mask.reshape(-1)).cuda())
    _check_grad(gg.cpu().numpy().astype(np.float64), gref, gabs, gfl[0], "terrain render_bwd",
                spec)
    assert np.count_nonzero(gref) > 50
    assert (np.abs(gref).reshape(-1, 5).sum(0) > 0).all()


# ---------------------------------------------------------------------------
def _zero_colour_case(which):
    if which == "global":
        spec, gt, init = I.config_tiny()
        spec.width, spec.height = 32, 24
        p = np.asarray(gt, np.float32).copy()
        p[[0, 2]] = 0.0  # red and blue base colour at their bound
        return spec, p
    spec = I.scene_textured(40, 32, 8, seed=2, depth=5, rr_start=3)
    p = I.fourier_params(spec, 3)
    p[0::spec.n_ch][::2] = 0.0  # every other texel's red channel
    return spec, p


LAMBERT_ZERO = pytest.mark.xfail(strict=True, reason=(
    "Lambert-only test mode at a base colour of exactly 0: the BSDF value of "
    "that channel vanishes, and the replay, which recovers the radiance a "
    "vertex's continuation carries from the path's remainder divided by f, "
    "drops the continuation derivative there (NEE derivatives are kept). The "
    "method's GGX + Lambert material never vanishes (its specular lobe has "
    "F >= F0 > 0), so the published material is unaffected"))


@pytest.mark.parametrize("which", ["global", "textured"])
@pytest.mark.parametrize("fd_shared", [False, True])
@pytest.mark.parametrize("flags", [0, pytest.param(O.LAMBERT_ONLY, marks=LAMBERT_ZERO)])
def test_base_colour_at_zero(ctx, which, fd_shared, flags):
    """Base-colour parameters at their lower bound 0 (where the projection
    puts them): gradient parity, and the derivative of those parameters is
    delivered (nonzero in the oracle, matched by the GPU)."""
    import torch
    from paper_2309_15676_amd import _lib as L
    _say("base colour 0", which, fd_shared, flags)
    spec, p = _zero_colour_case(which)
    lo, hi = spec.param_bounds()
    g = np.random.Generator(np.random.PCG64(4))
    p_prev = np.clip(p + g.normal(0, 0.02, p.shape).astype(np.float32), lo, hi)
    p_prev[p == 0.0] = 0.0  # both parameter vectors at the bound there
    T = I.target_image_synthetic(spec, 7)
    seed, it = 13, 4
    pd, ppd, Td = p.astype(np.float64), p_prev.astype(np.float64), T.astype(np.float64)
    oracle_pair = lambda m: O.rounding_sensitivity(  # noqa: E731
        spec, lambda: O.gradient_pair(spec, pd, ppd, Td, seed, it, flags=flags, mask=m,
                                      fd_shared=fd_shared))
    r0, f0 = oracle_pair(None)
    mask = ((r0["margin"] <= TAU) | O.ill_conditioned(r0, f0)).astype(np.uint8)
    assert mask.mean() <= 0.03
    ref, floor = oracle_pair(mask)
    prob = _problem(ctx, spec)
    prob.set_target(T)
    _set_pair(prob, p, p_prev, it)
    r = prob.estimate_gradients(seed, it, 2, 1, flags=flags,
                                mask=torch.from_numpy(mask.reshape(-1)).cuda(),
                                fd_mode=L.JSO_FD_SHARED if fd_shared else L.JSO_FD_REPLAY)
    zero = np.flatnonzero(p == 0.0)
    for key in ("F", "dF"):
        got = r[key].cpu().numpy().astype(np.float64)
        _check_grad(got, ref[key], ref[key + "_abs"], floor[key], key, spec)
    # the parameters at the bound receive their (nonzero) derivative
    Fz = ref["F"][zero]
    assert np.count_nonzero(Fz) > 0
    got = r["F"].cpu().numpy().astype(np.float64)[zero]
    big = np.abs(Fz) > 0.1 * ref["F_abs"][zero]
    assert big.any()
    np.testing.assert_allclose(got[big], Fz[big], rtol=1e-3)


# ---------------------------------------------------------------------------
def _uneven():
    """Three uneven problems: a global material, a texture, a ragged image."""
    tiny, gt, init = I.config_tiny()
    tiny.width, tiny.height = 40, 24
    t1 = I.scene_textured(48, 32, 16, seed=1, depth=4, rr_start=3)
    t2 = I.scene_textured(37, 21, 8, seed=2, depth=6, rr_start=3)
    return [(tiny, np.asarray(init, np.float32)), (t1, I.uniform_params(t1, 2, 0.2, 0.8)),
            (t2, I.uniform_params(t2, 4, 0.2, 0.8))]


def _fresh_state(prob, p, p_prev, it):
    """Optimiser state at iteration `it` with empty averages: after one step
    m2_F = <F>^2 and m2_D ||dpi||^2 = <dF>^2 exactly (first samples)."""
    st = prob.get_state()
    P = len(p)
    d = p.astype(np.float64) - p_prev.astype(np.float64)
    st.update(params=np.asarray(p, np.float32), params_prev=np.asarray(p_prev, np.float32),
              mean=np.zeros(P), var=np.zeros(P), alpha_prev=np.zeros(P), m2_F=np.zeros(P),
              m2_D=np.zeros(P), iteration=it, count_F=0, count_D=0,
              step_norm2=float(np.dot(d, d)))
    prob.set_state(st)
    return st["step_norm2"]


@pytest.mark.parametrize("mode", ["graph", "direct"])
def test_batched_problems_match_oracle(ctx, mode):
    """One batched iteration of three uneven problems (one launch per kernel
    for all of them) against the oracle: each problem's gradient samples, as
    the optimiser state reveals them, and its meta-estimator step.

    The batched step takes no pixel mask, so the few pixels whose paths take
    an FP32-unstable decision stay in: their oracle contribution (sum|contrib|
    over those pixels alone) is added, twice, to the tolerance of the
    parameters they touch."""
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd.problem import Batch, grad_step_many
    _say("batched vs oracle", mode)
    f32 = lambda v: float(np.float32(v))  # noqa: E731
    eta, bF, bD, seed, it = f32(0.01), f32(0.99), f32(0.9), 17, 5
    opts = L.step_opts(optimizer=L.JSO_OPT_META, eta=eta, beta_F=bF, beta_D=bD, seed=seed)
    probs, cases = [], []
    for k, (spec, p) in enumerate(_uneven()):
        lo, hi = spec.param_bounds()
        g = np.random.Generator(np.random.PCG64(20 + k))
        p_prev = np.clip(p + g.normal(0, 0.02, p.shape).astype(np.float32), lo, hi)
        T = I.target_image_synthetic(spec, 30 + k)
        prob = _problem(ctx, spec)
        prob.set_target(T)
        norm2 = _fresh_state(prob, p, p_prev, it)
        probs.append(prob)
        cases.append((spec, p, p_prev, T, norm2, lo, hi))
    if mode == "graph":
        b = Batch(probs, opts, use_graph=True)
        b.step(1)
        b.close()
    else:
        grad_step_many(probs, opts)
    needing = 0
    total = 0
    for prob, (spec, p, p_prev, T, norm2, lo, hi) in zip(probs, cases):
        st = prob.get_state()
        assert st["iteration"] == it + 1 and st["count_F"] == 1 and st["count_D"] == 1
        ref, floor = _oracle_pair(spec, p, p_prev, T, seed, it)
        bad = (ref["margin"] <= TAU) | O.ill_conditioned(ref, floor)
        only_bad = O.gradient_pair(spec, p.astype(np.float64), p_prev.astype(np.float64),
                                   T.astype(np.float64), seed, it, mask=(~bad).astype(np.uint8))
        tol = {}
        for key in ("F", "dF"):
            gabs = ref[key + "_abs"]
            tol[key] = (RTOL * gabs + 2 * floor[key] + 1e-12 * gabs.max() +
                        _neighbour_allowance(gabs, spec) + 2 * only_bad[key + "_abs"])
            needing += int((only_bad[key + "_abs"] > RTOL * gabs).sum())
            total += len(gabs)
        # the samples, as the first samples of the two averages reveal them
        F_gpu = np.sqrt(st["m2_F"])
        dF_gpu = np.sqrt(st["m2_D"] * norm2)
        for name, got, want, t in (("|F|", F_gpu, np.abs(ref["F"]), tol["F"]),
                                   ("|dF|", dF_gpu, np.abs(ref["dF"]), tol["dF"])):
            worst = int(np.argmax(np.abs(got - want) - t))
            assert np.all(np.abs(got - want) <= t), "%s param %d: %g vs %g (tol %g)" % (
                name, worst, got[worst], want[worst], t[worst])
        # the meta-estimator step of the oracle from the oracle's samples
        opt = OM.MetaOptimizer(p, lo, hi, eta, bF, bD)
        opt.params_prev = np.asarray(p_prev, np.float32)
        opt.iteration = it
        opt.step_norm2 = norm2
        opt.meta.i = it
        opt.meta.alpha_last = np.zeros(len(p))
        opt.step(ref["F"], ref["dF"])
        scale = np.abs(ref["F"]) + np.abs(ref["dF"])
        rel = np.minimum((tol["F"] + tol["dF"]) / np.maximum(scale, 1e-300), 1.0)
        # mean: a convex blend of <dF> and <F> (alpha <= 1/2)
        assert np.all(np.abs(st["mean"] - opt.meta.F_M) <= 2 * (tol["F"] + tol["dF"]))
        np.testing.assert_allclose(st["alpha_prev"][rel < 1e-3], opt.meta.alpha_last[rel < 1e-3],
                                   rtol=0, atol=1e-2)
        # the step is scale-free in (F, dF): a relative change r of the samples
        # moves it by at most ~4 r eta (and never by more than the full 2 eta)
        dp = np.abs(st["params"].astype(np.float64) - opt.params.astype(np.float64))
        assert np.all(dp <= np.minimum(4 * rel, 2.0) * eta + 1e-6), float(
            (dp / (np.minimum(4 * rel, 2.0) * eta + 1e-6)).max())
        np.testing.assert_array_equal(st["params_prev"], p)
    print("parameters needing the unstable-pixel allowance: %.2f%%" % (100 * needing / total),
          flush=True)
    # measured: 18% of these small textures' parameters are touched by an
    # unstable pixel (every texel a deep path crosses); the rest meet the
    # plain per-parameter bound
    assert needing <= 0.25 * total
