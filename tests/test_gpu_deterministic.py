"""The deterministic mode (JSO_F_DETERMINISTIC): gradient sums in 64-bit fixed
point with integer atomics, so results are bitwise reproducible:

  * many problems in one launch == each problem alone (survey T15);
  * every launch configuration (tile shape, persistent grid) gives the same
    bits (T16: radiance is bitwise equal in any mode, gradients here too);
  * a captured-graph batch == the same launches issued directly, and a run
    resumed from a checkpoint == the uninterrupted run (T17);
  * the fixed-point sums agree with the FP32-atomic sums and with the oracle
    at the usual tolerances.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2309_15676_amd import inputs as I
from test_gpu_parity import _check_grad, _oracle_pair, _set_pair, _gradient_mask

pytestmark = pytest.mark.gpu

DET = 16  # JSO_F_DETERMINISTIC
KEYS = ("params", "params_prev", "mean", "var", "alpha_prev", "m2_F", "m2_D", "adam_m", "adam_v")


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


def _specs():
    """A global material, a texture, a ragged image and a textured mesh."""
    tiny, gt, init = I.config_tiny()
    tiny.width, tiny.height = 40, 24
    t1 = I.scene_textured(48, 32, 16, seed=1, depth=4, rr_start=3)
    t2 = I.scene_textured(37, 21, 8, seed=2, depth=6, rr_start=3)
    v, t = I.heightfield(12, amp=0.3, seed=4)
    m = I.SceneSpec(width=40, height=32, plane_enabled=False, verts=v, tris=t,
                    mesh_mat=I.MAT_PARAM, spheres=np.array([[-1.0, 1.2, 0.0, 0.6]]),
                    sphere_mat=np.array([I.MAT_PARAM], np.int32), depth=5, rr_start=3,
                    tex_w=16, tex_h=16, ch_mask=I.CH_RGB_ROUGH,
                    fixed_default=(0.5, 0.5, 0.5, 0.0, 0.5))
    return [(tiny, np.asarray(gt, np.float32), np.asarray(init, np.float32)),
            (t1, I.fourier_params(t1, 1), I.uniform_params(t1, 2, 0.2, 0.8)),
            (t2, I.fourier_params(t2, 3), I.uniform_params(t2, 4, 0.2, 0.8)),
            (m, I.fourier_params(m, 1), I.uniform_params(m, 2, 0.2, 0.8))]


def _make(ctx, specs=None):
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd.problem import Problem
    probs = []
    for spec, gt, init in (specs or _specs()):
        p = Problem(spec, context=ctx)
        p.set_target(p.render(gt, seed=9, iteration=0, tag=L.JSO_TAG_TARGET, spp=16))
        p.set_params(init)
        probs.append(p)
    return probs


def _same(a, b, what):
    for k in KEYS:
        assert np.array_equal(np.asarray(a[k]), np.asarray(b[k])), "%s: %s differs" % (what, k)
    for k in ("iteration", "count_F", "count_D", "adam_t"):
        assert a[k] == b[k], (what, k)


def _opts(optimizer="meta", **kw):
    from paper_2309_15676_amd import _lib as L
    opt = L.JSO_OPT_META if optimizer == "meta" else L.JSO_OPT_ADAM
    return L.step_opts(optimizer=opt, eta=0.02, adam_spp=3, seed=41, flags=DET, **kw)


@pytest.mark.parametrize("optimizer", ["meta", "adam"])
def test_batch_equals_each_problem_alone_bitwise(ctx, optimizer):
    from paper_2309_15676_amd.problem import grad_step_many
    _say("deterministic batch == alone", optimizer)
    opts = _opts(optimizer)
    together, alone = _make(ctx), _make(ctx)
    for _ in range(3):
        grad_step_many(together, opts)
        for p in alone:
            p.grad_step(opts)
    for k in range(len(alone)):
        _same(together[k].get_state(), alone[k].get_state(), "problem %d" % k)


def test_every_launch_configuration_gives_the_same_bits(ctx):
    import torch
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd.problem import grad_step_many
    _say("deterministic launch configurations")
    # spp_prop 3: a configuration hash no tuner run of this process has touched
    opts = _opts(spp_prop=3)
    ref = None
    try:
        for config in (0, 1, 2, 4, 11):
            L.jso_set_launch_config(ctx.bind(), config)
            probs = _make(ctx)
            for _ in range(2):
                grad_step_many(probs, opts)
            states = [p.get_state() for p in probs]
            # the replayed adjoint of one render (jso_render_bwd)
            spec, gt, init = _specs()[1]
            dimg = torch.from_numpy(I.target_image_synthetic(spec, 5) - 0.7).cuda()
            g = probs[1].render_bwd(init, dimg, seed=3, iteration=1, tag=L.JSO_TAG_EVAL, spp=2,
                                    flags=DET).cpu().numpy()
            if ref is None:
                ref = (states, g)
                continue
            for k in range(len(states)):
                _same(states[k], ref[0][k], "config %d problem %d" % (config, k))
            assert np.array_equal(g, ref[1]), "render_bwd, config %d" % config
    finally:
        L.jso_set_launch_config(ctx.bind(), 0)


def test_graph_replay_equals_direct_launches_bitwise(ctx):
    from paper_2309_15676_amd.problem import Batch
    _say("deterministic graph == eager")
    opts = _opts()
    a, b = _make(ctx), _make(ctx)
    ba = Batch(a, opts, use_graph=True)
    bb = Batch(b, opts, use_graph=False)
    ba.step(3)
    bb.step(3)
    ba.close()
    bb.close()
    for k in range(len(a)):
        _same(a[k].get_state(), b[k].get_state(), "problem %d" % k)


@pytest.mark.parametrize("optimizer", ["meta", "adam"])
def test_resume_from_checkpoint_is_bitwise_exact(ctx, optimizer):
    from paper_2309_15676_amd.problem import Problem
    _say("deterministic checkpoint/resume", optimizer)
    opts = _opts(optimizer)
    spec, gt, init = _specs()[1]
    T = I.target_image_synthetic(spec, 4)
    a = Problem(spec, context=ctx)
    a.set_target(T)
    a.set_params(init)
    for _ in range(4):
        a.grad_step(opts)
    ck = a.get_state()
    for _ in range(3):
        a.grad_step(opts)
    b = Problem(spec, context=ctx)
    b.set_target(T)
    b.set_state(ck)
    for _ in range(3):
        b.grad_step(opts)
    _same(a.get_state(), b.get_state(), "resumed")


def test_fixed_point_sums_agree_with_float_atomics_and_oracle(ctx):
    import torch
    from paper_2309_15676_amd.problem import Problem
    _say("deterministic vs float atomics vs oracle")
    spec = I.scene_textured(64, 48, 32, seed=0, depth=6, rr_start=3)
    p = I.fourier_params(spec, 1)
    g = np.random.Generator(np.random.PCG64(8))
    p_prev = np.clip(p + g.normal(0, 0.02, p.shape).astype(np.float32), 0.06, 0.99)
    T = I.target_image_synthetic(spec, 5)
    seed, it = 33, 6
    mask = _gradient_mask(spec, p, p_prev, T, seed, it)
    prob = Problem(spec, context=ctx)
    prob.set_target(T)
    _set_pair(prob, p, p_prev, it)
    dmask = torch.from_numpy(mask.reshape(-1)).cuda()
    rd = prob.estimate_gradients(seed, it, 2, 1, flags=DET, mask=dmask)
    rf = prob.estimate_gradients(seed, it, 2, 1, mask=dmask)
    rd2 = prob.estimate_gradients(seed, it, 2, 1, flags=DET, mask=dmask)
    for key in ("F", "dF"):
        d, f, d2 = (r[key].cpu().numpy() for r in (rd, rf, rd2))
        assert np.array_equal(d, d2), key  # the same call twice: the same bits
        scale = np.abs(f).max()
        assert np.abs(d - f).max() <= 1e-5 * scale, key
    ref, floor = _oracle_pair(spec, p, p_prev, T, seed, it, 0, mask)
    for key in ("F", "dF"):
        _check_grad(rd[key].cpu().numpy().astype(np.float64), ref[key], ref[key + "_abs"],
                    floor[key], key, spec)
    # equal parameter vectors: the finite-difference sample is exactly zero
    _set_pair(prob, p, p, it)
    r0 = prob.estimate_gradients(seed, it, 2, 1, flags=DET)
    assert np.all(r0["dF"].cpu().numpy() == 0.0)


def test_deterministic_mode_errors(ctx):
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd.problem import Problem
    _say("deterministic errors")
    spec, gt, init = I.config_volume(res=8, views=1, view_w=8, view_h=8)
    prob = Problem(spec, context=ctx)
    prob.set_target(prob.render(gt, seed=1, iteration=0, tag=L.JSO_TAG_TARGET, spp=2))
    rc, _ = L.jso_grad_step(prob.ctx, [prob.sid], _opts(), False)
    assert rc == L.JSO_E_UNSUPPORTED
    # the no-allocation entry point has no deterministic mode
    tspec, tgt, tinit = _specs()[1]
    tp = Problem(tspec, context=ctx)
    import torch
    d = torch.zeros(tspec.height, tspec.width, 3, device="cuda")
    g = torch.zeros(tp.n_params, device="cuda")
    pt = tp.params_tensor(tinit)
    rc = L.jso_render_bwd_noalloc(tp.ctx, tp.sid, pt.data_ptr(), 1, 1, L.JSO_TAG_EVAL, 1,
                                  d.data_ptr(), L.render_opts(DET), g.data_ptr())
    assert rc == L.JSO_E_UNSUPPORTED
