"""GPU tests of many problems per launch: jso_grad_step over several problems
and jso_batch (descriptors uploaded once, optional HIP graph replay) against
stepping each problem on its own.

Gradients are summed with float atomics, whose order depends on block
scheduling, so two runs of the same step agree to float rounding, not bit
for bit: states are compared with a tolerance of 1e-5 of each array's scale
(one step of rounding noise through the FP64 meta-estimator state)."""
import sys

import numpy as np
import pytest

from paper_2309_15676_amd import inputs as I

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


def _specs():
    """Three uneven problems: a global material, two textures of different
    sizes, one with a ragged image (not a multiple of the 16x16 tile)."""
    tiny, gt, init = I.config_tiny()
    tiny.width, tiny.height = 40, 24
    t1 = I.scene_textured(48, 32, 16, seed=1, depth=4, rr_start=3)
    t2 = I.scene_textured(37, 21, 8, seed=2, depth=6, rr_start=3)
    return [
        (tiny, np.asarray(gt, np.float32), np.asarray(init, np.float32)),
        (t1, I.fourier_params(t1, 1), I.uniform_params(t1, 2, 0.2, 0.8)),
        (t2, I.fourier_params(t2, 3), I.uniform_params(t2, 4, 0.2, 0.8)),
    ]


def _make(ctx):
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd.problem import Problem
    probs = []
    for spec, gt, init in _specs():
        p = Problem(spec, context=ctx)
        p.set_target(p.render(gt, seed=9, iteration=0, tag=L.JSO_TAG_TARGET, spp=16))
        p.set_params(init)
        probs.append(p)
    return probs


def _close_states(a, b, what):
    for key in ("params", "params_prev", "mean", "var", "m2_F", "m2_D"):
        x, y = np.asarray(a[key], np.float64), np.asarray(b[key], np.float64)
        scale = max(np.abs(y).max(), 1e-30)
        assert np.abs(x - y).max() <= 1e-5 * scale, "%s %s: %g" % (what, key,
                                                                np.abs(x - y).max() / scale)
    assert a["iteration"] == b["iteration"], what


@pytest.mark.parametrize("optimizer", ["meta", "adam"])
def test_grad_step_over_several_problems_matches_one_by_one(ctx, optimizer):
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd.problem import grad_step_many
    _say("grad_step several problems", optimizer)
    opt = L.JSO_OPT_META if optimizer == "meta" else L.JSO_OPT_ADAM
    opts = L.step_opts(optimizer=opt, eta=0.02, adam_spp=3, seed=11)
    together, alone = _make(ctx), _make(ctx)
    for it in range(3):
        st = grad_step_many(together, opts, want_stats=True)
        for k, p in enumerate(alone):
            s1 = p.grad_step(opts, want_stats=True)
            assert st[k].iteration == s1.iteration == it + 1
            assert abs(st[k].loss - s1.loss) <= 1e-6 * max(s1.loss, 1e-30)
        for k in range(len(alone)):
            _close_states(together[k].get_state(), alone[k].get_state(), "problem %d it %d" % (k, it))


@pytest.mark.parametrize("use_graph", [True, False])
def test_batch_matches_grad_step_and_stops_at_its_limit(ctx, use_graph):
    import torch
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd.problem import Batch, grad_step_many
    _say("batch", "graph" if use_graph else "eager")
    opts = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.02, seed=5)
    batched, ref = _make(ctx), _make(ctx)
    limits = [2, 0, 4]
    b = Batch(batched, opts, max_iters=limits, use_graph=use_graph)
    assert b.active() == 3
    for it in range(5):
        b.step(1)
        # eager work and a synchronisation between replays
        junk = batched[1].render(batched[1].get_params(), seed=1, iteration=0, tag=L.JSO_TAG_EVAL,
                                 spp=1)
        torch.cuda.synchronize()
        assert torch.isfinite(junk).all()
        live = [p for p, m in zip(ref, limits) if m == 0 or it < m]
        grad_step_many(live, opts)
        for k, p in enumerate(batched):
            want = min(it + 1, limits[k]) if limits[k] else it + 1
            sb, sr = p.get_state(), ref[k].get_state()
            assert sb["iteration"] == want, (k, sb["iteration"], want)
            _close_states(sb, sr, "graph=%s problem %d after %d" % (use_graph, k, it + 1))
    assert b.active() == 1
    b.close()


@pytest.mark.parametrize("shape", [1, 2])
def test_tile_shapes_agree(ctx, shape):
    """Every path is traced and replayed identically whatever the tile shape:
    the image is bit-identical and the gradient equal up to atomic order."""
    import torch
    from paper_2309_15676_amd import _lib as L
    _say("tile shape", shape)
    probs = _make(ctx)
    try:
        for p, (spec, gt, init) in zip(probs, _specs()):
            dimg = torch.from_numpy(I.target_image_synthetic(spec, 5) - 0.7).cuda()
            L.jso_set_launch_config(ctx.bind(), 0)
            img0 = p.render(init, seed=3, iteration=1, tag=L.JSO_TAG_EVAL, spp=2)
            g0 = p.render_bwd(init, dimg, seed=3, iteration=1, tag=L.JSO_TAG_EVAL, spp=2)
            L.jso_set_launch_config(ctx.bind(), shape)
            img1 = p.render(init, seed=3, iteration=1, tag=L.JSO_TAG_EVAL, spp=2)
            g1 = p.render_bwd(init, dimg, seed=3, iteration=1, tag=L.JSO_TAG_EVAL, spp=2)
            assert torch.equal(img0, img1)
            scale = float(g0.abs().max())
            assert float((g1 - g0).abs().max()) <= 1e-5 * scale
    finally:
        L.jso_set_launch_config(ctx.bind(), 0)


def test_autotune_restores_state_and_picks_a_shape(ctx):
    import torch
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd.problem import Batch, grad_step_many
    _say("autotune")
    opts = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.02, seed=8)
    probs, ref = _make(ctx), _make(ctx)
    b = Batch(probs, opts, use_graph=True)
    b.step(2)
    grad_step_many(ref, opts)
    grad_step_many(ref, opts)
    before = [p.get_state() for p in probs]
    best, ms = b.autotune(2)
    assert 0 <= best < L.JSO_LAUNCH_CONFIGS and len(ms) == L.JSO_LAUNCH_CONFIGS
    assert all(m > 0 for m in ms), (best, ms)
    for p, st in zip(probs, before):
        after = p.get_state()
        for key in ("params", "params_prev", "mean", "var", "m2_F", "m2_D", "alpha_prev"):
            assert np.array_equal(after[key], st[key]), key
        assert after["iteration"] == st["iteration"]
    # the tuned batch keeps optimising like the reference
    b.step(1)
    torch.cuda.synchronize()
    grad_step_many(ref, opts)
    for k in range(len(probs)):
        _close_states(probs[k].get_state(), ref[k].get_state(), "after autotune %d" % k)
    b.close()


def _specs_with_mesh():
    """The three uneven problems plus a textured heightfield mesh (BVH
    traversal in the same launches)."""
    out = _specs()
    v, t = I.heightfield(12, amp=0.3, seed=4)
    m = I.SceneSpec(width=40, height=32, plane_enabled=False, verts=v, tris=t,
                    mesh_mat=I.MAT_PARAM, spheres=np.array([[-1.0, 1.2, 0.0, 0.6]]),
                    sphere_mat=np.array([I.MAT_PARAM], np.int32), depth=5, rr_start=3,
                    tex_w=16, tex_h=16, ch_mask=I.CH_RGB_ROUGH,
                    fixed_default=(0.5, 0.5, 0.5, 0.0, 0.5))
    out.append((m, I.fourier_params(m, 1), I.uniform_params(m, 2, 0.2, 0.8)))
    return out


@pytest.mark.parametrize("config", [3, 7, 11, 14])
def test_persistent_launches_match_plain_grid(ctx, config):
    """A persistent grid (blocks pulling tiles from a work queue) traces and
    replays the same paths as one block per tile: the optimiser states of
    several steps agree up to atomic order, for jso_grad_step and for a
    batch replayed from a captured graph (the queue resets itself between
    launches and replays)."""
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd.problem import Batch, Problem, grad_step_many
    _say("persistent config", L.config_name(config))
    # spp_prop 3: a configuration hash of its own, so no tuned entry applies
    opts = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.02, seed=21, spp_prop=3)

    def make():
        ps = []
        for spec, gt, init in _specs_with_mesh():
            p = Problem(spec, context=ctx)
            p.set_target(p.render(gt, seed=9, iteration=0, tag=L.JSO_TAG_TARGET, spp=16))
            p.set_params(init)
            ps.append(p)
        return ps

    try:
        L.jso_set_launch_config(ctx.bind(), 0)
        ref = make()
        for _ in range(3):
            grad_step_many(ref, opts)
        L.jso_set_launch_config(ctx.bind(), config)
        direct = make()
        for _ in range(3):
            grad_step_many(direct, opts)
        graph = make()
        b = Batch(graph, opts, use_graph=True)
        b.step(3)
        b.close()
        for k in range(len(ref)):
            sr = ref[k].get_state()
            _close_states(direct[k].get_state(), sr, "direct %s problem %d" % (config, k))
            _close_states(graph[k].get_state(), sr, "graph %s problem %d" % (config, k))
    finally:
        L.jso_set_launch_config(ctx.bind(), 0)


def test_launch_config_errors(ctx):
    from paper_2309_15676_amd import _lib as L
    lib = L.load()
    assert lib.jso_set_launch_config(ctx.bind(), -1) == L.JSO_E_INVALID
    assert lib.jso_set_launch_config(ctx.bind(), L.JSO_LAUNCH_CONFIGS) == L.JSO_E_INVALID
    assert lib.jso_set_launch_config(None, 0) == L.JSO_E_INVALID
    assert [L.config_name(c) for c in (0, 2, 3, 14)] == [
        "16x16", "8x8", "16x16 persistent x1", "8x8 persistent x8"]
