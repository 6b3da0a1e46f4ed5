"""Hit records (the forward pass of a replayed path stores what its first rays
hit and whether each vertex's shadow ray is blocked; the replay reads them
back instead of tracing those rays again): the replay takes a record only for
the bitwise same ray, so gradients with records equal the gradients of a
replay that traces every ray (JSO_F_NO_HIT_RECORDS) up to the order of the
float atomics.  Records exist in the kernels of triangle-mesh scenes (single
paths and replay pairs on lane pairs): checked on two mesh scenes
(wave-coherent camera rays, BVH shadow rays) and a terrain crop, through
jso_estimate_gradients, jso_render_bwd and whole meta-estimator steps; an
analytic scene (no records) checks that the flag changes nothing there.  The
agreement with the FP64 oracle is checked by the other parity tests, which
run with records."""
import sys

import numpy as np
import pytest

from paper_2309_15676_amd import inputs as I
from test_gpu_configs import _five_channel
from test_gpu_mesh import _mesh_texture, _mesh_vertex
from test_gpu_parity import _set_pair

pytestmark = pytest.mark.gpu

NO_RECS = 32  # JSO_F_NO_HIT_RECORDS
RTOL = 2e-5   # of the largest gradient element: FP32 atomics summed in another order


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


def _terrain_crop():
    v, t = I.heightfield(40, amp=0.35, seed=7)
    s = I.SceneSpec(width=64, height=48, plane_enabled=False, verts=v, tris=t,
                    mesh_mat=I.MAT_PARAM, spheres=np.array([[0.3, 0.9, -0.2, 0.35]]),
                    sphere_mat=np.array([I.MAT_PARAM], np.int32), depth=8, rr_start=3,
                    tex_w=32, tex_h=32, ch_mask=I.CH_ALL, fixed_default=(0.5, 0.5, 0.5, 0.0, 0.5))
    return s, I.fourier_params(s, 1), I.uniform_params(s, 2, 0.2, 0.8)


CASES = {"analytic": _five_channel, "mesh_texture": _mesh_texture,
         "mesh_vertex": _mesh_vertex, "terrain": _terrain_crop}


def _close(a, b, what):
    a, b = np.asarray(a, np.float64), np.asarray(b, np.float64)
    scale = np.abs(b).max()
    assert scale > 0, what
    err = np.abs(a - b).max()
    assert err <= RTOL * scale, "%s: max |diff| %.3g of scale %.3g" % (what, err, scale)


def _problem(ctx, spec, p, p_prev, it):
    from paper_2309_15676_amd.problem import Problem
    prob = Problem(spec, context=ctx)
    prob.set_target(I.target_image_synthetic(spec, 5))
    _set_pair(prob, p, p_prev, it)
    return prob


@pytest.mark.parametrize("name", list(CASES))
def test_estimators_with_records_equal_traced_replay(ctx, name):
    _say("hit records: estimators", name)
    spec, gt, init = CASES[name]()
    g = np.random.Generator(np.random.PCG64(8))
    lo, hi = spec.param_bounds()
    p_prev = np.clip(init + g.normal(0, 0.03, init.shape).astype(np.float32), lo, hi)
    prob = _problem(ctx, spec, init, p_prev, 6)
    for seed in (33, 34):
        r = prob.estimate_gradients(seed, 6, 2, 1)
        t = prob.estimate_gradients(seed, 6, 2, 1, flags=NO_RECS)
        # the primal images are the same (their loss sums differ in the order only)
        assert abs(r["loss"] - t["loss"]) <= 1e-9 * abs(t["loss"]), (r["loss"], t["loss"])
        for key in ("F", "dF"):
            _close(r[key].cpu().numpy(), t[key].cpu().numpy(), "%s seed %d %s" % (name, seed, key))


@pytest.mark.parametrize("name", ["mesh_texture", "terrain"])
def test_render_bwd_with_records_equals_traced_replay(ctx, name):
    import torch
    from paper_2309_15676_amd import _lib as L
    _say("hit records: render_bwd", name)
    spec, gt, init = CASES[name]()
    prob = _problem(ctx, spec, init, init, 1)
    dimg = torch.from_numpy(I.target_image_synthetic(spec, 3) - 0.6).cuda()
    a = prob.render_bwd(init, dimg, seed=3, iteration=2, tag=L.JSO_TAG_EVAL, spp=3)
    b = prob.render_bwd(init, dimg, seed=3, iteration=2, tag=L.JSO_TAG_EVAL, spp=3, flags=NO_RECS)
    _close(a.cpu().numpy(), b.cpu().numpy(), name)


def test_meta_steps_with_records_equal_traced_replay(ctx):
    from paper_2309_15676_amd import _lib as L
    _say("hit records: meta steps")
    spec, gt, init = _mesh_texture()
    a = _problem(ctx, spec, init, init, 0)
    b = _problem(ctx, spec, init, init, 0)
    opts = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, seed=5)
    opts_t = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, seed=5, flags=NO_RECS)
    for _ in range(3):
        a.grad_step(opts)
        b.grad_step(opts_t)
    sa, sb = a.get_state(), b.get_state()
    # three steps of the stabilised update from gradients that agree to
    # rounding: the parameters agree far inside the step size
    assert np.abs(np.asarray(sa["params"]) - np.asarray(sb["params"])).max() <= 1e-4
    assert sa["iteration"] == sb["iteration"] == 3
