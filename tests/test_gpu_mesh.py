"""GPU parity of triangle meshes (BVH traversal, two-sided shading, texture
and per-vertex parameter layouts) against the FP64 oracle's brute-force
intersection, through the C ABI.  Tolerances and the masking of unstable
pixels are those of the other parity tests: a pixel whose paths take a
decision within TAU of its threshold in the oracle (for a triangle: the
barycentric distance to the nearest edge) is left out."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2309_15676_amd import inputs as I
from test_gpu_parity import (TAU, _check_grad, _check_radiance, _gradient_mask, _oracle_pair,
                             _set_pair)

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


def _mesh_vertex(w=48, h=40, freq=8):
    """Displaced geodesic sphere with per-vertex RGB + roughness on a grey plane."""
    v, t = I.icosphere(freq, center=(0.0, 1.1, 0.0), radius=1.0, disp=0.12, seed=3)
    s = I.SceneSpec(width=w, height=h, plane_mat=0, fixed_mats=I.PLANE_GREY.copy(),
                    verts=v, tris=t, mesh_mat=I.MAT_PARAM, param_layout=I.LAYOUT_VERTEX,
                    depth=5, rr_start=3, ch_mask=I.CH_RGB_ROUGH,
                    fixed_default=(0.5, 0.5, 0.5, 0.0, 0.5),
                    spheres=np.array([[1.8, 0.5, 0.6, 0.5]]), sphere_mat=np.array([0], np.int32))
    return s, I.vertex_fourier_params(s, 1), I.vertex_fourier_params(s, 2, 0.2, 0.8)


def _mesh_texture(w=48, h=40):
    """Heightfield terrain (plane disabled) and two spheres sharing a 16x16
    texture, mapped to the mesh by planar UV."""
    v, t = I.heightfield(12, amp=0.3, seed=4)
    s = I.SceneSpec(width=w, height=h, plane_enabled=False, verts=v, tris=t,
                    mesh_mat=I.MAT_PARAM, spheres=np.array([[-1.0, 1.2, 0.0, 0.6],
                                                            [1.2, 1.0, -0.5, 0.5]]),
                    sphere_mat=np.array([I.MAT_PARAM, I.MAT_PARAM], np.int32),
                    depth=5, rr_start=3, tex_w=16, tex_h=16, ch_mask=I.CH_RGB_ROUGH,
                    fixed_default=(0.5, 0.5, 0.5, 0.0, 0.5))
    return s, I.fourier_params(s, 1), I.uniform_params(s, 2, 0.2, 0.8)


def _fixed_mesh(w=40, h=32):
    """A fixed-material mesh occluding the light over a parameterised plane."""
    v, t = I.icosphere(4, center=(0.8, 2.5, 0.8), radius=0.7, disp=0.0)
    s = I.SceneSpec(width=w, height=h, verts=v, tris=t, mesh_mat=0,
                    fixed_mats=np.array([[0.7, 0.3, 0.2, 0.0, 0.4]]), plane_mat=I.MAT_PARAM,
                    depth=4, tex_w=8, tex_h=8, ch_mask=I.CH_RGB_ROUGH,
                    fixed_default=(0.5, 0.5, 0.5, 0.0, 0.5))
    return s, I.fourier_params(s, 1), I.uniform_params(s, 2, 0.2, 0.8)


CASES = {"vertex": _mesh_vertex, "texture": _mesh_texture, "occluder": _fixed_mesh}


def _problem(ctx, spec):
    from paper_2309_15676_amd.problem import Problem
    return Problem(spec, context=ctx)


@pytest.mark.parametrize("name", ["vertex", "texture", "occluder"])
@pytest.mark.parametrize("flags", [0, O.NO_NEE])
def test_mesh_radiance_parity(ctx, name, flags):
    _say("mesh radiance", name, flags)
    spec, gt, init = CASES[name]()
    prob = _problem(ctx, spec)
    img = prob.render(gt, seed=21, iteration=4, tag=O.TAG_EVAL, spp=2, flags=flags).cpu().numpy()
    pd = gt.astype(np.float64)
    (ref, mg), floor = O.rounding_sensitivity(
        spec, lambda: O.render(spec, pd, 21, 4, O.TAG_EVAL, 2, flags)[0:2])
    _check_radiance(img, ref, mg, floor[0], max_unstable=0.02)


@pytest.mark.parametrize("name", ["vertex", "texture"])
@pytest.mark.parametrize("flags", [0, O.PARAM_INDEP])
def test_mesh_gradient_parity(ctx, name, flags):
    import torch
    _say("mesh gradient", name, flags)
    spec, p, _ = CASES[name]()
    g = np.random.Generator(np.random.PCG64(8))
    p_prev = np.clip(p + g.normal(0, 0.02, p.shape).astype(np.float32), 0.06, 0.99)
    T = I.target_image_synthetic(spec, 5)
    seed, it = 33, 6
    mask = _gradient_mask(spec, p, p_prev, T, seed, it, flags, max_frac=0.06)
    prob = _problem(ctx, spec)
    prob.set_target(T)
    _set_pair(prob, p, p_prev, it)
    r = prob.estimate_gradients(seed, it, 2, 1, flags=flags,
                                mask=torch.from_numpy(mask.reshape(-1)).to("cuda"))
    ref, floor = _oracle_pair(spec, p, p_prev, T, seed, it, flags, mask)
    _check_grad(r["F"].cpu().numpy().astype(np.float64), ref["F"], ref["F_abs"], floor["F"], "F",
                spec)
    _check_grad(r["dF"].cpu().numpy().astype(np.float64), ref["dF"], ref["dF_abs"], floor["dF"],
                "dF", spec)
    assert np.count_nonzero(ref["F"]) > 0 and np.count_nonzero(ref["dF"]) > 0


def test_mesh_fd_sample_bitwise_zero_for_equal_params(ctx):
    _say("mesh fd zero")
    spec, p, _ = _mesh_vertex()
    prob = _problem(ctx, spec)
    prob.set_target(I.target_image_synthetic(spec, 1))
    _set_pair(prob, p, p, 9)
    r = prob.estimate_gradients(seed=4, iteration=9)
    assert np.all(r["dF"].cpu().numpy() == 0.0)
    assert np.count_nonzero(r["F"].cpu().numpy()) > 0


def test_mesh_sphere_full_size_sampled(ctx):
    """The 200,000-triangle displaced sphere at 1024 x 1024 (per-vertex RGB +
    roughness, depth 8, roulette from vertex 3), in the launch configuration of
    a full optimisation step; radiance and gradients of a 16 x 16 crop centred
    on the sphere against the oracle's brute force over every triangle."""
    import torch
    _say("mesh sphere 200k, crop")
    spec = I.scene_mesh_sphere()
    assert len(spec.tris) == 200000 and spec.width == 1024
    p = I.vertex_fourier_params(spec, 1)
    crop = (504, 466, 520, 482)
    prob = _problem(ctx, spec)
    img = prob.render(p, seed=5, iteration=3, tag=O.TAG_EVAL, spp=1, crop=crop).cpu().numpy()
    pd = p.astype(np.float64)
    (ref, mg), floor = O.rounding_sensitivity(
        spec, lambda: O.render(spec, pd, 5, 3, O.TAG_EVAL, 1, crop=crop)[0:2])
    sl = (slice(crop[1], crop[3]), slice(crop[0], crop[2]))
    assert (img[sl] > 0).any(-1).mean() > 0.9  # the crop sees the sphere
    _check_radiance(img[sl], ref[sl], mg[sl], floor[0][sl], max_unstable=0.05)
    # pixels outside the crop are untouched
    out = np.ones(img.shape[:2], bool)
    out[sl] = False
    assert np.all(img[out] == 0)
    # gradient of the crop
    dimg = (I.target_image_synthetic(spec, 12) - 0.75).astype(np.float32)
    dd = dimg.astype(np.float64)
    (_, _, mg2, A), fl = O.rounding_sensitivity(
        spec, lambda: (None, None) + O.render_bwd(spec, pd, dd, 5, 3, O.TAG_EVAL, 1,
                                                  crop=crop)[2:4])
    mask = ((mg2 <= TAU) | O.ill_conditioned({"A": A}, {"A": fl[3]})).astype(np.uint8)
    (gref, gabs, _, _), gfl = O.rounding_sensitivity(
        spec, lambda: O.render_bwd(spec, pd, dd, 5, 3, O.TAG_EVAL, 1, crop=crop,
                                   mask=mask)[0:2] + (None, None))
    gg = prob.render_bwd(p, torch.from_numpy(dimg).cuda(), 5, 3, O.TAG_EVAL, 1, crop=crop,
                         mask=torch.from_numpy(mask.reshape(-1)).cuda())
    _check_grad(gg.cpu().numpy().astype(np.float64), gref, gabs, gfl[0], "render_bwd", spec)
    assert np.count_nonzero(gref) > 20


def test_mesh_sphere_adjoint_matches_central_differences(ctx):
    """Replayed adjoint of the full 1024 x 1024, 200,000-triangle scene (one
    sample per pixel, fixed seed) against central differences of the rendered
    loss J = sum dimg . I with h = 1e-3 on 64 random per-vertex parameters.
    Sampling that does not depend on the parameters makes J smooth in them;
    J(p + h) - J(p - h) is summed in FP64 from the two FP32 images, whose
    untouched pixels are bit-identical."""
    import torch
    from paper_2309_15676_amd import _lib as L
    _say("mesh sphere 200k, central differences")
    spec = I.scene_mesh_sphere()
    prob = _problem(ctx, spec)
    p = I.vertex_fourier_params(spec, 1)
    dimg = torch.from_numpy(I.target_image_synthetic(spec, 3) - 0.75).cuda()
    seed, it, tag, spp, flags = 9, 1, L.JSO_TAG_EVAL, 1, O.PARAM_INDEP
    g = prob.render_bwd(p, dimg, seed, it, tag, spp, flags=flags).cpu().numpy()
    live = np.flatnonzero(np.abs(g) > 1e-3 * np.abs(g).max())
    assert len(live) > 1000
    idx = np.random.Generator(np.random.PCG64(2)).choice(live, 64, replace=False)
    h = 1e-3
    d64 = dimg.double()
    worst = 0.0
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += h
        pm[i] -= h
        a = prob.render(pp, seed, it, tag, spp, flags=flags).double()
        b = prob.render(pm, seed, it, tag, spp, flags=flags).double()
        cd = float(((a - b) * d64).sum()) / (2 * h)
        err = abs(cd - g[i]) / abs(g[i])
        worst = max(worst, err)
        assert err <= 2e-2, (i, cd, g[i])
    print("central differences: worst relative error %.2e" % worst, flush=True)


def test_mesh_scene_errors(ctx):
    from paper_2309_15676_amd import _lib as L
    spec, _, _ = _mesh_vertex()
    bad = _mesh_vertex()[0]
    bad.tris = bad.tris.copy()
    bad.tris[5, 2] = len(bad.verts)
    with pytest.raises(L.JsoError):
        _problem(ctx, bad)
    bad = _mesh_vertex()[0]
    bad.plane_mat = I.MAT_PARAM
    with pytest.raises(L.JsoError):
        _problem(ctx, bad)
    # a good scene still loads after the failures
    prob = _problem(ctx, spec)
    assert prob.n_params == 4 * len(spec.verts)
