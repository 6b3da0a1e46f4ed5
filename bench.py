#!/usr/bin/env python3
"""Benchmark of the joint sampling-and-optimisation hot path on one MI355X.

Workload: the 512x512 textured inverse problem (plane + 8 spheres, one shared
256x256 texture of base colour RGB + roughness = 262,144 parameters, path
depth 6 with Russian roulette from vertex 3), optimised with the
meta-estimator at 2 proportional + 1 finite-difference samples per pixel.
A step is one call of jso_grad_step: primal renders for the adjoint images,
the replayed adjoint of 2 proportional paths and 1 finite-difference path
pair per pixel (4 differentiable paths per pixel), and the fused
meta-estimator + stabilised step.  Inputs are synthetic and already resident
on the GPU when the timed region starts.

Prints one JSON line.  `value` = differentiable paths/s (forward + replayed
adjoint); `roofline` = the dominant kernel (forward tracing or the replayed
adjoint, whichever takes longer): its algorithmic FP32 work (surface vertices
counted on the GPU x per-vertex FLOP figures) per launch over its HIP-event
launch time, against the FP32 vector peak, with `traffic` = HBM bytes per
launch from the committed rocprofv3 counter summary (null when the kernel
changed since it was taken);
`cpu_baseline` = the FP64 CPU oracle on the same workload for about 10 s.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published peaks
PEAK_HBM_GBS = 8000.0
PEAK_FP32_VECTOR_TFLOPS = 157.3

# Algorithmic FP32 work per surface vertex of a path: intersection of the
# continuation and shadow rays with the scene, texture fetch, BSDF evaluation
# and sampling, NEE with MIS, throughput update (forward); the replay repeats
# that and adds the material partials of both BSDF evaluations, the adjoint
# coefficients and the bilinear scatter weights.
FLOP_FORWARD_VERTEX = 600
FLOP_REPLAY_VERTEX = 1000

KERNEL_SOURCES = ("paper_2309_15676_amd/csrc/device.h", "paper_2309_15676_amd/csrc/kernels.h",
                  "paper_2309_15676_amd/csrc/kernels.hip")
TRAFFIC_SUMMARY = "profiles/%s_textured512_hbm_traffic.md"


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    path = os.path.join(ROOT, TRAFFIC_SUMMARY % kernel)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith("traffic-json: "):
                rec = json.loads(line[len("traffic-json: "):])
                if rec.get("source_sha256") == kernel_source_hash():
                    return rec["bytes_per_launch"]
    return None


def cpu_baseline(spec, params, target, seconds: float, seed: int):
    """The FP64 oracle, as it stands, timed on this host: whole iterations
    (proportional + finite-difference gradient samples on the full image, then
    the meta-estimator step) of the same workload, repeated until `seconds`
    have passed."""
    import numpy as np

    import oracle as O
    from oracle import meta as OM

    lo, hi = spec.param_bounds()
    opt = OM.MetaOptimizer(params, lo, hi, eta=float(np.float32(0.01)))
    # this host's share of cores (at most 16 worker threads)
    threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    t0 = time.perf_counter()
    iters = 0
    while True:
        r = O.gradient_pair(spec, opt.params.astype(np.float64),
                            opt.params_prev.astype(np.float64), target, seed, iters,
                            nthreads=threads)
        opt.step(r["F"], r["dF"])
        iters += 1
        dt = time.perf_counter() - t0
        if dt >= seconds or iters >= 1000:
            break
    paths = 4 * spec.n_pixels * iters - 2 * spec.n_pixels  # no FD pair at iteration 0
    out = dict(value=paths / dt, unit="differentiable paths/s", cores=threads, kind="oracle",
               sample="first %d iterations of the 512x512 workload from the same initial "
                      "texture (iteration 0 has no FD pair), %.1f s" % (iters, dt))
    # one thread, on a 64x64 crop at the image centre (a few seconds)
    crop = (224, 224, 288, 288)
    n = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < seconds / 4 and n < 200:
        O.gradient_pair(spec, params.astype(np.float64), params.astype(np.float64), target,
                        seed, 1 + n, crop=crop, nthreads=1)
        n += 1
    dt1 = time.perf_counter() - t0
    out["single_thread"] = dict(value=4 * 64 * 64 * n / dt1, unit="differentiable paths/s",
                                sample="%d iterations' gradient samples (prop + FD pair) on the "
                                       "central 64x64 crop, %.1f s" % (n, dt1))
    return out


def copy_calibration(mib: int):
    """A plain device copy of known size (mib MiB read + mib MiB written), run
    three times, for scaling the HBM byte counters of a profiled run."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()


META_BUDGET = 2.0  # meta-estimator wall-clock per run, in units of Adam's


def time_to_loss(prob, init, gt, target, args, iters: int, label: str, lam: float = 0.0,
                 etas=None):
    """Loss against wall-clock (grad_step calls only; evaluations off the
    clock) of plain Adam at 64 spp and of the meta-estimator at 2 proportional
    + 1 FD spp (replay pair, and shared path), same GPU, same process.  Every
    method runs at every learning rate of a grid: Adam for `iters`
    iterations, the meta-estimator for META_BUDGET times Adam's wall-clock.

    Reported: the time each method needs to reach Adam's best loss (the first
    time any learning rate reaches it: rates tuned per target, as the paper
    tunes each method's; speedup null when no rate reaches it within the
    budget), and the same for the losses Adam reaches after 1/8, 1/4 and 1/2
    of its iterations (speedup_by_level).  lam > 0: both methods
    precondition their texture gradients (Large Steps)."""
    import torch

    from paper_2309_15676_amd import _lib as L

    ev_seed, ev_spp = 777, 256
    T = target.float()
    every = max(iters // 40, 1)

    def eval_loss(p=None):
        p = prob.get_params() if p is None else p
        img = prob.render(p, seed=ev_seed, iteration=0, tag=L.JSO_TAG_EVAL, spp=ev_spp)
        return float(((img - T) ** 2).mean())

    floor = eval_loss(gt)  # the evaluation's own noise: loss at the ground truth

    def run(opts, n, every, seconds=None):
        prob.set_params(init)  # also resets the optimiser state
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        clock, hist = 0.0, [(0, 0.0, eval_loss())]
        done = 0
        while done < n and (seconds is None or clock < seconds):
            k = min(every, n - done)
            torch.cuda.synchronize()
            e0.record()
            for _ in range(k):
                prob.grad_step(opts)
            e1.record()
            torch.cuda.synchronize()
            clock += e0.elapsed_time(e1) / 1e3
            done += k
            hist.append((done, clock, eval_loss()))
        return hist

    def first(hist, level):
        return next(((h[0], h[1]) for h in hist if h[2] <= level), (None, None))

    grid = etas or [float(x) for x in args.ttl_etas.split(",")]
    adam = {}
    for eta in grid:
        o = L.step_opts(optimizer=L.JSO_OPT_ADAM, eta=eta, adam_spp=64, seed=args.seed + 1,
                        precond_lambda=lam)
        adam[eta] = run(o, iters, every)
        print("[bench]   %s: adam eta %g best %.4g" % (label[:24], eta, min(h[2] for h in adam[eta])),
              file=sys.stderr, flush=True)
    best_eta = min(adam, key=lambda e: min(h[2] for h in adam[e]))
    ha = adam[best_eta]
    target_loss = min(h[2] for h in ha)
    budget_s = ha[-1][1]
    runs = {}
    for name, mode in (("meta", L.JSO_FD_REPLAY), ("meta_fd_shared", L.JSO_FD_SHARED)):
        runs[name] = {}
        for eta in grid:
            o = L.step_opts(optimizer=L.JSO_OPT_META, eta=eta, beta_F=0.99, beta_D=0.9,
                            spp_prop=2, spp_fd=1, seed=args.seed + 2, precond_lambda=lam,
                            fd_mode=mode)
            runs[name][eta] = run(o, 10 ** 9, every * 4, seconds=META_BUDGET * budget_s)
            print("[bench]   %s: %s eta %g best %.4g" % (
                label[:24], name, eta, min(h[2] for h in runs[name][eta])), file=sys.stderr,
                flush=True)

    def time_to(hists, level):
        """(seconds, iterations, eta) of the learning rate that reaches `level`
        first, or Nones."""
        best = (None, None, None)
        for eta, h in hists.items():
            it, t = first(h, level)
            if t is not None and (best[0] is None or t < best[0]):
                best = (t, it, eta)
        return best

    def summary(name):
        h = runs[name]
        t, it, eta = time_to(h, target_loss)
        return {"spp": "2 prop + 1 FD" + (" (shared path)" if "shared" in name else ""),
                "seconds": t, "iterations": it, "eta": eta,
                "speedup": (t_adam / t) if t else None,
                "best_loss_by_eta": {str(e): min(x[2] for x in h[e]) for e in grid},
                "iterations_run_by_eta": {str(e): h[e][-1][0] for e in grid},
                "seconds_budget": META_BUDGET * budget_s}

    t_adam, it_adam, _ = time_to({best_eta: ha}, target_loss)
    levels = {}
    for frac in (8, 4, 2, 1):
        lv = next(h[2] for h in ha if h[0] >= iters // frac) if frac > 1 else target_loss
        ta, ia, ea = time_to(adam, lv)
        row = {"loss": lv, "adam_seconds": ta, "adam_eta": ea}
        for name in runs:
            tm, im, em = time_to(runs[name], lv)
            row.update({name + "_seconds": tm, name + "_iterations": im, name + "_eta": em,
                        name + "_speedup": (ta / tm) if tm else None})
        levels["adam_iters_%d" % (iters // frac)] = row
    return {
        "workload": label,
        "evaluation": "L2 of a %d-spp render (fixed evaluation stream) against the target, "
                      "off the clock" % ev_spp,
        "method": "each method's time to a loss is the first time any learning rate of the "
                  "grid reaches it (learning rates tuned per target); the meta-estimator runs "
                  "get %.0fx Adam's wall-clock" % META_BUDGET,
        "target_loss": target_loss,
        "loss_at_ground_truth": floor,
        "adam": {"spp": 64, "eta": best_eta, "iterations": it_adam, "seconds": t_adam,
                 "best_loss_by_eta": {str(e): min(h[2] for h in adam[e]) for e in grid},
                 "iteration_budget": iters, "seconds_budget": budget_s},
        "meta": summary("meta"),
        "meta_fd_shared": summary("meta_fd_shared"),
        "speedup": summary("meta")["speedup"],
        "speedup_by_level": levels,
        "precond_lambda": lam,
    }


def ablations(prob, init, target, iters: int, eta: float, seed: int, label: str):
    """The meta-estimator as published and with each ablation of the
    Experiments section (non-zero-centred variance EMAs, no alpha clipping,
    uncorrelated variance samples), same learning rate and random streams:
    evaluation loss (256 spp, fixed stream, off the clock) after `iters`
    iterations, the lowest loss seen, and the GPU time per iteration."""
    import torch

    from paper_2309_15676_amd import _lib as L

    T = target.float()

    def eval_loss():
        img = prob.render(prob.get_params(), seed=777, iteration=0, tag=L.JSO_TAG_EVAL,
                          spp=256)
        return float(((img - T) ** 2).mean())

    out = {"workload": label, "iterations": iters, "eta": eta}
    variants = {"published": 0, "non_zero_centred": L.JSO_ABLATE_CENTRED,
                "no_alpha_clip": L.JSO_ABLATE_NO_CLIP,
                "uncorrelated_variance": L.JSO_ABLATE_UNCORRELATED}
    every = max(iters // 10, 1)
    for name, ab in variants.items():
        prob.set_params(init)
        opts = L.step_opts(optimizer=L.JSO_OPT_META, eta=eta, seed=seed, ablate=ab)
        first = eval_loss()
        losses, ms = [], 0.0
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for done in range(0, iters, every):
            torch.cuda.synchronize()
            e0.record()
            for _ in range(min(every, iters - done)):
                prob.grad_step(opts)
            e1.record()
            torch.cuda.synchronize()
            ms += e0.elapsed_time(e1)
            losses.append(eval_loss())
        out[name] = {"initial_loss": first, "final_loss": losses[-1], "best_loss": min(losses),
                     "diverged": bool(losses[-1] > first or not all(map(math.isfinite, losses))),
                     "ms_per_iteration": ms / iters}
    return out


def large_time_to_rmse(context, args):
    """The 2048x2048 terrain problem (1.0M triangles + 32 spheres, 512x512
    texture of 5 channels): parameter-space RMSE against the ground truth
    over wall-clock (grad_step calls only) for the meta-estimator (2 prop +
    1 FD spp) and plain Adam at 32 and 64 spp.  The RMSE counts the
    observable parameters only: every channel of the texels that a 64-spp
    backward pass at the ground truth touches.  Each run stops at RMSE 1e-2,
    at 2000 iterations, or at args.large_ttl_seconds of GPU time."""
    import numpy as np
    import torch

    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd import inputs as I
    from paper_2309_15676_amd.problem import Problem

    spec, gt, init = I.config_large()
    prob = Problem(spec, context=context)
    target = prob.render(gt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET, spp=256)
    prob.set_target(target)
    ones = torch.ones(spec.height, spec.width, 3, device="cuda")
    g = prob.render_bwd(gt, ones, seed=99, iteration=0, tag=L.JSO_TAG_EVAL, spp=64)
    texel_seen = (g.abs().reshape(-1, spec.n_ch) > 0).any(dim=1)
    obs = texel_seen.repeat_interleave(spec.n_ch).cpu().numpy()
    gt64 = np.asarray(gt, np.float64)[obs]

    def rmse_of(p):
        return float(np.sqrt(np.mean((np.asarray(p)[obs].astype(np.float64) - gt64) ** 2)))

    def rmse():
        return rmse_of(prob.get_params())

    r0 = rmse_of(init)
    # RMSE 1e-2 and 95 / 90 / 85 / 80 % of the initial RMSE
    levels = [1e-2] + [f * r0 for f in (0.95, 0.9, 0.85, 0.8)]
    runs = {}
    for name, opts in (
            ("meta_eta0.003", L.step_opts(optimizer=L.JSO_OPT_META, eta=0.003, seed=args.seed)),
            ("meta_eta0.01", L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, seed=args.seed)),
            ("adam32_eta0.01", L.step_opts(optimizer=L.JSO_OPT_ADAM, eta=0.01, adam_spp=32,
                                           seed=args.seed)),
            ("adam64_eta0.01", L.step_opts(optimizer=L.JSO_OPT_ADAM, eta=0.01, adam_spp=64,
                                           seed=args.seed))):
        prob.set_params(init)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        clock, it, hist = 0.0, 0, [(0, 0.0, rmse())]
        chunk = 20 if opts.optimizer == L.JSO_OPT_META else 2
        while it < 2000 and clock < args.large_ttl_seconds and hist[-1][2] > 1e-2:
            torch.cuda.synchronize()
            e0.record()
            for _ in range(chunk):
                prob.grad_step(opts)
            e1.record()
            torch.cuda.synchronize()
            clock += e0.elapsed_time(e1) / 1e3
            it += chunk
            hist.append((it, clock, rmse()))
            if it % (50 * chunk) == 0:
                print("[bench]   large problem %s: %d iterations, %.1f s, rmse %.4g" % (
                    name, it, clock, hist[-1][2]), file=sys.stderr, flush=True)
        reach = {"%.4g" % lv: next((h[1] for h in hist if h[2] <= lv), None) for lv in levels}
        runs[name] = {"seconds_to_rmse": reach, "final_rmse": hist[-1][2],
                      "iterations": it, "seconds": clock,
                      "ms_per_iteration": 1e3 * clock / max(it, 1)}
        print("[bench] large problem %s: %s" % (name, json.dumps(runs[name])), file=sys.stderr,
              flush=True)
    del prob
    torch.cuda.empty_cache()
    return {"workload": "2048x2048 terrain (999,698 triangles) + 32 spheres, 512x512 texture "
                        "of RGB + metalness + roughness (1,310,720 params), depth 12, roulette "
                        "from vertex 3; target at 256 spp",
            "observable_params": int(obs.sum()), "total_params": spec.n_params,
            "initial_rmse": r0, "budget_seconds": args.large_ttl_seconds, "runs": runs}


def batched_throughput(ctx_problem, args):
    """64 independent problems of uneven size (image side 64-512, 5-65,536
    parameters, own seeds and iteration budgets): differentiable paths/s of
    one iteration for all of them, (a) as a batch replayed from a captured
    HIP graph with the tile shape picked by the autotuner, (b) as one
    jso_grad_step over all problems (one launch per kernel, tuned shape),
    (c) as one jso_grad_step per problem."""
    import torch

    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd import inputs as I
    from paper_2309_15676_amd.problem import Batch, Problem, grad_step_many

    cfg = I.config_batched(64, seed=args.seed)
    ctx = ctx_problem.context
    probs = []
    for k, c in enumerate(cfg):
        p = Problem(c["spec"], context=ctx)
        p.set_target(p.render(c["gt"], seed=1000 + k, iteration=0, tag=L.JSO_TAG_TARGET,
                              spp=args.batch_target_spp))
        p.set_params(c["init"])
        probs.append(p)
    opts = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, beta_F=0.99, beta_D=0.9,
                       spp_prop=2, spp_fd=1, seed=args.seed)
    pixels = sum(c["spec"].n_pixels for c in cfg)
    steps = args.batch_steps

    def timed(fn):
        fn(3)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        fn(steps)
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    b = Batch(probs, opts, max_iters=[c["max_iter"] for c in cfg], use_graph=True)
    shape, shape_ms = b.autotune(3)  # state is restored after each trial
    ms_graph = timed(lambda n: b.step(n))
    b.close()

    def together(n):
        for _ in range(n):
            grad_step_many(probs, opts)

    def one_by_one(n):
        for _ in range(n):
            for p in probs:
                p.grad_step(opts)

    ms_together = timed(together)
    ms_each = timed(one_by_one)
    paths = 4 * pixels
    return {
        "workload": "64 problems, image side log-uniform 64-512 (multiple of 8), 5-65,536 "
                    "parameters log-uniform (global material at <= 5, else an RGB + roughness "
                    "texture), own seeds, meta-estimator 2 prop + 1 FD spp",
        "pixels": pixels,
        "params": sum(c["spec"].n_params for c in cfg),
        "steps": steps,
        "autotune": {"tile": ["16x16", "16x8", "8x8"][shape],
                     "ms_per_iteration": {t: m for t, m in zip(["16x16", "16x8", "8x8"], shape_ms)}},
        "graph": {"ms_per_iteration": ms_graph, "paths_per_s": paths / (ms_graph / 1e3)},
        "one_launch_per_kernel": {"ms_per_iteration": ms_together,
                                  "paths_per_s": paths / (ms_together / 1e3)},
        "one_grad_step_per_problem": {"ms_per_iteration": ms_each,
                                      "paths_per_s": paths / (ms_each / 1e3)},
    }


META_BYTES_PER_PARAM = 108  # k_meta: reads 52 B, writes 56 B per parameter


def volume_workload(context, args):
    """The volume experiment's workload: a 256^3 emission-absorption volume
    (67.1M parameters: emission RGB + density per voxel) seen by 8 cameras of
    256x256.  Meta-estimator step time (replay pair and shared path; the
    march draws nothing from the parameters, so both trace the same rays),
    Adam at 2 and 4 spp (the paper places the meta-estimator's cost between
    them), k_meta against the HBM roofline at this parameter count, and the
    loss each reaches in the same wall-clock."""
    import torch
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd import inputs as I
    from paper_2309_15676_amd.problem import Problem
    t0 = time.time()
    spec, gt, init = I.config_volume()
    prob = Problem(spec, context=context)
    ctx = prob.ctx
    target = prob.render(gt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET, spp=16)
    prob.set_target(target)
    prob.set_params(init)
    load_s = time.time() - t0
    names = ((L.JSO_K_FORWARD, "forward"), (L.JSO_K_FINALIZE, "finalize"),
             (L.JSO_K_ADJOINT, "adjoint"), (L.JSO_K_META, "meta"), (L.JSO_K_ADAM, "adam"))

    def timed(opts, n):
        prob.set_params(init)
        for _ in range(2):
            prob.grad_step(opts)
        torch.cuda.synchronize()
        L.check(L.jso_set_timing(ctx, True), ctx)
        for k in range(L.JSO_K_COUNT):
            L.jso_get_kernel_time(ctx, k, reset=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            prob.grad_step(opts)
        e1.record()
        torch.cuda.synchronize()
        kt = {}
        for k, name in names:
            ms, calls = L.jso_get_kernel_time(ctx, k)
            if calls:
                kt[name] = {"ms_per_step": ms / n, "ms_per_launch": ms / calls}
        L.check(L.jso_set_timing(ctx, False), ctx)
        return e0.elapsed_time(e1) / n, kt

    n = args.volume_steps
    npix = spec.n_pixels
    out = {"workload": "256^3 emission-absorption volume (67,108,864 params: emission RGB + "
                       "density), 8 views of 256x256 (524,288 pixels), density scale 8 per unit "
                       "length, voxel-length segments (up to ~440 samples per ray)",
           "scene_load_s": load_s}
    meta = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, seed=args.seed)
    ms, kt = timed(meta, n)
    out["meta_step"] = {"ms": ms, "diff_paths_per_s": 4 * npix / (ms / 1e3), "kernel": kt}
    ms, kt = timed(L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, seed=args.seed,
                               fd_mode=L.JSO_FD_SHARED), n)
    out["meta_step_fd_shared"] = {"ms": ms, "kernel": kt}
    for spp in (2, 4):
        ms, kt = timed(L.step_opts(optimizer=L.JSO_OPT_ADAM, eta=0.01, adam_spp=spp,
                                   seed=args.seed), n)
        out["adam%d_step" % spp] = {"ms": ms, "kernel": kt}
    km = out["meta_step"]["kernel"]["meta"]["ms_per_launch"]
    bytes_meta = META_BYTES_PER_PARAM * spec.n_params
    out["k_meta_roofline"] = {"bound": "hbm", "bytes_per_launch": bytes_meta, "ms": km,
                              "achieved_GBs": bytes_meta / (km / 1e3) / 1e9,
                              "peak_GBs": PEAK_HBM_GBS,
                              "frac": bytes_meta / (km / 1e3) / 1e9 / PEAK_HBM_GBS}
    del prob
    torch.cuda.empty_cache()
    # equal wall-clock on a smaller grid (the 256^3 step is too slow for many
    # iterations in a bench run): the loss of a 16-spp evaluation render (off
    # the clock) after the same GPU time
    if args.volume_ttl_seconds > 0:
        R = args.volume_ttl_res
        spec, gt, init = I.config_volume(res=R, view_w=R, view_h=R)
        prob = Problem(spec, context=context)
        target = prob.render(gt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET, spp=64)
        prob.set_target(target)

        def eval_loss():
            img = prob.render(prob.get_params(), seed=777, iteration=0, tag=L.JSO_TAG_EVAL,
                              spp=16)
            return float(((img - target) ** 2).mean())

        def run(opts, seconds, every):
            prob.set_params(init)
            clock, it, hist = 0.0, 0, [(0, 0.0, eval_loss())]
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            while clock < seconds:
                torch.cuda.synchronize()
                e0.record()
                for _ in range(every):
                    prob.grad_step(opts)
                e1.record()
                torch.cuda.synchronize()
                clock += e0.elapsed_time(e1) / 1e3
                it += every
                hist.append((it, clock, eval_loss()))
            return hist

        prob.set_params(init)
        ttl = {"workload": "%d^3 volume, 8 views of %dx%d, same scene and initial volume" % (
                   R, R, R),
               "seconds": args.volume_ttl_seconds, "initial_loss": eval_loss(), "runs": {}}
        for name, mk in (("meta", lambda e: L.step_opts(optimizer=L.JSO_OPT_META, eta=e,
                                                         seed=args.seed + 2)),
                         ("adam2", lambda e: L.step_opts(optimizer=L.JSO_OPT_ADAM, eta=e,
                                                          adam_spp=2, seed=args.seed + 1)),
                         ("adam4", lambda e: L.step_opts(optimizer=L.JSO_OPT_ADAM, eta=e,
                                                          adam_spp=4, seed=args.seed + 1))):
            best = None
            for eta in (0.003, 0.01, 0.03, 0.1):
                h = run(mk(eta), args.volume_ttl_seconds, 10)
                print("[bench]   volume equal time: %s eta %g best %.4g after %d iterations" % (
                    name, eta, min(x[2] for x in h), h[-1][0]), file=sys.stderr, flush=True)
                row = {"eta": eta, "iterations": h[-1][0], "final_loss": h[-1][2],
                       "best_loss": min(x[2] for x in h),
                       "loss_curve": [(x[0], round(x[1], 4), x[2]) for x in h[:: max(len(h) // 8, 1)]]}
                if best is None or row["best_loss"] < best["best_loss"]:
                    best = row
            ttl["runs"][name] = best
        out["equal_time"] = ttl
        del prob
        torch.cuda.empty_cache()
    print("[bench] volume: %s" % json.dumps(out), file=sys.stderr, flush=True)
    return out


def mesh_workloads(context, args):
    """Throughput of the mesh workloads (BVH traversal): the 1024x1024,
    200,000-triangle displaced sphere with per-vertex RGB + roughness
    (replayed adjoint of one sample per pixel, and a full meta-estimator step),
    and the 2048x2048 scene of a 1.0M-triangle terrain + 32 spheres with a
    512x512x5 texture (meta-estimator step, depth 12)."""
    import torch
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd import inputs as I
    from paper_2309_15676_amd.problem import Problem
    ctx = context.bind()
    out = {}

    def timed(fn, n):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        L.check(L.jso_set_timing(ctx, True), ctx)
        for k in range(L.JSO_K_COUNT):
            L.jso_get_kernel_time(ctx, k, reset=True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        kt = {name: L.jso_get_kernel_time(ctx, k)[0] / n for k, name in
              ((L.JSO_K_FORWARD, "forward"), (L.JSO_K_FINALIZE, "finalize"),
               (L.JSO_K_ADJOINT, "adjoint"), (L.JSO_K_META, "meta"))}
        L.check(L.jso_set_timing(ctx, False), ctx)
        return e0.elapsed_time(e1) / n, kt

    t0 = time.time()
    spec = I.scene_mesh_sphere()
    prob = Problem(spec, context=context)
    load_s = time.time() - t0
    gt = I.vertex_fourier_params(spec, 1)
    init = I.uniform_params(spec, 2, 0.2, 0.8)
    prob.set_target(prob.render(gt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET, spp=64))
    prob.set_params(init)
    npix = spec.n_pixels
    dimg = torch.zeros(spec.height, spec.width, 3, device="cuda") + 0.25
    g = torch.zeros(spec.n_params, device="cuda")
    init_t = torch.from_numpy(init).cuda()
    ms_bwd, kt_bwd = timed(lambda: prob.render_bwd(init_t, dimg, 9, 1, L.JSO_TAG_EVAL, 1, out=g),
                           args.mesh_steps)
    opts = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, seed=args.seed)
    ms_step, kt_step = timed(lambda: prob.grad_step(opts), args.mesh_steps)
    opts_sh = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, seed=args.seed,
                          fd_mode=L.JSO_FD_SHARED)
    prob.set_params(init)
    ms_sh, kt_sh = timed(lambda: prob.grad_step(opts_sh), args.mesh_steps)
    out["sphere_200k"] = {
        "workload": "1024x1024, displaced geodesic sphere of 200,000 triangles on a grey "
                    "plane, per-vertex RGB + roughness (400,008 params), depth 8, roulette "
                    "from vertex 3",
        "scene_load_s": load_s,
        "adjoint_1spp": {"ms": ms_bwd, "diff_paths_per_s": npix / (ms_bwd / 1e3),
                         "kernel_ms": kt_bwd},
        "meta_step": {"ms": ms_step, "diff_paths_per_s": 4 * npix / (ms_step / 1e3),
                      "kernel_ms": kt_step},
        "meta_step_fd_shared": {"ms": ms_sh, "kernel_ms": kt_sh},
    }
    print("[bench] mesh sphere: %s" % json.dumps(out["sphere_200k"]), file=sys.stderr, flush=True)
    del prob
    torch.cuda.empty_cache()

    t0 = time.time()
    spec, gt, init = I.config_large()
    prob = Problem(spec, context=context)
    load_s = time.time() - t0
    prob.set_target(prob.render(gt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET, spp=16))
    prob.set_params(init)
    npix = spec.n_pixels
    ms_step, kt_step = timed(lambda: prob.grad_step(opts), max(2, args.mesh_steps // 2))
    prob.set_params(init)
    ms_sh, kt_sh = timed(lambda: prob.grad_step(opts_sh), max(2, args.mesh_steps // 2))
    out["terrain_1m"] = {
        "workload": "2048x2048, fractal terrain of 999,698 triangles + 32 spheres, 512x512 "
                    "texture of RGB + metalness + roughness (1,310,720 params), depth 12, "
                    "roulette from vertex 3, meta-estimator 2 prop + 1 FD spp",
        "scene_load_s": load_s,
        "meta_step": {"ms": ms_step, "diff_paths_per_s": 4 * npix / (ms_step / 1e3),
                      "kernel_ms": kt_step},
        "meta_step_fd_shared": {"ms": ms_sh, "kernel_ms": kt_sh},
    }
    print("[bench] terrain: %s" % json.dumps(out["terrain_1m"]), file=sys.stderr, flush=True)
    del prob
    torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--target-spp", type=int, default=4096)
    ap.add_argument("--cpu-seconds", type=float, default=10.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain copy of this many MiB (counter calibration)")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--ttl-iters", type=int, default=300,
                    help="Adam-64 iteration budget of the textured time-to-loss comparison "
                         "(0: skip the comparisons)")
    ap.add_argument("--ttl-etas", default="0.0003,0.001,0.003,0.01,0.03,0.1")
    ap.add_argument("--ttl-lambda", type=float, default=20.0,
                    help="also compare both methods with preconditioned texture gradients "
                         "(Large Steps) at this lambda (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="iterations timed for the 64-problem batch (0: skip it)")
    ap.add_argument("--batch-target-spp", type=int, default=256)
    ap.add_argument("--ablation-iters", type=int, default=1000,
                    help="meta-estimator iterations of the ablation runs on the textured "
                         "problem (the tiny problem runs 200; 0: skip)")
    ap.add_argument("--large-ttl-seconds", type=float, default=0.0,
                    help="GPU-seconds per run of the terrain time-to-RMSE comparison "
                         "(meta-estimator vs Adam at 32 and 64 spp; 0: skip)")
    ap.add_argument("--volume-steps", type=int, default=5,
                    help="timed calls per volume configuration (0 = skip the volume workload)")
    ap.add_argument("--volume-ttl-seconds", type=float, default=8.0,
                    help="GPU-seconds per run of the volume equal-time comparison (0: skip)")
    ap.add_argument("--volume-ttl-res", type=int, default=128,
                    help="voxels per side (and view size) of the equal-time comparison")
    ap.add_argument("--mesh-steps", type=int, default=10,
                    help="timed calls per mesh workload (0 = skip the mesh workloads)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: this build runs on one GPU; --gpus %d is not supported "
              "(the multi-GPU sharding is a design note, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd import inputs as I
    from paper_2309_15676_amd.problem import Problem

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    spec, gt, init = I.config_textured()
    prob = Problem(spec)
    # target image: ground-truth texture rendered at high spp (off the clock)
    print("[bench] rendering target at %d spp" % args.target_spp, file=sys.stderr, flush=True)
    target = prob.render(gt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET, spp=args.target_spp)
    prob.set_target(target)
    prob.set_params(init)
    opts = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, beta_F=0.99, beta_D=0.9, spp_prop=2,
                       spp_fd=1, seed=args.seed)
    ctx = prob.ctx
    for _ in range(args.warmup):
        prob.grad_step(opts)
    torch.cuda.synchronize()
    L.check(L.jso_set_timing(ctx, True), ctx)
    for k in range(L.JSO_K_COUNT):
        L.jso_get_kernel_time(ctx, k, reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        prob.grad_step(opts)
    e1.record()
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    ktimes = {name: L.jso_get_kernel_time(ctx, k) for k, name in
              ((L.JSO_K_FORWARD, "forward"), (L.JSO_K_FINALIZE, "finalize"),
               (L.JSO_K_ADJOINT, "adjoint"), (L.JSO_K_META, "meta"))}
    L.check(L.jso_set_timing(ctx, False), ctx)
    # work of the path-tracing launches, counted on the GPU (outside the timed region)
    L.check(L.jso_set_work_counting(ctx, True), ctx)
    L.jso_get_work(ctx, reset=True)
    n_count = 3
    for _ in range(n_count):
        prob.grad_step(opts)
    rep_paths, rep_verts, fwd_paths, fwd_verts = L.jso_get_work(ctx, reset=True)
    L.check(L.jso_set_work_counting(ctx, False), ctx)
    vpp = rep_verts / max(rep_paths, 1)
    st = prob.grad_step(opts, want_stats=True)
    print("[bench] kernel ms per step: %s; loss %.5g; %.4f vertices per path" % (
        {k: round(v[0] / max(v[1], 1), 4) for k, v in ktimes.items()}, st.loss, vpp),
        file=sys.stderr, flush=True)
    # the same step with the shared-path finite-difference sample (Eq. 5 as
    # written: one finite-difference path per pixel instead of two), reported
    # beside the headline figure
    opts_sh = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, beta_F=0.99, beta_D=0.9,
                          spp_prop=2, spp_fd=1, seed=args.seed, fd_mode=L.JSO_FD_SHARED)
    prob.set_params(init)
    for _ in range(args.warmup):
        prob.grad_step(opts_sh)
    L.check(L.jso_set_timing(ctx, True), ctx)
    for k in range(L.JSO_K_COUNT):
        L.jso_get_kernel_time(ctx, k, reset=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        prob.grad_step(opts_sh)
    e1.record()
    torch.cuda.synchronize()
    fd_shared = {"ms_per_step": e0.elapsed_time(e1) / args.steps,
                 "kernel_ms_per_step": {name: (lambda v: v[0] / max(v[1], 1))(
                     L.jso_get_kernel_time(ctx, k)) for k, name in
                     ((L.JSO_K_FORWARD, "forward"), (L.JSO_K_FINALIZE, "finalize"),
                      (L.JSO_K_ADJOINT, "adjoint"), (L.JSO_K_META, "meta"))},
                 "paths_traced_per_step": 3 * spec.n_pixels}
    L.check(L.jso_set_timing(ctx, False), ctx)
    prob.set_params(init)
    print("[bench] shared-path FD step: %s" % json.dumps(fd_shared), file=sys.stderr, flush=True)
    if args.copy_mib > 0:
        copy_calibration(args.copy_mib)

    npix = spec.n_pixels
    diff_paths = 4 * npix * args.steps
    value = diff_paths / (total_ms / 1e3)

    # CPU baseline: the oracle on this host
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline (%.0f s)" % args.cpu_seconds, file=sys.stderr,
              flush=True)
        Tn = target.cpu().numpy().astype(np.float64)
        cpu = cpu_baseline(spec, init, Tn, args.cpu_seconds, args.seed)
    bat = None
    if args.batch_steps > 0:
        print("[bench] 64-problem batch", file=sys.stderr, flush=True)
        bat = batched_throughput(prob, args)
        print("[bench] batch: %s" % json.dumps(bat), file=sys.stderr, flush=True)
    mesh = None
    if args.mesh_steps > 0:
        print("[bench] mesh workloads", file=sys.stderr, flush=True)
        mesh = mesh_workloads(prob.context, args)
    vol = None
    if args.volume_steps > 0:
        print("[bench] volume workload", file=sys.stderr, flush=True)
        vol = volume_workload(prob.context, args)
    large = None
    if args.large_ttl_seconds > 0:
        print("[bench] terrain time to RMSE", file=sys.stderr, flush=True)
        large = large_time_to_rmse(prob.context, args)
    ttl = None
    if args.ttl_iters > 0:
        print("[bench] time to loss: Adam-64 vs meta-estimator", file=sys.stderr, flush=True)
        ttl = {}
        # the paper's multivariate-material case: 5 global parameters
        tspec, tgt, tinit = I.config_tiny()
        tprob = Problem(tspec, context=prob.context)
        ttarget = tprob.render(tgt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET, spp=1024)
        tprob.set_target(ttarget)
        ttl["tiny"] = time_to_loss(
            tprob, tinit, tgt, ttarget, args, 200,
            "64x64, unit sphere on a grey plane, 5 global parameters (RGB, metalness, "
            "roughness), depth 3, target at 1024 spp")
        print("[bench] time to loss: %s" % json.dumps(ttl["tiny"]), file=sys.stderr, flush=True)
        ttl["textured"] = time_to_loss(
            prob, init, gt, target, args, args.ttl_iters,
            "the 512x512 textured problem (262,144 texel parameters, no preconditioning)")
        print("[bench] time to loss: %s" % json.dumps(ttl["textured"]), file=sys.stderr,
              flush=True)
        if args.ttl_lambda > 0:
            ttl["textured_preconditioned"] = time_to_loss(
                prob, init, gt, target, args, args.ttl_iters,
                "the 512x512 textured problem, both methods with Large-Steps preconditioned "
                "texture gradients", lam=args.ttl_lambda, etas=[0.01, 0.03, 0.1, 0.3])
            print("[bench] time to loss: %s" % json.dumps(ttl["textured_preconditioned"]),
                  file=sys.stderr, flush=True)
    abl = None
    if args.ablation_iters > 0:
        print("[bench] meta-estimator ablations", file=sys.stderr, flush=True)
        tspec, tgt, tinit = I.config_tiny()
        tprob = Problem(tspec, context=prob.context)
        ttarget = tprob.render(tgt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET, spp=1024)
        tprob.set_target(ttarget)
        abl = {"tiny": ablations(tprob, tinit, ttarget, 200, 0.01, args.seed + 2,
                                 "64x64, 5 global parameters"),
               "textured": ablations(prob, init, target, args.ablation_iters, 0.003,
                                     args.seed + 2, "512x512, 262,144 texel parameters")}
        print("[bench] ablations: %s" % json.dumps(abl), file=sys.stderr, flush=True)
    # roofline of the dominant kernel: algorithmic FP32 work per launch over
    # its average launch time
    cands = {
        "k_forward": (ktimes["forward"], fwd_verts / n_count * FLOP_FORWARD_VERTEX,
                      fwd_paths / n_count, fwd_verts / max(fwd_paths, 1)),
        "k_adjoint": (ktimes["adjoint"], rep_verts / n_count * FLOP_REPLAY_VERTEX,
                      rep_paths / n_count, vpp),
    }
    kname = max(cands, key=lambda k: cands[k][0][0])
    (k_ms, k_n), k_flop, k_paths, k_vpp = cands[kname]
    k_launch_ms = k_ms / max(k_n, 1)
    achieved = k_flop / (k_launch_ms / 1e3) / 1e12
    line = {
        "metric": "differentiable paths/s (fwd+adjoint); time-to-loss vs plain Adam, same GPU",
        "value": value,
        "unit": "differentiable paths/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total_ms / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32 (radiance/gradients), f64 (meta-estimator state)",
        "data": "synthetic",
        "config": {"workload": "textured 512x512, 256x256 RGB+roughness texture (262,144 params), "
                               "plane + 8 spheres, depth 6, roulette from vertex 3, "
                               "meta-estimator 2 prop + 1 FD spp",
                   "pixels": npix, "params": spec.n_params, "diff_paths_per_step": 4 * npix},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": PEAK_FP32_VECTOR_TFLOPS,
                     "unit": "TFLOP/s", "frac": achieved / PEAK_FP32_VECTOR_TFLOPS,
                     "traffic": measured_traffic(kname), "kernel": kname,
                     "kernel_ms": k_launch_ms, "paths_per_launch": k_paths,
                     "vertices_per_path": k_vpp},
        "vertices_per_s": value * vpp,
        "kernel_ms_per_step": {k: v[0] / max(v[1], 1) for k, v in ktimes.items()},
        "fd_shared_step": fd_shared,
        "cpu_baseline": cpu,
        "time_to_loss": ttl,
        "batched": bat,
        "meshes": mesh,
        "volume": vol,
        "ablations": abl,
        "large_time_to_rmse": large,
    }
    print(json.dumps(line))


if __name__ == "__main__":
    main()
