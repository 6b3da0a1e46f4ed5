#!/usr/bin/env python3
"""Benchmark of the joint sampling-and-optimisation hot path on one MI355X.

Workload (the headline): the 2048x2048 terrain problem -- a fractal
heightfield of 999,698 triangles and 32 spheres behind a four-wide BVH, one
512x512 texture of base colour RGB + metalness + roughness (1,310,720
parameters), path depth 12 with Russian roulette from vertex 3 -- optimised
with the meta-estimator at 2 proportional + 1 finite-difference samples per
pixel.  A step is one call of jso_grad_step: primal renders for the adjoint
images, the replayed adjoint of 2 proportional paths and 1 finite-difference
path pair per pixel (4 differentiable paths per pixel), and the fused
meta-estimator + stabilised step.  Inputs are synthetic and already resident
on the GPU when the timed region starts.

Prints one JSON line.  `value` = differentiable paths/s (forward + replayed
adjoint).  `roofline` = the dominant kernel of the step (forward tracing or
the replayed adjoint, whichever takes longer per launch; the other follows in
`roofline_other_kernel`): the adjoint against HBM (its algorithmic bytes per
launch over its HIP-event launch time, beside its FP32 atomic rate against
the measured atomic peak), the forward against the VALU lane-operation rate
(operations per vertex from rocprofv3 counters x vertices counted on the
GPU); `traffic` = HBM bytes per launch from the committed rocprofv3 counter
summary (null when the kernel changed since it was taken).
`microbenchmarks` = the measured copy bandwidth and atomic rates;
`cpu_baseline` = the FP64 CPU oracle on a crop of the same workload.
Extras: the 512x512 textured problem, time to loss against Adam-64, the
terrain's time to parameter RMSE, 64 problems in one batch, the meshes and
the volume.
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

# VALU lane operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (a
# wave64 instruction occupies a 16-lane SIMD for 4 cycles; the 157.3 TFLOP/s
# figure counts an FMA as 2 and packed FP32 as 2 more)
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# VALU lane operations the path kernels execute per surface vertex on the
# terrain workload (active lanes of every VALU instruction, traversal
# included), from rocprofv3 counters: SQ_INSTS_VALU x SQ_THREAD_CYCLES_VALU /
# SQ_ACTIVE_INST_VALU per dispatch over the dispatch's surface vertices
# (profiles/grad_step_terrain2048_kernel_trace_and_issue.md)
VALU_OPS_PER_VERTEX = {"k_forward": 6328.0, "k_adjoint": 2352.0}

KERNEL_SOURCES = ("paper_2309_15676_amd/csrc/device.h", "paper_2309_15676_amd/csrc/kernels.h",
                  "paper_2309_15676_amd/csrc/kernels.hip")
TRAFFIC_SUMMARY = "profiles/%s_terrain2048_hbm_traffic.md"
VOLUME_SUMMARY = "profiles/volume256_kernel_trace_traffic.md"


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profile_record(path: str, prefix: str):
    """The JSON record on the line starting with `prefix` of a committed
    rocprofv3 counter summary, or None when the kernel sources changed since
    the counters were taken (or there is no such summary)."""
    path = os.path.join(ROOT, path)
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        for line in fh:
            if line.startswith(prefix):
                rec = json.loads(line[len(prefix):])
                if rec.get("source_sha256") == kernel_source_hash():
                    return rec
    return None


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary, or None when the kernel sources changed since it was taken."""
    rec = profile_record(TRAFFIC_SUMMARY % kernel, "traffic-json: ")
    return rec["bytes_per_launch"] if rec else None


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


def time_to_loss(prob, init, gt, target, args, iters: int, seeds: int, label: str,
                 lam: float = 0.0, etas=None):
    """Wall-clock (grad_step calls only; evaluations off the clock) for the
    meta-estimator at 2 proportional + 1 FD spp (replay pair, and shared path)
    to reach plain Adam-64's loss, same GPU, same process.

    Reference loss: Adam at 64 spp runs `iters` iterations at every learning
    rate of the grid with optimisation seed 0; the rate with the lowest final
    evaluation loss is kept and run with seeds 1 .. seeds-1 too; the reference
    is the median over seeds of the final loss.  Each method's time is the
    first time its evaluation loss reaches the reference: Adam's with its
    tuned rate, the meta-estimator's with the rate that reaches it first for
    seed 0 (then run with the other seeds), within Adam's wall-clock (a run
    that does not get there within it is not faster).  Reported per seed and
    as medians (a run that never reaches the reference counts as infinite).
    lam > 0: both methods precondition their texture gradients (Large Steps)."""
    import torch

    from paper_2309_15676_amd import _lib as L

    ev_seed, ev_spp = 777, 256
    T = target.float()

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

    def median(xs):
        v = sorted(float("inf") if x is None else x for x in xs)
        m = v[len(v) // 2] if len(v) % 2 else 0.5 * (v[len(v) // 2 - 1] + v[len(v) // 2])
        return None if m == float("inf") else m

    def adam_opts(eta, k):
        return L.step_opts(optimizer=L.JSO_OPT_ADAM, eta=eta, adam_spp=64,
                           seed=args.seed + 1 + 100 * k, precond_lambda=lam)

    def meta_opts(eta, k, mode):
        return L.step_opts(optimizer=L.JSO_OPT_META, eta=eta, beta_F=0.99, beta_D=0.9,
                           spp_prop=2, spp_fd=1, seed=args.seed + 2 + 100 * k,
                           precond_lambda=lam, fd_mode=mode)

    grid = etas or [float(x) for x in args.ttl_etas.split(",")]
    every = max(iters // 20, 1)
    adam0 = {}
    for eta in grid:
        adam0[eta] = run(adam_opts(eta, 0), iters, every)
        print("[bench]   %s: adam eta %g final %.4g" % (label[:24], eta, adam0[eta][-1][2]),
              file=sys.stderr, flush=True)
    eta_a = min(adam0, key=lambda e: adam0[e][-1][2])
    adam_runs = [adam0[eta_a]] + [run(adam_opts(eta_a, k), iters, every)
                                  for k in range(1, seeds)]
    ref = median([h[-1][2] for h in adam_runs])
    adam_t = [first(h, ref)[1] for h in adam_runs]
    budget = max(h[-1][1] for h in adam_runs)
    out_runs = {}
    for name, mode in (("meta", L.JSO_FD_REPLAY), ("meta_fd_shared", L.JSO_FD_SHARED)):
        tuned = {}
        for eta in grid:
            tuned[eta] = run(meta_opts(eta, 0, mode), 10 ** 9, every, seconds=budget)
            print("[bench]   %s: %s eta %g best %.4g after %d iterations" % (
                label[:24], name, eta, min(h[2] for h in tuned[eta]), tuned[eta][-1][0]),
                file=sys.stderr, flush=True)
        reach = {e: first(h, ref)[1] for e, h in tuned.items()}
        ok = [e for e in grid if reach[e] is not None]
        eta_m = min(ok, key=lambda e: reach[e]) if ok else min(
            tuned, key=lambda e: min(h[2] for h in tuned[e]))
        hs = [tuned[eta_m]] + [run(meta_opts(eta_m, k, mode), 10 ** 9, every, seconds=budget)
                               for k in range(1, seeds)]
        ts = [first(h, ref)[1] for h in hs]
        its = [first(h, ref)[0] for h in hs]
        tm = median(ts)
        out_runs[name] = {
            "spp": "2 prop + 1 FD" + (" (shared path)" if mode == L.JSO_FD_SHARED else ""),
            "eta": eta_m, "seconds_per_seed": ts, "iterations_per_seed": its,
            "best_loss_per_seed": [min(h[2] for h in x) for x in hs],
            "seconds_median": tm,
            "speedup": (median(adam_t) / tm) if (tm and median(adam_t)) else None,
            "best_loss_by_eta_seed0": {str(e): min(h[2] for h in tuned[e]) for e in grid},
            "ms_per_iteration": 1e3 * hs[0][-1][1] / max(hs[0][-1][0], 1)}
    return {
        "workload": label,
        "evaluation": "L2 of a %d-spp render (fixed evaluation stream) against the target, "
                      "off the clock" % ev_spp,
        "protocol": "Adam-64 for %d iterations, learning rate tuned on seed 0 over %s (lowest "
                    "final loss), %d seeds; reference = median final loss; each method's time "
                    "= first evaluation at or below it, median over seeds; meta-estimator "
                    "rates tuned on seed 0 within Adam's wall-clock" % (iters, grid, seeds),
        "reference_loss": ref,
        "loss_at_ground_truth": floor,
        "adam": {"spp": 64, "eta": eta_a, "seconds_per_seed": adam_t,
                 "seconds_median": median(adam_t),
                 "final_loss_per_seed": [h[-1][2] for h in adam_runs],
                 "final_loss_by_eta_seed0": {str(e): adam0[e][-1][2] for e in grid},
                 "ms_per_iteration": 1e3 * adam_runs[0][-1][1] / max(adam_runs[0][-1][0], 1)},
        "meta": out_runs["meta"],
        "meta_fd_shared": out_runs["meta_fd_shared"],
        "speedup": out_runs["meta"]["speedup"],
        "speedup_fd_shared": out_runs["meta_fd_shared"]["speedup"],
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


def large_time_to_rmse(prob, gt, init, args):
    """The 2048x2048 terrain problem (1.0M triangles + 32 spheres, 512x512
    texture of 5 channels): parameter-space RMSE against the ground truth
    over wall-clock (grad_step calls only) for the meta-estimator (2 prop +
    1 FD spp, replay pair and shared path) and plain Adam at 32 and 64 spp.
    The RMSE counts the observable parameters only: every channel of the
    texels that a 64-spp backward pass at the ground truth touches.  Each
    run stops at RMSE 1e-2, at 2000 iterations, or at args.large_ttl_seconds
    of GPU time."""
    import numpy as np
    import torch

    from paper_2309_15676_amd import _lib as L

    spec = prob.spec
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
            ("meta_eta0.01", L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, seed=args.seed)),
            ("meta_fd_shared_eta0.01", L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01,
                                                   seed=args.seed, fd_mode=L.JSO_FD_SHARED)),
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
        reach = {"%.4g" % lv: next((h[1] for h in hist if h[2] <= lv), None) for lv in levels}
        runs[name] = {"seconds_to_rmse": reach, "final_rmse": hist[-1][2],
                      "iterations": it, "seconds": clock,
                      "ms_per_iteration": 1e3 * clock / max(it, 1)}
        print("[bench] large problem %s: %s" % (name, json.dumps(runs[name])), file=sys.stderr,
              flush=True)
    prob.set_params(init)
    return {"workload": "2048x2048 terrain (999,698 triangles) + 32 spheres, 512x512 texture "
                        "of RGB + metalness + roughness (1,310,720 params), depth 12, roulette "
                        "from vertex 3; target at %d spp" % args.large_target_spp,
            "observable_params": int(obs.sum()), "total_params": spec.n_params,
            "initial_rmse": r0, "budget_seconds": args.large_ttl_seconds, "runs": runs}


def batched_throughput(context, args):
    """64 independent problems of uneven size (image side 64-512, 5-65,536
    parameters, own seeds and iteration budgets): differentiable paths/s of
    one iteration for all of them, (a) as a batch replayed from a captured
    HIP graph with the launch configuration (tile shape, persistent grid)
    picked by the autotuner, and the same launches issued directly, (b) as one
    jso_grad_step over all problems (one launch per kernel, tuned configuration),
    (c) as one jso_grad_step per problem."""
    import numpy as np
    import torch

    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd import inputs as I
    from paper_2309_15676_amd.problem import Batch, Problem, grad_step_many

    cfg = I.config_batched(64, seed=args.seed)
    ctx = context
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
    best, config_ms = b.autotune(3)  # state is restored after each trial
    # the same launches issued directly (no graph), tuned configuration; the
    # two batches step the same problems in turn, so both see the same
    # optimisation states, each iteration timed on its own
    b1 = Batch(probs, opts, max_iters=[c["max_iter"] for c in cfg], use_graph=False)
    b.step(2)
    b1.step(2)
    torch.cuda.synchronize()
    t_graph, t_direct = [], []
    for _ in range(steps):
        for bb, out_t in ((b, t_graph), (b1, t_direct)):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            bb.step(1)
            e1.record()
            torch.cuda.synchronize()
            out_t.append(e0.elapsed_time(e1))
    ms_graph = float(np.median(t_graph))
    ms_direct = float(np.median(t_direct))
    # several iterations per replay call: consecutive graph launches
    ms_graph_run = timed(lambda n: b.step(n))
    b.close()
    b1.close()

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
        "autotune": {"best": L.config_name(best),
                     "ms_per_iteration": {L.config_name(c): m for c, m in enumerate(config_ms)}},
        "graph": {"ms_per_iteration": ms_graph, "paths_per_s": paths / (ms_graph / 1e3),
                  "config": L.config_name(best),
                  "ms_per_iteration_in_runs": ms_graph_run},
        "batch_direct_launches": {"ms_per_iteration": ms_direct, "config": L.config_name(best),
                                  "note": "median over iterations alternating with the graph's, "
                                          "on the same problems"},
        "one_launch_per_kernel": {"ms_per_iteration": ms_together,
                                  "paths_per_s": paths / (ms_together / 1e3)},
        "one_grad_step_per_problem": {"ms_per_iteration": ms_each,
                                      "paths_per_s": paths / (ms_each / 1e3)},
    }


META_BYTES_PER_PARAM = 108  # k_meta: reads 52 B, writes 56 B per parameter


def volume_workload(context, args, ub=None):
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
    # the replay is bound by the L2's atomic requests (one per 16-byte voxel row
    # and distinct 64-byte segment of an instruction): requests per launch from
    # the committed counter summary, against the rate of random 16-byte-row
    # atomics measured above
    ka = out["meta_step"]["kernel"]["adjoint"]["ms_per_launch"]
    rec = profile_record(VOLUME_SUMMARY, "atomics-json: ")
    req = rec["meta_adjoint_requests_per_launch"] if rec else None
    peak = ub["atomic_ops_per_s_rows"] / 4 if ub else None
    out["k_vol_adjoint_roofline"] = {
        "bound": "atomic", "ms": ka, "requests_per_launch": req,
        "achieved_requests_per_s": req / (ka / 1e3) if req else None,
        "peak_requests_per_s": peak,
        "frac": req / (ka / 1e3) / peak if req and peak else None}
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


KERNELS = ((0, "forward"), (4, "finalize"), (1, "adjoint"), (2, "meta"))  # JSO_K_* ids


def timed_steps(prob, opts, steps: int, warmup: int):
    """Wall-clock of `steps` grad_step calls (HIP events on torch's stream,
    which the context is bound to) and, over the same region, each kernel
    class's device time from the library's HIP events around its launches."""
    import torch

    from paper_2309_15676_amd import _lib as L
    ctx = prob.ctx
    for _ in range(warmup):
        prob.grad_step(opts)
    torch.cuda.synchronize()
    L.check(L.jso_set_timing(ctx, True), ctx)
    for k in range(L.JSO_K_COUNT):
        L.jso_get_kernel_time(ctx, k, reset=True)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(steps):
        prob.grad_step(opts)
    e1.record()
    torch.cuda.synchronize()
    kt = {name: L.jso_get_kernel_time(ctx, k) for k, name in KERNELS}
    L.check(L.jso_set_timing(ctx, False), ctx)
    return e0.elapsed_time(e1), kt


def counted_work(prob, opts, n: int):
    """Paths and surface vertices of the path launches, counted on the GPU
    over n further steps (outside any timed region), per step."""
    from paper_2309_15676_amd import _lib as L
    ctx = prob.ctx
    L.check(L.jso_set_work_counting(ctx, True), ctx)
    L.jso_get_work(ctx, reset=True)
    for _ in range(n):
        prob.grad_step(opts)
    rep_paths, rep_verts, fwd_paths, fwd_verts = L.jso_get_work(ctx, reset=True)
    L.check(L.jso_set_work_counting(ctx, False), ctx)
    return rep_paths / n, rep_verts / n, fwd_paths / n, fwd_verts / n


def microbenchmarks(context, n_params: int):
    """The roofline denominators measured on this GPU: a plain device copy of
    1 GiB (bytes read + written per second), and no-return FP32 atomic adds
    into a buffer of the headline's parameter count under five address
    patterns (operations per second), and the gap between dependent launches
    issued on a stream and replayed from a captured graph."""
    import torch

    from paper_2309_15676_amd import _lib as L
    ctx = context.bind()
    nbytes = 1 << 30
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    ms = L.jso_ub_copy(ctx, dst.data_ptr(), src.data_ptr(), nbytes, 5)
    out = {"copy_GBs": 2 * nbytes / (ms / 1e3) / 1e9, "copy_bytes": nbytes, "copy_ms": ms}
    del src, dst
    buf = torch.zeros(n_params, dtype=torch.float32, device="cuda")
    n_ops = 1 << 26
    for name, pat in (("random", L.JSO_UB_RANDOM), ("lines", L.JSO_UB_LINES),
                      ("rows", L.JSO_UB_ROWS), ("16_addresses", L.JSO_UB_16),
                      ("same_address", L.JSO_UB_SAME)):
        ms = L.jso_ub_atomics(ctx, buf.data_ptr(), n_params, pat, n_ops, 3)
        out["atomic_ops_per_s_" + name] = n_ops / (ms / 1e3)
    out["atomic_buffer_floats"] = n_params
    out["atomic_ops"] = n_ops
    del buf
    # gap between dependent launches: 64 one-block kernels issued on the
    # stream, and the same chain replayed from a captured graph
    ctr = torch.zeros(1, dtype=torch.int32, device="cuda")
    for name, graph in (("stream", False), ("graph", True)):
        ms = L.jso_ub_launch(ctx, ctr.data_ptr(), 64, graph, 20)
        out["launch_gap_us_" + name] = ms * 1e3 / 64
    expect = 64 * 21 * 2
    out["launch_chain_count_ok"] = int(ctr.item()) == expect
    del ctr
    torch.cuda.empty_cache()
    return out


def cpu_baseline_crop(spec, params, target, seed: int, crop, label: str):
    """The FP64 oracle, as it stands, on this host's share of cores (at most
    16 threads, the CPU share of one GPU): one iteration's gradient samples
    (2 proportional + 1 finite-difference pair per pixel) and the
    meta-estimator step on a crop of the workload, timed whole."""
    import numpy as np

    import oracle as O
    from oracle import meta as OM

    threads = max(1, min(len(os.sched_getaffinity(0)), 16))
    lo, hi = spec.param_bounds()
    opt = OM.MetaOptimizer(params, lo, hi, eta=float(np.float32(0.01)))
    prev = np.clip(np.asarray(params, np.float32) + np.float32(0.01), lo, hi)
    t0 = time.perf_counter()
    r = O.gradient_pair(spec, np.asarray(params, np.float64), prev.astype(np.float64), target,
                        seed, 1, crop=crop, nthreads=threads)
    opt.step(r["F"], r["dF"])
    dt = time.perf_counter() - t0
    px = (crop[2] - crop[0]) * (crop[3] - crop[1])
    return dict(value=4 * px / dt, unit="differentiable paths/s", cores=threads, kind="oracle",
                sample="one iteration (gradient samples of 2 proportional + 1 finite-difference "
                       "pair per pixel, brute-force intersection, then the meta-estimator step "
                       "over all %d parameters) on the %dx%d crop at (%d, %d) of %s, %.1f s" % (
                           spec.n_params, crop[2] - crop[0], crop[3] - crop[1], crop[0], crop[1],
                           label, dt))


def textured_extra(context, args):
    """The 512x512 textured problem (plane + 8 spheres, 256x256 RGB +
    roughness texture, 262,144 parameters, depth 6): meta-estimator step
    (replay pair and shared path), kernel times, and the adjoint against its
    HBM and atomic roofline."""
    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd import inputs as I
    from paper_2309_15676_amd.problem import Problem

    spec, gt, init = I.config_textured()
    prob = Problem(spec, context=context)
    target = prob.render(gt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET, spp=args.target_spp)
    prob.set_target(target)
    prob.set_params(init)
    opts = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, beta_F=0.99, beta_D=0.9, spp_prop=2,
                       spp_fd=1, seed=args.seed)
    total_ms, kt = timed_steps(prob, opts, args.steps, args.warmup)
    work = counted_work(prob, opts, 3)
    npix = spec.n_pixels
    out = {"workload": "textured 512x512, 256x256 RGB+roughness texture (262,144 params), "
                       "plane + 8 spheres, depth 6, roulette from vertex 3, meta-estimator 2 "
                       "prop + 1 FD spp",
           "ms_per_step": total_ms / args.steps,
           "diff_paths_per_s": 4 * npix * args.steps / (total_ms / 1e3),
           "kernel_ms_per_step": {k: v[0] / args.steps for k, v in kt.items()},
           "adjoint": adjoint_roofline(spec, prob, kt, work, None, args.steps),
           "vertices_per_replayed_path": work[1] / max(work[0], 1)}
    prob.set_params(init)
    opts_sh = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, beta_F=0.99, beta_D=0.9,
                          spp_prop=2, spp_fd=1, seed=args.seed, fd_mode=L.JSO_FD_SHARED)
    ms_sh, kt_sh = timed_steps(prob, opts_sh, args.steps, args.warmup)
    out["fd_shared_step"] = {"ms_per_step": ms_sh / args.steps,
                             "kernel_ms_per_step": {k: v[0] / args.steps
                                                    for k, v in kt_sh.items()},
                             "paths_traced_per_step": 3 * npix}
    prob.set_params(init)
    return out, prob, spec, gt, init, target


def scene_bytes(prob) -> int:
    """Bytes of the scene data a path launch reads at least once: the BVH
    (128-byte four-wide nodes, 48 bytes per triangle) of a mesh."""
    n_tris = len(prob.spec.tris) if len(prob.spec.tris) else 0
    if not n_tris:
        return 0
    # a four-wide hierarchy over leaves of a few triangles: at most n_tris / 3
    # nodes in practice; the exact count is not exported, so bound it by that
    return 48 * n_tris + 128 * (n_tris // 3)


def adjoint_roofline(spec, prob, kt, work, ub, steps):
    """k_adjoint against the bounds of its work per step.

    Algorithmic work of a step's replay (its one or two adjoint launches):
    every surface vertex scatters its material gradient into the 4 texels
    of its bilinear footprint, 4 n_ch FP32 atomics of 4 bytes; each replayed
    path reads its radiance slot (24 B), its pixel's adjoint colour (12 B)
    and the hit records of its camera ray and of each vertex's continuation
    ray (12 B each; records cover the first three rays, nearly every ray
    here); the parameters (4 B each) and the scene's BVH are read at least
    once.  HBM: those bytes over the launch time against 8 TB/s; atomics:
    the 4 n_ch atomics per vertex over the launch time against the measured
    peak of no-return FP32 atomics (coalesced 64-byte segments, and random
    addresses)."""
    # a step's replay is one launch, or two when it holds both replay pairs and
    # single paths (the pair kernel and the single-path kernel): the figures
    # below are per step, over the step's adjoint launches together
    ms, calls = kt["adjoint"]
    launch_ms = ms / max(steps, 1)
    rep_paths, rep_verts = work[0], work[1]
    n_ch = spec.n_ch
    atomics = rep_verts * 4 * n_ch
    bytes_ = (atomics * 4 + rep_paths * (24 + 12) + 12 * (rep_paths + rep_verts) +
              4 * spec.n_params + scene_bytes(prob))
    achieved = bytes_ / (launch_ms / 1e3) / 1e9
    out = {"bound": "hbm", "achieved": achieved, "peak": PEAK_HBM_GBS, "unit": "GB/s",
           "frac": achieved / PEAK_HBM_GBS, "kernel": "k_adjoint", "kernel_ms": launch_ms,
           "algorithmic_bytes": bytes_, "paths_per_launch": rep_paths,
           "vertices_per_launch": rep_verts, "vertices_per_path": rep_verts / max(rep_paths, 1),
           "atomics_per_launch": atomics,
           "atomics_per_s": atomics / (launch_ms / 1e3),
           "launches_per_step": calls / max(steps, 1)}
    if ub:
        out["atomic_frac_lines"] = out["atomics_per_s"] / ub["atomic_ops_per_s_lines"]
        out["atomic_frac_random"] = out["atomics_per_s"] / ub["atomic_ops_per_s_random"]
        out["frac_of_measured_copy"] = achieved / ub["copy_GBs"]
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=30)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--target-spp", type=int, default=4096,
                    help="samples per pixel of the 512x512 target render")
    ap.add_argument("--large-target-spp", type=int, default=64,
                    help="samples per pixel of the 2048x2048 target render")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-microbench", action="store_true")
    ap.add_argument("--copy-mib", type=int, default=0,
                    help="also run a plain copy of this many MiB (counter calibration)")
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--no-extras", action="store_true",
                    help="the headline only (no 512x512, batch, mesh, volume or time-to-loss "
                         "runs)")
    ap.add_argument("--ttl-iters", type=int, default=1000,
                    help="Adam-64 iteration budget of the textured time-to-loss comparison "
                         "(0: skip the comparisons)")
    ap.add_argument("--ttl-seeds", type=int, default=3,
                    help="optimisation seeds of the textured time-to-loss comparison (median)")
    ap.add_argument("--ttl-etas", default="0.001,0.003,0.01,0.03,0.1")
    ap.add_argument("--ttl-lambda", type=float, default=0.0,
                    help="also compare both methods with preconditioned texture gradients "
                         "(Large Steps) at this lambda (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=20,
                    help="iterations timed for the 64-problem batch (0: skip it)")
    ap.add_argument("--batch-target-spp", type=int, default=256)
    ap.add_argument("--ablation-iters", type=int, default=0,
                    help="meta-estimator iterations of the ablation runs on the textured "
                         "problem (the tiny problem runs 200; 0: skip)")
    ap.add_argument("--large-ttl-seconds", type=float, default=15.0,
                    help="GPU-seconds per run of the terrain time-to-RMSE comparison "
                         "(meta-estimator vs Adam at 32 and 64 spp; 0: skip)")
    ap.add_argument("--volume-steps", type=int, default=5,
                    help="timed calls per volume configuration (0 = skip the volume workload)")
    ap.add_argument("--volume-ttl-seconds", type=float, default=4.0,
                    help="GPU-seconds per run of the volume equal-time comparison (0: skip)")
    ap.add_argument("--volume-ttl-res", type=int, default=128,
                    help="voxels per side (and view size) of the equal-time comparison")
    ap.add_argument("--mesh-steps", type=int, default=10,
                    help="timed calls per mesh workload (0 = skip the mesh workloads)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py: the benchmark runs on one GPU; --gpus %d is not supported "
              "(the multi-GPU sharding is a design note, not built)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2309_15676_amd import _lib as L
    from paper_2309_15676_amd import inputs as I
    from paper_2309_15676_amd.problem import Context, Problem

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    context = Context(0)
    # ---- headline: the 2048x2048 terrain problem -------------------------
    t0 = time.time()
    spec, gt, init = I.config_large()
    prob = Problem(spec, context=context)
    load_s = time.time() - t0
    print("[bench] terrain loaded in %.1f s; rendering target at %d spp" % (
        load_s, args.large_target_spp), file=sys.stderr, flush=True)
    target = prob.render(gt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET,
                         spp=args.large_target_spp)
    prob.set_target(target)
    prob.set_params(init)
    opts = L.step_opts(optimizer=L.JSO_OPT_META, eta=0.01, beta_F=0.99, beta_D=0.9, spp_prop=2,
                       spp_fd=1, seed=args.seed)
    total_ms, ktimes = timed_steps(prob, opts, args.steps, args.warmup)
    work = counted_work(prob, opts, 2)
    st = prob.grad_step(opts, want_stats=True)
    npix = spec.n_pixels
    value = 4 * npix * args.steps / (total_ms / 1e3)
    print("[bench] terrain: %.3f ms per step, kernels %s, loss %.5g; per step: replayed "
          "paths %d, their vertices %d, forward paths %d, their vertices %d" % (
              total_ms / args.steps, {k: round(v[0] / args.steps, 3) for k, v in ktimes.items()},
              st.loss, *work), file=sys.stderr, flush=True)
    ub = None
    if not args.no_microbench:
        ub = microbenchmarks(context, spec.n_params)
        print("[bench] microbenchmarks: %s" % json.dumps(ub), file=sys.stderr, flush=True)
    adj = adjoint_roofline(spec, prob, ktimes, work, ub, args.steps)
    fwd_ms, fwd_calls = ktimes["forward"]
    fwd_launch_ms = fwd_ms / max(fwd_calls, 1)
    fwd_verts = work[3] * args.steps / max(fwd_calls, 1)
    fwd = {"kernel": "k_forward", "kernel_ms": fwd_launch_ms, "bound": "alu",
           "paths_per_launch": work[2] * args.steps / max(fwd_calls, 1),
           "vertices_per_launch": fwd_verts, "vertices_per_path": work[3] / max(work[2], 1),
           "achieved": None, "peak": PEAK_VALU_TOPS, "unit": "T VALU lane-op/s", "frac": None}
    if VALU_OPS_PER_VERTEX["k_forward"]:
        fwd["achieved"] = (fwd_verts * VALU_OPS_PER_VERTEX["k_forward"] /
                           (fwd_launch_ms / 1e3) / 1e12)
        fwd["frac"] = fwd["achieved"] / PEAK_VALU_TOPS
    if VALU_OPS_PER_VERTEX["k_adjoint"]:
        adj["alu_achieved_Tops"] = (adj["vertices_per_launch"] * VALU_OPS_PER_VERTEX["k_adjoint"]
                                    / (adj["kernel_ms"] / 1e3) / 1e12)
        adj["alu_frac"] = adj["alu_achieved_Tops"] / PEAK_VALU_TOPS
    # the dominant kernel's roofline leads; the other follows
    if fwd_launch_ms > adj["kernel_ms"]:
        roof, other = fwd, adj
    else:
        roof, other = adj, fwd
    roof = dict(roof)
    roof["traffic"] = measured_traffic(roof["kernel"])
    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] CPU oracle baseline", file=sys.stderr, flush=True)
        Tn = target.cpu().numpy().astype(np.float64)
        cpu = cpu_baseline_crop(spec, init, Tn, args.seed, (1016, 1100, 1032, 1116),
                                "the 2048x2048 terrain")
        print("[bench] CPU baseline: %s" % json.dumps(cpu), file=sys.stderr, flush=True)
    large = None
    if args.large_ttl_seconds > 0 and not args.no_extras:
        print("[bench] terrain time to RMSE", file=sys.stderr, flush=True)
        large = large_time_to_rmse(prob, gt, init, args)
    del prob, target
    torch.cuda.empty_cache()

    extras = {}
    if not args.no_extras:
        print("[bench] 512x512 textured problem", file=sys.stderr, flush=True)
        tex, tprob, tspec, tgt, tinit, ttarget = textured_extra(context, args)
        extras["textured_512"] = tex
        print("[bench] textured: %s" % json.dumps(tex), file=sys.stderr, flush=True)
        if args.ttl_iters > 0:
            print("[bench] time to loss: Adam-64 vs meta-estimator", file=sys.stderr, flush=True)
            ttl = {}
            sspec, sgt, sinit = I.config_tiny()
            sprob = Problem(sspec, context=context)
            starget = sprob.render(sgt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET, spp=1024)
            sprob.set_target(starget)
            ttl["tiny"] = time_to_loss(
                sprob, sinit, sgt, starget, args, 200, 1,
                "64x64, unit sphere on a grey plane, 5 global parameters (RGB, metalness, "
                "roughness), depth 3, target at 1024 spp")
            print("[bench] time to loss: %s" % json.dumps(ttl["tiny"]), file=sys.stderr,
                  flush=True)
            ttl["textured"] = time_to_loss(
                tprob, tinit, tgt, ttarget, args, args.ttl_iters, args.ttl_seeds,
                "the 512x512 textured problem (262,144 texel parameters, no preconditioning)")
            print("[bench] time to loss: %s" % json.dumps(ttl["textured"]), file=sys.stderr,
                  flush=True)
            if args.ttl_lambda > 0:
                ttl["textured_preconditioned"] = time_to_loss(
                    tprob, tinit, tgt, ttarget, args, args.ttl_iters, 1,
                    "the 512x512 textured problem, both methods with Large-Steps preconditioned "
                    "texture gradients", lam=args.ttl_lambda, etas=[0.01, 0.03, 0.1, 0.3])
            extras["time_to_loss"] = ttl
        if args.ablation_iters > 0:
            print("[bench] meta-estimator ablations", file=sys.stderr, flush=True)
            aspec, agt, ainit = I.config_tiny()
            aprob = Problem(aspec, context=context)
            atarget = aprob.render(agt, seed=12345, iteration=0, tag=L.JSO_TAG_TARGET, spp=1024)
            aprob.set_target(atarget)
            extras["ablations"] = {
                "tiny": ablations(aprob, ainit, atarget, 200, 0.01, args.seed + 2,
                                  "64x64, 5 global parameters"),
                "textured": ablations(tprob, tinit, ttarget, args.ablation_iters, 0.003,
                                      args.seed + 2, "512x512, 262,144 texel parameters")}
        del tprob
        torch.cuda.empty_cache()
        if args.batch_steps > 0:
            print("[bench] 64-problem batch", file=sys.stderr, flush=True)
            extras["batched"] = batched_throughput(context, args)
            print("[bench] batch: %s" % json.dumps(extras["batched"]), file=sys.stderr,
                  flush=True)
        if args.mesh_steps > 0:
            print("[bench] mesh workloads", file=sys.stderr, flush=True)
            extras["meshes"] = mesh_workloads(context, args)
        if args.volume_steps > 0:
            print("[bench] volume workload", file=sys.stderr, flush=True)
            extras["volume"] = volume_workload(context, args, ub)
    if args.copy_mib > 0:
        copy_calibration(args.copy_mib)
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
        "config": {"workload": "2048x2048 terrain: fractal heightfield of 999,698 triangles + "
                               "32 spheres, 512x512 texture of RGB + metalness + roughness "
                               "(1,310,720 params), depth 12, roulette from vertex 3, "
                               "meta-estimator 2 prop + 1 FD spp",
                   "pixels": npix, "params": spec.n_params, "triangles": len(spec.tris),
                   "diff_paths_per_step": 4 * npix},
        "roofline": roof,
        "roofline_other_kernel": other,
        "microbenchmarks": ub,
        "vertices_per_s": value * work[1] / max(work[0], 1),
        "kernel_ms_per_step": {k: v[0] / args.steps for k, v in ktimes.items()},
        "scene_load_s": load_s,
        "cpu_baseline": cpu,
        "large_time_to_rmse": large,
    }
    line.update(extras)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
