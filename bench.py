"""Benchmark of the TR-ScaledBRSGD hot path on one MI355X.

Workload (default): the ill-conditioned planted ring of the second synthetic
experiment at 400 x 400 x 400 (64M FP32 entries), ranks 10, each core's
mode-2 unfolding with singular values geometric from 1 to 1e-4, mini-batch
|F_n| = 4096 with H_n = F_n, uniform fibers, FP64 Gram and inverse.  One
step = mode pick, draws, sampled subchain, fiber gather, gradient, Gram,
inverse and update (every row of the single-problem hot path).

Prints one JSON line: steps/s of the --prec form (whole job), the same for
the other form (FP32 vs BF16 mixed), the dominant kernel's roofline (HIP
start/stop events recorded by each dispatch of the kernel itself), time
to RSE 1e-4 for
both forms (capped), the 64-problem batched workload (problem-steps/s with
the tuner's tile choice), and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import re
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": (157.3, "TFLOP/s"), "bf16": (2516.6, "TFLOP/s"), "f16": (2516.6, "TFLOP/s"),
        "f64": (78.6, "TFLOP/s")}
HBM_PEAK_GBS = 8000.0


def parse(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--prec", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--alpha", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=24.0,
                    help="CPU work of the oracle baseline, split between 1 thread and all threads")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the Gram/inverse branch on the main stream too")
    ap.add_argument("--ttt-steps", type=int, default=3000,
                    help="step cap of each time-to-target run (0: skip them)")
    ap.add_argument("--copy-probe", type=int, default=0, metavar="MIB",
                    help="only run 20 plain device copies of MIB MiB (counter calibration) and exit")
    ap.add_argument("--batch-steps", type=int, default=50,
                    help="timed steps of the 64-problem batched workload (0: skip it)")
    ap.add_argument("--autograd-steps", type=int, default=4000,
                    help="step cap of the differentiation workload's time-to-target runs (0: skip the leg)")
    ap.add_argument("--seeds", type=int, default=10,
                    help="time the headline step for seeds 0..SEEDS-1 too (mean and std; 0: skip)")
    ap.add_argument("--methods-budget", type=float, default=0.25,
                    help="seconds of GPU time per comparison method (0: skip the leg)")
    return ap.parse_args(argv)


def hip_events(n):
    import torch
    hip = C.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
    hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
    hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
    hip.hipEventDestroy.argtypes = [C.c_void_p]
    hip.hipEventRecord.argtypes = [C.c_void_p, C.c_void_p]
    evs = []
    for _ in range(n):
        e = C.c_void_p()
        assert hip.hipEventCreate(C.byref(e)) == 0
        evs.append(e)
    return hip, evs


def elapsed_ms(hip, a, b):
    out = C.c_float()
    assert hip.hipEventElapsedTime(C.byref(out), a, b) == 0
    return float(out.value)


def graph_schedule(K: int, G: int = 50):
    """Graph lengths and replay counts that time exactly K steps: full
    graphs of min(G, K) steps, then one graph of the remainder."""
    if K < 1:
        raise ValueError("--steps must be at least 1")
    g = min(G, K)
    plan = [(g, K // g)]
    if K % g:
        plan.append((K % g, 1))
    assert sum(n * r for n, r in plan) == K
    return plan


def replay_timed(solver, K: int, G: int = 50, hip=None, evs=None):
    """Capture the graphs of ``graph_schedule(K, G)`` (each capture runs
    one eager warm-up step first), replay each once untimed, then time
    exactly K steps of replays between two events on the current stream.
    Returns ms per step."""
    import torch
    plan = graph_schedule(K, G)
    graphs = [(solver.capture(n), r) for n, r in plan]
    for gr, _ in graphs:
        gr.replay()
    torch.cuda.synchronize()
    t_before = solver.t
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for gr, r in graphs:
        for _ in range(r):
            gr.replay()
    b.record()
    torch.cuda.synchronize()
    assert solver.t - t_before == K, (solver.t, t_before, K)
    ms = a.elapsed_time(b) / K
    del graphs
    return ms


def build_problem(seed, I, R, kappa, dev, kind="illcond"):
    """Planted 3-way ring at RMS 1 and the initial cores.  kind "illcond":
    each core's mode-2 unfolding U_n S V^T with singular values geometric
    from 1 to 1/kappa (second synthetic experiment); kind "gaussian":
    i.i.d. N(0, 1) cores (first synthetic experiment)."""
    import torch
    import tr_inputs as ti
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import cores_to_device
    N = 3
    true3 = (ti.illcond_cores(seed, N, I, R, kappa) if kind == "illcond"
             else ti.gaussian_cores(seed, N, I, R))
    desc = api.make_desc([I] * N, [R] * N, torch.float32)
    tcores = cores_to_device(true3, torch.float32, dev)
    X = api.tr_reconstruct(desc, tcores)
    ws = api.workspace(api.lib().tr_relerr_workspace_size(C.byref(desc)), dev)
    zero = [torch.zeros_like(c) for c in tcores]
    api.tr_relerr(desc, zero, X, ws=ws)          # ||X||^2 into ws[8:16]
    torch.cuda.synchronize()
    xx = float(ws[:16].view(torch.float64)[1].item())
    ms = xx / X.numel()
    # RMS 1: scale each core by ms^(-1/(2N)), then rebuild X.
    c = ms ** (-1.0 / (2 * N))
    true3 = [t * c for t in true3]
    tcores = cores_to_device(true3, torch.float32, dev)
    X = api.tr_reconstruct(desc, tcores, X)
    sig = (1.0 / R ** N) ** (1.0 / (2 * N))     # init: E[X^2] = sig^(2N) prod R_k = 1
    init3 = ti.gaussian_cores(seed + 1, N, I, R, scale=sig)
    return desc, X, true3, init3


BATCH_ETA = 0.2          # AdaGrad eta of the batched workload (both forms)
BATCH_TARGET = 1e-2      # RSE against the noise-free tensor, per problem


def batch_problem(b, dev):
    """One problem of the 64-problem workload: the planted tensor X_true
    (i.i.d. N(0,1) cores) rescaled to RMS 1, X = X_true + 40 dB noise (FP32),
    and the initial cores matched to X's second moment.  Deterministic in
    the instance's seed."""
    import torch
    import tr_inputs as ti
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import cores_to_device
    d32 = api.make_desc(b.I, b.R, torch.float32, torch.float32)
    true = cores_to_device(ti.gaussian_cores(b.seed, b.N, b.I, b.R), torch.float32, dev)
    Xt = api.tr_reconstruct(d32, true)
    Xt.div_(float(Xt.double().pow(2).mean().sqrt()))
    gen = torch.Generator(device=dev)
    gen.manual_seed(b.seed + 5)
    sigma = 10.0 ** (-40.0 / 20.0) * float(Xt.double().norm()) / (Xt.numel() ** 0.5)
    X = Xt + sigma * torch.randn(Xt.numel(), generator=gen, device=dev, dtype=torch.float32)
    sig = (float(X.double().pow(2).mean()) / float(np.prod(b.R))) ** (1.0 / (2 * b.N))
    init = ti.gaussian_cores(b.seed + 1, b.N, b.I, b.R, scale=sig)
    return d32, Xt, X, init


def build_batch(seed, dev):
    """The 64 independent planted problems (orders 3-5, sizes 16-128, ranks
    3-12, RMS 1, 40 dB noise, FP16 tensors, m = 1024, AdaGrad) as a TRBatch,
    with each problem's noise-free tensor (FP32) for the RSE."""
    import torch
    import tr_inputs as ti
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import TRBatch, cores_to_device
    insts = ti.batched_instances(seed)
    probs, truths = [], []
    for b in insts:
        d32, Xt, X, init = batch_problem(b, dev)
        d16 = api.make_desc(b.I, b.R, torch.float32, torch.float16)
        X16 = X.half()
        del X
        cores = cores_to_device(init, torch.float32, dev)
        reps = [api.tr_x_replicate(d16, X16, n) for n in range(b.N)]
        del X16
        truths.append((d32, Xt))
        probs.append(dict(cores=cores, Xrep=reps, I=b.I, R=b.R, m=1024,
                          rule=api.step_rule("adagrad", eta=BATCH_ETA), seed=b.seed))
    return TRBatch(probs, dev), insts, truths


def batch_time_to_target(B, truths, every=250, cap=4000):
    """Wall time until every problem's RSE (against its noise-free tensor)
    is <= BATCH_TARGET: ``every`` steps of all problems replay one captured
    graph, then the RSE of each problem not yet there is checked (the checks
    count).  Returns (seconds or None, steps, per-problem steps, worst ratio)."""
    import torch
    from paper_2303_16492_amd import api
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        B.run(every)
    reached = [None] * B.count
    steps = 0
    t0 = time.perf_counter()
    while steps < cap and any(r is None for r in reached):
        g.replay()
        steps += every
        for p, (d32, Xt) in enumerate(truths):
            if reached[p] is None and float(api.tr_relerr(d32, B.problems[p]["cores"], Xt)) <= BATCH_TARGET:
                reached[p] = steps
    wall = time.perf_counter() - t0
    done = all(r is not None for r in reached)
    del g
    return (round(wall, 4) if done else None), steps, reached, round(wall, 4)


def single_time_to_target(insts, dev, every=250, cap=4000):
    """The same problems stepped one at a time in FP32 (FP32 tensor, FP32
    matrix-core gradient, same AdaGrad eta, m = 1024), each to the same
    target; returns (total seconds, per-problem steps, steps/s of a single
    problem's step averaged over problems)."""
    import torch
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import TRSolver, cores_to_device
    total, per, rates = 0.0, [], []
    for b in insts:
        d32, Xt, X, init = batch_problem(b, dev)
        sol = TRSolver(cores_to_device(init, torch.float32, dev), X, b.I, b.R, 1024, law="U", scaled=False,
                       prec="f32", rule=api.step_rule("adagrad", eta=BATCH_ETA), seed=b.seed)
        snap = [c.clone() for c in sol.cores]
        g = sol.capture(every)
        for c, s_ in zip(sol.cores, snap):
            c.copy_(s_)
        for a in sol.accum:
            a.zero_()
        sol.t_dev.zero_()
        torch.cuda.synchronize()
        steps, ok = 0, False
        t0 = time.perf_counter()
        while steps < cap and not ok:
            g.replay()
            steps += every
            ok = float(api.tr_relerr(d32, sol.cores, Xt)) <= BATCH_TARGET
        wall = time.perf_counter() - t0
        total += wall
        per.append(steps if ok else None)
        rates.append(steps / wall)
        del g, sol, X, Xt
    torch.cuda.empty_cache()
    return round(total, 4), per, float(np.mean(rates))


AUTOGRAD_ETA = 0.005


def autograd_leg(dev, K=50, steps_cap=4000, every=250):
    """The differentiation workload: order 5, 32 per mode, ranks 8, planted
    Gaussian ring at RMS 1 + 30 dB noise, FP32, batches of B = 8192 sampled
    entries.  (1) Forward + backward through the torch.autograd.Function
    over the library's kernels, K pre-drawn batches: entries/s.  (2) Time
    to the target RSE (against the noise-free tensor) of the sampled-entry
    method (the same forward and backward kernels in the library's native
    loop, AdaGrad, every core per step, all entries observable) beside the
    plain FP32 fiber-sampling method (TR-BRSGD, AdaGrad, m = 256 fibers =
    8192 entries per step)."""
    import torch
    import tr_inputs as ti
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.autograd import tr_entry_loss
    from paper_2303_16492_amd.driver import TRSolver, cores_to_device
    N, I, R, B = 5, 32, 8, 8192
    desc = api.make_desc([I] * N, [R] * N, torch.float32)
    true = cores_to_device(ti.gaussian_cores(3, N, [I] * N, [R] * N), torch.float32, dev)
    Xt = api.tr_reconstruct(desc, true)
    Xt.div_(float(Xt.double().pow(2).mean().sqrt()))
    gen = torch.Generator(device=dev)
    gen.manual_seed(11)
    sigma = 10.0 ** (-30.0 / 20.0)
    X = Xt + sigma * torch.randn(Xt.numel(), generator=gen, device=dev, dtype=torch.float32)
    # local convergence: the planted cores (at the scale of the RMS-1 tensor)
    # with a 10% Gaussian perturbation; from i.i.d. random cores every form
    # stays at RSE ~1 on this order-5 ring for thousands of steps
    tc = ti.gaussian_cores(3, N, [I] * N, [R] * N)
    cfac = float(api.tr_reconstruct(desc, cores_to_device(tc, torch.float32, dev)).double().pow(2).mean().sqrt()) \
        ** (-1.0 / N)
    rng = np.random.default_rng(12)
    init = [cfac * c + 0.1 * cfac * np.sqrt(np.mean(c * c)) * rng.standard_normal(c.shape) for c in tc]
    P = N * I * R * R
    floor = sigma * (P / float(I ** N)) ** 0.5
    target = 10.0 * floor
    # (1) forward + backward through autograd
    cores = [c.requires_grad_() for c in cores_to_device(init, torch.float32, dev)]
    strides = torch.tensor([I ** k for k in range(N)], device=dev, dtype=torch.int64)
    batches = []
    for k in range(K):
        idx = torch.randint(0, I, (B, N), generator=gen, device=dev, dtype=torch.int64)
        batches.append((idx.to(torch.int32), X[(idx * strides).sum(1)].contiguous()))
    loss = tr_entry_loss(desc, batches[0][0], batches[0][1], cores)
    loss.backward()
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for idx, x in batches:
        loss = tr_entry_loss(desc, idx, x, cores)
        loss.backward()
    b.record()
    torch.cuda.synchronize()
    fb_ms = a.elapsed_time(b) / K
    del batches, cores
    # (2) time to target: the sampled-entry loop over every entry as observed
    obs_idx = torch.stack(torch.meshgrid(*[torch.arange(I, device=dev, dtype=torch.int32)] * N, indexing="ij"),
                          -1).flip(-1).reshape(-1, N).contiguous()          # first index fastest
    cfg = api.completion_config(B, rule=api.step_rule("adagrad", eta=AUTOGRAD_ETA), seed=7)
    runs = {}
    ecores = cores_to_device(init, torch.float32, dev)
    acc = [torch.zeros_like(c) for c in ecores]
    t_dev = torch.zeros(1, dtype=torch.int64, device=dev)
    st = torch.zeros(1, dtype=torch.int32, device=dev)
    ws = api.workspace(api.lib().tr_completion_workspace_size(C.byref(desc), C.byref(cfg)), dev)
    g = torch.cuda.CUDAGraph()
    sg = torch.cuda.Stream()
    sg.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=sg):
        api.tr_completion_run(desc, ecores, acc, obs_idx, X, cfg, t_dev, every, status=st, ws=ws)
    steps, rse = 0, float("nan")
    t0 = time.perf_counter()
    while steps < steps_cap:
        g.replay()
        steps += every
        rse = float(api.tr_relerr(desc, ecores, Xt))
        if rse <= target:
            break
    runs["sampled_entry"] = {"seconds": round(time.perf_counter() - t0, 4) if rse <= target else None,
                             "steps": steps, "rse_at_stop": rse, "entries_per_step": B}
    del g, obs_idx, ecores, acc
    sol = TRSolver(cores_to_device(init, torch.float32, dev), X, [I] * N, [R] * N, B // I, law="U",
                   scaled=False, prec="f32", rule=api.step_rule("adagrad", eta=AUTOGRAD_ETA), seed=7)
    snap = [c.clone() for c in sol.cores]
    g = sol.capture(every)
    for c, s_ in zip(sol.cores, snap):
        c.copy_(s_)
    for a_ in sol.accum:
        a_.zero_()
    sol.t_dev.zero_()
    torch.cuda.synchronize()
    steps, rse = 0, float("nan")
    t0 = time.perf_counter()
    while steps < steps_cap:
        g.replay()
        steps += every
        rse = float(api.tr_relerr(desc, sol.cores, Xt))
        if rse <= target:
            break
    runs["plain_fp32_fibers"] = {"seconds": round(time.perf_counter() - t0, 4) if rse <= target else None,
                                 "steps": steps, "rse_at_stop": rse, "entries_per_step": (B // I) * I}
    del g, sol
    return {"workload": "autograd-n5-i32-r8-b8192", "B": B, "noise_db": 30, "precision": "fp32",
            "fwd_bwd_ms_per_batch": round(fb_ms, 5), "fwd_bwd_entries_per_s": round(B / (fb_ms * 1e-3), 1),
            "fwd_bwd_timing": f"{K} pre-drawn batches through torch.autograd.Function (forward + backward kernels)",
            "start": "planted cores perturbed by 10% (local convergence)",
            "rule": f"AdaGrad eta {AUTOGRAD_ETA}, both forms",
            "target": {"rse_true": target, "floor_estimate": floor,
                       "reading": "10 x the noise floor (noise level x sqrt(parameters / entries)); AdaGrad's "
                                  "stochastic steps plateau near 5 x the floor in both forms"},
            "time_to_target": runs, "rse_every": every}


LAWS_ETA = 0.1   # AdaGrad eta of the four-law workload (every law)


def seeds_leg(args, I, R, kappa, m, dev, K, seeds=range(10)):
    """Steps/s of the headline step (the scaled method in ``args.prec``,
    same launch configuration) for every seed of ``seeds``: each seed plants
    its own ill-conditioned ring, initial cores and draws; exactly K steps
    replayed from HIP graphs after ``args.warmup`` eager steps.  Mean,
    sample standard deviation and median over the seeds."""
    import torch
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import TRSolver, cores_to_device
    N = 3
    rates, status = [], []
    for sd in seeds:
        _, X, _, init3 = build_problem(sd, I, R, kappa, dev)
        sol = TRSolver(cores_to_device(init3, torch.float32, dev), X, [I] * N, [R] * N, m, law="U", scaled=True,
                       prec=args.prec, rule=api.step_rule("fixed", alpha=args.alpha), seed=sd,
                       overlap=not args.no_overlap)
        if args.warmup > 0:
            sol.run(args.warmup)
        rates.append(1e3 / replay_timed(sol, K))
        status.append(int(sol.status.item()))
        del sol, X
    r = np.array(rates)
    return {"seeds": list(seeds), "prec": args.prec, "steps": K,
            "steps_per_s": [round(float(v), 2) for v in r],
            "mean": round(float(r.mean()), 2), "std": round(float(r.std(ddof=1)), 2) if r.size > 1 else 0.0,
            "median": round(float(np.median(r)), 2), "dev_status": status}


def laws_leg(dev, K, G=50, every=250, cap=5000):
    """The four-law workload: order 4, 64 per mode, ranks 5, planted Gaussian
    ring at RMS 1 + 40 dB noise, FP32 tensor and cores, m = 512 fibers,
    plain method (TR-BRSGD) with AdaGrad from random cores at the data's
    scale.  For each fiber law (uniform, Euclidean, leverage, optimal):
    (1) exactly K steps replayed from HIP graphs (steps/s; the E/L law
    refresh and the optimal law's per-step distribution are part of each
    step); (2) the time from the initial cores until the RSE against the
    noise-free tensor reaches 10x its noise floor sigma sqrt(P / J), P the
    number of core parameters, J = 64^4 entries (checks every ``every``
    steps, counted; the steps between checks replay one captured graph)."""
    import torch
    import tr_inputs as ti
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import TRSolver, cores_to_device
    N, I, R, m, db = 4, 64, 5, 512, 40.0
    desc = api.make_desc([I] * N, [R] * N, torch.float32)
    Xt = api.tr_reconstruct(desc, cores_to_device(ti.gaussian_cores(0, N, [I] * N, [R] * N), torch.float32, dev))
    Xt.div_(float(Xt.double().pow(2).mean().sqrt()))
    gen = torch.Generator(device=dev)
    gen.manual_seed(21)
    sigma = 10.0 ** (-db / 20.0)
    X = Xt + sigma * torch.randn(Xt.numel(), generator=gen, device=dev, dtype=torch.float32)
    # i.i.d. N(0, s^2) cores with E[X(i)^2] = s^(2N) R^N matched to mean(X^2)
    s = (float(X.double().pow(2).mean()) / float(R ** N)) ** (1.0 / (2 * N))
    init = ti.gaussian_cores(1, N, [I] * N, [R] * N, scale=s)
    floor = sigma * (N * I * R * R / float(I ** N)) ** 0.5
    target = 10.0 * floor
    xt2 = float(Xt.double().pow(2).sum())
    out = {"workload": "four-laws-n4-i64-r5-40db", "m": m, "method": "plain (TR-BRSGD)", "precision": "fp32",
           "rule": f"AdaGrad eta {LAWS_ETA}", "data": "planted Gaussian ring rescaled to RMS 1, 40 dB noise",
           "start": "i.i.d. Gaussian cores at the data's scale",
           "target": {"rse_true": target, "floor_estimate": floor,
                      "reading": "10 x the noise floor (noise level x sqrt(parameters / entries)); AdaGrad's "
                                 "stochastic steps plateau near 7 x the floor at this eta"},
           "rse_every": every, "laws": {}}
    rule = api.step_rule("adagrad", eta=LAWS_ETA)
    for law in ("U", "E", "L", "O"):
        sol = TRSolver(cores_to_device(init, torch.float32, dev), X, [I] * N, [R] * N, m, law=law, scaled=False,
                       prec="f32", rule=rule, seed=0)
        ms = replay_timed(sol, K, G)
        rate = {"steps_per_s": round(1e3 / ms, 2), "us_per_step": round(ms * 1e3, 3), "steps": K}
        del sol
        sol = TRSolver(cores_to_device(init, torch.float32, dev), X, [I] * N, [R] * N, m, law=law, scaled=False,
                       prec="f32", rule=rule, seed=0)
        graph = sol.capture(every)
        # undo the capture's warm-up step: the run starts from the initial cores at t = 0
        for c, c0 in zip(sol.cores, cores_to_device(init, torch.float32, dev)):
            c.copy_(c0)
        for a in sol.accum:
            a.zero_()
        sol.t_dev.zero_()
        sol.status.zero_()
        sol.rse(Xt, xt2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps, rse, hist = 0, float("nan"), []
        while steps < cap:
            graph.replay()
            steps += every
            rse = float(sol.rse(Xt, xt2))       # synchronises
            hist.append((steps, rse))
            if rse <= target:
                break
        wall = time.perf_counter() - t0
        status = int(sol.status.item())
        del graph, sol
        out["laws"][law] = {**rate, "time_to_target": {
            "reached": rse <= target, "seconds": round(wall, 4) if rse <= target else None, "steps": steps,
            "rse_at_stop": rse, "rse_trace": [[s_, float(f"{r_:.4e}")] for s_, r_ in hist[:: max(1, len(hist) // 8)]]},
            "dev_status": status}
        print(f"[bench] four-law workload, law {law}: {rate['us_per_step']} us/step, "
              f"rse {rse:.3e} after {steps} steps ({wall:.3f} s)", file=sys.stderr, flush=True)
    del X, Xt
    return out


def c1_time_to_target(dev, target=1e-4, every=10, cap=2000):
    """The plain FP64 workload (20^3, ranks 3, uniform fibers, m = 100,
    fixed step 0.2, noise-free planted ring): GPU time to RSE <= target
    (``every`` steps from one replayed graph, RSE checks counted)."""
    import torch
    import tr_inputs as ti
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import TRSolver, cores_to_device
    N, I, R, m = 3, 20, 3, 100
    desc = api.make_desc([I] * N, [R] * N, torch.float64)
    X = api.tr_reconstruct(desc, cores_to_device(ti.gaussian_cores(0, N, [I] * N, [R] * N), torch.float64, dev))
    sig = (float(X.pow(2).mean()) / float(R ** N)) ** (1.0 / (2 * N))
    init = ti.gaussian_cores(1, N, [I] * N, [R] * N, scale=sig)
    sol = TRSolver(cores_to_device(init, torch.float64, dev), X, [I] * N, [R] * N, m, prec="f64",
                   rule=api.step_rule("fixed", alpha=0.2), seed=0)
    snap = [c.clone() for c in sol.cores]
    g = sol.capture(every)
    for c, s_ in zip(sol.cores, snap):
        c.copy_(s_)
    sol.t_dev.zero_()
    torch.cuda.synchronize()
    steps, rse = 0, float("nan")
    t0 = time.perf_counter()
    while steps < cap:
        g.replay()
        steps += every
        rse = float(sol.rse())
        if rse <= target:
            break
    gpu_s = time.perf_counter() - t0
    return {"workload": "plain-fp64-n3-i20-r3", "target": target, "rse_every": every,
            "seconds": round(gpu_s, 5) if rse <= target else None, "steps": steps, "rse_at_stop": rse}


def c1_cpu_oracle(target=1e-4, every=10, cap=2000):
    """The oracle on the host: the same plain FP64 run to the same target."""
    import tr_inputs as ti
    from oracle import brsgd, tr
    N, I, R, m = 3, 20, 3, 100
    X = tr.full_tensor(ti.gaussian_cores(0, N, [I] * N, [R] * N))
    init = ti.gaussian_cores(1, N, [I] * N, [R] * N, scale=brsgd.init_scale(X, [R] * N))
    st = brsgd.State(init)
    t0 = time.perf_counter()
    hist = brsgd.run(st, X, brsgd.Config(m=m, alpha=0.2, seed=0), cap, rse_every=every, tol=target)
    return {"workload": "plain-fp64-n3-i20-r3", "target": target, "rse_every": every,
            "seconds": round(time.perf_counter() - t0, 4) if hist and hist[-1][1] <= target else None,
            "steps": hist[-1][0] if hist else None, "rse_at_stop": hist[-1][1] if hist else None}


def c3_local_cpu_oracle(seed, I, R, kappa, m, target=1e-4, every=50, wall_cap=40.0):
    """The oracle on the host, one BLAS thread (its faster setting at this
    size): the scaled method (alpha 1) on the ill-conditioned ring from the
    planted cores perturbed by 10% (the GPU leg's recipe), RSE checked every
    ``every`` steps (counted), until the target or ``wall_cap`` seconds."""
    import tr_inputs as ti
    from oracle import brsgd, tr
    from threadpoolctl import threadpool_limits
    N = 3
    true3 = ti.illcond_cores(seed, N, I, R, kappa)
    X = tr.full_tensor(true3)
    c = float(np.mean(X * X)) ** (-1.0 / (2 * N))
    true3 = [t * c for t in true3]
    X = X * c ** N
    rng = np.random.default_rng(12)
    init = [t + 0.1 * np.sqrt(np.mean(t * t)) * rng.standard_normal(t.shape) for t in true3]
    st = brsgd.State(init)
    cfg = brsgd.Config(m=m, variant="scaled", alpha=1.0, seed=seed)
    rse, steps = float("nan"), 0
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < wall_cap:
            for _ in range(every):
                brsgd.step(st, X, cfg)
            steps += every
            rse = tr.rse(st.cores, X)
            if rse <= target:
                break
        wall = time.perf_counter() - t0
    return {"workload": "scaled-illcond-n3-i400-r10", "start": "planted cores + 10% Gaussian perturbation",
            "target": target, "rse_every": every, "threads": 1, "wall_cap_s": wall_cap,
            "reached": rse <= target, "seconds": round(wall, 3) if rse <= target else None, "steps": steps,
            "rse_at_stop": rse}


def methods_leg(args, init3, X, I, R, m, dev, budget_s=0.25):
    """The paper's comparison (second synthetic experiment's table,
    qualitatively) on the benchmark problem: each method from the same
    initial cores for about ``budget_s`` of GPU time, RSE at the end."""
    import torch
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import TRSolver, TRSweeper, cores_to_device
    N = 3
    out = {}

    def rse_of(cores):
        return float(api.tr_relerr(api.make_desc([I] * N, [R] * N, torch.float32), cores, X))

    step_methods = {
        "TR-BRSGD-U (AdaGrad eta 1e-2)": dict(scaled=False, law="U", rule=api.step_rule("adagrad", eta=1e-2)),
        "TR-ScaledBRSGD-U (alpha 1)": dict(scaled=True, law="U", rule=api.step_rule("fixed", alpha=1.0)),
        "TR-ScaledBRSGD-L (alpha 1)": dict(scaled=True, law="L", rule=api.step_rule("fixed", alpha=1.0)),
    }
    for name, kw in step_methods.items():
        sol = TRSolver(cores_to_device(init3, torch.float32, dev), X, [I] * N, [R] * N, m, prec="f32", seed=args.seed,
                       **kw)
        sol.run(5)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        while time.perf_counter() - t0 < budget_s:
            sol.run(50)
            torch.cuda.synchronize()
            steps += 50
        wall = time.perf_counter() - t0
        out[name] = {"steps": steps + 5, "seconds": round(wall, 4), "rse": rse_of(sol.cores)}
        del sol
    sweep_methods = {
        "TR-GD (alpha 2e-5)": dict(method="gd", alpha=2e-5),
        "TR-ScaledGD (alpha 0.5)": dict(method="scaled-gd", alpha=0.5),
        "TR-ALS": dict(method="als"),
        "TR-ALS-Sampled-L (m 4096)": dict(method="als-sampled", m=m, law="L"),
    }
    for name, kw in sweep_methods.items():
        sw = TRSweeper(cores_to_device(init3, torch.float32, dev), X, [I] * N, [R] * N, prec="f32", seed=args.seed,
                       **kw)
        t0 = time.perf_counter()
        sweeps = 0
        while time.perf_counter() - t0 < budget_s:
            sw.sweep(1)
            torch.cuda.synchronize()
            sweeps += 1
        wall = time.perf_counter() - t0
        out[name] = {"sweeps": sweeps, "block_updates": sweeps * N, "seconds": round(wall, 4),
                     "rse": rse_of(sw.cores)}
        del sw
    torch.cuda.empty_cache()
    return {"workload": "scaled-illcond-n3-i400-r10", "budget_s_each": budget_s, "precision": "fp32",
            "methods": out}


def host_info():
    """CPU model, logical CPUs usable by this process, and memory of the
    host, read from the kernel's own files."""
    model = None
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    mem_gb = None
    try:
        for ln in open("/proc/meminfo"):
            if ln.startswith("MemTotal"):
                mem_gb = round(int(ln.split()[1]) / 2 ** 20, 1)
                break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": usable, "logical_cpus": os.cpu_count(), "mem_gb": mem_gb}


def cpu_baseline(seconds, seed, I, R, kappa, m, alpha, threads=None):
    """The oracle as it stands, on the same workload, for a bounded number
    of steps (about ``seconds`` of CPU work after one warm-up step), with
    the BLAS thread pools limited to ``threads`` (None: as configured);
    returns (steps/s, steps, threads actually used)."""
    import tr_inputs as ti
    from oracle import brsgd, tr
    from threadpoolctl import threadpool_info, threadpool_limits
    N = 3
    true3 = ti.illcond_cores(seed, N, I, R, kappa)
    X = tr.full_tensor(true3)
    c = float(np.mean(X * X)) ** (-1.0 / (2 * N))
    X = X * c ** N
    sig = (1.0 / R ** N) ** (1.0 / (2 * N))
    st = brsgd.State(ti.gaussian_cores(seed + 1, N, I, R, scale=sig))
    cfg = brsgd.Config(m=m, variant="scaled", alpha=alpha, seed=seed)
    with threadpool_limits(limits=threads):
        used = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
        brsgd.step(st, X, cfg)               # warm-up
        t0 = time.perf_counter()
        k = 0
        while time.perf_counter() - t0 < seconds:
            brsgd.step(st, X, cfg)
            k += 1
        dt = time.perf_counter() - t0
    return k / dt, k, used


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_scaled-illcond-n3-i400-r10.txt")
KERNEL_SOURCE = {"k_sweep": "sweep.hip", "k_grad_mfma_f32": "grad_mfma.hip", "k_grad_mfma_f32w": "grad_mfma.hip",
                 "k_grad_mixed": "grad_mixed.hip", "k_grad_mixed_w": "grad_mixed.hip"}


def measured_traffic(kernel):
    """Counter-measured HBM bytes per launch of ``kernel`` from the committed
    profile summary, or None if the kernel's source changed since."""
    import hashlib
    try:
        lines = open(TRAFFIC_FILE).read().splitlines()
    except OSError:
        return None
    src = os.path.join(ROOT, "paper_2303_16492_amd", "csrc", KERNEL_SOURCE[kernel])
    sha = hashlib.sha1(open(src, "rb").read()).hexdigest()
    for ln in lines:
        if ln.startswith("#") or "|" not in ln:
            continue
        name, _, _, _, nbytes, ksha = [x.strip() for x in ln.split("|")]
        if re.search(rf"\b{kernel}<", name) and ksha == sha:
            return int(nbytes)
    return None


def timed_run(args, prec, init3, X, I, R, m, dev, K, warmup, G=50, E=200):
    """The scaled method in precision ``prec`` from the initial cores:
    (1) E eager steps whose gradient and inverse dispatches record HIP
    start/stop events themselves (per-launch kernel execution times, as a
    kernel trace reports them); (2) exactly K timed steps replayed from HIP graphs
    (``graph_schedule``: graphs of min(G, K) steps plus a remainder graph),
    whose rate is the result."""
    import torch
    from paper_2303_16492_amd import _lib as L
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import TRSolver, cores_to_device
    N = 3
    cores = cores_to_device(init3, torch.float32, dev)
    solver = TRSolver(cores, X, [I] * N, [R] * N, m, law="U", scaled=True, prec=prec,
                      rule=api.step_rule("fixed", alpha=args.alpha), seed=args.seed,
                      overlap=not args.no_overlap)
    if warmup > 0:
        solver.run(warmup)
    torch.cuda.synchronize()
    hip, evs = hip_events(4 * E + 2)
    arr = lambda j: (C.c_void_p * E)(*[e.value for e in evs[2 + j * E:2 + (j + 1) * E]])
    gb, ge, ib, ie = arr(0), arr(1), arr(2), arr(3)
    opts = L.tr_run_opts()
    if solver.opts is not None:
        so = solver.opts
        opts.aux, opts.ev_fork, opts.ev_gram, opts.ev_join = so.aux, so.ev_fork, so.ev_gram, so.ev_join
    P = lambda a: C.cast(a, C.POINTER(C.c_void_p))
    opts.ev_begin, opts.ev_end, opts.ev_inv_begin, opts.ev_inv_end = P(gb), P(ge), P(ib), P(ie)
    stream = torch.cuda.current_stream()
    assert hip.hipEventRecord(evs[0], C.c_void_p(stream.cuda_stream)) == 0
    rc = api.lib().tr_run_ex(C.byref(solver.problem), C.byref(solver.config), C.c_void_p(solver.t_dev.data_ptr()),
                             E, None, C.c_void_p(solver.status.data_ptr()), C.c_void_p(solver.ws.data_ptr()),
                             solver.ws.numel(), C.c_void_p(stream.cuda_stream), C.byref(opts))
    assert rc == 0, rc
    assert hip.hipEventRecord(evs[1], C.c_void_p(stream.cuda_stream)) == 0
    torch.cuda.synchronize()
    eager_ms = elapsed_ms(hip, evs[0], evs[1]) / E
    grad_us = 1e3 * float(np.mean([elapsed_ms(hip, gb[i], ge[i]) for i in range(E)]))
    inv_us = (1e3 * float(np.mean([elapsed_ms(hip, ib[i], ie[i]) for i in range(E)]))
              if solver.opts is not None else None)
    for e in evs:
        hip.hipEventDestroy(e)
    ms = replay_timed(solver, K, G)
    rse = float(solver.rse())
    status = int(solver.status.item())
    del solver
    return dict(ms_per_step=ms, eager_ms_per_step=eager_ms, grad_us=grad_us, inv_us=inv_us, rse_after=rse,
                dev_status=status, graphs=graph_schedule(K, G))


def plain_rate(args, prec, init3, X, I, R, m, dev, K, G=50):
    """Steps/s of the plain method (TR-BRSGD, AdaGrad step) in precision
    ``prec`` on the same workload: draws, subchain, gradient, update; here
    the gradient kernel is on the critical path of every step.  Exactly K
    steps replayed from HIP graphs (``graph_schedule``)."""
    import torch
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import TRSolver, cores_to_device
    N = 3
    solver = TRSolver(cores_to_device(init3, torch.float32, dev), X, [I] * N, [R] * N, m, law="U", scaled=False,
                      prec=prec, rule=api.step_rule("adagrad", eta=1e-3), seed=args.seed)
    if args.warmup > 0:
        solver.run(args.warmup)
    ms = replay_timed(solver, K, G)
    status = int(solver.status.item())
    del solver
    return {"steps_per_s": round(1e3 / ms, 2), "us_per_step": round(ms * 1e3, 3), "steps": K, "dev_status": status}


def law_rate(args, law, init3, X, I, R, m, dev, K, G=50):
    """Steps/s of the scaled FP32 step with fibers drawn under ``law`` (E or
    L), including the refresh of the updated core's law after every step;
    exactly K steps replayed from HIP graphs (``graph_schedule``)."""
    import torch
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import TRSolver, cores_to_device
    N = 3
    solver = TRSolver(cores_to_device(init3, torch.float32, dev), X, [I] * N, [R] * N, m, law=law, scaled=True,
                      prec="f32", rule=api.step_rule("fixed", alpha=args.alpha), seed=args.seed,
                      overlap=not args.no_overlap)
    if args.warmup > 0:
        solver.run(args.warmup)
    ms = replay_timed(solver, K, G)
    status = int(solver.status.item())
    del solver
    return {"steps_per_s": round(1e3 / ms, 2), "us_per_step": round(ms * 1e3, 3), "steps": K, "dev_status": status}


# An RSE check runs after a replay only when the step's own loss estimate,
# as a relative error sqrt(2 loss / ||X||^2) (unbiased for the pre-update
# cores' squared error), is within this factor of the target.
RSE_TRIGGER = 30.0


def time_to_target(args, prec, init3, X, I, R, m, dev, target=1e-4, every=100, cap=None, scaled=True, alpha=None):
    """Wall time from the initial cores until an RSE check reaches
    ``target`` (checks after every ``every`` steps count toward the time
    when the last step's loss estimate triggers them; the steps between
    checks replay one captured graph), capped at ``cap`` (default
    args.ttt_steps) steps; the scaled method (default) or the plain one,
    fixed step ``alpha`` (default args.alpha)."""
    import torch
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import TRSolver, cores_to_device
    N = 3
    solver = TRSolver(cores_to_device(init3, torch.float32, dev), X, [I] * N, [R] * N, m, law="U", scaled=scaled,
                      prec=prec, rule=api.step_rule("fixed", alpha=args.alpha if alpha is None else alpha),
                      seed=args.seed, overlap=not args.no_overlap)
    # The ``every`` steps between checks run as one captured HIP graph, as in
    # the throughput measurement; the capture's warm-up step is undone (cores,
    # accumulators, step counter restored) before the timer starts.
    snap = [c.clone() for c in solver.cores]
    acc_snap = [a.clone() if a is not None else None for a in solver.accum]
    losses = torch.zeros(every, dtype=torch.float64, device=dev)
    graph = solver.capture(every, losses)
    xnorm2 = float(X.double().pow(2).sum())
    for c, s_ in zip(solver.cores, snap):
        c.copy_(s_)
    for a, s_ in zip(solver.accum, acc_snap):
        if a is not None:
            a.copy_(s_)
    solver.t_dev.zero_()
    solver.status.zero_()
    solver.rse()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    cap = args.ttt_steps if cap is None else cap
    steps, rse, hist, skipped = 0, float("nan"), [], 0
    while steps < cap:
        graph.replay()
        steps += every
        est = (2.0 * max(float(losses[-1]), 0.0) / xnorm2) ** 0.5   # synchronises
        if est > RSE_TRIGGER * target and steps < cap:
            skipped += 1
            continue
        rse = float(solver.rse())          # synchronises
        hist.append((steps, rse))
        if rse <= target:
            break
    wall = time.perf_counter() - t0
    del graph, solver
    return {"prec": prec, "target": target, "reached": rse <= target,
            "seconds": round(wall, 4) if rse <= target else None, "steps": steps,
            "rse_at_stop": rse, "wall_s_at_stop": round(wall, 4), "rse_every": every,
            "rse_trigger": f"loss estimate within {RSE_TRIGGER:g}x of the target", "rse_checks": len(hist),
            "rse_checks_skipped": skipped,
            "rse_trace": [[s_, float(f"{r_:.4e}")] for s_, r_ in hist[:: max(1, len(hist) // 10)]]}


def relerr_timing(desc, cores, X, reps=20):
    """Mean duration of one RSE evaluation (pack + matrix-core
    reconstruction against X + fixed-order finish) over ``reps`` calls on
    the current stream, bracketed by HIP events."""
    import torch
    from paper_2303_16492_amd import _lib as L
    from paper_2303_16492_amd import api
    ws = api.workspace(L.lib().tr_relerr_workspace_size(C.byref(desc)), X.device)
    out = torch.zeros(1, dtype=torch.float64, device=X.device)
    api.tr_relerr(desc, cores, X, rse=out, ws=ws)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        api.tr_relerr(desc, cores, X, rse=out, ws=ws)
    b.record()
    torch.cuda.synchronize()
    return a.elapsed_time(b) / reps * 1e3, float(out.item())


def step_roofline(main, plain, batched, laws4, I, R, m):
    """Whole-step fractions: the algorithmic lower bound of one step (what
    the method must compute or move, at the chip's peak) over the measured
    step time, for the workloads whose bound is not latency."""
    out = {}
    RR = R * R
    # 400^3, ranks 10, m = 4096: prediction and gradient contractions
    # 2 I m RR FMA plus the sampled Gram m RR^2 FMA on FP32 matrix cores
    fma = 2.0 * I * m * RR + m * RR * RR
    b_c3 = 2.0 * fma / (PEAK["f32"][0] * 1e12) * 1e6
    out["scaled_fp32"] = {"bound_us": round(b_c3, 3), "measured_us": round(main["ms_per_step"] * 1e3, 3),
                          "frac": round(b_c3 / (main["ms_per_step"] * 1e3), 4),
                          "basis": f"{fma / 1e6:.1f} M FMA at the FP32 matrix-core peak (the FP64 inverse's "
                                   f"RR^3/3 FMA and the HBM traffic, 0.9 us at 8 TB/s, below it)"}
    if plain and "f32" in plain:
        out["plain_fp32"] = {"bound_us": round(b_c3, 3), "measured_us": plain["f32"]["us_per_step"],
                             "frac": round(b_c3 / plain["f32"]["us_per_step"], 4), "basis": "as scaled_fp32"}
    if batched:
        # the 64-problem draw: fibers and cores of every problem's step, about 9.4 MB, at 8 TB/s
        b_c5 = 9.4e6 / (HBM_PEAK_GBS * 1e9) * 1e6
        ms = batched["ms_per_batch_step"] * 1e3
        out["batched_64"] = {"bound_us": round(b_c5, 3), "measured_us": round(ms, 3), "frac": round(b_c5 / ms, 4),
                             "basis": "about 9.4 MB of fibers and cores per step of all 64 problems at 8 TB/s"}
    if laws4 and "O" in laws4["laws"]:
        # law O: the residual of every column, J I RR = 64^4 25 FP64 FMA at the FP64 peak (10.7 us), above
        # the 64 MiB tensor read once at 8 TB/s (8.4 us)
        b_o = 2.0 * 64 ** 4 * 25 / (PEAK["f64"][0] * 1e12) * 1e6
        us = laws4["laws"]["O"]["us_per_step"]
        out["optimal_law_order4"] = {"bound_us": round(b_o, 3), "measured_us": us, "frac": round(b_o / us, 4),
                                     "basis": "419 M FP64 FMA of the law's residuals at the FP64 peak (the 64 MiB "
                                              "tensor read once: 8.4 us at 8 TB/s)"}
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "--gpus must be 1: the path runs on one GPU "
                          "(sharding over several GPUs is not implemented)"}))
        sys.exit(2)
    import torch

    dev = "cuda:0"
    if args.copy_probe > 0:
        # known-size traffic for scaling the FETCH_SIZE / WRITE_SIZE counters
        nbytes = args.copy_probe << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(20):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_probe_bytes": nbytes, "launches": 20}), flush=True)
        return
    I, R, kappa, m = 400, 10, 1e4, 4096
    N = 3
    desc, X, true3, init3 = build_problem(args.seed, I, R, kappa, dev)
    print(f"[bench] workload ready: {I}^3 rank {R}, m={m}", file=sys.stderr, flush=True)
    K = args.steps
    main = timed_run(args, args.prec, init3, X, I, R, m, dev, K, args.warmup)
    print(f"[bench] {args.prec}: {main['ms_per_step'] * 1e3:.2f} us/step, gradient {main['grad_us']:.2f} us, "
          f"inverse {main['inv_us']} us, rse {main['rse_after']:.3e}", file=sys.stderr, flush=True)
    other = "bf16" if args.prec == "f32" else "f32"
    alt = timed_run(args, other, init3, X, I, R, m, dev, K, args.warmup)
    print(f"[bench] {other}: {alt['ms_per_step'] * 1e3:.2f} us/step", file=sys.stderr, flush=True)
    plain = {pr: plain_rate(args, pr, init3, X, I, R, m, dev, K) for pr in ("f32", "bf16")}
    laws = {lw: law_rate(args, lw, init3, X, I, R, m, dev, K) for lw in ("E", "L")}
    print(f"[bench] scaled step under the Euclidean and leverage laws: {laws}", file=sys.stderr, flush=True)
    print(f"[bench] plain method: {plain}", file=sys.stderr, flush=True)
    ttt = []
    if args.ttt_steps > 0:
        for pr in ("f32", "bf16"):
            ttt.append(time_to_target(args, pr, init3, X, I, R, m, dev))
            print(f"[bench] time-to-target {pr}: {ttt[-1]['reached']} after {ttt[-1]['steps']} steps, "
                  f"rse {ttt[-1]['rse_at_stop']:.3e}", file=sys.stderr, flush=True)

    # The same workload from the planted cores perturbed by 10% (seeded):
    # local convergence, where the 1e-4 target is within reach of every form
    # (from random cores every method stalls near RSE 0.16 on this ring).
    local = None
    if args.ttt_steps > 0:
        rng = np.random.default_rng(12)
        linit = [t + 0.1 * np.sqrt(np.mean(t * t)) * rng.standard_normal(t.shape) for t in true3]
        local = {"workload": "scaled-illcond-n3-i400-r10", "start": "planted cores + 10% Gaussian perturbation",
                 "m": m, "law": "uniform", "alpha": 1.0, "scaled": [], "plain": []}
        for pr in ("f32", "bf16"):
            local["scaled"].append(time_to_target(args, pr, linit, X, I, R, m, dev, every=10, cap=2000))
            local["plain"].append(time_to_target(args, pr, linit, X, I, R, m, dev, every=250, cap=12000,
                                                 scaled=False, alpha=1.0))
            print(f"[bench] local time-to-target {pr}: scaled {local['scaled'][-1]['steps']} steps "
                  f"{local['scaled'][-1]['seconds']} s, plain {local['plain'][-1]['steps']} steps "
                  f"{local['plain'][-1]['seconds']} s", file=sys.stderr, flush=True)
        sc, pl = local["scaled"], local["plain"]
        local["mixed_speedup_scaled"] = (round(sc[0]["seconds"] / sc[1]["seconds"], 4)
                                         if sc[0]["reached"] and sc[1]["reached"] else None)
        local["mixed_speedup_plain"] = (round(pl[0]["seconds"] / pl[1]["seconds"], 4)
                                        if pl[0]["reached"] and pl[1]["reached"] else None)

    methods = None
    if args.methods_budget > 0:
        methods = methods_leg(args, init3, X, I, R, m, dev, budget_s=args.methods_budget)
        print(f"[bench] methods: {json.dumps(methods['methods'])}", file=sys.stderr, flush=True)

    # a9 on its own: one RSE evaluation at 400^3 (X read once, 2 I^3 R^2 FLOP)
    from paper_2303_16492_amd.driver import cores_to_device
    rcores = cores_to_device(init3, torch.float32, dev)
    rse_us, _ = relerr_timing(desc, rcores, X)
    rflops = 2.0 * I ** 3 * R * R
    rbytes = 4.0 * I ** 3
    # executed on the matrix cores: three FP16 products per K step, K padded to a multiple of 16
    xflops = 3 * 2.0 * I ** 3 * (16 * ((R * R + 15) // 16))
    relerr = {"kernel": "k_recon_mfma (+ k_recon_pack_h3, k_recon_finish)", "us_per_rse": round(rse_us, 2),
              "precision": "fp16 hi/lo split, three products per K step, fp32 accumulation, fp64 sums",
              "flops": rflops, "bytes": rbytes,
              "alg_tflops": round(rflops / (rse_us * 1e-6) / 1e12, 2),
              "mfma_flops_executed": xflops,
              "mfma_tflops": round(xflops / (rse_us * 1e-6) / 1e12, 2),
              "mfma_frac": round(xflops / (rse_us * 1e-6) / 1e12 / PEAK["f16"][0], 4),
              "hbm_gbs": round(rbytes / (rse_us * 1e-6) / 1e9, 1),
              "hbm_frac": round(rbytes / (rse_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    del rcores
    print(f"[bench] relerr: {rse_us:.1f} us per RSE", file=sys.stderr, flush=True)
    planted, planted_plain = [], []
    if args.ttt_steps > 0:
        # The same method on a planted ring with Gaussian cores at the same
        # size, where the 1e-4 target is within reach of both forms.
        pdesc, PX, _, pinit = build_problem(args.seed, I, R, kappa, dev, kind="gaussian")
        for pr in ("f32", "bf16"):
            planted.append(time_to_target(args, pr, pinit, PX, I, R, m, dev, every=10, cap=1000))
            print(f"[bench] planted time-to-target {pr}: {planted[-1]['reached']} after {planted[-1]['steps']} "
                  f"steps, {planted[-1]['wall_s_at_stop']} s, rse {planted[-1]['rse_at_stop']:.3e}",
                  file=sys.stderr, flush=True)
        # The plain method (the gradient on every step's critical path), fixed
        # step 1.0, RSE every 250 steps.
        for pr in ("f32", "bf16"):
            planted_plain.append(time_to_target(args, pr, pinit, PX, I, R, m, dev, every=250, cap=20000,
                                                scaled=False, alpha=1.0))
            print(f"[bench] planted plain-method time-to-target {pr}: {planted_plain[-1]['reached']} after "
                  f"{planted_plain[-1]['steps']} steps, {planted_plain[-1]['wall_s_at_stop']} s, "
                  f"rse {planted_plain[-1]['rse_at_stop']:.3e}", file=sys.stderr, flush=True)
        del PX

    RR = R * R
    flops = 4.0 * I * m * RR                       # prediction + gradient contractions
    bytes_alg = I * m * 4 + m * RR * 4 + I * RR * 4  # fibers + sampled rows + core
    peak, unit = PEAK[args.prec]
    g_ach = flops / (main["grad_us"] * 1e-6) / 1e12
    # FP32: the 16-byte-operand form (R_n R_{n+1} = 100, one 128-sample chunk per sample group)
    gkern = "k_grad_mfma_f32w" if args.prec == "f32" else "k_grad_mixed_w"
    grad_roof = {"bound": "mfma", "achieved": round(g_ach, 3), "peak": peak, "unit": unit,
                 "frac": round(g_ach / peak, 5), "traffic": measured_traffic(gkern),
                 "kernel": gkern,
                 "kernel_avg_us": round(main["grad_us"], 3), "flops_per_launch": flops,
                 "alg_bytes_per_launch": bytes_alg,
                 "alg_hbm_gbs": round(bytes_alg / (main["grad_us"] * 1e-6) / 1e9, 1)}
    inv_roof = None
    if main["inv_us"] is not None:
        # algorithmic work of the factorisation of the RR x RR system: RR^3 / 3 FMA (Cholesky); the
        # sweep executes 2 RR^3 FLOP, forming the explicit inverse that the update then applies
        inv_flops = 2.0 * RR ** 3 / 3.0
        i_ach = inv_flops / (main["inv_us"] * 1e-6) / 1e12
        inv_roof = {"bound": "mfma", "achieved": round(i_ach, 6), "peak": PEAK["f64"][0], "unit": "TFLOP/s",
                    "frac": round(i_ach / PEAK["f64"][0], 7), "traffic": measured_traffic("k_sweep"),
                    "kernel": "k_sweep", "kernel_avg_us": round(main["inv_us"], 3),
                    "flops_per_launch": round(inv_flops), "flops_executed_per_launch": 2.0 * RR ** 3,
                    "note": "one workgroup (the inverse is a chain of 100 dependent pivots in 13 blocks); "
                            "achieved counts the factorisation's RR^3/3 FMA; frac is against the whole chip's "
                            "FP64 peak"}
    # the dominant kernel: the longer of the two per step
    roof = inv_roof if inv_roof is not None and main["inv_us"] > main["grad_us"] else grad_roof

    batched = None
    if args.batch_steps > 0:
        print("[bench] building the 64-problem batch ...", file=sys.stderr, flush=True)
        del X
        torch.cuda.empty_cache()
        B, insts, truths = build_batch(args.seed, dev)
        torch.cuda.synchronize()
        tune = B.tune(steps=3, reps=2)
        print(f"[bench] batch tuned: {tune} -> chunk {B.chunk}, waves {B.waves}, splits {B.splits}",
              file=sys.stderr, flush=True)
        # timed: args.batch_steps steps of all problems replayed from one captured graph
        saved = B._state()
        B.run(1)                                  # warm-up (and the split workspace) before the capture
        gb = torch.cuda.CUDAGraph()
        sb = torch.cuda.Stream()
        sb.wait_stream(torch.cuda.current_stream())
        torch.cuda.synchronize()
        with torch.cuda.graph(gb, stream=sb):
            B.run(args.batch_steps)
        gb.replay()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        gb.replay()
        b.record()
        torch.cuda.synchronize()
        ms = a.elapsed_time(b) / args.batch_steps
        del gb
        B._restore(saved)
        torch.cuda.synchronize()
        tiles = {"chunk": B.chunk, "waves": B.waves, "splits": B.splits}
        print(f"[bench] batch: {ms * 1e3:.1f} us per step of all 64 problems (graph replay)", file=sys.stderr,
              flush=True)
        b_sec, b_steps, b_per, b_wall = batch_time_to_target(B, truths)
        print(f"[bench] batch time to RSE {BATCH_TARGET:g}: {b_sec} s ({b_steps} steps)", file=sys.stderr, flush=True)
        dev_status = int(B.status.max())
        del B, truths
        torch.cuda.empty_cache()
        s_sec, s_per, s_rate = single_time_to_target(insts, dev)
        print(f"[bench] same problems one at a time in FP32: {s_sec} s", file=sys.stderr, flush=True)
        batched = {"workload": "batched-64-planted-fp16", "problems": len(insts), "m": 1024,
                   "steps": args.batch_steps, "ms_per_batch_step": round(ms, 5),
                   "problem_steps_per_s": round(len(insts) * 1e3 / ms, 1),
                   "timing": "steps of all problems replayed from one captured graph",
                   "tiles": tiles,
                   "tuner_ms_per_step": {f"{c}x{w}x{sp}": round(v, 5) for (c, w, sp), v in tune.items()},
                   "precision": "fp16 tensors and matrix cores, fp32 accumulation, fp64 loss",
                   "data": "each planted tensor rescaled to RMS 1, 40 dB noise",
                   "rule": f"AdaGrad eta {BATCH_ETA}",
                   "time_to_target": {"target": f"RSE against the noise-free tensor <= {BATCH_TARGET:g} for every "
                                                f"problem (checks every 250 steps, counted)",
                                      "batched_seconds": b_sec, "batched_steps": b_steps,
                                      "single_fp32_seconds": s_sec,
                                      "single_fp32_steps_per_problem": s_per,
                                      "batched_steps_per_problem": b_per,
                                      "single_fp32_steps_per_s_avg": round(s_rate, 1),
                                      "speedup": (round(s_sec / b_sec, 3) if b_sec else None)},
                   "dev_status_or": dev_status}

    autograd = None
    if args.autograd_steps > 0:
        autograd = autograd_leg(dev, steps_cap=args.autograd_steps)
        print(f"[bench] autograd: {json.dumps(autograd)}", file=sys.stderr, flush=True)
    seeds = None
    if args.seeds > 0:
        seeds = seeds_leg(args, I, R, kappa, m, dev, max(K, 200), seeds=range(args.seeds))
        print(f"[bench] seeds 0-{args.seeds - 1}: {seeds['mean']} +- {seeds['std']} steps/s", file=sys.stderr,
              flush=True)
    laws4 = None
    if args.ttt_steps > 0:
        laws4 = laws_leg(dev, K)
        torch.cuda.empty_cache()
    c1 = None
    if args.ttt_steps > 0:
        c1 = c1_time_to_target(dev)
        print(f"[bench] plain fp64 time to target: {json.dumps(c1)}", file=sys.stderr, flush=True)

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu oracle baseline ...", file=sys.stderr, flush=True)
        host = host_info()
        half = args.cpu_seconds / 2.0
        v_all, k_all, th_all = cpu_baseline(half, args.seed, I, R, kappa, m, args.alpha, threads=host["nproc"])
        v_one, k_one, th_one = cpu_baseline(half, args.seed, I, R, kappa, m, args.alpha, threads=1)
        legs = {"threads_all": {"value": round(v_all, 4), "unit": "steps/s", "cores": th_all,
                                "sample": f"{k_all} oracle steps, {th_all} BLAS threads, about {half:g} s"},
                "threads_1": {"value": round(v_one, 4), "unit": "steps/s", "cores": th_one,
                              "sample": f"{k_one} oracle steps, 1 BLAS thread, about {half:g} s"}}
        best = max(legs.values(), key=lambda x: x["value"])
        c1_cpu = c1_cpu_oracle() if args.ttt_steps > 0 else None
        c3_cpu = c3_local_cpu_oracle(args.seed, I, R, kappa, m) if args.ttt_steps > 0 else None
        cpu = {"value": best["value"], "unit": "steps/s", "cores": best["cores"], "kind": "oracle",
               "time_to_target_plain_fp64": c1_cpu, "time_to_target_local": c3_cpu,
               "sample": f"oracle steps (FP64 numpy/scipy) of the same 400^3 scaled workload after 1 warm-up step; "
                         f"value is the faster of the two thread settings ({best['sample']})",
               **legs, "host": host}

    out = {
        "metric": "sampled-gradient steps/s + time to rel.err 1e-4: mixed vs plain FP32, 1 GPU",
        "value": round(1e3 / main["ms_per_step"], 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(main["ms_per_step"], 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "scaled-illcond-n3-i400-r10", "N": N, "I": I, "R": R, "kappa": kappa,
                   "m": m, "H_n": "F_n", "law": "uniform", "alpha": args.alpha, "prec": args.prec,
                   "overlap": not args.no_overlap},
        "roofline": roof,
        "roofline_gradient": grad_roof,
        "roofline_inverse": inv_roof,
        "cpu_baseline": cpu,
        "forms": {args.prec: {"steps_per_s": round(1e3 / main["ms_per_step"], 2), "rse_after": main["rse_after"],
                              "gradient_us": round(main["grad_us"], 3),
                              "inverse_us": None if main["inv_us"] is None else round(main["inv_us"], 3)},
                  other: {"steps_per_s": round(1e3 / alt["ms_per_step"], 2), "rse_after": alt["rse_after"],
                          "gradient_us": round(alt["grad_us"], 3),
                          "inverse_us": None if alt["inv_us"] is None else round(alt["inv_us"], 3)}},
        "timing": "value: K steps replayed from a captured HIP graph of 50 steps (the Gram/inverse branch forks "
                  "and joins as graph edges); kernel durations: HIP start/stop events recorded by every dispatch of "
                  "the inverse and gradient kernels themselves (hipExtLaunchKernelGGL) over 200 eager steps of the "
                  "same run",
        "eager_steps_per_s": round(1e3 / main["eager_ms_per_step"], 2),
        "forms_plain_method": plain,
        "forms_laws": laws,
        "four_laws": laws4,
        "seeds": seeds,
        "time_to_target": ttt,
        "time_to_target_local": local,
        "time_to_target_planted": {"workload": "planted-gaussian-n3-i400-r10", "method": "scaled", "m": m,
                                   "law": "uniform", "alpha": args.alpha, "runs": planted},
        "time_to_target_planted_plain": {"workload": "planted-gaussian-n3-i400-r10", "method": "plain", "m": m,
                                         "law": "uniform", "alpha": 1.0, "runs": planted_plain,
                                         "mixed_speedup": (round(planted_plain[0]["seconds"] / planted_plain[1]["seconds"], 4)
                                                           if len(planted_plain) == 2 and planted_plain[0]["reached"]
                                                           and planted_plain[1]["reached"] else None)},
        "relerr": relerr,
        "step_roofline": step_roofline(main, plain, batched, laws4, I, R, m),
        "batched": batched,
        "autograd": autograd,
        "time_to_target_plain_fp64": c1,
        "methods": methods,
        "rse_after": main["rse_after"],
        "dev_status": main["dev_status"],
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
