"""Benchmark of the TR-ScaledBRSGD hot path on one MI355X.

Workload (default): the ill-conditioned planted ring of the second synthetic
experiment at 400 x 400 x 400 (64M FP32 entries), ranks 10, each core's
mode-2 unfolding with singular values geometric from 1 to 1e-4, mini-batch
|F_n| = 4096 with H_n = F_n, uniform fibers, FP64 Cholesky of the 100 x 100
Gram.  One step = mode pick, draws, sampled subchain, fiber gather,
gradient, Gram, Cholesky solve and update (every row of the hot path).

Prints one JSON line: steps/s (whole job), the dominant kernel's roofline
(fused fiber-gather/gradient contraction, timed with HIP events around each
launch inside the timed region), the CPU oracle timed on a bounded sample,
and the RSE reached.
"""
from __future__ import annotations

import argparse
import ctypes as C
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK = {"f32": (157.3, "TFLOP/s"), "bf16": (2516.6, "TFLOP/s"), "f16": (2516.6, "TFLOP/s"),
        "f64": (78.6, "TFLOP/s")}
HBM_PEAK_GBS = 8000.0


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=1000)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--prec", default="f32", choices=["f32", "bf16"])
    ap.add_argument("--alpha", type=float, default=1.0)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-overlap", action="store_true",
                    help="run the Gram/inverse branch on the main stream too")
    return ap.parse_args()


def hip_events(n):
    import torch
    hip = C.CDLL(os.path.join(os.path.dirname(torch.__file__), "lib", "libamdhip64.so"))
    hip.hipEventCreate.argtypes = [C.POINTER(C.c_void_p)]
    hip.hipEventElapsedTime.argtypes = [C.POINTER(C.c_float), C.c_void_p, C.c_void_p]
    hip.hipEventDestroy.argtypes = [C.c_void_p]
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


def build_problem(seed, I, R, kappa, dev):
    import torch
    import tr_inputs as ti
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import cores_to_device
    N = 3
    true3 = ti.illcond_cores(seed, N, I, R, kappa)
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


def cpu_baseline(seconds, seed, I, R, kappa, m, alpha):
    """The oracle as it stands, on the same workload, for a bounded number
    of steps; returns (steps/s, steps, threads)."""
    import tr_inputs as ti
    from oracle import brsgd, tr
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] or [1])
    except Exception:
        threads = os.cpu_count() or 1
    N = 3
    true3 = ti.illcond_cores(seed, N, I, R, kappa)
    X = tr.full_tensor(true3)
    c = float(np.mean(X * X)) ** (-1.0 / (2 * N))
    X = X * c ** N
    sig = (1.0 / R ** N) ** (1.0 / (2 * N))
    st = brsgd.State(ti.gaussian_cores(seed + 1, N, I, R, scale=sig))
    cfg = brsgd.Config(m=m, variant="scaled", alpha=alpha, seed=seed)
    brsgd.step(st, X, cfg)               # warm-up
    t0 = time.perf_counter()
    k = 0
    while time.perf_counter() - t0 < seconds:
        brsgd.step(st, X, cfg)
        k += 1
    dt = time.perf_counter() - t0
    return k / dt, k, threads


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 "
                          "(multi-GPU sharding is a design note, not implemented)"}))
        sys.exit(2)
    import torch
    from paper_2303_16492_amd import _lib as L
    from paper_2303_16492_amd import api
    from paper_2303_16492_amd.driver import TRSolver, cores_to_device

    dev = "cuda:0"
    I, R, kappa, m = 400, 10, 1e4, 4096
    N = 3
    desc, X, true3, init3 = build_problem(args.seed, I, R, kappa, dev)
    cores = cores_to_device(init3, torch.float32, dev)
    solver = TRSolver(cores, X, [I] * N, [R] * N, m, law="U", scaled=True, prec=args.prec,
                      rule=api.step_rule("fixed", alpha=args.alpha), seed=args.seed,
                      overlap=not args.no_overlap)
    print(f"[bench] workload ready: {I}^3 rank {R}, m={m}, prec={args.prec}", file=sys.stderr, flush=True)
    solver.run(args.warmup)
    torch.cuda.synchronize()
    print(f"[bench] warmup {args.warmup} steps done", file=sys.stderr, flush=True)

    K = args.steps
    hip, evs = hip_events(2 * K + 2)
    begin = (C.c_void_p * K)(*[e.value for e in evs[2:2 + K]])
    end = (C.c_void_p * K)(*[e.value for e in evs[2 + K:2 + 2 * K]])
    opts = L.tr_run_opts()
    if solver.opts is not None:
        so = solver.opts
        opts.aux, opts.ev_fork, opts.ev_gram, opts.ev_join = so.aux, so.ev_fork, so.ev_gram, so.ev_join
    opts.ev_begin = C.cast(begin, C.POINTER(C.c_void_p))
    opts.ev_end = C.cast(end, C.POINTER(C.c_void_p))
    stream = torch.cuda.current_stream()
    torch.cuda.synchronize()
    assert hip.hipEventRecord(evs[0], C.c_void_p(stream.cuda_stream)) == 0
    rc = api.lib().tr_run_ex(C.byref(solver.problem), C.byref(solver.config), C.c_void_p(solver.t_dev.data_ptr()),
                             K, None, C.c_void_p(solver.status.data_ptr()), C.c_void_p(solver.ws.data_ptr()),
                             solver.ws.numel(), C.c_void_p(stream.cuda_stream), C.byref(opts))
    assert rc == 0, rc
    assert hip.hipEventRecord(evs[1], C.c_void_p(stream.cuda_stream)) == 0
    torch.cuda.synchronize()
    total_ms = elapsed_ms(hip, evs[0], evs[1])
    kern_ms = [elapsed_ms(hip, evs[2 + i], evs[2 + K + i]) for i in range(K)]
    kern_avg_us = 1e3 * float(np.mean(kern_ms))
    ms_per_step = total_ms / K
    rse = float(solver.rse())
    status = int(solver.status.item())
    print(f"[bench] timed {K} steps: {ms_per_step * 1e3:.2f} us/step, kernel {kern_avg_us:.2f} us, "
          f"rse {rse:.3e}", file=sys.stderr, flush=True)

    RR = R * R
    flops = 4.0 * I * m * RR                       # prediction + gradient contractions
    bytes_alg = I * m * 4 + m * RR * 4 + I * RR * 4  # fibers + sampled rows + core
    peak, unit = PEAK[args.prec]
    achieved = flops / (kern_avg_us * 1e-6) / 1e12
    roof = {"bound": "mfma", "achieved": round(achieved, 3), "peak": peak, "unit": unit,
            "frac": round(achieved / peak, 5), "traffic": None,
            "kernel": "k_grad_mfma_f32" if args.prec == "f32" else "k_grad_mixed", "kernel_avg_us": round(kern_avg_us, 3),
            "flops_per_launch": flops, "alg_bytes_per_launch": bytes_alg,
            "alg_hbm_gbs": round(bytes_alg / (kern_avg_us * 1e-6) / 1e9, 1)}

    cpu = None
    if not args.no_cpu_baseline:
        print("[bench] cpu oracle baseline ...", file=sys.stderr, flush=True)
        v, k, th = cpu_baseline(args.cpu_seconds, args.seed, I, R, kappa, m, args.alpha)
        cpu = {"value": round(v, 4), "unit": "steps/s", "cores": th, "kind": "oracle",
               "sample": f"{k} oracle steps (FP64 numpy/scipy) of the same 400^3 workload after 1 warm-up step"}

    out = {
        "metric": "sampled-gradient steps/s (TR-ScaledBRSGD, FP64 Cholesky), 1 GPU",
        "value": round(1e3 / ms_per_step, 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": args.prec,
        "data": "synthetic",
        "config": {"workload": "scaled-illcond-n3-i400-r10", "N": N, "I": I, "R": R, "kappa": kappa,
                   "m": m, "m_H": m, "law": "uniform", "alpha": args.alpha, "prec": args.prec,
                   "overlap": not args.no_overlap},
        "roofline": roof,
        "cpu_baseline": cpu,
        "rse_after": rse,
        "dev_status": status,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
