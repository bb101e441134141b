"""Whole iterations on the GPU against the oracle: the FP64 20^3 rank-3
trajectory with bit-exact index sets at every step, multi-step runs under
every law and step rule, graph replay and run-to-run bitwise equality."""
import numpy as np
import pytest
import torch

import tr_inputs as ti
from oracle import brsgd, tr
from gpu_util import DEV, flat_paper, fold, rel, rounded, say, to_dev, unfold

pytestmark = pytest.mark.gpu

from paper_2303_16492_amd import _lib as L  # noqa: E402
from paper_2303_16492_amd import api  # noqa: E402
from paper_2303_16492_amd.driver import TRSolver  # noqa: E402


def planted(N, I, R, dtype, seed=0, noise_db=None):
    Xt = tr.full_tensor(ti.gaussian_cores(seed, N, I, R))
    X = Xt if noise_db is None else brsgd.add_noise(Xt, ti.standard_normal(seed + 5, Xt.shape), noise_db)
    X = rounded(X, dtype)
    sig = brsgd.init_scale(X, [R] * N if np.isscalar(R) else R)
    init = [rounded(c, dtype) for c in ti.gaussian_cores(seed + 1, N, I, R, scale=sig)]
    return X, Xt, init


def test_fp64_trajectory_indices_bit_exact_every_step():
    """20^3, ranks 3, uniform fibers, m = 100, alpha = 0.2, 500 steps, seed 0:
    the per-call path draws the oracle's index sets and p_F at each of the
    500 steps; final cores within 1e-10 and the final RSE within 1e-12 (RSE
    units) of the oracle's."""
    N, I, R, m, steps = 3, 20, 3, 100, 500
    X, _, init = planted(N, I, R, torch.float64)
    desc = api.make_desc([I] * N, [R] * N, torch.float64)
    dX = to_dev(flat_paper(X), torch.float64)
    dcores = [to_dev(unfold(c), torch.float64) for c in init]
    st = brsgd.State(init)
    cfg = brsgd.Config(m=m, alpha=0.2, seed=0)
    rule = api.step_rule("fixed", alpha=0.2)
    g_buf = None
    for t in range(steps):
        n = api.tr_mode(0, t, N)
        trace = {}
        brsgd.step(st, X, cfg, trace=trace)
        assert trace["n"] == n
        idx, pF = api.tr_sample(desc, 0, t, n, m)
        S = api.tr_subchain(desc, n, dcores, idx, m)
        g, _, _ = api.tr_grad(desc, n, dcores[n], dX, idx, S, pF, m, L.TR_PREC_F64)
        api.tr_update(desc, n, dcores[n], g, rule=rule, t=t)
        if t % 100 == 0:
            say("trajectory step", t)
        assert np.array_equal(idx.cpu().numpy(), trace["idx"]), t
        assert np.array_equal(pF.cpu().numpy(), trace["pF"]), t
    for k in range(N):
        assert rel(dcores[k].cpu().numpy(), unfold(st.cores[k])) < 1e-10
    want = tr.rse(st.cores, X)
    assert want < 1e-8
    got = float(api.tr_relerr(desc, dcores, dX))
    # RSE units (relative to ||X||): the subtraction X_hat - X alone leaves
    # about u ||X|| of error in a residual of size RSE ||X||
    assert abs(got - want) < 1e-12, (got, want)
    assert abs(got - want) < 1e-3 * want, (got, want)


def _run_both(N, I, R, dtype, m, law, scaled, rule_kind, steps, seed=0, m_H=0, noise_db=40.0,
              alpha=0.1, eta=0.05, damping=0.0):
    X, _, init = planted(N, I, R, dtype, seed=seed, noise_db=noise_db)
    II = [I] * N if np.isscalar(I) else I
    RR_ = [R] * N if np.isscalar(R) else R
    dX = to_dev(flat_paper(X), dtype)
    dcores = [to_dev(unfold(c), dtype) for c in init]
    rule = api.step_rule(rule_kind, alpha=alpha, eta=eta, tau=50.0)
    prec = "f64" if dtype == torch.float64 else "f32"
    sol = TRSolver(dcores, dX, II, RR_, m, law=law, scaled=scaled, prec=prec, rule=rule,
                   damping=damping, m_H=m_H, seed=seed)
    sol.run(steps)
    st = brsgd.State(init)
    cfg = brsgd.Config(m=m, dist=law, variant="scaled" if scaled else "plain", rule=rule_kind,
                       alpha=alpha, eta=eta, tau=50.0, damping=damping, m_H=(m_H or None), seed=seed)
    for _ in range(steps):
        brsgd.step(st, X, cfg)
    torch.cuda.synchronize()
    return sol, st, X


@pytest.mark.parametrize("law", ["U", "E", "L", "O"])
def test_adagrad_run_each_law_fp64(law):
    say("run law fp64", law)
    sol, st, X = _run_both(4, [9, 8, 7, 10], [2, 3, 2, 3], torch.float64, 64, law, False, "adagrad", 40)
    assert sol.t == 40 and int(sol.status.item()) == st.status
    for k in range(4):
        assert rel(sol.cores[k].cpu().numpy(), unfold(st.cores[k])) < 1e-10


@pytest.mark.parametrize("law", ["U", "E", "L", "O"])
def test_adagrad_run_each_law_fp32(law):
    say("run law fp32", law)
    sol, st, X = _run_both(4, [9, 8, 7, 10], [2, 3, 2, 3], torch.float32, 64, law, False, "adagrad", 25)
    for k in range(4):
        assert rel(sol.cores[k].cpu().numpy(), unfold(st.cores[k])) < 1e-4


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32])
@pytest.mark.parametrize("m_H", [0, 150])
def test_scaled_run(dtype, m_H):
    say("scaled run", dtype, m_H)
    sol, st, X = _run_both(3, [30, 25, 28], [3, 3, 3], dtype, 200, "U", True, "fixed", 20, m_H=m_H,
                           alpha=0.5, noise_db=None)
    tol = 1e-9 if dtype == torch.float64 else 2e-4
    for k in range(3):
        assert rel(sol.cores[k].cpu().numpy(), unfold(st.cores[k])) < tol


def test_robbins_monro_run_fp64():
    sol, st, X = _run_both(3, [12, 10, 11], [2, 3, 2], torch.float64, 50, "E", False, "robbins-monro", 30,
                           alpha=0.05)
    for k in range(3):
        assert rel(sol.cores[k].cpu().numpy(), unfold(st.cores[k])) < 1e-10


def test_planted_recovery_fp64_on_gpu():
    """The device path recovers the planted 20^3 rank-3 ring to RSE <= 1e-10."""
    N, I, R = 3, 20, 3
    X, _, init = planted(N, I, R, torch.float64)
    dX = to_dev(flat_paper(X), torch.float64)
    sol = TRSolver([to_dev(unfold(c), torch.float64) for c in init], dX, [I] * N, [R] * N, 100,
                   prec="f64", rule=api.step_rule("fixed", alpha=0.2))
    sol.run(900)
    rse = float(sol.rse())
    say("planted rse", rse)
    assert rse <= 1e-10


def test_graph_replay_equals_eager_bitwise():
    dtype = torch.float32
    X, _, init = planted(3, [40, 30, 35], [3, 4, 3], dtype, noise_db=40.0)
    dX = to_dev(flat_paper(X), dtype)
    mk = lambda: TRSolver([to_dev(unfold(c), dtype) for c in init], dX, [40, 30, 35], [3, 4, 3], 256,
                          law="E", scaled=True, prec="f32", rule=api.step_rule("fixed", alpha=0.5))
    a = mk()
    a.run(1 + 3 * 5)
    b = mk()
    g = b.capture(5)            # one eager warm-up step + a 5-step graph
    for _ in range(3):
        g.replay()
        torch.cuda.synchronize()
        say("replay t", b.t)
    torch.cuda.synchronize()
    assert a.t == b.t == 16
    for k in range(3):
        assert torch.equal(a.cores[k], b.cores[k])


def test_runs_are_bitwise_reproducible():
    dtype = torch.float32
    X, _, init = planted(4, [9, 8, 7, 10], [2, 3, 2, 3], dtype, noise_db=40.0)
    dX = to_dev(flat_paper(X), dtype)
    outs = []
    for _ in range(2):
        s = TRSolver([to_dev(unfold(c), dtype) for c in init], dX, [9, 8, 7, 10], [2, 3, 2, 3], 128,
                     law="L", prec="f32", rule=api.step_rule("adagrad", eta=0.05))
        s.run(30)
        outs.append([c.clone() for c in s.cores])
    for a, b in zip(*outs):
        assert torch.equal(a, b)


def test_loss_estimates_written_per_step():
    dtype = torch.float64
    X, _, init = planted(3, [12, 10, 11], [2, 3, 2], dtype)
    dX = to_dev(flat_paper(X), dtype)
    s = TRSolver([to_dev(unfold(c), dtype) for c in init], dX, [12, 10, 11], [2, 3, 2], 64, prec="f64",
                 rule=api.step_rule("fixed", alpha=0.1))
    losses = torch.zeros(10, dtype=torch.float64, device=DEV)
    s.run(10, loss_out=losses)
    st = brsgd.State(init)
    cfg = brsgd.Config(m=64, alpha=0.1)
    ref = []
    for _ in range(10):
        tr_ = {}
        brsgd.step(st, X, cfg, trace=tr_)
        ref.append(tr_["loss"])
    assert rel(losses.cpu().numpy(), np.array(ref)) < 1e-10


@pytest.mark.parametrize("prec", ["bf16", "f16"])
def test_mixed_scaled_run_tracks_oracle(prec):
    """A few mixed-precision scaled steps stay within the 16-bit bar of the
    FP64 oracle's trajectory."""
    dtype = torch.float32
    X, _, init = planted(3, [30, 25, 28], [3, 3, 3], dtype, noise_db=None)
    dX = to_dev(flat_paper(X), dtype)
    sol = TRSolver([to_dev(unfold(c), dtype) for c in init], dX, [30, 25, 28], [3, 3, 3], 200, scaled=True,
                   prec=prec, rule=api.step_rule("fixed", alpha=0.5))
    sol.run(6)
    st = brsgd.State(init)
    cfg = brsgd.Config(m=200, variant="scaled", alpha=0.5)
    for _ in range(6):
        brsgd.step(st, X, cfg)
    torch.cuda.synchronize()
    for k in range(3):
        assert rel(sol.cores[k].cpu().numpy(), unfold(st.cores[k])) < 5e-3


@pytest.mark.parametrize("m_H", [0, 150])
@pytest.mark.parametrize("shape", [([30, 25, 28], [3, 4, 3]), ([28, 28, 28], [3, 3, 3])])
def test_overlapped_branch_equals_serial_bitwise(m_H, shape):
    """The Gram/inverse branch on a second stream changes no arithmetic: the
    same cores, step counter and loss as the one-stream run.  With an
    independent H draw and modes of one shape the branch forks before the
    step's own draws and its sample kernel draws the mode itself."""
    dtype = torch.float32
    I, R = shape
    X, _, init = planted(3, I, R, dtype, noise_db=40.0)
    dX = to_dev(flat_paper(X), dtype)
    outs = []
    for overlap in (False, True):
        s = TRSolver([to_dev(unfold(c), dtype) for c in init], dX, I, R, 200, scaled=True,
                     prec="f32", rule=api.step_rule("fixed", alpha=0.5), m_H=m_H, overlap=overlap)
        losses = torch.zeros(12, dtype=torch.float64, device=DEV)
        s.run(12, loss_out=losses)
        torch.cuda.synchronize()
        say("overlap", overlap, "t", s.t)
        outs.append(([c.clone() for c in s.cores], s.t, losses.clone()))
    (ca, ta, la), (cb, tb, lb) = outs
    assert ta == tb == 12
    assert torch.equal(la, lb)
    for a, b in zip(ca, cb):
        assert torch.equal(a, b)


@pytest.mark.parametrize("law", ["U", "E", "L", "O"])
def test_adagrad_run_each_law_at_full_size(law):
    """The four-law workload at its full size: order 4, 64 per mode, ranks 5,
    40 dB noise, FP32, m = 512, AdaGrad; a few whole steps on the GPU against
    the FP64 oracle."""
    say("run law full size", law)
    sol, st, X = _run_both(4, 64, 5, torch.float32, 512, law, False, "adagrad", 6, eta=0.05)
    assert sol.t == 6 and int(sol.status.item()) == st.status
    for k in range(4):
        assert rel(sol.cores[k].cpu().numpy(), unfold(st.cores[k])) < 1e-4, (law, k)


def test_optimal_law_run_fibers_longer_than_a_wavefront():
    """Law O through tr_run with mode sizes above 64 (two fiber rows per
    lane when the law's terms read the mode-major replicas) and mixed ranks:
    12 AdaGrad steps in FP64 against the oracle."""
    say("run law O, I up to 100")
    sol, st, X = _run_both(3, [70, 90, 100], [3, 4, 2], torch.float64, 64, "O", False, "adagrad", 12)
    assert sol.t == 12 and int(sol.status.item()) == st.status
    for k in range(3):
        assert rel(sol.cores[k].cpu().numpy(), unfold(st.cores[k])) < 1e-10, k


def test_optimal_law_run_fp16_tensor():
    """Law O through tr_run with an FP16 tensor and FP32 cores (the law's
    terms read the FP16 mode-major replicas): 8 AdaGrad steps against the
    oracle run on the FP16 values of X."""
    say("run law O, FP16 tensor")
    N, I, R, m, steps = 3, [40, 36, 44], [3, 4, 3], 128, 8
    Xt = tr.full_tensor(ti.gaussian_cores(3, N, I, R))
    X = rounded(brsgd.add_noise(Xt, ti.standard_normal(8, Xt.shape), 40.0), torch.float16)
    sig = brsgd.init_scale(X, R)
    init = [rounded(c, torch.float32) for c in ti.gaussian_cores(4, N, I, R, scale=sig)]
    dX = to_dev(flat_paper(X), torch.float16)
    dcores = [to_dev(unfold(c), torch.float32) for c in init]
    rule = api.step_rule("adagrad", eta=0.05)
    sol = TRSolver(dcores, dX, I, R, m, law="O", scaled=False, prec="f32", rule=rule, seed=2)
    sol.run(steps)
    st = brsgd.State(init)
    cfg = brsgd.Config(m=m, dist="O", rule="adagrad", eta=0.05, seed=2)
    for _ in range(steps):
        brsgd.step(st, X, cfg)
    torch.cuda.synchronize()
    assert sol.t == steps and int(sol.status.item()) == st.status
    for k in range(N):
        assert rel(sol.cores[k].cpu().numpy(), unfold(st.cores[k])) < 1e-4, k


def _graph_steps(sol, steps):
    """``steps`` steps from one captured graph of that length, replayed once
    (the capture itself runs one eager step first)."""
    g = sol.capture(steps)
    g.replay()
    torch.cuda.synchronize()
    return g


@pytest.mark.parametrize("prec,m_H", [("f32", None), ("bf16", None), ("f32", 150)])
def test_benchmarked_configuration_equal_shapes(prec, m_H):
    """The launch configuration the benchmark times, on a small problem:
    every mode with the same I_n and R_n R_{n+1} (the Gram, its reduction
    and the inverse then take mode 0's shape and never read the step
    counter), the Gram/inverse branch on a second stream, the mode slot
    published by the first kernel, graph capture and replay.  11 steps
    against the FP64 oracle's trajectory; with an independent H draw the
    branch forks before the step's draws."""
    dtype = torch.float32
    N, I, R, m = 3, 28, 3, 300
    X, _, init = planted(N, I, R, dtype, seed=3, noise_db=None)
    dX = to_dev(flat_paper(X), dtype)
    sol = TRSolver([to_dev(unfold(c), dtype) for c in init], dX, [I] * N, [R] * N, m, scaled=True, prec=prec,
                   rule=api.step_rule("fixed", alpha=0.5), seed=3, overlap=True, m_H=m_H or 0)
    assert sol.opts is not None
    _graph_steps(sol, 10)
    assert sol.t == 11
    st = brsgd.State(init)
    cfg = brsgd.Config(m=m, variant="scaled", alpha=0.5, seed=3, m_H=m_H)
    for _ in range(11):
        brsgd.step(st, X, cfg)
    tol = 2e-4 if prec == "f32" else 5e-3
    for k in range(N):
        e = rel(sol.cores[k].cpu().numpy(), unfold(st.cores[k]))
        say("equal shapes", prec, k, e)
        assert e < tol, (k, e)
    assert int(sol.status.item()) == st.status


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_benchmarked_configuration_full_size(prec):
    """The benchmark's workload and launch configuration: 400^3, ranks 10,
    each unfolding with singular values from 1 to 1e-4, |F_n| = 4096,
    alpha = 1, TRSolver with the second stream, captured one-step graphs
    replayed.  Each of 4 steps is checked against the oracle's step from the
    same (device) cores: the updated core within max(bar, 2^-22 cond(h)) of
    the oracle's (its Hessian's condition number amplifies the rounding of
    S), the other cores untouched, the step counter advanced."""
    dtype = torch.float32
    N, I, R, m = 3, 400, 10, 4096
    true3 = ti.illcond_cores(0, N, I, R, 1e4)
    X = tr.full_tensor(true3)
    X = rounded(X / np.sqrt(np.mean(X * X)), dtype)
    init = [rounded(c, dtype) for c in ti.gaussian_cores(1, N, I, R, scale=(1.0 / R ** N) ** (1 / (2 * N)))]
    dX = to_dev(flat_paper(X), dtype)
    sol = TRSolver([to_dev(unfold(c), dtype) for c in init], dX, [I] * N, [R] * N, m, scaled=True, prec=prec,
                   rule=api.step_rule("fixed", alpha=1.0), seed=0, overlap=True)
    g = sol.capture(1)               # t: 0 -> 1 (eager warm-up step)
    torch.cuda.synchronize()
    cfg = brsgd.Config(m=m, variant="scaled", alpha=1.0, seed=0)
    bar = 1e-5 if prec == "f32" else 5e-3
    for it in range(4):
        before = [fold(c.double().cpu().numpy(), R, R) for c in sol.cores]
        t = sol.t
        st = brsgd.State([c.copy() for c in before], t=t)
        trace = {}
        n = brsgd.step(st, X, cfg, trace=trace)
        g.replay()
        torch.cuda.synchronize()
        assert sol.t == t + 1
        cond = float(np.linalg.cond(trace["h"]))
        e = rel(sol.cores[n].double().cpu().numpy() - unfold(before[n]), trace["p"])
        say("full-size run", prec, "step", t, "mode", n, "rel", e, "cond(h)", f"{cond:.3e}")
        assert e < max(bar, 2.0 ** -22 * cond), (t, n, e, cond)
        for k in range(N):
            if k != n:
                assert np.array_equal(sol.cores[k].double().cpu().numpy(), unfold(before[k]))
    assert int(sol.status.item()) == 0


@pytest.mark.parametrize("schedule,eta0,tau", [("harmonic", 0.4, 3.0), ("geometric", 0.8, 0.7)])
@pytest.mark.parametrize("I,R", [([30, 25, 28], [3, 3, 3]), ([20, 20, 20], [3, 3, 3]), ([14, 13, 15], [12, 12, 12])])
def test_damping_schedule_run_fp64(schedule, eta0, tau, I, R):
    """Scaled runs with an iteration-specific damping eta^t (amended
    preconditioner): 12 FP64 steps against the oracle on the sweep route with
    unequal and equal mode shapes (the shape-only kernels then read t for
    eta^t) and on the Cholesky route (R_n R_{n+1} = 144)."""
    dtype = torch.float64
    X, _, init = planted(3, I, R, dtype, seed=2, noise_db=40.0)
    dX = to_dev(flat_paper(X), dtype)
    sol = TRSolver([to_dev(unfold(c), dtype) for c in init], dX, I, R, 300, scaled=True, prec="f64",
                   rule=api.step_rule("fixed", alpha=0.6), damping=eta0, damping_schedule=schedule,
                   damping_tau=tau, seed=2)
    g = sol.capture(5)             # one eager step, then a 5-step graph
    g.replay()
    g.replay()
    torch.cuda.synchronize()
    assert sol.t == 11
    st = brsgd.State(init)
    cfg = brsgd.Config(m=300, variant="scaled", alpha=0.6, damping=eta0, damping_schedule=schedule,
                       damping_tau=tau, seed=2)
    for _ in range(11):
        brsgd.step(st, X, cfg)
    for k in range(3):
        e = rel(sol.cores[k].cpu().numpy(), unfold(st.cores[k]))
        say("schedule", schedule, I, R, k, e)
        assert e < 1e-10, (k, e)


def test_large_damping_interpolates_to_the_plain_step():
    """eta^t -> infinity turns the scaled step into the plain one: with
    eta = 1e8 and alpha = eta alpha_0 the scaled GPU run follows the plain
    GPU run with alpha_0 (the limit named in the amended preconditioner's
    remark)."""
    dtype = torch.float64
    I, R = [30, 25, 28], [3, 3, 3]
    X, _, init = planted(3, I, R, dtype, seed=4, noise_db=40.0)
    dX = to_dev(flat_paper(X), dtype)
    eta, a0 = 1e8, 0.05
    runs = []
    for scaled in (True, False):
        s = TRSolver([to_dev(unfold(c), dtype) for c in init], dX, I, R, 200, scaled=scaled, prec="f64",
                     rule=api.step_rule("fixed", alpha=eta * a0 if scaled else a0), damping=eta if scaled else 0.0,
                     seed=4)
        s.run(8)
        torch.cuda.synchronize()
        runs.append([c.cpu().numpy() for c in s.cores])
    for a, b in zip(*runs):
        assert rel(a, b) < 1e-6
