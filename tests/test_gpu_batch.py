"""a11: many independent problems in one persistent launch.  Every problem
of a batch takes the oracle's step (same Philox draws, FP16 matrix-core
products with FP32 accumulation against the FP64 oracle), equals itself run
alone bit for bit, and the tile variants and graph replay agree."""
import numpy as np
import pytest
import torch

import tr_inputs as ti
from oracle import brsgd, tr
from gpu_util import DEV, rel, rounded, say, to_dev, unfold, flat_paper

pytestmark = pytest.mark.gpu

from paper_2303_16492_amd import api  # noqa: E402
from paper_2303_16492_amd.driver import TRBatch  # noqa: E402

TOL16 = 5e-3   # FP16 products, FP32 accumulation, against the FP64 oracle


def small_instances(seed, count, big=False):
    rng = np.random.default_rng(seed)
    out = []
    for p in range(count):
        N = int(rng.choice([3, 4, 5]))
        if big and p == 0:
            N, I, R = 3, [128, 20, 17], [12, 12, 12]     # largest I_n and R_n R_{n+1} = 144
        else:
            I = [int(x) for x in rng.integers(8, 19, size=N)]
            R = [int(x) for x in rng.integers(2, 6, size=N)]
        out.append(ti.BatchInstance(N=N, I=I, R=R, seed=int(rng.integers(0, 2**31))))
    return out


def build(instances, m, rule_kind="fixed", alpha=0.05, eta=0.02, noise_db=40.0):
    """Device problems plus the oracle's inputs (X rounded to FP16 once)."""
    probs, host = [], []
    for q, b in enumerate(instances):
        Xt = tr.full_tensor(ti.gaussian_cores(b.seed, b.N, b.I, b.R))
        X = brsgd.add_noise(Xt, ti.standard_normal(b.seed + 5, Xt.shape), noise_db)
        X = rounded(X, torch.float16)
        sig = brsgd.init_scale(X, b.R)
        init = [rounded(c, torch.float32) for c in ti.gaussian_cores(b.seed + 1, b.N, b.I, b.R, scale=sig)]
        desc = api.make_desc(b.I, b.R, torch.float32, torch.float16)
        dX = to_dev(flat_paper(X), torch.float16)
        reps = [api.tr_x_replicate(desc, dX, n) for n in range(b.N)]
        cores = [to_dev(unfold(c), torch.float32) for c in init]
        rule = api.step_rule(rule_kind, alpha=alpha, eta=eta)
        probs.append(dict(cores=cores, Xrep=reps, I=b.I, R=b.R, m=m, rule=rule, seed=b.seed))
        host.append((X, init, b))
    return probs, host


def oracle_steps(host, m, steps, rule_kind="fixed", alpha=0.05, eta=0.02):
    outs = []
    for X, init, b in host:
        st = brsgd.State([c.copy() for c in init])
        cfg = brsgd.Config(m=m, alpha=alpha, eta=eta, rule=rule_kind, seed=b.seed)
        losses = []
        for _ in range(steps):
            tr_ = {}
            brsgd.step(st, X, cfg, trace=tr_)
            losses.append(tr_["loss"])
        outs.append((st, losses))
    return outs


@pytest.mark.parametrize("splits", [1, 4, 16])
@pytest.mark.parametrize("rule_kind", ["fixed", "adagrad"])
def test_one_step_matches_oracle(rule_kind, splits):
    inst = small_instances(1, 6, big=True)
    probs, host = build(inst, m=100, rule_kind=rule_kind)
    B = TRBatch(probs)
    say("batch one step", rule_kind, splits, [b.N for b in inst])
    B.run(1, splits=splits)
    torch.cuda.synchronize()
    ref = oracle_steps(host, 100, 1, rule_kind)
    assert B.t_dev.cpu().tolist() == [1] * len(inst)
    for p, ((X, init, b), (st, losses)) in enumerate(zip(host, ref)):
        for k in range(b.N):
            got = probs[p]["cores"][k].cpu().numpy().astype(np.float64)
            want = unfold(st.cores[k])
            base = unfold(init[k])
            dw = want - base
            if np.linalg.norm(dw) == 0:
                assert np.array_equal(got, base), (p, k)     # cores other than n untouched
            else:
                assert rel(got - base, dw) < TOL16, (p, k, rel(got - base, dw))
        assert abs(float(B.loss[p]) - losses[-1]) <= TOL16 * abs(losses[-1])


@pytest.mark.parametrize("splits", [1, 4, 16])
def test_each_problem_equals_itself_alone(splits):
    inst = small_instances(2, 5)
    probs, _ = build(inst, m=70, rule_kind="adagrad")
    B = TRBatch(probs)
    B.run(4, splits=splits)
    torch.cuda.synchronize()
    together = [[c.clone() for c in pr["cores"]] for pr in probs]
    assert all(bool(torch.isfinite(c).all()) for cs in together for c in cs)
    for p, b in enumerate(inst):
        solo, _ = build([b], m=70, rule_kind="adagrad")
        S = TRBatch(solo)
        S.run(4, splits=splits)
        torch.cuda.synchronize()
        say("solo", p)
        for a, c in zip(together[p], solo[0]["cores"]):
            assert torch.equal(a, c)


def test_tile_variants_agree():
    inst = small_instances(3, 4)
    outs = []
    # every tile variant with one and four shares, plus six shares (the
    # apply then fetches the shares in two rounds, the second partly clamped)
    for (ch, wv), sp in [(v, 1) for v in TRBatch.VARIANTS] + [(v, 4) for v in TRBatch.VARIANTS] + [((64, 8), 6)]:
        probs, _ = build(inst, m=96)
        B = TRBatch(probs)
        B.run(3, ch, wv, sp)
        torch.cuda.synchronize()
        outs.append([[c.cpu().numpy() for c in pr["cores"]] for pr in probs])
    for other in outs[1:]:
        for pa, pb in zip(outs[0], other):
            for a, b in zip(pa, pb):
                assert rel(b, a) < 1e-5


@pytest.mark.parametrize("splits", [1, 4, 16])
def test_graph_replay_equals_eager_bitwise(splits):
    inst = small_instances(4, 4)
    pa, _ = build(inst, m=64, rule_kind="adagrad")
    A = TRBatch(pa)
    A.splits = splits
    A.run(6)
    torch.cuda.synchronize()
    assert all(bool(torch.isfinite(c).all()) for x in pa for c in x["cores"])
    pb, _ = build(inst, m=64, rule_kind="adagrad")
    Bb = TRBatch(pb)
    Bb.splits = splits
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        Bb.run(1)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    with torch.cuda.graph(g):
        Bb.run(1)
    for _ in range(5):
        g.replay()
        torch.cuda.synchronize()
    assert Bb.t_dev.cpu().tolist() == A.t_dev.cpu().tolist() == [6] * 4
    for x, y in zip(pa, pb):
        for a, b in zip(x["cores"], y["cores"]):
            assert torch.equal(a, b)


def test_trajectory_tracks_oracle_and_tuner_restores_state():
    inst = small_instances(5, 4)
    probs, host = build(inst, m=128, rule_kind="adagrad", eta=0.05)
    B = TRBatch(probs)
    before = [[c.clone() for c in pr["cores"]] for pr in probs]
    times = B.tune(steps=2, reps=1)
    say("tuned", times, "->", (B.chunk, B.waves))
    assert B.t_dev.cpu().tolist() == [0] * 4
    for x, pr in zip(before, probs):
        for a, b in zip(x, pr["cores"]):
            assert torch.equal(a, b)
    B.run(15)
    torch.cuda.synchronize()
    ref = oracle_steps(host, 128, 15, "adagrad", eta=0.05)
    for p, ((X, init, b), (st, _)) in enumerate(zip(host, ref)):
        got = [pr.cpu().numpy().astype(np.float64) for pr in probs[p]["cores"]]
        Xg = tr.full_tensor([unfold_back(g, b.R[k], b.R[(k + 1) % b.N]) for k, g in enumerate(got)])
        Xo = tr.full_tensor(st.cores)
        assert rel(Xg, Xo) < 2e-2, p


def unfold_back(G2, Rk, Rk1):
    return np.ascontiguousarray(G2.reshape(G2.shape[0], Rk1, Rk).transpose(2, 0, 1))


@pytest.mark.parametrize("splits", [1, 4, 16])
def test_full_batch_step_at_bench_configuration(splits):
    """The 64-problem workload the benchmark times (orders 3-5, sizes 16-128,
    ranks 3-12, FP16 tensors, m = 1024, AdaGrad) in its launch configuration
    (chunks of 64 samples, eight wavefronts, each problem's samples on one or
    four workgroups): one step of all problems; the smallest problem of each
    order, the problem with the largest R_n R_{n+1} and the one with the most
    entries are checked against the oracle, every problem advances its
    counter with no device flag raised."""
    inst = ti.batched_instances(0)
    sampled = {}
    for N in (3, 4, 5):
        p = min((q for q, b in enumerate(inst) if b.N == N), key=lambda q: int(np.prod(inst[q].I)))
        sampled[p] = None
    rr = [max(b.R[k] * b.R[(k + 1) % b.N] for k in range(b.N)) for b in inst]
    sampled[int(np.argmax(rr))] = None
    sampled[int(np.argmax([int(np.prod(b.I)) for b in inst]))] = None
    assert len(sampled) == 5
    m, eta = 1024, 0.05
    probs, host = [], {}
    for p, b in enumerate(inst):
        rule = api.step_rule("adagrad", eta=eta)
        if p in sampled:
            (X, init, _), = build([b], m, rule_kind="adagrad", eta=eta)[1]
            desc = api.make_desc(b.I, b.R, torch.float32, torch.float16)
            dX = to_dev(flat_paper(X), torch.float16)
            reps = [api.tr_x_replicate(desc, dX, n) for n in range(b.N)]
            cores = [to_dev(unfold(c), torch.float32) for c in init]
            host[p] = (X, init, b)
        else:   # not checked against the oracle: a noise-free planted tensor built on the device
            d32 = api.make_desc(b.I, b.R, torch.float32, torch.float32)
            d16 = api.make_desc(b.I, b.R, torch.float32, torch.float16)
            true = [to_dev(unfold(c), torch.float32) for c in ti.gaussian_cores(b.seed, b.N, b.I, b.R)]
            X16 = api.tr_reconstruct(d32, true).half()
            sig = (float(X16.float().pow(2).mean()) / float(np.prod(b.R))) ** (1.0 / (2 * b.N))
            cores = [to_dev(unfold(c), torch.float32) for c in ti.gaussian_cores(b.seed + 1, b.N, b.I, b.R, scale=sig)]
            reps = [api.tr_x_replicate(d16, X16, n) for n in range(b.N)]
            del X16
        probs.append(dict(cores=cores, Xrep=reps, I=b.I, R=b.R, m=m, rule=rule, seed=b.seed))
    B = TRBatch(probs)
    say("full batch step, sampled problems", sorted(sampled))
    B.run(1, chunk=64, waves=8, splits=splits)
    torch.cuda.synchronize()
    assert B.t_dev.cpu().tolist() == [1] * len(inst)
    assert int(B.status.max()) == 0
    for p in sorted(sampled):
        X, init, b = host[p]
        say("oracle step of problem", p, b.N, b.I, b.R)
        st = brsgd.State([c.copy() for c in init])
        trace = {}
        n = brsgd.step(st, X, brsgd.Config(m=m, eta=eta, rule="adagrad", seed=b.seed), trace=trace)
        for k in range(b.N):
            got = probs[p]["cores"][k].cpu().numpy().astype(np.float64)
            want, base = unfold(st.cores[k]), unfold(init[k])
            if k != n:
                assert np.array_equal(got, base), (p, k)
                continue
            # AdaGrad's first step is eta * sign(p) entrywise: an entry whose
            # direction is below the rounding of the 16-bit products (relative
            # 5e-3 of the largest) may take the other sign; every other entry
            # must agree to the FP32 rounding of the sum.
            dg, dw = got - base, want - base
            pdir = np.abs(trace["p"])
            flip = np.sign(dg) != np.sign(dw)
            assert np.all(pdir[flip] <= TOL16 * pdir.max()), (p, k, int(flip.sum()))
            assert rel(np.where(flip, 0.0, dg), np.where(flip, 0.0, dw)) < TOL16, (p, k)
        assert abs(float(B.loss[p]) - trace["loss"]) <= TOL16 * abs(trace["loss"]), p
    for pr in probs:
        for c in pr["cores"]:
            assert bool(torch.isfinite(c).all())
