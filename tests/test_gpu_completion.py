"""Tensor completion on the GPU (tr_completion_run) against the oracle:
a few steps with every core moved and with the block choice, with and
without the ridge term, fixed and AdaGrad rules, FP32 and FP16 observed
values; each step's loss; and recovery of a planted ring from 40% of its
entries."""
import numpy as np
import pytest
import torch

import tr_inputs as ti
from oracle import brsgd, completion, tr
from gpu_util import DEV, rel, rounded, say, to_dev, unfold

pytestmark = pytest.mark.gpu

from paper_2303_16492_amd import api  # noqa: E402


def _observed(sizes, ranks, frac, seed, xdt):
    X = tr.full_tensor(ti.gaussian_cores(seed, 3, sizes, ranks))
    mask = np.random.default_rng(seed + 10).random(X.shape) < frac
    obs_idx = np.argwhere(mask).astype(np.int32)
    obs_x = rounded(X[mask], xdt)
    return X, mask, obs_idx, obs_x


@pytest.mark.parametrize("xdt", [torch.float32, torch.float16])
@pytest.mark.parametrize("block,lam,rule", [(False, 0.0, "fixed"), (False, 0.05, "adagrad"), (True, 0.1, "fixed"),
                                            (True, 0.0, "adagrad")])
def test_completion_steps_match_oracle(block, lam, rule, xdt):
    sizes, ranks = [10, 9, 8], [2, 3, 2]
    X, mask, obs_idx, obs_x = _observed(sizes, ranks, 0.4, 3, xdt)
    init = [rounded(c, torch.float32) for c in ti.gaussian_cores(8, 3, sizes, ranks, scale=brsgd.init_scale(X, ranks))]
    steps, B = 6, 96
    cfg = completion.CompletionConfig(B=B, lam=lam, block=block, rule=rule, alpha=0.02, eta=0.05, seed=4)
    st = brsgd.State([c.copy() for c in init])
    losses = [completion.completion_step(st, obs_idx, obs_x, cfg) for _ in range(steps)]
    desc = api.make_desc(sizes, ranks, torch.float32, xdt)
    cores = [to_dev(unfold(c), torch.float32) for c in init]
    accum = [torch.zeros_like(c) for c in cores] if rule == "adagrad" else None
    t = torch.zeros(1, dtype=torch.int64, device=DEV)
    lo = torch.zeros(steps, dtype=torch.float64, device=DEV)
    c = api.completion_config(B, block=block, lam=lam, rule=api.step_rule(rule, alpha=0.02, eta=0.05), seed=4)
    say("completion", block, lam, rule, xdt)
    status = api.tr_completion_run(desc, cores, accum, to_dev(obs_idx, torch.int32), to_dev(obs_x, xdt), c, t, steps,
                                   loss_out=lo)
    torch.cuda.synchronize()
    assert int(t.item()) == steps and int(status.item()) == 0
    assert rel(lo.cpu().numpy(), np.array(losses)) < 1e-5
    for k in range(3):
        e = rel(cores[k].cpu().numpy(), unfold(st.cores[k]))
        say("  core", k, e)
        assert e < 1e-5, (k, e)


def test_completion_recovers_a_planted_ring():
    """10 x 9 x 8, ranks 2, 40% observed, AdaGrad eta = 0.5, B = 64, every
    core: the error on the never-observed entries falls below 1e-3 of their
    norm within 2500 steps (FP32), run as one captured graph of 500 steps
    replayed five times."""
    sizes, ranks = [10, 9, 8], [2, 2, 2]
    X, mask, obs_idx, obs_x = _observed(sizes, ranks, 0.4, 3, torch.float32)
    init = ti.gaussian_cores(8, 3, sizes, ranks, scale=brsgd.init_scale(X, ranks))
    desc = api.make_desc(sizes, ranks, torch.float32)
    cores = [to_dev(unfold(c), torch.float32) for c in init]
    accum = [torch.zeros_like(c) for c in cores]
    t = torch.zeros(1, dtype=torch.int64, device=DEV)
    c = api.completion_config(64, rule=api.step_rule("adagrad", eta=0.5), seed=5)
    di, dx = to_dev(obs_idx, torch.int32), to_dev(obs_x, torch.float32)
    ws = api.workspace(api.lib().tr_completion_workspace_size(api.C.byref(desc), api.C.byref(c)), DEV)
    status = torch.zeros(1, dtype=torch.int32, device=DEV)
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    torch.cuda.synchronize()
    with torch.cuda.graph(g, stream=s):
        api.tr_completion_run(desc, cores, accum, di, dx, c, t, 500, status=status, ws=ws)
    for _ in range(5):
        g.replay()
    torch.cuda.synchronize()
    assert int(t.item()) == 2500 and int(status.item()) == 0
    Xh = tr.full_tensor([np.ascontiguousarray(cc.double().cpu().numpy().reshape(sizes[k], ranks[(k + 1) % 3],
                                                                               ranks[k]).transpose(2, 0, 1))
                         for k, cc in enumerate(cores)])
    err = np.linalg.norm((Xh - X)[~mask]) / np.linalg.norm(X[~mask])
    say("completion held-out error", err)
    assert err < 1e-3, err
