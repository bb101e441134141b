"""tr_run_noalloc (the step driver on the library's own static device
scratch, for callers that cannot allocate) against tr_run_ex with a caller
workspace: the same steps give the same cores, accumulators, step counter and
loss estimates, bit for bit, on two calls in a row, the second on a smaller
problem (so the scratch holds the first call's contents); a problem whose
workspace exceeds the scratch is rejected before anything is enqueued."""
import ctypes as C

import numpy as np
import pytest
import torch

import tr_inputs as ti
from oracle import tr
from gpu_util import DEV, flat_paper, rounded, say, to_dev, unfold

pytestmark = pytest.mark.gpu

from paper_2303_16492_amd import _lib as L  # noqa: E402
from paper_2303_16492_amd import api  # noqa: E402
from paper_2303_16492_amd.driver import TRSolver  # noqa: E402


def _pair(I, R, m, scaled, rule, prec, law, steps, seed):
    """Run ``steps`` steps twice from the same state: tr_run_ex with the
    solver's workspace, then tr_run_noalloc; return both end states."""
    N = len(I)
    dtype = torch.float32
    Xt = tr.full_tensor(ti.gaussian_cores(seed, N, I, R))
    X = rounded(Xt + 0.01 * ti.standard_normal(seed + 2, Xt.shape), dtype)
    init = [rounded(c, dtype) for c in ti.gaussian_cores(seed + 1, N, I, R, scale=0.5)]
    dX = to_dev(flat_paper(X), dtype)
    outs = []
    for noalloc in (False, True):
        sol = TRSolver([to_dev(unfold(c), dtype) for c in init], dX, I, R, m, law=law, scaled=scaled, prec=prec,
                       rule=rule, seed=seed, overlap=scaled)
        losses = torch.zeros(steps, dtype=torch.float64, device=DEV)
        stream = C.c_void_p(torch.cuda.current_stream().cuda_stream)
        opts = C.byref(sol.opts) if sol.opts is not None else None
        if noalloc:
            rc = L.lib().tr_run_noalloc(C.byref(sol.problem), C.byref(sol.config), C.c_void_p(sol.t_dev.data_ptr()),
                                        steps, C.c_void_p(losses.data_ptr()), C.c_void_p(sol.status.data_ptr()),
                                        stream, opts)
        else:
            rc = L.lib().tr_run_ex(C.byref(sol.problem), C.byref(sol.config), C.c_void_p(sol.t_dev.data_ptr()),
                                   steps, C.c_void_p(losses.data_ptr()), C.c_void_p(sol.status.data_ptr()),
                                   C.c_void_p(sol.ws.data_ptr()), sol.ws.numel(), stream, opts)
        assert rc == 0, (noalloc, rc)
        torch.cuda.synchronize()
        outs.append(([c.clone() for c in sol.cores], [a.clone() for a in sol.accum if a is not None], sol.t,
                     losses.clone(), int(sol.status.item())))
        del sol
    return outs


def _assert_same(a, b):
    (ca, aa, ta, la, sa), (cb, ab, tb, lb, sb) = a, b
    assert ta == tb and sa == sb
    assert torch.equal(la, lb)
    for x, y in zip(ca, cb):
        assert torch.equal(x, y)
    for x, y in zip(aa, ab):
        assert torch.equal(x, y)


def test_noalloc_equals_workspace_run_twice_second_smaller():
    say("no-alloc call 1: scaled, 60x50x40, ranks 4, m 700")
    a, b = _pair([60, 50, 40], [4, 4, 4], 700, True, api.step_rule("fixed", alpha=0.5), "f32", "U", 9, 11)
    _assert_same(a, b)
    assert b[2] == 9
    say("no-alloc call 2: plain AdaGrad, leverage law, 20x17x15x9, ranks 2-3, m 100")
    a, b = _pair([20, 17, 15, 9], [2, 3, 2, 3], 100, False, api.step_rule("adagrad", eta=0.05), "f32", "L", 7, 12)
    _assert_same(a, b)
    assert b[2] == 7


def test_noalloc_rejects_a_problem_larger_than_its_scratch():
    """400^3 with ranks 16 and m = 60000: the step's workspace is far above
    TR_NOALLOC_SCRATCH_BYTES; the call returns TR_E_WORKSPACE and the step
    counter is untouched (nothing was enqueued)."""
    I, R, m = [400, 400, 400], [16, 16, 16], 60000
    desc = api.make_desc(I, R, torch.float32)
    p = L.tr_problem()
    p.desc = desc
    cores = [torch.zeros(I[k] * R[k] * R[(k + 1) % 3], dtype=torch.float32, device=DEV) for k in range(3)]
    X = torch.zeros(4, dtype=torch.float32, device=DEV)
    for k in range(3):
        p.cores[k] = cores[k].data_ptr()
    p.X = X.data_ptr()
    c = L.tr_config()
    c.m, c.m_H, c.law, c.scaled, c.prec = m, 0, L.TR_LAW_UNIFORM, 1, L.TR_PREC_F32
    c.rule = api.step_rule("fixed", alpha=1.0)
    assert api.tr_run_workspace_size(p, c) > L.TR_NOALLOC_SCRATCH_BYTES
    t = torch.zeros(1, dtype=torch.int64, device=DEV)
    st = torch.zeros(1, dtype=torch.int32, device=DEV)
    rc = L.lib().tr_run_noalloc(C.byref(p), C.byref(c), C.c_void_p(t.data_ptr()), 5, None,
                                C.c_void_p(st.data_ptr()), C.c_void_p(torch.cuda.current_stream().cuda_stream), None)
    torch.cuda.synchronize()
    assert rc == L.TR_E_WORKSPACE
    assert int(t.item()) == 0
