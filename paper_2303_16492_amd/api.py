"""Python binding of the C ABI (include/tr.h), one function per entry point
with the same name.  Arguments are torch tensors on the GPU; this module only
marshals them (pointers, sizes, the current stream) and allocates outputs and
workspaces the caller did not pass.  Every computation runs in the library's
HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import torch

from . import _lib as L
from ._lib import check, lib

DTYPE_CODE = {torch.float64: L.TR_F64, torch.float32: L.TR_F32,
              torch.float16: L.TR_F16, torch.bfloat16: L.TR_BF16}
CODE_DTYPE = {v: k for k, v in DTYPE_CODE.items()}


def paper_strides(I):
    s, out = 1, []
    for i in I:
        out.append(s)
        s *= int(i)
    return out


def make_desc(I, R, core_dtype=torch.float32, x_dtype=None, x_strides=None) -> L.tr_desc:
    """Descriptor of an order-N ring: sizes I, ranks R (core k is
    R[k] x I[k] x R[(k+1) % N]); X strides default to paper order."""
    N = len(I)
    d = L.tr_desc()
    d.N = N
    for k in range(N):
        d.I[k] = int(I[k])
        d.R[k] = int(R[k])
    strides = paper_strides(I) if x_strides is None else x_strides
    for k in range(N):
        d.x_stride[k] = int(strides[k])
    d.core_dtype = DTYPE_CODE[core_dtype]
    d.x_dtype = DTYPE_CODE[x_dtype if x_dtype is not None else core_dtype]
    return d


def rr(desc, n):
    return desc.R[n] * desc.R[(n + 1) % desc.N]


def J(desc, n):
    out = 1
    for k in range(desc.N):
        if k != n:
            out *= desc.I[k]
    return out


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _p(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _parr(ts):
    arr = (C.c_void_p * L.TR_MAX_ORDER)()
    for k, t in enumerate(ts):
        arr[k] = t.data_ptr() if t is not None else None
    return arr


def workspace(nbytes: int, device="cuda") -> torch.Tensor:
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


def step_rule(kind="fixed", alpha=1e-3, tau=1000.0, eta=1e-2, b=0.0, eps=0.0) -> L.tr_step:
    s = L.tr_step()
    s.kind = {"fixed": 0, "adagrad": 1, "robbins-monro": 2}[kind]
    s.alpha, s.tau, s.eta, s.b, s.eps = alpha, tau, eta, b, eps
    return s


def tr_mode(seed: int, step: int, N: int) -> int:
    return lib().tr_mode(seed, step, N)


def tr_sample(desc, seed, step, n, m, cdf=None, cdf_J=None, stream_tag=L.TR_STREAM_IDX,
              idx=None, pF=None, device="cuda"):
    if idx is None:
        idx = torch.empty((m, desc.N), dtype=torch.int32, device=device)
    if pF is None:
        pF = torch.empty(m, dtype=torch.float64, device=device)
    carr = None
    if cdf is not None:
        carr = C.cast(_parr(cdf), L.PVP)
    check("tr_sample", lib().tr_sample(C.byref(desc), seed, step, n, m, carr, _p(cdf_J), stream_tag,
                                       _p(idx), _p(pF), _stream()))
    return idx, pF


def tr_subchain(desc, n, cores, idx, m, S=None):
    if S is None:
        S = torch.empty((m, rr(desc, n)), dtype=CODE_DTYPE[desc.core_dtype], device=idx.device)
    check("tr_subchain", lib().tr_subchain(C.byref(desc), n, C.cast(_parr(cores), L.PVP), _p(idx), m,
                                           _p(S), _stream()))
    return S


def tr_grad(desc, n, core_n, X, idx, S, pF, m, prec, g=None, loss=None, gram=None, want_gram=False,
            ws=None):
    dev = core_n.device
    if g is None:
        g = torch.empty((desc.I[n], rr(desc, n)), dtype=core_n.dtype, device=dev)
    if loss is None:
        loss = torch.zeros((), dtype=torch.float64, device=dev)
    if want_gram and gram is None:
        gram = torch.empty((rr(desc, n), rr(desc, n)), dtype=torch.float64, device=dev)
    need = lib().tr_grad_workspace_size(C.byref(desc), m, prec)
    if ws is None:
        ws = workspace(need, dev)
    check("tr_grad", lib().tr_grad(C.byref(desc), n, _p(core_n), _p(X), _p(idx), _p(S), _p(pF), m, prec,
                                   _p(g), _p(loss), _p(gram), _p(ws), ws.numel(), _stream()))
    return g, loss, gram


def tr_gram(desc, n, S_H, pH, m_H, gram=None):
    dev = S_H.device
    if gram is None:
        gram = torch.empty((rr(desc, n), rr(desc, n)), dtype=torch.float64, device=dev)
    ws = workspace(lib().tr_gram_workspace_size(C.byref(desc), m_H), dev)
    check("tr_gram", lib().tr_gram(C.byref(desc), n, _p(S_H), _p(pH), m_H, _p(gram), _p(ws), ws.numel(),
                                   _stream()))
    return gram


def tr_update(desc, n, core_n, g, gram=None, damping=0.0, rule=None, t=0, accum=None, status=None):
    dev = core_n.device
    rule = rule if rule is not None else step_rule()
    if status is None:
        status = torch.zeros((), dtype=torch.int32, device=dev)
    ws = workspace(lib().tr_update_workspace_size(C.byref(desc), n, 1 if gram is not None else 0), dev)
    check("tr_update", lib().tr_update(C.byref(desc), n, _p(core_n), _p(g), _p(gram), float(damping),
                                       C.byref(rule), t, _p(accum), _p(status), _p(ws), ws.numel(),
                                       _stream()))
    return status


def tr_dist(desc, k, law, core_k, cdf=None, status=None):
    dev = core_k.device
    if cdf is None:
        cdf = torch.empty(desc.I[k], dtype=torch.int64, device=dev)
    if status is None:
        status = torch.zeros((), dtype=torch.int32, device=dev)
    ws = workspace(lib().tr_dist_workspace_size(C.byref(desc), k, law), dev)
    check("tr_dist", lib().tr_dist(C.byref(desc), k, law, _p(core_k), _p(cdf), _p(status), _p(ws),
                                   ws.numel(), _stream()))
    return cdf, status


def tr_dist_optimal(desc, n, cores, X, cdf_J=None, status=None):
    dev = X.device
    if cdf_J is None:
        cdf_J = torch.empty(J(desc, n), dtype=torch.int64, device=dev)
    if status is None:
        status = torch.zeros((), dtype=torch.int32, device=dev)
    ws = workspace(lib().tr_dist_optimal_workspace_size(C.byref(desc), n), dev)
    check("tr_dist_optimal", lib().tr_dist_optimal(C.byref(desc), n, C.cast(_parr(cores), L.PVP), _p(X),
                                                   _p(cdf_J), _p(status), _p(ws), ws.numel(), _stream()))
    return cdf_J, status


def tr_relerr(desc, cores, X_true, x_true_norm2=-1.0, rse=None, ws=None):
    dev = X_true.device
    if rse is None:
        rse = torch.zeros((), dtype=torch.float64, device=dev)
    if ws is None:
        ws = workspace(lib().tr_relerr_workspace_size(C.byref(desc)), dev)
    check("tr_relerr", lib().tr_relerr(C.byref(desc), C.cast(_parr(cores), L.PVP), _p(X_true),
                                       float(x_true_norm2), _p(rse), _p(ws), ws.numel(), _stream()))
    return rse


def tr_reconstruct(desc, cores, X=None):
    if X is None:
        numel = 1
        for k in range(desc.N):
            numel *= desc.I[k]
        X = torch.empty(numel, dtype=CODE_DTYPE[desc.x_dtype], device=cores[0].device)
    check("tr_reconstruct", lib().tr_reconstruct(C.byref(desc), C.cast(_parr(cores), L.PVP), _p(X),
                                                 _stream()))
    return X


def tr_x_replicate(desc, X, n, Xn=None):
    if Xn is None:
        Xn = torch.empty_like(X)
    check("tr_x_replicate", lib().tr_x_replicate(C.byref(desc), _p(X), n, _p(Xn), _stream()))
    return Xn


def tr_run(problem: L.tr_problem, config: L.tr_config, t_dev, steps, loss_out, status, ws):
    check("tr_run", lib().tr_run(C.byref(problem), C.byref(config), _p(t_dev), steps, _p(loss_out),
                                 _p(status), _p(ws), ws.numel(), _stream()))


def tr_run_ex(problem: L.tr_problem, config: L.tr_config, t_dev, steps, loss_out, status, ws, opts=None):
    """tr_run with options (an L.tr_run_opts or None)."""
    check("tr_run_ex", lib().tr_run_ex(C.byref(problem), C.byref(config), _p(t_dev), steps, _p(loss_out),
                                       _p(status), _p(ws), ws.numel(), _stream(),
                                       C.byref(opts) if opts is not None else None))


def tr_run_noalloc(problem: L.tr_problem, config: L.tr_config, t_dev, steps, loss_out, status, opts=None):
    """tr_run_ex on the library's own device scratch (no workspace)."""
    check("tr_run_noalloc", lib().tr_run_noalloc(C.byref(problem), C.byref(config), _p(t_dev), steps,
                                                 _p(loss_out), _p(status), _stream(),
                                                 C.byref(opts) if opts is not None else None))


def tr_sweep_run(problem: L.tr_problem, config: L.tr_sweep_config, t_dev, sweeps, status, ws):
    check("tr_sweep_run", lib().tr_sweep_run(C.byref(problem), C.byref(config), _p(t_dev), sweeps, _p(status),
                                             _p(ws), ws.numel(), _stream()))


def tr_sweep_workspace_size(problem, config) -> int:
    return lib().tr_sweep_workspace_size(C.byref(problem), C.byref(config))


def completion_config(B, block=False, lam=0.0, rule=None, seed=0) -> L.tr_completion_config:
    c = L.tr_completion_config()
    c.B, c.block, c.lam = int(B), int(bool(block)), float(lam)
    c.rule = rule if rule is not None else step_rule()
    c.seed = seed
    return c


def tr_completion_run(desc, cores, accum, obs_idx, obs_x, config, t_dev, steps, loss_out=None, status=None,
                      ws=None):
    dev = obs_idx.device
    if status is None:
        status = torch.zeros(1, dtype=torch.int32, device=dev)
    need = lib().tr_completion_workspace_size(C.byref(desc), C.byref(config))
    if ws is None:
        ws = workspace(need, dev)
    acc = C.cast(_parr(accum), L.PVP) if accum is not None else None
    check("tr_completion_run", lib().tr_completion_run(C.byref(desc), C.cast(_parr(cores), L.PVP), acc,
                                                       _p(obs_idx), _p(obs_x), int(obs_x.numel()), C.byref(config),
                                                       _p(t_dev), steps, _p(loss_out), _p(status), _p(ws),
                                                       ws.numel(), _stream()))
    return status


def tr_run_workspace_size(problem, config) -> int:
    return lib().tr_run_workspace_size(C.byref(problem), C.byref(config))


def tr_entry_fwd(desc, cores, idx, x, B, resid=None, loss=None, ws=None):
    dev = idx.device
    if resid is None:
        resid = torch.empty(B, dtype=torch.float32, device=dev)
    if loss is None:
        loss = torch.zeros((), dtype=torch.float64, device=dev)
    if ws is None:
        ws = workspace(lib().tr_entry_workspace_size(C.byref(desc), B), dev)
    check("tr_entry_fwd", lib().tr_entry_fwd(C.byref(desc), C.cast(_parr(cores), L.PVP), _p(idx), _p(x), B,
                                             _p(resid), _p(loss), _p(ws), ws.numel(), _stream()))
    return resid, loss


def tr_entry_bwd(desc, cores, idx, resid, B, scale=1.0, scale_dev=None, grads=None, ws=None):
    dev = idx.device
    if grads is None:
        grads = [torch.empty_like(c) for c in cores]
    if ws is None:
        ws = workspace(lib().tr_entry_workspace_size(C.byref(desc), B), dev)
    check("tr_entry_bwd", lib().tr_entry_bwd(C.byref(desc), C.cast(_parr(cores), L.PVP), _p(idx), _p(resid), B,
                                             float(scale), _p(scale_dev), C.cast(_parr(grads), L.PVP), _p(ws),
                                             ws.numel(), _stream()))
    return grads
