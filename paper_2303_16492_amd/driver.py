"""Problem object around ``tr_run``: device buffers for one decomposition
(cores, AdaGrad state, X and its mode-major replicas, CDF buffers, step
counter, status word, workspace) and the calls that advance it.

Algorithm TR-BRSGD / TR-ScaledBRSGD runs entirely in the library: the
object only owns memory and fills the C structs.  ``capture`` records K
steps in a HIP graph (torch.cuda.CUDAGraph on ROCm); replays advance the
device step counter, so successive replays continue the same trajectory.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from . import api

PREC = {"f64": L.TR_PREC_F64, "f32": L.TR_PREC_F32, "bf16": L.TR_PREC_BF16, "f16": L.TR_PREC_F16}
LAW = {"U": L.TR_LAW_UNIFORM, "L": L.TR_LAW_LEVERAGE, "E": L.TR_LAW_EUCLID, "O": L.TR_LAW_OPTIMAL}


def core_to_unfold(core3: np.ndarray) -> np.ndarray:
    """(R_k, I_k, R_{k+1}) array -> G_{k(2)} (I_k, R_k R_{k+1}), column r + R_k s."""
    Rk, Ik, Rk1 = core3.shape
    return np.ascontiguousarray(np.transpose(core3, (1, 2, 0)).reshape(Ik, Rk * Rk1))


def unfold_to_core(G2: np.ndarray, Rk: int, Rk1: int) -> np.ndarray:
    Ik = G2.shape[0]
    return np.ascontiguousarray(G2.reshape(Ik, Rk1, Rk).transpose(2, 0, 1))


def cores_to_device(cores3, dtype=torch.float32, device="cuda"):
    return [torch.from_numpy(core_to_unfold(np.asarray(c))).to(device=device, dtype=dtype) for c in cores3]


def cores_to_host(cores2, R):
    N = len(cores2)
    return [unfold_to_core(c.double().cpu().numpy(), R[k], R[(k + 1) % N]) for k, c in enumerate(cores2)]


class TRSolver:
    def __init__(self, cores, X, I, R, m, law="U", scaled=False, prec="f32", rule=None,
                 damping=0.0, m_H=0, seed=0, replicas=True, overlap=True):
        self.I, self.R = list(I), list(R)
        self.N = len(I)
        self.cores = cores
        self.X = X
        dev = X.device
        self.desc = api.make_desc(I, R, cores[0].dtype, X.dtype)
        self.rule = rule if rule is not None else api.step_rule()
        self.accum = ([torch.zeros_like(c) for c in cores] if self.rule.kind == 1 else [None] * self.N)
        self.reps = ([api.tr_x_replicate(self.desc, X, n) for n in range(self.N)] if replicas
                     else [None] * self.N)
        self.cdf = [None] * self.N
        self.cdf_J = None
        if law in ("L", "E"):
            self.cdf = [torch.empty(i, dtype=torch.int64, device=dev) for i in I]
        if law == "O":
            self.cdf_J = torch.empty(max(api.J(self.desc, n) for n in range(self.N)), dtype=torch.int64,
                                     device=dev)
        self.t_dev = torch.zeros(1, dtype=torch.int64, device=dev)
        self.status = torch.zeros(1, dtype=torch.int32, device=dev)
        p = L.tr_problem()
        p.desc = self.desc
        for k in range(self.N):
            p.cores[k] = cores[k].data_ptr()
            p.accum[k] = self.accum[k].data_ptr() if self.accum[k] is not None else None
            p.Xrep[k] = self.reps[k].data_ptr() if self.reps[k] is not None else None
            p.cdf[k] = self.cdf[k].data_ptr() if self.cdf[k] is not None else None
        p.X = X.data_ptr()
        p.cdf_J = self.cdf_J.data_ptr() if self.cdf_J is not None else None
        self.problem = p
        c = L.tr_config()
        c.m, c.m_H, c.law, c.scaled, c.prec = m, m_H, LAW[law], int(scaled), PREC[prec]
        c.damping, c.rule, c.seed = float(damping), self.rule, seed
        self.config = c
        self.ws = api.workspace(api.tr_run_workspace_size(p, c), dev)
        self.rse_ws = None
        # scaled steps: the Gram/inverse branch on a second stream (RR <= 128)
        self.opts = None
        if overlap and scaled:
            self.aux = torch.cuda.Stream(device=dev)
            self.events = [L.HipEvent(timing=False) for _ in range(3)]
            o = L.tr_run_opts()
            o.aux = self.aux.cuda_stream
            o.ev_fork, o.ev_gram, o.ev_join = (e.handle.value for e in self.events)
            self.opts = o

    def run(self, steps: int, loss_out=None):
        api.tr_run_ex(self.problem, self.config, self.t_dev, steps, loss_out, self.status, self.ws, self.opts)

    def capture(self, steps: int):
        """HIP graph of ``steps`` iterations (replay with graph.replay())."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run(1)            # warm-up outside capture; advances t once
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            self.run(steps)
        return g

    def rse(self, X_true=None, x_norm2=-1.0):
        Xt = self.X if X_true is None else X_true
        if self.rse_ws is None:
            self.rse_ws = api.workspace(L.lib().tr_relerr_workspace_size(C.byref(self.desc)), Xt.device)
        return api.tr_relerr(self.desc, self.cores, Xt, x_norm2, ws=self.rse_ws)

    @property
    def t(self) -> int:
        return int(self.t_dev.item())
