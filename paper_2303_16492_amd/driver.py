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
    SCHEDULE = {"constant": 0, "harmonic": 1, "geometric": 2}

    def __init__(self, cores, X, I, R, m, law="U", scaled=False, prec="f32", rule=None,
                 damping=0.0, m_H=0, seed=0, replicas=True, overlap=True, damping_schedule="constant",
                 damping_tau=1.0):
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
        c.damping_schedule, c.damping_tau = self.SCHEDULE[damping_schedule], float(damping_tau)
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

    def capture(self, steps: int, loss_out=None):
        """HIP graph of ``steps`` iterations (replay with graph.replay());
        with ``loss_out`` (``steps`` float64 on the device) every replay
        writes each step's loss estimate there."""
        g = torch.cuda.CUDAGraph()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(s):
            self.run(1)            # warm-up outside capture; advances t once
        torch.cuda.current_stream().wait_stream(s)
        torch.cuda.synchronize()
        with torch.cuda.graph(g):
            self.run(steps, loss_out)
        return g

    def rse(self, X_true=None, x_norm2=-1.0):
        Xt = self.X if X_true is None else X_true
        if self.rse_ws is None:
            self.rse_ws = api.workspace(L.lib().tr_relerr_workspace_size(C.byref(self.desc)), Xt.device)
        return api.tr_relerr(self.desc, self.cores, Xt, x_norm2, ws=self.rse_ws)

    @property
    def t(self) -> int:
        return int(self.t_dev.item())


METHOD = {"gd": L.TR_METHOD_GD, "scaled-gd": L.TR_METHOD_SCALED_GD, "als": L.TR_METHOD_ALS,
          "als-sampled": L.TR_METHOD_ALS_SAMPLED}


class TRSweeper(TRSolver):
    """The paper's comparison methods (TR-GD, TR-ScaledGD, TR-ALS,
    TR-ALS-Sampled) on the same problem buffers, advanced by whole sweeps
    through ``tr_sweep_run``."""

    def __init__(self, cores, X, I, R, method="als", m=0, law="U", prec="f32", alpha=1.0, damping=0.0, seed=0,
                 replicas=True):
        super().__init__(cores, X, I, R, max(m, 1), law=law, scaled=False, prec=prec, seed=seed, replicas=replicas,
                         overlap=False)
        sc = L.tr_sweep_config()
        sc.method, sc.m, sc.law, sc.prec = METHOD[method], m, LAW[law], PREC[prec]
        sc.alpha, sc.damping, sc.seed = alpha, damping, seed
        self.sweep_config = sc
        need = api.tr_sweep_workspace_size(self.problem, sc)
        if need == 0:
            raise ValueError("invalid sweep configuration")
        self.sweep_ws = api.workspace(need, X.device)

    def sweep(self, sweeps: int = 1):
        api.tr_sweep_run(self.problem, self.sweep_config, self.t_dev, sweeps, self.status, self.sweep_ws)


class TRBatch:
    """Many independent problems advanced together by ``tr_batch_run``.

    problems: list of dicts with keys cores (list of FP32 device G_{k(2)}),
    Xrep (list of FP16 mode-major replicas), I, R, m, rule (L.tr_step),
    seed.  The object owns the device table, the per-problem step counters,
    loss estimates and status words."""

    VARIANTS = ((32, 4), (32, 8), (64, 4), (64, 8))
    SPLITS = (1, 4, 8, 16)

    def __init__(self, problems, device="cuda"):
        self.count = len(problems)
        self.problems = problems
        self.t_dev = torch.zeros(self.count, dtype=torch.int64, device=device)
        self.loss = torch.zeros(self.count, dtype=torch.float64, device=device)
        self.status = torch.zeros(self.count, dtype=torch.int32, device=device)
        self.accum = []
        items = (L.tr_batch_item * self.count)()
        for p, pr in enumerate(problems):
            N = len(pr["I"])
            it = items[p]
            it.desc = api.make_desc(pr["I"], pr["R"], torch.float32, torch.float16)
            rule = pr["rule"]
            acc = [torch.zeros_like(c) for c in pr["cores"]] if rule.kind == 1 else [None] * N
            self.accum.append(acc)
            for k in range(N):
                it.cores[k] = pr["cores"][k].data_ptr()
                it.accum[k] = acc[k].data_ptr() if acc[k] is not None else None
                it.Xrep[k] = pr["Xrep"][k].data_ptr()
            it.t_dev = self.t_dev.data_ptr() + 8 * p
            it.loss = self.loss.data_ptr() + 8 * p
            it.dev_status = self.status.data_ptr() + 4 * p
            it.m, it.rule, it.seed = pr["m"], rule, pr["seed"]
        self.items = items
        self.table = api.workspace(L.lib().tr_batch_table_size(self.count), device)
        api.check("tr_batch_upload", L.lib().tr_batch_upload(items, self.count, C.c_void_p(self.table.data_ptr()),
                                                             self.table.numel(), api._stream()))
        self.chunk, self.waves, self.splits = 64, 4, 1
        self.split_ws = {}

    def run(self, steps: int, chunk=None, waves=None, splits=None):
        """``steps`` steps of every problem; splits > 1 spreads each problem's
        samples over that many workgroups (two launches per step)."""
        chunk, waves = chunk or self.chunk, waves or self.waves
        splits = splits or self.splits
        if splits == 1:
            api.check("tr_batch_run", L.lib().tr_batch_run(C.c_void_p(self.table.data_ptr()), self.count, steps,
                                                           chunk, waves, api._stream()))
            return
        if splits not in self.split_ws:
            self.split_ws[splits] = api.workspace(L.lib().tr_batch_split_workspace_size(self.count, splits),
                                                  self.table.device)
        ws = self.split_ws[splits]
        api.check("tr_batch_run_split", L.lib().tr_batch_run_split(
            C.c_void_p(self.table.data_ptr()), self.count, steps, chunk, waves, splits, C.c_void_p(ws.data_ptr()),
            ws.numel(), api._stream()))

    def _state(self):
        cores = [[c.clone() for c in pr["cores"]] for pr in self.problems]
        acc = [[a.clone() if a is not None else None for a in aa] for aa in self.accum]
        return cores, acc, self.t_dev.clone(), self.loss.clone(), self.status.clone()

    def _restore(self, st):
        cores, acc, t, loss, status = st
        for pr, cs in zip(self.problems, cores):
            for c, s in zip(pr["cores"], cs):
                c.copy_(s)
        for aa, ss in zip(self.accum, acc):
            for a, s in zip(aa, ss):
                if a is not None:
                    a.copy_(s)
        self.t_dev.copy_(t)
        self.loss.copy_(loss)
        self.status.copy_(status)

    def tune(self, steps: int = 3, reps: int = 2):
        """Time every (chunk, waves, splits) variant on this batch and keep
        the fastest; the problems' state is restored afterwards.  Returns
        {variant: ms per step}."""
        saved = self._state()
        times = {}
        for sp in self.SPLITS:
            for ch, wv in self.VARIANTS:
                self.run(1, ch, wv, sp)                  # warm-up (module load, caches)
                torch.cuda.synchronize()
                best = float("inf")
                for _ in range(reps):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record()
                    self.run(steps, ch, wv, sp)
                    b.record()
                    torch.cuda.synchronize()
                    best = min(best, a.elapsed_time(b) / steps)
                times[(ch, wv, sp)] = best
        self._restore(saved)
        torch.cuda.synchronize()
        self.chunk, self.waves, self.splits = min(times, key=times.get)
        return times
