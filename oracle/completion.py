"""Tensor completion in the ring format with a ridge regulariser, on the
sampled-entry loss (CPU oracle, FP64; test infrastructure only).

The concluding remarks name tensor completion and regularised problems as
uses of the doubly randomized framework.  Given observed entries (Omega: a
list of multi-indices with values), one step

* draws B observed entries uniformly with replacement: entry j of Omega
  with j = floor(r |Omega| / 2^64), r the Philox word of counter
  (t, b, 0, STREAM_ENTRY) under key (seed, 0);
* evaluates L = 1/(2B) sum_b r_b^2 + lambda/2 sum_k ||G_k||_F^2, r_b the
  residual Trace(G_1(i_1^b) ... G_N(i_N^b)) - x_b (tensor-ring format,
  Section 1);
* moves along p_k = -dL/dG_k with the step rule of ``brsgd.update``: every
  core, or with ``block`` only core n = the step's mode (the block choice of
  Algorithm TR-BRSGD).

dL/dG_k is the block gradient of ``eq:gradient`` restricted to the drawn
entries (``entry.entry_grads``) plus lambda G_k.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

from . import brsgd, entry, sampling, tr
from .philox import STREAM_ENTRY, draw_word, mulhi_np


@dataclass
class CompletionConfig:
    B: int
    lam: float = 0.0
    block: bool = False
    rule: str = "fixed"
    alpha: float = 1e-2
    tau: float = 1000.0
    eta: float = 1e-2
    b: float = 0.0
    eps: float = 0.0
    seed: int = 0

    def rule_config(self) -> brsgd.Config:
        return brsgd.Config(m=1, rule=self.rule, alpha=self.alpha, tau=self.tau, eta=self.eta, b=self.b,
                            eps=self.eps, seed=self.seed)


def draw_entries(seed: int, t: int, n_obs: int, B: int) -> np.ndarray:
    """Positions in Omega of the B entries drawn at step t."""
    r = draw_word(seed, t, np.arange(B, dtype=np.uint64), 0, STREAM_ENTRY)
    return mulhi_np(r, n_obs).astype(np.int64)


def regularised_loss(cores, idx, x, lam: float) -> float:
    L, _ = entry.entry_loss(cores, idx, x)
    return L + 0.5 * lam * sum(float(np.sum(c * c)) for c in cores)


def regularised_grads(cores, idx, x, lam: float):
    """dL/dG_k in core form for every k."""
    return [g + lam * c for g, c in zip(entry.entry_grads(cores, idx, x), cores)]


def completion_step(state: brsgd.State, obs_idx: np.ndarray, obs_x: np.ndarray, cfg: CompletionConfig,
                    trace: dict | None = None):
    """One step; returns the loss of the drawn batch before the update."""
    cores = state.cores
    N = len(cores)
    j = draw_entries(cfg.seed, state.t, len(obs_x), cfg.B)
    idx, x = obs_idx[j], obs_x[j]
    loss = regularised_loss(cores, idx, x, cfg.lam)
    grads = regularised_grads(cores, idx, x, cfg.lam)
    modes = [sampling.pick_mode(cfg.seed, state.t, N)] if cfg.block else list(range(N))
    rc = cfg.rule_config()
    for k in modes:
        G2 = tr.core_unfold2(cores[k])
        new, acc = brsgd.update(G2, -tr.core_unfold2(grads[k]), rc, state.t, state.accum[k])
        cores[k] = tr.core_fold2(new, cores[k].shape[0], cores[k].shape[2])
        state.accum[k] = acc
    if trace is not None:
        trace.update(j=j, loss=loss, grads=grads, modes=modes)
    state.t += 1
    return loss
