"""The paper's comparison methods, one sweep over the N cores at a time, in
plain numpy FP64 (CPU oracle; test infrastructure only).

* ``gd_sweep`` — TR-GD (the update rule after equation ``eq:gradient``):
  every core moves along its full block gradient, all N computed from the
  same iterate.
* ``scaled_gd_sweep`` — TR-ScaledGD (equation ``eq:scaled_gd``): the block
  gradient right-multiplied by the inverse of the Hessian block factor
  (G^{!=n}_[2])^T G^{!=n}_[2] of equation ``eq:hessian``, again all N from the
  same iterate; ``damping`` adds eta I to that factor.
* ``als_sweep`` — TR-ALS (Algorithm ``alg:tr_als``): for n = 1, ..., N in
  turn, core n becomes the least-squares solution of
  G^{!=n}_[2] Z_(2)^T = X_[n]^T with the other cores at their latest values.
* ``als_sampled_sweep`` — TR-ALS-Sampled (the sampled ALS subproblem that
  follows Algorithm ``alg:tr_als``): the same sweep on the rows F_n drawn by
  Algorithm SSDTP, each sampled row and fiber weighted by 1/sqrt(|F_n| p_f)
  (the importance-sampling weights of the sampled least-squares problem;
  the paper prints the subproblem without them).
"""
from __future__ import annotations

import numpy as np

from . import brsgd, sampling, tr
from .philox import STREAM_IDX


def gd_sweep(cores, X, alpha: float):
    """G_n <- G_n - alpha grad_n f(Y^t) for every n, all from Y^t."""
    grads = [tr.full_gradient(cores, X, n) for n in range(len(cores))]
    out = []
    for c, g in zip(cores, grads):
        out.append(tr.core_fold2(tr.core_unfold2(c) - alpha * g, c.shape[0], c.shape[2]))
    return out


def scaled_gd_sweep(cores, X, alpha: float, damping: float = 0.0):
    """G_n <- G_n - alpha grad_n f(Y^t) (Gs^T Gs + damping I)^{-1} for every
    n, all from Y^t (Gs = G^{!=n}_[2] at Y^t)."""
    out = []
    for n, c in enumerate(cores):
        g = tr.full_gradient(cores, X, n)
        H = tr.full_hessian_block(cores, n)
        if damping:
            H = H + damping * np.eye(H.shape[0])
        step = np.linalg.solve(H, g.T).T            # g H^{-1} (H symmetric)
        out.append(tr.core_fold2(tr.core_unfold2(c) - alpha * step, c.shape[0], c.shape[2]))
    return out


def als_sweep(cores, X):
    """One pass of Algorithm TR-ALS over n = 1, ..., N."""
    cores = [c.copy() for c in cores]
    for n in range(len(cores)):
        Gs = tr.subchain_unfold2(cores, n)
        Z, *_ = np.linalg.lstsq(Gs, tr.unfold_cyclic(X, n).T, rcond=None)
        R = cores[n].shape
        cores[n] = tr.core_fold2(Z.T, R[0], R[2])
    return cores


def als_sampled_sweep(cores, X, m: int, dist: str, seed: int, t0: int):
    """One pass of TR-ALS-Sampled over n = 1, ..., N: block n uses the draws
    of step t0 + n (the generator of Algorithm SSDTP with mode n fixed),
    the law ``dist`` of the other cores at their latest values, and solves
    the weighted sampled least-squares problem."""
    cores = [c.copy() for c in cores]
    sizes = tr.sizes_of(cores)
    for n in range(len(cores)):
        w_modes, w_J, _ = sampling.weights_for(dist, cores, n, X)
        idx, pF = sampling.draw(seed, t0 + n, n, m, sizes, w_modes, w_J, STREAM_IDX)
        S = brsgd.subchain_rows(cores, n, idx)
        XF = brsgd.gather_fibers(X, n, idx)
        wsq = 1.0 / np.sqrt(m * pF)
        Z, *_ = np.linalg.lstsq(S * wsq[:, None], (XF * wsq[None, :]).T, rcond=None)
        R = cores[n].shape
        cores[n] = tr.core_fold2(Z.T, R[0], R[2])
    return cores
