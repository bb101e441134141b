"""Sampled-entry loss and its gradient with respect to every core
(CPU oracle, FP64; test infrastructure only).

L = 1/(2B) * sum_b (X_hat(i^b) - x_b)^2 over a batch of B multi-indices,
X_hat(i) = Trace(G_1(i_1) ... G_N(i_N)) (tensor-ring format, Section 1).

The gradient with respect to G_{n(2)} is the block gradient of equation
``eq:gradient`` restricted to the sampled entries: with r_b the residual
and s_b the row of G^{!=n}_[2] at the fiber through i^b,
dL/dG_{n(2)}[i, :] = 1/B * sum_{b : i_n^b = i} r_b s_b.
"""
from __future__ import annotations

import numpy as np

from . import tr
from .brsgd import subchain_rows


def entry_values(cores, idx: np.ndarray) -> np.ndarray:
    """X_hat at each row of idx [B x N] by the chained slice product."""
    N = len(cores)
    T = cores[0][:, idx[:, 0], :]
    for k in range(1, N):
        T = tr.slices_hadamard(T, cores[k][:, idx[:, k], :])
    return np.einsum("aba->b", T)


def entry_loss(cores, idx: np.ndarray, x: np.ndarray):
    """(L, residuals r = X_hat - x)."""
    r = entry_values(cores, idx) - x
    return float(np.sum(r * r) / (2.0 * len(x))), r


def entry_grads(cores, idx: np.ndarray, x: np.ndarray):
    """Gradients dL/dG_k in core form (R_k, I_k, R_{k+1}) for every k."""
    B = idx.shape[0]
    _, r = entry_loss(cores, idx, x)
    out = []
    for n, core in enumerate(cores):
        S = subchain_rows(cores, n, idx)
        G2 = np.zeros((core.shape[1], S.shape[1]))
        np.add.at(G2, idx[:, n].astype(np.int64), (r / B)[:, None] * S)
        out.append(tr.core_fold2(G2, core.shape[0], core.shape[2]))
    return out
