"""Mode pick, the four sampling distributions and the fiber sampler
(CPU oracle, FP64; test infrastructure only).

Section 3.2 gives four laws for the mini-batch of mode-n fibers:

* uniform:   q = 1/J_n over all columns of X_[n];
* leverage:  p_k(i) = l_i(G_{k(2)}) / rank(G_{k(2)}) per core (Lemma
  "lev_est"), l_i the squared row norms of an orthonormal basis of the
  column space (Definition "Leverage Scores");
* Euclidean: p_k(i) = ||G_k(:, i, :)||_F^2 / ||G_k||_F^2 per core (Lemma
  "euc_est");
* optimal:   q(j) proportional to ||R_[n](:, j)||_2 * ||G^{!=n}_[2](j, :)||_2
  with R_[n] the full residual (equation ``eq:optimal_prob``).

For the three product laws, sampling a row of G^{!=n}_[2] is sampling one
slice index per core independently (end of Section 3.2); Algorithm SSDTP
draws them with replacement in the order n+1, ..., N, 1, ..., n-1 and
multiplies their probabilities into p_F in that order.

Readings where the paper is silent:

* every draw is a 64-bit word of Philox4x64-10, key (seed, 0), counter
  (step, sample, mode, stream); the mode of step t uses counter
  (t, 0, 0, STREAM_MODE) and is independent of the data;
* bounded draws are Lemire's floor(r * n / 2^64);
* a non-uniform law is turned into integer weights w_i = floor(p_i 2^40) + 1
  and sampled through their inclusive prefix sums C: u = floor(r W / 2^64),
  pick the first i with C_i > u; the probability used in D is w_i / W, the
  law actually sampled, so the estimate stays unbiased for it;
* a uniform mode contributes 1/I_k to p_F;
* the optimal law is not a product: j is drawn directly over [J_n]
  (counter slot k = n) and decoded into the multi-index by the cyclic order.
"""
from __future__ import annotations

import numpy as np

from . import tr
from .philox import STREAM_IDX, STREAM_MODE, draw_word, mulhi_np

QBITS = 40
TWO_Q = float(1 << QBITS)


def pick_mode(seed: int, t: int, N: int) -> int:
    """Mode of step t, uniform over the N modes (Algorithm TR-BRSGD)."""
    r = draw_word(seed, t, 0, 0, STREAM_MODE)
    return int(mulhi_np(r, N))


# ---------------------------------------------------------------- laws ----

def dist_uniform(I: int) -> np.ndarray:
    return np.full(I, 1.0 / I)


def dist_euclid(core: np.ndarray):
    """p(i) = ||G_k(:, i, :)||_F^2 / ||G_k||_F^2; (None, True) if the core is 0."""
    row = np.sum(core * core, axis=(0, 2))
    tot = float(np.sum(row))
    if not tot > 0.0:
        return None, True
    return row / tot, False


def dist_leverage(core: np.ndarray) -> np.ndarray:
    """p(i) = l_i(G_{k(2)}) / rank(G_{k(2)}); rank by numpy's default tolerance."""
    G2 = tr.core_unfold2(core)
    U, s, _ = np.linalg.svd(G2, full_matrices=False)
    rank = int(np.linalg.matrix_rank(G2))
    if rank == 0:
        return np.full(G2.shape[0], 1.0 / G2.shape[0])
    lev = np.sum(U[:, :rank] ** 2, axis=1)
    return lev / rank


def dist_optimal(cores, X: np.ndarray, n: int):
    """q over the J_n columns of X_[n] (equation ``eq:optimal_prob``),
    unsquared norms, at the current cores; (None, True) if every term is 0."""
    Gs = tr.subchain_unfold2(cores, n)
    Gn = tr.core_unfold2(cores[n])
    Rn = Gn @ Gs.T - tr.unfold_cyclic(X, n)
    a = np.linalg.norm(Rn, axis=0) * np.linalg.norm(Gs, axis=1)
    tot = float(np.sum(a))
    if not tot > 0.0:
        return None, True
    return a / tot, False


def quantize(p: np.ndarray) -> np.ndarray:
    """Integer weights w_i = floor(p_i * 2^40) + 1 (uint64)."""
    return (np.floor(np.asarray(p, dtype=np.float64) * TWO_Q)).astype(np.uint64) + np.uint64(1)


def weights_for(dist: str, cores, n: int, X=None):
    """Per-mode integer weights (None for uniform modes) and, for the optimal
    law, the weights over J_n.  Returns (w_modes, w_J, zero_flag)."""
    N = len(cores)
    w = [None] * N
    if dist == "U":
        return w, None, False
    if dist == "O":
        q, zero = dist_optimal(cores, X, n)
        if zero:
            return w, None, True
        return w, quantize(q), False
    zero_any = False
    for k in range(N):
        if k == n:
            continue
        if dist == "E":
            p, zero = dist_euclid(cores[k])
            zero_any |= zero
            w[k] = None if zero else quantize(p)
        elif dist == "L":
            w[k] = quantize(dist_leverage(cores[k]))
        else:
            raise ValueError(dist)
    return w, None, zero_any


# -------------------------------------------------------------- sampler ---

def _cdf_pick(r: np.ndarray, w: np.ndarray):
    C = np.cumsum(w.astype(np.uint64), dtype=np.uint64)
    W = C[-1]
    if int(W) >= (1 << 53):
        raise ValueError("weight total must stay below 2^53")
    u = mulhi_np(r, W)
    i = np.searchsorted(C, u, side="right")
    p = w[i].astype(np.float64) / float(W)
    return i, p


def draw(seed: int, t: int, n: int, m: int, sizes, w_modes=None, w_J=None,
         stream: int = STREAM_IDX):
    """Algorithm SSDTP's index draw: idx [m x N] int32 (column n = -1) and
    p_F [m] float64."""
    N = len(sizes)
    idx = np.full((m, N), -1, dtype=np.int32)
    pF = np.ones(m, dtype=np.float64)
    f = np.arange(m, dtype=np.uint64)
    order = tr.cyclic_order(N, n)
    if w_J is not None:
        r = draw_word(seed, t, f, n, stream)
        j, p = _cdf_pick(r, np.asarray(w_J, dtype=np.uint64))
        rem = j.astype(np.int64)
        for k in order:
            idx[:, k] = (rem % sizes[k]).astype(np.int32)
            rem //= sizes[k]
        return idx, p
    for k in order:
        r = draw_word(seed, t, f, k, stream)
        wk = None if w_modes is None else w_modes[k]
        if wk is None:
            i = mulhi_np(r, sizes[k]).astype(np.int64)
            p = np.full(m, 1.0 / sizes[k])
        else:
            i, p = _cdf_pick(r, np.asarray(wk, dtype=np.uint64))
        idx[:, k] = i.astype(np.int32)
        pF = pF * p
    return idx, pF


def law_of(w_modes, sizes, n):
    """Probability vector over the J_n columns of X_[n] implied by per-mode
    weights (product law; uniform where weights are None)."""
    N = len(sizes)
    order = tr.cyclic_order(N, n)
    q = np.ones(1)
    for k in order:
        wk = w_modes[k] if w_modes is not None else None
        pk = (np.full(sizes[k], 1.0 / sizes[k]) if wk is None
              else wk.astype(np.float64) / float(np.sum(wk.astype(np.uint64))))
        q = np.outer(pk, q).ravel()   # earlier modes fastest
    return q
