"""TR-BRSGD and TR-ScaledBRSGD, one step at a time, in plain numpy FP64
(CPU oracle; test infrastructure only).

Each function follows one passage of the paper:

* ``subchain_rows`` — Algorithm SSDTP: start from identity slices and take
  the slices-Hadamard product with the sampled slices of the cores
  n+1, ..., N, 1, ..., n-1;
* ``gather_fibers`` — Algorithm SSDTP, last step: the sampled mode-n fibers,
  one per sample (paired indexing);
* ``stoch_grad`` — equation ``eq:S_gradient``, taken literally with the
  1/(|F_n| J_n) factor, so E[g] = grad f / J_n (the lemma on unbiasedness
  drops this J_n; step sizes are therefore stated in these units);
* ``stoch_hessian`` — equation ``eq:S_hessian`` read as 1/(|H_n| J_n),
  plus the damping term of the amended preconditioner remark;
* ``scaled_direction`` — equation ``eq:scaledsg_direction``, p = -g h^{-1};
* ``update`` — equation ``eq:update_brsgd`` (fixed or Robbins-Monro alpha)
  or the AdaGrad remark (per-core, per-entry accumulator including the
  current step, updated only when the core is chosen);
* ``step``/``run`` — Algorithm TR-BRSGD, with the scaled direction when
  ``variant == "scaled"``.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

from . import sampling, tr
from .philox import STREAM_H, STREAM_IDX

DEV_NONFINITE = 1
DEV_NOT_SPD = 2
DEV_ZERO_DIST = 4
DEV_DAMPED = 8


@dataclass
class Config:
    m: int
    dist: str = "U"            # U, L, E, O
    variant: str = "plain"     # plain | scaled
    rule: str = "fixed"        # fixed | adagrad | robbins-monro
    alpha: float = 1e-3        # fixed alpha, or alpha_0 for Robbins-Monro
    tau: float = 1000.0        # Robbins-Monro: alpha_t = alpha_0 / (1 + t/tau)
    eta: float = 1e-2          # AdaGrad eta
    b: float = 0.0
    eps: float = 0.0
    damping: float = 0.0       # eta^0 of the amended preconditioner
    damping_schedule: str = "constant"   # constant | harmonic | geometric
    damping_tau: float = 1.0   # harmonic: eta^t = eta^0 / (1 + t/tau); geometric: eta^t = eta^0 tau^t
    m_H: int | None = None     # None: H_n = F_n
    seed: int = 0


@dataclass
class State:
    cores: list
    accum: list = None
    t: int = 0
    status: int = 0

    def __post_init__(self):
        self.cores = [np.array(c, dtype=np.float64) for c in self.cores]
        if self.accum is None:
            self.accum = [np.zeros((c.shape[1], c.shape[0] * c.shape[2])) for c in self.cores]


def subchain_rows(cores, n: int, idx: np.ndarray) -> np.ndarray:
    """Sampled rows S = G^{!=n}_[2](F_n, :) (m x R_n R_{n+1}),
    S[f, r + R_n*s] = M_f[s, r], M_f = G_{n+1}(i_{n+1}) ... G_{n-1}(i_{n-1})."""
    N = len(cores)
    m = idx.shape[0]
    Rn1 = cores[(n + 1) % N].shape[0]
    T = np.repeat(np.eye(Rn1)[:, None, :], m, axis=1)       # (R_{n+1}, m, R_{n+1})
    for k in tr.cyclic_order(N, n):
        T = tr.slices_hadamard(T, cores[k][:, idx[:, k], :])
    Rn = T.shape[2]
    return T.transpose(1, 0, 2).reshape(m, Rn1 * Rn)


def gather_fibers(X: np.ndarray, n: int, idx: np.ndarray) -> np.ndarray:
    """X_[n](:, F_n) (I_n x m): fiber f is X(i_1, ..., :, ..., i_N)."""
    N = X.ndim
    Xm = np.moveaxis(X, n, 0)
    sel = tuple(idx[:, k].astype(np.int64) for k in range(N) if k != n)
    return np.asarray(Xm[(slice(None),) + sel])


def J_of(sizes, n: int) -> int:
    return int(np.prod([s for k, s in enumerate(sizes) if k != n], dtype=object))


def stoch_grad(Gn2: np.ndarray, S: np.ndarray, XF: np.ndarray, pF: np.ndarray, Jn: int):
    """g = (G S^T D S - X_F D S) / (|F| J_n), D = diag(1/p_F)
    (equation ``eq:S_gradient``); also the unbiased estimate of f,
    sum_f ||x_f - G s_f||^2 / (2 |F| p_f)."""
    m = S.shape[0]
    DS = S / pF[:, None]
    g = (Gn2 @ (S.T @ DS) - XF @ DS) / (m * float(Jn))
    E = XF - Gn2 @ S.T
    loss = float(np.sum(np.sum(E * E, axis=0) / (2.0 * m * pF)))
    return g, loss


def stoch_hessian(S_H: np.ndarray, p_H: np.ndarray, Jn: int, damping: float = 0.0):
    """h = S_H^T D S_H / (|H| J_n) + eta I (``eq:S_hessian`` and the amended
    preconditioner)."""
    mH = S_H.shape[0]
    h = S_H.T @ (S_H / p_H[:, None]) / (mH * float(Jn))
    if damping:
        h = h + damping * np.eye(h.shape[0])
    return h


def scaled_direction(g: np.ndarray, h: np.ndarray):
    """p = -g h^{-1} by Cholesky; if h is not positive definite, retry with
    eta = 10^(k-10) tr(h)/RR for k = 0..6.  Returns (p, status bits)."""
    RR = h.shape[0]
    try:
        c = scipy.linalg.cho_factor(h, lower=True, check_finite=True)
        return -scipy.linalg.cho_solve(c, g.T).T, 0
    except (np.linalg.LinAlgError, ValueError):
        pass
    base = float(np.trace(h)) / RR
    for k in range(7):
        eta = 10.0 ** (k - 10) * base
        try:
            c = scipy.linalg.cho_factor(h + eta * np.eye(RR), lower=True)
            return -scipy.linalg.cho_solve(c, g.T).T, DEV_DAMPED
        except (np.linalg.LinAlgError, ValueError):
            continue
    return np.zeros_like(g), DEV_NOT_SPD


def damping_at(cfg: Config, t: int) -> float:
    """eta^t of the amended preconditioner (the remark after
    ``eq:scaledsg_direction``: a damping specific to iteration t, >= 0).
    The paper fixes no schedule; besides a constant, a harmonic decay
    eta^0 / (1 + t/tau) and a geometric decay eta^0 tau^t (0 < tau <= 1)."""
    if cfg.damping_schedule == "harmonic":
        return cfg.damping / (1.0 + t / cfg.damping_tau)
    if cfg.damping_schedule == "geometric":
        return cfg.damping * cfg.damping_tau ** t
    return cfg.damping


def update(Gn2: np.ndarray, p: np.ndarray, cfg: Config, t: int, accum: np.ndarray | None):
    """New G_{n(2)} (and AdaGrad accumulator) from the direction p."""
    if cfg.rule == "adagrad":
        A = accum + p * p
        base = cfg.b + A
        denom = np.power(base, 0.5 + cfg.eps, where=base > 0, out=np.ones_like(base))
        stepm = np.where(base > 0, cfg.eta / denom, 0.0)
        return Gn2 + stepm * p, A
    if cfg.rule == "robbins-monro":
        a = cfg.alpha / (1.0 + t / cfg.tau)
    else:
        a = cfg.alpha
    return Gn2 + a * p, accum


def step(state: State, X: np.ndarray, cfg: Config, n: int | None = None, trace: dict | None = None):
    """One iteration of Algorithm TR-BRSGD (plain or scaled direction)."""
    cores = state.cores
    N = len(cores)
    sizes = tr.sizes_of(cores)
    if n is None:
        n = sampling.pick_mode(cfg.seed, state.t, N)
    w_modes, w_J, zero = sampling.weights_for(cfg.dist, cores, n, X)
    if zero:
        state.status |= DEV_ZERO_DIST
    idx, pF = sampling.draw(cfg.seed, state.t, n, cfg.m, sizes, w_modes, w_J, STREAM_IDX)
    S = subchain_rows(cores, n, idx)
    XF = gather_fibers(X, n, idx)
    Jn = J_of(sizes, n)
    Gn2 = tr.core_unfold2(cores[n])
    g, loss = stoch_grad(Gn2, S, XF, pF, Jn)
    h = None
    if cfg.variant == "scaled":
        if cfg.m_H is None:
            S_H, p_H = S, pF
        else:
            idx_H, p_H = sampling.draw(cfg.seed, state.t, n, cfg.m_H, sizes, w_modes, w_J, STREAM_H)
            S_H = subchain_rows(cores, n, idx_H)
        h = stoch_hessian(S_H, p_H, Jn, damping_at(cfg, state.t))
        p, st = scaled_direction(g, h)
        state.status |= st
    else:
        p = -g
    new, acc = update(Gn2, p, cfg, state.t, state.accum[n])
    if not np.all(np.isfinite(new)):
        state.status |= DEV_NONFINITE
    R = cores[n].shape
    cores[n] = tr.core_fold2(new, R[0], R[2])
    state.accum[n] = acc
    if trace is not None:
        trace.update(n=n, idx=idx, pF=pF, S=S, XF=XF, g=g, loss=loss, h=h, p=p,
                     w_modes=w_modes, w_J=w_J)
    state.t += 1
    return n


def run(state: State, X: np.ndarray, cfg: Config, steps: int, X_true=None,
        rse_every: int = 0, tol: float = 0.0):
    """Steps until ``steps`` are done or the RSE (checked every ``rse_every``
    steps) reaches ``tol``; returns [(t, rse), ...]."""
    hist = []
    ref = X if X_true is None else X_true
    for _ in range(steps):
        step(state, X, cfg)
        if rse_every and state.t % rse_every == 0:
            e = tr.rse(state.cores, ref)
            hist.append((state.t, e))
            if e <= tol:
                break
    return hist


def init_scale(X: np.ndarray, ranks) -> float:
    """sigma with E[X(i)^2] = sigma^(2N) prod R_k for i.i.d. N(0, sigma^2)
    cores, matched to mean(X^2) (random initialisation)."""
    N = len(ranks)
    ms = float(np.mean(X * X))
    return (ms / float(np.prod(ranks))) ** (1.0 / (2 * N))


def add_noise(X_true: np.ndarray, E: np.ndarray, snr_db: float) -> np.ndarray:
    """X = X_true + sigma E with sigma = 10^(-SNR/20) ||X_true||_F / sqrt(#X)."""
    sig = 10.0 ** (-snr_db / 20.0) * np.linalg.norm(X_true) / np.sqrt(X_true.size)
    return X_true + sig * E
