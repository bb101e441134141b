"""Pins of the completion oracle (CPU only): the regularised gradient
against central differences of the regularised loss (exact: the loss is
quadratic in each scalar of the cores), unbiasedness over every single-entry
draw against the differences of the full-Omega loss, the draw as Lemire's
bound on numpy's Philox words, and recovery of a planted ring from 40% of
its entries."""
import numpy as np
import pytest

import tr_inputs as ti
from oracle import brsgd, completion, entry, tr
from oracle.philox import STREAM_ENTRY

SIZES, RANKS = [7, 6, 8], [2, 3, 2]


def _observed(seed, frac):
    true = ti.gaussian_cores(seed, 3, SIZES, RANKS)
    X = tr.full_tensor(true)
    rng = np.random.default_rng(seed + 7)
    mask = rng.random(X.shape) < frac
    obs_idx = np.argwhere(mask).astype(np.int32)
    return true, X, obs_idx, X[mask]


def test_regularised_gradient_is_central_difference():
    _, X, obs_idx, obs_x = _observed(1, 0.5)
    cores = ti.gaussian_cores(3, 3, SIZES, RANKS, scale=0.7)
    lam, h = 0.3, 1e-3
    g = completion.regularised_grads(cores, obs_idx[:40], obs_x[:40], lam)
    rng = np.random.default_rng(4)
    for k in range(3):
        for _ in range(6):
            pos = tuple(int(rng.integers(0, s)) for s in cores[k].shape)
            cp = [c.copy() for c in cores]
            cm = [c.copy() for c in cores]
            cp[k][pos] += h
            cm[k][pos] -= h
            fd = (completion.regularised_loss(cp, obs_idx[:40], obs_x[:40], lam)
                  - completion.regularised_loss(cm, obs_idx[:40], obs_x[:40], lam)) / (2 * h)
            assert abs(fd - g[k][pos]) < 1e-9 * max(1.0, abs(fd))


def test_single_entry_gradient_is_unbiased_for_the_full_omega_loss():
    """B = 1: averaging the drawn-entry gradient over every position of Omega
    (each drawn with probability 1/|Omega|) gives the gradient of the loss
    over all of Omega, checked by central differences of that loss."""
    _, X, obs_idx, obs_x = _observed(2, 0.3)
    cores = ti.gaussian_cores(5, 3, SIZES, RANKS, scale=0.7)
    mean = [np.zeros_like(c) for c in cores]
    for j in range(len(obs_x)):
        gj = entry.entry_grads(cores, obs_idx[j:j + 1], obs_x[j:j + 1])
        for a, b in zip(mean, gj):
            a += b / len(obs_x)
    h = 1e-3
    for k in range(3):
        pos = (1, 2, 0)
        cp = [c.copy() for c in cores]
        cm = [c.copy() for c in cores]
        cp[k][pos] += h
        cm[k][pos] -= h
        fd = (entry.entry_loss(cp, obs_idx, obs_x)[0] - entry.entry_loss(cm, obs_idx, obs_x)[0]) / (2 * h)
        assert abs(fd - mean[k][pos]) < 1e-9 * max(1.0, abs(fd))


def test_draw_is_lemire_bound_on_numpy_philox():
    """Position b of step t is floor(r |Omega| / 2^64) with r the first word
    numpy's Philox4x64 returns for counter (t, b, 0, STREAM_ENTRY) and key
    (seed, 0) (numpy advances the counter before a block: start one below)."""
    seed, t, n_obs, B = 11, 5, 1234, 9
    got = completion.draw_entries(seed, t, n_obs, B)
    for b in range(B):
        c = np.array([t - 1, b, 0, STREAM_ENTRY], dtype=np.uint64)   # word 0 is the lowest; t > 0
        r = int(np.random.Philox(counter=c, key=[seed, 0]).random_raw(1)[0])
        assert got[b] == (r * n_obs) >> 64


def test_block_step_moves_only_the_drawn_mode_as_the_full_step_would():
    """With ``block`` only core n (the step's mode) changes, and it changes
    exactly as in the step that moves every core (same draws, same rule)."""
    _, X, obs_idx, obs_x = _observed(6, 0.5)
    init = ti.gaussian_cores(9, 3, SIZES, RANKS, scale=0.6)
    outs = []
    for block in (True, False):
        st = brsgd.State([c.copy() for c in init], t=4)
        tr_ = {}
        completion.completion_step(st, obs_idx, obs_x, completion.CompletionConfig(B=32, lam=0.1, block=block,
                                                                                   alpha=0.05, seed=2), trace=tr_)
        outs.append((st.cores, tr_["modes"]))
    (cb, mb), (ca, _) = outs
    n = mb[0]
    for k in range(3):
        if k == n:
            assert np.array_equal(cb[k], ca[k])
        else:
            assert np.array_equal(cb[k], init[k])


def test_planted_completion_from_40_percent():
    """A planted 10 x 9 x 8 ring of ranks 2 from 40% of its entries: AdaGrad
    steps (eta = 0.5) on batches of 64 observed entries, every core moved
    per step, bring the error on the entries never observed below 1e-4 of
    their norm within 2500 steps."""
    sizes, ranks = [10, 9, 8], [2, 2, 2]
    X = tr.full_tensor(ti.gaussian_cores(3, 3, sizes, ranks))
    mask = np.random.default_rng(10).random(X.shape) < 0.4
    obs_idx = np.argwhere(mask).astype(np.int32)
    obs_x = X[mask]
    st = brsgd.State(ti.gaussian_cores(8, 3, sizes, ranks, scale=brsgd.init_scale(X, ranks)))
    cfg = completion.CompletionConfig(B=64, rule="adagrad", eta=0.5, seed=5)
    for _ in range(2500):
        completion.completion_step(st, obs_idx, obs_x, cfg)
    Xh = tr.full_tensor(st.cores)
    err = np.linalg.norm((Xh - X)[~mask]) / np.linalg.norm(X[~mask])
    assert err < 1e-4, err
