"""Pins of the oracle's tensor-ring algebra (Section 2 definitions) against
brute force, closed forms and invariants; no GPU needed."""
import itertools
import json
import os

import numpy as np
import pytest

import tr_inputs as ti
from oracle import brsgd, tr

SMALL = [
    (3, [3, 4, 2], [2, 3, 1]),
    (3, [2, 2, 2], [1, 1, 1]),
    (4, [3, 2, 4, 2], [2, 1, 3, 2]),
    (4, [2, 3, 2, 3], [3, 2, 2, 1]),
]


@pytest.mark.parametrize("N,I,R", SMALL)
def test_unfolding_identity_vs_trace(N, I, R):
    """X_[n] = G_{n(2)} (G^{!=n}_[2])^T against element-wise Trace (T1)."""
    cores = ti.gaussian_cores(7, N, I, R)
    Xb = tr.full_tensor_by_trace(cores)
    assert np.allclose(tr.full_tensor(cores), Xb, rtol=0, atol=1e-12)
    for n in range(N):
        Xn = tr.core_unfold2(cores[n]) @ tr.subchain_unfold2(cores, n).T
        # column order by a pure-python multi-index, independent of reshape
        for idx in itertools.product(*[range(s) for s in I]):
            j = tr.cyclic_column(idx, I, n)
            assert abs(Xn[idx[n], j] - Xb[idx]) < 1e-12
        assert np.allclose(tr.unfold_cyclic(Xb, n), Xn, atol=1e-12)


@pytest.mark.parametrize("N,I,R", SMALL)
def test_cyclic_shift_invariance(N, I, R):
    """TR(G_2..G_N, G_1)(i_2..i_N, i_1) = TR(G_1..G_N)(i_1..i_N) (T2)."""
    cores = ti.gaussian_cores(3, N, I, R)
    X = tr.full_tensor(cores)
    shifted = cores[1:] + cores[:1]
    Xs = tr.full_tensor(shifted)
    assert np.allclose(np.moveaxis(X, 0, -1), Xs, atol=1e-12)


def test_rank_one_ring_is_outer_product():
    """All ranks 1: the ring is the outer product of the N vectors."""
    cores = ti.gaussian_cores(5, 3, [4, 3, 5], 1)
    a, b, c = (cc[0, :, 0] for cc in cores)
    assert np.allclose(tr.full_tensor(cores), np.einsum("i,j,k->ijk", a, b, c), atol=1e-13)


def test_classical_unfolding_is_column_permutation():
    """X_(n) and X_[n] hold the same fibers, columns ordered differently."""
    X = ti.standard_normal(0, (3, 4, 2, 5))
    for n in range(4):
        A = tr.unfold_classical(X, n)
        for idx in itertools.product(*[range(s) for s in X.shape]):
            rest = [idx[k] for k in range(4) if k != n]
            col = tr.multi_index(rest, [X.shape[k] for k in range(4) if k != n])
            assert A[idx[n], col] == X[idx]


@pytest.mark.parametrize("N,I,R", SMALL)
def test_sampled_subchain_rows_are_rows_of_full_subchain(N, I, R):
    """SSDTP's slices-Hadamard rows = rows of the full G^{!=n}_[2] (T3)."""
    cores = ti.gaussian_cores(11, N, I, R)
    rng = np.random.default_rng(0)
    for n in range(N):
        Gs = tr.subchain_unfold2(cores, n)
        idx = np.stack([rng.integers(0, I[k], 17) for k in range(N)], 1).astype(np.int32)
        idx[:, n] = -1
        S = brsgd.subchain_rows(cores, n, idx)
        for f in range(17):
            j = tr.cyclic_column(idx[f], I, n)
            assert np.allclose(S[f], Gs[j], atol=1e-13)


def test_fiber_gather_matches_unfolding():
    X = ti.standard_normal(1, (3, 4, 2, 5))
    rng = np.random.default_rng(1)
    for n in range(4):
        idx = np.stack([rng.integers(0, X.shape[k], 9) for k in range(4)], 1).astype(np.int32)
        idx[:, n] = -1
        XF = brsgd.gather_fibers(X, n, idx)
        Xn = tr.unfold_cyclic(X, n)
        for f in range(9):
            assert np.array_equal(XF[:, f], Xn[:, tr.cyclic_column(idx[f], X.shape, n)])


def test_gauge_transform_leaves_tensor_unchanged():
    """G_n x_3 A and A^{-1} x_1 G_{n+1} give the same ring (RSE ~ 0)."""
    cores = ti.gaussian_cores(2, 3, [4, 5, 3], [2, 3, 2])
    X = tr.full_tensor(cores)
    A = np.eye(3) + 0.3 * ti.standard_normal(9, (3, 3))
    g = [c.copy() for c in cores]
    g[0] = np.einsum("ris,st->rit", g[0], A)
    g[1] = np.einsum("ts,sir->tir", np.linalg.inv(A), g[1])
    assert tr.rse(g, X) < 1e-13
    assert tr.rse(cores, X) == 0.0


def test_golden_integer_ring():
    """Hand-checkable integer ring stored under tests/golden (entries are
    Trace of products of small integer slices, exact in FP64)."""
    path = os.path.join(os.path.dirname(__file__), "golden", "integer_ring_n3.json")
    with open(path) as fh:
        gold = json.load(fh)
    cores = [np.array(c, dtype=np.float64) for c in gold["cores"]]
    X = tr.full_tensor(cores)
    assert np.array_equal(X, np.array(gold["X"], dtype=np.float64))
    for hand in gold["hand_entries"]:
        assert X[tuple(hand["index"])] == hand["value"]
    G = tr.full_gradient(cores, np.zeros_like(X), 1)
    assert np.array_equal(G, np.array(gold["grad_mode2_at_zero_X"], dtype=np.float64))
