"""Pins of the four sampling laws (Section 3.2): closed forms, an independent
QR route to the leverage scores, the special case I_k <= R_k R_{k+1}, and the
two estimate lemmas checked by brute force on the full subchain."""
import numpy as np
import pytest

import tr_inputs as ti
from oracle import sampling, tr


def test_euclid_closed_form_and_zero_core():
    core = ti.standard_normal(0, (3, 7, 2))
    p, zero = sampling.dist_euclid(core)
    assert not zero
    want = np.array([sum(core[r, i, s] ** 2 for r in range(3) for s in range(2)) for i in range(7)])
    assert np.allclose(p, want / want.sum(), rtol=1e-14)
    assert abs(p.sum() - 1) < 1e-15
    p, zero = sampling.dist_euclid(np.zeros((2, 4, 2)))
    assert zero and p is None


def test_leverage_matches_qr_route():
    """Full column rank: l_i = ||Q(i,:)||^2 from a QR factorisation, an
    independent routine from the oracle's SVD."""
    core = ti.standard_normal(1, (2, 11, 3))
    p = sampling.dist_leverage(core)
    Q, _ = np.linalg.qr(tr.core_unfold2(core))
    want = np.sum(Q * Q, axis=1) / 6
    assert np.allclose(p, want, rtol=1e-12)
    assert abs(p.sum() - 1) < 1e-14


def test_leverage_is_uniform_when_rows_do_not_exceed_columns():
    core = ti.standard_normal(2, (3, 8, 4))        # I = 8 <= RR = 12, full row rank
    p = sampling.dist_leverage(core)
    assert np.allclose(p, np.full(8, 1 / 8), rtol=1e-12)


def test_leverage_rank_deficient():
    core = ti.standard_normal(3, (2, 9, 2))
    G2 = tr.core_unfold2(core)
    G2[:, 3] = G2[:, 0] + G2[:, 1]                 # rank 3
    core = tr.core_fold2(G2, 2, 2)
    p = sampling.dist_leverage(core)
    Q, _ = np.linalg.qr(G2[:, :3])
    assert np.allclose(p, np.sum(Q * Q, axis=1) / 3, rtol=1e-10)


@pytest.mark.parametrize("n", [0, 1, 2, 3])
def test_leverage_estimate_lemma(n):
    """q^{!=n}(i) >= beta_n p^{!=n}(i), exact leverage of G^{!=n}_[2] by SVD
    (lemma lev_est)."""
    sizes, ranks = [5, 4, 6, 5], [2, 2, 1, 2]
    cores = ti.gaussian_cores(4, 4, sizes, ranks)
    w = [None if k == n else sampling.dist_leverage(cores[k]) for k in range(4)]
    q = np.ones(1)
    for k in tr.cyclic_order(4, n):
        q = np.outer(w[k], q).ravel()
    Gs = tr.subchain_unfold2(cores, n)
    U, s, _ = np.linalg.svd(Gs, full_matrices=False)
    rk = np.linalg.matrix_rank(Gs)
    pfull = np.sum(U[:, :rk] ** 2, axis=1) / rk
    N = 4
    beta = 1.0 / (ranks[n] * ranks[(n + 1) % N] *
                  np.prod([ranks[k] ** 2 for k in range(N) if k not in (n, (n + 1) % N)]))
    assert np.all(q >= beta * pfull * (1 - 1e-12))


@pytest.mark.parametrize("n", [0, 2])
def test_euclid_estimate_lemma_first_inequality(n):
    """prod_k ||G_k(i_k)||_F^2 >= ||G^{!=n}(:, i, :)||_F^2 (submultiplicativity,
    the first inequality in the proof of lemma euc_est)."""
    sizes, ranks = [3, 4, 3, 2], [2, 3, 2, 2]
    cores = ti.gaussian_cores(5, 4, sizes, ranks)
    Gs = tr.subchain_unfold2(cores, n)
    order = tr.cyclic_order(4, n)
    slice_norm = [np.sum(c ** 2, axis=(0, 2)) for c in cores]
    prod = np.ones(1)
    for k in order:
        prod = np.outer(slice_norm[k], prod).ravel()
    assert np.all(prod >= np.sum(Gs ** 2, axis=1) * (1 - 1e-12))


def test_optimal_law_closed_form_and_zero_residual():
    sizes, ranks = [3, 4, 2], [2, 1, 2]
    cores = ti.gaussian_cores(6, 3, sizes, ranks)
    X = ti.standard_normal(7, sizes)
    q, zero = sampling.dist_optimal(cores, X, 1)
    assert not zero
    Xn = tr.unfold_cyclic(X, 1)
    Gs = tr.subchain_unfold2(cores, 1)
    Gn = tr.core_unfold2(cores[1])
    a = np.array([np.linalg.norm(Gn @ Gs[j] - Xn[:, j]) * np.linalg.norm(Gs[j])
                  for j in range(Gs.shape[0])])
    assert np.allclose(q, a / a.sum(), rtol=1e-12)
    Xexact = tr.fold_cyclic(Gn @ Gs.T, 1, sizes)   # residual exactly zero
    q, zero = sampling.dist_optimal(cores, Xexact, 1)
    assert zero and q is None
