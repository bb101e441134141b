"""Pins of the oracle's random draws: Philox4x64-10 against numpy's Philox
(library routine), Lemire's bound against exact integers, the integer-CDF
sampler against brute force and chi-square, the product law of Section 3.2
(sampling each core independently = sampling rows of G^{!=n}_[2])."""
import numpy as np
import pytest
from scipy import stats

import tr_inputs as ti
from oracle import philox, sampling, tr


def _numpy_block(ctr, key):
    c = list(ctr)
    # numpy increments the counter before each block: start one below.
    for w in range(4):
        if c[w] > 0:
            c[w] -= 1
            break
        c[w] = (1 << 64) - 1
    bg = np.random.Philox(counter=c, key=list(key))
    return [int(x) for x in bg.random_raw(4)]


def test_philox_matches_numpy_library():
    rng = np.random.default_rng(123)
    for _ in range(50):
        ctr = [int(x) for x in rng.integers(0, 2**63, 4, dtype=np.uint64)]
        ctr[0] |= 1  # avoid a borrow through all words in the helper
        key = [int(x) for x in rng.integers(0, 2**63, 2, dtype=np.uint64)]
        want = _numpy_block(ctr, key)
        assert list(philox.philox_int(ctr, key)) == want
        got = philox.philox_np(*[np.uint64(c) for c in ctr], key[0], key[1])
        assert [int(x) for x in got] == want


def test_philox_vectorised_equals_scalar():
    t = np.arange(40, dtype=np.uint64)
    f = (t * np.uint64(7919)) ^ np.uint64(0xDEADBEEF)
    got = philox.philox_np(t, f, 3, philox.STREAM_IDX, 99, 0)
    for i in range(40):
        want = philox.philox_int((int(t[i]), int(f[i]), 3, philox.STREAM_IDX), (99, 0))
        assert tuple(int(g[i]) for g in got) == want


def test_lemire_bound_exact():
    rng = np.random.default_rng(5)
    r = rng.integers(0, 2**64 - 1, 1000, dtype=np.uint64, endpoint=True)
    for n in (1, 3, 20, 400, 2**40 + 12345, 2**53 - 1):
        got = philox.mulhi_np(r, n)
        want = [(int(x) * n) >> 64 for x in r]
        assert [int(x) for x in got] == want
        assert int(got.max()) < n


def test_mode_pick_uniform():
    N = 5
    modes = [sampling.pick_mode(42, t, N) for t in range(5000)]
    counts = np.bincount(modes, minlength=N)
    assert stats.chisquare(counts).pvalue > 1e-6
    assert modes == [sampling.pick_mode(42, t, N) for t in range(5000)]


def test_cdf_pick_first_exceeding_brute_force():
    w = ti.int_weights(3, 17, 1, 50)
    C = np.cumsum(w)
    rng = np.random.default_rng(9)
    r = rng.integers(0, 2**64 - 1, 3000, dtype=np.uint64, endpoint=True)
    i, p = sampling._cdf_pick(r, w)
    for rr, ii, pp in zip(r, i, p):
        u = (int(rr) * int(C[-1])) >> 64
        want = next(k for k in range(len(w)) if int(C[k]) > u)
        assert ii == want
        assert pp == float(w[ii]) / float(C[-1])


def test_weighted_draw_chi_square_and_product_probability():
    """Index frequencies follow w/W per mode (T15), p_F = prod p_k(i_k)."""
    sizes = [6, 5, 7]
    w = [ti.int_weights(10 + k, s, 1, 1000) for k, s in enumerate(sizes)]
    n = 1
    m = 40000
    idx, pF = sampling.draw(7, 3, n, m, sizes, w)
    assert np.all(idx[:, n] == -1)
    want = np.ones(m)
    for k in tr.cyclic_order(3, n):
        counts = np.bincount(idx[:, k], minlength=sizes[k])
        exp = w[k].astype(float) / w[k].astype(float).sum() * m
        assert stats.chisquare(counts, exp).pvalue > 1e-6
        want = want * (w[k].astype(float) / float(w[k].sum()))[idx[:, k]]
    assert np.array_equal(pF, want)


def test_uniform_draw_probability_and_range():
    sizes = [4, 9, 3, 8]
    idx, pF = sampling.draw(1, 0, 2, 5000, sizes)
    for k in (3, 0, 1):
        assert idx[:, k].min() >= 0 and idx[:, k].max() < sizes[k]
        assert stats.chisquare(np.bincount(idx[:, k], minlength=sizes[k])).pvalue > 1e-6
    want = 1.0 * (1.0 / 8) * (1.0 / 4) * (1.0 / 9)
    assert np.all(pF == want)


def test_product_law_equals_row_law():
    """Drawing one slice per core with p_k samples row j of G^{!=n}_[2]
    with q(j) = prod p_k(i_k) (end of Section 3.2)."""
    sizes = [3, 4, 2]
    n = 0
    w = [None, ti.int_weights(1, 4, 1, 20), ti.int_weights(2, 2, 1, 20)]
    q = sampling.law_of(w, sizes, n)
    assert abs(q.sum() - 1) < 1e-15
    m = 60000
    idx, pF = sampling.draw(3, 0, n, m, sizes, w)
    cols = np.array([tr.cyclic_column(r, sizes, n) for r in idx])
    counts = np.bincount(cols, minlength=len(q))
    assert stats.chisquare(counts, q * m).pvalue > 1e-6
    assert np.allclose(pF, q[cols], rtol=1e-15)


def test_direct_draw_decodes_cyclic_multi_index():
    sizes = [3, 4, 5]
    n = 1
    J = 15
    w_J = ti.int_weights(4, J, 1, 100)
    idx, pF = sampling.draw(2, 5, n, 20000, sizes, w_J=w_J)
    assert np.all(idx[:, n] == -1)
    cols = np.array([tr.cyclic_column(r, sizes, n) for r in idx])
    p = w_J.astype(float) / float(w_J.sum())
    assert np.array_equal(pF, p[cols])
    assert stats.chisquare(np.bincount(cols, minlength=J), p * 20000).pvalue > 1e-6


def test_quantize_rule():
    p = np.array([0.0, 2.0**-40, 0.5, 0.25 - 2.0**-50, 1.0])
    w = sampling.quantize(p)
    assert [int(x) for x in w] == [1, 2, 2**39 + 1, 2**38, 2**40 + 1]


def test_draws_reproducible_and_step_dependent():
    sizes = [7, 7, 7]
    a = sampling.draw(0, 10, 0, 64, sizes)[0]
    b = sampling.draw(0, 10, 0, 64, sizes)[0]
    c = sampling.draw(0, 11, 0, 64, sizes)[0]
    d = sampling.draw(1, 10, 0, 64, sizes)[0]
    assert np.array_equal(a, b)
    assert not np.array_equal(a, c) and not np.array_equal(a, d)
