"""Pins of the oracle's sampled-entry loss and all-core gradient: element-wise
Trace, central finite differences (exact: the loss is quadratic in each
scalar) and the full block gradient eq:gradient when every entry is
sampled once."""
import itertools

import numpy as np

import tr_inputs as ti
from oracle import entry, tr

SIZES, RANKS = [3, 4, 2, 3], [2, 3, 1, 2]


def test_entry_values_equal_trace():
    cores = ti.gaussian_cores(0, 4, SIZES, RANKS)
    idx = ti.entry_indices(1, SIZES, 30)
    v = entry.entry_values(cores, idx)
    for b in range(30):
        assert abs(v[b] - tr.entry_by_trace(cores, idx[b])) < 1e-12


def test_entry_grads_equal_central_differences():
    cores = ti.gaussian_cores(2, 4, SIZES, RANKS)
    idx = ti.entry_indices(3, SIZES, 50)
    x = ti.standard_normal(4, 50)
    grads = entry.entry_grads(cores, idx, x)
    h = 1e-3
    rng = np.random.default_rng(0)
    for k in range(4):
        for _ in range(8):
            pos = tuple(int(rng.integers(0, s)) for s in cores[k].shape)
            vals = []
            for sgn in (1, -1):
                cc = [c.copy() for c in cores]
                cc[k][pos] += sgn * h
                vals.append(entry.entry_loss(cc, idx, x)[0])
            fd = (vals[0] - vals[1]) / (2 * h)
            assert abs(fd - grads[k][pos]) < 1e-9 * max(1.0, abs(fd))


def test_entry_grads_equal_block_gradient_when_every_entry_once():
    cores = ti.gaussian_cores(5, 4, SIZES, RANKS)
    X = ti.standard_normal(6, SIZES)
    idx = np.array(list(itertools.product(*[range(s) for s in SIZES])), dtype=np.int32)
    x = np.array([X[tuple(r)] for r in idx])
    grads = entry.entry_grads(cores, idx, x)
    B = len(x)
    for n in range(4):
        G = tr.full_gradient(cores, X, n) / B
        want = tr.core_fold2(G, cores[n].shape[0], cores[n].shape[2])
        assert np.allclose(grads[n], want, rtol=1e-11, atol=1e-14)
