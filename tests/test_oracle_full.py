"""Pins of the comparison methods' oracle (TR-GD, TR-ScaledGD, TR-ALS,
TR-ALS-Sampled), each against something other than its own formula: finite
differences of the objective, numpy's least-squares routine, the fixed point
at a planted ring, the monotone decrease of alternating least squares, and
exact recovery (CPU only)."""
import numpy as np
import pytest

import tr_inputs as ti
from oracle import brsgd, full, tr

SIZES, RANKS = [6, 5, 7], [2, 3, 2]


def _problem(seed, noise=0.1):
    true = ti.gaussian_cores(seed, 3, SIZES, RANKS)
    Xt = tr.full_tensor(true)
    X = Xt + noise * ti.standard_normal(seed + 1, Xt.shape)
    init = ti.gaussian_cores(seed + 2, 3, SIZES, RANKS, scale=0.8)
    return true, X, init


def test_gd_sweep_moves_along_the_joint_gradient():
    """All blocks from the same iterate: (G - G_new) / alpha is the joint
    gradient of f, so its inner product with any direction V equals the
    central difference of f along V (exact: f is a polynomial of degree 2N
    in the cores and the difference is taken at a tiny step)."""
    _, X, cores = _problem(1)
    alpha = 1e-3
    new = full.gd_sweep(cores, X, alpha)
    rng = np.random.default_rng(3)
    V = [rng.standard_normal(c.shape) for c in cores]
    h = 1e-5
    fp = tr.objective([c + h * v for c, v in zip(cores, V)], X)
    fm = tr.objective([c - h * v for c, v in zip(cores, V)], X)
    fd = (fp - fm) / (2 * h)
    ip = sum(float(np.sum((c - nc) / alpha * v)) for c, nc, v in zip(cores, new, V))
    assert abs(ip - fd) < 1e-6 * max(1.0, abs(fd)), (ip, fd)


def test_gd_sweep_fixed_point_at_planted_ring():
    true, _, _ = _problem(4)
    X = tr.full_tensor(true)
    new = full.gd_sweep(true, X, 0.1)
    for a, b in zip(new, true):
        assert np.allclose(a, b, rtol=0, atol=1e-12)


def test_scaled_gd_unit_step_is_blockwise_least_squares():
    """alpha = 1: every block jumps to the least-squares solution with the
    other cores at the sweep's starting iterate (numpy's lstsq)."""
    _, X, cores = _problem(5)
    new = full.scaled_gd_sweep(cores, X, 1.0)
    for n in range(3):
        Gs = tr.subchain_unfold2(cores, n)
        Z, *_ = np.linalg.lstsq(Gs, tr.unfold_cyclic(X, n).T, rcond=None)
        assert np.allclose(tr.core_unfold2(new[n]), Z.T, rtol=1e-9, atol=1e-10)


def test_scaled_gd_damping_limit_is_plain_gd():
    """eta (G - G_new(eta)) / alpha -> grad f as eta -> infinity."""
    _, X, cores = _problem(6)
    errs = []
    for eta in (1e3, 1e6, 1e9):
        new = full.scaled_gd_sweep(cores, X, 0.5, damping=eta)
        for n in range(3):
            g = tr.full_gradient(cores, X, n)
            e = np.linalg.norm(eta * (tr.core_unfold2(cores[n]) - tr.core_unfold2(new[n])) / 0.5 - g)
            errs.append(e / np.linalg.norm(g))
    assert errs[-1] < 1e-5 and errs[0] > errs[-1]


def test_als_sweep_monotone_and_block_optimal():
    """Each block update minimises f over that block, so f never increases
    over a sweep and the block gradient of the last block is zero after it."""
    _, X, cores = _problem(7)
    f_prev = tr.objective(cores, X)
    for _ in range(5):
        cores = full.als_sweep(cores, X)
        f = tr.objective(cores, X)
        assert f <= f_prev * (1 + 1e-12)
        f_prev = f
        g = tr.full_gradient(cores, X, 2)
        assert np.linalg.norm(g) < 1e-9 * max(1.0, np.linalg.norm(tr.core_unfold2(cores[2])))


def test_als_recovers_a_planted_ring():
    """A planted 8 x 9 x 10 ring of ranks 2 (from a start where alternating
    least squares does not stall in a swamp) is recovered to RSE <= 1e-10."""
    sizes, ranks = [8, 9, 10], [2, 2, 2]
    true = ti.gaussian_cores(0, 3, sizes, ranks)
    init = ti.gaussian_cores(2, 3, sizes, ranks, scale=0.8)
    X = tr.full_tensor(true)
    cores = init
    for _ in range(60):
        cores = full.als_sweep(cores, X)
        if tr.rse(cores, X) < 1e-10:
            break
    assert tr.rse(cores, X) < 1e-10


@pytest.mark.parametrize("dist", ["U", "L", "E"])
def test_als_sampled_fixed_point_and_equal_to_unit_scaled_step(dist):
    """At the planted ring every sampled subproblem has the true core as an
    exact solution (zero residual), so a sweep changes nothing; off it, block
    n equals TR-ScaledBRSGD's step with alpha = 1 and H_n = F_n from the same
    draws (the weighted sampled least-squares problem)."""
    true, _, init = _problem(9)
    X = tr.full_tensor(true)
    m = 60
    new = full.als_sampled_sweep(true, X, m, dist, seed=3, t0=0)
    for a, b in zip(new, true):
        assert np.allclose(a, b, rtol=1e-8, atol=1e-9)
    new = full.als_sampled_sweep(init, X, m, dist, seed=3, t0=10)
    st = brsgd.State([c.copy() for c in init], t=10)
    cfg = brsgd.Config(m=m, dist=dist, variant="scaled", alpha=1.0, seed=3)
    for n in range(3):
        brsgd.step(st, X, cfg, n=n)
        assert np.allclose(st.cores[n], new[n], rtol=1e-8, atol=1e-9)
