"""Pins of the oracle's gradient, Hessian, direction and update rules
against closed forms, finite differences, exact enumeration of the
sampling law and library least squares (Section 3)."""
import numpy as np
import pytest

import tr_inputs as ti
from oracle import brsgd, sampling, tr

SIZES = [4, 3, 5]
RANKS = [2, 3, 2]


def _problem(seed=0, noise=0.3):
    cores = ti.gaussian_cores(seed, 3, SIZES, RANKS)
    X = tr.full_tensor(ti.gaussian_cores(seed + 100, 3, SIZES, RANKS))
    X = X + noise * ti.standard_normal(seed + 200, X.shape)
    return cores, X


@pytest.mark.parametrize("n", [0, 1, 2])
def test_full_gradient_equals_central_difference(n):
    """eq:gradient against central differences of f; f is quadratic in each
    block, so the difference is exact up to rounding (T4)."""
    cores, X = _problem(1)
    G = tr.full_gradient(cores, X, n)
    Gn2 = tr.core_unfold2(cores[n])
    h = 0.5
    fd = np.zeros_like(G)
    for i in range(G.shape[0]):
        for c in range(G.shape[1]):
            for sgn in (1, -1):
                P = Gn2.copy()
                P[i, c] += sgn * h
                cc = list(cores)
                cc[n] = tr.core_fold2(P, cores[n].shape[0], cores[n].shape[2])
                fd[i, c] += sgn * tr.objective(cc, X)
    fd /= 2 * h
    assert np.allclose(G, fd, rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_stochastic_gradient_with_all_columns_is_full_over_J(n):
    """eq:S_gradient with F = every column once and p = 1/J_n equals
    grad f / J_n exactly (T5; the literal 1/(|F| J_n) factor)."""
    cores, X = _problem(2)
    Jn = brsgd.J_of(SIZES, n)
    Gs = tr.subchain_unfold2(cores, n)
    g, loss = brsgd.stoch_grad(tr.core_unfold2(cores[n]), Gs, tr.unfold_cyclic(X, n),
                               np.full(Jn, 1.0 / Jn), Jn)
    assert np.allclose(g, tr.full_gradient(cores, X, n) / Jn, rtol=1e-12, atol=1e-13)
    assert np.isclose(loss, tr.objective(cores, X), rtol=1e-12)


def _laws(cores, X, n):
    out = {}
    for d in ("U", "E", "L", "O"):
        w, wJ, _ = sampling.weights_for(d, cores, n, X)
        q = (wJ.astype(float) / float(wJ.sum())) if wJ is not None else sampling.law_of(w, SIZES, n)
        out[d] = q
    return out


def _single_sample(cores, X, n, j, q):
    Gs = tr.subchain_unfold2(cores, n)
    Xn = tr.unfold_cyclic(X, n)
    Jn = Gs.shape[0]
    return brsgd.stoch_grad(tr.core_unfold2(cores[n]), Gs[j:j + 1], Xn[:, j:j + 1],
                            np.array([q[j]]), Jn)


@pytest.mark.parametrize("n", [0, 2])
def test_unbiased_gradient_by_enumeration(n):
    """E[g] = grad f / J_n and E[loss_est] = f for every law (T6)."""
    cores, X = _problem(3)
    full = tr.full_gradient(cores, X, n)
    Jn = brsgd.J_of(SIZES, n)
    for d, q in _laws(cores, X, n).items():
        Eg = np.zeros_like(full)
        El = 0.0
        for j in range(Jn):
            g, l = _single_sample(cores, X, n, j, q)
            Eg += q[j] * g
            El += q[j] * l
        assert np.allclose(Eg, full / Jn, rtol=1e-10, atol=1e-12), d
        assert np.isclose(El, tr.objective(cores, X), rtol=1e-10), d


@pytest.mark.parametrize("n", [1])
def test_variance_formula_and_optimal_law(n):
    """Variance of eq:var (paper's scale, i.e. J_n^2 times the literal g's),
    its optimum eq:optimal_var at the law eq:optimal_prob, and no other law
    below it (T7)."""
    cores, X = _problem(4)
    Jn = brsgd.J_of(SIZES, n)
    full = tr.full_gradient(cores, X, n)
    Gs = tr.subchain_unfold2(cores, n)
    Rres = tr.core_unfold2(cores[n]) @ Gs.T - tr.unfold_cyclic(X, n)
    a = np.linalg.norm(Rres, axis=0) * np.linalg.norm(Gs, axis=1)
    laws = _laws(cores, X, n)
    exact_q = a / a.sum()
    laws["O-exact"] = exact_q
    var = {}
    for d, q in laws.items():
        v = 0.0
        for j in range(Jn):
            g, _ = _single_sample(cores, X, n, j, q)
            v += q[j] * np.sum((Jn * g - full) ** 2)
        formula = np.sum(a ** 2 / q) - np.sum(full ** 2)
        assert np.isclose(v, formula, rtol=1e-9), d
        var[d] = v
    opt = a.sum() ** 2 - np.sum(full ** 2)
    assert np.isclose(var["O-exact"], opt, rtol=1e-12)
    assert np.isclose(var["O"], opt, rtol=1e-8)   # 2^-40 quantisation
    for d in ("U", "E", "L"):
        assert var[d] >= opt * (1 - 1e-12)


def test_unbiased_hessian_by_enumeration():
    """E[h] = Gs^T Gs / J_n for S_hessian read with 1/(|H| J_n) (T10)."""
    cores, X = _problem(5)
    n = 0
    Jn = brsgd.J_of(SIZES, n)
    Gs = tr.subchain_unfold2(cores, n)
    for d, q in _laws(cores, X, n).items():
        Eh = np.zeros((Gs.shape[1],) * 2)
        for j in range(Jn):
            Eh += q[j] * brsgd.stoch_hessian(Gs[j:j + 1], np.array([q[j]]), Jn)
        assert np.allclose(Eh, Gs.T @ Gs / Jn, rtol=1e-10, atol=1e-12), d


def test_scaled_step_alpha_one_is_weighted_least_squares():
    """alpha = 1, H = F: the scaled step is the importance-weighted sampled
    least-squares solution (numpy lstsq); with every column once it is the
    exact ALS block update (T11)."""
    cores, X = _problem(6)
    n = 1
    Jn = brsgd.J_of(SIZES, n)
    idx, pF = sampling.draw(0, 0, n, 40, SIZES)
    S = brsgd.subchain_rows(cores, n, idx)
    XF = brsgd.gather_fibers(X, n, idx)
    G = tr.core_unfold2(cores[n])
    g, _ = brsgd.stoch_grad(G, S, XF, pF, Jn)
    p, st = brsgd.scaled_direction(g, brsgd.stoch_hessian(S, pF, Jn))
    assert st == 0
    wsq = 1.0 / np.sqrt(pF)
    Z, *_ = np.linalg.lstsq(S * wsq[:, None], (XF * wsq[None, :]).T, rcond=None)
    assert np.allclose(G + p, Z.T, rtol=1e-9, atol=1e-10)
    Gs = tr.subchain_unfold2(cores, n)
    g, _ = brsgd.stoch_grad(G, Gs, tr.unfold_cyclic(X, n), np.full(Jn, 1.0 / Jn), Jn)
    p, _ = brsgd.scaled_direction(g, brsgd.stoch_hessian(Gs, np.full(Jn, 1.0 / Jn), Jn))
    Zals, *_ = np.linalg.lstsq(Gs, tr.unfold_cyclic(X, n).T, rcond=None)
    assert np.allclose(G + p, Zals.T, rtol=1e-9, atol=1e-10)


def test_damping_limit_recovers_plain_direction():
    """eta * p(eta) -> -g as eta -> infinity (amended preconditioner, T12)."""
    cores, X = _problem(7)
    n = 2
    Jn = brsgd.J_of(SIZES, n)
    idx, pF = sampling.draw(1, 0, n, 30, SIZES)
    S = brsgd.subchain_rows(cores, n, idx)
    g, _ = brsgd.stoch_grad(tr.core_unfold2(cores[n]), S, brsgd.gather_fibers(X, n, idx), pF, Jn)
    errs = []
    for eta in (1e2, 1e4, 1e6):
        p, _ = brsgd.scaled_direction(g, brsgd.stoch_hessian(S, pF, Jn, damping=eta))
        errs.append(np.linalg.norm(eta * p + g) / np.linalg.norm(g))
    assert errs[0] > errs[1] > errs[2] and errs[2] < 1e-5


def test_damping_fallback_on_singular_gram():
    """|H| < R_n R_{n+1}: h is singular, Cholesky fails, damping is used."""
    cores, X = _problem(8)
    n = 0
    Jn = brsgd.J_of(SIZES, n)
    idx, pF = sampling.draw(2, 0, n, 3, SIZES)       # 3 rows < RR = 6
    S = brsgd.subchain_rows(cores, n, idx)
    g, _ = brsgd.stoch_grad(tr.core_unfold2(cores[n]), S, brsgd.gather_fibers(X, n, idx), pF, Jn)
    h = brsgd.stoch_hessian(S, pF, Jn)
    p, st = brsgd.scaled_direction(g, h)
    assert st in (0, brsgd.DEV_DAMPED)
    assert np.all(np.isfinite(p))
    if st == brsgd.DEV_DAMPED:
        ok = [k for k in range(7)
              if np.all(np.linalg.eigvalsh(h + 10.0 ** (k - 10) * np.trace(h) / 6 * np.eye(6)) > 0)]
        assert ok


def test_adagrad_first_step_and_scale_invariance():
    """b = eps = 0: the first AdaGrad step is eta * sign(p) entrywise, and the
    update does not change when p is scaled (T13)."""
    rng = np.random.default_rng(0)
    G = rng.standard_normal((5, 4))
    p = rng.standard_normal((5, 4))
    p[0, 0] = 0.0
    cfg = brsgd.Config(m=1, rule="adagrad", eta=0.3)
    new, A = brsgd.update(G, p, cfg, 0, np.zeros_like(G))
    assert np.allclose(new - G, 0.3 * np.sign(p), rtol=1e-15, atol=0)
    new2, _ = brsgd.update(new, 2 * p, cfg, 1, A)
    new2s, _ = brsgd.update(new, 2000 * p, cfg, 1, 1e6 * A)
    assert np.allclose(new2, new2s, rtol=1e-13)


def test_fixed_and_robbins_monro_rules():
    G = np.ones((2, 2))
    p = np.full((2, 2), 2.0)
    c = brsgd.Config(m=1, alpha=0.25)
    assert np.array_equal(brsgd.update(G, p, c, 5, None)[0], G + 0.5)
    c = brsgd.Config(m=1, rule="robbins-monro", alpha=0.5, tau=10.0)
    assert np.allclose(brsgd.update(G, p, c, 10, None)[0], G + 0.5)
