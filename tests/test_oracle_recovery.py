"""End-to-end pins of the oracle's Algorithm TR-BRSGD: exact recovery of a
planted ring in FP64, mode relabelling invariance, noise and
initialisation recipes."""
import numpy as np

import tr_inputs as ti
from oracle import brsgd, sampling, tr


def _planted(N=3, I=20, R=3):
    X = tr.full_tensor(ti.gaussian_cores(0, N, I, R))
    sig = brsgd.init_scale(X, [R] * N)
    return X, ti.gaussian_cores(1, N, I, R, scale=sig)


def test_plain_recovers_planted_ring_to_tol():
    """Plain TR-BRSGD, uniform fibers, m = 100, fixed alpha = 0.2 on the
    20^3 rank-3 planted ring reaches RSE <= 1e-10 (the paper's tol) (T14)."""
    X, init = _planted()
    st = brsgd.State(init)
    hist = brsgd.run(st, X, brsgd.Config(m=100, alpha=0.2, seed=0), 1500, rse_every=50, tol=1e-10)
    assert hist[-1][1] <= 1e-10, hist[-5:]


def test_scaled_recovers_planted_ring_to_tol():
    X, init = _planted()
    st = brsgd.State(init)
    hist = brsgd.run(st, X, brsgd.Config(m=100, variant="scaled", alpha=1.0, seed=0),
                     800, rse_every=50, tol=1e-10)
    assert hist[-1][1] <= 1e-10, hist[-5:]


def test_adagrad_recovers_planted_ring():
    X, init = _planted()
    st = brsgd.State(init)
    hist = brsgd.run(st, X, brsgd.Config(m=100, rule="adagrad", eta=0.3, seed=0),
                     3000, rse_every=100, tol=1e-9)
    assert hist[-1][1] <= 1e-9, hist[-5:]


def test_mode_relabelling_invariance():
    """A step on mode n equals a step on mode 1 of the cyclically shifted
    problem fed the same fibers (T17)."""
    sizes, ranks = [4, 5, 3, 6], [2, 3, 2, 1]
    cores = ti.gaussian_cores(2, 4, sizes, ranks)
    X = ti.standard_normal(3, sizes)
    for n in range(4):
        idx, pF = sampling.draw(5, 0, n, 25, sizes)
        S = brsgd.subchain_rows(cores, n, idx)
        XF = brsgd.gather_fibers(X, n, idx)
        g, l = brsgd.stoch_grad(tr.core_unfold2(cores[n]), S, XF, pF, brsgd.J_of(sizes, n))
        perm = [(n + d) % 4 for d in range(4)]
        cs = [cores[k] for k in perm]
        Xs = X.transpose(perm)
        idx_s = idx[:, perm]
        S2 = brsgd.subchain_rows(cs, 0, idx_s)
        XF2 = brsgd.gather_fibers(Xs, 0, idx_s)
        g2, l2 = brsgd.stoch_grad(tr.core_unfold2(cs[0]), S2, XF2, pF,
                                  brsgd.J_of([sizes[k] for k in perm], 0))
        assert np.allclose(S, S2, rtol=1e-14, atol=1e-15)
        assert np.array_equal(XF, XF2)
        assert np.allclose(g, g2, rtol=1e-13, atol=1e-15) and np.isclose(l, l2, rtol=1e-13)


def test_noise_recipe_hits_requested_snr():
    X = tr.full_tensor(ti.gaussian_cores(0, 3, 12, 2))
    E = ti.standard_normal(1, X.shape)
    Xn = brsgd.add_noise(X, E, 40.0)
    snr = 20 * np.log10(np.linalg.norm(X) / np.linalg.norm(Xn - X))
    assert abs(snr - 40.0) < 0.3


def test_init_scale_matches_second_moment():
    """For i.i.d. N(0, s^2) cores, E[X(i)^2] = s^(2N) prod R_k."""
    N, I, R = 3, 30, [3, 4, 2]
    X = tr.full_tensor(ti.gaussian_cores(9, N, I, R, scale=0.7))
    est = brsgd.init_scale(X, R)
    assert abs(est - 0.7) < 0.07


def test_step_records_trace_and_status():
    X, init = _planted(3, 8, 2)
    st = brsgd.State(init)
    tr_ = {}
    n = brsgd.step(st, X, brsgd.Config(m=16, dist="E", alpha=0.1), trace=tr_)
    assert st.t == 1 and tr_["n"] == n and tr_["S"].shape == (16, 4)
    assert st.status == 0
