"""Closed-form pins of the oracle pieces that whole-run tests cannot tell
apart from plausible mistakes (CPU only):

* the RSE of Section 4, ||TR(G) - X_true||_F / ||X_true||_F, at values
  other than 0 (a squared or unsquared ratio, or a swapped denominator,
  gives different numbers);
* the AdaGrad rule of the remark after Algorithm TR-BRSGD with b > 0 and
  eps > 0, on entries whose result is a hand-worked number;
* the damping fallback of the amended preconditioner (eta added to the
  stochastic Hessian of eq:S_hessian) on matrices whose first positive
  definite rung of the ladder eta_k = 10^(k-10) tr(h)/RR is known.
"""
import json
import os

import numpy as np
import pytest

import tr_inputs as ti
from oracle import brsgd, tr

HERE = os.path.dirname(os.path.abspath(__file__))


def _golden_ring():
    with open(os.path.join(HERE, "golden", "integer_ring_n3.json")) as fh:
        gold = json.load(fh)
    return [np.array(c, dtype=np.float64) for c in gold["cores"]], np.array(gold["X"], dtype=np.float64)


# ------------------------------------------------------------------ RSE ----

def test_rse_of_zero_cores_is_one():
    """TR(0) = 0, so the error is ||X_true|| and the ratio is exactly 1."""
    cores = ti.gaussian_cores(3, 3, [4, 3, 5], [2, 3, 2])
    X = tr.full_tensor(cores)
    zero = [np.zeros_like(c) for c in cores]
    assert tr.rse(zero, X) == 1.0


def test_rse_of_half_and_double_scaled_targets():
    """X_true = 2 TR(G): error TR(G), norm 2 ||TR(G)|| -> exactly 1/2.
    X_true = -TR(G): error 2 TR(G), norm ||TR(G)|| -> exactly 2.
    (Scaling by 2 is exact in binary floating point.)"""
    cores = ti.gaussian_cores(4, 3, [5, 4, 3], [3, 2, 2])
    X = tr.full_tensor(cores)
    assert tr.rse(cores, 2.0 * X) == 0.5
    assert tr.rse(cores, -X) == 2.0


def test_rse_hand_value_on_integer_ring():
    """The golden 2x2x2 integer ring has entries 9, 0, -6, 0, -3, 3, 2, -2
    (sum of squares 143).  Changing X_true(0,0,0) from 9 to 7 leaves an
    error of norm 2 and ||X_true||^2 = 143 - 81 + 49 = 111, so
    RSE = 2 / sqrt(111) = 0.189832...; changing X_true(1,0,0) from -3 to 1
    as well gives error sqrt(4 + 16) and ||X_true||^2 = 111 - 9 + 1 = 103."""
    cores, X = _golden_ring()
    assert float(np.sum(X * X)) == 143.0
    Xt = X.copy()
    Xt[0, 0, 0] = 7.0
    assert abs(tr.rse(cores, Xt) - 0.1898315991504998) < 1e-15
    Xt[1, 0, 0] = 1.0
    assert abs(tr.rse(cores, Xt) - np.sqrt(20.0 / 103.0)) < 1e-15
    assert abs(tr.rse(cores, Xt) - 0.44065264923923175) < 1e-15


# -------------------------------------------------------------- AdaGrad ----

def test_adagrad_with_b_and_eps_hand_values():
    """eta = 1/2, b = 7, eps = 1/4, fresh accumulator.
    Entry p = 3:  A = 9,  b + A = 16, 16^(3/4) = 8   -> step 0.5*3/8  = 0.1875.
    Entry p = -1: A = 1,  b + A = 8,  8^(3/4) = 2^(9/4) -> step -0.5/2^(9/4).
    Entry p = 0:  A = 0,  b + A = 7 > 0                -> step 0.
    Second call with p = 9 on the first entry: A = 9 + 81 = 90, b + A = 97
    -> step 4.5 / 97^(3/4)."""
    cfg = brsgd.Config(m=1, rule="adagrad", eta=0.5, b=7.0, eps=0.25)
    G = np.array([[1.0, -2.0, 0.5]])
    p = np.array([[3.0, -1.0, 0.0]])
    new, A = brsgd.update(G, p, cfg, 0, np.zeros_like(G))
    assert np.array_equal(A, [[9.0, 1.0, 0.0]])
    assert new[0, 0] == 1.0 + 0.1875
    assert abs(new[0, 1] - (-2.0 - 0.5 * 2.0 ** -2.25)) < 1e-15
    assert new[0, 2] == 0.5
    new2, A2 = brsgd.update(new, np.array([[9.0, 0.0, 0.0]]), cfg, 1, A)
    assert A2[0, 0] == 90.0
    assert abs(new2[0, 0] - (1.1875 + 4.5 * 97.0 ** -0.75)) < 1e-15
    assert abs(4.5 * 97.0 ** -0.75 - 0.14559072646615961) < 1e-15


def test_adagrad_zero_denominator_entries_do_not_move():
    """b = 0 and an entry whose accumulated p is still 0: b + A = 0, and the
    rule leaves that entry unchanged instead of dividing by zero."""
    cfg = brsgd.Config(m=1, rule="adagrad", eta=1.0, b=0.0, eps=0.1)
    G = np.array([[2.0, 3.0]])
    new, A = brsgd.update(G, np.array([[0.0, 4.0]]), cfg, 0, np.zeros_like(G))
    assert new[0, 0] == 2.0
    assert abs(new[0, 1] - (3.0 + 4.0 * 16.0 ** -0.6)) < 1e-15


# ------------------------------------------------------- damping ladder ----

def _ladder_matrix(c):
    """h = diag(4/3 + c/3 (three times), -c): tr(h)/4 = 1 exactly up to
    rounding of the first three entries, smallest eigenvalue -c."""
    a = (4.0 + c) / 3.0
    return np.diag([a, a, a, -c])


@pytest.mark.parametrize("c, k_first", [(3e-6, 5), (3e-9, 2), (5e-10, 1), (5e-11, 0)])
def test_damping_ladder_takes_the_first_positive_definite_rung(c, k_first):
    """With tr(h)/RR = 1, rung k adds 10^(k-10); h + eta_k I is positive
    definite exactly when 10^(k-10) > c.  The direction must then be
    -g (h + 10^(k_first-10) I)^{-1}: entrywise -g_j / (h_jj + eta) here."""
    h = _ladder_matrix(c)
    base = float(np.trace(h)) / 4.0
    assert abs(base - 1.0) < 1e-15
    g = np.array([[1.0, -2.0, 0.5, 3.0], [0.25, 1.0, -1.0, 2.0]])
    p, st = brsgd.scaled_direction(g, h)
    assert st == brsgd.DEV_DAMPED
    eta = 10.0 ** (k_first - 10) * base
    want = -g / (np.diag(h) + eta)[None, :]
    assert np.allclose(p, want, rtol=1e-12, atol=0)
    # the previous rung would not have been positive definite
    if k_first > 0:
        assert -c + 10.0 ** (k_first - 11) * base < 0


def test_damping_ladder_in_a_rotated_basis():
    """Q h Q^T has the same spectrum, so the same rung (k = 5) is taken;
    the expected direction comes from the eigendecomposition of h."""
    h0 = _ladder_matrix(3e-6)
    Q, _ = np.linalg.qr(ti.standard_normal(21, (4, 4)))
    h = Q @ h0 @ Q.T
    h = 0.5 * (h + h.T)
    g = ti.standard_normal(22, (3, 4))
    p, st = brsgd.scaled_direction(g, h)
    assert st == brsgd.DEV_DAMPED
    base = float(np.trace(h)) / 4.0
    lam, V = np.linalg.eigh(h)
    want = -(g @ V) / (lam + 1e-5 * base)[None, :] @ V.T
    assert np.allclose(p, want, rtol=1e-9, atol=1e-12)


def test_damping_ladder_exhausted_leaves_no_update():
    """Smallest eigenvalue -1 with tr(h)/RR about 1: even the last rung
    (10^-4) is not enough; the direction is zero and NOT_SPD is reported."""
    h = _ladder_matrix(1.0)
    g = np.ones((2, 4))
    p, st = brsgd.scaled_direction(g, h)
    assert st == brsgd.DEV_NOT_SPD
    assert np.array_equal(p, np.zeros_like(g))


def test_positive_definite_h_is_not_damped():
    h = _ladder_matrix(-0.5)       # diag(7/6, 7/6, 7/6, 0.5): positive definite
    g = np.ones((1, 4))
    p, st = brsgd.scaled_direction(g, h)
    assert st == 0
    assert np.allclose(p, -g / np.diag(h)[None, :], rtol=1e-15)


# ------------------------------------------------------- damping schedule ----

def test_damping_schedules_hand_values():
    """eta^t of the amended preconditioner: harmonic eta^0 = 2, tau = 4 gives
    2, 1.6, 1 at t = 0, 1, 4; geometric eta^0 = 8, tau = 1/2 gives 8, 4, 1 at
    t = 0, 1, 3; constant stays at eta^0."""
    c = brsgd.Config(m=1, damping=2.0, damping_schedule="harmonic", damping_tau=4.0)
    assert [brsgd.damping_at(c, t) for t in (0, 1, 4)] == [2.0, 1.6, 1.0]
    c = brsgd.Config(m=1, damping=8.0, damping_schedule="geometric", damping_tau=0.5)
    assert [brsgd.damping_at(c, t) for t in (0, 1, 3)] == [8.0, 4.0, 1.0]
    c = brsgd.Config(m=1, damping=0.3)
    assert brsgd.damping_at(c, 10 ** 6) == 0.3


def test_scheduled_step_equals_constant_damping_at_that_step():
    """A scaled step at t = 3 under the geometric schedule (eta^0 = 8,
    tau = 1/2) is the step under the constant damping 1 at the same t (the
    schedule only picks eta^t)."""
    cores = ti.gaussian_cores(5, 3, [6, 5, 7], [2, 3, 2])
    X = tr.full_tensor(ti.gaussian_cores(6, 3, [6, 5, 7], [2, 3, 2]))
    outs = []
    for cfg in (brsgd.Config(m=40, variant="scaled", alpha=0.5, damping=8.0, damping_schedule="geometric",
                             damping_tau=0.5, seed=2),
                brsgd.Config(m=40, variant="scaled", alpha=0.5, damping=1.0, seed=2)):
        st = brsgd.State([c.copy() for c in cores], t=3)
        n = brsgd.step(st, X, cfg)
        outs.append(st.cores[n])
    assert np.array_equal(outs[0], outs[1])
