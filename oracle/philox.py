"""Philox4x64-10 and Lemire's bounded integers, written from their published
definitions, for the CPU oracle (test infrastructure only).

Philox4x64-R is the counter-based generator of Salmon, Moraes, Dror and Shaw,
"Parallel random numbers: as easy as 1, 2, 3" (SC'11): a 256-bit counter and
a 128-bit key go through R rounds of a multiply/xor bijection, the key being
bumped by two Weyl constants between rounds.  The paper on tensor-ring
decomposition draws its mode and its fibers at random but fixes no generator;
this counter-based one makes every draw a pure function of
(seed, step, sample, mode, stream), so that any implementation can reproduce
it exactly.

Bounded integers follow Lemire, "Fast random integer generation in an
interval" (ACM TOMACS 2019): floor(r * n / 2^64) for a 64-bit uniform r.

Two implementations live here: ``philox_int`` with Python integers (obviously
correct, slow) and ``philox_np`` vectorised with numpy uint64 limbs.  Tests
pin both against ``numpy.random.Philox`` and against each other.
"""
from __future__ import annotations

import numpy as np

M0 = 0xD2E7470EE14C6C93
M1 = 0xCA5A826395121157
W0 = 0x9E3779B97F4A7C15
W1 = 0xBB67AE8584CAA73B
MASK64 = (1 << 64) - 1
ROUNDS = 10

# Stream tags: the fourth counter word separates independent uses.
STREAM_MODE = 0
STREAM_IDX = 1
STREAM_H = 2
STREAM_ENTRY = 3


def philox_int(ctr, key, rounds: int = ROUNDS):
    """One Philox4x64 block with Python integers; returns 4 ints."""
    c0, c1, c2, c3 = (int(x) & MASK64 for x in ctr)
    k0, k1 = (int(x) & MASK64 for x in key)
    for rnd in range(rounds):
        if rnd > 0:
            k0 = (k0 + W0) & MASK64
            k1 = (k1 + W1) & MASK64
        p0 = M0 * c0
        p1 = M1 * c2
        hi0, lo0 = p0 >> 64, p0 & MASK64
        hi1, lo1 = p1 >> 64, p1 & MASK64
        c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    return c0, c1, c2, c3


_U = np.uint64
_M32 = _U(0xFFFFFFFF)
_S32 = _U(32)


def _mulhilo(a: int, b: np.ndarray):
    """(hi, lo) of the 128-bit product of the constant ``a`` with uint64 ``b``."""
    a_lo = _U(a & 0xFFFFFFFF)
    a_hi = _U(a >> 32)
    b_lo = b & _M32
    b_hi = b >> _S32
    ll = a_lo * b_lo
    lh = a_lo * b_hi
    hl = a_hi * b_lo
    hh = a_hi * b_hi
    mid = (ll >> _S32) + (lh & _M32) + (hl & _M32)
    lo = (ll & _M32) | ((mid & _M32) << _S32)
    hi = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return hi, lo


def philox_np(c0, c1, c2, c3, k0: int, k1: int, rounds: int = ROUNDS):
    """Vectorised Philox4x64: counters are broadcastable uint64 arrays."""
    c0, c1, c2, c3 = np.broadcast_arrays(*(np.asarray(c, dtype=np.uint64) for c in (c0, c1, c2, c3)))
    c0, c1, c2, c3 = (c.copy() for c in (c0, c1, c2, c3))
    k0 = int(k0) & MASK64
    k1 = int(k1) & MASK64
    with np.errstate(over="ignore"):
        for rnd in range(rounds):
            if rnd > 0:
                k0 = (k0 + W0) & MASK64
                k1 = (k1 + W1) & MASK64
            hi0, lo0 = _mulhilo(M0, c0)
            hi1, lo1 = _mulhilo(M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ _U(k0), lo1, hi0 ^ c3 ^ _U(k1), lo0
    return c0, c1, c2, c3


def mulhi_np(r: np.ndarray, n) -> np.ndarray:
    """Lemire's bounded integer floor(r * n / 2^64) for uint64 r and n < 2^64."""
    r = np.asarray(r, dtype=np.uint64)
    n = np.asarray(n, dtype=np.uint64)
    r, n = np.broadcast_arrays(r, n)
    out = np.empty(r.shape, dtype=np.uint64)
    flat_r = r.ravel()
    flat_n = n.ravel()
    with np.errstate(over="ignore"):
        r_lo = flat_r & _M32
        r_hi = flat_r >> _S32
        n_lo = flat_n & _M32
        n_hi = flat_n >> _S32
        ll = r_lo * n_lo
        lh = r_lo * n_hi
        hl = r_hi * n_lo
        hh = r_hi * n_hi
        mid = (ll >> _S32) + (lh & _M32) + (hl & _M32)
        out.ravel()[:] = hh + (lh >> _S32) + (hl >> _S32) + (mid >> _S32)
    return out


def mulhi_int(r: int, n: int) -> int:
    """Lemire's bounded integer with Python integers."""
    return (int(r) * int(n)) >> 64


def draw_word(seed: int, t, f, k, stream: int) -> np.ndarray:
    """First output word of Philox4x64-10 with key (seed, 0) and counter
    (t, f, k, stream); arguments broadcast."""
    w0, _, _, _ = philox_np(t, f, k, stream, seed, 0)
    return w0
