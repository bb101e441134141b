"""Seeded synthetic inputs shared by the CPU oracle, the tests and the benchmark.

This module only draws random numbers and shapes.  It holds none of the
decomposition's arithmetic: no tensor-ring contraction, no unfolding, no
sampling law, no gradient.  Each consumer (the oracle on the CPU, the HIP
library on the GPU) builds the planted tensor from these cores with its own
code.

Cores are returned in their natural three-way form, ``core[r, i, s]`` with
shape ``(R_k, I_k, R_{k+1})`` and ``R_{N+1} = R_1`` (tensor-ring format of
the paper's introduction).  Every generator takes an explicit integer seed
and uses ``numpy.random.default_rng`` so that the same call returns the same
arrays on every machine.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "ring_ranks",
    "gaussian_cores",
    "illcond_cores",
    "standard_normal",
    "int_weights",
    "entry_indices",
    "BatchInstance",
    "batched_instances",
    "WORKLOADS",
]


def ring_ranks(N: int, R) -> list[int]:
    """Expand a scalar rank to the N ring ranks R_1..R_N (R_{N+1} = R_1)."""
    if np.isscalar(R):
        return [int(R)] * N
    R = [int(r) for r in R]
    if len(R) != N:
        raise ValueError("need one rank per mode")
    return R


def _sizes(N: int, I) -> list[int]:
    if np.isscalar(I):
        return [int(I)] * N
    I = [int(i) for i in I]
    if len(I) != N:
        raise ValueError("need one size per mode")
    return I


def gaussian_cores(seed: int, N: int, I, R, scale: float = 1.0) -> list[np.ndarray]:
    """Cores with i.i.d. N(0, scale^2) entries (synthetic-data section: each
    planted core has standard-normal entries; also the random initialisation).
    """
    rng = np.random.default_rng(seed)
    I = _sizes(N, I)
    R = ring_ranks(N, R)
    out = []
    for k in range(N):
        shape = (R[k], I[k], R[(k + 1) % N])
        out.append(scale * rng.standard_normal(shape))
    return out


def illcond_cores(seed: int, N: int, I, R: int, kappa: float) -> list[np.ndarray]:
    """Ill-conditioned cores of the second synthetic experiment.

    Each core's mode-2 unfolding is U_n * S * V^T: U_n (I_n x R^2) has
    orthonormal columns from the QR factorisation of a Gaussian matrix, S is
    diagonal with entries decreasing geometrically from 1 to 1/kappa, and V
    (R^2 x R^2, orthogonal) is shared by all cores.  The unfolding's column
    c maps to core[r, i, s] with c = r + R*s (first index fastest).
    """
    rng = np.random.default_rng(seed)
    I = _sizes(N, I)
    RR = R * R
    if any(i < RR for i in I):
        raise ValueError("ill-conditioned generator needs I_n >= R^2")
    sv = np.geomspace(1.0, 1.0 / kappa, RR)
    V, _ = np.linalg.qr(rng.standard_normal((RR, RR)))
    cores = []
    for k in range(N):
        U, _ = np.linalg.qr(rng.standard_normal((I[k], RR)))
        G2 = (U * sv) @ V.T                       # I_k x R^2
        core = G2.reshape(I[k], R, R, order="F")  # [i, r, s], c = r + R*s
        cores.append(np.ascontiguousarray(core.transpose(1, 0, 2)))
    return cores


def standard_normal(seed: int, shape, dtype=np.float64) -> np.ndarray:
    """I.i.d. N(0,1) array (noise, initial values)."""
    rng = np.random.default_rng(seed)
    return rng.standard_normal(shape, dtype=np.float64).astype(dtype, copy=False)


def int_weights(seed: int, n: int, low: int = 1, high: int = 1 << 40) -> np.ndarray:
    """Random positive integer weights in [low, high), uint64 (sampler tests)."""
    rng = np.random.default_rng(seed)
    return rng.integers(low, high, size=n, dtype=np.uint64)


def entry_indices(seed: int, I, B: int) -> np.ndarray:
    """B uniform multi-indices drawn with replacement, int32 array [B, N]."""
    rng = np.random.default_rng(seed)
    cols = [rng.integers(0, int(i), size=B) for i in I]
    return np.stack(cols, axis=1).astype(np.int32)


@dataclass
class BatchInstance:
    """One problem of the batched workload: order, sizes and ranks."""
    N: int
    I: list[int]
    R: list[int]
    seed: int = 0
    extra: dict = field(default_factory=dict)


def batched_instances(seed: int, count: int = 64, orders=(3, 4, 5),
                      size_range=(16, 128), rank_range=(3, 12),
                      max_entries: int = 1 << 27) -> list[BatchInstance]:
    """Independent problems of uneven order, size and rank.

    N is uniform over ``orders``; each I_n is uniform over ``size_range``
    (inclusive) and each R_n over ``rank_range`` (inclusive), i.i.d. per mode.
    Sizes are redrawn until prod(I_n) <= max_entries so that every dense
    tensor fits in device memory next to the others.
    """
    rng = np.random.default_rng(seed)
    out = []
    for p in range(count):
        N = int(rng.choice(orders))
        while True:
            I = [int(x) for x in rng.integers(size_range[0], size_range[1] + 1, size=N)]
            if int(np.prod(I, dtype=np.int64)) <= max_entries:
                break
        R = [int(x) for x in rng.integers(rank_range[0], rank_range[1] + 1, size=N)]
        out.append(BatchInstance(N=N, I=I, R=R, seed=int(rng.integers(0, 2**31))))
    return out


# The five workloads, by what they are.  Sizes follow the paper's synthetic
# experiments scaled to the shapes named in the design notes.
WORKLOADS = {
    "plain-fp64-n3-i20-r3": dict(N=3, I=20, R=3, m=100, steps=500, dtype="f64",
                                 noise_db=None, dist="U", variant="plain"),
    "adagrad-fp32-n4-i64-r5": dict(N=4, I=64, R=5, m=512, dtype="f32",
                                   noise_db=40.0, dist=("U", "L", "E", "O"),
                                   variant="plain", rule="adagrad"),
    "scaled-illcond-n3-i400-r10": dict(N=3, I=400, R=10, m=4096, dtype="f32",
                                       kappa=1e4, noise_db=None, dist="U",
                                       variant="scaled"),
    "autograd-n5-i32-r8": dict(N=5, I=32, R=8, B=8192, dtype="f32", noise_db=30.0),
    "batched-64": dict(count=64, m=1024, dtype="f16", noise_db=40.0),
}
