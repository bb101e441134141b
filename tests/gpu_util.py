"""Helpers shared by the GPU parity tests (not a test module)."""
import sys

import numpy as np
import torch

import tr_inputs as ti
from oracle import tr

DEV = "cuda"
TOL = {torch.float64: 1e-12, torch.float32: 1e-5, torch.bfloat16: 5e-3, torch.float16: 5e-3}


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = np.linalg.norm(b)
    return float(np.linalg.norm(a - b) / (nb if nb > 0 else 1.0))


def rounded(a, dtype):
    """numpy float64 array holding exactly the values of ``a`` cast to dtype."""
    return torch.from_numpy(np.asarray(a, dtype=np.float64)).to(dtype).double().numpy()


def unfold(core3):
    Rk, Ik, Rk1 = core3.shape
    return np.ascontiguousarray(np.transpose(core3, (1, 2, 0)).reshape(Ik, Rk * Rk1))


def fold(G2, Rk, Rk1):
    return np.ascontiguousarray(G2.reshape(G2.shape[0], Rk1, Rk).transpose(2, 0, 1))


def to_dev(a, dtype):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype)


def flat_paper(X):
    """Paper-order (first index fastest) flat copy of a numpy tensor."""
    return np.asarray(X).reshape(-1, order="F")


def problem(seed, N, I, R, dtype, noise=0.2):
    """Cores and a target tensor, rounded to ``dtype`` (oracle inputs) and
    uploaded (GPU inputs)."""
    I = list(I) if not np.isscalar(I) else [int(I)] * N
    R = list(R) if not np.isscalar(R) else [int(R)] * N
    cores = [rounded(c, dtype) for c in ti.gaussian_cores(seed, N, I, R, scale=0.7)]
    X = tr.full_tensor(ti.gaussian_cores(seed + 1, N, I, R, scale=0.7))
    X = rounded(X + noise * ti.standard_normal(seed + 2, X.shape), dtype)
    dcores = [to_dev(unfold(c), dtype) for c in cores]
    dX = to_dev(flat_paper(X), dtype)
    return I, R, cores, X, dcores, dX
