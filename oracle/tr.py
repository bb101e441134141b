"""Tensor-ring algebra in plain numpy, FP64 (CPU oracle; test infrastructure).

Everything is 0-based.  A tensor X of shape (I_1, ..., I_N) is a numpy array
indexed X[i_1, ..., i_N]; linear multi-indices put the first index fastest
(Definition "Multi-index").  A core is a numpy array core[r, i, s] of shape
(R_k, I_k, R_{k+1}) with R_{N+1} = R_1 (tensor-ring format of Section 1).

Layouts fixed by the paper's definitions:

* Classical mode-2 unfolding of a core, G_{k(2)} (I_k x R_k R_{k+1}):
  G_{k(2)}[i, r + R_k*s] = core[r, i, s].
* Cyclic mode-n unfolding X_[n] (Definition "Mode-n Unfolding"): row i_n,
  column = multi-index of (i_{n+1}, ..., i_N, i_1, ..., i_{n-1}).
* Subchain tensor G^{!=n} (Definition "Subchain Tensor"), shape
  (R_{n+1}, J_n, R_n), the subchain product of the cores n+1, ..., N, 1, ...,
  n-1; its cyclic mode-2 unfolding G^{!=n}_[2] (J_n x R_n R_{n+1}) has
  G^{!=n}_[2][j, r + R_n*s] = G^{!=n}[s, j, r].

With these, X_[n] = G_{n(2)} (G^{!=n}_[2])^T  (the per-block least-squares
form of the objective in Section 2).
"""
from __future__ import annotations

import itertools

import numpy as np

__all__ = [
    "ranks_of", "sizes_of", "cyclic_order", "core_unfold2", "core_fold2",
    "subchain_product", "slices_hadamard", "subchain_tensor", "subchain_unfold2",
    "unfold_cyclic", "unfold_classical", "fold_cyclic", "full_tensor",
    "entry_by_trace", "full_tensor_by_trace", "objective", "full_gradient",
    "full_hessian_block", "rse", "multi_index", "cyclic_column",
]


def ranks_of(cores):
    """R_1..R_N (left ranks)."""
    return [c.shape[0] for c in cores]


def sizes_of(cores):
    return [c.shape[1] for c in cores]


def cyclic_order(N: int, n: int):
    """Modes n+1, ..., N, 1, ..., n-1 (0-based: n+1..N-1, 0..n-1)."""
    return [(n + d) % N for d in range(1, N)]


def core_unfold2(core: np.ndarray) -> np.ndarray:
    """Classical mode-2 unfolding G_{k(2)}: [i, r + R_k*s] = core[r, i, s]."""
    Rk, Ik, Rk1 = core.shape
    return core.transpose(1, 2, 0).reshape(Ik, Rk * Rk1)


def core_fold2(G2: np.ndarray, Rk: int, Rk1: int) -> np.ndarray:
    """Inverse of ``core_unfold2``."""
    Ik = G2.shape[0]
    return np.ascontiguousarray(G2.reshape(Ik, Rk1, Rk).transpose(2, 0, 1))


def multi_index(idx, sizes) -> int:
    """Linear index of (i_1..i_K) with the first index fastest."""
    lin, stride = 0, 1
    for i, s in zip(idx, sizes):
        lin += int(i) * stride
        stride *= int(s)
    return lin


def cyclic_column(idx, sizes, n: int) -> int:
    """Column of X_[n] that holds the fiber through multi-index ``idx``."""
    N = len(sizes)
    order = cyclic_order(N, n)
    return multi_index([idx[k] for k in order], [sizes[k] for k in order])


def subchain_product(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Mode-2 subchain product (Definition "Subchain Product").

    A: (I1, J1, K), B: (K, J2, I2) -> (I1, J1*J2, I2) whose lateral slice at
    the multi-index j1 + J1*j2 is A(j1) @ B(j2).
    """
    I1, J1, K = A.shape
    K2, J2, I2 = B.shape
    assert K == K2
    # every pair (j1, j2) at once: T[a, j2, j1, b] = sum_k A[a, j1, k] B[k, j2, b],
    # and the (j2, j1) axes flattened with j1 fastest give the multi-index
    T = np.einsum("ajk,kcb->acjb", A, B)
    return T.reshape(I1, J2 * J1, I2)


def slices_hadamard(A: np.ndarray, B: np.ndarray) -> np.ndarray:
    """Mode-2 slices-Hadamard product (Definition "Slices-Hadamard Product"):
    lateral slice j of the result is A(j) @ B(j)."""
    assert A.shape[1] == B.shape[1] and A.shape[2] == B.shape[0]
    return np.einsum("ajk,kjb->ajb", A, B)


def subchain_tensor(cores, n: int) -> np.ndarray:
    """G^{!=n} = G_{n+1} [x] ... [x] G_N [x] G_1 [x] ... [x] G_{n-1}."""
    order = cyclic_order(len(cores), n)
    T = cores[order[0]]
    for k in order[1:]:
        T = subchain_product(T, cores[k])
    return T


def subchain_unfold2(cores, n: int) -> np.ndarray:
    """G^{!=n}_[2] (J_n x R_n R_{n+1}); [j, r + R_n*s] = G^{!=n}[s, j, r]."""
    T = subchain_tensor(cores, n)         # (R_{n+1}, J_n, R_n)
    Rn1, Jn, Rn = T.shape
    return T.transpose(1, 0, 2).reshape(Jn, Rn1 * Rn)   # [j, s, r] -> s*Rn + r


def unfold_cyclic(X: np.ndarray, n: int) -> np.ndarray:
    """X_[n] (Definition "Mode-n Unfolding")."""
    N = X.ndim
    axes = [n] + cyclic_order(N, n)
    Y = X.transpose(axes)
    return Y.reshape(X.shape[n], -1, order="F")


def fold_cyclic(Xn: np.ndarray, n: int, sizes) -> np.ndarray:
    """Inverse of ``unfold_cyclic``."""
    N = len(sizes)
    axes = [n] + cyclic_order(N, n)
    Y = Xn.reshape([sizes[a] for a in axes], order="F")
    return np.ascontiguousarray(Y.transpose(np.argsort(axes)))


def unfold_classical(X: np.ndarray, n: int) -> np.ndarray:
    """X_(n) (Definition "Classical Mode-n Unfolding")."""
    N = X.ndim
    axes = [n] + [k for k in range(N) if k != n]
    return X.transpose(axes).reshape(X.shape[n], -1, order="F")


def full_tensor(cores) -> np.ndarray:
    """TR(cores) through X_[1] = G_{1(2)} (G^{!=1}_[2])^T."""
    sizes = sizes_of(cores)
    X1 = core_unfold2(cores[0]) @ subchain_unfold2(cores, 0).T
    return fold_cyclic(X1, 0, sizes)


def entry_by_trace(cores, idx) -> float:
    """X(i_1..i_N) = Trace(G_1(i_1) ... G_N(i_N)) with explicit loops."""
    M = None
    for k, i in enumerate(idx):
        S = cores[k][:, int(i), :]
        if M is None:
            M = S.copy()
        else:
            Rm, Rk = M.shape
            Rk2, Rn = S.shape
            assert Rk == Rk2
            P = np.zeros((Rm, Rn))
            for a in range(Rm):
                for b in range(Rn):
                    acc = 0.0
                    for c in range(Rk):
                        acc += M[a, c] * S[c, b]
                    P[a, b] = acc
            M = P
    return float(sum(M[d, d] for d in range(M.shape[0])))


def full_tensor_by_trace(cores) -> np.ndarray:
    sizes = sizes_of(cores)
    X = np.empty(sizes)
    for idx in itertools.product(*[range(s) for s in sizes]):
        X[idx] = entry_by_trace(cores, idx)
    return X


def objective(cores, X) -> float:
    """f = 1/2 ||TR(cores) - X||_F^2 (objective of Section 2)."""
    D = full_tensor(cores) - X
    return 0.5 * float(np.sum(D * D))


def full_gradient(cores, X, n: int) -> np.ndarray:
    """Full block gradient (equation ``eq:gradient``):
    G_{n(2)} Gs^T Gs - X_[n] Gs with Gs = G^{!=n}_[2]."""
    Gs = subchain_unfold2(cores, n)
    Gn = core_unfold2(cores[n])
    return Gn @ (Gs.T @ Gs) - unfold_cyclic(X, n) @ Gs


def full_hessian_block(cores, n: int) -> np.ndarray:
    """Gs^T Gs, the factor of the n-th diagonal Hessian block
    (equation ``eq:hessian``: Gs^T Gs kron I_{I_n})."""
    Gs = subchain_unfold2(cores, n)
    return Gs.T @ Gs


def rse(cores, X_true) -> float:
    """Relative square error ||TR(cores) - X_true||_F / ||X_true||_F
    (evaluation measure of Section 4)."""
    D = full_tensor(cores) - X_true
    return float(np.sqrt(np.sum(D * D)) / np.sqrt(np.sum(X_true * X_true)))
