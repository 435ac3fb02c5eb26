"""Brute-force checkers used to pin the oracle: independent nodes / derivative matrix built from numpy's
polynomial routines, and the volume operator assembled densely by Kronecker products."""
from __future__ import annotations

import numpy as np


def np_nodes(n: int):
    """Gauss-Legendre nodes and weights on [0, 1] from numpy.polynomial.legendre.leggauss."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def np_dmatrix(n: int) -> np.ndarray:
    """D[i, j] = l_j'(xi_i), built from monomial coefficients of each Lagrange polynomial."""
    xi, _ = np_nodes(n)
    D = np.zeros((n, n))
    for j in range(n):
        others = np.delete(xi, j)
        coef = np.poly(others) / np.prod(xi[j] - others) if n > 1 else np.array([1.0])
        dcoef = np.polyder(coef) if n > 1 else np.array([0.0])
        D[:, j] = np.polyval(dcoef, xi)
    return D


def axis_operator(M: np.ndarray, axis: int, n: int) -> np.ndarray:
    """Kronecker form of applying M along spatial axis (0 = x fastest, 2 = z slowest) of node index
    (z*n + y)*n + x."""
    I = np.eye(n)
    mats = [I, I, I]  # order (z, y, x) in the Kronecker product
    mats[2 - axis] = M
    return np.kron(np.kron(mats[0], mats[1]), mats[2])


def dense_Vd(N: int, m: int, h: float, d: int, B3: np.ndarray, A3: np.ndarray | None = None,
             D: np.ndarray | None = None) -> np.ndarray:
    """Dense (n^3 m) x (n^3 m) matrix of V_d = -(1/h)[ (K_d x I_m) diag(A_d) + diag(B_d) (K_d x I_m) ].
    B3/A3: per-node matrices [3, n^3, m, m]."""
    n = N + 1
    nn = n ** 3
    if D is None:
        D = np_dmatrix(n)
    Kd = np.kron(axis_operator(D, d, n), np.eye(m))
    Bblk = np.zeros((nn * m, nn * m))
    for k in range(nn):
        Bblk[k * m:(k + 1) * m, k * m:(k + 1) * m] = B3[d, k]
    V = Bblk @ Kd
    if A3 is not None:
        Ablk = np.zeros((nn * m, nn * m))
        for k in range(nn):
            Ablk[k * m:(k + 1) * m, k * m:(k + 1) * m] = A3[d, k]
        V = V + Kd @ Ablk
    return -V / h


def dense_V(N, m, h, B3, A3=None, D=None):
    return sum(dense_Vd(N, m, h, d, B3, A3, D) for d in range(3))


def per_node_B(physics_B, params_nodes):
    """Stack preset matrices [3, m, m] per node into [3, n^3, m, m] using a callable physics_B(par)."""
    mats = np.stack([physics_B(p) for p in params_nodes], axis=1)
    return mats
