"""Reverse-mode derivative of the Chebyshev filter Y = sum_j a_j T_j(L~) X.

The forward recurrence is Z_0 = X, Z_1 = L~ Z_0, Z_{j+1} = 2 L~ Z_j - Z_{j-1} and
Y = sum_j a_j Z_j, with L~ = alpha I - beta A, alpha = 2 / lmax - 1, beta = 2 / lmax.
Given G = dl/dY, the adjoints Zb_j = dl/dZ_j satisfy (Zb_{m+1} = Zb_{m+2} = 0)
    Zb_j = a_j G + 2 L~^T Zb_{j+1} - Zb_{j+2}   (j = m .. 1)
    Zb_0 = a_0 G +   L~^T Zb_1     - Zb_2,
and
    dl/dX   = Zb_0
    dl/da_j = <G, Z_j>
    dl/dL~  = Zb_1 Z_0^T + sum_{j=1..m-1} 2 Zb_{j+1} Z_j^T
    dl/dA   = -beta dl/dL~, read on A's stored entries (each directed entry its own
              parameter; lmax and the cut-off are held fixed).

The chain to the edge weights (normalized Laplacian, Sec. 2.1: A = D^{-1/2} W D^{-1/2},
d = W 1).  With s = d^{-1/2}, G_e = dl/dA_e and, for every node i,
    q_i = sum over the stored entries e of row i of  G_e A_e + G_m(e) A_m(e)
(m(e) the mirror entry (j, i) of e = (i, j)), an entry W_ij taken as its own parameter has
    dl/dW_ij = G_ij s_i s_j - q_i s_i^2 / 2,
because A_ab depends on W_ij directly (a = i, b = j) and through d_i (row i and column i of
A).  The weight of an undirected edge {i, j} is one parameter stored twice, so its gradient
is the sum over the pair: dl/dw_ij = dl/dW_ij + dl/dW_ji.

Parity pins (tests/test_oracle_adjoint.py): central finite differences in FP64, the
Daleckii-Krein divided-difference formula for the derivative of a matrix function, and
dl/dX = h(L~)^T G; for the weight chain, central finite differences of the loss through
A(W) with both stored copies of an edge weight moved together.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .chebyshev import filter_recurrence
from .operator import scaled_laplacian


def filter_backward(A: sp.csr_matrix, lmax: float, a: np.ndarray, X: np.ndarray,
                    G: np.ndarray):
    """Returns (dX, da, dA_vals) with dA_vals aligned to A.data."""
    A = sp.csr_matrix(A)
    Lt = scaled_laplacian(A, lmax)
    LtT = Lt.T.tocsr()
    beta = 2.0 / lmax
    G = np.asarray(G, dtype=np.float64)
    _, Z = filter_recurrence(A, lmax, a, X, return_iterates=True)
    m = len(a) - 1
    da = np.array([np.sum(G * Zj) for Zj in Z])
    Zb = [None] * (m + 3)
    zero = np.zeros_like(G)
    Zb[m + 1] = zero
    Zb[m + 2] = zero
    for j in range(m, 0, -1):
        Zb[j] = a[j] * G + 2.0 * (LtT @ Zb[j + 1]) - Zb[j + 2]
    Zb[0] = a[0] * G + (LtT @ Zb[1] if m >= 1 else zero) - (Zb[2] if m >= 2 else zero)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    cols = A.indices
    dLt = np.zeros(A.nnz)
    if m >= 1:
        dLt += np.einsum("ij,ij->i", Zb[1][rows], Z[0][cols])
        for j in range(1, m):
            dLt += 2.0 * np.einsum("ij,ij->i", Zb[j + 1][rows], Z[j][cols])
    return Zb[0], da, -beta * dLt


def mirror_index(n, rowptr, colidx) -> np.ndarray:
    """For every stored entry e = (i, j) of a structurally symmetric CSR pattern, the index of
    the entry (j, i)."""
    rowptr = np.asarray(rowptr, dtype=np.int64)
    colidx = np.asarray(colidx, dtype=np.int64)
    nnz = int(rowptr[-1])
    idx = sp.csr_matrix((np.arange(nnz, dtype=np.float64) + 1.0, colidx, rowptr), shape=(n, n))
    T = idx.T.tocsr()  # entry (i, j) of T holds 1 + the index of (j, i)
    T.sort_indices()
    return (T.data - 1.0).astype(np.int64)


def weight_gradient(n, rowptr, colidx, w, dA: np.ndarray) -> np.ndarray:
    """dl/dw per stored entry of W (the same value on (i, j) and (j, i)) from dl/dA_e, for
    the normalized Laplacian (module header)."""
    from .operator import normalized_adjacency

    A, s = normalized_adjacency(n, rowptr, colidx, w)
    dA = np.asarray(dA, dtype=np.float64)
    rows = np.repeat(np.arange(n), np.diff(np.asarray(rowptr, dtype=np.int64)))
    cols = np.asarray(colidx, dtype=np.int64)
    mir = mirror_index(n, rowptr, colidx)
    ga = dA * A.data
    q = np.zeros(n)
    np.add.at(q, rows, ga + ga[mir])
    g = dA * s[rows] * s[cols] - 0.5 * q[rows] * s[rows] ** 2
    return g + g[mir]
