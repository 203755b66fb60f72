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

Parity pins (tests/test_oracle_adjoint.py): central finite differences in FP64, the
Daleckii-Krein divided-difference formula for the derivative of a matrix function, and
dl/dX = h(L~)^T G.
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
