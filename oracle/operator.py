"""Graph operators of Sec. 2.1, in FP64.

The graph is G = (V, E, W), simple, symmetric, with positive weights.  The normalized
Laplacian is L = I - D^{-1/2} W D^{-1/2} with D the diagonal degree matrix.  An isolated
node has degree 0; its D^{-1/2} entry is taken to be 0 (the paper does not cover this
case), so that its row of L is the identity row and its eigenvalue is 1.

Parity pins: the cycle graph (eigenvalues 1 - cos(2 pi j / n)) and disjoint cliques
(eigenvalue 0 with multiplicity k) in tests/test_oracle_operator.py.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def weight_matrix(n, rowptr, colidx, w) -> sp.csr_matrix:
    return sp.csr_matrix((np.asarray(w, dtype=np.float64), np.asarray(colidx, dtype=np.int64),
                          np.asarray(rowptr, dtype=np.int64)), shape=(n, n))


def degrees(W: sp.csr_matrix) -> np.ndarray:
    """d_i = sum_j W_ij."""
    return np.asarray(W.sum(axis=1)).ravel()


def inv_sqrt_degrees(deg: np.ndarray) -> np.ndarray:
    """D^{-1/2} with 0^{-1/2} := 0."""
    out = np.zeros_like(deg)
    pos = deg > 0
    out[pos] = 1.0 / np.sqrt(deg[pos])
    return out


def normalized_adjacency(n, rowptr, colidx, w) -> tuple[sp.csr_matrix, np.ndarray]:
    """A = D^{-1/2} W D^{-1/2} (same sparsity pattern and entry order as W) and D^{-1/2}."""
    W = weight_matrix(n, rowptr, colidx, w)
    dis = inv_sqrt_degrees(degrees(W))
    # A_ij = W_ij d_i^{-1/2} d_j^{-1/2}, on W's exact pattern and entry order
    A = sp.csr_matrix((np.asarray(W.data) * dis[np.repeat(np.arange(n), np.diff(W.indptr))]
                       * dis[W.indices], W.indices.copy(), W.indptr.copy()), shape=(n, n))
    return A, dis


def laplacian(A: sp.csr_matrix) -> sp.csr_matrix:
    """L = I - A."""
    n = A.shape[0]
    return (sp.identity(n, format="csr") - A).tocsr()


def scaled_laplacian(A: sp.csr_matrix, lmax: float) -> sp.csr_matrix:
    """L~ = (2 / lmax) L - I, which maps the spectrum [0, lmax] onto [-1, 1]."""
    n = A.shape[0]
    return ((2.0 / lmax) * laplacian(A) - sp.identity(n, format="csr")).tocsr()


def dense_spectrum(A: sp.csr_matrix) -> tuple[np.ndarray, np.ndarray]:
    """Eigenvalues (ascending) and orthonormal eigenvectors of L, by dense symmetric eigh."""
    L = laplacian(A).toarray()
    L = 0.5 * (L + L.T)
    lam, U = np.linalg.eigh(L)
    return lam, U


def isolated_count(n, rowptr) -> int:
    return int(np.sum(np.diff(np.asarray(rowptr)) == 0))
