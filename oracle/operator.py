"""Graph operators of Sec. 2.1, in FP64.

The graph is G = (V, E, W), simple, symmetric, with positive weights.  The normalized
Laplacian is L = I - D^{-1/2} W D^{-1/2} with D the diagonal degree matrix.  An isolated
node has degree 0; its D^{-1/2} entry is taken to be 0 (the paper does not cover this
case), so that its row of L is the identity row and its eigenvalue is 1.

The combinatorial Laplacian L = D - W (Sec. 2.1 names it beside the normalized one) has
no fixed spectral bound; the bound used with it is Anderson and Morley's
lambda_max(L) <= max over edges (i, j) of d_i + d_j (Linear Multilinear Algebra 18, 1985).

Every function of the oracle that takes the normalized adjacency A (L = I - A) also takes
an ExplicitLaplacian, which carries L itself.

Parity pins (tests/test_oracle_chebyshev.py, tests/test_oracle_laplacian.py): the cycle
graph (normalized eigenvalues 1 - cos(2 pi j / n), combinatorial 2 - 2 cos(2 pi j / n)),
disjoint cliques (eigenvalue 0 with multiplicity k; combinatorial eigenvalue s on the rest),
the star graph and regular bipartite graphs where the Anderson-Morley bound is attained.
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


class ExplicitLaplacian:
    """A Laplacian given as a matrix, accepted in place of the normalized adjacency."""

    def __init__(self, L: sp.csr_matrix):
        self.L = sp.csr_matrix(L, dtype=np.float64)
        self.shape = self.L.shape


def combinatorial_laplacian(n, rowptr, colidx, w) -> ExplicitLaplacian:
    """L = D - W."""
    W = weight_matrix(n, rowptr, colidx, w)
    return ExplicitLaplacian((sp.diags(degrees(W)) - W).tocsr())


def anderson_morley_bound(n, rowptr, colidx, w) -> float:
    """max over stored entries (i, j) of d_i + d_j, an upper bound of lambda_max(D - W); 0
    for a graph without edges."""
    W = weight_matrix(n, rowptr, colidx, w)
    if W.nnz == 0:
        return 0.0
    deg = degrees(W)
    rows = np.repeat(np.arange(n), np.diff(W.indptr))
    return float(np.max(deg[rows] + deg[W.indices]))


def laplacian(A) -> sp.csr_matrix:
    """L = I - A, or the matrix an ExplicitLaplacian carries."""
    if isinstance(A, ExplicitLaplacian):
        return A.L
    n = A.shape[0]
    return (sp.identity(n, format="csr") - A).tocsr()


def scaled_laplacian(A, lmax: float) -> sp.csr_matrix:
    """L~ = (2 / lmax) L - I, which maps the spectrum [0, lmax] onto [-1, 1]."""
    n = A.shape[0]
    return ((2.0 / lmax) * laplacian(A) - sp.identity(n, format="csr")).tocsr()


def dense_spectrum(A) -> tuple[np.ndarray, np.ndarray]:
    """Eigenvalues (ascending) and orthonormal eigenvectors of L, by dense symmetric eigh."""
    L = laplacian(A).toarray()
    L = 0.5 * (L + L.T)
    lam, U = np.linalg.eigh(L)
    return lam, U


def isolated_count(n, rowptr) -> int:
    return int(np.sum(np.diff(np.asarray(rowptr)) == 0))
