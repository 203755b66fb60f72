"""Graph similarity of consecutive snapshots (Sec. 4, definition of the two metrics; Thm 4.1;
Cor. 4.1), in FP64.  Test infrastructure: nothing in the product imports this module.

* Edge similarity: rho_e = ||L_t - L_{t-1}||_F, a sum over the union of the two sparsity
  patterns (and the diagonal for L = D - W).
* (rho, k)-spectral similarity: rho_s = ||H_k^t - H_k^{t-1}||_F with H_k the orthogonal
  projector onto the first k eigenvectors of L.
* Estimate of rho_s from filtered signals (a reading; the paper gives the metric, not an
  estimator): the polynomial low-pass h with cut-off lambda stands in for H_k on both
  graphs, and Hutchinson's identity E ||M P||_F^2 = sigma^2 s ||M||_F^2 for P with i.i.d.
  entries of variance sigma^2 (s columns) gives
      rho_hat^2 = ||h(L_t) P - h(L_{t-1}) P||_F^2 / (sigma^2 s).

Thm 4.1 adds (1 + delta) p gamma to the CSC error when a fraction p of the features is
reused, with gamma = rho_s (or sqrt(2) rho_e / alpha through Cor. 4.1).  The refresh rule of
the dynamic method compares p * rho_hat with a budget.

Parity pins (tests/test_oracle_similarity.py): hand-computed edge distances, symmetry and the
triangle inequality, the exact matrix-function distance from dense eigendecompositions, the
estimator's mean over many probe draws, the projector distance of disjoint-clique graphs in
closed form, and Cor. 4.1 linking the two metrics.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from . import chebyshev, operator


def edge_distance(A1, A2) -> float:
    """||L(A2) - L(A1)||_F for two operators of the same kind (normalized adjacency or an
    ExplicitLaplacian)."""
    D = (operator.laplacian(A2) - operator.laplacian(A1)).tocsr()
    return float(np.sqrt(np.sum(np.asarray(D.data, dtype=np.float64) ** 2)))


def projector(A, k: int) -> np.ndarray:
    """H_k = U_k U_k^T from a dense eigendecomposition of L."""
    _, U = operator.dense_spectrum(A)
    return U[:, :k] @ U[:, :k].T


def spectral_distance(A1, A2, k: int) -> float:
    """||H_k(L2) - H_k(L1)||_F."""
    return float(np.linalg.norm(projector(A2, k) - projector(A1, k)))


def filter_distance_exact(A1, lmax1: float, a1, A2, lmax2: float, a2) -> float:
    """||h2(L2) - h1(L1)||_F from dense eigendecompositions (h_i = sum_j a_i[j] T_j)."""
    lam1, U1 = operator.dense_spectrum(A1)
    lam2, U2 = operator.dense_spectrum(A2)
    M1 = (U1 * chebyshev.response(a1, lam1, lmax1)) @ U1.T
    M2 = (U2 * chebyshev.response(a2, lam2, lmax2)) @ U2.T
    return float(np.linalg.norm(M2 - M1))


def filter_distance_estimate(A1, lmax1: float, a1, A2, lmax2: float, a2, P: np.ndarray,
                             sigma2: float) -> float:
    """Hutchinson estimate of ||h2(L2) - h1(L1)||_F with probes P (n x s)."""
    P = np.asarray(P, dtype=np.float64)
    Y1 = chebyshev.filter_recurrence(A1, lmax1, a1, P)
    Y2 = chebyshev.filter_recurrence(A2, lmax2, a2, P)
    return float(np.sqrt(np.sum((Y2 - Y1) ** 2) / (sigma2 * P.shape[1])))
