"""Chebyshev approximation of the ideal low-pass filter (Sec. 2.2, Sec. 3.2).

The ideal filter H_k keeps the first k eigenvectors: its response is the step
g(lambda) = 1[lambda <= lambda_c] with the cut-off between lambda_k and lambda_{k+1}.
It is replaced by a degree-m polynomial h(lambda) = sum_{j=0..m} a_j T_j(x) with
x = 2 lambda / lmax - 1 (Sec. 3.2 and the cost O(|E| d m) of Sec. 2.2).

Readings where the paper is silent
  * coefficients are those of the Chebyshev series of the step, truncated at degree m,
    with the "folded" convention a_0 = c_0 / 2 (so h = sum a_j T_j);
  * optional Jackson damping multiplies a_j by the Jackson kernel g_j (Weisse et al.,
    Rev. Mod. Phys. 78, 2006), which keeps h inside [0, 1] and monotone in lambda_c;
  * "order m" means degree m: m + 1 coefficients and m products with the operator.

Parity pins (tests/test_oracle_chebyshev.py): the closed form against numerical
quadrature of the Chebyshev projection integral, the special cut-offs lambda_c = lmax
(h = 1) and lambda_c = 0 (h = 0), Jackson g_0 = 1 and range/monotonicity, the
recurrence against the dense identity U h(Lambda) U^T X and the cycle graph's Fourier
eigenvectors, and the error bound eq. (static_filtering).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .operator import scaled_laplacian


def jackson_damping(m: int) -> np.ndarray:
    """Jackson kernel g_0..g_m for a degree-m expansion."""
    j = np.arange(m + 1, dtype=np.float64)
    M = m + 2.0
    return ((M - j) * np.cos(np.pi * j / M) + np.sin(np.pi * j / M) / np.tan(np.pi / M)) / M


def step_coefficients(m: int, lmax: float, lam_c: float, damping: str = "jackson") -> np.ndarray:
    """Folded Chebyshev coefficients of g(lambda) = 1[lambda <= lam_c] on [0, lmax].

    With x = 2 lambda / lmax - 1 = cos(theta), the step is 1[theta >= theta_c] where
    theta_c = arccos(2 lam_c / lmax - 1).  The series coefficients are
    c_j = (2 / pi) * int_{theta_c}^{pi} cos(j theta) d theta, hence
    a_0 = c_0 / 2 = 1 - theta_c / pi and a_j = -2 sin(j theta_c) / (j pi).
    """
    if m < 0:
        raise ValueError("m must be >= 0")
    x_c = np.clip(2.0 * lam_c / lmax - 1.0, -1.0, 1.0)
    th = np.arccos(x_c)
    a = np.empty(m + 1, dtype=np.float64)
    a[0] = 1.0 - th / np.pi
    j = np.arange(1, m + 1, dtype=np.float64)
    a[1:] = -2.0 * np.sin(j * th) / (j * np.pi)
    if damping == "jackson":
        a *= jackson_damping(m)
    elif damping != "none":
        raise ValueError(damping)
    return a


def cheb_eval(a: np.ndarray, x) -> np.ndarray:
    """sum_j a_j T_j(x) with T_j(x) = cos(j arccos x), for x in [-1, 1]."""
    x = np.clip(np.asarray(x, dtype=np.float64), -1.0, 1.0)
    th = np.arccos(x)
    j = np.arange(len(a), dtype=np.float64)
    return np.cos(np.multiply.outer(th, j)) @ a


def response(a: np.ndarray, lam, lmax: float) -> np.ndarray:
    """h(lambda) for eigenvalues lambda of L."""
    return cheb_eval(a, 2.0 * np.asarray(lam, dtype=np.float64) / lmax - 1.0)


def filter_recurrence(A: sp.csr_matrix, lmax: float, a: np.ndarray, X: np.ndarray,
                      return_iterates: bool = False):
    """Y = sum_j a_j T_j(L~) X by the three-term recurrence
    Z_0 = X, Z_1 = L~ X, Z_{j+1} = 2 L~ Z_j - Z_{j-1}."""
    Lt = scaled_laplacian(A, lmax)
    X = np.asarray(X, dtype=np.float64)
    m = len(a) - 1
    Z_prev = X
    Y = a[0] * Z_prev
    iters = [Z_prev]
    if m >= 1:
        Z = Lt @ X
        Y = Y + a[1] * Z
        iters.append(Z)
        for j in range(1, m):
            Z_next = 2.0 * (Lt @ Z) - Z_prev
            Y = Y + a[j + 1] * Z_next
            Z_prev, Z = Z, Z_next
            iters.append(Z)
    if return_iterates:
        return Y, iters
    return Y


def filter_dense(lam: np.ndarray, U: np.ndarray, a: np.ndarray, lmax: float,
                 X: np.ndarray) -> np.ndarray:
    """U h(Lambda) U^T X from a full eigendecomposition of L."""
    h = response(a, lam, lmax)
    return U @ (h[:, None] * (U.T @ X))


def ideal_lowpass(U: np.ndarray, k: int, X: np.ndarray) -> np.ndarray:
    """Psi = H_k X = U_k U_k^T X (eq. Hk)."""
    Uk = U[:, :k]
    return Uk @ (Uk.T @ X)


def static_filtering_bound(lam: np.ndarray, a: np.ndarray, lmax: float, k: int,
                           X: np.ndarray) -> float:
    """Right side of eq. (static_filtering): ||h(Lambda) - I_{n x k} I_{k x n}||_2 ||X||_F."""
    h = response(a, lam, lmax)
    ideal = np.zeros_like(h)
    ideal[:k] = 1.0
    return float(np.max(np.abs(h - ideal)) * np.linalg.norm(X))
