"""Eigencount and the dichotomy on lambda_k (Sec. 3.2 and Sec. 4.1).

The number of eigenvalues below a cut-off lambda is estimated from filtered random
signals: with probes P (n x n_s, i.i.d. entries of variance sigma^2),
    c(lambda) = (1 / (sigma^2 n_s)) * sum_s p_s^T h_lambda(L) p_s,
Hutchinson's estimator of trace h_lambda(L), where h_lambda is the polynomial filter
with cut-off lambda.  The dichotomy halves a bracket [lo, hi] a fixed number of times,
moving lo up when c(mid) < k and hi down otherwise, and returns hi.

Two equivalent ways to evaluate c(lambda) for many cut-offs with the same probes:
  * literal: filter P at every candidate and take <P, h_lambda(L) P>;
  * moments: mu_j = sum_s p_s^T T_j(L~) p_s once, then c = sum_j a_j(lambda) mu_j / (sigma^2 n_s).
The doubling identities T_j^2 = (T_{2j} + T_0) / 2 and T_{j+1} T_j = (T_{2j+1} + T_1) / 2
give mu_0..mu_{2J+1} from J + 1 products of the operator (L~ symmetric).

Readings where the paper is silent: the estimator is Hutchinson's quadratic form; the
same probes serve every candidate; the bisection takes a fixed number of steps with no
early exit; the dynamic refinement uses a one-sided bracket starting at the previous
cut-off; acceptance is |c - k| <= tau.

Parity pins (tests/test_oracle_eigcount.py): literal vs moments, doubled vs direct
moments, the exact trace tr(P^T U h(Lambda) U^T P) from a dense eigendecomposition, the
true count #{lambda_i <= lambda} within its deterministic and statistical bounds, and
monotonicity of the damped count in lambda.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .chebyshev import filter_recurrence, step_coefficients
from .operator import scaled_laplacian


def moments_direct(A: sp.csr_matrix, lmax: float, m: int, P: np.ndarray) -> np.ndarray:
    """mu_j = <P, T_j(L~) P> (summed over probe columns) for j = 0..m."""
    _, iters = filter_recurrence(A, lmax, np.zeros(m + 1), P, return_iterates=True)
    P = np.asarray(P, dtype=np.float64)
    return np.array([np.sum(P * Z) for Z in iters])


def moments_doubled(A: sp.csr_matrix, lmax: float, m: int, P: np.ndarray) -> np.ndarray:
    """mu_0..mu_m from floor(m / 2) + 1 operator products using the doubling identities."""
    Lt = scaled_laplacian(A, lmax)
    P = np.asarray(P, dtype=np.float64)
    J = m // 2
    mu = np.zeros(2 * J + 2)
    Z_prev = P
    Z = Lt @ P
    mu[0] = np.sum(P * P)
    mu[1] = np.sum(Z * P)
    for j in range(1, J + 1):
        # Z holds T_j P, Z_prev holds T_{j-1} P
        Z_next = 2.0 * (Lt @ Z) - Z_prev
        mu[2 * j] = 2.0 * np.sum(Z * Z) - mu[0]
        mu[2 * j + 1] = 2.0 * np.sum(Z_next * Z) - mu[1]
        Z_prev, Z = Z, Z_next
    return mu[: m + 1]


def count_from_moments(a: np.ndarray, mu: np.ndarray, sigma2: float, n_s: int) -> float:
    return float(np.dot(a, mu[: len(a)]) / (sigma2 * n_s))


def count_literal(A, lmax: float, a: np.ndarray, P: np.ndarray, sigma2: float) -> float:
    """<P, h(L) P> / (sigma^2 n_s), filtering the probes at this cut-off."""
    Y = filter_recurrence(A, lmax, a, P)
    return float(np.sum(np.asarray(P, dtype=np.float64) * Y) / (sigma2 * P.shape[1]))


def bisect(count_fn, k: float, lo: float, hi: float, steps: int):
    """Fixed-step dichotomy: mid = (lo + hi) / 2; c(mid) < k -> lo = mid else hi = mid.

    Returns (lambda_c = hi, c(hi), trace) where trace lists (mid, c(mid)) per step.
    """
    trace = []
    for _ in range(steps):
        mid = 0.5 * (lo + hi)
        c = count_fn(mid)
        trace.append((mid, c))
        if c < k:
            lo = mid
        else:
            hi = mid
    return hi, count_fn(hi), trace


def eigcount_bisect(mu: np.ndarray, m: int, lmax: float, damping: str, sigma2: float,
                    n_s: int, k: float, steps: int, lo: float, hi: float):
    """Dichotomy for lambda_k driven by precomputed moments mu_0..mu_m."""
    def c(lam):
        return count_from_moments(step_coefficients(m, lmax, lam, damping), mu, sigma2, n_s)
    return bisect(c, k, lo, hi, steps)


def accept_tolerance(k: int, n_s: int) -> float:
    """tau = max(0.5, 2 sqrt(2 k / n_s)): twice the standard deviation of Hutchinson's
    estimator on a rank-k projector with n_s Gaussian probes."""
    return max(0.5, 2.0 * np.sqrt(2.0 * k / n_s))
