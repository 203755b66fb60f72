"""Compressive k-means (Sec. 2.2, Step 2), in FP64.  Test infrastructure only.

Instead of clustering all n feature rows, cluster a random subset of nodes and infer the
other assignments by Tikhonov-regularised interpolation of the k cluster indicators.  The
paper only outlines the step (a sample of O(k log k) nodes from a variable-density
distribution, Tikhonov interpolation costing graph filterings); the readings taken here,
after Puy et al. (random sampling of bandlimited graph signals, 2016) and Tremblay et al.
(compressive spectral clustering, 2016):

  * sampling density p_i = ||theta_i||^2 / ||Theta||_F^2 (the features estimate the local
    coherence ||U_k^T delta_i||^2), n' i.i.d. draws with replacement, node i drawn for a
    uniform u when C_{i-1} <= u W < C_i with C the prefix sums of ||theta_i||^2 and W = C_n;
  * k-means (k-means++ then Lloyd) on the n' sampled rows;
  * interpolation of each reduced indicator y_j (y_j[s] = 1 if sample s is in cluster j):
        x_j = argmin_x ||P^{-1/2} (M x - y_j)||^2 + gamma x^T L^r x,
    i.e. (M^T P^{-1} M + gamma L^r) x_j = M^T P^{-1} y_j, where M selects the sampled rows
    and P = diag(n' p_{omega_s}) (so M^T P^{-1} M is diagonal, sum over a node's draws of
    1 / (n' p_i));
  * node i is assigned to argmax_j x_j[i] (ties to the lowest j).

The exact minimiser is computed by a dense linear solve (small n only).

Parity pins (tests/test_oracle_compressive.py): the inverse-CDF draw by hand and its
frequencies, the interpolation of a clique indicator on a regular graph (exact: the
indicator lies in the null space of L and matches every sample), the optimality condition,
gamma -> 0 reproducing the samples, and agreement with full k-means on a separable SBM.
"""

from __future__ import annotations

import numpy as np

from . import kmeans, operator


def sampling_weights(F: np.ndarray) -> np.ndarray:
    """||theta_i||^2 per row."""
    F = np.asarray(F, dtype=np.float64)
    return np.sum(F * F, axis=1)


def draw(weights: np.ndarray, u: np.ndarray) -> np.ndarray:
    """Inverse-CDF draws: node i for each u with C_{i-1} <= u W < C_i."""
    C = np.cumsum(np.asarray(weights, dtype=np.float64))
    return np.searchsorted(C, np.asarray(u) * C[-1], side="right").astype(np.int64)


def interpolation_system(A, idx: np.ndarray, weights: np.ndarray, r: int, gamma: float):
    """Diagonal of M^T P^{-1} M (length n) and the dense matrix gamma L^r."""
    n = A.shape[0]
    p = np.asarray(weights, dtype=np.float64) / np.sum(weights)
    s = np.zeros(n)
    np.add.at(s, idx, 1.0 / (len(idx) * p[idx]))
    L = operator.laplacian(A).toarray()
    Lr = np.linalg.matrix_power(L, r)
    return s, gamma * Lr, p


def interpolate(A, idx: np.ndarray, weights: np.ndarray, labels_s: np.ndarray, k: int, r: int,
                gamma: float) -> np.ndarray:
    """X (n x k): column j solves (M^T P^{-1} M + gamma L^r) x = M^T P^{-1} y_j."""
    n = A.shape[0]
    s, G, p = interpolation_system(A, idx, weights, r, gamma)
    B = np.zeros((n, k))
    np.add.at(B, (idx, np.asarray(labels_s, dtype=np.int64)), 1.0 / (len(idx) * p[idx]))
    return np.linalg.solve(np.diag(s) + G, B)


def compressive_kmeans(A, F: np.ndarray, k: int, n_sample: int, u_sample: np.ndarray,
                       u_seed: np.ndarray, lloyd_iters: int, r: int, gamma: float):
    """Labels of all n nodes, plus the intermediate results (samples, their labels, X)."""
    w = sampling_weights(F)
    idx = draw(w, u_sample[:n_sample])
    Fs = np.asarray(F, dtype=np.float64)[idx]
    C0 = Fs[kmeans.kmeanspp(Fs, k, u_seed)]
    lab_s, _, _ = kmeans.lloyd(Fs, C0, lloyd_iters)
    X = interpolate(A, idx, w, lab_s, k, r, gamma)
    return np.argmax(X, axis=1).astype(np.int32), idx, lab_s, X
