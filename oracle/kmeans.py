"""k-means on the rows of a feature matrix (Sec. 2.1).

The k-means problem of eq. (SC_cost) looks for the indicator matrix X minimising
||F - X X^T F||_F; its value C(X; F) is the square root of the usual sum of squared
distances to the cluster means.  The paper fixes no solver; the readings used here:
  * assignment: label_i = argmin_c sum_t (f_it - mu_ct)^2 in the direct form, exact ties
    to the lowest centroid index;
  * update: the mean of the rows assigned to a cluster; an empty cluster keeps its
    previous centroid;
  * seeding: k-means++ (Arthur and Vassilvitskii, 2007) with caller-supplied uniforms:
    the first centre is row floor(u_0 n); centre j is the first row i whose cumulative
    squared distance to the chosen centres exceeds u_j times the total;
  * Lloyd: a fixed number of assign/update rounds.

Parity pins (tests/test_oracle_kmeans.py): brute force over all assignments of tiny
inputs, the cost identity ||F - X X^T F||_F = sqrt(sum of squared distances to the
means), monotone Lloyd objective, and well separated clusters recovered exactly.
"""

from __future__ import annotations

import numpy as np


def sq_distances(F: np.ndarray, C: np.ndarray) -> np.ndarray:
    """D2[i, c] = sum_t (F[i, t] - C[c, t])^2, direct form in FP64."""
    F = np.asarray(F, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    out = np.empty((F.shape[0], C.shape[0]))
    for c in range(C.shape[0]):
        diff = F - C[c]
        out[:, c] = np.sum(diff * diff, axis=1)
    return out


def assign(F: np.ndarray, C: np.ndarray):
    """Labels (lowest index on exact ties) and the squared distance to the chosen centroid."""
    D2 = sq_distances(F, C)
    lab = np.argmin(D2, axis=1)  # argmin returns the first minimum
    return lab.astype(np.int32), D2[np.arange(D2.shape[0]), lab]


def update(F: np.ndarray, labels: np.ndarray, C_prev: np.ndarray):
    """Cluster means; an empty cluster keeps its previous centroid.  Returns (C, counts)."""
    F = np.asarray(F, dtype=np.float64)
    k = C_prev.shape[0]
    counts = np.bincount(labels, minlength=k)
    sums = np.zeros((k, F.shape[1]))
    np.add.at(sums, labels, F)
    C = np.array(C_prev, dtype=np.float64, copy=True)
    nz = counts > 0
    C[nz] = sums[nz] / counts[nz, None]
    return C, counts


def kmeanspp(F: np.ndarray, k: int, u: np.ndarray):
    """k-means++ seeding driven by the uniforms u_0..u_{k-1} in [0, 1).

    Returns the chosen row indices.
    """
    F = np.asarray(F, dtype=np.float64)
    n = F.shape[0]
    idx = [min(int(np.floor(u[0] * n)), n - 1)]
    d2 = np.sum((F - F[idx[0]]) ** 2, axis=1)
    for j in range(1, k):
        cs = np.cumsum(d2)
        total = cs[-1]
        if total <= 0.0:
            nxt = idx[-1]
        else:
            nxt = int(np.searchsorted(cs, u[j] * total, side="right"))
            nxt = min(nxt, n - 1)
        idx.append(nxt)
        d2 = np.minimum(d2, np.sum((F - F[nxt]) ** 2, axis=1))
    return np.array(idx, dtype=np.int64)


def lloyd(F: np.ndarray, C0: np.ndarray, iters: int):
    """``iters`` rounds of (assign, update), then a final assignment.

    Returns (labels, centroids, objective per round) where the objective is the sum of
    squared distances of each assignment.
    """
    C = np.array(C0, dtype=np.float64)
    obj = []
    for _ in range(iters):
        lab, d2 = assign(F, C)
        obj.append(float(np.sum(d2)))
        C, _ = update(F, lab, C)
    lab, d2 = assign(F, C)
    obj.append(float(np.sum(d2)))
    return lab, C, obj


def indicator(labels: np.ndarray, k: int) -> np.ndarray:
    """X_ij = 1 / sqrt(s_j) if i is in cluster j, else 0 (s_j the cluster size)."""
    n = labels.shape[0]
    X = np.zeros((n, k))
    counts = np.bincount(labels, minlength=k)
    for j in range(k):
        if counts[j] > 0:
            X[labels == j, j] = 1.0 / np.sqrt(counts[j])
    return X


def cost(Phi: np.ndarray, labels: np.ndarray) -> float:
    """C(X; Phi) = sqrt(sum_c sum_{i in c} ||phi_i - mean_c phi||^2)."""
    Phi = np.asarray(Phi, dtype=np.float64)
    total = 0.0
    for c in np.unique(labels):
        rows = Phi[labels == c]
        total += float(np.sum((rows - rows.mean(axis=0)) ** 2))
    return float(np.sqrt(total))
