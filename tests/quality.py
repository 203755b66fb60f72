"""Clustering quality of static CSC against SC (Thm 3.1, Lemma 3.1 and Thm 3.2 of Sec. 3.1).

Shared by the CPU pins (tests/test_oracle_theory.py) and the GPU test
(tests/test_gpu_quality.py).  With Phi = U_k the first k eigenvectors of L, the cost of an
assignment is C(X; Phi) = ||Phi - X X^T Phi||_F (eq. CSC_cost); C_Phi is SC's own cost, here
the best of 50 seeded k-means++ restarts of Lloyd on Phi (k-means is a heuristic, so the
optimum of the theorems is approximated from above).  For features Psi~ of d filtered
signals R, three checks:
  * Thm 3.1 at t = 3 (probability >= 1 - e^{-4.5}): C <= C_Phi + 2 sqrt(k/d)(sqrt(k) + 3).
    Every assignment has C <= ||Phi||_F = sqrt(k), so the bound says nothing when it is at
    least sqrt(k) (k = 5: for every d < 55); it is informative at d = 256 (2.13 < 2.24).
  * Lemma 3.1's deterministic chain with the ideal features Psi = H_k R and Thm 3.2's
    equality ||Psi - Phi I Q||_F = ||Sigma - I||_F (Sigma the singular values of U_k^T R):
    C <= C_Phi + 2 (||Psi~ - Psi||_F + ||Sigma - I||_F).
  * the assignment is as good as the oracle's static CSC on the same signals: C <= C_oracle +
    0.05.  Thm 3.1 speaks of optimal k-means; both sides approximate it by the best of
    RESTARTS seeded k-means++ + 20 Lloyd runs (lowest k-means objective on the features),
    because a single run can stop in a local optimum that merges two clusters (C near 1.1
    instead of 0.67 on C1) on features of either precision.  Features of another precision
    can still reach another optimum of nearly the same cost, hence the slack; the wrong
    assignments below cost at least 0.35 more than SC's 0.67 on C1.
A random labelling, two clusters merged, or half of a cluster moved fails at least one.
"""

from __future__ import annotations

import numpy as np

from oracle import chebyshev, kmeans, operator, philox
from workloads import sbm, seed_for

K = 5
M = 50
RESTARTS = 8


def c1_graph():
    """The C1 graph: SBM N = 1000, k = 5 equal blocks, degree 16, ratio 0.1."""
    return sbm(1000, K, 16.0, 0.1, seed=seed_for(1, "graph"))


def sc_reference(g, restarts: int = 50):
    """(A, eigenvalues, Phi = U_k, C_Phi) from a dense eigendecomposition."""
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    lam, U = operator.dense_spectrum(A)
    Phi = U[:, :K]
    best = np.inf
    for s in range(restarts):
        u = philox.uniforms(K, seed_for(1, "kmeans"), 1000 + s)
        lab, _, _ = kmeans.lloyd(Phi, Phi[kmeans.kmeanspp(Phi, K, u)], 30)
        best = min(best, kmeans.cost(Phi, lab))
    return A, lam, U, best


def signals(n: int, d: int, store: str) -> np.ndarray:
    """The d signals of variance 1/d both sides draw (Philox stream 1), as stored."""
    return np.asarray(philox.gaussian_block(n, d, 1 / np.sqrt(d), seed_for(1, "signals"), 1,
                                            dtype="bf16" if store == "bf16" else np.float32),
                      dtype=np.float64)


def kmeans_stream(r: int) -> int:
    """Philox stream of the k-means++ uniforms of restart r (both sides)."""
    return 2 + 16 * r


def oracle_csc(A, lam_c: float, R: np.ndarray):
    """Static CSC in the oracle: filter at lam_c, then the best (lowest objective) of RESTARTS
    runs of k-means++ (Philox streams kmeans_stream(r)) + 20 Lloyd rounds."""
    a = chebyshev.step_coefficients(M, 2.0, lam_c, "jackson")
    Y = chebyshev.filter_recurrence(A, 2.0, a, R)
    best, best_obj = None, np.inf
    for r in range(RESTARTS):
        u = philox.uniforms(K, seed_for(1, "kmeans"), kmeans_stream(r))
        lab, _, obj = kmeans.lloyd(Y, Y[kmeans.kmeanspp(Y, K, u)], 20)
        if obj[-1] < best_obj:
            best, best_obj = lab, obj[-1]
    return Y, best


def bounds(U, C_phi: float, R: np.ndarray, features: np.ndarray):
    """(Thm 3.1 bound at t = 3, Lemma 3.1 chain bound) for features of the signals R."""
    d = R.shape[1]
    Psi = chebyshev.ideal_lowpass(U, K, R)
    S = np.linalg.svd(U[:, :K].T @ R, compute_uv=False)
    thm = C_phi + 2.0 * np.sqrt(K / d) * (np.sqrt(K) + 3.0)
    chain = C_phi + 2.0 * (np.linalg.norm(features - Psi) + np.linalg.norm(S - 1.0))
    return thm, chain


def quality_ok(Phi, labels, thm: float, chain: float, c_oracle: float, slack: float = 0.05):
    """All three checks of the module header for one assignment; returns (ok, cost)."""
    c = kmeans.cost(Phi, labels)
    return (c <= thm and c <= chain and c <= c_oracle + slack), c


def corruptions(labels: np.ndarray, seed: int = 0):
    """Wrong assignments: random labels, clusters 0 and 1 merged, half of cluster 0 moved."""
    rng = np.random.default_rng(seed)
    rnd = rng.integers(0, K, labels.shape[0]).astype(np.int32)
    merged = labels.copy()
    merged[merged == 1] = 0
    half = labels.copy()
    idx = np.where(labels == 0)[0]
    half[idx[: len(idx) // 2]] = 1
    return {"random": rnd, "merged": merged, "half": half}
