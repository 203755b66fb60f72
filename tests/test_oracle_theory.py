"""The paper's theorems as pins of the oracle's features and costs (Sec. 3, Sec. 4.2)."""

import numpy as np
import pytest

from oracle import chebyshev, kmeans, operator
from workloads import DynamicSBM, gaussian_block, sbm


@pytest.fixture(scope="module")
def c1():
    g = sbm(1000, 5, 16.0, 0.1, seed=20170703)
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    lam, U = operator.dense_spectrum(A)
    return g, A, lam, U


def _thm32_Q(Uk, R):
    """The unitary Q of Thm. 3.2's proof: R' = Uk^T R = QL S QR^T, Q = diag(QL, I) QR^T."""
    k = Uk.shape[1]
    d = R.shape[1]
    Rp = Uk.T @ R
    QL, S, QRt = np.linalg.svd(Rp, full_matrices=True)
    B = np.eye(d)
    B[:k, :k] = QL
    return B @ QRt, S


def test_thm32_feature_error_equals_singular_value_error(c1):
    g, A, lam, U = c1
    k, d = 5, 32
    R = gaussian_block(g.n, d, 1 / np.sqrt(d), seed=20170704).astype(np.float64)
    Psi = chebyshev.ideal_lowpass(U, k, R)
    Uk = U[:, :k]
    Q, S = _thm32_Q(Uk, R)
    I_kd = np.eye(k, d)
    lhs = np.linalg.norm(Psi - Uk @ I_kd @ Q)
    rhs = np.linalg.norm(S - 1.0)
    assert lhs == pytest.approx(rhs, rel=1e-10)


def test_cor32_bound_failure_rate():
    # ||Sigma - I||_F <= sqrt(k/d)(sqrt(k) + t) fails with probability <= exp(-t^2/2)
    k, d, t = 5, 32, 1.5
    fails = 0
    trials = 200
    rng = np.random.default_rng(9)
    for _ in range(trials):
        Rp = rng.standard_normal((k, d)) / np.sqrt(d)
        S = np.linalg.svd(Rp, compute_uv=False)
        if np.linalg.norm(S - 1.0) > np.sqrt(k / d) * (np.sqrt(k) + t):
            fails += 1
    assert fails / trials <= np.exp(-t * t / 2) + 0.05


def test_lemma31_chain_on_c1(c1):
    # C_Psi~ <= C_Phi + 2 (||Psi~ - Psi||_F + ||Sigma - I||_F), with C_Phi the best of many
    # k-means++ restarts on U_k (Lloyd is a heuristic, so this reports a margin).
    g, A, lam, U = c1
    k, d = 5, 256
    R = gaussian_block(g.n, d, 1 / np.sqrt(d), seed=20170705).astype(np.float64)
    lc = 0.5 * (lam[k - 1] + lam[k])
    a = chebyshev.step_coefficients(50, 2.0, lc, "jackson")
    Yt = chebyshev.filter_recurrence(A, 2.0, a, R)
    Psi = chebyshev.ideal_lowpass(U, k, R)
    Phi = U[:, :k]
    rng = np.random.default_rng(10)
    best_phi = np.inf
    for _ in range(20):
        C0 = Phi[kmeans.kmeanspp(Phi, k, rng.random(k))]
        lab, _, _ = kmeans.lloyd(Phi, C0, 30)
        best_phi = min(best_phi, kmeans.cost(Phi, lab))
    C0 = Yt[kmeans.kmeanspp(Yt, k, rng.random(k))]
    lab_t, _, _ = kmeans.lloyd(Yt, C0, 20)
    c_psi = kmeans.cost(Phi, lab_t)
    _, S = _thm32_Q(Phi, R)
    bound = best_phi + 2 * (np.linalg.norm(Yt - Psi) + np.linalg.norm(S - 1.0))
    assert c_psi <= bound
    # and Thm. 3.1's probabilistic form at t = 3 (probability >= 1 - e^{-4.5})
    assert c_psi <= best_phi + 2 * np.sqrt(k / d) * (np.sqrt(k) + 3.0) + 2 * np.linalg.norm(Yt - Psi)


def test_cor41_projector_perturbation_bound():
    g0 = sbm(300, 3, 30.0, 0.03, seed=21)
    dyn = DynamicSBM(g0, seed=22)
    g1 = dyn.step(0.02, 0.0)
    k = 3
    A0, _ = operator.normalized_adjacency(g0.n, g0.rowptr, g0.colidx, g0.w)
    A1, _ = operator.normalized_adjacency(g1.n, g1.rowptr, g1.colidx, g1.w)
    lam0, U0 = operator.dense_spectrum(A0)
    lam1, U1 = operator.dense_spectrum(A1)
    H0 = U0[:, :k] @ U0[:, :k].T
    H1 = U1[:, :k] @ U1[:, :k].T
    alpha = min(lam1[k - 1], lam0[k] - lam1[k - 1])
    assert alpha > 0
    dL = (operator.laplacian(A1) - operator.laplacian(A0)).toarray()
    assert np.linalg.norm(H1 - H0) <= np.sqrt(2) / alpha * np.linalg.norm(dL)


@pytest.mark.parametrize("d", [32, 256])
def test_quality_checks_accept_csc_and_reject_wrong_assignments(d):
    # the checks of tests/quality.py on the oracle's own static CSC: its assignment passes,
    # random labels, two merged clusters and half a cluster moved do not
    import quality as Q
    g = Q.c1_graph()
    A, lam, U, c_phi = Q.sc_reference(g)
    R = Q.signals(g.n, d, "f32")
    lam_c = 0.5 * (lam[Q.K - 1] + lam[Q.K])
    Y, lab = Q.oracle_csc(A, lam_c, R)
    Phi = U[:, :Q.K]
    thm, chain = Q.bounds(U, c_phi, R, Y)
    ok, c = Q.quality_ok(Phi, lab, thm, chain, kmeans.cost(Phi, lab))
    assert ok
    assert (thm < np.sqrt(Q.K)) == (d == 256)
    for bad in Q.corruptions(lab).values():
        assert not Q.quality_ok(Phi, bad, thm, chain, c)[0]
