"""Pins of the oracle's eigencount and dichotomy (Sec. 3.2, Sec. 4.1)."""

import numpy as np
import pytest

from oracle import chebyshev, eigcount, operator
from workloads import gaussian_block, sbm


@pytest.fixture(scope="module")
def small():
    g = sbm(400, 4, 14.0, 0.1, seed=11)
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    lam, U = operator.dense_spectrum(A)
    return g, A, lam, U


def test_literal_equals_moments(small):
    g, A, lam, U = small
    m = 40
    P = gaussian_block(g.n, 12, 0.5, seed=3).astype(np.float64)
    mu = eigcount.moments_direct(A, 2.0, m, P)
    for lc in [0.1, 0.35, 0.8, 1.6]:
        a = chebyshev.step_coefficients(m, 2.0, lc, "jackson")
        c1 = eigcount.count_literal(A, 2.0, a, P, 0.25)
        c2 = eigcount.count_from_moments(a, mu, 0.25, 12)
        assert c2 == pytest.approx(c1, rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("m", [1, 2, 7, 40, 41])
def test_doubled_moments_equal_direct(small, m):
    g, A, lam, U = small
    P = gaussian_block(g.n, 5, 1.0, seed=4).astype(np.float64)
    d = eigcount.moments_direct(A, 2.0, m, P)
    k = eigcount.moments_doubled(A, 2.0, m, P)
    assert np.max(np.abs(d - k)) <= 1e-9 * np.max(np.abs(d))


def test_moments_match_dense_trace(small):
    g, A, lam, U = small
    m = 30
    P = gaussian_block(g.n, 8, 1.0, seed=5).astype(np.float64)
    mu = eigcount.moments_direct(A, 2.0, m, P)
    x = 2.0 * lam / 2.0 - 1.0
    PU = U.T @ P
    for j in [0, 1, 2, 13, 30]:
        exact = np.sum((np.cos(j * np.arccos(np.clip(x, -1, 1)))[:, None]) * PU * PU)
        assert mu[j] == pytest.approx(exact, rel=1e-10, abs=1e-9)


def test_count_near_true_count(small):
    g, A, lam, U = small
    m = 80
    n_s = 3000
    sigma = 1.0
    P = gaussian_block(g.n, n_s, sigma, seed=6).astype(np.float64)
    mu = eigcount.moments_direct(A, 2.0, m, P)
    for lc in [0.3, 0.7, 1.2]:
        a = chebyshev.step_coefficients(m, 2.0, lc, "jackson")
        h = chebyshev.response(a, lam, 2.0)
        c = eigcount.count_from_moments(a, mu, sigma ** 2, n_s)
        # Hutchinson: variance of the estimate is 2 sum h^2 / n_s for Gaussian probes
        assert abs(c - h.sum()) <= 4.0 * np.sqrt(2.0 * np.sum(h ** 2) / n_s)
        true = np.sum(lam <= lc)
        assert abs(h.sum() - true) <= np.sum(np.abs(h - (lam <= lc))) + 1e-9


def test_damped_count_monotone_in_cutoff(small):
    g, A, lam, U = small
    m = 50
    P = gaussian_block(g.n, 24, 0.2, seed=7).astype(np.float64)
    mu = eigcount.moments_direct(A, 2.0, m, P)
    cs = [eigcount.count_from_moments(chebyshev.step_coefficients(m, 2.0, lc, "jackson"), mu,
                                      0.04, 24) for lc in np.linspace(0, 2, 200)]
    assert np.all(np.diff(cs) >= -1e-9)
    assert cs[-1] == pytest.approx(g.n, rel=0.2)


def test_bisect_on_known_staircase():
    # count(lambda) = number of thresholds below lambda: the dichotomy finds the k-th one
    thr = np.sort(np.random.default_rng(0).random(20) * 2)
    lam_c, c, trace = eigcount.bisect(lambda x: float(np.sum(thr <= x)), 7, 0.0, 2.0, 30)
    assert len(trace) == 30
    assert thr[6] <= lam_c <= thr[6] + 2.0 / 2 ** 29
    assert c >= 7


def test_bisect_brackets_lambda_k(small):
    g, A, lam, U = small
    m = 80
    P = gaussian_block(g.n, 400, 1.0, seed=8).astype(np.float64)
    mu = eigcount.moments_direct(A, 2.0, m, P)
    lc, c, _ = eigcount.eigcount_bisect(mu, m, 2.0, "jackson", 1.0, 400, 4, 16, 0.0, 2.0)
    # with many probes the cut-off lands near the k-th eigenvalue gap of this graph
    assert lam[2] < lc < lam[5]
    assert c >= 4
