"""Pins of the oracle's combinatorial Laplacian L = D - W (Sec. 2.1) and of the spectrum bound
used with it, and of filtering, eigencount and dynamic CSC on that operator."""

import numpy as np
import pytest

from oracle import chebyshev, dynamic, eigcount, operator, philox
from workloads import DynamicSBM, cycle_graph, disjoint_cliques, edges_to_graph, sbm


def _comb(g):
    return operator.combinatorial_laplacian(g.n, g.rowptr, g.colidx, g.w)


def _am(g):
    return operator.anderson_morley_bound(g.n, g.rowptr, g.colidx, g.w)


def _keys(n, pairs):
    return np.sort(np.array([min(i, j) * n + max(i, j) for i, j in pairs], dtype=np.int64))


def test_weighted_path_by_hand():
    # W = [[0, 2, 0], [2, 0, 3], [0, 3, 0]]: D = diag(2, 5, 3)
    g = edges_to_graph(3, _keys(3, [(0, 1), (1, 2)]), weights=np.array([2.0, 3.0]))
    L = _comb(g).L.toarray()
    assert np.array_equal(L, [[2, -2, 0], [-2, 5, -3], [0, -3, 3]])
    assert _am(g) == 8.0


@pytest.mark.parametrize("n", [8, 64])
def test_cycle_spectrum_and_fourier_modes(n):
    """Even cycle: eigenvalues 2 - 2 cos(2 pi j / n); 2-regular bipartite, so the bound 4 is
    attained; each Fourier pair is scaled by h at its eigenvalue."""
    g = cycle_graph(n)
    L = _comb(g)
    lam, _ = operator.dense_spectrum(L)
    ref = np.sort(2.0 - 2.0 * np.cos(2 * np.pi * np.arange(n) / n))
    assert np.allclose(lam, ref, atol=1e-12)
    assert _am(g) == 4.0 == pytest.approx(lam[-1], abs=1e-12)
    x = np.arange(n)
    a = chebyshev.step_coefficients(40, 4.0, 1.3, "jackson")
    for j in [0, 1, n // 4, n // 2]:
        X = np.stack([np.cos(2 * np.pi * j * x / n), np.sin(2 * np.pi * j * x / n)], axis=1)
        Y = chebyshev.filter_recurrence(L, 4.0, a, X)
        hj = chebyshev.response(a, 2.0 - 2.0 * np.cos(2 * np.pi * j / n), 4.0)
        assert np.allclose(Y, hj * X, atol=1e-12)


def test_disjoint_cliques_block_means():
    """k cliques K_s: eigenvalue 0 on block-constant vectors, s on the zero-mean rest."""
    k, s = 3, 7
    g = disjoint_cliques(k, s)
    L = _comb(g)
    lam, _ = operator.dense_spectrum(L)
    assert np.allclose(lam[:k], 0.0, atol=1e-12) and np.allclose(lam[k:], s, atol=1e-12)
    lmax = _am(g)
    assert lmax == 2.0 * (s - 1)
    rng = np.random.default_rng(2)
    X = rng.standard_normal((g.n, 4))
    means = np.zeros_like(X)
    for c in range(k):
        means[g.labels == c] = X[g.labels == c].mean(axis=0)
    a = chebyshev.step_coefficients(30, lmax, 2.0, "jackson")
    Y = chebyshev.filter_recurrence(L, lmax, a, X)
    assert np.allclose(Y, chebyshev.response(a, 0.0, lmax) * means
                       + chebyshev.response(a, float(s), lmax) * (X - means), atol=1e-12)


def test_star_attains_bound():
    """Star K_{1,n-1}: eigenvalues 0, 1 (n - 2 times), n; the bound (n - 1) + 1 = n."""
    n = 9
    g = edges_to_graph(n, _keys(n, [(0, i) for i in range(1, n)]))
    lam, _ = operator.dense_spectrum(_comb(g))
    assert np.allclose(lam, [0.0] + [1.0] * (n - 2) + [float(n)], atol=1e-12)
    assert _am(g) == float(n)


def test_complete_bipartite_spectrum():
    """K_{a,b}: eigenvalues 0, a (b - 1 times), b (a - 1 times), a + b = the bound."""
    a_, b_ = 3, 5
    n = a_ + b_
    g = edges_to_graph(n, _keys(n, [(i, a_ + j) for i in range(a_) for j in range(b_)]))
    lam, _ = operator.dense_spectrum(_comb(g))
    ref = np.sort([0.0] + [a_] * (b_ - 1) + [b_] * (a_ - 1) + [a_ + b_])
    assert np.allclose(lam, ref, atol=1e-12)
    assert _am(g) == a_ + b_


def test_bound_above_spectrum_on_random_graphs():
    for seed in range(3):
        g = sbm(300, 3, 12.0, 0.2, seed=90 + seed)
        lam, _ = operator.dense_spectrum(_comb(g))
        assert lam[-1] <= _am(g) + 1e-9
        assert lam[0] == pytest.approx(0.0, abs=1e-9)


def test_recurrence_and_eigencount_on_combinatorial():
    g = sbm(400, 4, 10.0, 0.1, seed=95)
    L = _comb(g)
    lmax = _am(g)
    lam, U = operator.dense_spectrum(L)
    a = chebyshev.step_coefficients(60, lmax, 0.5 * (lam[3] + lam[4]), "jackson")
    R = philox.gaussian_block(g.n, 8, 1.0, 5, 1)
    Y = chebyshev.filter_recurrence(L, lmax, a, R)
    assert np.allclose(Y, chebyshev.filter_dense(lam, U, a, lmax, R), atol=1e-10)
    mu = eigcount.moments_direct(L, lmax, 60, R)
    exact = np.sum(R * chebyshev.filter_dense(lam, U, a, lmax, R))
    assert eigcount.count_from_moments(a, mu, 1.0, 8) == pytest.approx(exact / 8, rel=1e-10)
    assert np.allclose(eigcount.moments_doubled(L, lmax, 60, R), mu, rtol=1e-9, atol=1e-8)


def test_dynamic_combinatorial_p_zero_is_static_per_snapshot():
    g0 = sbm(500, 3, 12.0, 0.1, seed=96)
    dyn = DynamicSBM(g0, seed=97)
    seq = [g0] + [dyn.step(0.02, 0.01) for _ in range(3)]
    run = dynamic.DynamicCSC(500, 16, 3, 0.0, 30, seed=98, lloyd_iters=5, tau=0.0,
                             laplacian="combinatorial")
    for t, g in enumerate(seq, start=1):
        res = run.step(g)
        lmax = _am(g)
        R = philox.gaussian_block(500, 16, 0.25, 98, dynamic.stream_id(t, dynamic.SIGNALS))
        a = chebyshev.step_coefficients(30, lmax, res.lam, "jackson")
        assert np.allclose(run.theta, chebyshev.filter_recurrence(_comb(g), lmax, a, R), atol=1e-12)
        # the count at the chosen cut-off is Hutchinson's form on the snapshot's own spectrum
        lam, U = operator.dense_spectrum(_comb(g))
        exact = np.sum(R * chebyshev.filter_dense(lam, U, a, lmax, R)) / (0.25 ** 2 * 16)
        assert res.count == pytest.approx(exact, rel=1e-9)
        assert 0.0 < res.lam < lmax
