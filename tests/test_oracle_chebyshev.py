"""Pins of the oracle's Chebyshev coefficients and filter (Sec. 2.2, Sec. 3.2)."""

import numpy as np
import pytest

from oracle import chebyshev, operator
from workloads import cycle_graph, disjoint_cliques, gaussian_block, sbm


def _quadrature_coeffs(m, lmax, lam_c, npts=4_000_000):
    """Chebyshev projection c_j = (2/pi) int_0^pi g(lmax (cos t + 1) / 2) cos(j t) dt by
    the midpoint rule, folded (a_0 = c_0 / 2)."""
    t = (np.arange(npts) + 0.5) * (np.pi / npts)
    g = ((np.cos(t) + 1.0) * lmax / 2.0 <= lam_c).astype(np.float64)
    c = np.array([(2.0 / npts) * np.sum(g * np.cos(j * t)) for j in range(m + 1)])
    c[0] *= 0.5
    return c


@pytest.mark.parametrize("lam_c", [0.43, 0.9, 1.5])
def test_coefficients_match_quadrature(lam_c):
    a = chebyshev.step_coefficients(50, 2.0, lam_c, damping="none")
    q = _quadrature_coeffs(50, 2.0, lam_c)
    assert np.max(np.abs(a - q)) < 2e-6


def test_coefficients_other_lmax():
    a = chebyshev.step_coefficients(20, 1.7, 0.6, damping="none")
    q = _quadrature_coeffs(20, 1.7, 0.6)
    assert np.max(np.abs(a - q)) < 2e-6


@pytest.mark.parametrize("damping", ["none", "jackson"])
def test_special_cutoffs(damping):
    lam = np.linspace(0, 2, 101)
    a_all = chebyshev.step_coefficients(30, 2.0, 2.0, damping)
    a_none = chebyshev.step_coefficients(30, 2.0, 0.0, damping)
    assert np.allclose(chebyshev.response(a_all, lam, 2.0), 1.0, atol=1e-13)
    assert np.allclose(chebyshev.response(a_none, lam, 2.0), 0.0, atol=1e-13)


def test_jackson_kernel_known_values():
    for m in [1, 5, 50, 150]:
        g = chebyshev.jackson_damping(m)
        assert g[0] == pytest.approx(1.0, abs=1e-15)
        # the Jackson kernel's first damping factor is cos(pi / (N + 1)) for N = m + 1 moments
        assert g[1] == pytest.approx(np.cos(np.pi / (m + 2)), abs=1e-14)
        assert np.all(np.diff(g) < 0) and np.all(g > 0)


def test_jackson_response_in_unit_interval_and_monotone_in_cutoff():
    # The derivative of the damped step with respect to theta_c is minus the Jackson
    # kernel, which is non-negative: h lies in [0, 1] and grows with the cut-off.
    lam = np.linspace(0, 2, 2001)
    for m in [10, 50, 120]:
        prev = None
        for lc in np.linspace(0.0, 2.0, 81):
            h = chebyshev.response(chebyshev.step_coefficients(m, 2.0, lc, "jackson"), lam, 2.0)
            assert h.min() >= -1e-12 and h.max() <= 1 + 1e-12
            if prev is not None:
                assert np.all(h >= prev - 1e-12)
            prev = h
        hu = chebyshev.response(chebyshev.step_coefficients(m, 2.0, 0.55, "none"), lam, 2.0)
        assert hu.min() < -1e-3  # Gibbs overshoot of the undamped series


def test_undamped_converges_to_step_away_from_cutoff():
    lam = np.array([0.2, 0.3, 0.8, 1.5])
    h = chebyshev.response(chebyshev.step_coefficients(400, 2.0, 0.55, "none"), lam, 2.0)
    assert np.allclose(h, [1, 1, 0, 0], atol=0.02)


@pytest.fixture(scope="module")
def c1_graph():
    g = sbm(1000, 5, 16.0, 0.1, seed=20170703)
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    lam, U = operator.dense_spectrum(A)
    return g, A, lam, U


def test_recurrence_matches_dense_identity(c1_graph):
    g, A, lam, U = c1_graph
    R = gaussian_block(g.n, 32, 1 / np.sqrt(32), seed=20170704).astype(np.float64)
    for damping in ["none", "jackson"]:
        a = chebyshev.step_coefficients(50, 2.0, 0.5 * (lam[4] + lam[5]), damping)
        Y = chebyshev.filter_recurrence(A, 2.0, a, R)
        Yd = chebyshev.filter_dense(lam, U, a, 2.0, R)
        assert np.linalg.norm(Y - Yd) / np.linalg.norm(Yd) < 1e-12


def test_static_filtering_bound_holds(c1_graph):
    g, A, lam, U = c1_graph
    k = 5
    R = gaussian_block(g.n, 32, 1 / np.sqrt(32), seed=20170704).astype(np.float64)
    Psi = chebyshev.ideal_lowpass(U, k, R)
    for damping in ["none", "jackson"]:
        a = chebyshev.step_coefficients(50, 2.0, 0.5 * (lam[4] + lam[5]), damping)
        Y = chebyshev.filter_recurrence(A, 2.0, a, R)
        err = np.linalg.norm(Y - Psi)
        assert err <= chebyshev.static_filtering_bound(lam, a, 2.0, k, R) + 1e-12


def test_cycle_graph_fourier_eigenvectors():
    n = 64
    g = cycle_graph(n)
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    x = np.arange(n)
    a = chebyshev.step_coefficients(40, 2.0, 0.7, "jackson")
    for j in [0, 1, 5, 16, 31, 32]:
        lam_j = 1.0 - np.cos(2 * np.pi * j / n)
        X = np.stack([np.cos(2 * np.pi * j * x / n), np.sin(2 * np.pi * j * x / n)], axis=1)
        Y = chebyshev.filter_recurrence(A, 2.0, a, X)
        hj = chebyshev.response(a, lam_j, 2.0)
        assert np.allclose(Y, hj * X, atol=1e-12)


def test_disjoint_cliques_two_eigenspaces():
    k, s = 4, 9
    g = disjoint_cliques(k, s)
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    rng = np.random.default_rng(1)
    X = rng.standard_normal((g.n, 3))
    means = np.zeros_like(X)
    for c in range(k):
        means[g.labels == c] = X[g.labels == c].mean(axis=0)
    a = chebyshev.step_coefficients(30, 2.0, 0.5, "jackson")
    Y = chebyshev.filter_recurrence(A, 2.0, a, X)
    h0 = chebyshev.response(a, 0.0, 2.0)
    h1 = chebyshev.response(a, s / (s - 1.0), 2.0)
    assert np.allclose(Y, h0 * means + h1 * (X - means), atol=1e-12)


def test_isolated_node_convention():
    # path 0-1 plus an isolated node 2: its Laplacian row is the identity row (eigenvalue 1)
    from workloads import edges_to_graph
    g = edges_to_graph(3, np.array([0 * 3 + 1]))
    A, dis = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    assert dis[2] == 0.0
    L = operator.laplacian(A).toarray()
    assert np.allclose(L, [[1, -1, 0], [-1, 1, 0], [0, 0, 1]])
    assert operator.isolated_count(g.n, g.rowptr) == 1
