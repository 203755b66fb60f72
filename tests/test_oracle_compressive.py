"""Pins of the oracle's compressive k-means (Sec. 2.2, Step 2)."""

import numpy as np
import pytest

from oracle import chebyshev, compressive, kmeans, operator, philox
from workloads import disjoint_cliques, sbm


def _A(g):
    return operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)[0]


def test_inverse_cdf_draw_by_hand():
    w = np.array([1.0, 2.0, 3.0, 4.0])  # prefix sums 1, 3, 6, 10
    u = np.array([0.0, 0.05, 0.1, 0.29, 0.3, 0.59, 0.6, 0.999])
    assert compressive.draw(w, u).tolist() == [0, 0, 1, 1, 2, 2, 3, 3]


def test_draw_frequencies_follow_the_density():
    rng = np.random.default_rng(5)
    w = rng.random(20) ** 2
    u = philox.uniforms(200_000, 7, 3)
    idx = compressive.draw(w, u)
    freq = np.bincount(idx, minlength=20) / len(u)
    p = w / w.sum()
    assert np.all(np.abs(freq - p) <= 5 * np.sqrt(p * (1 - p) / len(u)))


def test_clique_indicators_are_interpolated_exactly():
    """Equal cliques form a regular graph: each clique indicator is in the null space of L
    and matches every sample, so it is the unique minimiser."""
    g = disjoint_cliques(3, 8)
    A = _A(g)
    idx = np.array([0, 3, 9, 12, 12, 20])
    labels_s = g.labels[idx]
    w = np.linspace(1.0, 2.0, g.n)
    for r in (1, 2, 4):
        X = compressive.interpolate(A, idx, w, labels_s, 3, r, 0.01)
        E = np.zeros((g.n, 3))
        E[np.arange(g.n), g.labels] = 1.0
        assert np.allclose(X, E, atol=1e-10)


def test_small_gamma_reproduces_the_samples_and_optimality_holds():
    g = sbm(300, 3, 12.0, 0.1, seed=61)
    A = _A(g)
    rng = np.random.default_rng(62)
    idx = np.unique(rng.integers(0, g.n, size=40))
    labels_s = g.labels[idx]
    w = rng.random(g.n) + 0.5
    X = compressive.interpolate(A, idx, w, labels_s, 3, 2, 1e-9)
    Y = np.zeros((len(idx), 3))
    Y[np.arange(len(idx)), labels_s] = 1.0
    assert np.allclose(X[idx], Y, atol=1e-5)
    # first-order condition of the objective at gamma = 0.1: the gradient vanishes
    gam = 0.1
    X = compressive.interpolate(A, idx, w, labels_s, 3, 2, gam)
    p = w / w.sum()
    L = operator.laplacian(A).toarray()
    wt = 1.0 / (len(idx) * p[idx])
    resid = X[idx] - Y
    grad = gam * (L @ L @ X)
    np.add.at(grad, idx, wt[:, None] * resid)
    assert np.max(np.abs(grad)) <= 1e-10 * max(1.0, np.max(np.abs(X)))


def test_agrees_with_full_kmeans_on_a_separable_sbm():
    g = sbm(800, 3, 24.0, 0.02, seed=63)
    A = _A(g)
    lam, U = operator.dense_spectrum(A)
    R = philox.gaussian_block(g.n, 32, 1 / np.sqrt(32), 64, 1)
    a = chebyshev.step_coefficients(80, 2.0, 0.5 * (lam[2] + lam[3]), "jackson")
    F = chebyshev.filter_recurrence(A, 2.0, a, R)
    lab, idx, lab_s, X = compressive.compressive_kmeans(
        A, F, 3, 60, philox.uniforms(60, 65, 3), philox.uniforms(3, 65, 2), 20, 4, 1e-3)
    full, _, _ = kmeans.lloyd(F, F[kmeans.kmeanspp(F, 3, philox.uniforms(3, 66, 2))], 20)
    # agreement up to a permutation of the cluster ids
    conf = np.zeros((3, 3))
    np.add.at(conf, (lab, full), 1)
    assert conf.max(axis=1).sum() / g.n >= 0.97
    assert len(np.unique(lab)) == 3
    conf = np.zeros((3, 3))
    np.add.at(conf, (lab, g.labels), 1)
    assert conf.max(axis=1).sum() / g.n >= 0.95  # and with the planted partition
