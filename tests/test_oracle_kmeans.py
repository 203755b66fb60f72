"""Pins of the oracle's k-means (Sec. 2.1, eq. SC_cost)."""

import itertools

import numpy as np
import pytest

from oracle import kmeans


def test_assign_matches_brute_force_loop():
    rng = np.random.default_rng(0)
    F = rng.standard_normal((50, 6))
    C = rng.standard_normal((7, 6))
    lab, d2 = kmeans.assign(F, C)
    for i in range(50):
        best, bestc = None, -1
        for c in range(7):
            v = sum((F[i, t] - C[c, t]) ** 2 for t in range(6))
            if best is None or v < best:
                best, bestc = v, c
        assert lab[i] == bestc
        assert d2[i] == pytest.approx(best, rel=1e-14)


def test_exact_ties_go_to_lowest_index():
    F = np.array([[0.0, 0.0], [1.0, 1.0]])
    C = np.array([[1.0, 1.0], [0.0, 0.0], [0.0, 0.0], [1.0, 1.0]])
    lab, _ = kmeans.assign(F, C)
    assert list(lab) == [1, 0]


def test_cost_identity_with_indicator_matrix():
    rng = np.random.default_rng(1)
    F = rng.standard_normal((30, 4))
    lab = rng.integers(0, 5, size=30)
    X = kmeans.indicator(lab, 5)
    lhs = np.linalg.norm(F - X @ X.T @ F)
    assert lhs == pytest.approx(kmeans.cost(F, lab), rel=1e-12)
    # X has orthonormal non-empty columns
    nz = np.bincount(lab, minlength=5) > 0
    assert np.allclose((X.T @ X)[np.ix_(nz, nz)], np.eye(nz.sum()))


def test_lloyd_reaches_brute_force_optimum_on_tiny_input():
    rng = np.random.default_rng(2)
    F = np.concatenate([rng.standard_normal((3, 2)) + [5, 0], rng.standard_normal((4, 2)) - [5, 0],
                        rng.standard_normal((2, 2)) + [0, 8]])
    k = 3
    best = np.inf
    for lab in itertools.product(range(k), repeat=F.shape[0]):
        lab = np.array(lab)
        if len(np.unique(lab)) < k:
            continue
        best = min(best, kmeans.cost(F, lab))
    found = np.inf
    for s in range(10):
        u = np.random.default_rng(100 + s).random(k)
        C0 = F[kmeans.kmeanspp(F, k, u)]
        lab, C, obj = kmeans.lloyd(F, C0, 10)
        found = min(found, kmeans.cost(F, lab))
    assert found == pytest.approx(best, rel=1e-12)


def test_lloyd_objective_non_increasing():
    rng = np.random.default_rng(3)
    F = rng.standard_normal((500, 8))
    u = rng.random(6)
    C0 = F[kmeans.kmeanspp(F, 6, u)]
    _, _, obj = kmeans.lloyd(F, C0, 20)
    assert np.all(np.diff(obj) <= 1e-9 * obj[0])


def test_empty_cluster_keeps_previous_centroid():
    F = np.array([[0.0], [1.0]])
    C_prev = np.array([[0.5], [100.0]])
    lab = np.array([0, 0])
    C, counts = kmeans.update(F, lab, C_prev)
    assert C[1, 0] == 100.0 and C[0, 0] == 0.5 and list(counts) == [2, 0]


def test_kmeanspp_picks_by_cumulative_distance():
    F = np.array([[0.0], [1.0], [3.0], [10.0]])
    # first centre floor(0.3 * 4) = 1; squared distances to it: 1, 0, 4, 81 (cum 1, 1, 5, 86)
    idx = kmeans.kmeanspp(F, 2, np.array([0.3, 4.5 / 86]))
    assert list(idx) == [1, 2]
    idx = kmeans.kmeanspp(F, 2, np.array([0.3, 0.5]))
    assert list(idx) == [1, 3]


def test_separated_clusters_recovered():
    rng = np.random.default_rng(4)
    centers = rng.standard_normal((5, 10)) * 20
    truth = rng.integers(0, 5, size=400)
    F = centers[truth] + rng.standard_normal((400, 10))
    C0 = F[kmeans.kmeanspp(F, 5, rng.random(5))]
    lab, _, _ = kmeans.lloyd(F, C0, 20)
    # identical partitions up to relabelling
    pairs = set(zip(truth.tolist(), lab.tolist()))
    assert len(pairs) == 5
