"""Pins of the oracle's graph-similarity metrics (Sec. 4 definitions, Thm 4.1, Cor. 4.1)."""

import numpy as np
import pytest

from oracle import chebyshev, operator, philox, similarity
from workloads import DynamicSBM, disjoint_cliques, edges_to_graph, sbm


def _A(g):
    return operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)[0]


def _C(g):
    return operator.combinatorial_laplacian(g.n, g.rowptr, g.colidx, g.w)


def _keys(n, pairs):
    return np.sort(np.array([min(i, j) * n + max(i, j) for i, j in pairs], dtype=np.int64))


def test_edge_distance_by_hand():
    # path 0-1-2 vs triangle 0-1-2
    n = 3
    p = edges_to_graph(n, _keys(n, [(0, 1), (1, 2)]))
    t = edges_to_graph(n, _keys(n, [(0, 1), (1, 2), (0, 2)]))
    # combinatorial: L_path = [[1,-1,0],[-1,2,-1],[0,-1,1]], L_tri = [[2,-1,-1],[-1,2,-1],[-1,-1,2]]
    # difference [[1,0,-1],[0,0,0],[-1,0,1]] -> Frobenius 2
    assert similarity.edge_distance(_C(p), _C(t)) == pytest.approx(2.0, abs=1e-15)
    # normalized: A_path has 1/sqrt(2) on (0,1), (1,2); A_tri has 1/2 everywhere off the diagonal
    d2 = 4 * (0.5 - 1 / np.sqrt(2)) ** 2 + 2 * 0.5 ** 2
    assert similarity.edge_distance(_A(p), _A(t)) == pytest.approx(np.sqrt(d2), abs=1e-15)


def test_edge_distance_is_a_metric():
    g0 = sbm(400, 3, 10.0, 0.1, seed=31)
    dyn = DynamicSBM(g0, seed=32)
    g1 = dyn.step(0.05, 0.01)
    g2 = dyn.step(0.05, 0.01)
    for op in (_A, _C):
        d01 = similarity.edge_distance(op(g0), op(g1))
        assert similarity.edge_distance(op(g0), op(g0)) == 0.0
        assert d01 == similarity.edge_distance(op(g1), op(g0)) > 0.0
        assert similarity.edge_distance(op(g0), op(g2)) <= d01 + similarity.edge_distance(op(g1), op(g2)) + 1e-12


def test_projector_distance_of_cliques_in_closed_form():
    """Two cliques of s nodes, then node s - 1 moved to the other clique (sizes s - 1, s + 1).
    L = D - W has the block indicators as its null space, so H_2 is the projector onto the
    normalized indicators and ||H' - H||_F^2 = 4 - 2 tr(H' H) with
    tr(H' H) = (s - 1) / s + 1 / (s (s + 1)) + s / (s + 1)."""
    s = 6
    g0 = disjoint_cliques(2, s)
    n = 2 * s
    blocks = [list(range(s - 1)), list(range(s - 1, n))]
    pairs = [(i, j) for b in blocks for ii, i in enumerate(b) for j in b[ii + 1:]]
    g1 = edges_to_graph(n, _keys(n, pairs))
    H0 = similarity.projector(_C(g0), 2)
    E = np.zeros((n, 2))
    for c in range(2):
        E[g0.labels == c, c] = 1.0 / np.sqrt(s)
    assert np.allclose(H0, E @ E.T, atol=1e-12)
    tr = (s - 1) / s + 1 / (s * (s + 1)) + s / (s + 1)
    assert similarity.spectral_distance(_C(g0), _C(g1), 2) == pytest.approx(np.sqrt(4 - 2 * tr), abs=1e-12)
    assert similarity.spectral_distance(_C(g0), _C(g0), 2) == pytest.approx(0.0, abs=1e-12)


def test_filter_distance_estimate_is_unbiased():
    g0 = sbm(300, 3, 12.0, 0.1, seed=33)
    g1 = DynamicSBM(g0, seed=34).step(0.1, 0.05)
    A0, A1 = _A(g0), _A(g1)
    lam, _ = operator.dense_spectrum(A0)
    a = chebyshev.step_coefficients(60, 2.0, 0.5 * (lam[2] + lam[3]), "jackson")
    exact = similarity.filter_distance_exact(A0, 2.0, a, A1, 2.0, a)
    # mean of rho_hat^2 over independent probe blocks -> exact^2
    est2 = []
    for t in range(40):
        P = philox.gaussian_block(300, 16, 0.25, 35, t)
        est2.append(similarity.filter_distance_estimate(A0, 2.0, a, A1, 2.0, a, P, 0.0625) ** 2)
    est2 = np.array(est2)
    sem = est2.std(ddof=1) / np.sqrt(len(est2))
    assert abs(est2.mean() - exact ** 2) <= 4 * sem
    # identical graphs estimate exactly zero
    P = philox.gaussian_block(300, 8, 0.25, 36, 0)
    assert similarity.filter_distance_estimate(A0, 2.0, a, A0, 2.0, a, P, 0.0625) == 0.0


def test_filter_distance_tracks_projector_distance_with_a_gap():
    """With a clear eigengap and a high order, h is close to H_k on both graphs, so the filter
    distance approaches the projector distance rho_s."""
    g0 = sbm(300, 3, 30.0, 0.03, seed=37)
    g1 = DynamicSBM(g0, seed=38).step(0.05, 0.01)
    A0, A1 = _A(g0), _A(g1)
    lam0, _ = operator.dense_spectrum(A0)
    lam1, _ = operator.dense_spectrum(A1)
    lc = 0.25 * (lam0[2] + lam1[2] + lam0[3] + lam1[3])
    a = chebyshev.step_coefficients(400, 2.0, lc, "jackson")
    rho_s = similarity.spectral_distance(A0, A1, 3)
    rho_h = similarity.filter_distance_exact(A0, 2.0, a, A1, 2.0, a)
    assert rho_h == pytest.approx(rho_s, rel=0.05, abs=2e-3)


def test_cor41_links_the_two_metrics():
    g0 = sbm(300, 3, 30.0, 0.03, seed=39)
    g1 = DynamicSBM(g0, seed=40).step(0.02, 0.0)
    A0, A1 = _A(g0), _A(g1)
    lam0, _ = operator.dense_spectrum(A0)
    lam1, _ = operator.dense_spectrum(A1)
    alpha = min(lam1[2], lam0[3] - lam1[2])
    assert similarity.spectral_distance(A0, A1, 3) <= np.sqrt(2) / alpha * similarity.edge_distance(A0, A1)


def test_dynamic_similarity_and_refresh_rule():
    from oracle import dynamic
    g0 = sbm(500, 3, 14.0, 0.08, seed=41)
    dyn = DynamicSBM(g0, seed=42)
    seq = [g0, dyn.step(0.01, 0.005), dyn.step(0.3, 0.2), dyn.step(0.01, 0.005)]
    run = dynamic.DynamicCSC(500, 24, 3, 0.5, 40, seed=43, lloyd_iters=5, sim_probes=6)
    res = [run.step(g) for g in seq]
    assert res[0].rho_edge == -1.0 and res[0].rho_hat == -1.0
    for t in range(1, 4):
        assert res[t].rho_edge == pytest.approx(similarity.edge_distance(_A(seq[t - 1]), _A(seq[t])), rel=1e-12)
        assert not res[t].refreshed
    # the heavy perturbation at t = 3 stands out in both metrics
    assert res[2].rho_edge > 5 * max(res[1].rho_edge, res[3].rho_edge)
    assert res[2].rho_hat > 2 * max(res[1].rho_hat, res[3].rho_hat)
    # the estimate is the Hutchinson form of the two filters at lambda_{t-1}
    R = philox.gaussian_block(500, 6, 1 / np.sqrt(24), 43, dynamic.stream_id(2, dynamic.SIGNALS))
    a = chebyshev.step_coefficients(40, 2.0, res[0].lam, "jackson")
    ref = similarity.filter_distance_estimate(_A(seq[0]), 2.0, a, _A(seq[1]), 2.0, a, R, 1 / 24)
    assert res[1].rho_hat == pytest.approx(ref, rel=1e-12)
    # a budget between the quiet and the heavy snapshots refreshes exactly the heavy one, which
    # is then static CSC on its own signal stream
    budget = 0.5 * 0.5 * (res[2].rho_hat + max(res[1].rho_hat, res[3].rho_hat))
    run = dynamic.DynamicCSC(500, 24, 3, 0.5, 40, seed=43, lloyd_iters=5, sim_probes=6,
                             refresh_budget=budget)
    res2 = [run.step(g) for g in seq[:3]]
    assert [r.refreshed for r in res2] == [False, False, True]
    static = dynamic.DynamicCSC(500, 24, 3, 0.5, 40, seed=43, lloyd_iters=5)
    lam, cnt = static._static(_A(seq[2]), 2.0, 3)
    assert lam == res2[2].lam and cnt == res2[2].count
    assert np.array_equal(run.theta, static.theta) and run.cursor == 0
