"""GPU parity of the graph-similarity metrics (Sec. 4) and of the refresh rule of dynamic CSC
(Thm 4.1) against the FP64 oracle, through the C ABI."""

import numpy as np
import pytest
import torch

from oracle import dynamic, operator, similarity
from workloads import DynamicSBM, sbm
from helpers import rel_fro, say

pytestmark = pytest.mark.gpu


def _A(g):
    return operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)[0]


def _C(g):
    return operator.combinatorial_laplacian(g.n, g.rowptr, g.colidx, g.w)


@pytest.fixture(scope="module")
def pair():
    g0 = sbm(3000, 6, 12.0, 0.1, seed=101)
    dyn = DynamicSBM(g0, seed=102)
    return g0, dyn.step(0.05, 0.02)


def test_edge_distance_normalized(csc, pair):
    g0, g1 = pair
    say("edge distance, normalized")
    G0, G1 = csc.Graph.from_workload(g0), csc.Graph.from_workload(g1)
    ref = similarity.edge_distance(_A(g0), _A(g1))
    d = G0.distance(G1)
    say(f"  gpu {d:.9f} oracle {ref:.9f}")
    assert d == pytest.approx(ref, rel=1e-5)
    assert G1.distance(G0) == d
    assert G0.distance(G0) == 0.0
    B0 = csc.Graph.from_workload(g0, val_dtype=torch.bfloat16)
    B1 = csc.Graph.from_workload(g1, val_dtype=torch.bfloat16)
    assert B0.distance(B1) == pytest.approx(ref, rel=1e-2)


def test_edge_distance_combinatorial_is_exact(csc, pair):
    """Unit weights and integer degrees: every term is an integer, so the FP64 sum is exact."""
    g0, g1 = pair
    G0 = csc.Graph.from_workload(g0, laplacian=csc.LAP_COMBINATORIAL)
    G1 = csc.Graph.from_workload(g1, laplacian=csc.LAP_COMBINATORIAL)
    assert G0.distance(G1) == similarity.edge_distance(_C(g0), _C(g1))


def test_edge_distance_argument_errors(csc, pair):
    g0, g1 = pair
    G0 = csc.Graph.from_workload(g0)
    with pytest.raises(csc.CscError, match="Laplacian kinds"):
        G0.distance(csc.Graph.from_workload(g1, laplacian=csc.LAP_COMBINATORIAL))
    with pytest.raises(csc.CscError, match="different sizes"):
        G0.distance(csc.Graph.from_workload(sbm(100, 2, 5.0, 0.1, seed=103)))


@pytest.fixture(scope="module")
def seq():
    g0 = sbm(2000, 3, 14.0, 0.08, seed=104)
    dyn = DynamicSBM(g0, seed=105)
    return [g0, dyn.step(0.01, 0.005), dyn.step(0.3, 0.2), dyn.step(0.01, 0.005), dyn.step(0.01, 0.005)]


@pytest.mark.parametrize("keep", [0, 1])
def test_dynamic_similarity_matches_oracle(csc, seq, keep):
    say(f"dynamic similarity tracking keep_iterates={keep}")
    k, m, d, p, seed = 3, 40, 24, 0.5, 106
    orc = dynamic.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, storage=np.float32,
                             sim_probes=6)
    gpu = csc.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, keep_iterates=keep,
                         sim_probes=6)
    for t, g in enumerate(seq, start=1):
        lab, lam, ref, cnt = gpu.step(csc.Graph.from_workload(g))
        r = orc.step(g)
        re_, rh, rf = gpu.similarity(t)
        say(f"  t={t} rho_e {re_:.6f}/{r.rho_edge:.6f} rho_hat {rh:.6f}/{r.rho_hat:.6f}")
        assert lam == r.lam and ref == r.refined and not rf
        if t == 1:
            assert re_ == -1.0 and rh == -1.0
        else:
            assert re_ == pytest.approx(r.rho_edge, rel=1e-5)
            assert rh == pytest.approx(r.rho_hat, rel=1e-3)
    assert rel_fro(gpu.features().double().cpu().numpy(), orc.theta) <= 1e-5


@pytest.mark.parametrize("batch", [1, 4])
def test_refresh_rule_matches_oracle(csc, seq, batch):
    say(f"refresh rule batch={batch}")
    k, m, d, p, seed = 3, 40, 24, 0.5, 107
    probe = dynamic.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, storage=np.float32,
                               sim_probes=6)
    rh = [probe.step(g).rho_hat for g in seq]
    quiet = max(rh[1], rh[3], rh[4])
    assert rh[2] > 2 * quiet
    budget = p * 0.5 * (rh[2] + quiet)
    orc = dynamic.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, storage=np.float32,
                             sim_probes=6, refresh_budget=budget)
    res = [orc.step(g) for g in seq]
    assert [r.refreshed for r in res] == [False, False, True, False, False]
    gpu = csc.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, keep_iterates=1,
                         sim_probes=6, refresh_budget=budget, batch=batch, use_graph=batch > 1)
    Gs = [csc.Graph.from_workload(g) for g in seq]
    labels, lams, refs, cnts = gpu.steps(Gs)
    for t, r in enumerate(res, start=1):
        _, _, rf = gpu.similarity(t)
        assert rf == r.refreshed
        assert lams[t - 1] == r.lam and refs[t - 1] == r.refined
        assert cnts[t - 1] == pytest.approx(r.count, rel=1e-4, abs=1e-4)
    assert rel_fro(gpu.features().double().cpu().numpy(), orc.theta) <= 1e-5


def test_similarity_on_combinatorial_snapshots(csc, seq):
    k, m, d, p, seed = 3, 80, 24, 0.5, 108
    orc = dynamic.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, storage=np.float32,
                             laplacian="combinatorial")
    gpu = csc.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, keep_iterates=0,
                         track_similarity=True)
    for t, g in enumerate(seq, start=1):
        _, lam, _, _ = gpu.step(csc.Graph.from_workload(g, laplacian=csc.LAP_COMBINATORIAL))
        r = orc.step(g)
        assert lam == r.lam
        re_, rh, rf = gpu.similarity(t)
        assert rh == -1.0 and not rf
        assert re_ == (r.rho_edge if t > 1 else -1.0)
