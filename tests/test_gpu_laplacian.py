"""GPU parity of the combinatorial Laplacian L = D - W (Sec. 2.1) against the FP64 oracle:
spectrum bound, filter (every kernel shape, heavy rows), moments, eigencount and dynamic CSC."""

import numpy as np
import pytest
import torch

from oracle import chebyshev, dynamic, eigcount, operator
from workloads import DynamicSBM, edges_to_graph, gaussian_block, sbm
from helpers import rel_fro, say

pytestmark = pytest.mark.gpu

TOL_F32 = 1e-5


def _comb(g):
    return operator.combinatorial_laplacian(g.n, g.rowptr, g.colidx, g.w)


def _am(g):
    return operator.anderson_morley_bound(g.n, g.rowptr, g.colidx, g.w)


@pytest.fixture(scope="module")
def cg(csc):
    g = sbm(1500, 5, 14.0, 0.1, seed=81)
    return g, csc.Graph.from_workload(g, laplacian=csc.LAP_COMBINATORIAL), _comb(g)


def test_spectrum_bound_matches_oracle(csc, cg):
    g, G, L = cg
    say("combinatorial spectrum bound")
    assert G.lmax() == _am(g)
    lam, _ = operator.dense_spectrum(L)
    est = G.lmax(200)
    say(f"  bound {G.lmax():.3f} power estimate {est:.4f} true {lam[-1]:.4f}")
    assert lam[-1] * 0.999 <= est <= G.lmax()
    # weighted graph: the bound is an FP64 maximum of degree sums, equal to the oracle's
    rng = np.random.default_rng(82)
    gw = sbm(700, 3, 9.0, 0.2, seed=83)
    keys = np.unique(np.minimum(np.repeat(np.arange(gw.n), np.diff(gw.rowptr)), gw.colidx.astype(np.int64)) * gw.n
                     + np.maximum(np.repeat(np.arange(gw.n), np.diff(gw.rowptr)), gw.colidx.astype(np.int64)))
    gw = edges_to_graph(gw.n, keys, weights=rng.integers(1, 9, size=keys.size).astype(np.float64))
    Gw = csc.Graph.from_workload(gw, laplacian=csc.LAP_COMBINATORIAL)
    assert Gw.lmax() == _am(gw)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("w", [1, 7, 64])
def test_filter_parity(csc, cg, variant, w):
    g, G, L = cg
    say(f"combinatorial filter variant={variant} w={w}")
    lmax = G.lmax()
    lam, _ = operator.dense_spectrum(L)
    a = chebyshev.step_coefficients(80, lmax, 0.5 * (lam[4] + lam[5]), "jackson")
    X = gaussian_block(g.n, w, 1 / np.sqrt(w), seed=84)
    G.set_variant(variant)
    Y = csc.cheb_filter(G, a, torch.from_numpy(X).cuda()).cpu().numpy()
    G.set_variant(-1)
    ref = chebyshev.filter_recurrence(L, lmax, a, X.astype(np.float64))
    assert rel_fro(Y, ref) <= TOL_F32


def test_filter_bf16s_iterates(csc, cg):
    g, G, L = cg
    say("combinatorial filter, BF16 copies with FP32 state")
    lmax = G.lmax()
    a = chebyshev.step_coefficients(60, lmax, 1.0, "jackson")
    X = torch.from_numpy(gaussian_block(g.n, 32, 0.2, seed=85)).cuda().to(torch.bfloat16)
    Y = csc.cheb_filter(G, a, X, iter_dtype="bf16s").cpu().numpy()
    ref = chebyshev.filter_recurrence(L, lmax, a, X.float().cpu().numpy().astype(np.float64))
    assert rel_fro(Y, ref) <= 2e-2


def test_heavy_rows_and_isolated_nodes(csc):
    """A hub of degree 3000 (cooperative heavy-block path) and isolated nodes (zero rows)."""
    rng = np.random.default_rng(86)
    n = 5003
    keys = set(range(1, 3001))
    u = rng.integers(3001, n - 10, size=20000)
    v = rng.integers(3001, n - 10, size=20000)
    for a_, b_ in zip(u, v):
        if a_ != b_:
            keys.add(int(min(a_, b_)) * n + int(max(a_, b_)))
    g = edges_to_graph(n, np.array(sorted(keys), dtype=np.int64))
    G = csc.Graph.from_workload(g, laplacian=csc.LAP_COMBINATORIAL)
    lmax = G.lmax()
    assert lmax == _am(g) >= 3001
    X = gaussian_block(n, 20, 0.3, seed=87)
    a = chebyshev.step_coefficients(40, lmax, 0.02 * lmax, "jackson")
    L = _comb(g)
    ref = chebyshev.filter_recurrence(L, lmax, a, X.astype(np.float64))
    mu_ref = eigcount.moments_direct(L, lmax, 40, X.astype(np.float64))
    for variant in range(4):
        G.set_variant(variant)
        Y, mu = csc.cheb_filter(G, a, torch.from_numpy(X).cuda(), moments=True)
        assert rel_fro(Y.cpu().numpy(), ref) <= TOL_F32
        assert np.max(np.abs(mu.cpu().numpy() - mu_ref)) <= 1e-5 * np.max(np.abs(mu_ref))
    G.set_variant(-1)


def test_eigcount_matches_oracle(csc, cg):
    g, G, L = cg
    say("combinatorial eigencount")
    lmax = G.lmax()
    P = gaussian_block(g.n, 32, 1 / np.sqrt(32), seed=88)
    m, k = 120, 5
    lam, cnt, trace, mu = csc.eigcount(G, m, torch.from_numpy(P).cuda(), sigma2=1 / 32.0, k=k, n_cand=16)
    mu_ref = eigcount.moments_direct(L, lmax, m, P.astype(np.float64))
    lam_ref, cnt_ref, trace_ref = eigcount.eigcount_bisect(mu_ref, m, lmax, "jackson", 1 / 32.0, 32,
                                                           k, 16, 0.0, lmax)
    tr = np.array(trace_ref)
    for i in range(16):
        if (trace[i, 1] < k) != (tr[i, 1] < k):
            assert abs(tr[i, 1] - k) < 1e-5 * np.sum(np.abs(mu_ref)) / (32 / 32.0)
            return
        assert trace[i, 0] == tr[i, 0]
    assert lam == lam_ref
    assert cnt == pytest.approx(cnt_ref, rel=1e-4)


def test_adjoint_refuses_combinatorial(csc, cg):
    g, G, L = cg
    X = torch.zeros((g.n, 4), device="cuda")
    with pytest.raises(csc.CscError, match="normalized"):
        csc.filter_backward(G, np.ones(3), X, X)


@pytest.mark.parametrize("keep,batch", [(0, 1), (1, 1), (1, 4)])
def test_dynamic_matches_oracle(csc, keep, batch):
    say(f"combinatorial dynamic keep_iterates={keep} batch={batch}")
    g0 = sbm(2000, 4, 20.0, 0.05, seed=89)
    dyn = DynamicSBM(g0, seed=90)
    seq = [g0] + [dyn.step(0.01, 0.005) for _ in range(4)]
    k, m, d, p, seed = 4, 80, 32, 0.5, 91
    orc = dynamic.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, storage=np.float32,
                             laplacian="combinatorial")
    gpu = csc.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, keep_iterates=keep,
                         batch=batch, use_graph=batch > 1)
    Gs = [csc.Graph.from_workload(g, laplacian=csc.LAP_COMBINATORIAL) for g in seq]
    if batch > 1:
        labels, lams, refs, cnts = gpu.steps(Gs)
        outs = list(zip(labels, lams, refs, cnts))
    else:
        outs = None
    for t, g in enumerate(seq, start=1):
        lab, lam, ref, cnt = outs[t - 1] if outs else gpu.step(Gs[t - 1])
        r = orc.step(g)
        say(f"  t={t} lmax={Gs[t - 1].lmax():.1f} lam gpu={lam:.6f} oracle={r.lam:.6f} refined {ref}/{r.refined}")
        assert ref == r.refined
        assert lam == r.lam
        assert cnt == pytest.approx(r.count, rel=1e-4, abs=1e-4)
    theta = gpu.features().double().cpu().numpy()
    assert rel_fro(theta, orc.theta) <= 1e-5
