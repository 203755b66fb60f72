"""Pins of the oracle's dynamic CSC (Algorithm 1, Sec. 4.1)."""

import numpy as np
import pytest

from oracle import chebyshev, dynamic, kmeans, operator, philox
from workloads import DynamicSBM, sbm


@pytest.fixture(scope="module")
def seq():
    g0 = sbm(600, 3, 20.0, 0.05, seed=41)
    dyn = DynamicSBM(g0, seed=42)
    return [g0] + [dyn.step(0.01, 0.005) for _ in range(3)]


@pytest.mark.parametrize("p", [0.5, 0.3, 0.75])
def test_reused_columns_are_bit_identical(seq, p):
    """Exactly the q d columns at the ring cursor (modulo d) are replaced each snapshot; the
    p d others are the previous snapshot's columns, bit for bit (p = 0.3 wraps around)."""
    run = dynamic.DynamicCSC(600, 16, 3, p, 30, seed=43, lloyd_iters=5)
    run.step(seq[0])
    prev = run.theta.copy()
    for t in range(1, 4):
        repl = (run.cursor + np.arange(run.qd)) % 16
        run.step(seq[t])
        kept = np.setdiff1d(np.arange(16), repl)
        assert kept.size == 16 - run.qd
        assert np.array_equal(run.theta[:, kept], prev[:, kept])
        assert not np.any(np.all(run.theta[:, repl] == prev[:, repl], axis=0))
        prev = run.theta.copy()


def test_p_zero_is_static_csc_per_snapshot(seq):
    run = dynamic.DynamicCSC(600, 16, 3, 0.0, 30, seed=44, lloyd_iters=5, tau=0.0)
    for t, g in enumerate(seq, start=1):
        res = run.step(g)
        A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
        R = philox.gaussian_block(600, 16, 0.25, 44, dynamic.stream_id(t, dynamic.SIGNALS))
        a = chebyshev.step_coefficients(30, 2.0, res.lam, "jackson")
        assert np.allclose(run.theta, chebyshev.filter_recurrence(A, 2.0, a, R), atol=1e-13)


def test_forced_refine(seq):
    run = dynamic.DynamicCSC(600, 16, 3, 0.5, 30, seed=45, lloyd_iters=5, tau=0.0)
    for g in seq:
        assert run.step(g).refined
    run = dynamic.DynamicCSC(600, 16, 3, 0.5, 30, seed=45, lloyd_iters=5, tau=1e9)
    res = [run.step(g) for g in seq]
    assert res[0].refined and not any(r.refined for r in res[1:])
    assert all(r.lam == res[0].lam for r in res)


def test_corrupted_lambda_is_refined(seq):
    run = dynamic.DynamicCSC(600, 64, 3, 0.5, 40, seed=46, lloyd_iters=5)
    run.step(seq[0])
    good = run.lam
    run.lam = 1.9  # far above lambda_k: the count of the new columns is far above k
    res = run.step(seq[1])
    assert res.refined and res.lam < 1.9
    assert abs(res.lam - good) < 0.3


def test_dynamic_quality_close_to_sc(seq):
    # Thm. 4.1 bounds C_Theta - C_Phi by 2 sqrt(k/d)(sqrt(k) + c) + 2 sqrt((1 + delta) p) rho
    # (the proof's squared form), which is loose here; the multiplicative error of Sec. 5.2
    # is also checked against a sanity threshold.
    run = dynamic.DynamicCSC(600, 64, 3, 0.5, 60, seed=47, lloyd_iters=20)
    errs = []
    for g in seq:
        res = run.step(g)
        A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
        lam, U = operator.dense_spectrum(A)
        Phi = U[:, :3]
        rng = np.random.default_rng(48)
        best = np.inf
        for _ in range(10):
            lab, _, _ = kmeans.lloyd(Phi, Phi[kmeans.kmeanspp(Phi, 3, rng.random(3))], 30)
            best = min(best, kmeans.cost(Phi, lab))
        c = kmeans.cost(Phi, res.labels)
        errs.append((c - best) / best)
        assert c - best <= 2 * np.sqrt(3 / 64) * (np.sqrt(3) + 3.0) + 2 * np.sqrt(2 * 0.5) * 2 * np.sqrt(3)
    assert max(errs) < 0.25
