"""Sanity of the seeded input generators (shapes, symmetry, degrees, determinism)."""

import numpy as np
import scipy.sparse as sp

from workloads import DynamicSBM, block_sizes_zipf, chung_lu, gaussian_block, sbm


def _check_csr(g):
    W = sp.csr_matrix((g.w, g.colidx, g.rowptr), shape=(g.n, g.n))
    assert abs(W - W.T).sum() == 0
    assert W.diagonal().sum() == 0
    for r in range(0, g.n, max(1, g.n // 50)):
        c = g.colidx[g.rowptr[r]:g.rowptr[r + 1]]
        assert np.all(np.diff(c) > 0)
    assert np.all(g.w > 0)


def test_sbm_degree_and_determinism():
    g = sbm(2000, 4, 10.0, 0.1, seed=1)
    _check_csr(g)
    assert abs(g.nnz / g.n - 10.0) < 0.5
    g2 = sbm(2000, 4, 10.0, 0.1, seed=1)
    assert np.array_equal(g.colidx, g2.colidx)
    # intra-block fraction of edges matches q1 / q2
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    intra = np.mean(g.labels[rows] == g.labels[g.colidx])
    assert abs(intra - 1 / (1 + 0.1 * 3)) < 0.05


def test_zipf_sizes():
    s = block_sizes_zipf(1_000_000, 50, 1.2)
    assert s.sum() == 1_000_000 and s[0] > 300_000 and s[-1] > 2000
    assert np.all(np.diff(s) <= 0)


def test_dynamic_sequence_changes_little():
    g = sbm(3000, 5, 12.0, 0.1, seed=2)
    dyn = DynamicSBM(g, seed=3)
    g1 = dyn.step(0.01, 0.005)
    _check_csr(g1)
    k0, k1 = g.edge_keys(), g1.edge_keys()
    changed = len(np.setxor1d(k0, k1)) / len(k0)
    assert 0.01 < changed < 0.06
    assert np.sum(g.labels != g1.labels) == 15


def test_chung_lu_power_law():
    g = chung_lu(20000, 20, 20.0, 2.5, 0.1, seed=4)
    _check_csr(g)
    deg = np.diff(g.rowptr)
    assert abs(deg.mean() - 20.0) < 1.0
    assert deg.max() > 10 * deg.mean()


def test_gaussian_block():
    x = gaussian_block(1000, 16, 0.25, seed=5)
    assert x.dtype == np.float32 and x.shape == (1000, 16)
    assert abs(x.std() - 0.25) < 0.01
