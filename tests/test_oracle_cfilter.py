"""The oracle's multi-core C filter against the Python oracle's recurrence (Sec. 2.2, Step 1)."""

import numpy as np
import pytest

from oracle import cfilter, chebyshev, operator
from workloads import gaussian_block, sbm
from helpers import oracle_A, rel_fro


@pytest.fixture(scope="module")
def graph():
    return sbm(3000, 6, 12.0, 0.1, seed=17)


@pytest.mark.parametrize("m", [0, 1, 2, 60])
@pytest.mark.parametrize("w", [1, 7])
def test_c_filter_equals_python_recurrence(graph, m, w):
    A = oracle_A(graph)
    X = gaussian_block(graph.n, w, 0.3, seed=m + w).astype(np.float64)
    a = chebyshev.step_coefficients(m, 2.0, 0.4, "jackson")
    Y, used = cfilter.filter_recurrence_c(A, 2.0, a, X)
    assert used >= 1
    assert rel_fro(Y, chebyshev.filter_recurrence(A, 2.0, a, X)) <= 1e-13


def test_c_filter_combinatorial_and_lmax(graph):
    g = graph
    L = operator.combinatorial_laplacian(g.n, g.rowptr, g.colidx, g.w)
    lmax = operator.anderson_morley_bound(g.n, g.rowptr, g.colidx, g.w)
    X = gaussian_block(g.n, 3, 1.0, seed=5).astype(np.float64)
    a = chebyshev.step_coefficients(30, lmax, 0.3 * lmax, "none")
    Y, _ = cfilter.filter_recurrence_c(L, lmax, a, X)
    assert rel_fro(Y, chebyshev.filter_recurrence(L, lmax, a, X)) <= 1e-13


def test_c_filter_same_bits_for_any_thread_count(graph):
    A = oracle_A(graph)
    X = gaussian_block(graph.n, 5, 0.3, seed=3).astype(np.float64)
    a = chebyshev.step_coefficients(40, 2.0, 0.5, "jackson")
    Y1, u1 = cfilter.filter_recurrence_c(A, 2.0, a, X, threads=1)
    Y4, u4 = cfilter.filter_recurrence_c(A, 2.0, a, X, threads=4)
    assert (u1, u4) == (1, 4)
    assert np.array_equal(Y1, Y4)
