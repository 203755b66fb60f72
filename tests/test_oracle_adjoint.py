"""Pins of the oracle's filter adjoint: finite differences, Daleckii-Krein, h(L~)^T G."""

import numpy as np
import pytest
import scipy.sparse as sp

from oracle import adjoint, chebyshev, operator
from workloads import sbm


@pytest.fixture(scope="module")
def tiny():
    g = sbm(60, 3, 6.0, 0.2, seed=31)
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    rng = np.random.default_rng(32)
    X = rng.standard_normal((g.n, 3))
    G = rng.standard_normal((g.n, 3))
    a = chebyshev.step_coefficients(7, 2.0, 0.6, "jackson")
    return A, X, G, a


def _loss(A, a, X, G, lmax=2.0):
    return float(np.sum(G * chebyshev.filter_recurrence(A, lmax, a, X)))


def test_finite_differences(tiny):
    A, X, G, a = tiny
    dX, da, dA = adjoint.filter_backward(A, 2.0, a, X, G)
    h = 1e-6
    rng = np.random.default_rng(33)
    for _ in range(6):
        i, c = rng.integers(0, X.shape[0]), rng.integers(0, X.shape[1])
        Xp, Xm = X.copy(), X.copy()
        Xp[i, c] += h
        Xm[i, c] -= h
        fd = (_loss(A, a, Xp, G) - _loss(A, a, Xm, G)) / (2 * h)
        assert dX[i, c] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    for j in range(len(a)):
        ap, am = a.copy(), a.copy()
        ap[j] += h
        am[j] -= h
        fd = (_loss(A, ap, X, G) - _loss(A, am, X, G)) / (2 * h)
        assert da[j] == pytest.approx(fd, rel=1e-6, abs=1e-8)
    for e in rng.integers(0, A.nnz, size=8):
        Ap, Am = A.copy(), A.copy()
        Ap.data[e] += h
        Am.data[e] -= h
        fd = (_loss(Ap, a, X, G) - _loss(Am, a, X, G)) / (2 * h)
        assert dA[e] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def test_lmax_not_two(tiny):
    A, X, G, a = tiny
    lmax = 1.9
    dX, da, dA = adjoint.filter_backward(A, lmax, a, X, G)
    h = 1e-6
    e = 5
    Ap, Am = A.copy(), A.copy()
    Ap.data[e] += h
    Am.data[e] -= h
    fd = (_loss(Ap, a, X, G, lmax) - _loss(Am, a, X, G, lmax)) / (2 * h)
    assert dA[e] == pytest.approx(fd, rel=1e-6, abs=1e-8)


def _cheb_derivative_coeffs(a):
    """Coefficients of f' for f = sum a_j T_j (textbook recurrence d_{j-1} = d_{j+1} + 2 j a_j,
    with the j = 0 term halved)."""
    m = len(a) - 1
    d = np.zeros(m + 2)
    for j in range(m, 0, -1):
        d[j - 1] = d[j + 1] + 2 * j * a[j]
    d[0] *= 0.5
    return d[:m]


def test_daleckii_krein(tiny):
    A, X, G, a = tiny
    Lt = operator.scaled_laplacian(A, 2.0).toarray()
    x, V = np.linalg.eigh(0.5 * (Lt + Lt.T))
    f = chebyshev.cheb_eval(a, x)
    fp = chebyshev.cheb_eval(_cheb_derivative_coeffs(a), x) if len(a) > 1 else 0 * x
    dx = x[:, None] - x[None, :]
    close = np.abs(dx) < 1e-9
    Gam = np.where(close, 0.5 * (fp[:, None] + fp[None, :]),
                   (f[:, None] - f[None, :]) / np.where(close, 1.0, dx))
    grad_Lt = V @ (Gam * (V.T @ G @ X.T @ V)) @ V.T
    _, _, dA = adjoint.filter_backward(A, 2.0, a, X, G)
    rows = np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))
    expect = -1.0 * grad_Lt[rows, A.indices]  # dA = -beta dL~ with beta = 2 / lmax = 1
    assert np.max(np.abs(dA - expect)) <= 1e-10 * np.max(np.abs(expect))


def test_input_gradient_is_filter_transpose(tiny):
    A, X, G, a = tiny
    dX, _, _ = adjoint.filter_backward(A, 2.0, a, X, G)
    lam, U = operator.dense_spectrum(A)
    expect = chebyshev.filter_dense(lam, U, a, 2.0, G)
    assert np.allclose(dX, expect, atol=1e-12)


def test_weight_chain_finite_differences():
    """dl/dw of an undirected edge weight (both stored copies moved together), through
    A = D^{-1/2} W D^{-1/2} and the degrees, against central differences of the loss."""
    g = sbm(60, 3, 6.0, 0.2, seed=31)
    rng = np.random.default_rng(34)
    w = g.w * rng.uniform(0.5, 2.0, size=g.w.shape)
    mir = adjoint.mirror_index(g.n, g.rowptr, g.colidx)
    w = 0.5 * (w + w[mir])  # symmetric weights
    X = rng.standard_normal((g.n, 3))
    G = rng.standard_normal((g.n, 3))
    a = chebyshev.step_coefficients(9, 2.0, 0.7, "jackson")
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, w)
    _, _, dA = adjoint.filter_backward(A, 2.0, a, X, G)
    dw = adjoint.weight_gradient(g.n, g.rowptr, g.colidx, w, dA)
    assert np.array_equal(dw, dw[mir])
    h = 1e-6

    def loss(wv):
        Av, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, wv)
        return _loss(Av, a, X, G)

    for e in rng.integers(0, len(w), size=10):
        wp, wm = w.copy(), w.copy()
        for q in {int(e), int(mir[e])}:
            wp[q] += h
            wm[q] -= h
        fd = (loss(wp) - loss(wm)) / (2 * h)
        assert dw[e] == pytest.approx(fd, rel=1e-6, abs=1e-9)


def test_mirror_index_is_an_involution():
    g = sbm(200, 4, 8.0, 0.2, seed=35)
    mir = adjoint.mirror_index(g.n, g.rowptr, g.colidx)
    assert np.array_equal(mir[mir], np.arange(len(mir)))
    rows = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    assert np.array_equal(rows[mir], g.colidx) and np.array_equal(g.colidx[mir], rows)
