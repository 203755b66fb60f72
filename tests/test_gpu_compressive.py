"""GPU parity of compressive k-means (Sec. 2.2, Step 2) against the FP64 oracle, through the
C ABI.  The draws are index work and must match exactly; the sampled rows' k-means follows the
usual near-tie rule; the interpolation is an iterative solve of an ill-conditioned system in
FP32, compared with the oracle's exact minimiser within the error that its residual allows."""

import numpy as np
import pytest
import torch

from oracle import chebyshev, compressive, kmeans as okm, operator, philox
from workloads import sbm
from helpers import say

pytestmark = pytest.mark.gpu

SEED, S_STREAM, K_STREAM = 121, 3, 2


def _features(g, k, d=32, m=80, seed=122):
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    lam, _ = operator.dense_spectrum(A)
    R = philox.gaussian_block(g.n, d, 1 / np.sqrt(d), seed, 1)
    a = chebyshev.step_coefficients(m, 2.0, 0.5 * (lam[k - 1] + lam[k]), "jackson")
    return A, chebyshev.filter_recurrence(A, 2.0, a, R).astype(np.float32)


@pytest.mark.parametrize("r,gamma,ns", [(2, 1e-2, 150), (4, 1e-3, 200)])
def test_matches_oracle(csc, r, gamma, ns):
    say(f"compressive k-means r={r} gamma={gamma} n_sample={ns}")
    k = 4
    g = sbm(2000, k, 16.0, 0.1, seed=123)
    A, F = _features(g, k)
    G = csc.Graph.from_workload(g)
    lab, samp, slab, X, its = csc.compressive_kmeans(
        G, torch.from_numpy(F).cuda(), k, ns, r=r, gamma=gamma, cg_iters=2000, cg_tol=1e-6,
        seed=SEED, sample_stream=S_STREAM, kmeans_stream=K_STREAM, details=True)
    Fd = F.astype(np.float64)
    ref_lab, ref_idx, ref_slab, ref_X = compressive.compressive_kmeans(
        A, Fd, k, ns, philox.uniforms(ns, SEED, S_STREAM), philox.uniforms(k, SEED, K_STREAM),
        20, r, gamma)
    assert np.array_equal(samp.cpu().numpy(), ref_idx)
    agree_s = np.mean(slab.cpu().numpy() == ref_slab)
    X = X.cpu().numpy()
    err = np.max(np.abs(X - ref_X)) / np.max(np.abs(ref_X))
    lab = lab.cpu().numpy()
    agree = np.mean(lab == ref_lab)
    say(f"  CG iterations {its}, sample-label agreement {agree_s:.4f}, max rel error of X {err:.2e}, "
        f"label agreement {agree:.4f}")
    assert agree_s == 1.0
    assert its < 2000
    assert err <= 2e-2
    # a label may differ only where the oracle's two largest interpolants are within that error
    top2 = np.sort(ref_X, axis=1)[:, -2:]
    margin = (top2[:, 1] - top2[:, 0]) / np.max(np.abs(ref_X))
    assert np.all(margin[lab != ref_lab] <= 2 * err)


def test_agrees_with_full_kmeans_on_separable_graphs(csc):
    k = 5
    g = sbm(6000, k, 30.0, 0.02, seed=124)
    _, F = _features(g, k)
    G = csc.Graph.from_workload(g)
    Ft = torch.from_numpy(F).cuda()
    lab = csc.compressive_kmeans(G, Ft, k, 150, seed=SEED).cpu().numpy()
    full, _ = csc.kmeans(Ft, k, 20, seed=SEED, stream_id=K_STREAM)
    full = full.cpu().numpy()
    conf = np.zeros((k, k))
    np.add.at(conf, (lab, full), 1)
    say(f"  agreement with full k-means {conf.max(axis=1).sum() / g.n:.4f}")
    assert conf.max(axis=1).sum() / g.n >= 0.97


def test_combinatorial_graph_and_errors(csc):
    k = 3
    g = sbm(1500, k, 16.0, 0.05, seed=125)
    _, F = _features(g, k)
    G = csc.Graph.from_workload(g, laplacian=csc.LAP_COMBINATORIAL)
    Ft = torch.from_numpy(F).cuda()
    lab, _, _, _, its = csc.compressive_kmeans(G, Ft, k, 100, r=1, gamma=1e-2, details=True)
    conf = np.zeros((k, k))
    np.add.at(conf, (lab.cpu().numpy(), g.labels), 1)
    say(f"  combinatorial: {its} CG iterations, agreement with the planted partition "
        f"{conf.max(axis=1).sum() / g.n:.4f}")
    assert conf.max(axis=1).sum() / g.n >= 0.9
    with pytest.raises(csc.CscError, match="n_sample"):
        csc.compressive_kmeans(G, Ft, k, 2)
    with pytest.raises(csc.CscError, match="gamma"):
        csc.compressive_kmeans(G, Ft, k, 100, gamma=0.0)
