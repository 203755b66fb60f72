"""GPU parity of dynamic CSC (Algorithm 1), the filter adjoint and lmax."""

import numpy as np
import pytest
import torch

from oracle import adjoint, chebyshev, dynamic, kmeans as okm, operator
from workloads import DynamicSBM, gaussian_block, sbm
from helpers import oracle_A, rel_fro, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def seq():
    g0 = sbm(2000, 4, 20.0, 0.05, seed=51)
    dyn = DynamicSBM(g0, seed=52)
    return [g0] + [dyn.step(0.01, 0.005) for _ in range(4)]


# (0.97, 32): one fresh column per snapshot (q d = 1); (0.5, 256): the widest feature block
@pytest.mark.parametrize("keep", [0, 1])
@pytest.mark.parametrize("p,d,tau", [(0.5, 32, 1e-12), (0.5, 64, None), (0.75, 64, None), (0.0, 16, None),
                                     (0.3, 40, None), (0.3, 40, 1e-12), (0.97, 32, None),
                                     (0.5, 256, None)])
def test_dynamic_matches_oracle(csc, seq, p, d, tau, keep):
    say(f"dynamic parity p={p} d={d} tau={tau} keep_iterates={keep}")
    k, m, seed = 4, 40, 53
    orc = dynamic.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10,
                             tau=tau, storage=np.float32)
    gpu = csc.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, tau=tau or 0.0,
                         keep_iterates=keep)
    for t, g in enumerate(seq, start=1):
        G = csc.Graph.from_workload(g)
        lab, lam, ref, cnt = gpu.step(G)
        r = orc.step(g)
        say(f"  t={t} lam gpu={lam:.6f} oracle={r.lam:.6f} refined {ref}/{r.refined} count {cnt:.4f}/{r.count:.4f}")
        assert ref == r.refined
        assert lam == r.lam
        assert cnt == pytest.approx(r.count, rel=1e-4, abs=1e-4)
        theta = gpu.features().double().cpu().numpy()
        assert rel_fro(theta, orc.theta) <= 1e-5
        # labels: equal up to near-ties; compare k-means cost on the oracle's features
        c_gpu = okm.cost(orc.theta, lab.cpu().numpy())
        c_orc = okm.cost(orc.theta, r.labels)
        agree = np.mean(lab.cpu().numpy() == r.labels)
        assert agree > 0.99 or c_gpu == pytest.approx(c_orc, rel=1e-3)


@pytest.mark.parametrize("batch", [1, 4])
@pytest.mark.parametrize("iters", [torch.float32, torch.bfloat16, "bf16s", torch.float16, "f16s"])
def test_dynamic_16bit_forms_cluster_like_the_oracle(csc, seq, iters, batch):
    """Dynamic CSC with BF16 signals and features in every iterate form (kept basis, one
    snapshot at a time or four per batched, graph-replayed recurrence) against the FP64
    oracle's dynamic CSC on the same Philox draws: on the last snapshot the assignment's
    cost C(X; U_k) (eq. CSC_cost) must be within 0.05 of the oracle's.  The SBM (N = 2000,
    k = 4, degree 20, ratio 0.05) is well separated, so both sit near SC's cost, while the
    wrong assignments of tests/quality.py (a random labelling, two clusters merged, half a
    cluster moved) cost at least 0.3 more and fail the same check."""
    import quality as Q

    k, m, d, p, seed = 4, 40, 64, 0.5, 54
    say(f"dynamic 16-bit features, iterates {iters}, batch {batch}")
    gpu = csc.DynamicCSC(2000, d, k, p, m, seed=seed, feat_dtype=torch.bfloat16,
                         iter_dtype=iters, keep_iterates=1, batch=batch, use_graph=batch > 1)
    orc = dynamic.DynamicCSC(2000, d, k, p, m, seed=seed, storage=np.float32)
    labels, lams, _, _ = gpu.steps([csc.Graph.from_workload(g) for g in seq])
    for g in seq:
        r = orc.step(g)
    lam_d, U = operator.dense_spectrum(oracle_A(seq[-1]))
    Phi = U[:, :k]
    lab = labels[-1].cpu().numpy()
    c_gpu, c_orc = okm.cost(Phi, lab), okm.cost(Phi, r.labels)
    say(f"  lambda gpu {lams[-1]:.5f} oracle {r.lam:.5f}; cost gpu {c_gpu:.4f} oracle {c_orc:.4f}")
    assert c_gpu <= c_orc + 0.05
    for name, bad in Q.corruptions(lab).items():
        cb = okm.cost(Phi, bad)
        say(f"  wrong assignment {name}: cost {cb:.4f}")
        assert cb > c_orc + 0.05


@pytest.mark.parametrize("m,w,ckpt", [(0, 3, 0), (1, 5, 0), (7, 16, 3), (30, 20, 0), (60, 64, 8)])
def test_adjoint_matches_oracle(csc, m, w, ckpt):
    say(f"adjoint parity m={m} w={w} ckpt={ckpt}")
    g = sbm(1500, 4, 10.0, 0.1, seed=55)
    A = oracle_A(g)
    G = csc.Graph.from_workload(g)
    X = gaussian_block(g.n, w, 0.3, seed=56)
    Gr = gaussian_block(g.n, w, 1.0, seed=57)
    a = chebyshev.step_coefficients(m, 2.0, 0.4, "jackson")
    dX, da, dA = csc.filter_backward(G, a, torch.from_numpy(X).cuda(), torch.from_numpy(Gr).cuda(),
                                     ckpt_every=ckpt)
    rX, rda, rdA = adjoint.filter_backward(A, 2.0, a, X.astype(np.float64), Gr.astype(np.float64))
    assert rel_fro(dX.cpu().numpy(), rX) <= 1e-5
    assert rel_fro(da.cpu().numpy(), rda) <= 1e-5
    if m > 0:
        assert rel_fro(dA.cpu().numpy(), rdA) <= 1e-5
    else:
        assert np.all(dA.cpu().numpy() == 0)


def test_weight_chain_matches_oracle_and_finite_differences(csc):
    """The chain from dl/dA to the symmetric edge weights (Sec. 2.1, A = D^{-1/2} W D^{-1/2})
    on C4's gradient-check graph (SBM N = 2000, k = 4, degree 10) with random symmetric
    weights: the GPU chain of the GPU's dA against the oracle chain of the oracle's dA, and
    the oracle's chain against FP64 central differences of the loss on a few edges."""
    from workloads import seed_for
    say("weight chain, C4 gradient-check graph")
    g = sbm(2000, 4, 10.0, 0.1, seed=seed_for(4, "graph") + 7)
    rng = np.random.default_rng(71)
    mir = adjoint.mirror_index(g.n, g.rowptr, g.colidx)
    w = g.w * rng.uniform(0.5, 2.0, size=g.w.shape)
    w = 0.5 * (w + w[mir])
    g.w = w
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, w)
    G = csc.Graph.from_workload(g)
    X = gaussian_block(g.n, 8, 0.3, seed=72)
    Gr = gaussian_block(g.n, 8, 1.0, seed=73)
    a = chebyshev.step_coefficients(30, 2.0, 0.5, "jackson")
    _, _, dA = csc.filter_backward(G, a, torch.from_numpy(X).cuda(), torch.from_numpy(Gr).cuda())
    dW = csc.weight_gradient(G, dA).cpu().numpy()
    _, _, rdA = adjoint.filter_backward(A, 2.0, a, X.astype(np.float64), Gr.astype(np.float64))
    rdW = adjoint.weight_gradient(g.n, g.rowptr, g.colidx, w, rdA)
    err = rel_fro(dW, rdW)
    say(f"  dW relative error {err:.3e}")
    assert err <= 1e-5
    assert np.array_equal(dW, dW[mir])

    def loss(wv):
        Av, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, wv)
        return float(np.sum(Gr * chebyshev.filter_recurrence(Av, 2.0, a, X.astype(np.float64))))

    h = 1e-6
    for e in rng.integers(0, len(w), size=4):
        wp, wm = w.copy(), w.copy()
        for q in {int(e), int(mir[e])}:
            wp[q] += h
            wm[q] -= h
        fd = (loss(wp) - loss(wm)) / (2 * h)
        assert rdW[e] == pytest.approx(fd, rel=1e-6, abs=1e-8)
        assert dW[e] == pytest.approx(fd, rel=1e-4, abs=1e-6)


def test_adjoint_c4_full_size_sampled_columns(csc):
    """C4 at full size (SBM N=200k, degree 20, w=64, m=60, checkpoints every 8 iterates):
    the adjoint is column-separable, so the 64-column run is checked on two sampled columns
    against a two-column run, and that run against the FP64 oracle."""
    from workloads import seed_for
    say("adjoint C4 full size, sampled columns")
    g = sbm(200_000, 20, 20.0, 0.1, seed=seed_for(4, "graph"))
    A = oracle_A(g)
    G = csc.Graph.from_workload(g)
    X = gaussian_block(g.n, 64, 0.125, seed=seed_for(4, "signals"))
    Gr = gaussian_block(g.n, 64, 1.0, seed=seed_for(4, "probes"))
    a = chebyshev.step_coefficients(60, 2.0, 0.5, "jackson")
    dX, da, dA = csc.filter_backward(G, a, torch.from_numpy(X).cuda(), torch.from_numpy(Gr).cuda(),
                                     ckpt_every=8)
    cols = [5, 40]
    Xs, Gs = np.ascontiguousarray(X[:, cols]), np.ascontiguousarray(Gr[:, cols])
    dXs, das, dAs = csc.filter_backward(G, a, torch.from_numpy(Xs).cuda(), torch.from_numpy(Gs).cuda(),
                                        ckpt_every=8)
    assert np.allclose(dX.cpu().numpy()[:, cols], dXs.cpu().numpy(), rtol=1e-6, atol=1e-9)
    rX, rda, rdA = adjoint.filter_backward(A, 2.0, a, Xs.astype(np.float64), Gs.astype(np.float64))
    assert rel_fro(dXs.cpu().numpy(), rX) <= 1e-5
    assert rel_fro(das.cpu().numpy(), rda) <= 1e-5
    assert rel_fro(dAs.cpu().numpy(), rdA) <= 1e-5
    assert np.all(np.isfinite(da.cpu().numpy())) and np.all(np.isfinite(dA.cpu().numpy()))


def test_autograd_function(csc):
    from paper_1706_03591_amd import cheb_filter_autograd
    g = sbm(800, 3, 10.0, 0.1, seed=58)
    A = oracle_A(g)
    G = csc.Graph.from_workload(g)
    X = torch.from_numpy(gaussian_block(g.n, 8, 0.3, seed=59)).cuda().requires_grad_(True)
    a = torch.tensor(chebyshev.step_coefficients(12, 2.0, 0.5, "jackson"), dtype=torch.float64,
                     requires_grad=True)
    vals = torch.from_numpy(A.data.astype(np.float32)).cuda().requires_grad_(True)
    W = torch.from_numpy(gaussian_block(g.n, 8, 1.0, seed=60)).cuda()
    Y = cheb_filter_autograd(X, a, G, edge_vals=vals)
    loss = (Y * W).sum()
    loss.backward()
    rX, rda, rdA = adjoint.filter_backward(A, 2.0, a.detach().numpy(), X.detach().cpu().double().numpy(),
                                           W.cpu().double().numpy())
    assert rel_fro(X.grad.cpu().numpy(), rX) <= 1e-5
    assert rel_fro(a.grad.numpy(), rda) <= 1e-5
    assert rel_fro(vals.grad.cpu().numpy(), rdA) <= 1e-5


def test_lmax_estimate_is_upper_bound(csc):
    g = sbm(600, 3, 8.0, 0.2, seed=61)
    A = oracle_A(g)
    lam, _ = operator.dense_spectrum(A)
    G = csc.Graph.from_workload(g)
    assert G.lmax(0) == 2.0
    est = G.lmax(100)
    say(f"  lmax est {est:.6f} true {lam[-1]:.6f}")
    assert lam[-1] * 0.999 <= est <= 2.0


# batch 1 with kept iterates: the sequence call starts each next recurrence beside the
# current k-means (one buffer), which must not change any result
@pytest.mark.parametrize("batch,use_graph,iters,p,d", [(1, True, torch.float32, 0.5, 32),
                                                       (1, False, "bf16s", 0.5, 32),
                                                       (1, False, torch.float32, 0.3, 40),
                                                       (3, False, torch.float32, 0.5, 32),
                                                       (4, True, torch.float32, 0.5, 32),
                                                       (4, True, "bf16s", 0.5, 32),
                                                       (4, True, torch.float32, 0.3, 40)])
def test_batched_and_graph_forms_equal_sequential(csc, seq, batch, use_graph, iters, p, d):
    say(f"batched dynamic batch={batch} graph={use_graph} iterates={iters} p={p} d={d}")
    k, m, seed = 4, 40, 62
    ref = csc.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, keep_iterates=1,
                         iter_dtype=iters)
    G_ref = [csc.Graph.from_workload(g) for g in seq]
    ref_out = [ref.step(G) for G in G_ref]
    ref_theta = ref.features()
    bat = csc.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, keep_iterates=1,
                         batch=batch, use_graph=use_graph, iter_dtype=iters)
    G_bat = [csc.Graph.from_workload(g) for g in seq]
    labels, lams, refs, cnts = bat.steps(G_bat)
    for t in range(len(seq)):
        assert lams[t] == ref_out[t][1]
        assert refs[t] == ref_out[t][2]
        assert cnts[t] == ref_out[t][3]
        assert torch.equal(labels[t], ref_out[t][0])
    assert torch.equal(bat.features(), ref_theta)


# one-pass batches (no kept iterates): a batch is filtered at the cut-off in force when it
# starts, with its moments; decisions come from the moments, and snapshots whose cut-off
# changed within the batch are filtered again.  Against one snapshot at a time without kept
# iterates: the same cut-offs, refinements and labels, bit-identical features (the same
# kernels in the same order).  The accepted counts are two estimates of the same quantity,
# the moment series here and <R, Y> with the stored output Y there, so they differ by the
# rounding of Y and of the iterates: up to 1e-5 relative with FP32 iterates, 5e-3 with
# 16-bit ones (the acceptance half-width is at least 0.5).  tau = 1e-12 refines every
# snapshot, so every block is filtered again.
@pytest.mark.parametrize("batch,use_graph,iters,p,d,tau", [(4, True, torch.float32, 0.5, 32, None),
                                                           (3, False, torch.float16, 0.3, 40, None),
                                                           (4, True, "bf16s", 0.5, 32, 1e-12),
                                                           (2, True, "f16s", 0.75, 64, None),
                                                           (4, False, torch.float32, 0.5, 32, 1e-12)])
def test_onepass_batches_equal_sequential(csc, seq, batch, use_graph, iters, p, d, tau):
    say(f"one-pass batches batch={batch} graph={use_graph} iterates={iters} p={p} d={d} tau={tau}")
    k, m, seed = 4, 40, 63
    ref = csc.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, keep_iterates=0,
                         iter_dtype=iters, tau=tau or 0.0)
    ref_out = [ref.step(csc.Graph.from_workload(g)) for g in seq]
    bat = csc.DynamicCSC(2000, d, k, p, m, seed=seed, lloyd_iters=10, keep_iterates=0,
                         batch=batch, use_graph=use_graph, iter_dtype=iters, tau=tau or 0.0)
    labels, lams, refs, cnts = bat.steps([csc.Graph.from_workload(g) for g in seq])
    for t in range(len(seq)):
        say(f"  t={t + 1} lambda {lams[t]:.6f} refined {refs[t]} count {cnts[t]:.5f} / {ref_out[t][3]:.5f}")
        assert lams[t] == ref_out[t][1]
        assert refs[t] == ref_out[t][2]
        assert torch.equal(labels[t], ref_out[t][0])
        if refs[t]:
            # both the count at the refined cut-off from the same doubled moments (computed by
            # the batched and by the single step kernel)
            assert cnts[t] == pytest.approx(ref_out[t][3], rel=1e-12)
        elif iters == torch.float32:
            assert cnts[t] == pytest.approx(ref_out[t][3], rel=1e-5)
        else:
            assert cnts[t] == pytest.approx(ref_out[t][3], abs=5e-3)
    assert torch.equal(bat.features(), ref.features())


@pytest.mark.parametrize("variant", [0, 1, 2])
def test_dynamic_kernel_shape_does_not_change_results(csc, seq, variant):
    """The row-group x column-tile shape (the autotuner's choice) changes only the order of
    block partial sums, never the per-element arithmetic of the recurrence."""
    say(f"dynamic variant={variant}")
    k, m, d, seed = 4, 40, 32, 62
    ref = csc.DynamicCSC(2000, d, k, 0.5, m, seed=seed, lloyd_iters=10, keep_iterates=1)
    alt = csc.DynamicCSC(2000, d, k, 0.5, m, seed=seed, lloyd_iters=10, keep_iterates=1,
                         variant=variant)
    for g in seq:
        G1, G2 = csc.Graph.from_workload(g), csc.Graph.from_workload(g)
        l1, lam1, r1, c1 = ref.step(G1)
        l2, lam2, r2, c2 = alt.step(G2)
        assert c2 == pytest.approx(c1, rel=1e-9, abs=1e-9)
        assert lam2 == lam1 and r2 == r1
        assert torch.equal(l1, l2)
    assert torch.equal(ref.features(), alt.features())


def test_autotuned_variant_drives_dynamic_state(csc, seq):
    say("autotune -> dynamic variant")
    G = csc.Graph.from_workload(seq[0])
    v = G.autotune(16, torch.float32)
    assert 0 <= v < 4
    dyn = csc.DynamicCSC(2000, 32, 4, 0.5, 40, seed=62, lloyd_iters=10, keep_iterates=1, variant=v)
    lab, lam, _, cnt = dyn.step(G)
    assert 0.0 < lam < 2.0 and lab.min() >= 0 and lab.max() < 4
    with pytest.raises(csc.CscError):
        csc.DynamicCSC(2000, 32, 4, 0.5, 40, seed=62, variant=4)
