"""GPU parity of the Philox draws and of k-means (assign, update, k-means++, Lloyd)."""

import numpy as np
import pytest
import torch

from oracle import kmeans as okm
from oracle import philox
from workloads import gaussian_block
from helpers import near_tie_exempt, say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("dtype", [torch.float64, torch.float32, torch.bfloat16])
def test_randn_matches_oracle_philox(csc, dtype):
    say(f"randn parity {dtype}")
    n, w = 3001, 7
    X = csc.randn(n, w, seed=123456789012, stream_id=(5 << 32) + 17, sigma=0.3, dtype=dtype)
    ref = philox.gaussian_block(n, w, 0.3, 123456789012, (5 << 32) + 17)
    got = X.double().cpu().numpy()
    if dtype == torch.float64:
        assert np.max(np.abs(got - ref)) <= 1e-13
    elif dtype == torch.float32:
        assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)) <= 1.2e-7
    else:
        assert np.max(np.abs(got - ref) / np.maximum(np.abs(ref), 1e-30)) <= 8e-3
    part = csc.randn(100, w, seed=123456789012, stream_id=(5 << 32) + 17, sigma=0.3,
                     dtype=torch.float64, row0=2000)
    assert np.array_equal(part.cpu().numpy(), X.double().cpu().numpy()[2000:2100]) or dtype != torch.float64


def test_uniforms_bit_exact(csc):
    u = csc.uniforms(1000, seed=42, stream_id=34).cpu().numpy()
    assert np.array_equal(u, philox.uniforms(1000, 42, 34))


def _mixture(n, d, k, seed, spread=6.0):
    rng = np.random.default_rng(seed)
    centers = rng.standard_normal((k, d)) * spread
    lab = rng.integers(0, k, size=n)
    return (centers[lab] + rng.standard_normal((n, d))).astype(np.float32)


# (4099, 256, 240): the largest d and k the k-means calls take (two centroid chunks per
# 256-row panel)
@pytest.mark.parametrize("n,d,k", [(5000, 32, 5), (20011, 128, 50), (3000, 256, 200), (777, 17, 1),
                                   (4099, 256, 240)])
def test_assign_matches_oracle(csc, n, d, k):
    say(f"kmeans assign n={n} d={d} k={k}")
    F = _mixture(n, d, max(k, 2), seed=n)
    C = F[np.random.default_rng(1).choice(n, size=k, replace=False)] + 0.01
    lab, best = csc.kmeans_assign(torch.from_numpy(F).cuda(), torch.from_numpy(C).cuda())
    lab = lab.cpu().numpy()
    ref, d2 = okm.assign(F.astype(np.float64), C.astype(np.float64))
    exempt, ok_tie = near_tie_exempt(F.astype(np.float64), C.astype(np.float64), lab)
    mism = (lab != ref) & ~(exempt & ok_tie)
    assert mism.sum() == 0
    assert np.allclose(best.cpu().numpy(), d2, rtol=1e-6)


@pytest.mark.parametrize("n,d,k,bf", [(5000, 32, 5, False), (20011, 128, 50, True), (3000, 256, 200, False),
                                      (777, 17, 3, False)])
def test_assign_fused_sums_and_counts(csc, n, d, k, bf):
    """The optional Lloyd partial sums of the assignment call: for the labels it returns,
    sums[c] = sum of the rows labelled c and counts[c] their number (Sec. 2.1, the update
    step of k-means); FP64 sums in the oracle, one FP32 rounding on the GPU."""
    say(f"kmeans assign with sums n={n} d={d} k={k} bf16={bf}")
    F = _mixture(n, d, max(k, 2), seed=n + 1)
    Ft = torch.from_numpy(F).cuda()
    if bf:
        Ft = Ft.to(torch.bfloat16)
    C = F[np.random.default_rng(2).choice(n, size=k, replace=False)] + 0.01
    lab, _, S, cnt = csc.kmeans_assign(Ft, torch.from_numpy(C).cuda(), sums=True)
    lab = lab.cpu().numpy()
    F64 = Ft.double().cpu().numpy()
    ref = np.zeros((k, d))
    np.add.at(ref, lab, F64)
    assert np.array_equal(cnt.cpu().numpy(), np.bincount(lab, minlength=k))
    scale = np.abs(F64).max() * n * 2.0 ** -40  # fixed-point resolution of the sums
    err = np.abs(S.cpu().numpy().astype(np.float64) - ref)
    assert np.all(err <= 2.0 ** -24 * np.abs(ref) + 2 * scale)
    # the same labels as the call without sums
    lab2, _ = csc.kmeans_assign(Ft, torch.from_numpy(C).cuda())
    assert np.array_equal(lab2.cpu().numpy(), lab)


def test_assign_exact_ties_lowest_index(csc):
    F = np.array([[0.0, 0.0], [1.0, 1.0], [0.5, 0.5]], dtype=np.float32)
    C = np.array([[1.0, 1.0], [0.0, 0.0], [0.0, 0.0], [1.0, 1.0]], dtype=np.float32)
    lab, _ = csc.kmeans_assign(torch.from_numpy(F).cuda(), torch.from_numpy(C).cuda())
    assert lab.cpu().tolist() == [1, 0, 0]


@pytest.mark.parametrize("n,d,k", [(4000, 64, 8), (20011, 128, 50), (3000, 256, 200), (9001, 48, 150)])
def test_assign_bf16_features(csc, n, d, k):
    # (3000, 256, 200) and (9001, 48, 150) need several LDS chunks of centroids (two row tiles
    # per wave)
    say(f"kmeans assign bf16 n={n} d={d} k={k}")
    F = _mixture(n, d, max(k, 2), seed=3)
    Fb = torch.from_numpy(F).cuda().to(torch.bfloat16)
    C = F[np.random.default_rng(4).choice(n, size=k, replace=False)] + 0.01
    lab, _ = csc.kmeans_assign(Fb, torch.from_numpy(C).cuda())
    F64 = Fb.double().cpu().numpy()
    ref, _ = okm.assign(F64, C.astype(np.float64))
    exempt, ok_tie = near_tie_exempt(F64, C.astype(np.float64), lab.cpu().numpy())
    assert np.sum((lab.cpu().numpy() != ref) & ~(exempt & ok_tie)) == 0


@pytest.mark.parametrize("n,d,k,dtype", [(5000, 32, 5, torch.float32), (100003, 128, 50, torch.float32),
                                         (3000, 256, 200, torch.float32), (9001, 50, 20, torch.float32),
                                         (20011, 200, 130, torch.float32),
                                         (100003, 128, 50, torch.bfloat16),
                                         (600000, 256, 200, torch.bfloat16)])
def test_update_matches_oracle(csc, n, d, k, dtype):
    # d = 50: rows not in whole 16-byte pieces (masked loads); d = 200, k = 130: 32-column
    # groups, the last one partly past d; N = 600000: 586 row blocks (not a multiple of the
    # eight XCDs) times eight column groups
    say(f"kmeans update n={n} d={d} k={k} {dtype}")
    F = torch.from_numpy(_mixture(n, d, k, seed=n + 1)).to(dtype)
    rng = np.random.default_rng(2)
    lab = rng.integers(0, k, size=n).astype(np.int32)
    lab[lab == k - 1] = 0  # cluster k-1 empty: keeps its previous centroid
    C0 = rng.standard_normal((k, d)).astype(np.float32)
    Cg = torch.from_numpy(C0.copy()).cuda()
    Fg = F.cuda()
    counts = csc.kmeans_update(Fg, torch.from_numpy(lab).cuda(), Cg)
    ref, rc = okm.update(F.double().numpy(), lab, C0.astype(np.float64))
    assert np.array_equal(counts.cpu().numpy(), rc)
    got = Cg.cpu().numpy()
    assert np.array_equal(got[k - 1], C0[k - 1])
    assert np.max(np.abs(got - ref)) <= 1e-5 * max(1.0, np.max(np.abs(ref)))
    Cg2 = torch.from_numpy(C0.copy()).cuda()
    csc.kmeans_update(Fg, torch.from_numpy(lab).cuda(), Cg2)
    assert torch.equal(Cg, Cg2)
    # the same rows with a leading dimension of d + 8 (row-wise max scan, and unaligned rows
    # where (d + 8) x element size is not a multiple of 16 bytes): fixed-point sums, same bits
    Fp = torch.zeros((n, d + 8), dtype=dtype, device="cuda")
    Fp[:, :d] = Fg
    Cg3 = torch.from_numpy(C0.copy()).cuda()
    csc.kmeans_update(Fp[:, :d], torch.from_numpy(lab).cuda(), Cg3)
    assert torch.equal(Cg, Cg3)


def _fixed_point_centroids(F64, lab, k, C0):
    """The update's arithmetic written out in numpy: each value rounded half to even to a
    multiple of 2^-S (S = 62 - e - ceil(log2 n), kept within [-60, 120], max |F| < 2^e), the
    integers of each label added exactly, the sum scaled back in FP64, divided by the count
    and rounded once to FP32; labels outside [0, k) ignored, empty clusters unchanged."""
    n = F64.shape[0]
    _, e = np.frexp(np.float32(np.abs(F64).max()))
    S = int(np.clip(62 - int(e) - (n - 1).bit_length(), -60, 120))
    ok = (lab >= 0) & (lab < k)
    lv = lab[ok]
    order = np.argsort(lv, kind="stable")
    y = np.rint(np.ldexp(F64[ok][order], S)).astype(np.int64)
    cnt = np.bincount(lv, minlength=k)
    C = C0.copy()
    nz = np.flatnonzero(cnt)
    starts = np.concatenate([[0], np.cumsum(cnt)[:-1]])[nz]
    sums = np.add.reduceat(y, starts, axis=0)
    C[nz] = (np.ldexp(sums.astype(np.float64), -S) / cnt[nz, None]).astype(np.float32)
    return C, cnt


@pytest.mark.parametrize("n,d,k,dtype,ld_pad", [(600000, 256, 200, torch.bfloat16, 0),
                                                (100003, 128, 3, torch.float32, 0),
                                                (3000, 256, 200, torch.float32, 0),
                                                (9001, 50, 20, torch.bfloat16, 0),
                                                (20000, 17, 5, torch.float32, 3),
                                                (2000, 32, 1, torch.float32, 0),
                                                (511, 8, 3, torch.bfloat16, 0)])
def test_update_sums_are_exact_fixed_point(csc, n, d, k, dtype, ld_pad):
    """The Lloyd update (Sec. 2.1, the update step of k-means) returns, bit for bit, the means
    of the 64-bit fixed-point sums: large n with FP64 runs inside a chunk, small n with each
    value converted on its own, labels of 30 000+ rows over many chunks, masked rows (d = 50,
    d = 17 with a leading dimension of d + 3), out-of-range labels and an empty cluster."""
    say(f"kmeans update exact n={n} d={d} k={k} {dtype} ld=d+{ld_pad}")
    rng = np.random.default_rng(n + k)
    F = torch.from_numpy(_mixture(n, d, k, seed=n + 7)).to(dtype)
    lab = rng.integers(0, k, size=n).astype(np.int32)
    if k > 1:
        lab[lab == k - 1] = 0  # cluster k - 1 empty: keeps its previous centroid
    lab[rng.choice(n, size=n // 100, replace=False)] = -1
    lab[rng.choice(n, size=n // 100, replace=False)] = k
    C0 = rng.standard_normal((k, d)).astype(np.float32)
    ref, rcnt = _fixed_point_centroids(F.double().numpy(), lab, k, C0)
    if ld_pad:
        Fg = torch.zeros((n, d + ld_pad), dtype=dtype, device="cuda")
        Fg[:, :d] = F.cuda()
        Fg = Fg[:, :d]
    else:
        Fg = F.cuda()
    Cg = torch.from_numpy(C0.copy()).cuda()
    counts = csc.kmeans_update(Fg, torch.from_numpy(lab).cuda(), Cg)
    assert np.array_equal(counts.cpu().numpy(), rcnt)
    assert np.array_equal(Cg.cpu().numpy().view(np.uint32), ref.view(np.uint32))


def test_update_without_valid_labels_keeps_centroids(csc):
    """Every label outside [0, k): no cluster has a row, so every centroid stays as it was
    and every count is zero (no chunk to sum)."""
    n, d, k = 3000, 40, 7
    F = torch.from_numpy(_mixture(n, d, k, seed=11)).cuda()
    lab = np.where(np.arange(n) % 2 == 0, -1, k).astype(np.int32)
    C0 = np.random.default_rng(12).standard_normal((k, d)).astype(np.float32)
    Cg = torch.from_numpy(C0.copy()).cuda()
    counts = csc.kmeans_update(F, torch.from_numpy(lab).cuda(), Cg)
    assert np.array_equal(counts.cpu().numpy(), np.zeros(k, dtype=np.int32))
    assert np.array_equal(Cg.cpu().numpy(), C0)


@pytest.mark.parametrize("n,d,k,dtype", [(3000, 16, 6, torch.float32), (50000, 64, 20, torch.float32),
                                         (3000, 200, 8, torch.float32),
                                         (20011, 128, 40, torch.bfloat16),
                                         (6001, 256, 60, torch.bfloat16)])
def test_kmeanspp_matches_oracle(csc, n, d, k, dtype):
    # the BF16 cases read one (d = 128) or two (d = 256) 16-byte pieces per lane; well
    # separated mixtures make the triangle-inequality skip fire on most rows of later passes
    say(f"kmeans++ n={n} d={d} k={k} {dtype}")
    F = torch.from_numpy(_mixture(n, d, k, seed=7)).to(dtype)
    Fn = F.double().numpy()
    u = csc.uniforms(k, seed=99, stream_id=2)
    C, idx = csc.kmeans_seed(F.cuda(), u, k)
    ref = okm.kmeanspp(Fn, k, philox.uniforms(k, 99, 2))
    assert idx.cpu().numpy().tolist() == ref.tolist()
    assert np.array_equal(C.double().cpu().numpy(), Fn[ref])


def test_lloyd_matches_oracle(csc):
    n, d, k = 20000, 32, 10
    F = _mixture(n, d, k, seed=8, spread=3.0)
    lab, C, obj = csc.kmeans(torch.from_numpy(F).cuda(), k, iters=20, seed=5, stream_id=2,
                             objective=True)
    u = philox.uniforms(k, 5, 2)
    C0 = F.astype(np.float64)[okm.kmeanspp(F, k, u)]
    rlab, rC, robj = okm.lloyd(F.astype(np.float64), C0, 20)
    # identical decisions unless a near-tie steered them apart; the objective then agrees
    agree = np.mean(lab.cpu().numpy() == rlab)
    say(f"  lloyd label agreement {agree:.6f}, obj {obj[-1]:.6f} vs {robj[-1]:.6f}")
    assert agree > 0.999
    assert obj[-1] == pytest.approx(robj[-1], rel=1e-5)
    assert np.all(np.diff(obj) <= 1e-6 * obj[0])
