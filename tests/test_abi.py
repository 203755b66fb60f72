"""The C ABI without a GPU: the library loads, exports every declared entry point, and its
host-only calls (coefficients, dichotomy, argument validation) behave as specified."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

from oracle import chebyshev, eigcount

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "csc.h")
LIB = os.path.join(ROOT, "paper_1706_03591_amd", "libcsc.so")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(csc_[a-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def pkg():
    if not os.path.exists(LIB):
        pytest.fail("libcsc.so is not built (python -m paper_1706_03591_amd.build)")
    import paper_1706_03591_amd as p
    return p


def test_exports_every_declared_symbol(pkg):
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (csc_[a-z0-9_]+)", out))
    missing = [s for s in _declared() if s not in exported]
    assert not missing, missing
    assert len(_declared()) >= 30


def test_binding_covers_every_symbol(pkg):
    for name in _declared():
        assert hasattr(pkg.lib, name)


def test_coefficients_match_oracle(pkg):
    for m, lc, damp in [(0, 0.3, "none"), (1, 1.2, "jackson"), (50, 0.43, "jackson"),
                        (120, 0.55, "none"), (150, 1.999, "jackson")]:
        a = pkg.cheb_coeffs(m, 2.0, lc, pkg.DAMP_JACKSON if damp == "jackson" else pkg.DAMP_NONE)
        ref = chebyshev.step_coefficients(m, 2.0, lc, damp)
        assert np.max(np.abs(a - ref)) <= 1e-14


def test_host_dichotomy_matches_oracle(pkg):
    from workloads import gaussian_block, sbm
    from helpers import oracle_A
    g = sbm(300, 3, 10.0, 0.1, seed=5)
    A = oracle_A(g)
    P = gaussian_block(g.n, 16, 0.25, seed=6).astype(np.float64)
    m = 30
    mu = eigcount.moments_direct(A, 2.0, m, P)
    for lo, hi, k in [(0.0, 2.0, 3), (0.2, 2.0, 3), (0.0, 0.3, 2)]:
        lam, cnt, trace = pkg.eigcount_from_moments(mu, m, 1 / 16.0, 16, k, 16, lo, hi)
        rl, rc, rt = eigcount.eigcount_bisect(mu, m, 2.0, "jackson", 1 / 16.0, 16, k, 16, lo, hi)
        assert lam == rl
        assert cnt == pytest.approx(rc, rel=1e-12)
        assert np.allclose(trace, np.array(rt), rtol=1e-12)


def test_host_argument_errors(pkg):
    CscError = pkg.CscError
    with pytest.raises(CscError, match="CSC_E_ARG"):
        pkg.cheb_coeffs(-1, 2.0, 0.5)
    with pytest.raises(CscError, match="CSC_E_ARG"):
        pkg.cheb_coeffs(10, 2.0, 2.5)
    with pytest.raises(CscError, match="CSC_E_ARG"):
        pkg.cheb_coeffs(10, -1.0, 0.5)
    with pytest.raises(CscError, match="CSC_E_ARG"):
        pkg.eigcount_from_moments(np.ones(5), 4, 1.0, 4, 2, 8, lo=1.5, hi=1.0)
    lib = pkg.lib
    out = ctypes.c_void_p()
    assert lib.csc_graph_create(0, 0, 0, None, None, None, 0, 0, 1, None, ctypes.byref(out)) == 1
    assert b"n must be" in lib.csc_last_error()
    assert lib.csc_graph_create(4, 0, 0, None, None, None, 0, 0, 1, None, ctypes.byref(out)) == 1
    assert b"null CSR" in lib.csc_last_error()
    # the Laplacian kind is checked before anything touches the (here fake) device pointer
    fake = ctypes.c_void_p(256)
    assert lib.csc_graph_create(4, 0, 0, fake, None, None, 0, 7, 1, None, ctypes.byref(out)) == 1
    assert b"Laplacian kind" in lib.csc_last_error()
    opts = pkg.binding.DynOpts(lmax=0, tau=0, n_cand=0, lloyd_iters=-1, init=0, iter_dt=0,
                               keep_iterates=0)
    # p = 1 leaves no fresh columns, p < 0 is meaningless, and p close to 1 rounds q d to 0
    assert lib.csc_dyn_create(100, 8, 2, 1.0, 10, 1, 0, 1, ctypes.byref(opts), ctypes.byref(out)) == 1
    assert lib.csc_dyn_create(100, 8, 2, -0.1, 10, 1, 0, 1, ctypes.byref(opts), ctypes.byref(out)) == 1
    assert lib.csc_dyn_create(100, 8, 2, 0.95, 10, 1, 0, 1, ctypes.byref(opts), ctypes.byref(out)) == 1
    # similarity options: probes beyond the fresh block, or a refresh budget without probes
    bad = pkg.binding.DynOpts(keep_iterates=0, lloyd_iters=-1, sim_probes=5)
    assert lib.csc_dyn_create(100, 8, 2, 0.5, 10, 1, 0, 1, ctypes.byref(bad), ctypes.byref(out)) == 1
    assert b"sim_probes" in lib.csc_last_error()
    bad = pkg.binding.DynOpts(keep_iterates=0, lloyd_iters=-1, refresh_budget=0.1)
    assert lib.csc_dyn_create(100, 8, 2, 0.5, 10, 1, 0, 1, ctypes.byref(bad), ctypes.byref(out)) == 1
    assert lib.csc_dyn_create(100, 8, 2, 0.5, 10, 1, 5, 1, ctypes.byref(opts), ctypes.byref(out)) == 3
    # k-means sizes beyond 256 columns or 240 centroids are refused before any device access
    assert lib.csc_kmeans_assign(fake, 0, 257, 10, 257, fake, 5, fake, None, None, None, fake,
                                 1 << 30, None) == 1
    assert b"d must be <= 256" in lib.csc_last_error()
    assert lib.csc_kmeans_assign(fake, 0, 256, 1000, 256, fake, 241, fake, None, None, None, fake,
                                 1 << 30, None) == 1
    assert b"k must be <= 240" in lib.csc_last_error()
    # null handles
    assert lib.csc_cheb_filter(None, 2.0, 3, None, None, 0, 1, None, 0, 1, 1, 0, None, None, 0, None) == 1
    assert lib.csc_graph_destroy(None) == 0


def test_workspace_queries_are_monotone(pkg):
    lib = pkg.lib
    a = lib.csc_cheb_filter_workspace_bytes(1000, 16, 0)
    b = lib.csc_cheb_filter_workspace_bytes(2000, 16, 0)
    c = lib.csc_cheb_filter_workspace_bytes(1000, 200, 0)  # sized for every tile shape
    assert 0 < a < b and a < c
    assert lib.csc_kmeans_workspace_bytes(1000, 32, 5) < lib.csc_kmeans_workspace_bytes(10000, 32, 5)
    assert lib.csc_cheb_backward_workspace_bytes(1000, 8, 20, 0) > 0


def test_version(pkg):
    assert pkg.version() >= 10000


def test_iterate_mode_codes(pkg):
    import torch

    from paper_1706_03591_amd import binding

    assert binding._it(torch.float32) == binding.F32
    assert binding._it(torch.bfloat16) == binding.BF16
    assert binding._it("bf16s") == binding.BF16S == 3
    with pytest.raises(ValueError):
        binding._it("fp8")


def test_bf16s_workspace_holds_fp32_state(pkg):
    lib = pkg.lib
    n, w = 1000, 64
    f32 = lib.csc_cheb_filter_workspace_bytes(n, w, 0)
    b16 = lib.csc_cheb_filter_workspace_bytes(n, w, 1)
    b16s = lib.csc_cheb_filter_workspace_bytes(n, w, 3)
    # two BF16 copies plus two FP32 state arrays on top of the BF16 layout
    assert b16s >= b16 + 2 * n * w * 4
    assert f32 > 0


def test_dyn_state_header_layout(pkg):
    """The exported state starts with a 64-byte csc_dyn_header; null handles are rejected."""
    H = pkg.binding.DynHeader
    assert ctypes.sizeof(H) == 64
    assert H.lam.offset == 56 and H.seed.offset == 48 and H.t.offset == 36
    lib = pkg.lib
    assert lib.csc_dyn_state_bytes(None) == 0
    buf = ctypes.create_string_buffer(64)
    assert lib.csc_dyn_export(None, buf, 64, None) == 1
    assert lib.csc_dyn_import(None, buf, 64, None) == 1
