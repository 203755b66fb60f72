"""The allocation-free k-means assignment (csc_kmeans_assign_noalloc) against the workspace
entry point csc_kmeans_assign, through the C ABI: two calls in a row on one device, the
second with a smaller input, must each give the same labels and distances bit for bit (the
same kernels; only where the split centroids live differs)."""

import ctypes as C

import numpy as np
import pytest
import torch

from helpers import say

pytestmark = pytest.mark.gpu


def _noalloc(lib):
    f = lib.csc_kmeans_assign_noalloc
    f.argtypes = [C.c_void_p, C.c_int, C.c_int64, C.c_int64, C.c_int, C.c_void_p, C.c_int,
                  C.c_void_p, C.c_void_p, C.c_void_p]
    f.restype = C.c_int
    return f


def _mixture(n, d, k, seed):
    rng = np.random.default_rng(seed)
    centers = rng.standard_normal((k, d)) * 3.0
    return (centers[rng.integers(0, k, n)] + rng.standard_normal((n, d))).astype(np.float32)


@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_noalloc_assign_equals_workspace_assign(csc, dtype):
    f = _noalloc(csc.lib)
    for n, d, k in [(30011, 256, 200), (4001, 48, 7)]:
        say(f"no-alloc assign n={n} d={d} k={k} {dtype}")
        F = torch.from_numpy(_mixture(n, d, k, seed=n)).cuda().to(dtype)
        Cc = F[torch.from_numpy(np.random.default_rng(1).choice(n, k, replace=False)).cuda()].float() + 0.01
        lab_ref, best_ref = csc.kmeans_assign(F, Cc)
        lab = torch.full((n,), -1, dtype=torch.int32, device="cuda")
        best = torch.full((n,), -1.0, dtype=torch.float32, device="cuda")
        st = f(F.data_ptr(), csc.binding._dt(F), F.stride(0), n, d, Cc.data_ptr(), k,
               lab.data_ptr(), best.data_ptr(), None)
        torch.cuda.synchronize()
        assert st == 0, csc.lib.csc_last_error().decode()
        assert torch.equal(lab, lab_ref)
        assert torch.equal(best, best_ref)


def test_noalloc_assign_rejects_what_its_scratch_cannot_hold(csc):
    f = _noalloc(csc.lib)
    n, d, k = 1000, 300, 8
    F = torch.zeros((n, d), dtype=torch.float32, device="cuda")
    Cc = torch.zeros((k, d), dtype=torch.float32, device="cuda")
    lab = torch.empty(n, dtype=torch.int32, device="cuda")
    st = f(F.data_ptr(), 0, d, n, d, Cc.data_ptr(), k, lab.data_ptr(), None, None)
    assert st == 1  # CSC_E_ARG
    assert "256" in csc.lib.csc_last_error().decode()
