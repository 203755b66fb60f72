"""Python binding of libcsc (argument marshalling only).

Every call goes to the HIP library through its C ABI (``include/csc.h``); PyTorch only
provides device memory and the current stream.  The library must be built
(``python -m paper_1706_03591_amd.build``); importing this module without it raises.
"""

from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcsc.so")

F32, BF16, F64, BF16S, F16, F16S = 0, 1, 2, 3, 4, 5
# iterate storage modes: a torch dtype (float32, bfloat16, float16), or "bf16s" / "f16s"
# (BF16 / binary16 copies for the gathers and the kept basis, FP32 recurrence state)
BF16S_ITER = "bf16s"
F16S_ITER = "f16s"
DAMP_NONE, DAMP_JACKSON = 0, 1
LAP_NORMALIZED, LAP_COMBINATORIAL = 0, 1

_TORCH_DT = {torch.float32: F32, torch.bfloat16: BF16, torch.float64: F64}
_DT_TORCH = {F32: torch.float32, BF16: torch.bfloat16, F64: torch.float64}


_ITER_MODES = {torch.float32: F32, torch.bfloat16: BF16, torch.float16: F16,
               BF16S_ITER: BF16S, F16S_ITER: F16S}


def _it(iter_dtype) -> int:
    """Iterate-mode code of a torch dtype or of "bf16s" / "f16s"."""
    key = iter_dtype.lower() if isinstance(iter_dtype, str) else iter_dtype
    try:
        return _ITER_MODES[key]
    except KeyError:
        raise ValueError(f"unknown iterate mode {iter_dtype!r}") from None

STATUS = {0: "CSC_OK", 1: "CSC_E_ARG", 2: "CSC_E_GRAPH", 3: "CSC_E_DTYPE", 4: "CSC_E_NOMEM",
          5: "CSC_E_HIP", 6: "CSC_E_STATE"}


class CscError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is not built; run `python -m paper_1706_03591_amd.build`")

lib = C.CDLL(LIB_PATH)

vp, i64, i32, u64, dbl, sz = C.c_void_p, C.c_int64, C.c_int, C.c_uint64, C.c_double, C.c_size_t
pdbl, pi64, pint = C.POINTER(C.c_double), C.POINTER(C.c_int64), C.POINTER(C.c_int)


class DynHeader(C.Structure):
    """csc_dyn_header: the fixed-size head of an exported dynamic state."""
    _fields_ = [("magic", C.c_uint64), ("n", C.c_int64), ("d", C.c_int32), ("k", C.c_int32),
                ("m", C.c_int32), ("qd", C.c_int32), ("feat_dt", C.c_int32), ("t", C.c_int32),
                ("cursor", C.c_int32), ("reserved", C.c_int32), ("seed", C.c_uint64),
                ("lam", C.c_double)]


class DynOpts(C.Structure):
    _fields_ = [("lmax", C.c_double), ("tau", C.c_double), ("n_cand", C.c_int),
                ("lloyd_iters", C.c_int), ("init", C.c_int), ("iter_dt", C.c_int),
                ("keep_iterates", C.c_int), ("batch", C.c_int), ("use_graph", C.c_int),
                ("variant", C.c_int), ("track_similarity", C.c_int), ("sim_probes", C.c_int),
                ("refresh_budget", C.c_double)]


_SIGS = {
    "csc_last_error": ([], C.c_char_p),
    "csc_version": ([], C.c_int),
    "csc_graph_create": ([i64, i64, i64, vp, vp, vp, i32, i32, i32, vp, C.POINTER(vp)], i32),
    "csc_graph_update": ([vp, i64, vp, vp, vp, i32, vp], i32),
    "csc_graph_destroy": ([vp], i32),
    "csc_graph_info": ([vp, pi64, pi64, pi64], i32),
    "csc_graph_arrays": ([vp, C.POINTER(vp), C.POINTER(vp), C.POINTER(vp), pint, C.POINTER(vp),
                          C.POINTER(vp)], i32),
    "csc_lmax": ([vp, i32, pdbl, vp], i32),
    "csc_graph_distance": ([vp, vp, pdbl, vp], i32),
    "csc_cheb_coeffs": ([i32, dbl, dbl, i32, pdbl], i32),
    "csc_cheb_filter_workspace_bytes": ([i64, i32, i32], sz),
    "csc_cheb_filter": ([vp, dbl, i32, pdbl, vp, i32, i64, vp, i32, i64, i32, i32, vp, vp, sz,
                         vp], i32),
    "csc_cheb_moments": ([vp, dbl, i32, vp, i32, i64, i32, i32, vp, vp, sz, vp], i32),
    "csc_eigcount": ([vp, dbl, i32, i32, vp, i32, i64, i32, dbl, dbl, i32, dbl, dbl, i32, pdbl,
                      pdbl, pdbl, pdbl, vp, sz, vp], i32),
    "csc_eigcount_from_moments": ([pdbl, i32, dbl, i32, dbl, i32, dbl, i32, dbl, dbl, pdbl, pdbl,
                                   pdbl], i32),
    "csc_dot_workspace_bytes": ([i64], sz),
    "csc_dot": ([vp, i32, i64, vp, i32, i64, i64, i32, vp, vp, sz, vp], i32),
    "csc_randn": ([vp, i32, i64, i32, i64, i64, u64, u64, dbl, vp], i32),
    "csc_uniforms": ([vp, i32, u64, u64, vp], i32),
    "csc_kmeans_workspace_bytes": ([i64, i32, i32], sz),
    "csc_kmeans_assign": ([vp, i32, i64, i64, i32, vp, i32, vp, vp, vp, vp, vp, sz, vp], i32),
    "csc_kmeans_assign_noalloc": ([vp, i32, i64, i64, i32, vp, i32, vp, vp, vp], i32),
    "csc_kmeans_update": ([vp, i32, i64, i64, i32, vp, i32, vp, vp, vp, sz, vp], i32),
    "csc_kmeans_seed": ([vp, i32, i64, i64, i32, i32, vp, vp, vp, vp, sz, vp], i32),
    "csc_compressive_workspace_bytes": ([i64, i32, i32, i32], sz),
    "csc_compressive_kmeans": ([vp, vp, i32, i64, i32, i32, i32, i32, dbl, i32, i32, dbl, u64, u64,
                                u64, vp, vp, vp, vp, pint, vp, sz, vp], i32),
    "csc_kmeans": ([vp, i32, i64, i64, i32, i32, i32, i32, u64, u64, vp, vp, pdbl, vp, sz, vp],
                   i32),
    "csc_dyn_create": ([i64, i32, i32, dbl, i32, i32, i32, u64, C.POINTER(DynOpts), C.POINTER(vp)],
                       i32),
    "csc_dynamic_step": ([vp, vp, vp, pdbl, pint, pdbl, vp], i32),
    "csc_dynamic_steps": ([vp, C.POINTER(vp), i32, C.POINTER(vp), pdbl, pint, pdbl, vp], i32),
    "csc_dyn_features": ([vp, C.POINTER(vp), pint, pi64, C.POINTER(vp)], i32),
    "csc_dyn_similarity": ([vp, i32, pdbl, pdbl, pint], i32),
    "csc_dyn_state_bytes": ([vp], sz),
    "csc_dyn_export": ([vp, vp, sz, vp], i32),
    "csc_dyn_import": ([vp, vp, sz, vp], i32),
    "csc_dyn_destroy": ([vp], i32),
    "csc_cheb_backward_workspace_bytes": ([i64, i32, i32, i32], sz),
    "csc_cheb_filter_backward": ([vp, dbl, i32, pdbl, vp, i64, vp, i64, i32, vp, i64, vp, vp, i32,
                                  vp, sz, vp], i32),
    "csc_weight_grad_workspace_bytes": ([i64], sz),
    "csc_weight_grad": ([vp, vp, vp, vp, sz, vp], i32),
    "csc_gather_probe": ([vp, vp, i64, vp, i32, vp, vp], i32),
    "csc_timing_enable": ([i32], i32),
    "csc_timing_reset": ([], i32),
    "csc_timing_read": ([pdbl, pi64, pdbl], i32),
    "csc_autotune": ([vp, i32, i32, vp, sz, vp, pint], i32),
    "csc_set_variant": ([vp, i32, i32], i32),
}

for _name, (_args, _res) in _SIGS.items():
    _f = getattr(lib, _name)
    _f.argtypes = _args
    _f.restype = _res


def _check(st: int):
    if st != 0:
        raise CscError(st, lib.csc_last_error().decode())


def _stream(stream=None):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dt(t: torch.Tensor) -> int:
    try:
        return _TORCH_DT[t.dtype]
    except KeyError:
        raise CscError(3, f"unsupported dtype {t.dtype}") from None


def _ld(t: torch.Tensor) -> int:
    if t.dim() != 2 or t.stride(1) != 1:
        raise CscError(1, "blocks must be 2-D with unit column stride")
    return t.stride(0)


def _dbl_array(a) -> C.Array:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.float64))
    return (C.c_double * len(a))(*a.tolist())


_WS: dict = {}


def workspace(nbytes: int, device=None) -> torch.Tensor:
    """A cached device scratch buffer of at least ``nbytes`` bytes."""
    device = torch.device(device or "cuda")
    key = (device.index if device.index is not None else torch.cuda.current_device())
    buf = _WS.get(key)
    if buf is None or buf.numel() < nbytes:
        buf = torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)
        _WS[key] = buf
    return buf


def release_workspace():
    """Drop the cached scratch buffers and return cached device memory to the driver (the
    dynamic state sizes its kept basis from the free memory it sees)."""
    _WS.clear()
    torch.cuda.empty_cache()


def version() -> int:
    return lib.csc_version()


# ----------------------------------------------------------------------------------
# graph


class Graph:
    """Device operator of a CSR weight matrix W: the normalized adjacency
    A = D^{-1/2} W D^{-1/2} (L = I - A), or with laplacian=LAP_COMBINATORIAL, W and D
    (L = D - W)."""

    def __init__(self, n: int, rowptr, colidx, w, val_dtype=torch.float32, validate: bool = True,
                 nnz_capacity: int | None = None, stream=None, laplacian: int = 0):
        self.n = int(n)
        self.val_dtype = val_dtype
        self.laplacian = int(laplacian)
        rp, ci, ww = self._to_device(rowptr, colidx, w)
        nnz = int(ci.numel())
        cap = int(nnz_capacity if nnz_capacity is not None else nnz)
        h = C.c_void_p()
        _check(lib.csc_graph_create(self.n, nnz, cap, _ptr(rp), _ptr(ci), _ptr(ww),
                                    _TORCH_DT[val_dtype], self.laplacian, int(validate),
                                    _stream(stream), C.byref(h)))
        self.h = h
        self.nnz = nnz
        self._src = (rp, ci, ww)

    @staticmethod
    def _to_device(rowptr, colidx, w):
        dev = torch.device("cuda")
        rp = torch.as_tensor(np.asarray(rowptr, dtype=np.int64) if not torch.is_tensor(rowptr) else rowptr,
                             dtype=torch.int64).to(dev).contiguous()
        ci = torch.as_tensor(np.asarray(colidx, dtype=np.int32) if not torch.is_tensor(colidx) else colidx,
                             dtype=torch.int32).to(dev).contiguous()
        ww = torch.as_tensor(np.asarray(w, dtype=np.float64) if not torch.is_tensor(w) else w,
                             dtype=torch.float64).to(dev).contiguous()
        return rp, ci, ww

    @classmethod
    def from_workload(cls, g, **kw):
        return cls(g.n, g.rowptr, g.colidx, g.w, **kw)

    def update(self, rowptr, colidx, w, validate: bool = True, stream=None):
        rp, ci, ww = self._to_device(rowptr, colidx, w)
        _check(lib.csc_graph_update(self.h, int(ci.numel()), _ptr(rp), _ptr(ci), _ptr(ww),
                                    int(validate), _stream(stream)))
        self.nnz = int(ci.numel())
        self._src = (rp, ci, ww)

    def update_device(self, rp: torch.Tensor, ci: torch.Tensor, ww: torch.Tensor,
                      validate: bool = False, stream=None):
        """Rebuild from device-resident CSR tensors (int64, int32, float64)."""
        _check(lib.csc_graph_update(self.h, int(ci.numel()), _ptr(rp), _ptr(ci), _ptr(ww),
                                    int(validate), _stream(stream)))
        self.nnz = int(ci.numel())
        self._src = (rp, ci, ww)

    def info(self):
        n, nnz, iso = C.c_int64(), C.c_int64(), C.c_int64()
        _check(lib.csc_graph_info(self.h, C.byref(n), C.byref(nnz), C.byref(iso)))
        return n.value, nnz.value, iso.value

    def arrays(self):
        """Copies of the device operator: (rowptr int32, colidx int32, values, dinv, mirror)."""
        rp, ci, vals, dinv, mir = C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_void_p(), C.c_void_p()
        vdt = C.c_int()
        _check(lib.csc_graph_arrays(self.h, C.byref(rp), C.byref(ci), C.byref(vals), C.byref(vdt),
                                    C.byref(dinv), C.byref(mir)))
        torch.cuda.synchronize()
        out = {}
        for name, ptr, count, dt in [("rowptr", rp, self.n + 1, torch.int32),
                                     ("colidx", ci, self.nnz, torch.int32),
                                     ("vals", vals, self.nnz, _DT_TORCH[vdt.value]),
                                     ("dinv", dinv, self.n, torch.float64),
                                     ("mirror", mir, self.nnz, torch.int32)]:
            t = torch.empty(count, dtype=dt, device="cuda")
            nbytes = count * t.element_size()
            if nbytes:
                _copy_d2d(t.data_ptr(), ptr.value, nbytes)
            out[name] = t
        return out

    def set_values(self, vals: torch.Tensor):
        """Overwrite A's stored values (float32 graphs; one value per CSR entry)."""
        if self.val_dtype != torch.float32 or vals.dtype != torch.float32 or vals.numel() != self.nnz:
            raise CscError(1, "set_values needs float32 values, one per entry")
        ptr = C.c_void_p()
        _check(lib.csc_graph_arrays(self.h, None, None, C.byref(ptr), None, None, None))
        torch.cuda.current_stream().synchronize()
        _copy_d2d(ptr.value, vals.contiguous().data_ptr(), self.nnz * 4)

    def lmax(self, iters: int = 0, stream=None) -> float:
        v = C.c_double()
        _check(lib.csc_lmax(self.h, int(iters), C.byref(v), _stream(stream)))
        return v.value

    def distance(self, other: "Graph", stream=None) -> float:
        """Edge similarity ||L(other) - L(self)||_F."""
        v = C.c_double()
        _check(lib.csc_graph_distance(self.h, other.h, C.byref(v), _stream(stream)))
        return v.value

    def autotune(self, w: int, iter_dtype=torch.float32, stream=None) -> int:
        need = lib.csc_cheb_filter_workspace_bytes(self.n, w, _it(iter_dtype))
        need += 2 * ((self.n * w * 4 + 255) // 256 * 256) + 4096
        ws = workspace(need)
        v = C.c_int()
        _check(lib.csc_autotune(self.h, int(w), _it(iter_dtype), _ptr(ws), ws.numel(),
                                _stream(stream), C.byref(v)))
        return v.value

    def set_variant(self, variant: int, iter_dtype=torch.float32):
        _check(lib.csc_set_variant(self.h, _it(iter_dtype), int(variant)))

    def close(self):
        if getattr(self, "h", None):
            lib.csc_graph_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _copy_d2d(dst: int, src: int, nbytes: int):
    hip = _hip()
    st = hip.hipMemcpy(C.c_void_p(dst), C.c_void_p(src), C.c_size_t(nbytes), 3)
    if st != 0:
        raise CscError(5, f"hipMemcpy failed ({st})")


_HIP = None


def _hip():
    global _HIP
    if _HIP is None:
        _HIP = C.CDLL("libamdhip64.so")
        _HIP.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        _HIP.hipMemcpy.restype = C.c_int
    return _HIP


# ----------------------------------------------------------------------------------
# coefficients, filter, eigencount


def cheb_coeffs(m: int, lmax: float, lambda_c: float, damping: int = DAMP_JACKSON) -> np.ndarray:
    a = (C.c_double * (m + 1))()
    _check(lib.csc_cheb_coeffs(int(m), float(lmax), float(lambda_c), int(damping), a))
    return np.frombuffer(a, dtype=np.float64).copy()


def cheb_filter(g: Graph, a, X: torch.Tensor, out: torch.Tensor | None = None,
                out_dtype=torch.float32, iter_dtype=torch.float32, lmax: float | None = None,
                moments: bool = False, stream=None):
    """Y = sum_j a_j T_j(L~) X (row-major blocks).  Returns Y, or (Y, moments) if asked.
    lmax None: the graph's own spectrum bound."""
    n, w = X.shape
    lmax = g.lmax() if lmax is None else lmax
    if out is None:
        out = torch.empty((n, w), dtype=out_dtype, device=X.device)
    a = np.asarray(a, dtype=np.float64)
    m = len(a) - 1
    mom = torch.empty(m + 1, dtype=torch.float64, device=X.device) if moments else None
    need = lib.csc_cheb_filter_workspace_bytes(n, w, _it(iter_dtype))
    ws = workspace(need, X.device)
    _check(lib.csc_cheb_filter(g.h, float(lmax), m, _dbl_array(a), _ptr(X), _dt(X), _ld(X),
                               _ptr(out), _dt(out), _ld(out), int(w), _it(iter_dtype),
                               _ptr(mom), _ptr(ws), ws.numel(), _stream(stream)))
    return (out, mom) if moments else out


def cheb_moments(g: Graph, m: int, P: torch.Tensor, iter_dtype=torch.float32,
                 lmax: float | None = None, stream=None) -> torch.Tensor:
    n, w = P.shape
    lmax = g.lmax() if lmax is None else lmax
    mom = torch.empty(m + 1, dtype=torch.float64, device=P.device)
    need = lib.csc_cheb_filter_workspace_bytes(n, w, _it(iter_dtype))
    ws = workspace(need, P.device)
    _check(lib.csc_cheb_moments(g.h, float(lmax), int(m), _ptr(P), _dt(P), _ld(P), int(w),
                                _it(iter_dtype), _ptr(mom), _ptr(ws), ws.numel(),
                                _stream(stream)))
    return mom


def eigcount(g: Graph, m: int, P: torch.Tensor, sigma2: float, k: float, n_cand: int = 16,
             lo: float = 0.0, hi: float | None = None, damping: int = DAMP_JACKSON,
             lmax: float | None = None, iter_dtype=torch.float32, stream=None):
    """Returns (lambda_c, count, trace (n_cand x 2), moments)."""
    n, w = P.shape
    lmax = g.lmax() if lmax is None else lmax
    hi = lmax if hi is None else hi
    need = lib.csc_cheb_filter_workspace_bytes(n, w, _it(iter_dtype)) + (m + 1) * 8 + 512
    ws = workspace(need, P.device)
    lam, cnt = C.c_double(), C.c_double()
    trace = (C.c_double * (2 * max(n_cand, 1)))()
    mom = (C.c_double * (m + 1))()
    _check(lib.csc_eigcount(g.h, float(lmax), int(m), int(damping), _ptr(P), _dt(P), _ld(P), int(w),
                            float(sigma2), float(k), int(n_cand), float(lo), float(hi),
                            _it(iter_dtype), C.byref(lam), C.byref(cnt), trace, mom,
                            _ptr(ws), ws.numel(), _stream(stream)))
    tr = np.frombuffer(trace, dtype=np.float64).reshape(-1, 2)[:n_cand].copy()
    return lam.value, cnt.value, tr, np.frombuffer(mom, dtype=np.float64).copy()


def eigcount_from_moments(mu, m: int, sigma2: float, n_probe: int, k: float, n_cand: int = 16,
                          lo: float = 0.0, hi: float = 2.0, damping: int = DAMP_JACKSON,
                          lmax: float = 2.0):
    lam, cnt = C.c_double(), C.c_double()
    trace = (C.c_double * (2 * max(n_cand, 1)))()
    _check(lib.csc_eigcount_from_moments(_dbl_array(mu), int(m), float(lmax), int(damping),
                                         float(sigma2), int(n_probe), float(k), int(n_cand),
                                         float(lo), float(hi), C.byref(lam), C.byref(cnt), trace))
    return lam.value, cnt.value, np.frombuffer(trace, dtype=np.float64).reshape(-1, 2)[:n_cand].copy()


def dot(X: torch.Tensor, Y: torch.Tensor, stream=None) -> float:
    n, w = X.shape
    res = torch.empty(1, dtype=torch.float64, device=X.device)
    ws = workspace(lib.csc_dot_workspace_bytes(n), X.device)
    _check(lib.csc_dot(_ptr(X), _dt(X), _ld(X), _ptr(Y), _dt(Y), _ld(Y), n, w, _ptr(res),
                       _ptr(ws), ws.numel(), _stream(stream)))
    return float(res.item())


def randn(n: int, w: int, seed: int, stream_id: int, sigma: float = 1.0, dtype=torch.float32,
          out: torch.Tensor | None = None, row0: int = 0, stream=None) -> torch.Tensor:
    if out is None:
        out = torch.empty((n, w), dtype=dtype, device="cuda")
    _check(lib.csc_randn(_ptr(out), _dt(out), int(n), int(w), _ld(out), int(row0), int(seed),
                         int(stream_id), float(sigma), _stream(stream)))
    return out


def uniforms(count: int, seed: int, stream_id: int, stream=None) -> torch.Tensor:
    u = torch.empty(count, dtype=torch.float64, device="cuda")
    _check(lib.csc_uniforms(_ptr(u), int(count), int(seed), int(stream_id), _stream(stream)))
    return u


# ----------------------------------------------------------------------------------
# k-means


def kmeans_assign(F: torch.Tensor, Cc: torch.Tensor, sums: bool = False, best_d2: bool = True,
                  stream=None):
    """(labels, best squared distances or None) and, with sums=True, also the Lloyd partial
    sums (k x d float32) and counts (k int32) of the new assignment."""
    n, d = F.shape
    k = Cc.shape[0]
    labels = torch.empty(n, dtype=torch.int32, device=F.device)
    best = torch.empty(n, dtype=torch.float32, device=F.device) if best_d2 else None
    S = torch.empty((k, d), dtype=torch.float32, device=F.device) if sums else None
    cnt = torch.empty(k, dtype=torch.int32, device=F.device) if sums else None
    ws = workspace(lib.csc_kmeans_workspace_bytes(n, d, k), F.device)
    _check(lib.csc_kmeans_assign(_ptr(F), _dt(F), _ld(F), n, d, _ptr(Cc.contiguous()), k,
                                 _ptr(labels), _ptr(best), _ptr(S), _ptr(cnt), _ptr(ws),
                                 ws.numel(), _stream(stream)))
    if sums:
        return labels, best, S, cnt
    return labels, best


def kmeans_update(F: torch.Tensor, labels: torch.Tensor, Cc: torch.Tensor, stream=None):
    """Updates Cc (float32, k x d) in place; returns the cluster sizes."""
    n, d = F.shape
    k = Cc.shape[0]
    counts = torch.empty(k, dtype=torch.int32, device=F.device)
    ws = workspace(lib.csc_kmeans_workspace_bytes(n, d, k), F.device)
    _check(lib.csc_kmeans_update(_ptr(F), _dt(F), _ld(F), n, d, _ptr(labels), k, _ptr(Cc),
                                 _ptr(counts), _ptr(ws), ws.numel(), _stream(stream)))
    return counts


def kmeans_seed(F: torch.Tensor, u: torch.Tensor, k: int, stream=None):
    n, d = F.shape
    Cc = torch.empty((k, d), dtype=torch.float32, device=F.device)
    idx = torch.empty(k, dtype=torch.int32, device=F.device)
    ws = workspace(lib.csc_kmeans_workspace_bytes(n, d, k), F.device)
    _check(lib.csc_kmeans_seed(_ptr(F), _dt(F), _ld(F), n, d, k, _ptr(u), _ptr(Cc), _ptr(idx),
                               _ptr(ws), ws.numel(), _stream(stream)))
    return Cc, idx


def kmeans(F: torch.Tensor, k: int, iters: int = 20, seed: int = 0, stream_id: int = 0,
           C0: torch.Tensor | None = None, objective: bool = False, stream=None):
    n, d = F.shape
    Cc = torch.empty((k, d), dtype=torch.float32, device=F.device) if C0 is None else C0.clone()
    labels = torch.empty(n, dtype=torch.int32, device=F.device)
    obj = (C.c_double * (iters + 1))() if objective else None
    ws = workspace(lib.csc_kmeans_workspace_bytes(n, d, k), F.device)
    _check(lib.csc_kmeans(_ptr(F), _dt(F), _ld(F), n, d, int(k), int(iters),
                          0 if C0 is None else 1, int(seed), int(stream_id), _ptr(Cc),
                          _ptr(labels), obj, _ptr(ws), ws.numel(), _stream(stream)))
    if objective:
        return labels, Cc, np.frombuffer(obj, dtype=np.float64).copy()
    return labels, Cc


def compressive_kmeans(g: "Graph", F: torch.Tensor, k: int, n_sample: int, r: int = 4,
                       gamma: float = 1e-3, lloyd_iters: int = 20, cg_iters: int = 500,
                       cg_tol: float = 1e-6, seed: int = 0, sample_stream: int = 3,
                       kmeans_stream: int = 2, details: bool = False, stream=None):
    """Labels of all nodes from k-means on n_sample drawn nodes and Tikhonov interpolation.
    With details: (labels, samples, sample labels, X (n x k), CG iterations)."""
    n, d = F.shape
    labels = torch.empty(n, dtype=torch.int32, device=F.device)
    samp = torch.empty(n_sample, dtype=torch.int32, device=F.device) if details else None
    slab = torch.empty(n_sample, dtype=torch.int32, device=F.device) if details else None
    X = torch.empty((n, k), dtype=torch.float32, device=F.device) if details else None
    its = C.c_int()
    ws = workspace(lib.csc_compressive_workspace_bytes(n, d, k, n_sample), F.device)
    _check(lib.csc_compressive_kmeans(g.h, _ptr(F), _dt(F), _ld(F), d, int(k), int(n_sample), int(r),
                                      float(gamma), int(lloyd_iters), int(cg_iters), float(cg_tol),
                                      int(seed), int(sample_stream), int(kmeans_stream),
                                      _ptr(labels), _ptr(samp), _ptr(slab), _ptr(X), C.byref(its),
                                      _ptr(ws), ws.numel(), _stream(stream)))
    if details:
        return labels, samp, slab, X, its.value
    return labels


# ----------------------------------------------------------------------------------
# dynamic CSC


class DynamicCSC:
    def __init__(self, n: int, d: int, k: int, p: float, m: int, seed: int,
                 damping: int = DAMP_JACKSON, feat_dtype=torch.float32, iter_dtype=torch.float32,
                 lmax: float = 0.0, tau: float = 0.0, n_cand: int = 16, lloyd_iters: int = 20,
                 init: int = 0, keep_iterates: int = -1, batch: int = 1, use_graph: bool = False,
                 variant: int = -1, track_similarity: bool = False, sim_probes: int = 0,
                 refresh_budget: float = 0.0):
        opts = DynOpts(lmax=lmax, tau=tau, n_cand=n_cand, lloyd_iters=lloyd_iters, init=init,
                       iter_dt=_it(iter_dtype), keep_iterates=keep_iterates, batch=batch,
                       use_graph=int(bool(use_graph)), variant=int(variant),
                       track_similarity=int(bool(track_similarity)), sim_probes=int(sim_probes),
                       refresh_budget=float(refresh_budget))
        h = C.c_void_p()
        if keep_iterates < 0:
            release_workspace()
        _check(lib.csc_dyn_create(int(n), int(d), int(k), float(p), int(m), int(damping),
                                  _TORCH_DT[feat_dtype], int(seed), C.byref(opts), C.byref(h)))
        self.h = h
        self.n, self.d, self.k = n, d, k
        self.feat_dtype = feat_dtype

    def step(self, g: Graph, labels: torch.Tensor | None = None, stream=None):
        if labels is None:
            labels = torch.empty(self.n, dtype=torch.int32, device="cuda")
        lam, cnt = C.c_double(), C.c_double()
        ref = C.c_int()
        _check(lib.csc_dynamic_step(self.h, g.h, _ptr(labels), C.byref(lam), C.byref(ref),
                                    C.byref(cnt), _stream(stream)))
        return labels, lam.value, bool(ref.value), cnt.value

    def steps(self, graphs, labels=None, stream=None):
        """Several snapshots in order (batched recurrences when the state was created with
        batch > 1).  Returns (labels list, lambdas, refined, counts)."""
        S = len(graphs)
        if labels is None:
            labels = [torch.empty(self.n, dtype=torch.int32, device="cuda") for _ in range(S)]
        gh = (C.c_void_p * S)(*[g.h.value for g in graphs])
        lp = (C.c_void_p * S)(*[lab.data_ptr() for lab in labels])
        lam = (C.c_double * S)()
        ref = (C.c_int * S)()
        cnt = (C.c_double * S)()
        _check(lib.csc_dynamic_steps(self.h, gh, S, lp, lam, ref, cnt, _stream(stream)))
        return labels, list(lam), [bool(x) for x in ref], list(cnt)

    def export_state(self, stream=None) -> bytearray:
        """Checkpoint: header, Theta, centroids and labels in one host buffer."""
        nb = lib.csc_dyn_state_bytes(self.h)
        buf = bytearray(nb)
        cbuf = (C.c_char * nb).from_buffer(buf)
        _check(lib.csc_dyn_export(self.h, C.cast(cbuf, vp), nb, _stream(stream)))
        return buf

    def import_state(self, buf, stream=None):
        """Resume from a buffer written by export_state (same parameters and seed)."""
        buf = bytearray(buf)
        cbuf = (C.c_char * len(buf)).from_buffer(buf)
        _check(lib.csc_dyn_import(self.h, C.cast(cbuf, vp), len(buf), _stream(stream)))

    @staticmethod
    def header(buf) -> DynHeader:
        """A writable view of the header at the start of an exported state."""
        return DynHeader.from_buffer(buf)

    def similarity(self, t: int):
        """(rho_edge, rho_hat, refreshed) of snapshot t (1-based); -1 where not computed."""
        re_, rh, rf = C.c_double(), C.c_double(), C.c_int()
        _check(lib.csc_dyn_similarity(self.h, int(t), C.byref(re_), C.byref(rh), C.byref(rf)))
        return re_.value, rh.value, bool(rf.value)

    def features(self) -> torch.Tensor:
        th, dt, ld, cp = C.c_void_p(), C.c_int(), C.c_int64(), C.c_void_p()
        _check(lib.csc_dyn_features(self.h, C.byref(th), C.byref(dt), C.byref(ld), C.byref(cp)))
        torch.cuda.synchronize()
        out = torch.empty((self.n, self.d), dtype=_DT_TORCH[dt.value], device="cuda")
        _copy_d2d(out.data_ptr(), th.value, out.numel() * out.element_size())
        return out

    def centroids(self) -> torch.Tensor:
        th, dt, ld, cp = C.c_void_p(), C.c_int(), C.c_int64(), C.c_void_p()
        _check(lib.csc_dyn_features(self.h, C.byref(th), C.byref(dt), C.byref(ld), C.byref(cp)))
        torch.cuda.synchronize()
        out = torch.empty((self.k, self.d), dtype=torch.float32, device="cuda")
        _copy_d2d(out.data_ptr(), cp.value, out.numel() * 4)
        return out

    def close(self):
        if getattr(self, "h", None):
            lib.csc_dyn_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# ----------------------------------------------------------------------------------
# adjoint


def filter_backward(g: Graph, a, X: torch.Tensor, G: torch.Tensor, lmax: float | None = None,
                    ckpt_every: int = 0, want_dx: bool = True, want_da: bool = True,
                    want_dA: bool = True, stream=None):
    """(dX, da, dA) of l = <G, sum_j a_j T_j(L~) X>; FP32 in, FP32/FP64 out."""
    n, w = X.shape
    lmax = g.lmax() if lmax is None else lmax
    a = np.asarray(a, dtype=np.float64)
    m = len(a) - 1
    dX = torch.empty((n, w), dtype=torch.float32, device=X.device) if want_dx else None
    da = torch.empty(m + 1, dtype=torch.float64, device=X.device) if want_da else None
    dA = torch.empty(g.nnz, dtype=torch.float32, device=X.device) if want_dA else None
    need = lib.csc_cheb_backward_workspace_bytes(n, w, m, int(ckpt_every))
    ws = workspace(need, X.device)
    _check(lib.csc_cheb_filter_backward(g.h, float(lmax), m, _dbl_array(a), _ptr(X), _ld(X),
                                        _ptr(G), _ld(G), int(w), _ptr(dX), _ld(dX) if dX is not None else w,
                                        _ptr(da), _ptr(dA), int(ckpt_every), _ptr(ws), ws.numel(),
                                        _stream(stream)))
    return dX, da, dA


# ----------------------------------------------------------------------------------
# measurement


def timing_enable(on: bool = True):
    _check(lib.csc_timing_enable(int(on)))


def timing_reset():
    _check(lib.csc_timing_reset())


def timing_read():
    ms, n, b = C.c_double(), C.c_int64(), C.c_double()
    _check(lib.csc_timing_read(C.byref(ms), C.byref(n), C.byref(b)))
    return ms.value, n.value, b.value


def weight_gradient(g: "Graph", dA: torch.Tensor, stream=None) -> torch.Tensor:
    """dl/dw per stored entry (float64, the symmetric edge weight's derivative, equal on both
    copies of an edge) from dl/dA_e (float32, one per stored entry)."""
    dW = torch.empty(dA.numel(), dtype=torch.float64, device=dA.device)
    ws = workspace(lib.csc_weight_grad_workspace_bytes(g.n), dA.device)
    _check(lib.csc_weight_grad(g.h, _ptr(dA.contiguous()), _ptr(dW), _ptr(ws), ws.numel(),
                               _stream(stream)))
    return dW


def gather_probe(rowptr: torch.Tensor, colidx: torch.Tensor, table: torch.Tensor, row_bytes: int,
                 out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """The random-gather probe over a CSR pattern (int32 device tensors) and a table of rows
    of row_bytes bytes; returns the per-lane XORs (uint32 as int32)."""
    n = rowptr.numel() - 1
    if out is None:
        out = torch.empty(n * (row_bytes // 16), dtype=torch.int32, device=rowptr.device)
    _check(lib.csc_gather_probe(_ptr(rowptr), _ptr(colidx), n, _ptr(table), int(row_bytes),
                                _ptr(out), _stream(stream)))
    return out
