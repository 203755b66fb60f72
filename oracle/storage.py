"""Storage-rounding emulation of the Chebyshev filter (Sec. 2.2, Step 1; eq. static_filtering).

TEST INFRASTRUCTURE ONLY (see the package header).  The paper fixes no precision.  A GPU
form stores some quantities in a narrower format than FP64: the operator's values, the
signals, the recurrence state Z_j, the copies of Z_j that the sparse product gathers, the
running sum Y (or the kept iterates Y is recombined from) and the output.  Rounding at those
points alone already moves the result away from the exact filter, by an amount that no
kernel can beat: the storage floor of the form.  This module computes it by running the
oracle's FP64 three-term recurrence with exactly those roundings and nothing else (every
arithmetic operation stays FP64).

Rounding is to nearest, ties to even, to a given number of significant bits: 53 (FP64,
no rounding), 24 (FP32), 11 (FP16), 8 (BF16).  For FP16 the exponent range is modelled as
IEEE binary16 has it: below 2^-14 values are rounded to the subnormal grid of spacing 2^-24,
and results of magnitude 2^16 or more (after rounding) overflow to infinity.  For FP32 and
BF16 it is not: their range (down to about 1e-38) holds every iterate of these signals.

Formats of one form (each a key of FORMAT_BITS, or an int number of bits):
  val     the stored values of A (normalized adjacency, L = I - A);
  state   the iterates Z_j as carried by the recurrence;
  gather  the copies of Z_j read by the sparse product (None: the state itself);
  combine "acc": Y summed step by step in a running sum stored in `acc`, with the
          coefficients rounded to `acc` too (the one-pass filter);
          "basis": every iterate kept in `basis` and Y = sum_j a_j Z_j formed in FP64 in the
          order j = 0..m afterwards (the kept-basis filter);
  out     the output.
The input block X is taken as given: a caller that stores the signals in BF16 passes the
rounded block, and compares with the exact filter of that same block.

With every format FP64 the result equals chebyshev.filter_recurrence bit for bit: the
sparse product is written as L~ G + diag(L~) (Z - G), whose second term is exactly zero
when the gathered copy is the state itself, and every other operation is the same FP64
operation in the same order.

Parity pins (tests/test_oracle_storage.py): the rounding against np.float32 casts, against
the integer-arithmetic BF16 rounding of oracle.philox and against hand-computed ties;
bit-identity with filter_recurrence when nothing is rounded (both combine modes); an error
that scales with the unit roundoff (2^-14 against 2^-18 of the state: a ratio of about 16);
output rounding alone bounded by half an ulp per entry.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .operator import scaled_laplacian

FORMAT_BITS = {"f64": 53, "f32": 24, "f16": 11, "bf16": 8}


def _bits(fmt) -> int:
    if fmt is None:
        return 53
    if isinstance(fmt, (int, np.integer)):
        if not 1 <= int(fmt) <= 53:
            raise ValueError("bits must be in [1, 53]")
        return int(fmt)
    return FORMAT_BITS[fmt]


def round_sig(x, fmt) -> np.ndarray:
    """x rounded to nearest (ties to even) with the significant bits of `fmt` (and, for
    "f16", binary16's subnormal grid and overflow)."""
    x = np.asarray(x, dtype=np.float64)
    bits = _bits(fmt)
    if bits >= 53:
        return x.copy()
    m, e = np.frexp(x)                      # x = m 2^e, 0.5 <= |m| < 1 (m = 0 for x = 0)
    r = np.ldexp(np.rint(np.ldexp(m, bits)), e - bits)  # np.rint rounds half to even
    if isinstance(fmt, str) and fmt == "f16":
        sub = np.abs(x) < 2.0 ** -14
        r = np.where(sub, np.ldexp(np.rint(np.ldexp(x, 24)), -24), r)
        r = np.where(np.abs(r) >= 2.0 ** 16, np.copysign(np.inf, x), r)
    return r


def round_values(A: sp.csr_matrix, fmt) -> sp.csr_matrix:
    """A with its stored values rounded (same pattern and entry order)."""
    return sp.csr_matrix((round_sig(A.data, fmt), A.indices.copy(), A.indptr.copy()), shape=A.shape)


def stored_operator(A: sp.csr_matrix, lmax: float, val="f64") -> sp.csr_matrix:
    """L~ built from A's values rounded to `val` (what filter_stored multiplies by)."""
    return scaled_laplacian(round_values(A, val), lmax)


def filter_stored(A: sp.csr_matrix, lmax: float, a: np.ndarray, X: np.ndarray, *, val="f64",
                  state="f64", gather=None, combine="acc", acc="f64", basis="f64",
                  out="f64", Lt=None) -> np.ndarray:
    """Y = sum_j a_j T_j(L~) X with the roundings of one storage form (module header).
    Lt: stored_operator(A, lmax, val), when the caller has it already (large graphs)."""
    if combine not in ("acc", "basis"):
        raise ValueError(combine)
    if Lt is None:
        Lt = stored_operator(A, lmax, val)
    dg = Lt.diagonal()[:, None]
    X = np.asarray(X, dtype=np.float64)
    gfmt = state if gather is None else gather
    m = len(a) - 1
    coef = round_sig(a, acc) if combine == "acc" else np.asarray(a, dtype=np.float64)

    def product(Z):
        G = round_sig(Z, gfmt)
        return Lt @ G + dg * (Z - G)

    def add(Y, j, Z):
        if combine == "acc":
            return round_sig(Y + coef[j] * Z, acc)
        return Y + coef[j] * round_sig(Z, basis)

    Z_prev = round_sig(X, state)
    Y = round_sig(coef[0] * Z_prev, acc) if combine == "acc" else coef[0] * round_sig(Z_prev, basis)
    if m >= 1:
        Z = round_sig(product(Z_prev), state)
        Y = add(Y, 1, Z)
        for j in range(1, m):
            Z_next = round_sig(2.0 * product(Z) - Z_prev, state)
            Y = add(Y, j + 1, Z_next)
            Z_prev, Z = Z, Z_next
    return round_sig(Y, out)


# The storage forms of the library's filter paths, by the formats of the module header.
# "onepass" forms accumulate Y in FP32 during the recurrence; "basis" forms keep every
# iterate and recombine them in FP64.
FORMS = {
    "fp32_onepass": dict(val="f32", state="f32", combine="acc", acc="f32", out="f32"),
    "fp32_basis": dict(val="f32", state="f32", combine="basis", basis="f32", out="f32"),
    "bf16io_onepass": dict(val="bf16", state="f32", combine="acc", acc="f32", out="bf16"),
    "bf16io_basis": dict(val="bf16", state="f32", combine="basis", basis="f32", out="bf16"),
    "bf16_onepass": dict(val="bf16", state="bf16", combine="acc", acc="f32", out="bf16"),
    "bf16_basis": dict(val="bf16", state="bf16", combine="basis", basis="bf16", out="bf16"),
    "bf16s_onepass": dict(val="bf16", state="f32", gather="bf16", combine="acc", acc="f32",
                          out="bf16"),
    "bf16s_basis": dict(val="bf16", state="f32", gather="bf16", combine="basis", basis="f32",
                        out="bf16"),
    "bf16s_basis_bf16copies": dict(val="bf16", state="f32", gather="bf16", combine="basis",
                                   basis="bf16", out="bf16"),
    "f16_onepass": dict(val="bf16", state="f16", combine="acc", acc="f32", out="bf16"),
    "f16_basis": dict(val="bf16", state="f16", combine="basis", basis="f16", out="bf16"),
    "f16s_onepass": dict(val="bf16", state="f32", gather="f16", combine="acc", acc="f32",
                         out="bf16"),
    "f16s_basis": dict(val="bf16", state="f32", gather="f16", combine="basis", basis="f32",
                       out="bf16"),
    "f16s_basis_f16copies": dict(val="bf16", state="f32", gather="f16", combine="basis",
                                 basis="f16", out="bf16"),
}


def form_inputs(form: str) -> str:
    """Storage of the signal block a form filters: "f32" or "bf16"."""
    return "f32" if form.startswith("fp32") else "bf16"
