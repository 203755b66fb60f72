"""Pins of the storage-rounding emulator (oracle.storage) against what the arithmetic fixes."""

import numpy as np
import pytest

from oracle import chebyshev, operator, philox, storage
from workloads import sbm


@pytest.fixture(scope="module")
def small():
    g = sbm(2000, 4, 12.0, 0.1, seed=61)
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    X = np.random.default_rng(62).standard_normal((g.n, 6)) / 8.0
    return A, X


def test_round_sig_identity_and_float32():
    x = np.random.default_rng(1).standard_normal(10_000) * 10.0 ** np.random.default_rng(2).integers(-20, 20, 10_000)
    assert np.array_equal(storage.round_sig(x, "f64"), x)
    # 24 significant bits is IEEE binary32 (round to nearest even) in the normal range
    assert np.array_equal(storage.round_sig(x, "f32"), x.astype(np.float32).astype(np.float64))


def test_round_sig_bf16_matches_integer_rounding():
    # on values exactly representable in FP32 (no double rounding), 8 significant bits equal
    # the bit-pattern rounding of the upper half of binary32 words
    f = (np.random.default_rng(3).standard_normal(20_000) * 3.0).astype(np.float32)
    assert np.array_equal(storage.round_sig(f.astype(np.float64), "bf16"),
                          philox.round_bf16(f).astype(np.float64))


def test_round_sig_f16_matches_numpy_half():
    # IEEE binary16: 11 significant bits in the normal range, the 2^-24 grid below 2^-14,
    # overflow to infinity from 65520 on (65504 is the largest finite value)
    rng = np.random.default_rng(4)
    x = np.concatenate([rng.standard_normal(20_000) * 3.0,
                        rng.standard_normal(20_000) * 2.0 ** -16,
                        rng.standard_normal(2_000) * 3e4,
                        [65504.0, 65519.0, 65520.0, -65536.0, 2.0 ** -25, 3 * 2.0 ** -26, 0.0]])
    with np.errstate(over="ignore"):
        want = x.astype(np.float16).astype(np.float64)
    assert np.array_equal(storage.round_sig(x, "f16"), want)


def test_round_sig_hand_ties():
    # 8 significant bits: the ulp of [1, 2) is 2^-7
    x = np.array([1 + 2.0 ** -8, 1 + 3 * 2.0 ** -8, 1 + 2.0 ** -8 + 2.0 ** -30, -(1 + 2.0 ** -8), 0.0])
    want = np.array([1.0, 1 + 2.0 ** -6, 1 + 2.0 ** -7, -1.0, 0.0])
    assert np.array_equal(storage.round_sig(x, "bf16"), want)


@pytest.mark.parametrize("combine", ["acc", "basis"])
def test_no_rounding_is_the_recurrence_bit_for_bit(small, combine):
    A, X = small
    a = chebyshev.step_coefficients(40, 2.0, 0.4, "jackson")
    ref = chebyshev.filter_recurrence(A, 2.0, a, X)
    got = storage.filter_stored(A, 2.0, a, X, combine=combine)
    assert np.array_equal(got, ref)
    # also with a spectrum bound that leaves a diagonal in L~
    ref = chebyshev.filter_recurrence(A, 1.9, a, X)
    assert np.array_equal(storage.filter_stored(A, 1.9, a, X, combine=combine), ref)


def test_error_scales_with_unit_roundoff(small):
    # rounding the state to b bits adds errors proportional to 2^-b: 4 more bits, ~16x less
    A, X = small
    a = chebyshev.step_coefficients(40, 2.0, 0.45, "jackson")
    ref = chebyshev.filter_recurrence(A, 2.0, a, X)
    e = {b: np.linalg.norm(storage.filter_stored(A, 2.0, a, X, state=b) - ref) for b in (14, 18)}
    assert 8.0 <= e[14] / e[18] <= 32.0
    # the same for the gathered copies alone
    e = {b: np.linalg.norm(storage.filter_stored(A, 2.0, a, X, state="f64", gather=b) - ref)
         for b in (10, 14)}
    assert 8.0 <= e[10] / e[14] <= 32.0


def test_output_rounding_alone_is_half_an_ulp(small):
    A, X = small
    a = chebyshev.step_coefficients(30, 2.0, 0.5, "jackson")
    ref = chebyshev.filter_recurrence(A, 2.0, a, X)
    got = storage.filter_stored(A, 2.0, a, X, out="bf16")
    assert np.all(np.abs(got - ref) <= 2.0 ** -8 * np.abs(ref))
    assert np.linalg.norm(got - ref) > 0.0


def test_value_rounding_is_a_perturbed_operator(small):
    # rounding A's values only equals the exact filter of the rounded operator
    A, X = small
    a = chebyshev.step_coefficients(30, 2.0, 0.5, "jackson")
    Ab = storage.round_values(A, "bf16")
    assert np.array_equal(storage.filter_stored(A, 2.0, a, X, val="bf16"),
                          chebyshev.filter_recurrence(Ab, 2.0, a, X))


def test_basis_forms_floor_ordering(small):
    # near the cut-off the recombination of BF16 copies is far worse than FP32 slots
    A, X = small
    a = chebyshev.step_coefficients(60, 2.0, 0.3, "jackson")
    Xb = philox.round_bf16(X).astype(np.float64)
    ref = chebyshev.filter_recurrence(A, 2.0, a, Xb)
    err = {f: np.linalg.norm(storage.filter_stored(A, 2.0, a, Xb, **storage.FORMS[f]) - ref) /
           np.linalg.norm(ref) for f in ("bf16s_basis", "bf16s_basis_bf16copies", "bf16io_basis")}
    assert err["bf16io_basis"] < err["bf16s_basis"] < err["bf16s_basis_bf16copies"]
