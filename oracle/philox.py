"""Philox4x32-10 (Salmon, Moraes, Dror and Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC 2011) and the Gaussian draw built on it.

Philox4x32 works on a 128-bit counter (four 32-bit words) and a 64-bit key.  One round
multiplies words 0 and 2 by the constants 0xD2511F53 and 0xCD9E8D57 into 64-bit
products (hi, lo) and outputs (hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0); between rounds
the key is advanced by the Weyl constants (0x9E3779B9, 0xBB67AE85).  Ten rounds.

Gaussian entries (this library's own convention, shared by both sides only through this
definition): for row i and column pair q of a block, with 64-bit seed S and 64-bit
stream id T, the counter is (i, q, T_lo, T_hi) and the key (S_lo, S_hi).  The output
words (x0, x1, x2, x3) give two uniforms in (0, 1)
    u1 = ((x1 * 2^32 + x0) >> 11) * 2^-53 + 2^-54,   u2 likewise from (x3, x2),
and Box-Muller gives column 2q = sigma sqrt(-2 ln u1) cos(2 pi u2) and column
2q + 1 = sigma sqrt(-2 ln u1) sin(2 pi u2), computed in FP64 and rounded once to the
storage type.  A scalar uniform for index j of stream T uses counter (j, 0, T_lo, T_hi)
and the same u1 formula.

Parity pin: the known-answer vectors of the Random123 distribution
(tests/golden/philox4x32_10_kat.txt).
"""

from __future__ import annotations

import numpy as np

M0 = np.uint64(0xD2511F53)
M1 = np.uint64(0xCD9E8D57)
W0 = np.uint32(0x9E3779B9)
W1 = np.uint32(0xBB67AE85)
MASK32 = np.uint64(0xFFFFFFFF)


def philox4x32_10(ctr: np.ndarray, key: np.ndarray) -> np.ndarray:
    """ctr: (..., 4) uint32; key: (..., 2) uint32 (broadcastable).  Returns (..., 4) uint32."""
    c = [np.asarray(ctr[..., i], dtype=np.uint32) for i in range(4)]
    k0 = np.asarray(key[..., 0], dtype=np.uint32)
    k1 = np.asarray(key[..., 1], dtype=np.uint32)
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:
                k0 = (k0 + W0).astype(np.uint32)
                k1 = (k1 + W1).astype(np.uint32)
            p0 = M0 * c[0].astype(np.uint64)
            p1 = M1 * c[2].astype(np.uint64)
            hi0 = (p0 >> np.uint64(32)).astype(np.uint32)
            lo0 = (p0 & MASK32).astype(np.uint32)
            hi1 = (p1 >> np.uint64(32)).astype(np.uint32)
            lo1 = (p1 & MASK32).astype(np.uint32)
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return np.stack(c, axis=-1)


def _split64(x: int):
    x = int(x) & 0xFFFFFFFFFFFFFFFF
    return np.uint32(x & 0xFFFFFFFF), np.uint32(x >> 32)


def _u53(lo: np.ndarray, hi: np.ndarray) -> np.ndarray:
    v = (hi.astype(np.uint64) << np.uint64(32)) | lo.astype(np.uint64)
    return (v >> np.uint64(11)).astype(np.float64) * 2.0 ** -53 + 2.0 ** -54


def gaussian_block(n: int, w: int, sigma: float, seed: int, stream: int,
                   dtype=np.float64, row0: int = 0) -> np.ndarray:
    """Rows row0 .. row0 + n - 1 of the n x w Gaussian block of (seed, stream)."""
    s_lo, s_hi = _split64(seed)
    t_lo, t_hi = _split64(stream)
    npair = (w + 1) // 2
    rows = np.arange(row0, row0 + n, dtype=np.uint64).astype(np.uint32)
    ctr = np.zeros((n, npair, 4), dtype=np.uint32)
    ctr[..., 0] = rows[:, None]
    ctr[..., 1] = np.arange(npair, dtype=np.uint32)[None, :]
    ctr[..., 2] = t_lo
    ctr[..., 3] = t_hi
    key = np.array([s_lo, s_hi], dtype=np.uint32)
    x = philox4x32_10(ctr, key)
    u1 = _u53(x[..., 0], x[..., 1])
    u2 = _u53(x[..., 2], x[..., 3])
    r = np.sqrt(-2.0 * np.log(u1))
    z = np.empty((n, 2 * npair))
    z[:, 0::2] = r * np.cos(2.0 * np.pi * u2)
    z[:, 1::2] = r * np.sin(2.0 * np.pi * u2)
    z = sigma * z[:, :w]
    if dtype == "bf16":
        return round_bf16(z)
    return z.astype(dtype)


def uniforms(count: int, seed: int, stream: int) -> np.ndarray:
    """Scalar uniforms u_0..u_{count-1} in (0, 1) of (seed, stream)."""
    s_lo, s_hi = _split64(seed)
    t_lo, t_hi = _split64(stream)
    ctr = np.zeros((count, 4), dtype=np.uint32)
    ctr[:, 0] = np.arange(count, dtype=np.uint32)
    ctr[:, 2] = t_lo
    ctr[:, 3] = t_hi
    x = philox4x32_10(ctr, np.array([s_lo, s_hi], dtype=np.uint32))
    return _u53(x[:, 0], x[:, 1])


def round_bf16(x: np.ndarray) -> np.ndarray:
    """Round to bfloat16 (nearest, ties to even) via float32; returned as float32 values."""
    f = np.asarray(x, dtype=np.float32)
    b = f.view(np.uint32).astype(np.uint64)
    lsb = (b >> np.uint64(16)) & np.uint64(1)
    b = (b + np.uint64(0x7FFF) + lsb) >> np.uint64(16) << np.uint64(16)
    return (b & np.uint64(0xFFFFFFFF)).astype(np.uint32).view(np.float32)
