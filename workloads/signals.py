"""Seeded Gaussian signal blocks (the random matrix R of Sec. 2.2 and eigencount probes)."""

from __future__ import annotations

import numpy as np


def seed_for(config: int, purpose: str) -> int:
    """Seed recipe ``20170603 + 100 * config + offset`` (graph 0, signals 1, probes 2,
    k-means 3, perturbation 4)."""
    off = {"graph": 0, "signals": 1, "probes": 2, "kmeans": 3, "perturb": 4}[purpose]
    return 20170603 + 100 * int(config) + off


def gaussian_block(n: int, w: int, sigma: float, seed: int, dtype=np.float32,
                   chunk_rows: int = 1 << 18) -> np.ndarray:
    """Row-major n x w block of i.i.d. N(0, sigma^2) entries rounded to ``dtype``.

    Drawn in FP64 and rounded once; generated in row chunks to bound host memory.
    """
    rng = np.random.default_rng(seed)
    out = np.empty((n, w), dtype=dtype)
    for r0 in range(0, n, chunk_rows):
        r1 = min(n, r0 + chunk_rows)
        out[r0:r1] = (rng.standard_normal((r1 - r0, w)) * sigma).astype(dtype)
    return out
