"""Shared helpers for the tests: oracle operators built from workload graphs, error norms."""

from __future__ import annotations

import sys

import numpy as np

from oracle import operator


def rel_fro(x, ref) -> float:
    x = np.asarray(x, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    return float(np.linalg.norm(x - ref) / max(np.linalg.norm(ref), 1e-300))


def oracle_A(g):
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    return A


def say(*args):
    """Print and flush, so that a failing GPU step is named in the log."""
    print(*args, flush=True)
    sys.stdout.flush()


def near_tie_exempt(F64, C64, gpu_labels, tol=1e-6):
    """Rows whose two smallest oracle distances (FP64, on the same features) are within
    tol * d2 of each other may take either label."""
    from oracle import kmeans as okm
    D2 = okm.sq_distances(F64, C64)
    srt = np.sort(D2, axis=1)
    d1 = srt[:, 0]
    d2 = srt[:, 1] if D2.shape[1] > 1 else np.full_like(d1, np.inf)
    exempt = (d2 - d1) <= tol * d2
    chosen = D2[np.arange(D2.shape[0]), gpu_labels]
    ok_tie = np.abs(chosen - d1) <= tol * np.maximum(d2, 1e-300)
    return exempt, ok_tie
