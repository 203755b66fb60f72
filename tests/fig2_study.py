"""Reuse-fraction study of Sec. 5.2 (Fig. 2(a)): multiplicative k-means cost error of dynamic
CSC against spectral clustering, as a function of the reused fraction p.

Workload (Sec. 5.2): SBM with n = 1000, mean degree s = 25, e = q2/q1 = 1/6; every snapshot
relabels 1% of the nodes and redraws 3% of the edges.  The paper gives k and d only for its
scaling runs (k = 2 log n, d = 30 log n); the same rule is used here: k = 14, d = 207.

Error (Thm 4.1 and Sec. 5.2): (C(X_Theta; Phi) - C_Phi) / C_Phi, where Phi = U_k of the
snapshot's normalized Laplacian, X_Theta is the partition dynamic CSC returns, and C_Phi is
the k-means cost of spectral clustering, taken as the best of several k-means++ restarts of
Lloyd on Phi.  C is the Frobenius form ||Phi - X X^T Phi||_F.

Test infrastructure: spectral clustering comes from the FP64 oracle, the method under study
from either the oracle or the HIP library.  Run as a script to print the table:

    python -m tests.fig2_study --backend hip --reps 20
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import time

import numpy as np

from oracle import dynamic, kmeans as okm, operator
from workloads.graphs import DynamicSBM, sbm

N, S, E = 1000, 25.0, 1.0 / 6.0
K = int(round(2 * math.log(N)))
D = int(round(30 * math.log(N)))
M = 50
RELABEL, REDRAW = 0.01, 0.03


def snapshots(rep: int, T: int):
    g0 = sbm(N, K, S, E, seed=7000 + rep)
    dyn = DynamicSBM(g0, seed=8000 + rep)
    return [g0] + [dyn.step(REDRAW, RELABEL) for _ in range(T - 1)]


def sc_cost(g, restarts: int, seed: int):
    """Phi = U_k by dense eigh, and the best k-means cost over k-means++ restarts."""
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    _, U = operator.dense_spectrum(A)
    Phi = U[:, :K]
    rng = np.random.default_rng(seed)
    best = math.inf
    for _ in range(restarts):
        C0 = Phi[okm.kmeanspp(Phi, K, rng.random(K))]
        lab = okm.lloyd(Phi, C0, 50)[0]
        best = min(best, okm.cost(Phi, lab))
    return Phi, best


def make_method(backend: str, p: float, seed: int):
    if backend == "oracle":
        orc = dynamic.DynamicCSC(N, D, K, p, M, seed=seed)
        return lambda g: orc.step(g).labels
    import torch
    import paper_1706_03591_amd as csc
    gpu = csc.DynamicCSC(N, D, K, p, M, seed=seed, keep_iterates=0)
    return lambda g: gpu.step(csc.Graph.from_workload(g))[0].cpu().numpy()


def _log(*a):
    print(*a, flush=True)


def run(backend: str, ps, reps: int, T: int, restarts: int, log=_log):
    """errors[p] = list over (rep, t >= 2) of the multiplicative error; static[p] likewise at t = 1."""
    dyn_err = {p: [] for p in ps}
    first_err = {p: [] for p in ps}
    for rep in range(reps):
        t0 = time.time()
        snaps = snapshots(rep, T)
        base = [sc_cost(g, restarts, 9000 + 31 * rep + t) for t, g in enumerate(snaps)]
        for p in ps:
            step = make_method(backend, p, seed=100 + rep)
            for t, (g, (Phi, c_sc)) in enumerate(zip(snaps, base)):
                err = (okm.cost(Phi, step(g)) - c_sc) / c_sc
                (first_err if t == 0 else dyn_err)[p].append(err)
        log(f"rep {rep}: {time.time() - t0:.1f} s")
    return dyn_err, first_err


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--backend", choices=["oracle", "hip"], default="hip")
    ap.add_argument("--reps", type=int, default=20)
    ap.add_argument("--T", type=int, default=6)
    ap.add_argument("--restarts", type=int, default=20)
    ap.add_argument("--ps", default="0,0.1,0.2,0.3,0.4,0.5")
    ap.add_argument("--json", default=None)
    a = ap.parse_args(argv)
    ps = [float(x) for x in a.ps.split(",")]
    dyn_err, first_err = run(a.backend, ps, a.reps, a.T, a.restarts)
    rows = []
    print(f"n={N} k={K} d={D} m={M} s={S} e={E:.4f}, {a.reps} replications x {a.T - 1} dynamic steps")
    print("| p | q d | mean error, dynamic steps | std | max | mean error, first snapshot |")
    print("|---|---|---|---|---|---|")
    for p in ps:
        e = np.array(dyn_err[p])
        f = np.array(first_err[p])
        rows.append(dict(p=p, qd=int(round((1 - p) * D)), mean=float(e.mean()), std=float(e.std()),
                         max=float(e.max()), first=float(f.mean())))
        print(f"| {p:.1f} | {rows[-1]['qd']} | {e.mean():.4f} | {e.std():.4f} | {e.max():.4f} | {f.mean():.4f} |")
    if a.json:
        with open(a.json, "w") as fh:
            json.dump(dict(n=N, k=K, d=D, m=M, reps=a.reps, T=a.T, restarts=a.restarts,
                           backend=a.backend, rows=rows), fh, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
