"""Writes the expected values of the full-size parity tests (tests/test_gpu_fullsize.py).

    python tests/golden/make_fullsize.py c3      (about 10 minutes on 4 cores)
    python tests/golden/make_fullsize.py c5 3    (about 50 minutes on 3 workers, 40 GB of RAM)

Calls only the FP64 oracle (oracle/) and the seeded input generators (workloads/).  For
each case it stores, on 10,000 sampled rows of 4 sampled columns of one snapshot's fresh
signal block:
  * the exact filter h(L) R (Sec. 2.2, Step 1; Jackson-damped step at the cut-off) of the
    signals as a form stores them: FP32, or rounded to BF16 (ref_<cut-off>_<f32|bf16>.npy
    inside <case>_fullsize.npz);
  * the storage floor of every form of oracle.storage.FORMS: the relative Frobenius error,
    on the same rows and columns, of the FP64 recurrence rounded only where that form stores
    values (<case>_floors.json).

C3: dynamic SBM, N = 1,000,000, k = 50 Zipf(1.2) blocks, degree 16, ratio 0.1; snapshot 5 of
the sequence (4 perturbations of 1% rewired edges and 0.5% moved nodes); d = 128 (signal
variance 1/128), the 64 fresh signals of snapshot 5 (Philox stream 16 * 5 + 1, seed 20170904);
m = 120; cut-offs 0.5 and 0.4 (the sequence's own cut-off is near 0.385).
C5: Chung-Lu, N = 8,000,000, 200 communities, exponent 2.5, degree 20, ratio 0.1; snapshot 2
(0.5% of the edges rewired); d = 256, the 64 fresh signals of snapshot 2 (stream 16 * 2 + 1,
seed 20171104); m = 150; cut-off 0.45 (the sequence's own is near 0.446).
"""

from __future__ import annotations

import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import cfilter, chebyshev, operator, philox, storage  # noqa: E402
from workloads import DynamicSBM, block_sizes_zipf, chung_lu, sbm, seed_for  # noqa: E402
from workloads.graphs import rewire_model_free  # noqa: E402

COLS = [0, 21, 42, 63]
N_ROWS = 10_000
ROW_SEED = 7

CASES = {
    "c3": dict(n=1_000_000, d=128, m=120, t=5, cutoffs=[0.5, 0.4], config=3),
    "c5": dict(n=8_000_000, d=256, m=150, t=2, cutoffs=[0.45], config=5),
}
# forms whose floors each case records (the paths its benchmark and tests run)
CASE_FORMS = {
    "c3": list(storage.FORMS),
    "c5": ["fp32_onepass", "bf16io_onepass", "bf16_onepass", "bf16s_onepass",
           "bf16s_basis_bf16copies", "f16_onepass", "f16_basis", "f16s_onepass",
           "f16s_basis_f16copies"],
}


def case_graph(case: str):
    """The snapshot a case filters on (workloads only)."""
    if case == "c3":
        n = CASES[case]["n"]
        g = sbm(n, 50, 16.0, 0.1, seed=seed_for(3, "graph"), sizes=block_sizes_zipf(n, 50, 1.2))
        dyn = DynamicSBM(g, seed=seed_for(3, "perturb"))
        for _ in range(CASES[case]["t"] - 1):
            g = dyn.step(0.01, 0.005)
        return g
    g = chung_lu(CASES[case]["n"], 200, 20.0, 2.5, 0.1, seed=seed_for(5, "graph"))
    return rewire_model_free(g, 0.005, seed_for(5, "perturb") + 2, 0.1)


def case_signals(case: str, store: str) -> np.ndarray:
    """The 4 sampled columns of the fresh block, as the library draws it (Philox, FP64,
    rounded once to the storage type)."""
    c = CASES[case]
    R = philox.gaussian_block(c["n"], 64, 1.0 / np.sqrt(c["d"]), seed_for(c["config"], "signals"),
                              16 * c["t"] + 1, dtype="bf16" if store == "bf16" else np.float32)
    return np.asarray(R[:, COLS], dtype=np.float64)


def case_rows(case: str) -> np.ndarray:
    return np.sort(np.random.default_rng(ROW_SEED).choice(CASES[case]["n"], N_ROWS, replace=False))


_W = {}


def _job(job):
    kind, lam, name = job
    A, X, rows, m = _W["A"], _W["X"], _W["rows"], _W["m"]
    a = chebyshev.step_coefficients(m, 2.0, lam, "jackson")
    t0 = time.perf_counter()
    form = storage.FORMS[name]
    Y = storage.filter_stored(A, 2.0, a, X[storage.form_inputs(name)], **form,
                              Lt=_W["Lt"][form["val"]])
    print(f"  {kind} {name} cut-off {lam}: {time.perf_counter() - t0:.0f} s", flush=True)
    return job, Y[rows]


def main(case: str, workers: int = 4):
    c = CASES[case]
    t0 = time.perf_counter()
    g = case_graph(case)
    A, _ = operator.normalized_adjacency(g.n, g.rowptr, g.colidx, g.w)
    print(f"{case}: graph n={g.n} nnz={g.nnz} ({time.perf_counter() - t0:.0f} s)", flush=True)
    _W.update(A=A, X={s: case_signals(case, s) for s in ("f32", "bf16")}, rows=case_rows(case),
              m=c["m"])
    # the exact filters: the oracle's multi-core C recurrence (the same FP64 operations as
    # chebyshev.filter_recurrence, pinned to it)
    res = {}
    Lt = operator.scaled_laplacian(A, 2.0)
    for lam in c["cutoffs"]:
        a = chebyshev.step_coefficients(c["m"], 2.0, lam, "jackson")
        for s in ("f32", "bf16"):
            t1 = time.perf_counter()
            Y, used = cfilter.filter_recurrence_c(None, 2.0, a, _W["X"][s], Lt=Lt)
            res[("ref", lam, s)] = Y[_W["rows"]]
            print(f"  ref {s} cut-off {lam}: {time.perf_counter() - t1:.0f} s on {used} threads", flush=True)
    del Lt
    # the storage forms: each worker shares the parent's operators (built once per value
    # format, before the fork)
    _W["Lt"] = {v: storage.stored_operator(A, 2.0, v)
                for v in sorted({storage.FORMS[f]["val"] for f in CASE_FORMS[case]})}
    jobs = [("form", lam, f) for lam in c["cutoffs"] for f in CASE_FORMS[case]]
    with mp.get_context("fork").Pool(workers) as pool:
        res.update(dict(pool.imap_unordered(_job, jobs, chunksize=1)))
    refs = {f"ref_{lam}_{s}": res[("ref", lam, s)] for lam in c["cutoffs"] for s in ("f32", "bf16")}
    floors = {}
    for lam in c["cutoffs"]:
        for f in CASE_FORMS[case]:
            ref = refs[f"ref_{lam}_{storage.form_inputs(f)}"]
            Y = res[("form", lam, f)]
            floors[f"{f}@{lam}"] = float(np.linalg.norm(Y - ref) / np.linalg.norm(ref))
    gains = {f"{lam}_{s}": float(np.linalg.norm(refs[f"ref_{lam}_{s}"]) /
                                 np.linalg.norm(_W["X"][s][_W["rows"]]))
             for lam in c["cutoffs"] for s in ("f32", "bf16")}
    np.savez(os.path.join(HERE, f"{case}_fullsize.npz"), rows=_W["rows"], cols=np.array(COLS), **refs)
    meta = dict(case=case, n=int(g.n), nnz=int(g.nnz), m=c["m"], d=c["d"], snapshot=c["t"],
                cutoffs=c["cutoffs"], cols=COLS, n_rows=N_ROWS, row_seed=ROW_SEED,
                signal_seed=seed_for(c["config"], "signals"), signal_stream=16 * c["t"] + 1,
                damping="jackson", lmax=2.0, gain=gains, floors=floors,
                script="tests/golden/make_fullsize.py")
    with open(os.path.join(HERE, f"{case}_floors.json"), "w") as f:
        json.dump(meta, f, indent=1)
    print(json.dumps(floors, indent=1))
    print(f"{case}: done in {time.perf_counter() - t0:.0f} s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "c3",
         int(sys.argv[2]) if len(sys.argv) > 2 else 4)
