"""Benchmark: dynamic compressive spectral clustering on one MI355X.

Workload (default): the dynamic SBM sequence N = 1,000,000, k = 50 blocks of Zipf(1.2)
sizes, mean degree 16, inter/intra ratio 0.1; each snapshot rewires 1% of the edges and
moves 0.5% of the nodes; d = 128 signals, Chebyshev degree m = 120, reuse p = 0.5.  A step
is one dynamic snapshot (Algorithm 1 steps 4-8: operator build, q d = 64 fresh signals,
filter, eigencount, refinement when needed, k-means with 20 Lloyd rounds), with every
snapshot's CSR already resident in HBM.  The storage forms (FORMS below) run on the same
snapshots: FP32 everywhere; BF16 signals/features/values with FP32 iterates (bf16io), BF16
iterates (bf16), BF16 gathered copies with an FP32 recurrence state (bf16s), binary16
iterates (f16, the headline) or binary16 copies with an FP32 state (f16s); each with a
suffix b for the fresh blocks of several snapshots in one batched, graph-replayed recurrence,
and b1p for batches without kept iterates.

Printed: one JSON line.  `value` is the whole-job rate of the Chebyshev step kernels'
algorithmic bytes (GB/s over the timed wall clock) of the headline form; `roofline` gives
the step kernel's own rate from HIP events on its stream; `errors_vs_fp64_oracle` is each
form's error on the columns its last timed snapshot wrote; `cpu_baseline` times the FP64
oracle (its multi-core C recurrence) filtering a 4-column sample of that snapshot on all host
cores and on one.
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_GBPS = 8000.0


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=12)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=None, help="nodes (default: the workload's configuration)")
    ap.add_argument("--k", type=int, default=None)
    ap.add_argument("--d", type=int, default=None)
    ap.add_argument("--m", type=int, default=None)
    ap.add_argument("--p", type=float, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-error", action="store_true")
    ap.add_argument("--forms", default="fp32,bf16io,bf16,bf16s,bf16b,bf16sb,f16,f16s,f16b,f16sb",
                    help="comma list of " + ", ".join(f"{k}: {v[5]}" for k, v in FORMS.items()))
    ap.add_argument("--headline", default="f16")
    ap.add_argument("--init", choices=["pp", "warm"], default="pp",
                    help="k-means start per snapshot: k-means++ (pp) or the previous labels' means")
    ap.add_argument("--batch", type=int, default=4, help="snapshots per batched recurrence")
    ap.add_argument("--workload", choices=["c3", "c2", "c4", "c5", "ckm", "psweep", "kassign", "gather"],
                    default="c3")
    ap.add_argument("--ps", default="0,0.25,0.5,0.75", help="psweep: reused fractions p")
    ap.add_argument("--n-sample", type=int, default=0,
                    help="ckm: sampled nodes (0: ceil(4 k ln k))")
    ap.add_argument("--probe", metavar="FORM",
                    help="counter probe: snapshot 1 and one batch of FORM's dynamic steps on the "
                         "C3 sequence, then a plain 1 GiB device copy (run under rocprofv3 --pmc)")
    ap.add_argument("--traffic", nargs=2, metavar=("FETCH_CSV", "WRITE_CSV"),
                    help="turn two rocprofv3 counter_collection.csv files (FETCH_SIZE, WRITE_SIZE) "
                         "of --probe FORM into profiles/k_step_c3_traffic.json")
    args = ap.parse_args()
    # the configuration table (workloads/configs.py) supplies the sizes of each workload
    from workloads import CONFIGS

    cfg = {"c2": 2, "c4": 4, "c5": 5, "kassign": 5}.get(args.workload, 3)
    c = CONFIGS[cfg]
    for key in ("n", "k", "d", "m", "p"):
        if getattr(args, key) is None:
            setattr(args, key, c.get(key, 0.5))
    args.config = c
    return args


# name -> (features/signals, iterates, operator values, batched, hipGraph replay, description)
FORMS = {
    "fp32": ("float32", "float32", "float32", False, False, "FP32 everywhere"),
    "bf16": ("bfloat16", "bfloat16", "bfloat16", False, False,
             "BF16 signals, features, operator values and recurrence iterates; FP32 arithmetic "
             "and accumulation"),
    "bf16io": ("bfloat16", "float32", "bfloat16", False, False,
               "BF16 signals, features and operator values; FP32 iterates"),
    "bf16b": ("bfloat16", "bfloat16", "bfloat16", True, True,
              "the bf16 form with the fresh blocks of --batch snapshots filtered in one batched "
              "recurrence replayed from a HIP graph"),
    "fp32g": ("float32", "float32", "float32", False, True, "FP32 with HIP-graph replay"),
    "bf16s": ("bfloat16", "bf16s", "bfloat16", False, False,
              "BF16 signals, features, operator values and gathered iterate copies; the "
              "recurrence state, arithmetic and accumulation FP32"),
    "bf16sb": ("bfloat16", "bf16s", "bfloat16", True, True,
               "the bf16s form with the fresh blocks of --batch snapshots filtered in one "
               "batched recurrence replayed from a HIP graph"),
    "f16": ("bfloat16", "float16", "bfloat16", False, False,
            "BF16 signals, features and operator values; IEEE binary16 recurrence iterates; "
            "FP32 arithmetic and accumulation"),
    "f16b": ("bfloat16", "float16", "bfloat16", True, True,
             "the f16 form with the fresh blocks of --batch snapshots filtered in one batched "
             "recurrence replayed from a HIP graph"),
    "f16s": ("bfloat16", "f16s", "bfloat16", False, False,
             "BF16 signals, features and operator values; binary16 gathered iterate copies; the "
             "recurrence state, arithmetic and accumulation FP32"),
    "f16sb": ("bfloat16", "f16s", "bfloat16", True, True,
              "the f16s form with the fresh blocks of --batch snapshots filtered in one batched "
              "recurrence replayed from a HIP graph"),
}
for _f in ("fp32", "f16", "f16s", "bf16s"):
    _b = FORMS[_f]
    FORMS[_f + "b1p"] = (_b[0], _b[1], _b[2], True, True,
                         f"the {_f} form with the fresh blocks of --batch snapshots filtered in one "
                         f"batched one-pass recurrence (FP32 running sum, no kept iterates) replayed "
                         f"from a HIP graph; snapshots whose cut-off changed are filtered again")
SPLIT_MODES = ("bf16s", "f16s")
# forms that keep no iterates (one-pass recurrences)
ONEPASS = {f for f in FORMS if f.endswith("b1p")}


def torch_types(form):
    """(features, iterates, values) of a form; iterates may be a split-mode string."""
    import torch

    fdt, idt, vdt = FORMS[form][:3]
    return getattr(torch, fdt), (idt if idt in SPLIT_MODES else getattr(torch, idt)), getattr(torch, vdt)


def kernel_digest() -> str:
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_1706_03591_amd", "csrc", "k_cheb.hip"), "rb") as f:
        h.update(f.read())
    return h.hexdigest()[:16]


def traffic_path(workload: str) -> str:
    return os.path.join(ROOT, "profiles", f"k_step_{workload}_traffic.json")


def load_traffic(digest: str, form: str, workload: str = "c3"):
    """HBM bytes per step launch from the committed counter summary of this workload, if it
    was taken on this exact kernel source; else None."""
    path = traffic_path(workload)
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_sha256_16") != digest:
        return None
    return rec.get("bytes_per_launch", {}).get(form)


def build_sequence(args, T):
    import numpy as np

    from workloads import DynamicSBM, block_sizes_zipf, sbm, seed_for

    t0 = time.perf_counter()
    c = args.config
    if args.workload == "c5":
        from workloads import chung_lu
        from workloads.graphs import rewire_model_free

        g = chung_lu(args.n, args.k, c["degree"], c["exponent"], c["ratio"], seed=seed_for(5, "graph"))
        log(f"[bench] snapshot 1: nnz {g.nnz} ({time.perf_counter() - t0:.1f} s)")
        seq = [g]
        for t in range(2, T + 1):
            seq.append(rewire_model_free(seq[-1], c["rewire"], seed_for(5, "perturb") + t, c["ratio"]))
            log(f"[bench] snapshot {t}: nnz {seq[-1].nnz} ({time.perf_counter() - t0:.1f} s)")
        return seq, np
    sizes = block_sizes_zipf(args.n, args.k, c["zipf_s"])
    g = sbm(args.n, args.k, c["degree"], c["ratio"], seed=seed_for(3, "graph"), sizes=sizes)
    log(f"[bench] snapshot 1: nnz {g.nnz} ({time.perf_counter() - t0:.1f} s)")
    dyn = DynamicSBM(g, seed=seed_for(3, "perturb"))
    seq = [g]
    for t in range(2, T + 1):
        seq.append(dyn.step(c["rewire"], c["move"]))
        log(f"[bench] snapshot {t}: nnz {seq[-1].nnz} ({time.perf_counter() - t0:.1f} s)")
    return seq, np


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: the path is single-GPU by design (column sharding "
              "across GPUs is not built); run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.traffic:
        return traffic_summary(args)
    if args.probe:
        return run_probe(args)
    {"c3": run_dynamic, "c5": run_dynamic, "c2": run_static, "c4": run_adjoint,
     "ckm": run_compressive, "psweep": run_psweep, "kassign": run_kassign,
     "gather": run_gather}[args.workload](args)


def run_probe(args):
    """Snapshot 1 plus one batch of the form's dynamic steps, then a 1 GiB device copy whose
    counter readings calibrate FETCH_SIZE / WRITE_SIZE to bytes."""
    import torch

    import paper_1706_03591_amd as csc
    from workloads import seed_for

    fdt, idt, vdt, batched, graph, _ = FORMS[args.probe]
    feat, iters, vals = torch_types(args.probe)
    T = 1 + args.batch
    seq, _ = build_sequence(args, T)
    dev = torch.device("cuda")
    cap = max(g.nnz for g in seq)
    Gs = [csc.Graph(args.n, *(torch.from_numpy(a).to(dev) for a in (g.rowptr, g.colidx, g.w)),
                    val_dtype=vals, validate=False, nnz_capacity=cap) for g in seq]
    cid = 5 if args.workload == "c5" else 3
    dyn = csc.DynamicCSC(args.n, args.d, args.k, args.p, args.m, seed=seed_for(cid, "signals"),
                         feat_dtype=feat, iter_dtype=iters, batch=args.batch if batched else 1,
                         use_graph=graph, keep_iterates=1 if batched else -1)
    dyn.step(Gs[0])
    if batched:
        dyn.steps(Gs[1:])
    else:
        for G in Gs[1:]:
            dyn.step(G)
    torch.cuda.synchronize()
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    log("[bench] probe done")


def traffic_summary(args):
    """HBM bytes per launch of the dominant step kernel: FETCH_SIZE and WRITE_SIZE (KiB per
    dispatch, summed over the counter's instances) scaled by what the same counters read for
    the plain 1 GiB copy of the probe."""
    import csv
    import statistics

    form = args.probe or args.headline
    kname = "k_step_batch"  # the stored-basis step of every form at C3

    def per_dispatch(path, counter):
        out = {}
        with open(path) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                name, v = out.get(r["Dispatch_Id"], (r["Kernel_Name"], 0.0))
                out[r["Dispatch_Id"]] = (name, v + float(r["Counter_Value"]))
        return list(out.values())

    fetch = per_dispatch(args.traffic[0], "FETCH_SIZE")
    write = per_dispatch(args.traffic[1], "WRITE_SIZE")
    gib_kib = float(1 << 20)
    # the probe's 1 GiB copy is the largest copy dispatch (the others move labels and CSR)
    cf = max(v for n, v in fetch if "copyBuffer" in n)
    cw = max(v for n, v in write if "copyBuffer" in n)
    sf, sw = gib_kib / cf, gib_kib / cw
    # (rocprofv3 leaves names with binary16 template arguments mangled)
    sel = lambda rows: [v for n, v in rows if kname in n]  # noqa: E731
    stf, stw = sel(fetch), sel(write)
    per_launch = (statistics.mean(stf) * sf + statistics.mean(stw) * sw) * 1024.0
    path = traffic_path(args.workload)
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        rec = {}
    digest = kernel_digest()
    if rec.get("kernel_sha256_16") != digest:
        rec = {"kernel_sha256_16": digest, "bytes_per_launch": {}, "detail": {}}
    rec["bytes_per_launch"][form] = per_launch
    rec["detail"][form] = {
        "kernel": kname, "launches": len(stf),
        "fetch_kib_raw_mean": statistics.mean(stf), "write_kib_raw_mean": statistics.mean(stw),
        "copy_fetch_kib_raw": cf, "copy_write_kib_raw": cw,
        "scale_fetch": sf, "scale_write": sw,
    }
    with open(path, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps({"form": form, "bytes_per_launch": per_launch, **rec["detail"][form]}))


def _time_form(args, form, p, resident, cap, cid):
    """Snapshot 1, the warm-up snapshots, then the timed snapshots of one storage form at
    reuse fraction p; returns the form's record and the timed snapshots' labels."""
    import torch

    import paper_1706_03591_amd as csc
    from workloads import seed_for

    dev = torch.device("cuda")
    T = 1 + args.warmup + args.steps
    fdt, idt, vdt, batched, graph, _ = FORMS[form]
    feat, iters, vals = torch_types(form)
    rp, ci, ww = resident[0]
    G = csc.Graph(args.n, rp, ci, ww, val_dtype=vals, validate=True, nnz_capacity=cap)
    # kernel shape of the fresh block's recurrence, timed on snapshot 1
    qd = int(round((1 - p) * args.d))
    variant = G.autotune(qd, iter_dtype=iters)
    dyn = csc.DynamicCSC(args.n, args.d, args.k, p, args.m, seed=seed_for(cid, "signals"),
                         feat_dtype=feat, iter_dtype=iters, batch=args.batch if batched else 1,
                         use_graph=graph, variant=variant,
                         keep_iterates=0 if form in ONEPASS else (1 if batched else -1),
                         init=1 if args.init == "warm" else 0)
    labels = torch.empty(args.n, dtype=torch.int32, device=dev)
    _, lam, ref, cnt = dyn.step(G, labels)
    log(f"[bench] {form}: snapshot 1 lambda {lam:.5f} count {cnt:.2f}")
    for t in range(2, 2 + args.warmup):
        G.update_device(*resident[t - 1], validate=False)
        dyn.step(G, labels)
    timed = list(range(2 + args.warmup, T + 1))
    labs = [torch.empty(args.n, dtype=torch.int32, device=dev) for _ in timed]
    # every form runs the timed snapshots through the sequence call (Algorithm 1 over the
    # list): batched forms advance several recurrences per launch, and a state with one
    # buffer of kept iterates starts each next recurrence beside the current k-means
    Gs = [G] + [csc.Graph(args.n, rp, ci, ww, val_dtype=vals, validate=False, nnz_capacity=cap)
                for _ in range(len(timed) - 1)]
    torch.cuda.synchronize()
    csc.timing_reset()
    csc.timing_enable(True)
    refines = 0
    lams = []
    t0 = time.perf_counter()
    for q, t in enumerate(timed):
        Gs[q].update_device(*resident[t - 1], validate=False)
    labs, lams, refs, _ = dyn.steps(Gs, labs)
    refines = sum(refs)
    labels = labs[-1]
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    # the last timed snapshot's fresh columns as the timed path wrote them into Theta: the
    # ring's cursor starts at column 0 on snapshot 2 and advances by q d per snapshot
    rows, cols = error_sample(args, qd)
    c0 = ((T - 2) * qd) % args.d
    idx = torch.tensor([(c0 + c) % args.d for c in cols], device=dev)
    theta_sample = (dyn.features().index_select(0, torch.from_numpy(rows).to(dev))
                    .index_select(1, idx).double().cpu().numpy())
    kms, launches, kbytes = csc.timing_read()
    csc.timing_enable(False)
    log(f"[bench] {form}: {wall / args.steps * 1e3:.2f} ms/snapshot, step kernels "
        f"{kms / launches * 1e3:.1f} us/launch, {kbytes / (kms * 1e-3) / 1e9:.0f} GB/s, "
        f"refines {refines}")
    entry = dict(
        ms_per_snapshot=wall / args.steps * 1e3,
        gbps_whole=kbytes / wall / 1e9,
        step_kernel_gbps=kbytes / (kms * 1e-3) / 1e9,
        step_kernel_us=kms / launches * 1e3,
        step_launches=launches,
        bytes_per_launch=kbytes / launches,
        refines=refines,
        lambda_last=lams[-1] if lams else None,
        storage=dict(signals=fdt, features=fdt, values=vdt, iterates=idt, accumulate="float32"),
        batch=args.batch if batched else 1,
        hip_graph=graph,
        autotuned_variant=variant,
        G=G,
        theta_sample=theta_sample,
    )
    del dyn
    if batched:
        del Gs
    return entry, labs


def error_sample(args, qd):
    """(rows, cols) of the error sample: 10k rows drawn with the probe seed, 4 fresh columns."""
    import numpy as np

    from workloads import seed_for

    cid = 5 if args.workload == "c5" else 3
    cols = [0, 21, 42, 63] if qd >= 64 else list(range(min(4, qd)))
    rows = np.sort(np.random.default_rng(seed_for(cid, "probes")).choice(args.n, 10_000, replace=False))
    return rows, cols


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def timed_path_errors(args, gl, T, cid, forms):
    """Per form: the relative Frobenius error of the timed path's last fresh columns against
    the FP64 oracle (the multi-core C filter of oracle/), and the CPU baseline: that oracle
    filter timed on all host cores and on one."""
    import numpy as np

    from oracle import cfilter, chebyshev, operator, philox
    from workloads import seed_for

    qd = int(round((1 - args.p) * args.d))
    rows, cols = error_sample(args, qd)
    A, _ = operator.normalized_adjacency(gl.n, gl.rowptr, gl.colidx, gl.w)
    sig = {}
    for store in ("f32", "bf16"):
        R = philox.gaussian_block(args.n, qd, 1.0 / np.sqrt(args.d), seed_for(cid, "signals"),
                                  16 * T + 1, dtype="bf16" if store == "bf16" else np.float32)
        sig[store] = np.asarray(R[:, cols], dtype=np.float64)
    cache, errors, cpu = {}, {}, None
    for form, rec in forms.items():
        store = "bf16" if FORMS[form][0] == "bfloat16" else "f32"
        lam = rec["lambda_last"]
        key = (lam, store)
        if key not in cache:
            a = chebyshev.step_coefficients(args.m, 2.0, lam, "jackson")
            log(f"[bench] oracle: FP64 filter of {len(cols)} columns of snapshot {T} at cut-off "
                f"{lam:.6f} ({store} signals)")
            t0 = time.perf_counter()
            Y, used = cfilter.filter_recurrence_c(A, 2.0, a, sig[store])
            t_all = time.perf_counter() - t0
            cache[key] = Y[rows]
            if cpu is None:
                t0 = time.perf_counter()
                cfilter.filter_recurrence_c(A, 2.0, a, sig[store], threads=1)
                t_one = time.perf_counter() - t0
                nnz = gl.nnz + gl.n  # L~ stores the diagonal too
                alg = args.m * (nnz * 12.0 + 8.0 * (gl.n + 1) + gl.n * len(cols) * (3 * 8 + 2 * 8))
                cpu = dict(value=round(alg / t_all / 1e9, 3), unit="GB/s", cores=used, kind="oracle",
                           one_core_value=round(alg / t_one / 1e9, 3), cpu_model=cpu_model(),
                           nproc=os.cpu_count(),
                           sample=f"FP64 C/OpenMP three-term filter of the oracle, {len(cols)} of the "
                                  f"{qd} fresh columns of snapshot {T} (N={gl.n}, nnz={gl.nnz}, "
                                  f"m={args.m}): {t_all:.2f} s on {used} threads, {t_one:.2f} s on "
                                  f"one; the {qd}-column filter of one snapshot extrapolates to "
                                  f"{t_all * qd / len(cols):.1f} s on {used} threads",
                           seconds=round(t_all, 3), seconds_one_core=round(t_one, 3))
        ref = cache[key]
        got = rec["theta_sample"]
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        gain = float(np.linalg.norm(ref) / np.linalg.norm(sig[store][rows]))
        errors[form] = dict(rel_fro_vs_fp64=err, cut_off=lam, snapshot=T,
                            output_over_input=gain, signals=store)
        log(f"[bench] {form}: timed-path error {err:.3e} of the output at cut-off {lam:.5f} "
            f"(the filter keeps {gain:.4f} of the input)")
    return errors, cpu


def golden_errors(args, resident, cap, forms):
    """Per form: snapshot 2's fresh block (4 columns, 10k rows) filtered by a dynamic state in
    the form's configuration with the cut-off fixed through an imported state, against the
    committed FP64 expected values and storage floors of the C5 case."""
    import numpy as np
    import torch

    import paper_1706_03591_amd as csc
    from workloads import seed_for

    gdir = os.path.join(ROOT, "tests", "golden")
    with open(os.path.join(gdir, "c5_floors.json")) as f:
        meta = json.load(f)
    gold = np.load(os.path.join(gdir, "c5_fullsize.npz"))
    lam = meta["cutoffs"][0]
    rows, cols = gold["rows"], gold["cols"]
    seed = seed_for(5, "signals")
    qd = int(round((1 - args.p) * args.d))
    floor_of = {"fp32": "fp32_onepass", "bf16s": "bf16s_basis_bf16copies", "f16": "f16_basis",
                "f16s": "f16s_basis_f16copies", "f16b1p": "f16_onepass", "f16sb1p": "f16s_onepass",
                "bf16sb1p": "bf16s_onepass", "fp32b1p": "fp32_onepass", "bf16": "bf16_basis",
                "bf16io": "bf16io_onepass"}
    errors = {}
    for form in forms:
        feat, iters, vals = torch_types(form)
        batched = FORMS[form][3]
        keep = 0 if form in ONEPASS else (1 if batched else -1)
        G = csc.Graph(args.n, *resident[1], val_dtype=vals, validate=False, nnz_capacity=cap)
        st = csc.DynamicCSC(args.n, args.d, args.k, args.p, args.m, seed=seed, feat_dtype=feat,
                            iter_dtype=iters, tau=1e9, keep_iterates=keep,
                            batch=args.batch if batched else 1, use_graph=FORMS[form][4],
                            lloyd_iters=1)
        buf = bytearray(csc.lib.csc_dyn_state_bytes(st.h))
        h = csc.DynamicCSC.header(buf)
        h.magic, h.n, h.d, h.k, h.m, h.qd = 0x31304E5944435343, args.n, args.d, args.k, args.m, qd
        h.feat_dt, h.t, h.cursor, h.seed, h.lam = (0 if feat == torch.float32 else 1), 1, 0, seed, lam
        st.import_state(buf)
        _, lams, _, _ = st.steps([G])
        th = st.features()
        got = th.index_select(0, torch.from_numpy(rows).cuda()).index_select(
            1, torch.from_numpy(cols).cuda()).double().cpu().numpy()
        del th, st, G
        torch.cuda.empty_cache()
        ref = gold[f"ref_{lam}_{'f32' if feat == torch.float32 else 'bf16'}"]
        err = float(np.linalg.norm(got - ref) / np.linalg.norm(ref))
        fl = meta["floors"].get(f"{floor_of.get(form, '')}@{lam}")
        errors[form] = dict(rel_fro_vs_fp64=err, cut_off=lam, snapshot=2, storage_floor=fl,
                            source="tests/golden/c5_fullsize.npz (10k rows x 4 columns)")
        log(f"[bench] {form}: error {err:.3e} of the output at cut-off {lam} (snapshot 2; floor {fl})")
    return errors


def run_dynamic(args):
    import numpy as np
    import torch

    import paper_1706_03591_amd as csc
    from workloads import seed_for

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    T = 1 + args.warmup + args.steps
    cid = 5 if args.workload == "c5" else 3
    seq, _ = build_sequence(args, T)
    dev = torch.device("cuda")
    resident = []
    for g in seq:
        resident.append((torch.from_numpy(g.rowptr).to(dev), torch.from_numpy(g.colidx).to(dev),
                         torch.from_numpy(g.w).to(dev)))
    cap = max(g.nnz for g in seq)
    torch.cuda.synchronize()
    log(f"[bench] {T} snapshots resident on the GPU, max nnz {cap}")

    forms = {}
    digest = kernel_digest()
    final_labels = {}
    all_labels = {}
    for form in args.forms.split(","):
        forms[form], labs = _time_form(args, form, args.p, resident, cap, cid)
        final_labels[form] = labs[-1].cpu().numpy()
        all_labels[form] = [x.cpu().numpy() for x in labs]

    # error of the timed path: the last timed snapshot's fresh columns (4 of them, 10k sampled
    # rows) as each form wrote them into Theta, against the FP64 oracle's filter of the same
    # Philox signals on the same snapshot at the cut-off that form's snapshot used; the
    # oracle runs double as the CPU baseline
    errors, cpu = {}, None
    if not args.no_error:
        if args.workload == "c5":
            # the oracle over 8M nodes and 160M entries takes minutes per cut-off even on all
            # host cores, so at C5 each form filters snapshot 2's fresh block at the fixed
            # cut-off of the committed expected values (tests/golden/make_fullsize.py)
            errors = golden_errors(args, resident, cap, forms)
        else:
            errors, cpu = timed_path_errors(args, seq[-1], T, cid, forms)
    head = forms[args.headline]
    traffic = load_traffic(digest, args.headline, args.workload)
    achieved = head["step_kernel_gbps"]
    out = {
        "metric": "Chebyshev SpMM HBM GB/s (% peak) & ms/dynamic snapshot, BF16 vs FP32 at tol",
        "value": round(head["gbps_whole"], 2),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_snapshot"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": (f"dynamic SBM N={args.n}, k={args.k} Zipf(1.2) blocks, degree 16, ratio 0.1, "
                         f"1% edges rewired + 0.5% nodes moved per snapshot; d={args.d}, m={args.m}, "
                         f"p={args.p}; step = one dynamic snapshot") if args.workload == "c3" else
                        (f"dynamic Chung-Lu N={args.n}, exponent 2.5, degree 20, {args.k} planted "
                         f"communities, ratio 0.1, 0.5% edges rewired per snapshot; d={args.d}, "
                         f"m={args.m}, p={args.p}; step = one dynamic snapshot"),
            "n": args.n, "nnz_max": cap, "d": args.d, "m": args.m, "p": args.p, "k": args.k,
            "storage": FORMS[args.headline][5], "parallelism": "single GPU",
            "kmeans_init": "k-means++" if args.init == "pp" else "previous labels' means",
        },
        "roofline": {
            "bound": "hbm",
            "kernel": ("k_step_batch<%s> (fused Chebyshev SpMM + three-term update, %s)" % (
                FORMS[args.headline][1], "one-pass: FP32 running sum" if args.headline in ONEPASS
                else "iterates kept for recombination")),
            "achieved": round(achieved, 1),
            "peak": PEAK_GBPS,
            "unit": "GB/s",
            "frac": round(achieved / PEAK_GBPS, 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": round(head["bytes_per_launch"]),
            "avg_launch_us": round(head["step_kernel_us"], 2),
            # the measured HBM-side bytes over the live launch time: the rate to compare with
            # the random-gather ceiling of the gather workload
            "traffic_rate_tb_s": (round(traffic / (head["step_kernel_us"] * 1e-6) / 1e12, 3)
                                  if traffic else None),
            "note": ("live launches run beside the previous snapshot's recombination and k-means "
                     "on a second stream; the gathers fetch each neighbour row from beyond L2, so "
                     "traffic exceeds the algorithmic bytes"),
        },
        "forms": {f: {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()
                      if k not in ("G", "theta_sample")}
                  for f, r in forms.items()},
        "errors_vs_fp64_oracle": errors,
        "cpu_baseline": None if args.no_cpu_baseline else cpu,
        "kernel_sha256_16": digest,
        "headline_note": (
            f"value and roofline count the {args.headline} form's own algorithmic bytes; 16-bit "
            f"iterates move half of FP32's per step, so a faster form can show fewer GB/s: "
            + ", ".join(f"{f} {r['ms_per_snapshot']:.1f} ms" for f, r in forms.items())
            + " per snapshot"),
    }
    if "fp32" in forms:
        out["speedup_per_snapshot_vs_fp32"] = {
            f: round(forms["fp32"]["ms_per_snapshot"] / r["ms_per_snapshot"], 4) for f, r in forms.items() if f != "fp32"}
    # clustering quality against the planted partition of each timed snapshot
    from sklearn.metrics import adjusted_rand_score, normalized_mutual_info_score

    timed = list(range(2 + args.warmup, T + 1))
    quality = {}
    for f, labs in all_labels.items():
        nmi = [normalized_mutual_info_score(seq[t - 1].labels, lab) for t, lab in zip(timed, labs)]
        ari = [adjusted_rand_score(seq[t - 1].labels, lab) for t, lab in zip(timed, labs)]
        quality[f] = dict(nmi_mean=round(float(np.mean(nmi)), 5), nmi_std=round(float(np.std(nmi)), 5),
                          ari_mean=round(float(np.mean(ari)), 5), ari_std=round(float(np.std(ari)), 5))
    out["quality_vs_planted_timed_snapshots"] = quality
    if "fp32" in final_labels:
        # agreement of the last snapshot's partition with the FP32 form's, up to relabelling
        ref = final_labels["fp32"]
        agree = {}
        for f, lab in final_labels.items():
            if f == "fp32":
                continue
            cont = np.zeros((args.k, args.k), dtype=np.int64)
            np.add.at(cont, (ref, lab), 1)
            agree[f] = round(float(cont.max(axis=1).sum()) / len(ref), 5)
        out["label_agreement_vs_fp32_last_snapshot"] = agree
    print(json.dumps(out), flush=True)


def _line(args, metric, value, unit, ms, extra):
    out = {"metric": metric, "value": round(value, 3), "unit": unit, "n_gpus": 1, "steps": args.steps,
           "warmup": args.warmup, "ms_per_step": round(ms, 3), "higher_is_better": True,
           "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic"}
    out.update(extra)
    print(json.dumps(out), flush=True)


def run_static(args):
    """C2: static CSC on an SBM (N=200k, k=20, degree 20): eigencount with 24 probes and a
    16-step dichotomy (one moment pass), the filter of 64 signals at the found cut-off (m=100),
    k-means++ and 20 Lloyd rounds.  A step is one full static CSC."""
    import numpy as np
    import torch

    import paper_1706_03591_amd as csc
    from workloads import gaussian_block, sbm, seed_for

    g = sbm(args.n, args.k, args.config["degree"], args.config["ratio"], seed=seed_for(2, "graph"))
    log(f"[bench] C2 graph nnz {g.nnz}")
    G = csc.Graph.from_workload(g)
    variant = G.autotune(args.d)
    R = torch.from_numpy(gaussian_block(args.n, args.d, 1 / np.sqrt(args.d), seed=seed_for(2, "signals"))).cuda()
    P = torch.from_numpy(gaussian_block(args.n, 24, 1 / np.sqrt(args.d), seed=seed_for(2, "probes"))).cuda()
    Y = torch.empty_like(R)

    def once():
        lam, cnt, _, _ = csc.eigcount(G, args.m, P, sigma2=1.0 / args.d, k=args.k, n_cand=16)
        a = csc.cheb_coeffs(args.m, 2.0, lam)
        csc.cheb_filter(G, a, R, out=Y)
        lab, C = csc.kmeans(Y, args.k, iters=20, seed=seed_for(2, "kmeans"), stream_id=2)
        return lam, cnt

    for _ in range(args.warmup):
        once()
    torch.cuda.synchronize()
    csc.timing_reset()
    csc.timing_enable(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lam, cnt = once()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    kms, launches, kbytes = csc.timing_read()
    csc.timing_enable(False)
    _line(args, "static CSC: Chebyshev SpMM GB/s & ms per clustering", kbytes / (wall * args.steps) / 1e9,
          "GB/s", wall * 1e3,
          {"config": {"workload": f"static SBM N={args.n}, k={args.k}, degree 20, ratio 0.1; 24 probes, "
                                  f"16 dichotomy steps, d={args.d}, m={args.m}, 20 Lloyd rounds",
                      "nnz": g.nnz, "lambda": lam, "count": cnt, "autotuned_variant": variant},
           "roofline": {"bound": "hbm", "achieved": round(kbytes / (kms * 1e-3) / 1e9, 1),
                        "peak": PEAK_GBPS, "unit": "GB/s",
                        "frac": round(kbytes / (kms * 1e-3) / 1e9 / PEAK_GBPS, 4),
                        "avg_launch_us": round(kms / launches * 1e3, 2), "traffic": None}})


def run_adjoint(args):
    """C4: Chebyshev filter forward (m=60, 64 signals) and its adjoint (dX, the 61 coefficient
    gradients and one gradient per stored edge value, checkpoints every 8 iterates) on the
    N=200k SBM.  A step is one forward plus one backward."""
    import numpy as np
    import torch

    import paper_1706_03591_amd as csc
    from workloads import gaussian_block, sbm, seed_for

    g = sbm(args.n, args.k, args.config["degree"], args.config["ratio"], seed=seed_for(4, "graph"))
    G = csc.Graph.from_workload(g)
    X = torch.from_numpy(gaussian_block(args.n, args.d, 1 / np.sqrt(args.d), seed=seed_for(4, "signals"))).cuda()
    Gr = torch.from_numpy(gaussian_block(args.n, args.d, 1.0, seed=seed_for(4, "probes"))).cuda()
    a = csc.cheb_coeffs(args.m, 2.0, 0.5)
    Y = torch.empty_like(X)

    def once():
        csc.cheb_filter(G, a, X, out=Y)
        return csc.filter_backward(G, a, X, Gr, ckpt_every=8)

    for _ in range(args.warmup):
        once()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        once()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    nnz = g.nnz
    nw = args.n * args.d
    fwd = args.m * (nnz * 8 + 4 * (args.n + 1) + nw * 20)
    # backward: checkpointed forward (3 streams + G read per step), segment recompute (same),
    # adjoint steps (2 gathers + 2 streams + G read + one dA read-modify-write per entry)
    bwd = args.m * (nnz * 8 + nw * 16) * 2 + args.m * (nnz * 16 + nw * 20)
    rate = (fwd + bwd) / wall / 1e9
    _line(args, "Chebyshev filter forward+backward: algorithmic GB/s & ms per pair",
          rate, "GB/s", wall * 1e3,
          {"config": {"workload": f"SBM N={args.n}, k={args.k}, degree 20; w={args.d}, m={args.m}, "
                                  f"checkpoint every 8 iterates; dX, da and dA", "nnz": nnz},
           "roofline": {"bound": "hbm", "kernel": "forward steps + checkpointed recompute + fused "
                                                  "adjoint (whole pair)",
                        "achieved": round(rate, 1), "peak": PEAK_GBPS, "unit": "GB/s",
                        "frac": round(rate / PEAK_GBPS, 4), "traffic": None,
                        "algorithmic_bytes": round(fwd + bwd)}})


def run_psweep(args):
    """Time side of the reuse study (Sec. 5.2, Fig. 2(b)) at C3 scale: ms per dynamic snapshot
    of the headline form as the reused fraction p grows, on the C3 sequence.  The value is the
    time saved at the largest p relative to p = 0 (the paper reports up to 25%)."""
    import torch

    T = 1 + args.warmup + args.steps
    seq, _ = build_sequence(args, T)
    dev = torch.device("cuda")
    resident = [(torch.from_numpy(g.rowptr).to(dev), torch.from_numpy(g.colidx).to(dev),
                 torch.from_numpy(g.w).to(dev)) for g in seq]
    cap = max(g.nnz for g in seq)
    ps = [float(x) for x in args.ps.split(",")]
    rows = []
    for p in ps:
        entry, _ = _time_form(args, args.headline, p, resident, cap, 3)
        rows.append(dict(p=p, qd=int(round((1 - p) * args.d)),
                         ms_per_snapshot=round(entry["ms_per_snapshot"], 3),
                         step_kernel_us=round(entry["step_kernel_us"], 1),
                         refines=entry["refines"], batch=entry["batch"]))
        del entry
        torch.cuda.empty_cache()
    base = rows[0]["ms_per_snapshot"]
    for r in rows:
        r["saved_vs_first"] = round(1.0 - r["ms_per_snapshot"] / base, 4)
    last = rows[-1]
    _line(args, f"time saved per dynamic snapshot by reusing a fraction p of the features "
                f"(C3, {args.headline}), p={ps[-1]} vs p={ps[0]}",
          100.0 * last["saved_vs_first"], "%", last["ms_per_snapshot"],
          {"config": {"workload": f"dynamic SBM N={args.n}, k={args.k} Zipf(1.2) blocks, degree 16, "
                                  f"ratio 0.1; d={args.d}, m={args.m}; p in {ps}",
                      "form": args.headline},
           "sweep": rows})


def run_compressive(args):
    """Full k-means against compressive k-means on the C3 features: snapshot 1 of the C3
    sequence (N=1M, k=50 Zipf blocks) through static CSC gives Theta (d=128, FP32); a step is
    one clustering of Theta, timed for both with HIP events on the current stream."""
    import math

    import numpy as np
    import torch
    from sklearn.metrics import normalized_mutual_info_score

    import paper_1706_03591_amd as csc
    from workloads import seed_for

    seq, _ = build_sequence(args, 1)
    g = seq[0]
    G = csc.Graph.from_workload(g)
    dyn = csc.DynamicCSC(args.n, args.d, args.k, args.p, args.m, seed=seed_for(3, "signals"),
                         keep_iterates=0)
    dyn.step(G)
    F = dyn.features().contiguous()
    del dyn
    ns = args.n_sample or int(math.ceil(4 * args.k * math.log(args.k)))
    seed = seed_for(3, "kmeans")

    def full():
        return csc.kmeans(F, args.k, 20, seed=seed, stream_id=2)[0]

    def comp():
        return csc.compressive_kmeans(G, F, args.k, ns, seed=seed, details=True)

    def timed(fn):
        for _ in range(args.warmup):
            out = fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            out = fn()
        e1.record()
        torch.cuda.synchronize()
        return out, e0.elapsed_time(e1) / args.steps

    lab_f, ms_f = timed(full)
    (lab_c, _, _, _, its), ms_c = timed(comp)
    lf, lc = lab_f.cpu().numpy(), lab_c.cpu().numpy()
    conf = np.zeros((args.k, args.k))
    np.add.at(conf, (lc, lf), 1)
    log(f"[bench] full k-means {ms_f:.2f} ms, compressive {ms_c:.2f} ms ({its} CG iterations)")
    _line(args, "k-means on the C3 features: compressive (sampling + Tikhonov) ms per clustering",
          ms_c, "ms", ms_c,
          {"higher_is_better": False,
           "config": {"workload": f"C3 snapshot 1 features: N={args.n}, k={args.k} Zipf(1.2) blocks, "
                                  f"d={args.d}, m={args.m}; full: k-means++ + 20 Lloyd rounds; "
                                  f"compressive: {ns} sampled nodes, 20 Lloyd rounds, r=4, "
                                  f"gamma=1e-3, PCG to 1e-6",
                      "n_sample": ns},
           "full_kmeans_ms": round(ms_f, 3), "cg_iterations": its,
           "agreement_with_full": round(float(conf.max(axis=1).sum() / args.n), 5),
           "nmi_vs_planted": {"full": round(float(normalized_mutual_info_score(g.labels, lf)), 5),
                              "compressive": round(float(normalized_mutual_info_score(g.labels, lc)), 5)}})


def run_kassign(args):
    """The k-means assignment at C5's shape (Sec. 2.1, eq. SC_cost): N = 8M BF16 rows of
    d = 256 columns against k = 200 FP32 centroids.  The rows are a seeded synthetic mixture
    (k centres of N(0, 1) entries, each row its centre plus N(0, 1) noise, rounded to BF16);
    the centroids are k rows of it.  A step is one assignment call; the whole k-means
    (k-means++ and 20 Lloyd rounds) is timed too.  The roofline compares the rows' bytes per
    call with HBM peak and the split-precision cross products with BF16 matrix-core peak."""
    import torch

    import paper_1706_03591_amd as csc

    n, d, k = args.n, args.d, args.k
    gen = torch.Generator(device="cuda").manual_seed(20171105)
    centers = torch.randn((k, d), generator=gen, device="cuda")
    lab = torch.randint(0, k, (n,), generator=gen, device="cuda")
    F = torch.empty((n, d), dtype=torch.bfloat16, device="cuda")
    for r0 in range(0, n, 1 << 20):
        r1 = min(n, r0 + (1 << 20))
        F[r0:r1] = (centers[lab[r0:r1]] + torch.randn((r1 - r0, d), generator=gen, device="cuda")).to(torch.bfloat16)
    del lab
    Cc = F[torch.randperm(n, generator=gen, device="cuda")[:k]].float().contiguous()
    # as k-means calls it: labels only (no per-row distances)
    for _ in range(args.warmup):
        csc.kmeans_assign(F, Cc, best_d2=False)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(args.steps):
        csc.kmeans_assign(F, Cc, best_d2=False)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / args.steps
    # one Lloyd update call on the labels of that assignment (the call scans max |F| for its
    # fixed-point scale each time; inside k-means that scan runs once)
    labels, _ = csc.kmeans_assign(F, Cc, best_d2=False)
    Cu = Cc.clone()
    for _ in range(args.warmup):
        csc.kmeans_update(F, labels, Cu)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(args.steps):
        csc.kmeans_update(F, labels, Cu)
    e1.record()
    torch.cuda.synchronize()
    upd_ms = e0.elapsed_time(e1) / args.steps
    t0 = time.perf_counter()
    csc.kmeans(F, k, 20, seed=7, stream_id=2)
    torch.cuda.synchronize()
    km_ms = (time.perf_counter() - t0) * 1e3
    kp = (k + 15) // 16 * 16
    flops = 2.0 * n * kp * d * 2  # the rows against the centroids' hi and mid BF16 parts
    gbps = n * d * 2 / (ms * 1e-3) / 1e9
    log(f"[bench] assignment {ms:.3f} ms ({gbps:.0f} GB/s of rows, {flops / (ms * 1e-3) / 1e12:.0f} "
        f"TFLOP/s of split products); Lloyd update call {upd_ms:.3f} ms; k-means++ + 20 Lloyd "
        f"rounds {km_ms:.1f} ms")
    _line(args, "k-means assignment at C5 shape: ms per call", ms, "ms", ms,
          {"higher_is_better": False, "dtype": "bf16 rows, fp32 centroids (split bf16 products)",
           "config": {"workload": f"synthetic BF16 mixture N={n}, d={d}, k={k}; one assignment call",
                      "n": n, "d": d, "k": k},
           "roofline": {"bound": "hbm", "kernel": "k_assign_mf (BF16 rows, two row tiles)",
                        "achieved": round(gbps, 1), "peak": PEAK_GBPS, "unit": "GB/s",
                        "frac": round(gbps / PEAK_GBPS, 4), "traffic": None,
                        "mfma_tflops": round(flops / (ms * 1e-3) / 1e12, 1),
                        "mfma_frac_bf16_dense": round(flops / (ms * 1e-3) / 2.5e15, 4)},
           "kmeans_20_lloyd_ms": round(km_ms, 2),
           "lloyd_update_call_ms": round(upd_ms, 3),
           "lloyd_update_note": "one csc_kmeans_update call on the assignment's labels, including "
                                "its scan of max |F| (4.1 GB); within k-means that scan runs once"})


def run_gather(args):
    """Ceiling of the recurrence step's neighbour gathers (csc_gather_probe: the step kernel's
    gather loop with nothing else).  On the CSR of C3's first snapshot (N = 1M, 16M entries)
    with 128-byte rows (64 binary16 or BF16 columns, the f16 step's tile), and on random
    patterns of degree 16 over 1M rows whose columns address tables of 1M or 4M rows of 64 to
    512 bytes (64 MB to 2 GB: inside and beyond the 256 MB MALL).  Rates count the requested
    bytes, nnz x row bytes.  The f16 step kernel on the same C3 CSR is timed beside it."""
    import numpy as np
    import torch

    import paper_1706_03591_amd as csc

    dev = torch.device("cuda")
    seq, _ = build_sequence(args, 1)
    g = seq[0]

    def timed(fn, reps=None):
        reps = reps or args.steps
        for _ in range(args.warmup):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps * 1e-3

    def probe(rowptr, colidx, n_table, row_bytes):
        # host-side checks of what the kernel assumes before it runs
        assert rowptr[0] == 0 and np.all(np.diff(rowptr) >= 0) and rowptr[-1] == len(colidx)
        assert colidx.min() >= 0 and colidx.max() < n_table
        rp = torch.from_numpy(rowptr.astype(np.int32)).to(dev)
        ci = torch.from_numpy(colidx.astype(np.int32)).to(dev)
        table = torch.randint(0, 1 << 30, (n_table * row_bytes // 4,), dtype=torch.int32, device=dev)
        out = torch.empty((len(rowptr) - 1) * (row_bytes // 16), dtype=torch.int32, device=dev)
        t = timed(lambda: csc.gather_probe(rp, ci, table, row_bytes, out))
        req = len(colidx) * row_bytes
        del table, out
        torch.cuda.empty_cache()
        return t, req / t / 1e12

    rows = []
    t_c3, tb_c3 = probe(g.rowptr, g.colidx, g.n, 128)
    rows.append(dict(pattern="C3 snapshot 1", n_rows=g.n, nnz=g.nnz, n_table=g.n, row_bytes=128,
                     table_mb=g.n * 128 / 2**20, us=round(t_c3 * 1e6, 1), tb_s=round(tb_c3, 3)))
    log(f"[bench] gather probe, C3 CSR, 128-byte rows: {t_c3 * 1e6:.1f} us, {tb_c3:.2f} TB/s requested")
    rng = np.random.default_rng(20171106)
    n_rows, deg = 1_000_000, 16
    rowptr = np.arange(n_rows + 1, dtype=np.int64) * deg
    for n_table in (1_000_000, 4_000_000):
        colidx = np.sort(rng.integers(0, n_table, size=(n_rows, deg)), axis=1).ravel()
        for rb in (64, 128, 256, 512):
            t, tb = probe(rowptr, colidx, n_table, rb)
            rows.append(dict(pattern="uniform random, degree 16", n_rows=n_rows, nnz=n_rows * deg,
                             n_table=n_table, row_bytes=rb, table_mb=n_table * rb / 2**20,
                             us=round(t * 1e6, 1), tb_s=round(tb, 3)))
            log(f"[bench] gather probe, random, table {n_table} x {rb} B ({n_table * rb / 2**20:.0f} MB): "
                f"{t * 1e6:.1f} us, {tb:.2f} TB/s requested")
    # the f16 step kernel on the C3 CSR (64 columns, m steps, timed by the library's events)
    G = csc.Graph.from_workload(g, val_dtype=torch.bfloat16)
    X = csc.randn(g.n, 64, 7, 1, sigma=0.125, dtype=torch.bfloat16)
    a = csc.cheb_coeffs(args.m, 2.0, 0.4)
    G.set_variant(1, torch.float16)  # one 64-column tile: 128-byte rows
    csc.cheb_filter(G, a, X, out_dtype=torch.bfloat16, iter_dtype=torch.float16)
    torch.cuda.synchronize()
    csc.timing_reset()
    csc.timing_enable(True)
    for _ in range(3):
        csc.cheb_filter(G, a, X, out_dtype=torch.bfloat16, iter_dtype=torch.float16)
    torch.cuda.synchronize()
    kms, launches, kbytes = csc.timing_read()
    csc.timing_enable(False)
    step_us = kms / launches * 1e3
    gather_req = g.nnz * 128
    step_tb = gather_req / (step_us * 1e-6) / 1e12
    log(f"[bench] f16 one-pass step on the same CSR: {step_us:.1f} us per step; its gathers alone "
        f"would take {t_c3 * 1e6:.1f} us at the probe's rate")
    # a plain 1 GiB copy, whose FETCH_SIZE / WRITE_SIZE readings calibrate the counters when
    # this workload runs under rocprofv3 --pmc
    src = torch.empty(1 << 28, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)
    torch.cuda.synchronize()
    del src, dst
    _line(args, "random-gather ceiling: requested TB/s of 128-byte neighbour rows on the C3 CSR",
          tb_c3, "TB/s", t_c3 * 1e3,
          {"config": {"workload": "csc_gather_probe on C3 snapshot 1 (N=1M, 16M entries) and random "
                                  "degree-16 patterns; tables of 64-512-byte rows",
                      "n": g.n, "nnz": g.nnz},
           "sweep": rows,
           "f16_step": {"us_per_step": round(step_us, 1), "gather_requested_tb_s": round(step_tb, 3),
                        "algorithmic_bytes_per_step": round(kbytes / launches),
                        "gather_share_of_probe_time": round(t_c3 * 1e6 / step_us, 3)}})


if __name__ == "__main__":
    main()
