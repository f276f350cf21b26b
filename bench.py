"""Benchmark of the sparsified-NetMF hot path on one MI355X.

One step = one full embedding (sparsifier -> trunc_log -> fast randomized SVD
-> Chebyshev propagation) of the workload, inputs resident in HBM, through the
C ABI (lne_embed).  Prints ONE JSON line.

  value            accepted PathSampling samples per second of whole step
  roofline         dominant kernel: algorithmic bytes per launch / average
                   launch time (HIP events on the library stream, timed region)
  cpu_baseline     the oracle (plain C sampler + aggregator) on a bounded edge
                   sample of the same workload, on the host cores
"""
from __future__ import annotations

import argparse
import json
import math
import os
import subprocess
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def kernel_bytes(name, ctx_info):
    """Algorithmic HBM bytes of one launch of `name` (per-unit figure x units).

    Both sparse x dense products use the gather model: row offsets, 8 bytes
    of structure per nonzero, one gathered k-wide dense row per nonzero and
    two n x k dense streams (operand in, product out),
        B_gather = 8 (n + 1) + 8 nnz + e k nnz + 2 e n k,
    with e the element size: the rSVD product at k = k' over the nonzeros of
    the sparsified matrix, the propagation product at k = d over the graph's
    arcs.  The epilogue streams the recurrence adds to some propagation
    launches are not counted here (`graph_spmm_streams` reports them)."""
    n, nnz_M, kp, arcs, d, P = (ctx_info[k] for k in ("n", "nnz_M", "kp", "arcs", "d", "pairs"))
    es = ctx_info["es"]
    if name == "spmm":
        return 8 * (n + 1) + 8 * nnz_M + es * kp * nnz_M + 2 * es * n * kp
    if name == "graph_spmm":
        return 8 * (n + 1) + 8 * arcs + es * d * arcs + 2 * es * n * d
    if name == "radix_scatter":
        # read and write (key, weight) per item, plus the per-tile digit counts
        # and offsets
        return P * (8 + 4) * 2 + (P // 4096 + 1) * 256 * 12
    if name == "radix_hist":
        return P * 8
    if name == "sym_merge":
        # row offsets of both triangles, the upper triangle's (col, value) and
        # the lower's (key, value) per entry read, (col, value) written
        return 24 * (n + 1) + ctx_info["nnz_counts"] * (8 + 12 + 8) // 2
    if name == "reduce_trunc_log":
        # (key, weight) per item read, (column, value) per distinct pair
        # written, row offsets
        return P * 12 + ctx_info["nnz_counts"] * (4 + es) + 8 * (n + 1)
    return None


def graph_spmm_streams(K):
    """Dense n x d streams the Chebyshev recurrence of order K moves per
    propagation, launch by launch.  Every term runs Z = B T (T in, Z out: 2
    streams) and then the term's update with the accumulator (Z, the two
    earlier terms and the accumulator in, the new term and the accumulator
    out: 6; the first term has one earlier term and starts the accumulator
    without reading it: 4); the final D^-1 A product adds 2.  Returns
    (launches, streams)."""
    if K <= 0:
        return 0, 0
    return 2 * K + 1, 2 + 4 + 8 * (K - 1) + 2


# Counter summary of the dominant kernels (profiles/): FETCH_SIZE and
# WRITE_SIZE per launch and the calibration factors of a plain copy.
COUNTERS = os.path.join(ROOT, "profiles", "counters_large.json")
KERNEL_SOURCE = {"spmm": "k_spmm.hip", "graph_spmm": "k_spmm.hip",
                 "radix_scatter": "k_sort.hip", "radix_hist": "k_sort.hip",
                 "reduce_trunc_log": "k_sort.hip"}


# Library kernels by the name bench.py and the counter summary use: a pattern
# on the (demangled) kernel name and the source file that defines it.
KERNEL_CLASSES = {
    "spmm": (r"\bk_spmm<", "k_spmm.hip"),
    "graph_spmm": (r"\bk_graph_spmm<", "k_spmm.hip"),
    "radix_scatter": (r"\bk_scatter\b", "k_sort.hip"),
    "radix_hist": (r"\bk_hist\b", "k_sort.hip"),
    "reduce_trunc_log": (r"\bk_reduce_tl\b", "k_sort.hip"),
    "sym_merge": (r"\bk_sym_merge\b", "k_sort.hip"),
    "sample_count": (r"\bk_sample_count<", "k_sample.hip"),
    "sample_emit": (r"\bk_sample_emit<", "k_sample.hip"),
}


def _rocprof_files(root, suffix):
    out = []
    for d, _, files in os.walk(root):
        out += [os.path.join(d, f) for f in files if f.endswith(suffix)]
    return sorted(out)


def _col(row, *names):
    """Value of the first of `names` present in a csv row (case-insensitive)."""
    low = {k.lower(): v for k, v in row.items() if k}
    for nm in names:
        if nm.lower() in low:
            return low[nm.lower()]
    raise KeyError(names)


def _short_name(name):
    """Kernel name without namespaces, return type and argument list."""
    import re
    name = re.sub(r"^void\s+", "", name).replace("(anonymous namespace)::", "")
    depth, cut = 0, len(name)
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            cut = i
            break
    name = name[:cut]
    return re.sub(r"^(?:\w+::)+", "", name)


def summarize_kernel_trace(root, steps, title, command):
    """Markdown table of a `rocprofv3 --kernel-trace --stats` run: calls,
    average and per-step milliseconds and share of every kernel, from its
    kernel_stats.csv (or, without one, from the kernel trace itself)."""
    import csv
    rows = {}
    stats = _rocprof_files(root, "kernel_stats.csv")
    if stats:
        for path in stats:
            with open(path, newline="") as f:
                for r in csv.DictReader(f):
                    nm = _short_name(_col(r, "Name", "Kernel_Name", "KernelName"))
                    calls = int(float(_col(r, "Calls")))
                    tot = float(_col(r, "TotalDurationNs", "Total_Duration_Ns"))
                    c0, t0 = rows.get(nm, (0, 0.0))
                    rows[nm] = (c0 + calls, t0 + tot)
    else:
        for path in _rocprof_files(root, "kernel_trace.csv"):
            with open(path, newline="") as f:
                for r in csv.DictReader(f):
                    nm = _short_name(_col(r, "Kernel_Name", "KernelName", "Name"))
                    dt = float(_col(r, "End_Timestamp")) - float(_col(r, "Start_Timestamp"))
                    c0, t0 = rows.get(nm, (0, 0.0))
                    rows[nm] = (c0 + 1, t0 + dt)
    if not rows:
        raise SystemExit(f"no kernel_stats.csv or kernel_trace.csv under {root}")
    total = sum(t for _, t in rows.values())
    lines = [f"# {title}", "", f"Command (from the repository root, `TMPDIR=/tmp`): `{command}`",
             "", f"Per-step figures divide the totals by {steps} (the embedding steps the "
             "profiled command ran, warm-up included).", "",
             "| kernel | calls | avg ms | ms per step | share |", "|---|---|---|---|---|"]
    for nm, (calls, tot) in sorted(rows.items(), key=lambda kv: -kv[1][1]):
        if tot / total < 0.001:
            continue
        lines.append(f"| `{nm[:90]}` | {calls} | {tot / calls / 1e6:.3f} | "
                     f"{tot / steps / 1e6:.1f} | {100 * tot / total:.1f}% |")
    return "\n".join(lines) + "\n"


def summarize_counters(fetch_root, write_root, calib_bytes, workload, commands):
    """FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the library kernels
    from two `rocprofv3 --pmc` runs, averaged per launch of each kernel class,
    with the calibration factors of the largest plain device copy
    (`calib_bytes` long) that the runs made, and the sha256 of each kernel's
    source so that a changed kernel invalidates its figures."""
    import csv
    import hashlib
    import re

    def per_dispatch(root, counter):
        """[(dispatch id, kernel name, counter value)] in dispatch order."""
        vals = {}
        for path in _rocprof_files(root, "counter_collection.csv"):
            with open(path, newline="") as f:
                for r in csv.DictReader(f):
                    if _col(r, "Counter_Name") != counter:
                        continue
                    did = int(float(_col(r, "Dispatch_Id", "Correlation_Id")))
                    key = (path, did)
                    nm = _col(r, "Kernel_Name", "KernelName")
                    v = float(_col(r, "Counter_Value"))
                    vals[key] = (did, nm, vals.get(key, (did, nm, 0.0))[2] + v)
        return sorted(vals.values())

    out = {"workload": workload, "commands": commands, "kernels": {}}
    factors = {}
    for counter, root in (("FETCH_SIZE", fetch_root), ("WRITE_SIZE", write_root)):
        disp = [(nm, v) for _, nm, v in per_dispatch(root, counter)]
        # the calibration: bench.py --calib-copy-mib copies the buffer three
        # times before any other device copy of the run
        copies = [v for nm, v in disp if "copyBuffer" in nm][:3]
        if len(copies) < 3:
            raise SystemExit(f"no calibration copies in the {counter} run (use --calib-copy-mib)")
        factors[counter] = calib_bytes / (sorted(copies)[1] * 1024.0)
        for cls, (pat, src) in KERNEL_CLASSES.items():
            v = [x for nm, x in disp if re.search(pat, nm)]
            if not v:
                continue
            ent = out["kernels"].setdefault(cls, {"source": src})
            ent["launches"] = len(v)
            ent[("fetch" if counter == "FETCH_SIZE" else "write") + "_kib_per_launch"] = \
                sum(v) / len(v)
    out["fetch_factor"] = factors["FETCH_SIZE"]
    out["write_factor"] = factors["WRITE_SIZE"]
    out["calibration"] = (f"median of the run's first three device copies ({calib_bytes} bytes "
                          f"each)")
    for ent in out["kernels"].values():
        with open(os.path.join(ROOT, "paper_2302_07084_amd", "csrc", ent["source"]), "rb") as f:
            ent["source_sha256"] = hashlib.sha256(f.read()).hexdigest()
    return out


def counters_markdown(summ, title):
    lines = [f"# {title}", "", "Commands: " + " and ".join(f"`{c}`" for c in summ["commands"]) +
             " (one counter per run).", "",
             f"Calibration: {summ['calibration']} -> read factor {summ['fetch_factor']:.3f}, "
             f"write factor {summ['write_factor']:.3f}.", "",
             "| kernel | launches | FETCH KiB/launch | WRITE KiB/launch | HBM bytes/launch "
             "(calibrated) |", "|---|---|---|---|---|"]
    for cls, e in summ["kernels"].items():
        fk, wk = e.get("fetch_kib_per_launch", 0.0), e.get("write_kib_per_launch", 0.0)
        tot = (fk * summ["fetch_factor"] + wk * summ["write_factor"]) * 1024
        lines.append(f"| `{cls}` | {e['launches']} | {fk:,.0f} | {wk:,.0f} | {tot / 1e9:,.1f} GB |")
    return "\n".join(lines) + "\n"


def measured_traffic(name):
    """HBM bytes per launch of `name` from the committed counter summary, or
    None when there is none or the kernel source changed since it was taken."""
    import hashlib
    try:
        with open(COUNTERS) as f:
            summ = json.load(f)
        ent = summ["kernels"][name]
        src = os.path.join(ROOT, "paper_2302_07084_amd", "csrc", ent["source"])
        with open(src, "rb") as f:
            if hashlib.sha256(f.read()).hexdigest() != ent["source_sha256"]:
                return None
        return (ent["fetch_kib_per_launch"] * summ["fetch_factor"] +
                ent["write_kib_per_launch"] * summ["write_factor"]) * 1024.0
    except (OSError, KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="large")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--report", choices=["precision", "automl", "mfma", "linkpred", "weighted",
                                         "ablation", "host", "hbm"],
                    default=None,
                    help="precision: the FP32 and BF16-MFMA paths against the FP64 path; "
                         "automl: trials/s and time to an equal score of the plain "
                         "sequential search and the batched surrogate search; mfma: "
                         "achieved matrix-core rate of the dense rSVD steps; linkpred: "
                         "held-out edges ranked against corrupted ones (MR, MRR, HITS@10, "
                         "AUC) and the ranking kernel's rate; weighted: the embedding step on "
                         "the workload's graph with integer weights beside the unweighted one; "
                         "ablation: stage times and micro-F1 of the vanilla and fast randomized "
                         "SVD (q = 1, 2, 5) over sample sizes; host: the embedding step with "
                         "the sparsifier in pinned host memory (streamed over PCIe) beside "
                         "the in-HBM step; hbm: the rates of plain device copies, fills and "
                         "sums of 4 GiB (the practical streaming ceiling beside the 8 TB/s "
                         "peak)")
    ap.add_argument("--flags", type=int, default=0,
                    help="extra LNE_FLAG_* bits for the timed step (default 0: the paper's "
                         "method; 4 = sparse-sign test matrix, 2 = vanilla randomized SVD)")
    ap.add_argument("--relabel", type=int, default=None,
                    help="permute the workload's vertex ids with this seed first (the "
                         "generators number vertices in degree order; real graphs do not)")
    ap.add_argument("--automl-trials", type=int, default=64)
    ap.add_argument("--automl-seeds", type=int, default=3,
                    help="independent repetitions of the AutoML report (95%% intervals)")
    ap.add_argument("--pretrain-trials", type=int, default=64,
                    help="surrogate pretraining trials per family graph (8 graphs)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run a plain device copy of this size first (counter calibration)")
    ap.add_argument("--summarize-trace", metavar="DIR", default=None,
                    help="print a markdown summary of a rocprofv3 --kernel-trace --stats "
                         "output directory (no GPU work)")
    ap.add_argument("--summarize-counters", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    default=None,
                    help="summarise two rocprofv3 --pmc runs (FETCH_SIZE, then WRITE_SIZE) "
                         "into the counter JSON that the roofline's traffic field reads "
                         "(no GPU work; --calib-copy-mib gives the calibration copy's size)")
    ap.add_argument("--summary-steps", type=int, default=1,
                    help="embedding steps the profiled command ran (per-step figures)")
    ap.add_argument("--summary-title", default="Kernel time")
    ap.add_argument("--summary-command", action="append", default=[],
                    help="the profiled command, recorded in the summary (repeatable)")
    ap.add_argument("--summary-out", default=None,
                    help="write the summary here (markdown; .json for --summarize-counters "
                         "also writes a .md beside it)")
    args = ap.parse_args()
    if args.summarize_trace:
        text = summarize_kernel_trace(args.summarize_trace, args.summary_steps,
                                      args.summary_title, " && ".join(args.summary_command))
        if args.summary_out:
            with open(args.summary_out, "w") as f:
                f.write(text)
        print(text)
        return
    if args.summarize_counters:
        summ = summarize_counters(args.summarize_counters[0], args.summarize_counters[1],
                                  args.calib_copy_mib << 20, args.workload, args.summary_command)
        md = counters_markdown(summ, args.summary_title)
        if args.summary_out:
            with open(args.summary_out, "w") as f:
                json.dump(summ, f, indent=1)
            with open(os.path.splitext(args.summary_out)[0] + ".md", "w") as f:
                f.write(md)
        print(md)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_2302_07084_amd as lne
    from synth import workload

    if args.report == "precision":
        precision_report(args.workload if args.workload != "large" else "precision")
        return
    if args.report == "mfma":
        mfma_report()
        return
    if args.report == "automl":
        automl_report(args.workload if args.workload != "large" else "batched",
                      args.automl_trials, args.pretrain_trials, args.automl_seeds)
        return
    if args.report == "linkpred":
        linkpred_report(args.workload)
        return
    if args.report == "weighted":
        weighted_report(args.workload, seconds=args.cpu_seconds)
        return
    if args.report == "ablation":
        ablation_report(args.workload if args.workload != "large" else "batched")
        return
    if args.report == "hbm":
        hbm_report()
        return
    if args.report == "host":
        host_report(args.workload)
        return

    if args.calib_copy_mib:
        # a plain copy of known size: its FETCH_SIZE / WRITE_SIZE counters
        # calibrate the counters of the library kernels
        nb = args.calib_copy_mib << 20
        src = torch.ones(nb // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        log(f"calibration copy of {nb} bytes done")
        del src, dst

    t0 = time.time()
    log(f"generating workload '{args.workload}'")
    g, p = workload(args.workload, device="cuda")
    if args.relabel is not None:
        from synth import relabel
        g = relabel(g, args.relabel, device="cuda")
    if args.flags:
        p = dict(p, flags=int(p.get("flags", 0)) | args.flags)
    log(f"graph n={g.n} m={g.m} in {time.time() - t0:.1f}s; params T={p['T']} M={p['M']} "
        f"d={p['d']} q={p['q']} precision={p['precision']}")
    rp = torch.from_numpy(g.rowptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    torch.cuda.synchronize()

    ctx = lne.Context()
    X = torch.empty((g.n, p["d"]), dtype=torch.float64 if p["precision"] == "f64" else torch.float32,
                    device="cuda")
    stats = None
    for i in range(args.warmup):
        _, stats = lne.embed(ctx, rp, col, p, out=X)
        torch.cuda.synchronize()
        log(f"warmup {i} done: {stats}")

    ctx.prof_enable(True)
    ctx.prof_reset()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        _, stats = lne.embed(ctx, rp, col, p, out=X)
        log(f"step {i} enqueued")
    torch.cuda.synchronize()
    t_end = time.perf_counter()
    ms_per_step = (t_end - t_start) * 1e3 / args.steps
    log(f"timed {args.steps} steps: {ms_per_step:.1f} ms/step")

    names = ["validate_graph", "row_up", "fill_edges", "sample_count", "fold_stats", "sample_emit", "scan",
             "radix_hist", "radix_scatter", "heads", "reduce", "degrees", "reduce_trunc_log", "drop_zeros",
             "rowptr_tail", "concat_rows", "trunc_log_count", "trunc_log_fill", "gaussian",
             "sparse_omega", "spmm_sparse_omega", "weight_check", "weight_guide",
             "spmm", "gram", "gram_reduce", "chol_inv", "project", "sym_eig", "eig_weights",
             "w_to_bf16", "graph_spmm", "dense_scale", "axpby", "sym_bounds", "sym_rowlen",
             "sym_merge"]
    prof = {}
    for nm in names:
        ms, cnt = ctx.prof_get(nm)
        if cnt:
            prof[nm] = {"ms_per_step": ms / args.steps, "launches_per_step": cnt / args.steps,
                        "avg_ms": ms / cnt}
    ctx.prof_enable(False)

    kp = p["d"] + p["oversample"]
    es = 8 if p["precision"] == "f64" else 4
    info = dict(n=g.n, nnz_M=stats["nnz_log"], kp=kp, arcs=g.n_arcs, d=p["d"],
                pairs=stats["entries"], es=es, nnz_counts=stats["nnz_counts"])
    dominant = max(prof, key=lambda k: prof[k]["ms_per_step"])
    rl_name = dominant if kernel_bytes(dominant, info) is not None else "spmm"
    nbytes = kernel_bytes(rl_name, info)
    # the counters were taken on the generator's vertex order
    traffic = measured_traffic(rl_name) if args.relabel is None else None
    # achieved rate: the algorithmic bytes, or the measured HBM bytes where
    # the caches served part of them (min of the two), over the launch time
    counted = min(nbytes, traffic) if traffic else nbytes
    achieved = counted / (prof[rl_name]["avg_ms"] * 1e-3) / 1e9
    spmm_gbs = kernel_bytes("spmm", info) / (prof["spmm"]["avg_ms"] * 1e-3) / 1e9
    spmm_min = (8 * (g.n + 1) + 8 * stats["nnz_log"] + 2 * es * g.n * kp) / (prof["spmm"]["avg_ms"] * 1e-3) / 1e9
    gsp = None
    if "graph_spmm" in prof:
        launches, streams = graph_spmm_streams(p["cheb_k"])
        # the gather model plus the epilogue streams each launch really moves
        # (on average over the propagation's launches)
        b_streams = (kernel_bytes("graph_spmm", info) - 2 * es * g.n * p["d"]
                     + streams / launches * es * g.n * p["d"])
        gsp = {"bytes_gather_model": kernel_bytes("graph_spmm", info),
               "bytes_with_epilogue_streams": b_streams,
               "streams_per_launch": streams / launches,
               "avg_launch_ms": prof["graph_spmm"]["avg_ms"],
               "gbs_gather_model": kernel_bytes("graph_spmm", info) / (prof["graph_spmm"]["avg_ms"] * 1e-3) / 1e9,
               "gbs_with_epilogue_streams": b_streams / (prof["graph_spmm"]["avg_ms"] * 1e-3) / 1e9}
    sampler_ms = sum(prof.get(k, {}).get("ms_per_step", 0.0) for k in ("sample_count", "sample_emit"))
    # the sparsifier stage: sampling, the pair sort and the aggregation with
    # Eq. (1) fused (the embedding builds no separate count matrix)
    sparsifier_ms = sum(prof.get(k, {}).get("ms_per_step", 0.0) for k in (
        "validate_graph", "row_up", "fill_edges", "sample_count", "fold_stats", "sample_emit",
        "scan", "radix_hist", "radix_scatter", "heads", "reduce", "degrees", "reduce_trunc_log",
        "drop_zeros", "rowptr_tail", "concat_rows", "sym_bounds", "sym_rowlen", "sym_merge"))

    value = stats["accepted"] / (ms_per_step * 1e-3)
    out = {
        "metric": "sampled edges/s (accepted PathSampling samples per second of the whole "
                  "embedding step) + rSVD SpMM GB/s vs HBM peak",
        "value": value,
        "unit": "sampled edges/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if p["precision"] != "f64" else "f64",
        "data": "synthetic (seeded generator)",
        "config": {"workload": f"{args.workload}: Chung-Lu power-law n={g.n} m={g.m} "
                               f"gamma=2.1, T={p['T']}, s={list(map(float, p['s']))}, "
                               f"M={p['M']} (4Tm), d={p['d']}, q={p['q']}, k={p['cheb_k']}",
                   "n": g.n, "m": g.m, "T": p["T"], "M": p["M"], "d": p["d"],
                   "oversample": p["oversample"], "q": p["q"], "precision": p["precision"],
                   "flags": int(p.get("flags", 0)), "relabel": args.relabel,
                   "parallelism": "single GPU"},
        "roofline": {"kernel": rl_name, "bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "bytes_per_launch": nbytes, "bytes_counted": counted,
                     "avg_launch_ms": prof[rl_name]["avg_ms"],
                     "model": "gather: 8(n+1) + 8 nnz + e k nnz + 2 e n k; achieved = "
                              "min(model, traffic) / average launch time"},
        "graph_spmm": gsp,
        "stats": stats,
        "sampler_edges_per_s": stats["accepted"] / (sampler_ms * 1e-3) if sampler_ms else None,
        "gpu_same_scope": {"value": stats["accepted"] / (sparsifier_ms * 1e-3) if sparsifier_ms else None,
                           "unit": "sampled edges/s (sampling + aggregation stages)",
                           "ms_per_step": sparsifier_ms},
        "attempted_samples_per_s": stats["attempted"] / (ms_per_step * 1e-3),
        "spmm_gbs_gather_model": spmm_gbs,
        "spmm_gbs_min_model": spmm_min,
        "spmm_frac_hbm_peak": spmm_gbs / HBM_PEAK_GBS,
        "kernels": prof,
    }

    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(g, p, args.cpu_seconds)
    print(json.dumps(out), flush=True)


def _principal_angle(A, B):
    import numpy as np
    qa, _ = np.linalg.qr(A)
    qb, _ = np.linalg.qr(B)
    r = qb - qa @ (qa.T @ qb)
    return float(np.arcsin(min(1.0, np.linalg.norm(r, 2))))


def _procrustes(X, Xref):
    import numpy as np
    U, _, Vt = np.linalg.svd(X.T @ Xref)
    return float(np.linalg.norm(X @ (U @ Vt) - Xref) / np.linalg.norm(Xref))


def ablation_report(name, mults=(0.077, 1, 5, 10, 50, 100)):
    """Stage times and accuracy of the randomized-SVD variants over sample
    sizes on a labelled graph, the shape of the paper's running-time table and
    its power-iteration ablation: the vanilla randomized SVD (q = 1) and the
    fast one with q = 1, 2, 5, each at M = mult T m.  The embedding step is
    timed whole (fused aggregation); the rSVD and the propagation are timed
    again on their own, and the sparsifier stage is the remainder.  Accuracy:
    micro-F1 of one-vs-rest logistic regression on the GPU, 10% training
    labels, 3 seeded splits."""
    import numpy as np
    import torch

    import paper_2302_07084_amd as lne
    from paper_2302_07084_amd import search
    from synth import workload

    g, p = workload(name, device="cuda")
    ctx = lne.Context()
    task = search.Task.make(ctx, g, p, train_ratio=0.1, n_splits=3, seed=7)
    variants = (("vanilla rSVD, q=1", 1, lne.FLAG_VANILLA_RSVD), ("fast rSVD, q=1", 1, 0),
                ("fast rSVD, q=2", 2, 0), ("fast rSVD, q=5", 5, 0),
                ("fast rSVD, q=1, sparse-sign Omega", 1, lne.FLAG_SPARSE_OMEGA),
                ("fast rSVD, q=2, sparse-sign Omega", 2, lne.FLAG_SPARSE_OMEGA))
    out = {"report": "ablation", "workload": name, "n": g.n, "m": g.m, "T": p["T"], "d": p["d"],
           "oversample": p["oversample"], "cheb_k": p["cheb_k"], "precision": p["precision"],
           "scoring": "one-vs-rest logistic regression on GPU, 10% training labels, 3 splits, "
                      "micro-F1", "rows": []}

    def sync_time(fn):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fn()
        torch.cuda.synchronize()
        return r, time.perf_counter() - t0

    for mult in mults:
        M = int(round(mult * p["T"] * g.m))
        for label, q, flags in variants:
            pp = dict(p, M=M, q=q, flags=flags)
            lne.embed(ctx, task.rp, task.col, pp)                 # warm-up (tuning)
            (X, st), t_embed = sync_time(lambda: lne.embed(ctx, task.rp, task.col, pp))
            f1 = float(np.mean([lne.score_micro_f1(ctx, X, task.labels, tr, te)
                                for tr, te in task.splits]))
            counts, _ = lne.sparsify(ctx, task.rp, task.col, pp)
            Mm = lne.trunc_log(ctx, task.rp, task.col, pp, counts)
            counts.free()
            lne.rsvd(ctx, Mm, pp, want=("X0",))
            (_, _, _, X0), t_rsvd = sync_time(lambda: lne.rsvd(ctx, Mm, pp, want=("X0",)))
            Mm.free()
            _, t_prop = sync_time(lambda: lne.propagate(ctx, task.rp, task.col, pp, X0))
            row = {"variant": label, "M_over_Tm": mult, "M": M, "q": q,
                   "accepted": st["accepted"], "nnz": st["nnz_log"], "seconds": t_embed,
                   "sparsifier_s": max(t_embed - t_rsvd - t_prop, 0.0), "rsvd_s": t_rsvd,
                   "propagation_s": t_prop, "micro_f1": f1}
            out["rows"].append(row)
            log(f"ablation: M={mult}Tm {label}: {t_embed:.3f}s (rsvd {t_rsvd:.3f}s) F1 {f1:.4f}")
            del X, X0
    print(json.dumps(out), flush=True)


def weighted_report(name, wmax=16, steps=2, seconds=15.0):
    """The whole embedding step (sparsify, truncated log, rSVD, propagation) on
    the workload's graph with symmetric integer weights 1..wmax (a hash of
    each pair) beside the same step unweighted, in one process: sampled edges
    per second, the per-kernel time of each, and the weighted oracle's sampler
    and aggregator on a bounded block of the same edges (host cores)."""
    import numpy as np
    import torch

    import paper_2302_07084_amd as lne
    from synth import Graph, pair_weights, workload

    g, p = workload(name, device="cuda")
    w = pair_weights(g, wmax, seed=int(p["seed"]) + 1, device="cuda")
    log(f"weighted: '{name}' n={g.n} m={g.m}, weights 1..{wmax}, vol {int(w.sum(dtype=np.uint64))}")
    rp = torch.from_numpy(g.rowptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    wd = torch.from_numpy(w.astype(np.int32)).cuda()
    ctx = lne.Context()
    X = torch.empty((g.n, p["d"]), dtype=torch.float32, device="cuda")
    out = {"report": "weighted", "workload": name, "n": g.n, "m": g.m, "weights": f"1..{wmax}",
           "T": p["T"], "M": p["M"], "d": p["d"], "precision": p["precision"], "runs": {}}
    for label, weight in (("unweighted", None), ("weighted", wd)):
        _, st = lne.embed(ctx, rp, col, p, out=X, weight=weight)      # warm-up, tuning
        torch.cuda.synchronize()
        ctx.prof_enable(True)
        ctx.prof_reset()
        t0 = time.perf_counter()
        for _ in range(steps):
            _, st = lne.embed(ctx, rp, col, p, out=X, weight=weight)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        ker = {}
        for nm in ("sample_count", "sample_emit", "radix_scatter", "reduce_trunc_log", "spmm",
                   "graph_spmm", "weight_check", "weight_guide"):
            ms, cnt = ctx.prof_get(nm)
            if cnt:
                ker[nm] = ms / steps
        ctx.prof_enable(False)
        out["runs"][label] = {"ms_per_step": dt * 1e3, "sampled_edges_per_s": st["accepted"] / dt,
                              "accepted": st["accepted"], "nnz_log": st["nnz_log"],
                              "kernels_ms_per_step": ker}
        log(f"weighted: {label} {dt * 1e3:.1f} ms/step, {st['accepted'] / dt:.3g} sampled edges/s")
    gw = Graph(g.n, g.rowptr, g.col, None, name + "-w", w)
    out["cpu_baseline"] = cpu_baseline(gw, p, seconds)
    print(json.dumps(out), flush=True)


def host_report(name, steps=2):
    """The embedding step with the sparsified matrix kept in pinned host
    memory (the path for graphs whose sparsifier exceeds HBM: its row chunks
    stream over PCIe for each of the q + 1 products of the randomized SVD)
    beside the same step with the matrix in HBM; both give the same
    embedding bit for bit (checked here).  Reports ms per step, the bytes
    moved over PCIe per step (the matrix once to the host, q + 1 times back)
    and their rate counted over the extra time plus the in-HBM products'."""
    import torch

    import paper_2302_07084_amd as lne
    from synth import workload

    g, p = workload(name, device="cuda")
    rp = torch.from_numpy(g.rowptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    ctx = lne.Context()
    out = {"report": "host", "workload": name, "n": g.n, "m": g.m, "T": p["T"], "M": p["M"],
           "d": p["d"], "q": p["q"], "precision": p["precision"], "runs": {}}
    Xs = {}
    for label, flags in (("hbm", 0), ("host", lne.FLAG_HOST_SPARSIFIER)):
        pp = dict(p, flags=flags)
        X, st = lne.embed(ctx, rp, col, pp)                 # warm-up, tuning
        torch.cuda.synchronize()
        ctx.prof_enable(True)
        ctx.prof_reset()
        t0 = time.perf_counter()
        for _ in range(steps):
            X, st = lne.embed(ctx, rp, col, pp, out=X)
        torch.cuda.synchronize()
        dt = (time.perf_counter() - t0) / steps
        spmm_ms, cnt = ctx.prof_get("spmm")
        ctx.prof_enable(False)
        Xs[label] = X
        out["runs"][label] = {"ms_per_step": dt * 1e3, "sampled_edges_per_s": st["accepted"] / dt,
                              "nnz_log": st["nnz_log"], "spmm_ms_per_step": spmm_ms / steps}
        log(f"host: {label} {dt * 1e3:.1f} ms/step (spmm {spmm_ms / steps:.1f} ms), "
            f"nnz {st['nnz_log']}")
    nnz = out["runs"]["host"]["nnz_log"]
    es = 8 if p["precision"] == "f64" else 4
    matrix = nnz * (4 + es) + 8 * (g.n + 1)
    moved = matrix * (1 + p["q"] + 1)
    extra = (out["runs"]["host"]["ms_per_step"] - out["runs"]["hbm"]["ms_per_step"]
             + out["runs"]["hbm"]["spmm_ms_per_step"]) * 1e-3
    out["matrix_bytes"] = matrix
    out["pcie_bytes_per_step"] = moved
    out["pcie_gb_per_s"] = moved / extra / 1e9 if extra > 0 else None
    out["bit_identical"] = bool((Xs["host"] == Xs["hbm"]).all())
    log(f"host: {moved / 1e9:.1f} GB over PCIe per step, {out['pcie_gb_per_s']} GB/s effective, "
        f"identical {out['bit_identical']}")
    print(json.dumps(out), flush=True)


def linkpred_report(name, held_out=10_000, K=1000, hits_k=10, oracle_edges=500):
    """Link-prediction evaluation, the protocol of the paper's very-large-graph
    runs: hold out edges, embed the training graph with T = 2, d = 32 and no
    spectral propagation, and rank every held-out edge against K corrupted
    edges (uniform destinations).  Reports MR / MRR / HITS@10 / AUC of the
    embedding and of a random one, the embedding time, the ranking kernel's
    time and gather rate, and the oracle's ranking of a sample of the edges
    (timed on the host, checked against the kernel's counts)."""
    import numpy as np
    import torch

    import paper_2302_07084_amd as lne
    from oracle import linkpred
    from synth import workload, holdout_edges, corrupt_destinations

    g, p = workload(name, device="cuda")
    t0 = time.perf_counter()
    train, pos = holdout_edges(g, held_out, seed=31)
    neg = corrupt_destinations(pos, g.n, K, seed=32)
    t_split = time.perf_counter() - t0
    n, m = g.n, g.m
    del g
    log(f"linkpred: '{name}' n={n} m={m}, {held_out} held-out edges x {K} corrupted "
        f"(split {t_split:.1f}s)")
    rp = torch.from_numpy(train.rowptr).cuda()
    col = torch.from_numpy(train.col).cuda()
    pp = dict(p, T=2, s=[0.5, 0.5], d=32, cheb_k=0, precision="f32",
              M=int(round(p["M"] / (p["T"] * m) * 2 * train.m)))
    ctx = lne.Context()
    X, st = lne.embed(ctx, rp, col, pp)            # warm-up (launch-shape tuning)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    X, st = lne.embed(ctx, rp, col, pp)
    torch.cuda.synchronize()
    t_embed = time.perf_counter() - t0
    pd = torch.from_numpy(pos).cuda()
    nd = torch.from_numpy(neg).cuda()
    lne.link_rank(ctx, X, pd, nd, hits_k)           # warm-up
    ctx.prof_enable(True)
    ctx.prof_reset()
    reps = 5
    for _ in range(reps):
        met, above, ties = lne.link_rank(ctx, X, pd, nd, hits_k)
    ms, cnt = ctx.prof_get("link_rank")
    ctx.prof_enable(False)
    ms_rank = ms / cnt
    torch.manual_seed(0)
    met_rand, _, _ = lne.link_rank(ctx, torch.randn_like(X), pd, nd, hits_k)
    # algorithmic bytes: every scored row once (h (K + 1) + h rows of d floats)
    # plus the corrupted ids
    d = X.shape[1]
    bytes_launch = held_out * (K + 2) * d * 4 + held_out * K * 4 + held_out * 8
    # the oracle beside it, on the first edges
    Xh = X.double().cpu().numpy()
    t0 = time.perf_counter()
    _, oa, ot = linkpred.link_metrics(Xh, pos[:oracle_edges], neg[:oracle_edges], hits_k)
    t_oracle = time.perf_counter() - t0
    agree = bool(np.array_equal(above[:oracle_edges].cpu().numpy(), oa) and
                 np.array_equal(ties[:oracle_edges].cpu().numpy(), ot))
    out = {"report": "linkpred", "workload": name, "n": n, "m": m, "train_m": train.m,
           "held_out": held_out, "corrupted_per_edge": K, "T": 2, "d": d,
           "M": pp["M"], "propagation": False, "embed_seconds": t_embed,
           "accepted_samples": st["accepted"], "metrics": met, "random_embedding": met_rand,
           "rank_kernel": {"ms": ms_rank, "scored_pairs_per_s": held_out * (K + 1) / (ms_rank / 1e3),
                           "gbs_gather_model": bytes_launch / (ms_rank / 1e3) / 1e9,
                           "frac_hbm_peak": bytes_launch / (ms_rank / 1e3) / 8e12},
           "oracle": {"edges": oracle_edges, "seconds": t_oracle,
                      "scored_pairs_per_s": oracle_edges * (K + 1) / t_oracle,
                      "counts_equal_kernel": agree}}
    log(f"linkpred: embed {t_embed:.2f}s, rank {ms_rank:.3f} ms; MRR {met['mrr']:.4f} "
        f"(random {met_rand['mrr']:.4f}), AUC {met['auc']:.4f}; oracle agrees: {agree}")
    print(json.dumps(out), flush=True)


def precision_report(name):
    """Runs the workload's sparsifier, fast randomized SVD and propagation in
    FP64, FP32 and BF16 (dense rSVD steps on BF16 MFMA, FP64 Cholesky and
    eigen-solves) and reports each result's error against the FP64 run."""
    import numpy as np
    import torch

    import paper_2302_07084_amd as lne
    from synth import workload

    g, p = workload(name, device="cuda")
    log(f"precision report on '{name}': n={g.n} m={g.m} M={p['M']} d={p['d']} q={p['q']}")
    rp = torch.from_numpy(g.rowptr).cuda()
    col = torch.from_numpy(g.col).cuda()
    ctx = lne.Context()
    res = {}
    for prec in ("f64", "f32", "bf16"):
        pp = dict(p, precision=prec)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        counts, st = lne.sparsify(ctx, rp, col, pp)
        M = lne.trunc_log(ctx, rp, col, pp, counts)
        counts.free()
        torch.cuda.synchronize()
        t_sp = time.perf_counter() - t0
        # untimed warm-ups: the launch-shape tuner times every SpMM variant on
        # the first product of a new shape
        lne.rsvd(ctx, M, dict(pp, q=1), want=("S",))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        U, S, V, X0 = lne.rsvd(ctx, M, pp)
        torch.cuda.synchronize()
        t_rs = time.perf_counter() - t0
        nnz = M.nnz
        M.free()
        lne.propagate(ctx, rp, col, dict(pp, cheb_k=1), X0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        X = lne.propagate(ctx, rp, col, pp, X0)
        torch.cuda.synchronize()
        t_pr = time.perf_counter() - t0
        t0, t1, t2, t3 = 0.0, t_sp, t_sp + t_rs, t_sp + t_rs + t_pr
        res[prec] = dict(U=U.double().cpu().numpy(), S=S.cpu().numpy(), X0=X0.double().cpu().numpy(),
                         X=X.double().cpu().numpy(), t_sparsify=t1 - t0, t_rsvd=t2 - t1,
                         t_propagate=t3 - t2, nnz=nnz, stats=st)
        log(f"{prec}: sparsify {t1 - t0:.2f}s rsvd {t2 - t1:.2f}s propagate {t3 - t2:.2f}s nnz={nnz}")
        del U, S, V, X0, X
        torch.cuda.empty_cache()
    ref = res["f64"]
    S = ref["S"]
    gaps = (S[:-1] - S[1:]) / S[0]
    dprime = int(max([i + 1 for i in range(len(gaps)) if gaps[i] >= 1e-3] or [1]))
    kp = p["d"] + p["oversample"]
    out = {"report": "precision", "workload": name, "n": g.n, "m": g.m, "M": p["M"], "d": p["d"],
           "q": p["q"], "oversample": p["oversample"], "d_prime": dprime,
           "gap_at_d_prime": float(gaps[dprime - 1]), "results": {}}
    for prec, u in (("f32", 2.0 ** -24), ("bf16", 2.0 ** -8)):
        r = res[prec]
        # every stored n x k' block is rounded entry by entry, so the factorised products
        # move by at most about 4 sqrt(k') u s_1: the principal angle of the top d' vectors
        # is then at most 4 sqrt(k') u / gap (the bar of the precision tests)
        bar = 4 * math.sqrt(kp) * u / max(float(gaps[dprime - 1]), 1e-12)
        out["results"][prec] = {
            "sigma_max_rel_err": float(np.max(np.abs(r["S"] - S) / S)),
            "U_principal_angle_top_dprime": _principal_angle(r["U"][:, :dprime], ref["U"][:, :dprime]),
            "X0_procrustes_rel_err": _procrustes(r["X0"], ref["X0"]),
            "X_procrustes_rel_err": _procrustes(r["X"], ref["X"]),
            "angle_bar": bar,
            "seconds": {"sparsify_trunc_log": r["t_sparsify"], "rsvd": r["t_rsvd"],
                        "propagate": r["t_propagate"]},
        }
    out["results"]["f64"] = {"seconds": {"sparsify_trunc_log": ref["t_sparsify"],
                                         "rsvd": ref["t_rsvd"], "propagate": ref["t_propagate"]},
                             "nnz": ref["nnz"], "stats": ref["stats"]}
    print(json.dumps(out), flush=True)


MFMA_PEAK_TFLOPS = {"f64": 78.6, "f32": 78.6, "bf16": 2500.0}   # FP32 data runs on FP64 MFMA


def hbm_report():
    """Practical streaming rates of this GPU's HBM: torch's device copy (read
    + write), fill (write) and sum (read) of 4 GiB, best of five HIP-event
    timed runs each.  Context for the roofline fractions, which divide by the
    published 8 TB/s."""
    import torch

    n = 1 << 30   # float32 elements: 4 GiB
    a = torch.empty(n, dtype=torch.float32, device="cuda")
    a.uniform_()
    b = torch.empty_like(a)
    out = {"report": "hbm", "bytes": 4 * n, "peak_GBps": HBM_PEAK_GBS, "cases": []}
    for name, fn, nbytes in (("copy (read + write)", lambda: b.copy_(a), 8 * n),
                             ("fill (write)", lambda: b.fill_(1.0), 4 * n),
                             ("sum (read)", lambda: a.sum(), 4 * n)):
        fn()
        torch.cuda.synchronize()
        best = float("inf")
        for _ in range(5):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1))
        gbps = nbytes / (best * 1e-3) / 1e9
        out["cases"].append({"op": name, "ms": best, "GBps": gbps, "of_peak": gbps / HBM_PEAK_GBS})
        log(f"hbm {name}: {best:.3f} ms, {gbps:.0f} GB/s")
    print(json.dumps(out), flush=True)


def mfma_ceiling():
    """Runs tests/probe/mfma_ceiling (built by __graft_entry__.build()): the
    rate of register-only back-to-back MFMAs at 1 to 8 waves per SIMD, the
    most a kernel made of the same instruction can reach on this chip.
    Returns its JSON with the best rate per instruction, or None if the probe
    is not built."""
    exe = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tests", "probe",
                       "mfma_ceiling")
    if not os.path.exists(exe):
        log("mfma ceiling probe not built; reporting against the published peaks only")
        return None
    r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
    if r.returncode != 0:
        raise RuntimeError(f"mfma_ceiling failed ({r.returncode}): {r.stderr.strip()}")
    res = json.loads(r.stdout.strip().splitlines()[-1])
    best = {}
    for x in res["results"]:
        best[x["mfma"]] = max(best.get(x["mfma"], 0.0), x["tflops"])
    res["max_tflops"] = best
    log("mfma ceiling (register-only, best over waves per SIMD): " +
        ", ".join(f"{k} {v:.1f} TFLOP/s" for k, v in best.items()))
    return res


def mfma_report():
    """Achieved matrix-core rate of the dense steps of the fast randomized SVD
    (Gram Y^T Y and projection Y W on MFMA) at the shapes of the large
    workload (n = 1e7, k' = 138, FP32 data on FP64 MFMA) and of the precision
    workload (n = 1e6, k' = 266, FP32 and BF16), from HIP-event times of the
    kernels inside eigSVD (one Gram, one k' x k' eigen-solve, one projection
    U = Y V S^-1)."""
    ceiling = mfma_ceiling()     # a child process, before this one touches the GPU
    import torch

    import paper_2302_07084_amd as lne

    ctx = lne.Context()
    out = {"report": "mfma", "peak_tflops": MFMA_PEAK_TFLOPS, "cases": []}
    if ceiling:
        out["ceiling"] = ceiling
    for dt, n, k in (("f32", 10_000_000, 138), ("f32", 1_000_000, 266), ("bf16", 1_000_000, 266),
                     ("f64", 1_000_000, 266)):
        tdt = {"f64": torch.float64, "f32": torch.float32, "bf16": torch.bfloat16}[dt]
        ld = (k + 7) // 8 * 8
        Y = torch.zeros((n, ld), dtype=tdt, device="cuda")
        Y[:, :k] = torch.randn((n, k), dtype=torch.float32, device="cuda").to(tdt)
        Yk = Y[:, :k]
        lne.eigsvd(ctx, Yk)                  # warm-up
        torch.cuda.synchronize()
        ctx.prof_enable(True)
        ctx.prof_reset()
        reps = 3
        for _ in range(reps):
            lne.eigsvd(ctx, Yk)
        torch.cuda.synchronize()
        gms, gcnt = ctx.prof_get("gram")
        pms, pcnt = ctx.prof_get("project")
        ctx.prof_enable(False)
        # useful flops: Gram n k (k + 1) (upper triangle), projection 2 n k k
        gflop = n * k * (k + 1) * gcnt
        pflop = 2 * n * k * k * pcnt
        peak = MFMA_PEAK_TFLOPS[dt]
        case = {"dtype": dt, "n": n, "k": k, "gram_launches": gcnt, "project_launches": pcnt,
                "gram_tflops": gflop / (gms * 1e-3) / 1e12, "project_tflops": pflop / (pms * 1e-3) / 1e12,
                "gram_avg_ms": gms / gcnt, "project_avg_ms": pms / pcnt}
        case["gram_frac_peak"] = case["gram_tflops"] / peak
        case["project_frac_peak"] = case["project_tflops"] / peak
        top = (ceiling or {}).get("max_tflops", {}).get(
            "bf16_16x16x32" if dt == "bf16" else "f64_16x16x4")
        if top:
            case["gram_frac_ceiling"] = case["gram_tflops"] / top
            case["project_frac_ceiling"] = case["project_tflops"] / top
        out["cases"].append(case)
        log(f"mfma {dt} n={n} k={k}: gram {case['gram_tflops']:.1f} TFLOP/s, "
            f"project {case['project_tflops']:.1f} TFLOP/s (peak {peak})")
        del Y, Yk
        torch.cuda.empty_cache()
    print(json.dumps(out), flush=True)


def _ci95(x):
    """Mean and half-width of the 95% t-interval of the values x."""
    import numpy as np
    import scipy.stats
    x = np.asarray([v for v in x if v is not None], dtype=float)
    if len(x) == 0:
        return None, None
    if len(x) == 1:
        return float(x[0]), None
    return float(x.mean()), float(scipy.stats.t.ppf(0.975, len(x) - 1) * x.std(ddof=1) /
                                  math.sqrt(len(x)))


def automl_report(name, budget, pretrain_per_graph, seeds=3):
    """Hyperparameter search on the batched-trials workload, two arms on the
    same GPU, the same search space, scorer and splits:
      plain      one trial after another, each with its own sampling pass
                 (random proposals, as a plain sequential search)
      batched    one shared sampling pass, rounds of 16 trials run as one
                 batch (HIP graph replay) and scored in one call, proposed by
                 the surrogate (pretrained on a family of smaller graphs,
                 refitted after each round)
    Repeated over `seeds` seeds (pretraining trials, surrogate initialisation
    and both arms' proposals drawn anew; the graphs stay the same).  Per seed:
    trials/s with and without scoring and the wall time each arm needs to
    reach the better arm's best score minus its 95% interval over the scoring
    splits; over the seeds: means with 95% t-intervals."""
    import numpy as np
    import torch

    import paper_2302_07084_amd as lne
    from paper_2302_07084_amd import search
    from synth import workload

    ctx = lne.Context()
    t0 = time.perf_counter()
    family = []
    for i, (blocks, size, intra) in enumerate([(20, 1000, 0.30), (20, 1000, 0.36), (40, 500, 0.32),
                                                (40, 500, 0.40), (25, 1600, 0.28), (25, 1600, 0.34),
                                                (50, 800, 0.31), (50, 800, 0.37)]):
        g, p = workload(name, sizes=[size] * blocks, intra=intra, seed=100 + i)
        family.append(search.Task.make(ctx, g, p, train_ratio=0.1, n_splits=3, seed=100 + i))
    t_fam = time.perf_counter() - t0
    log(f"automl: {len(family)} family graphs in {t_fam:.1f}s")
    g, p = workload(name, device="cuda")
    task = search.Task.make(ctx, g, p, train_ratio=0.1, n_splits=3, seed=0)
    log(f"automl: target graph n={g.n} m={g.m}, budget {budget} trials per arm, {seeds} seeds")
    # warm both paths once so that neither arm pays first-launch costs
    w = search.sample_trials(np.random.default_rng(9), 1)
    search.plain_sequential_search(ctx, task, w)
    torch.cuda.synchronize()

    def best_ci(sc):
        m = sc.mean(axis=1)
        i = int(np.argmax(m))
        half = 1.96 * sc[i].std(ddof=1) / math.sqrt(sc.shape[1]) if sc.shape[1] > 1 else 0.0
        return float(m[i]), float(half)

    runs = []
    for seed in range(seeds):
        t0 = time.perf_counter()
        F, y = search.pretrain_pairs(ctx, family, pretrain_per_graph,
                                     np.random.default_rng(seed))
        t_pairs = time.perf_counter() - t0
        sur = search.Surrogate(ctx, seed=seed)
        sur.set_scaler(F)
        sur.add(F, y)
        t0 = time.perf_counter()
        loss = sur.fit(epochs=800)
        torch.cuda.synchronize()
        t_fit = time.perf_counter() - t0
        log(f"automl seed {seed}: surrogate pretrained on {len(y)} trials ({t_pairs:.1f}s batched "
            f"runs, {t_fit:.1f}s fit, loss {loss})")
        trials_a = search.sample_trials(np.random.default_rng(1000 + seed), budget)
        sa, ta, ea = search.plain_sequential_search(ctx, task, trials_a)
        log(f"automl seed {seed}: plain arm {ta[-1]:.1f}s, best {sa.mean(axis=1).max():.4f}")
        tb, sb, stb, eb, setup = search.batched_surrogate_search(
            ctx, task, sur, budget, np.random.default_rng(2000 + seed))
        log(f"automl seed {seed}: batched arm {stb[-1]:.1f}s (set-up {setup:.1f}s), "
            f"best {sb.mean(axis=1).max():.4f}")
        ba, ca = best_ci(sa)
        bb, cb = best_ci(sb)
        target = (ba - ca) if ba >= bb else (bb - cb)

        def time_to(sc, stamps):
            run = np.maximum.accumulate(sc.mean(axis=1))
            hit = np.flatnonzero(run >= target)
            return float(stamps[hit[0]]) if len(hit) else None

        def arm(sc, stamps, embed_s, extra):
            return dict(extra, trials=len(stamps), seconds=float(stamps[-1]),
                        trials_per_s=len(stamps) / float(stamps[-1]),
                        trials_per_s_embedding_only=len(stamps) / embed_s,
                        best_micro_f1=float(sc.mean(axis=1).max()),
                        mean_micro_f1=float(sc.mean()), seconds_to_target=time_to(sc, stamps))

        r = {"seed": seed, "target_micro_f1": target,
             "arms": {"plain_sequential": arm(sa, ta, ea, {"proposals": "random"}),
                      "batched_surrogate": arm(sb, stb, eb, {"proposals": "surrogate, 25% random",
                                                             "per_round": 16,
                                                             "setup_seconds": setup})},
             "surrogate_pretraining": {"graphs": 8, "trials": int(len(y)),
                                       "batched_run_seconds": t_pairs, "fit_seconds": t_fit}}
        a, b = r["arms"]["plain_sequential"], r["arms"]["batched_surrogate"]
        r["speedup_trials_per_s"] = b["trials_per_s"] / a["trials_per_s"]
        r["speedup_time_to_target"] = (a["seconds_to_target"] / b["seconds_to_target"]
                                       if a["seconds_to_target"] and b["seconds_to_target"] else None)
        runs.append(r)

    def agg(key, arm_name=None):
        vals = [(r["arms"][arm_name][key] if arm_name else r[key]) for r in runs]
        m, h = _ci95(vals)
        return {"mean": m, "ci95": h, "values": vals}

    summary = {"plain_trials_per_s": agg("trials_per_s", "plain_sequential"),
               "batched_trials_per_s": agg("trials_per_s", "batched_surrogate"),
               "speedup_trials_per_s": agg("speedup_trials_per_s"),
               "plain_seconds_to_target": agg("seconds_to_target", "plain_sequential"),
               "batched_seconds_to_target": agg("seconds_to_target", "batched_surrogate"),
               "plain_best_micro_f1": agg("best_micro_f1", "plain_sequential"),
               "batched_best_micro_f1": agg("best_micro_f1", "batched_surrogate"),
               "plain_reached_target": sum(r["arms"]["plain_sequential"]["seconds_to_target"]
                                           is not None for r in runs),
               "batched_reached_target": sum(r["arms"]["batched_surrogate"]["seconds_to_target"]
                                             is not None for r in runs)}
    out = {"report": "automl", "workload": name, "n": g.n, "m": g.m, "T": p["T"], "M": p["M"],
           "d": p["d"], "q": p["q"], "budget": budget, "seeds": seeds,
           "scoring": "one-vs-rest logistic regression on GPU, 10% training labels, 3 seeded "
                      "splits, micro-F1", "summary": summary, "runs": runs}
    print(json.dumps(out), flush=True)


def host_cpu_info():
    """CPU model, logical CPUs of the machine and CPUs this process may run
    on (its affinity mask)."""
    import platform
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        allowed = len(os.sched_getaffinity(0))
    except AttributeError:
        allowed = os.cpu_count() or 1
    return {"model": model, "nproc_machine": os.cpu_count(), "nproc_allowed": allowed}


def cpu_baseline(g, p, seconds):
    """The oracle's sampler + aggregator (plain C, POSIX threads) on a
    contiguous block of edges from the middle of the same workload's edge list
    (the first edges all belong to the largest hub), sized to about `seconds`
    of work on all the threads it may use, then the same block on one thread.
    Threads: the CPUs in this process's affinity mask, capped by
    OMP_NUM_THREADS (the host's CPU share per GPU) when that is set.  Scope:
    the sampling and aggregation stages (count CSR) only, in accepted
    samples per second; the GPU's rate over the same stages is reported beside
    it (`gpu_same_scope`)."""
    import oracle
    info = host_cpu_info()
    cap = os.environ.get("OMP_NUM_THREADS")
    threads = info["nproc_allowed"]
    if cap and cap.isdigit() and int(cap) > 0:
        threads = min(threads, int(cap))
    e0 = g.m // 2
    cnt = max(1000, g.m // 10000)
    while True:
        e1 = min(g.m, e0 + cnt)
        t0 = time.perf_counter()
        _, _, _, att, acc = oracle.count_csr(g, p, nthreads=threads, e_begin=e0, e_end=e1)
        dt = time.perf_counter() - t0
        log(f"cpu baseline: edges [{e0}, {e1}), {acc} accepted samples in {dt:.2f}s "
            f"on {threads} threads")
        if dt >= seconds * 0.6 or e1 >= g.m:
            break
        cnt = int(cnt * min(50.0, max(1.5, seconds / max(dt, 1e-3))))
    # one thread on a block with a tenth of the work per thread
    e1s = min(g.m, e0 + max(1000, (e1 - e0) // max(threads, 1) // 2))
    t0 = time.perf_counter()
    _, _, _, att1, acc1 = oracle.count_csr(g, p, nthreads=1, e_begin=e0, e_end=e1s)
    dt1 = time.perf_counter() - t0
    log(f"cpu baseline: one thread, edges [{e0}, {e1s}), {acc1} accepted samples in {dt1:.2f}s")
    return {"value": acc / dt, "unit": "sampled edges/s (sampling + aggregation stages)",
            "cores": threads, "kind": "oracle",
            "sample": f"all {att} sample slots of edges [{e0}, {e1}) of {g.m} "
                      f"(sampled, walked and aggregated to a count CSR), {dt:.1f}s",
            "single_thread": {"value": acc1 / dt1, "edges": [e0, e1s], "seconds": dt1},
            "host": info}


if __name__ == "__main__":
    main()
