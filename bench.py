"""Benchmark of the fused PageRank path on one MI355X.

A step is one full PageRank solve (FP32 ranks, FP64 residual and dangling
sums, uniform dangling redistribution, damping 0.85, L1 tolerance 1e-6) on
an R-MAT scale-22 graph (edge factor 16, a/b/c/d = .57/.19/.19/.05, seed
22, self-loops and duplicates removed) that is already resident in HBM,
through GrM_pagerank in nonblocking mode, i.e. one fused kernel per
iteration.  value = GTEPS = edges x iterations / solve time.

Also reported on the same JSON line: the unfused (blocking) solve, the FP64
fused solve and the FP32-vs-FP64 error, the roofline of the fused kernel
(algorithmic bytes per launch over its event-timed average duration), a
streaming-copy probe, and the CPU oracle timed on a bounded sample.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
DAMPING = 0.85


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def fused_bytes_per_pass(n: int, m: int, b: int) -> int:
    """Algorithmic bytes of one fused pass: row pointers, column indices,
    the gathered operand (compulsory n*b), x_old, d, and the two outputs
    (new ranks and their pre-scaled copy)."""
    return 4 * (n + 1) + 4 * m + 5 * n * b


def blocking_bytes_per_pass(n: int, m: int, b: int) -> int:
    """Unfused: mult (3n) + mxv (rowptr, col, gather n, write n) + apply (2n)
    + absdiff (3n) + reduce (n) + masked reduce (2n)."""
    return 4 * (n + 1) + 4 * m + 13 * n * b


COPY_BYTES = 1 << 30  # bytes read and written by one launch of the copy probe
# fused FP32 kernel of each plan kind: name, committed profile summary of
# the scale-22 pass, sources whose hash the summary records
FUSED_KERNELS = {
    0: ("fused_pr_kernel<float, ...>", None, ("kernels.hip",)),
    1: ("fused_wave_kernel<float, ...>", "fused_wave_kernel_rmat22.md", ("kernels.hip",)),
    2: ("fused_stripe_kernel", "fused_stripe_kernel_rmat22.md", ("stripe.hip",)),
    3: ("cold_fill_kernel+fused_stripe_kernel", "fused_stripe_kernel_twophase_rmat22.md", ("stripe.hip",)),
}
TRAFFIC_KERNELS = {"fused_wave_kernel<float": 1, "fused_stripe_kernel": 2, "cold_fill_kernel+fused_stripe_kernel": 3}


def kernel_source_sha(kind: int = 1) -> str:
    """sha256 over the sources that define the fused kernel of a plan kind."""
    import hashlib
    h = hashlib.sha256()
    for f in FUSED_KERNELS[kind][2] + ("kernels.h", "device_util.h", "ops_device.h"):
        with open(os.path.join(ROOT, "paper_2509_14211_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def recorded_traffic(kind: int):
    """HBM-side bytes per launch of the fused FP32 kernel of a plan kind as
    recorded in the committed profile summary, or None when the summary is
    missing or the kernel sources changed since the counters were taken."""
    if FUSED_KERNELS[kind][1] is None:
        return None
    try:
        text = open(os.path.join(ROOT, "profiles", FUSED_KERNELS[kind][1])).read()
    except OSError:
        return None
    kv = {}
    for line in text.splitlines():
        if line.startswith("- ") and ": " in line:
            k, v = line[2:].split(": ", 1)
            kv[k.strip()] = v.strip()
    if kv.get("source_sha256") != kernel_source_sha(kind):
        return None
    try:
        return int(kv["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def summarize_rocprof(dirs, traffic_kernel: str = "fused_wave_kernel<float", min_write_kib: float = 0.0,
                      min_launch_us: float = 20.0) -> None:
    """Kernel statistics (from --kernel-trace --stats) and per-dispatch PMC
    counters (from --pmc runs) found under the given directories, as
    Markdown tables; with FETCH_SIZE and WRITE_SIZE runs that include the
    copy probe, also the calibrated traffic per launch of the fused kernels.
    With min_write_kib, only the traffic kernel's launches whose WRITE_SIZE
    reaches it are counted (matched by launch order between the two runs):
    the fused passes, when plain mxv launches of the same kernel (blocking
    mode) share the profile.  min_launch_us: the trace table also averages
    the launches at least this long (the passes of the larger graph when
    two graphs share a profile)."""
    import collections
    import csv
    import glob
    parts = traffic_kernel.split("+")  # a pass of several kernels: their traffic adds up
    counters = collections.defaultdict(list)
    for d in dirs:
        stats = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)
        for p in stats:
            print("### kernel statistics (%s)\n" % os.path.basename(p))
            print("| kernel | calls | average (us) | min (us) | max (us) | share |")
            print("|---|---|---|---|---|---|")
            for r in list(csv.DictReader(open(p)))[:15]:
                print("| %s | %s | %.2f | %.2f | %.2f | %.2f%% |" % (
                    r["Name"][:90], r["Calls"], float(r["AverageNs"]) / 1e3, float(r["MinNs"]) / 1e3,
                    float(r["MaxNs"]) / 1e3, float(r["Percentage"])))
            print()
        traces = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)
        for p in traces:
            dur = collections.defaultdict(list)
            for r in csv.DictReader(open(p)):
                dur[r["Kernel_Name"]].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
            print("### launches of the fused kernels (%s)\n" % os.path.basename(p))
            print("| kernel | launches | mean (us) | launches > %g us | their mean (us) |" % min_launch_us)
            print("|---|---|---|---|---|")
            for k, v in dur.items():
                if "fused" in k or any(part in k for part in parts):
                    act = [x for x in v if x > min_launch_us]
                    print("| %s | %d | %.2f | %d | %.2f |" % (k[:90], len(v), sum(v) / len(v), len(act),
                                                            sum(act) / max(len(act), 1)))
            print()
        pmcs = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        for p in pmcs:
            vals = collections.defaultdict(list)
            for r in sorted(csv.DictReader(open(p)), key=lambda r: int(r["Dispatch_Id"])):
                vals[(r["Kernel_Name"], r["Counter_Name"])].append(float(r["Counter_Value"]))
            print("### counters per dispatch (%s)\n" % os.path.basename(p))
            print("| kernel | counter | dispatches | mean | max |")
            print("|---|---|---|---|---|")
            for (k, c), v in sorted(vals.items()):
                if "fused" in k or "stream_copy" in k or any(part in k for part in parts):
                    print("| %s | %s | %d | %.1f | %.1f |" % (k[:90], c, len(v), sum(v) / len(v), max(v)))
                    counters[(k, c)] = v
            print()
    copy = [k for (k, c) in counters if "stream_copy" in k]
    if not copy:
        return
    ck = copy[0]
    f_copy = sum(counters[(ck, "FETCH_SIZE")]) / max(len(counters[(ck, "FETCH_SIZE")]), 1)
    w_copy = sum(counters[(ck, "WRITE_SIZE")]) / max(len(counters[(ck, "WRITE_SIZE")]), 1)
    if not f_copy or not w_copy:
        return
    f_scale = COPY_BYTES / (f_copy * 1024.0)
    w_scale = COPY_BYTES / (w_copy * 1024.0)
    picked = []
    for part in parts:
        # the matching kernel (template instance) with the most launches
        # that pass the write filter
        best = None
        for k in sorted({k for (k, c) in counters if part in k}):
            fv, wv = counters.get((k, "FETCH_SIZE"), []), counters.get((k, "WRITE_SIZE"), [])
            if not fv or len(fv) != len(wv):
                continue
            keep = [i for i, w in enumerate(wv) if w >= min_write_kib]
            if keep and (best is None or len(keep) > len(best[3])):
                best = (k, fv, wv, keep)
        if best is None:
            print("### calibrated traffic of %s: no launch of %s passes the filters\n" % (traffic_kernel, part))
            return
        picked.append(best)
    print("### calibrated traffic of %s\n" % traffic_kernel)
    print("The copy probe reads and writes %d bytes per launch; its counters give the scale of each "
          "counter (bytes per KiB reported).\n" % COPY_BYTES)
    print("- copy_fetch_kib: %.1f" % f_copy)
    print("- copy_write_kib: %.1f" % w_copy)
    print("- fetch_scale: %.4f" % (f_scale * 1.0))
    print("- write_scale: %.4f" % (w_scale * 1.0))
    traffic = 0.0
    for k, fv, wv, keep in picked:
        f_k = sum(fv[i] for i in keep) / len(keep)
        w_k = sum(wv[i] for i in keep) / len(keep)
        traffic += f_k * 1024.0 * f_scale + w_k * 1024.0 * w_scale
        print("- kernel: %s" % k[:90])
        print("- kernel_fetch_kib_per_launch: %.1f" % f_k)
        print("- kernel_write_kib_per_launch: %.1f" % w_k)
        if len(keep) != len(wv):
            print("- launches_counted: %d of %d (WRITE_SIZE >= %.0f KiB)" % (len(keep), len(wv), min_write_kib))
    print("- traffic_bytes_per_launch: %d" % int(round(traffic)))
    if traffic_kernel in TRAFFIC_KERNELS:
        print("- source_sha256: %s" % kernel_source_sha(TRAFFIC_KERNELS[traffic_kernel]))
    print()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--scale", type=int, default=22)
    ap.add_argument("--tol", type=float, default=1e-6)
    ap.add_argument("--check-every", type=int, default=8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-blocking", action="store_true",
                    help="scale25 / web legs: skip the blocking solves (for profiling the fused passes alone)")
    ap.add_argument("--cpu-seconds", type=float, default=8.0,
                    help="target length of the one-thread CPU oracle sample (whole solves)")
    ap.add_argument("--ppr-k", type=int, default=64, help="seed sets of the batched PPR leg")
    ap.add_argument("--ppr-itermax", type=int, default=1000,
                    help="pass limit of the batched and sequential PPR solves (with --tol 0 every column "
                         "runs this many passes at full width: a fixed-width run for profiling)")
    ap.add_argument("--ppr-stream", type=int, default=512,
                    help="seed sets streamed through the ppr-k column slots (0: skip)")
    ap.add_argument("--many", type=int, default=256, help="graphs of the many-graph leg")
    ap.add_argument("--warm-train-sets", type=int, default=256,
                    help="seed sets per training graph of the warm-start leg (0: skip it)")
    ap.add_argument("--skip-extras", action="store_true",
                    help="time only the headline fused solve (for profiling); same as --legs none")
    ap.add_argument("--legs", default="all",
                    help="comma list of extra legs to run: blocking (also FP64), m0, ppr, many, fusion, bfs, "
                         "scale25, web, warm; "
                         "or all / none")
    ap.add_argument("--traffic-kernel", default="fused_wave_kernel<float",
                    help="kernel (name substring) whose calibrated traffic --summarize-rocprof reports")
    ap.add_argument("--min-write-kib", type=float, default=0.0,
                    help="with --summarize-rocprof: count only traffic-kernel launches writing at least this")
    ap.add_argument("--min-launch-us", type=float, default=20.0,
                    help="with --summarize-rocprof: also average the fused launches at least this long")
    ap.add_argument("--summarize-rocprof", metavar="DIR", nargs="+",
                    help="print a text summary of the rocprofv3 CSV files under the DIRs and exit")
    args = ap.parse_args()
    if args.summarize_rocprof:
        summarize_rocprof(args.summarize_rocprof, args.traffic_kernel, args.min_write_kib, args.min_launch_us)
        return

    legs = {"blocking", "m0", "ppr", "many", "fusion", "bfs", "scale25", "web", "warm"} if args.legs == "all" else (
        set() if args.legs == "none" else set(args.legs.split(",")))
    if args.skip_extras:
        legs = set()

    def leg(name):
        return name in legs

    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2509_14211_amd import api, grb

    torch.cuda.init()
    dev = torch.cuda.get_device_properties(0)
    log("device:", dev.name, "CUs:", dev.multi_processor_count)
    stream = torch.cuda.current_stream()

    out = {}
    with api.Context(grb.GrB_NONBLOCKING):
        t0 = time.perf_counter()
        g = api.rmat_graph(args.scale)
        torch.cuda.synchronize()
        setup_s = time.perf_counter() - t0
        n, m = g.n, g.m
        log("graph: scale %d n %d m %d (setup %.2fs)" % (args.scale, n, m, setup_s))

        def solve(dtype, check_every=args.check_every):
            return api.pagerank(g, dtype, DAMPING, args.tol, 1000, grb.GrM_DANGLING_UNIFORM,
                                None, check_every)

        # ---- plan selection (the autotuner times candidate tile plans on this
        # graph, like the paper's warm-up run that fills its code cache)
        tuned = {}
        for dt, name in ((torch.float32, "GrB_FP32"), (torch.float64, "GrB_FP64")):
            t0 = time.perf_counter()
            cfg, us = grb.GrM_autotune_pagerank(g.AT, g.outdeg, grb.builtin(name),
                                                os.environ.get("NBGRB_TUNE_CACHE"))
            tuned[name] = dict(cfg, us_per_pass=round(us, 2),
                               tune_s=round(time.perf_counter() - t0, 3))
            log("autotune %s: %s (%.1f us/pass)" % (name, cfg, us))
        out["plan"] = tuned

        def pass_time_us(dtype, k1=4, k2=20):
            """Time of one fused pass: two single-batch runs of k1 and k2 passes
            (tolerance 0, no early stop) timed with HIP events on the library's
            stream; their difference over k2 - k1 cancels the setup."""
            t = []
            for k in (k1, k2, k1, k2):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                api.pagerank(g, dtype, DAMPING, 0.0, k, grb.GrM_DANGLING_UNIFORM, None, k)
                e1.record(stream)
                torch.cuda.synchronize()
                t.append(e0.elapsed_time(e1))
            return ((t[1] - t[0]) + (t[3] - t[2])) / 2 * 1e3 / (k2 - k1)

        def timed(dtype, steps, warmup):
            for _ in range(warmup):
                solve(dtype)
            torch.cuda.synchronize()
            ev = [torch.cuda.Event(enable_timing=True) for _ in range(steps + 1)]
            iters = []
            ev[0].record(stream)
            x = None
            for k in range(steps):
                x, it, res = solve(dtype)
                iters.append(it)
                ev[k + 1].record(stream)
            torch.cuda.synchronize()
            per = [ev[k].elapsed_time(ev[k + 1]) for k in range(steps)]
            timed.min_ms = min(per)
            ms = ev[0].elapsed_time(ev[steps]) / steps
            return x, iters, ms, res

        # ---- headline: fused FP32
        grb.GrM_set_mode(grb.GrB_NONBLOCKING)
        x32, iters32, ms32, res32 = timed(torch.float32, args.steps, args.warmup)
        min32 = timed.min_ms
        it32 = iters32[-1]
        gteps = m * it32 / (ms32 * 1e-3) / 1e9
        log("fused fp32: %d iterations, %.3f ms/solve, %.1f GTEPS" % (it32, ms32, gteps))

        # ---- roofline of the fused pass
        kind32 = tuned["GrB_FP32"]["kernel"]
        avg_us = pass_time_us(torch.float32)
        bpp = fused_bytes_per_pass(n, m, 4)
        achieved = bpp / (avg_us * 1e-6) / 1e9
        log("fused pass: %.2f us, %.1f GB/s algorithmic" % (avg_us, achieved))
        out["roofline"] = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                           "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                           # the committed counters cover the scale-22 graph only
                           "traffic": recorded_traffic(kind32) if args.scale == 22 else None,
                           "kernel": FUSED_KERNELS[kind32][0],
                           "bytes_per_launch": bpp, "avg_launch_us": round(avg_us, 3)}
        if out["roofline"]["traffic"]:
            # fabric-side rate of the same pass: counter bytes over the pass time
            out["roofline"]["traffic_gbs"] = round(out["roofline"]["traffic"] / (avg_us * 1e-6) / 1e9, 1)

        # ---- streaming copy probe (1 GiB)
        nb = 1 << 30
        a = torch.empty(nb // 4, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        grb.GrM_stream_copy(b, a, nb)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(10):
            grb.GrM_stream_copy(b, a, nb)
        e1.record(stream)
        torch.cuda.synchronize()
        copy_gbs = 2 * nb * 10 / (e0.elapsed_time(e1) * 1e-3) / 1e9
        del a, b
        log("stream copy: %.1f GB/s" % copy_gbs)
        out["stream_copy_gbs"] = round(copy_gbs, 1)
        out["roofline"]["frac_of_copy"] = round(achieved / copy_gbs, 4)

        if leg("blocking"):
            # ---- unfused (blocking) FP32
            grb.GrM_set_mode(grb.GrB_BLOCKING)
            xb, itersb, msb, _ = timed(torch.float32, max(2, args.steps // 2), 1)
            grb.GrM_set_mode(grb.GrB_NONBLOCKING)
            gteps_b = m * itersb[-1] / (msb * 1e-3) / 1e9
            log("blocking fp32: %d iterations, %.3f ms/solve, %.1f GTEPS" % (itersb[-1], msb, gteps_b))
            # ---- fused FP64 and the FP32 error against it
            x64, iters64, ms64, _ = timed(torch.float64, 2, 1)
            gteps64 = m * iters64[-1] / (ms64 * 1e-3) / 1e9
            err = float((x32.double() - x64).abs().sum().item())
            log("fused fp64: %d iterations, %.3f ms/solve; |x32-x64|_1 = %.3e" % (iters64[-1], ms64, err))
            out["unfused"] = {"gteps": round(gteps_b, 2), "ms_per_solve": round(msb, 4),
                              "iterations": itersb[-1],
                              "bytes_per_iteration": blocking_bytes_per_pass(n, m, 4)}
            out["fused_vs_unfused_speedup"] = round(msb / ms32, 3)
            out["fp64_fused"] = {"gteps": round(gteps64, 2), "ms_per_solve": round(ms64, 4),
                                 "iterations": iters64[-1]}
            out["l1_fp32_vs_fp64"] = err

        # ---- batched personalised PageRank: 64 seed sets (sizes 1..16) as one
        # SpMM solve vs 64 sequential single-vector solves, same tolerance
        if leg("ppr") and args.ppr_k > 0:
            import synthetic
            sets = [s.tolist() for s in synthetic.ppr_seed_sets(n, args.ppr_k, seed=7)]
            f32 = grb.builtin("GrB_FP32")
            X = torch.empty(n * len(sets), dtype=torch.float32, device="cuda")
            grb.GrM_ppr_batch(X, f32, sets, g.AT, g.outdeg, DAMPING, args.tol, args.ppr_itermax)  # warm-up
            torch.cuda.synchronize()
            reps = 3
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            for _ in range(reps):
                pit, col_it, col_res = grb.GrM_ppr_batch(X, f32, sets, g.AT, g.outdeg, DAMPING,
                                                         args.tol, args.ppr_itermax)
            e1.record(stream)
            torch.cuda.synchronize()
            batch_ms = e0.elapsed_time(e1) / reps
            # sequential single-vector solves of the first few sets, scaled
            nseq = min(8, len(sets))
            r = grb.GrB_Vector_new(f32, n)
            seq_ms = 0.0
            for s_ in sets[:nseq]:
                v = torch.zeros(n, dtype=torch.float32, device="cuda")
                v[torch.as_tensor(s_, dtype=torch.long)] = 1.0 / len(s_)
                vv = api.vector_from_tensor(v)
                torch.cuda.synchronize()
                e0.record(stream)
                grb.GrM_ppr(r, g.AT, g.outdeg, vv, DAMPING, args.tol, args.ppr_itermax)
                e1.record(stream)
                torch.cuda.synchronize()
                seq_ms += e0.elapsed_time(e1)
                grb.GrB_Vector_free(vv)
            grb.GrB_Vector_free(r)
            seq_per_query = seq_ms / nseq
            # algorithmic bytes: the pattern and d once per pass, and per
            # column-pass the gathered w, x_old, x_new and w_new (columns
            # stop at their own converged pass; the product narrows)
            col_passes = int(np.sum(col_it[col_it > 0])) + int(np.sum(col_it <= 0)) * pit
            alg_bytes = (4 * (n + 1) + 4 * m + 4 * n) * pit + 4 * n * 4 * col_passes
            del X
            log("ppr batch: %d sets, %d passes, %.2f ms -> %.1f queries/s; sequential %.2f ms/query "
                "(%.1f queries/s)" % (len(sets), pit, batch_ms, len(sets) / batch_ms * 1e3,
                                      seq_per_query, 1e3 / seq_per_query))
            out["ppr"] = {"queries_per_s": round(len(sets) / batch_ms * 1e3, 1), "k": len(sets),
                          "passes": pit, "column_passes": col_passes,
                          "ms_per_batch": round(batch_ms, 3),
                          "sequential_queries_per_s": round(1e3 / seq_per_query, 1),
                          "batch_vs_sequential_speedup": round(seq_per_query * len(sets) / batch_ms, 2),
                          "algorithmic_gbs": round(alg_bytes / (batch_ms * 1e-3) / 1e9, 1),
                          "max_col_resid": float(col_res.max())}
            # a stream of seed sets through the same 64 column slots: a
            # converged column is written out and restarts with the next set
            if args.ppr_stream > 0:
                ssets = [s_.tolist() for s_ in synthetic.ppr_seed_sets(n, args.ppr_stream, seed=8)]
                Xs = torch.empty(n * len(ssets), dtype=torch.float32, device="cuda")
                torch.cuda.synchronize()
                e0.record(stream)
                s_it, s_ps, s_res = grb.GrM_ppr_stream(Xs, f32, ssets, g.AT, g.outdeg, DAMPING, args.tol, 1000,
                                                       grb.GrM_DANGLING_UNIFORM, len(sets), 2)
                e1.record(stream)
                torch.cuda.synchronize()
                stream_ms = e0.elapsed_time(e1)
                del Xs
                log("ppr stream: %d sets through %d slots, %.1f ms -> %.1f queries/s (mean %.1f passes per set, "
                    "first converged at %.1f)" % (len(ssets), len(sets), stream_ms, len(ssets) / stream_ms * 1e3,
                                                  s_ps.mean(), s_it.mean()))
                out["ppr"]["stream"] = {"sets": len(ssets), "slots": len(sets), "ms": round(stream_ms, 2),
                                        "queries_per_s": round(len(ssets) / stream_ms * 1e3, 1),
                                        "mean_passes_per_set": round(float(s_ps.mean()), 2),
                                        "mean_first_converged_pass": round(float(s_it.mean()), 2),
                                        "max_resid": float(s_res.max())}
                # the workload's figure stays the 64-set batch (one SpMM
                # solve); the stream is a separate configuration
                out["ppr"]["stream_queries_per_s"] = out["ppr"]["stream"]["queries_per_s"]

        # ---- many small graphs: one persistent, graph-captured launch vs the
        # same graphs solved one after another
        if leg("many") and args.many > 0:
            import synthetic
            specs = synthetic.many_graph_specs(args.many)
            t0 = time.perf_counter()
            mgs = [api.rmat_graph(sc, 16, sd) for sc, sd in specs]
            mg = grb.GrM_Multigraph_new([x.AT for x in mgs])
            torch.cuda.synchronize()
            pack_s = time.perf_counter() - t0
            off = grb.GrM_Multigraph_offsets(mg, len(mgs))
            f32 = grb.builtin("GrB_FP32")
            Xm = torch.empty(int(off[-1]), dtype=torch.float32, device="cuda")
            grb.GrM_pagerank_many(Xm, f32, mg, len(mgs), DAMPING, args.tol, 1000)  # capture
            reps = 5
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            torch.cuda.synchronize()
            e0.record(stream)
            for _ in range(reps):
                grb.GrM_pagerank_many(Xm, f32, mg, len(mgs), DAMPING, args.tol, 1000)
            e1.record(stream)
            torch.cuda.synchronize()
            many_ms = e0.elapsed_time(e1) / reps
            its, res = grb.GrM_pagerank_many(Xm, f32, mg, len(mgs), DAMPING, args.tol, 1000)
            edges = sum(x.m for x in mgs)
            for x in mgs:  # sequential baseline: warm every plan first
                api.pagerank(x, torch.float32, DAMPING, args.tol, 1000)
            torch.cuda.synchronize()
            e0.record(stream)
            seq_it = 0
            for x in mgs:
                _, it_, _ = api.pagerank(x, torch.float32, DAMPING, args.tol, 1000)
                seq_it += it_
            e1.record(stream)
            torch.cuda.synchronize()
            seq_ms = e0.elapsed_time(e1)
            log("many graphs: %d graphs, %d vertices, %d edges; one launch %.3f ms (%.0f graphs/s, "
                "%.1f GTEPS); sequential %.2f ms; pack %.1fs" % (
                    len(mgs), int(off[-1]), edges, many_ms, len(mgs) / many_ms * 1e3,
                    float((its.astype(np.int64) * np.array([x.m for x in mgs])).sum()) / (many_ms * 1e-3) / 1e9,
                    seq_ms, pack_s))
            out["many_graphs"] = {"graphs": len(mgs), "vertices": int(off[-1]), "edges": int(edges),
                                  "ms_per_launch": round(many_ms, 4),
                                  "graphs_per_s": round(len(mgs) / many_ms * 1e3, 1),
                                  "gteps": round(float((its.astype(np.int64) * np.array(
                                      [x.m for x in mgs])).sum()) / (many_ms * 1e-3) / 1e9, 2),
                                  "sequential_ms": round(seq_ms, 3),
                                  "speedup_vs_sequential": round(seq_ms / many_ms, 2),
                                  "max_resid": float(res.max()), "max_iters": int(its.max())}
            grb.GrM_Multigraph_free(mg)
            for x in mgs:
                x.free()
            del Xm

        # ---- the smallest configuration: R-MAT scale 10, FP64 to 1e-9, the
        # fused nonblocking loop vs the blocking one (time and launches)
        if leg("m0"):
            g10 = api.rmat_graph(10)
            res0 = {}
            for mode in (grb.GrB_NONBLOCKING, grb.GrB_BLOCKING):
                grb.GrM_set_mode(mode)
                api.pagerank(g10, torch.float64, DAMPING, 1e-9, 1000, grb.GrM_DANGLING_UNIFORM, None, 8)
                torch.cuda.synchronize()
                grb.GrM_reset_stats()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                reps = 20
                for _ in range(reps):
                    _, it10, _ = api.pagerank(g10, torch.float64, DAMPING, 1e-9, 1000, grb.GrM_DANGLING_UNIFORM,
                                              None, 8)
                e1.record(stream)
                torch.cuda.synchronize()
                st = grb.GrM_get_stats()
                res0[mode] = (e0.elapsed_time(e1) / reps, it10, st["kernels"] / reps, st["fused_launches"] / reps)
            grb.GrM_set_mode(grb.GrB_NONBLOCKING)
            g10.free()
            fz, bl = res0[grb.GrB_NONBLOCKING], res0[grb.GrB_BLOCKING]
            log("scale 10 fp64: fused %.3f ms (%d passes, %.1f kernels/solve), blocking %.3f ms (%.1f kernels/solve)" % (
                fz[0], fz[1], fz[2], bl[0], bl[2]))
            out["scale10_fp64"] = {"iterations": fz[1], "fused_ms": round(fz[0], 4), "blocking_ms": round(bl[0], 4),
                                   "fused_kernels_per_solve": fz[2], "blocking_kernels_per_solve": bl[2],
                                   "fused_passes_per_solve": fz[3],
                                   "fused_vs_unfused_speedup": round(bl[0] / fz[0], 2)}

        # ---- generated elementwise fusion: w = |x .* (y + 1) - 2 z| / 3 over
        # 2^26 FP32 entries, one generated kernel vs five per-op kernels
        if leg("fusion"):
            ne = 1 << 26
            f = grb.builtin
            xs = [torch.rand(ne, device="cuda") for _ in range(3)]
            vx, vy, vz = (api.vector_from_tensor(t_) for t_ in xs)
            w = grb.GrB_Vector_new(f("GrB_FP32"), ne)

            def chain():
                t1 = grb.GrB_Vector_new(f("GrB_FP32"), ne)
                grb.GrB_Vector_apply_BinaryOp2nd_FP64(t1, None, None, f("GrB_PLUS_FP32"), vy, 1.0)
                t2 = grb.GrB_Vector_new(f("GrB_FP32"), ne)
                grb.GrB_Vector_eWiseMult_BinaryOp(t2, None, None, f("GrB_TIMES_FP32"), vx, t1)
                t3 = grb.GrB_Vector_new(f("GrB_FP32"), ne)
                grb.GrB_Vector_apply_BinaryOp1st_FP64(t3, None, None, f("GrB_TIMES_FP32"), 2.0, vz)
                t4 = grb.GrB_Vector_new(f("GrB_FP32"), ne)
                grb.GrB_Vector_eWiseAdd_BinaryOp(t4, None, None, f("GrM_ABSDIFF_FP32"), t2, t3)
                grb.GrB_Vector_apply_BinaryOp2nd_FP64(w, None, None, f("GrB_DIV_FP32"), t4, 3.0)
                for h in (t1, t2, t3, t4):
                    grb.GrB_Vector_free(h)
                grb.GrB_Vector_wait(w)

            res_f = {}
            for level in (1, 0):
                grb.GrM_set_fusion(level)
                t0 = time.perf_counter()
                chain()
                torch.cuda.synchronize()
                first_s = time.perf_counter() - t0
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(10):
                    chain()
                e1.record(stream)
                torch.cuda.synchronize()
                res_f[level] = (e0.elapsed_time(e1) / 10, first_s)
            grb.GrM_set_fusion(1)
            for h in (vx, vy, vz, w):
                grb.GrB_Vector_free(h)
            del xs
            fused_b, perop_b = 16 * ne, 48 * ne
            log("elementwise chain over %d: generated %.3f ms (%.1f GB/s), per-op %.3f ms; first call %.2fs" % (
                ne, res_f[1][0], fused_b / (res_f[1][0] * 1e-3) / 1e9, res_f[0][0], res_f[1][1]))
            out["ewise_fusion"] = {"n": ne, "ops": 5, "generated_ms": round(res_f[1][0], 4),
                                   "per_op_ms": round(res_f[0][0], 4),
                                   "speedup": round(res_f[0][0] / res_f[1][0], 2),
                                   "generated_gbs": round(fused_b / (res_f[1][0] * 1e-3) / 1e9, 1),
                                   "per_op_gbs": round(perop_b / (res_f[0][0] * 1e-3) / 1e9, 1),
                                   "first_call_s": round(res_f[1][1], 3)}

        def big_graph_leg(gx, dang, tol, itermax, reps):
            """Fused solve to tolerance (autotuned plan), the pass time from
            two fixed-length runs, and the blocking solve, all FP32."""
            f32 = grb.builtin("GrB_FP32")
            cfg, _ = grb.GrM_autotune_pagerank(gx.AT, gx.outdeg, f32, os.environ.get("NBGRB_TUNE_CACHE"))

            def solve_x():
                return api.pagerank(gx, torch.float32, DAMPING, tol, itermax, dang, None, args.check_every)

            def time_x(k):
                solve_x()
                torch.cuda.synchronize()
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                for _ in range(k):
                    xx, it_, res_ = solve_x()
                e1.record(stream)
                torch.cuda.synchronize()
                return e0.elapsed_time(e1) / k, it_, res_, xx

            ms_x, it_x, res_x, xx = time_x(reps)
            t = []
            for k in (4, 20, 4, 20):
                e0 = torch.cuda.Event(enable_timing=True)
                e1 = torch.cuda.Event(enable_timing=True)
                e0.record(stream)
                api.pagerank(gx, torch.float32, DAMPING, 0.0, k, dang, None, k)
                e1.record(stream)
                torch.cuda.synchronize()
                t.append(e0.elapsed_time(e1))
            us_x = ((t[1] - t[0]) + (t[3] - t[2])) / 2 * 1e3 / 16
            bpp_x = fused_bytes_per_pass(gx.n, gx.m, 4)
            msb_x, itb_x = None, None
            if not args.no_blocking:
                grb.GrM_set_mode(grb.GrB_BLOCKING)
                msb_x, itb_x, _, _ = time_x(max(1, reps - 1))
                grb.GrM_set_mode(grb.GrB_NONBLOCKING)
            gbs = bpp_x / (us_x * 1e-6) / 1e9
            return {"n": gx.n, "m": gx.m, "plan": cfg, "iterations": it_x, "resid": res_x,
                    "rank_sum": float(xx.double().sum().item()), "ms_per_solve": round(ms_x, 3),
                    "gteps": round(gx.m * it_x / (ms_x * 1e-3) / 1e9, 2),
                    "pass_us": round(us_x, 2), "bytes_per_pass": bpp_x,
                    "achieved_gbs": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                    "blocking_ms_per_solve": round(msb_x, 3) if msb_x else None, "blocking_iterations": itb_x,
                    "fused_vs_unfused_speedup": round(msb_x / ms_x, 3) if msb_x else None}

        # ---- the HBM-bound size: R-MAT scale 25, fused vs blocking (FP32)
        if leg("scale25"):
            t0 = time.perf_counter()
            g25 = api.rmat_graph(25)
            torch.cuda.synchronize()
            setup25 = time.perf_counter() - t0
            r25 = big_graph_leg(g25, grb.GrM_DANGLING_UNIFORM, args.tol, 1000, 3)
            g25.free()
            r25.pop("rank_sum")
            r25.pop("resid")
            log("scale 25: n %d m %d (setup %.1fs); fused %d passes %.2f ms (%.1f GTEPS), pass %.1f us = "
                "%.1f GB/s; blocking %.2f ms" % (r25["n"], r25["m"], setup25, r25["iterations"],
                                                 r25["ms_per_solve"], r25["gteps"], r25["pass_us"],
                                                 r25["achieved_gbs"], r25["blocking_ms_per_solve"] or 0.0))
            out["scale25"] = r25

        # ---- the web-crawl-shaped graph at the size of the paper's data set
        # (50.6M pages, about 1.93B links after merging repeats), in the
        # paper's dangling-drop mode with the GAP benchmark's tolerance
        if leg("web"):
            import synthetic
            t0 = time.perf_counter()
            gw = api.web_graph(synthetic.WEB_N, synthetic.WEB_SEED, synthetic.WEB_MODEL)
            torch.cuda.synchronize()
            setupw = time.perf_counter() - t0
            rw = big_graph_leg(gw, grb.GrM_DANGLING_DROP, synthetic.WEB_TOL, synthetic.WEB_ITERMAX, 3)
            gw.free()
            rw["setup_s"] = round(setupw, 2)
            rw["dangling"] = "drop"
            rw["tol"] = synthetic.WEB_TOL
            log("web: n %d m %d (setup %.1fs); fused %d passes %.2f ms (%.1f GTEPS), pass %.1f us = %.1f GB/s; "
                "blocking %.2f ms" % (rw["n"], rw["m"], setupw, rw["iterations"], rw["ms_per_solve"],
                                      rw["gteps"], rw["pass_us"], rw["achieved_gbs"],
                                      rw["blocking_ms_per_solve"] or 0.0))
            out["web"] = rw

        # ---- vectors with missing entries: breadth-first search on the
        # headline graph, loop drivers chosen by the fill estimates (push for
        # sparse frontiers, pull for dense ones) vs pull at every level
        if leg("bfs"):
            rp_a, _ = api.csr_of(g.A)
            outdeg_h = np.diff(rp_a.cpu().numpy().astype(np.int64))
            del rp_a
            rng_b = np.random.default_rng(17)
            cands = np.nonzero(outdeg_h > 0)[0]
            sources = [int(s_) for s_ in rng_b.choice(cands, 4, replace=False)]

            def run_bfs(policy):
                grb.GrM_set_format_policy(policy)
                lv, _ = api.bfs_levels(g, sources[0])  # warm-up (transposed pattern, plans)
                grb.GrB_Vector_free(lv)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                traversed, depths, lvs = 0, [], []
                stats0 = grb.GrM_get_stats()
                for s_ in sources:
                    lv, depth = api.bfs_levels(g, s_)
                    lvs.append(lv)
                    depths.append(depth)
                torch.cuda.synchronize()
                dt = (time.perf_counter() - t0) / len(sources)
                st = grb.GrM_get_stats()
                # the reached vertices' out-edges, counted after the timed region
                for lv in lvs:
                    idx_b, _ = grb.GrB_Vector_extractTuples(lv)
                    grb.GrB_Vector_free(lv)
                    traversed += int(outdeg_h[idx_b].sum())
                grb.GrM_set_format_policy(0)
                return dt, traversed / len(sources), depths, st["mxv_push"] - stats0["mxv_push"], \
                    st["mxv_pull"] - stats0["mxv_pull"]

            dt_e, tr_e, depths, push_e, pull_e = run_bfs(0)
            dt_p, tr_p, _, push_p, pull_p = run_bfs(1)
            log("bfs: %.2f ms per search (push %d / pull %d levels), pull only %.2f ms; %.2f GTEPS" %
                (dt_e * 1e3, push_e, pull_e, dt_p * 1e3, tr_e / dt_e / 1e9))
            out["bfs"] = {"sources": len(sources), "depths": depths,
                          "ms_per_search": round(dt_e * 1e3, 3), "gteps": round(tr_e / dt_e / 1e9, 2),
                          "push_levels": push_e, "pull_levels": pull_e,
                          "pull_only_ms_per_search": round(dt_p * 1e3, 3),
                          "speedup_vs_pull_only": round(dt_p / dt_e, 2),
                          "edges_per_search": int(tr_e),
                          "timing": "host clock around whole searches on the device, including the "
                                    "per-level count read-back; the levels' extraction to the host is "
                                    "not timed"}

        # ---- learned warm start (reduced size): train on scale-20 graphs,
        # then warm vs teleport start on the headline graph, both to tol;
        # the warm time includes the walk features and the prediction.
        if leg("warm") and args.warm_train_sets > 0:
            from paper_2509_14211_amd import warmstart
            t0 = time.perf_counter()
            ws = warmstart.WarmStart("bf16")
            tr = []
            for gs in (1000, 1001):
                gt = api.rmat_graph(20, seed=gs)
                tr += ws.train([gt], [warmstart.seed_sets(gt.n, args.warm_train_sets, gs)], epochs=1,
                               lr=3e-3, graph_seeds=[gs])
                gt.free()
            train_s = time.perf_counter() - t0
            ev = ws.evaluate(g, warmstart.seed_sets(n, 64, 5000), tol=args.tol, graph_seed=args.scale)
            ws.close()
            log("warm start: trained in %.1fs (KL %.4f); iterations warm %.2f vs teleport %.2f; "
                "%.2f vs %.2f ms per query" % (train_s, tr[-1], ev["mean_iters_warm"], ev["mean_iters_teleport"],
                                               ev["ms_warm"], ev["ms_teleport"]))
            out["warm_start"] = {"train": "2 R-MAT scale-20 graphs x %d seed sets, 1 epoch, BF16 activations" %
                                          args.warm_train_sets,
                                 "train_s": round(train_s, 2), "final_kl": round(tr[-1], 5),
                                 "eval_sets": ev["sets"], "mean_iters_warm": ev["mean_iters_warm"],
                                 "mean_iters_teleport": ev["mean_iters_teleport"],
                                 "ms_per_query_warm": round(ev["ms_warm"], 3),
                                 "ms_per_query_teleport": round(ev["ms_teleport"], 3),
                                 "ms_per_query_features": round(ev["ms_features"], 3),
                                 "fallbacks": ev["fallbacks"],
                                 "pays_in_wall_time": ev["pays"],
                                 "result": ("the learned start is faster in wall time" if ev["pays"] else
                                            "negative: features and prediction cost more wall time than "
                                            "the passes the learned start saves")}

        # ---- CPU oracle: solves to the same tolerance on the same graph, 1
        # warm-up + 16 timed at the host's thread count and a bounded sample
        # at one thread; the GPU error against it at the same pass count.
        if not args.no_cpu_baseline:
            import oracle
            threads = min(16, os.cpu_count() or 1)
            oracle.set_threads(threads)
            t0 = time.perf_counter()
            og = oracle.rmat_graph(args.scale)
            build_s = time.perf_counter() - t0
            ref = oracle.pagerank(og, DAMPING, tol=args.tol)  # warm-up
            runs = 16
            t0 = time.perf_counter()
            for _ in range(runs):
                ref = oracle.pagerank(og, DAMPING, tol=args.tol)
            cpu_s = (time.perf_counter() - t0) / runs
            cpu_gteps = og.m * ref.iters / cpu_s / 1e9
            # one thread: solves to tolerance until about cpu_seconds have
            # passed (at least one; the result does not depend on the thread
            # count)
            oracle.set_threads(1)
            runs1, t1 = 0, 0.0
            while runs1 == 0 or (t1 < args.cpu_seconds and runs1 < 16):
                t0 = time.perf_counter()
                r1 = oracle.pagerank(og, DAMPING, tol=args.tol)
                t1 += time.perf_counter() - t0
                runs1 += 1
            cpu1_s = t1 / runs1
            oracle.set_threads(threads)
            model = ""
            try:
                with open("/proc/cpuinfo") as f_:
                    model = next((ln.split(":", 1)[1].strip() for ln in f_ if ln.startswith("model name")), "")
            except OSError:
                pass
            k = ref.iters
            xk, itk, _ = api.pagerank(g, torch.float32, DAMPING, 0.0, k, grb.GrM_DANGLING_UNIFORM, None, 8)
            errk = float(np.abs(xk.double().cpu().numpy() - ref.x).sum())
            log("oracle: %d passes to tol %g, %.3fs per solve on %d threads (%.3f GTEPS), %.2fs on one; "
                "graph build %.1fs; GPU fp32 L1 error at %d passes: %.3e"
                % (k, args.tol, cpu_s, threads, cpu_gteps, cpu1_s, build_s, k, errk))
            out["cpu_baseline"] = {"value": round(cpu_gteps, 4), "unit": "GTEPS", "cores": threads,
                                   "kind": "oracle",
                                   "sample": "blocking FP64 solves of the same R-MAT scale-%d graph to L1 %g "
                                             "(%d passes): 1 warm-up + %d timed, %.3f s each"
                                             % (args.scale, args.tol, k, runs, cpu_s),
                                   "seconds_to_tol": round(cpu_s, 4),
                                   "one_thread_value": round(og.m * r1.iters / cpu1_s / 1e9, 4),
                                   "one_thread_seconds_to_tol": round(cpu1_s, 3),
                                   "one_thread_sample": "%d solves to L1 %g, no warm-up" % (runs1, args.tol),
                                   "host_cpus": os.cpu_count(), "host_model": model}
            out["l1_fp32_vs_oracle_fixed_passes"] = errk
        g.free()

    line = {
        "metric": "fused PageRank GTEPS & %HBM peak vs unfused at 1e-6 L1; PPR queries/s",
        "value": round(gteps, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms32, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "R-MAT scale %d (n=%d, m=%d after dedup), FP32 ranks + FP64 "
                               "reductions, damping 0.85, tol %g, uniform dangling"
                               % (args.scale, n, m, args.tol),
                   "iterations": it32, "graph_setup_s": round(setup_s, 3),
                   "ms_per_step_min": round(min32, 4)},
    }
    line.update(out)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
