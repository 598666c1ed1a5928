#!/usr/bin/env python3
"""Benchmark one wavelet-tree build on one MI355X.

A step is one complete build (every kernel of wt_build: histogram, node
tables, one pass per level with bitmaps, rank directory and next-level
order) of one synthetic sequence that is already resident in HBM.  The
default workload is n = 2^28 uint8 symbols, sigma = 256, with Zipf(1.1)
symbol frequencies over a seeded permutation of the alphabet.

Prints one JSON line: symbols/s of whole builds (K timed builds with no
instrumentation inside a build), the roofline of the dominant kernel (the
level pass) from HIP events recorded on the build's stream around every
launch in a second pass of K timed builds, and the sequential CPU oracle
timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

import wtgen  # noqa: E402

HBM_PEAK_GBPS = 8000.0
METRIC = "input symbols/s and % HBM roofline per wtree build; p50/p99 build latency served"

WORKLOADS = {
    "c1": "n=2^20 uint8 sigma=256 uniform",
    "c2": "n=2^28 uint8 sigma=256 Zipf(1.1) over a seeded permutation of the alphabet",
    "c3": "n=2^28 uint32 sigma=2^20 half uniform, half 64 Gaussian clusters (sd 2^10)",
    "c4": "4096 sequences, n = 2^U with U ~ U[10, 22], sigma from {4, 20, 256, 2^16} "
          "(u8/u8/u8/u16), uniform symbols; one batched build",
    "c5": "serving: Poisson build requests, n = 2^U with U ~ U[12, 26], sigma from {4, 256, 2^16, 2^20} "
          "(u8/u8/u16/u32), Zipf(1.0) symbols, 10 rank/select queries per tree, HBM-footprint admission",
}


def kernel_source_hash() -> str:
    """Hash of the kernel sources and the tuning table (the counter figures in
    profiles/traffic.json are keyed by it)."""
    from paper_1610_05994_amd.profiling import kernel_source_hash as h
    return h()


def instrumented_pass(steps, step):
    """Per-kernel durations: `steps` more steps with a HIP event recorded on
    the build's stream before and after every launch (wt_prof_enable).  Each
    record between two kernels idles the stream for several microseconds, so
    these steps are timed apart from the ones that give `value`; their own
    wall time per step is returned beside the records."""
    import torch
    from paper_1610_05994_amd import wtree
    wtree.wt_prof_enable(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    recs = wtree.wt_prof_read()
    wtree.wt_prof_enable(False)
    return (t1 - t0) * 1e3 / steps, recs


def calib_copy(args, dev):
    """One plain device copy of --calib-copy-mib MiB: in a counter run, what
    FETCH_SIZE and WRITE_SIZE read for it scales the kernels' readings."""
    import torch
    if args.calib_copy_mib:
        src = torch.empty(args.calib_copy_mib << 20, dtype=torch.uint8, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst


def copy_reference(dev, stream, mib: int = 256, copies: int = 10, reps: int = 3):
    """A plain device-to-device copy of `mib` MiB on the build's stream (read +
    write bytes over its duration; `copies` back to back between one event
    pair, so that the events' own cost is spread thin; median of `reps`): the
    bandwidth a pass that reads and writes what it moves can reach on this
    GPU, for scale beside the roofline's 8 TB/s."""
    import torch
    src = torch.empty(mib << 20, dtype=torch.uint8, device=dev)
    dst = torch.empty_like(src)
    times = []
    with torch.cuda.stream(stream):
        dst.copy_(src)  # warm
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            for _ in range(copies):
                dst.copy_(src)
            b.record(stream)
            b.synchronize()
            times.append(a.elapsed_time(b) / copies)
    del src, dst
    ms = statistics.median(times)
    return {"gbps": 2 * (mib << 20) / (ms / 1e3) / 1e9, "bytes": 2 * (mib << 20),
            "how": "torch device-to-device copies of %d MiB on the build's stream, %d back to back per "
                   "event pair, median of %d" % (mib, copies, reps)}


def per_level_rows(lvl):
    """Level-pass launches grouped by tree level: average duration and
    algorithmic GB/s (a folded pass, which also writes the next level's
    bitmap, shows as the last row with fewer bytes)."""
    by = {}
    for r in lvl:
        e = by.setdefault(r["level"], [0, 0.0, 0])
        e[0] += 1
        e[1] += r["ms"]
        e[2] += r["bytes"]
    rows = []
    for level in sorted(by):
        k, ms, b = by[level]
        rows.append({"level": level, "avg_us": round(ms * 1e3 / k, 2),
                     "gbps": round(b / (ms / 1e3) / 1e9, 1) if ms > 0 else None})
    return rows


def load_traffic_entry(workload: str):
    """The committed rocprofv3 counter figures of a workload, or None when the
    kernel source changed since they were taken."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        data = json.load(f)
    ent = data.get(workload)
    if not ent or ent.get("kernel_hash") != kernel_source_hash():
        return None
    return ent


def load_batch_traffic():
    """HBM bytes per batched build of the batched kernels (counters), or None."""
    ent = load_traffic_entry("c4")
    return ent.get("bytes_per_batched_build") if ent else None


def load_traffic(workload: str):
    """HBM bytes per level launch (counters), or None."""
    ent = load_traffic_entry(workload)
    return ent.get("bytes_per_level_launch") if ent else None


def whole_build_traffic(args, ms_per_step: float):
    """HBM bytes that every kernel of one build moves (rocprofv3 FETCH_SIZE and
    WRITE_SIZE, scaled by a plain copy's readings) over the measured time per
    build, or None for variants and when the counters are stale."""
    if args.matrix or args.buffered or args.arity == 4 or args.huffman:
        return None
    ent = load_traffic_entry(args.workload)
    if not ent or "bytes_per_build" not in ent:
        return None
    b = ent["bytes_per_build"]
    gbps = b / (ms_per_step / 1e3) / 1e9
    return {"bytes": b, "gbps": gbps, "frac_of_peak": gbps / HBM_PEAK_GBPS}


def host_facts() -> dict:
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else None
    return {"cpu_model": model, "nproc": os.cpu_count(), "cores_available": aff}


def _workload_input(workload: str, lg: int):
    return wtgen.workload(workload if not lg else "%s@lg%d" % (workload, lg))


def cpu_baseline(workload: str, lg: int, runs: int, matrix: bool = False, arity: int = 2):
    """The sequential oracle on the workload (its full size unless lg is
    set), on one host core: the calling thread is pinned to one CPU of its
    affinity set while it runs."""
    import oracle
    S, sigma = _workload_input(workload, lg)
    build = oracle.build_matrix if matrix else (oracle.build4 if arity == 4 else oracle.build)
    build(S[:4096], sigma)  # load + warm the library
    pinned = None
    if hasattr(os, "sched_setaffinity"):
        saved = os.sched_getaffinity(0)
        pinned = min(saved)
        os.sched_setaffinity(0, {pinned})
    try:
        times = []
        for _ in range(runs):
            t0 = time.perf_counter()
            build(S, sigma)
            times.append(time.perf_counter() - t0)
        med = statistics.median(times)
        # the paper times construction without the rank structures: the same
        # oracle with the directories switched off (one run)
        t0 = time.perf_counter()
        if arity == 4:
            build(S, sigma, with_dir=False)
        else:
            build(S, sigma, with_ranks=False)
        plain = time.perf_counter() - t0
    finally:
        if pinned is not None:
            os.sched_setaffinity(0, saved)
    n = S.shape[0]
    return {
        "value": n / med,
        "unit": "symbols/s",
        "cores": 1,
        "kind": "oracle",
        "sample": "first-principles sequential oracle (gcc -O2, one thread pinned to CPU %s) on the whole "
                  "workload input (n=%d), median of %d runs of %.2f s each, bitmaps + rank directories"
                  % (pinned, n, runs, med),
        "value_without_directories": n / plain,
        "host": host_facts(),
    }


def cpu_multicore(workload: str, lg: int, runs: int):
    """The paper's parallel algorithms (pwt, dd) on every host core, on the
    same bounded sample as the oracle baseline."""
    from paper_1610_05994_amd import cpu_baseline as cb
    S, sigma = _workload_input(workload, lg)
    threads = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    threads = int(os.environ.get("OMP_NUM_THREADS", threads))
    out = {}
    for algo in cb.ALGOS:
        cb.build(S[:4096], sigma, algo, threads)
        times = []
        for _ in range(runs):
            t0 = time.perf_counter()
            rc, _, _ = cb.build(S, sigma, algo, threads)
            times.append(time.perf_counter() - t0)
            assert rc == 0
        med = statistics.median(times)
        out[algo] = {"value": S.shape[0] / med, "unit": "symbols/s", "cores": threads,
                     "sample": "n=%d symbols of the workload, median of %d runs of %.3f s" % (S.shape[0], runs, med)}
    return out


def main() -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--matrix", action="store_true",
                    help="build the wavelet matrix of the workload instead of the wavelet tree (c1-c3)")
    ap.add_argument("--arity", type=int, default=2, choices=[2, 4],
                    help="4: build the 4-ary wavelet tree of the workload (c1-c3)")
    ap.add_argument("--huffman", action="store_true",
                    help="build the Huffman-shaped wavelet tree of the workload (c1-c3): each step counts the "
                         "symbols on the GPU, reads the counts back, derives the code on the host and builds")
    ap.add_argument("--buffered", type=int, default=0, metavar="LG",
                    help="buffered build of the workload (c1-c3) in buffers of 2^LG symbols, read from "
                         "page-locked host memory (PCIe included in the step) or, with --buffered-source "
                         "device, from HBM")
    ap.add_argument("--buffered-source", default="host", choices=["host", "device"])
    ap.add_argument("--cpu-sample-lg", type=int, default=0,
                    help="time the CPU baselines on 2^LG symbols of the workload (0: its full size)")
    ap.add_argument("--cpu-runs", type=int, default=0,
                    help="timed runs of each CPU baseline (default: 5, and 3 for the large-alphabet c3)")
    ap.add_argument("--no-extra", action="store_true",
                    help="default line only: skip the c3 and c4 measurements added to it under 'extra'")
    ap.add_argument("--input-cache", default="",
                    help="directory to keep the generated input between runs (.npy)")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="run one plain device copy of this size first (counter calibration)")
    ap.add_argument("--batched-only", action="store_true",
                    help="c4: skip the one-build-call-per-sequence comparison (counter runs)")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py measures one GPU only: the build runs on a single MI355X and this "
              "benchmark takes no multi-GPU configuration (--gpus 1).", file=sys.stderr)
        return 2

    if args.workload == "c4":
        print(json.dumps(bench_batch(args)), flush=True)
        return 0
    if args.workload == "c5":
        return bench_serve(args)
    default = args.workload == "c2" and not (args.matrix or args.buffered or args.arity == 4 or args.huffman)
    out = bench_single(args)
    if out is None:
        return 2
    if not args.no_cpu_baseline:
        lg = args.cpu_sample_lg
        print("bench: CPU oracle baseline on n=2^%s" % (lg if lg else "full"), file=sys.stderr, flush=True)
        runs = args.cpu_runs or (3 if args.workload == "c3" else 5)
        out["cpu_baseline"] = cpu_baseline(args.workload, lg, runs, args.matrix, args.arity)
        out["cpu_multicore"] = cpu_multicore(args.workload, lg, runs)
    if default and not args.no_extra:
        out["extra"] = extra_workloads(args)
    print(json.dumps(out), flush=True)
    return 0


def extra_workloads(args) -> dict:
    """The other workloads, measured in the same run as the headline line
    with fewer steps: the large-alphabet single build (c3) and the batched
    build (c4) with time per build, symbols/s, the level-pass roofline, the
    compulsory-byte fraction and, for the batch, its speedup over one build
    call per sequence; the short single build (c1) with its latency; and the
    serving loop (c5) with its sustained rate and latency percentiles."""
    import torch
    ex = {}
    a1 = argparse.Namespace(**vars(args))
    a1.workload, a1.steps, a1.warmup = "c1", 20, 3
    r1 = bench_single(a1)
    ex["c1"] = {"workload": r1["config"]["workload"], "steps": a1.steps, "ms_per_step": r1["ms_per_step"],
                "symbols_per_s": r1["value"], "build_latency_ms": r1["build_latency_ms"]}
    del r1
    torch.cuda.empty_cache()
    a3 = argparse.Namespace(**vars(args))
    a3.workload, a3.steps, a3.warmup = "c3", max(5, args.steps // 4), 1
    r3 = bench_single(a3)
    ex["c3"] = {"workload": r3["config"]["workload"], "steps": a3.steps, "ms_per_step": r3["ms_per_step"],
                "symbols_per_s": r3["value"], "build_latency_ms": r3["build_latency_ms"],
                "roofline": {k: r3["roofline"][k] for k in ("bound", "achieved", "peak", "unit", "frac", "traffic",
                                                             "kernel", "avg_launch_us", "frac_of_copy")},
                "compulsory_bytes": r3["compulsory_bytes"], "whole_build_traffic": r3["whole_build_traffic"]}
    del r3
    torch.cuda.empty_cache()
    a4 = argparse.Namespace(**vars(args))
    a4.workload, a4.steps, a4.warmup = "c4", 6, 2
    r4 = bench_batch(a4)
    ex["c4"] = {"workload": r4["config"]["workload"], "steps": a4.steps, "ms_per_step": r4["ms_per_step"],
                "symbols_per_s": r4["value"], "roofline": r4["roofline"], "compulsory_bytes": r4["compulsory_bytes"],
                "one_call_per_sequence": r4["one_call_per_sequence"]}
    torch.cuda.empty_cache()
    a5 = argparse.Namespace(**vars(args))
    a5.workload, a5.warmup = "c5", 1
    r5 = serve_result(a5)
    sv = r5["serving"]
    ex["c5"] = {"workload": r5["config"]["workload"], "sustained_symbols_per_s": r5["value"],
                "latency_ms": r5["latency_ms"], "saturation_ms": sv["saturation"]["seconds"] * 1e3,
                "loads": {k: {q: v[q] for q in ("p50_ms", "p99_ms", "symbols_per_s", "qps")}
                          for k, v in sv["loads"].items()},
                "one_call_per_request": r5["one_call_per_request"]}
    return ex


def bench_single(args):
    """One single-build workload (c1-c3, or a variant): returns the JSON
    object of its line, without the CPU baselines."""
    import torch

    from paper_1610_05994_amd import wtree

    dev = torch.device("cuda:0")
    print("bench: generating workload %s" % args.workload, file=sys.stderr, flush=True)
    S, sigma = None, None
    if args.input_cache:
        path = os.path.join(args.input_cache, "%s.npy" % args.workload)
        if os.path.exists(path):
            S = np.load(path)
            sigma = {"c1": 256, "c2": 256, "c3": 1 << 20}[args.workload]
    if S is None:
        S, sigma = wtgen.workload(args.workload)
        if args.input_cache:
            os.makedirs(args.input_cache, exist_ok=True)
            np.save(os.path.join(args.input_cache, "%s.npy" % args.workload), S)
    n, width = S.shape[0], S.dtype.itemsize
    if sum(bool(x) for x in (args.buffered, args.arity == 4, args.matrix, args.huffman)) > 1:
        print("bench.py: --matrix, --arity 4, --huffman and --buffered are separate variants", file=sys.stderr)
        return None
    if args.buffered and args.buffered_source == "host":
        view = {1: np.uint8, 2: np.int16, 4: np.int32}[width]
        dS = torch.from_numpy(S.view(view)).pin_memory()
    else:
        dS = wtree.to_device(S, dev)
    if args.huffman:
        counts_dev = torch.empty(sigma, dtype=torch.int64, device=dev)
        counts_host = torch.empty(sigma, dtype=torch.int64).pin_memory()
        counts0 = np.bincount(S.astype(np.int64), minlength=sigma).astype(np.uint64)
        rc, tb, wb = wtree.wt_huffman_footprint(counts0, n, sigma, width)
    elif args.buffered:
        rc, tb, wb = wtree.wt_buffered_footprint(n, sigma, width, 1 << args.buffered)
    elif args.arity == 4:
        rc, tb, wb = wtree.wt_multiary_footprint(n, sigma, width)
    else:
        rc, tb, wb = wtree.wt_footprint(n, sigma, width)
    assert rc == wtree.WT_OK
    tree_mem = torch.empty(tb, dtype=torch.uint8, device=dev)
    work_mem = torch.empty(wb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream(device=dev)
    sh = int(stream.cuda_stream)

    calib_copy(args, dev)

    build_fn = wtree.wt_build_matrix if args.matrix else (wtree.wt_build_multiary if args.arity == 4 else wtree.wt_build)
    if args.buffered:
        def build_fn(S_ptr, n, sigma, width, t_ptr, tb, w_ptr, wb, sh):
            return wtree.wt_build_buffered(S_ptr, n, sigma, width, 1 << args.buffered, t_ptr, tb, w_ptr, wb, sh)
    fn_name = "wt_build_buffered" if args.buffered else build_fn.__name__
    if args.huffman:
        def build_fn(S_ptr, n, sigma, width, t_ptr, tb, w_ptr, wb, sh):
            # the whole method: counts on the GPU, read back, code on the host, build
            rc = wtree.wt_histogram(S_ptr, n, sigma, width, counts_dev.data_ptr(), sh)
            if rc != wtree.WT_OK:
                return rc, 0
            with torch.cuda.stream(stream):
                counts_host.copy_(counts_dev, non_blocking=True)
            stream.synchronize()
            return wtree.wt_build_huffman(S_ptr, n, sigma, width, counts_host.numpy().view(np.uint64), t_ptr, tb,
                                          w_ptr, wb, sh)
        fn_name = "wt_build_huffman"

    def one_build():
        rc, h = build_fn(dS.data_ptr(), n, sigma, width, tree_mem.data_ptr(), tb, work_mem.data_ptr(), wb, sh)
        if rc != wtree.WT_OK:
            raise wtree.WtError(rc, fn_name)
        return h

    print("bench: warmup %d" % args.warmup, file=sys.stderr, flush=True)
    for _ in range(args.warmup):
        wtree.wt_free(one_build())
    torch.cuda.synchronize()

    # sanity: the last warm-up tree decodes sampled positions back to S
    h = one_build()
    if wtree.wt_tree_status(h) != wtree.WT_OK:
        raise RuntimeError("build reported an error")
    pos = torch.from_numpy(np.random.Generator(np.random.PCG64(1)).integers(0, n, 4096)).to(dev)
    sym = torch.empty(4096, dtype=torch.int32, device=dev)
    assert wtree.wt_access_batch(h, pos.data_ptr(), sym.data_ptr(), 4096, sh) == wtree.WT_OK
    torch.cuda.synchronize()
    want = torch.from_numpy(S[pos.cpu().numpy()].astype(np.int64))
    assert torch.equal(sym.cpu().to(torch.int64) & 0xFFFFFFFF, want), "sampled access mismatch"
    huff_info = None
    if args.huffman:
        rc, info = wtree.wt_huffman_levels(h, sigma)
        assert rc == wtree.WT_OK
        huff_info = {"levels": info["levels"], "bits_per_symbol": sum(info["sizes"]) / max(1, n),
                     "balanced_levels": max(0, (sigma - 1).bit_length()), "tree_bytes": tb}
    wtree.wt_free(h)

    print("bench: timing %d steps" % args.steps, file=sys.stderr, flush=True)
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        h = one_build()
        ev[k][1].record(stream)
        wtree.wt_free(h)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    ms_instrumented, recs = instrumented_pass(args.steps, lambda: wtree.wt_free(one_build()))
    copy_ref = copy_reference(dev, stream)
    step_ms = sorted(a.elapsed_time(b) for a, b in ev)
    p50 = float(np.percentile(step_ms, 50))
    p99 = float(np.percentile(step_ms, 99))
    value = n / (ms_per_step / 1e3)

    lvl_kernel = "quad" if args.arity == 4 else "level"  # the pass that moves the symbols
    lvl = [r for r in recs if r["kernel"] == lvl_kernel]
    lvl_ms = sum(r["ms"] for r in lvl)
    lvl_bytes = sum(r["bytes"] for r in lvl)
    launches = len(lvl)
    achieved = lvl_bytes / (lvl_ms / 1e3) / 1e9 if lvl_ms > 0 else 0.0
    fams = {}
    for r in recs:
        f = fams.setdefault(r["kernel"], {"launches": 0, "ms": 0.0})
        f["launches"] += 1
        f["ms"] += r["ms"]
    for f in fams.values():
        f["avg_us"] = round(f["ms"] * 1e3 / f["launches"], 2)
        f["ms_per_step"] = round(f["ms"] / args.steps, 4)
        del f["ms"]
    traffic = None if (args.matrix or args.buffered or args.arity == 4 or args.huffman) else load_traffic(args.workload)
    levels = max(0, (sigma - 1).bit_length())
    qmin = n * width + (tb - 256)  # read S once + write every bitmap word and rank entry once
    qmin_gbps = qmin / (p50 / 1e3) / 1e9

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "symbols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {1: "u8", 2: "u16", 4: "u32"}[width],
        "data": "synthetic",
        "config": {"workload": "%s: %s%s%s" % (args.workload, WORKLOADS[args.workload],
                                               ("; wavelet matrix" if args.matrix else "") +
                                               ("; 4-ary wavelet tree" if args.arity == 4 else "") +
                                               ("; Huffman-shaped wavelet tree (histogram, code and build "
                                                "in every step)" if args.huffman else ""),
                                               ("; buffered build, 2^%d-symbol buffers from %s" % (
                                                   args.buffered, "page-locked host memory (PCIe included)"
                                                   if args.buffered_source == "host" else "HBM"))
                                               if args.buffered else ""), "n": n, "sigma": sigma,
                   "width_bytes": width, "levels": levels, "seed": wtgen.SEED_BASE + int(args.workload[1]) - 1},
        "roofline": {
            "bound": "hbm",
            "achieved": achieved,
            "peak": HBM_PEAK_GBPS,
            "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBPS,
            "traffic": traffic,
            "kernel": ("k_quad (one four-way split per digit level)" if args.arity == 4
                       else "k_level (one launch per tree level)"),
            "avg_launch_us": lvl_ms * 1e3 / max(launches, 1),
            "algorithmic_bytes_per_launch": lvl_bytes / max(launches, 1),
            "per_level": per_level_rows(lvl),
            "copy_reference": copy_ref,
            "frac_of_copy": (achieved / copy_ref["gbps"]) if copy_ref else None,
        },
        "build_latency_ms": {"p50": p50, "p99": p99},
        "instrumented_ms_per_step": ms_instrumented,
        "compulsory_bytes": {"bytes": qmin, "gbps_at_p50": qmin_gbps, "frac_of_peak": qmin_gbps / HBM_PEAK_GBPS},
        "whole_build_traffic": whole_build_traffic(args, ms_per_step),
        "kernels": fams,
    }
    if huff_info:
        out["huffman"] = huff_info
    if args.buffered:
        mg = [r for r in recs if r["kernel"] == "merge"]
        mg_ms = sum(r["ms"] for r in mg)
        out["buffered"] = {
            "buffer_syms": 1 << args.buffered,
            "buffers": -(-n // (1 << args.buffered)),
            "source": args.buffered_source,
            "input_gbps": n * width / (ms_per_step / 1e3) / 1e9,
            "merge_avg_us": mg_ms * 1e3 / max(1, len(mg)),
            "merge_gbps": (sum(r["bytes"] for r in mg) / (mg_ms / 1e3) / 1e9) if mg_ms > 0 else None,
            "workspace_bytes": wb,
        }
    return out


def bench_batch(args) -> dict:
    """Batched build of many uneven sequences vs one build call per sequence."""
    import torch

    from paper_1610_05994_amd import wtree

    dev = torch.device("cuda:0")
    calib_copy(args, dev)
    m = int(os.environ.get("WT_BENCH_BATCH", "4096"))
    print("bench: generating %d sequences" % m, file=sys.stderr, flush=True)
    specs = wtgen.batch_specs(m, wtgen.SEED_BASE + 3)
    Ss = wtgen.batch_inputs(specs)
    total = sum(d["n"] for d in specs)
    dS = [wtree.to_device(S, dev) for S in Ss]
    descs = [(d["n"], d["sigma"], d["width"]) for d in specs]
    trees, tbytes = [], []
    max_work = 256
    for d in descs:
        rc, tb, wb = wtree.wt_footprint(*d)
        trees.append(torch.empty(tb, dtype=torch.uint8, device=dev))
        tbytes.append(tb)
        max_work = max(max_work, wb)
    rc, bw = wtree.wt_batch_footprint(descs)
    assert rc == wtree.WT_OK
    work = torch.empty(bw, dtype=torch.uint8, device=dev)
    work1 = torch.empty(max_work, dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream(device=dev)
    sh = int(stream.cuda_stream)
    sptr = [x.data_ptr() for x in dS]
    tptr = [x.data_ptr() for x in trees]

    def batched():
        rc, hs = wtree.wt_build_batch(sptr, descs, tptr, tbytes, work.data_ptr(), bw, sh)
        if rc != wtree.WT_OK:
            raise wtree.WtError(rc, "wt_build_batch")
        return hs

    def one_by_one():
        hs = []
        for q, d in enumerate(descs):
            rc, h = wtree.wt_build(sptr[q], d[0], d[1], d[2], tptr[q], tbytes[q], work1.data_ptr(), max_work, sh)
            if rc != wtree.WT_OK:
                raise wtree.WtError(rc, "wt_build")
            hs.append(h)
        return hs

    def timed(fn, steps, warmup):
        for _ in range(warmup):
            for h in fn():
                wtree.wt_free(h)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            for h in fn():
                wtree.wt_free(h)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) * 1e3 / steps

    print("bench: batched", file=sys.stderr, flush=True)
    ms_batch = timed(batched, args.steps, args.warmup)

    def batched_step():
        for h in batched():
            wtree.wt_free(h)

    ms_batch_instrumented, recs = instrumented_pass(args.steps, batched_step)
    # sanity: sampled positions of a few trees decode back to their sequences
    hs = batched()
    torch.cuda.synchronize()
    for q in range(0, m, max(1, m // 16)):
        n = descs[q][0]
        if n == 0:
            continue
        assert wtree.wt_tree_status(hs[q]) == wtree.WT_OK
        pos = torch.from_numpy(np.random.Generator(np.random.PCG64(q)).integers(0, n, 64)).to(dev)
        sym = torch.empty(64, dtype=torch.int32, device=dev)
        assert wtree.wt_access_batch(hs[q], pos.data_ptr(), sym.data_ptr(), 64, sh) == wtree.WT_OK
        torch.cuda.synchronize()
        want = torch.from_numpy(Ss[q][pos.cpu().numpy()].astype(np.int64))
        assert torch.equal(sym.cpu().to(torch.int64) & 0xFFFFFFFF, want), "batched access mismatch"
    for h in hs:
        wtree.wt_free(h)
    ms_single = None
    if not getattr(args, "batched_only", False):
        print("bench: one build call per sequence", file=sys.stderr, flush=True)
        ms_single = timed(one_by_one, max(1, args.steps // 4), 1)

    lvl = [r for r in recs if r["kernel"] in ("batch_level", "batch_small", "batch_mid")]
    lvl_ms = sum(r["ms"] for r in lvl)
    lvl_bytes = sum(r["bytes"] for r in lvl)
    achieved = lvl_bytes / (lvl_ms / 1e3) / 1e9 if lvl_ms > 0 else 0.0
    # compulsory bytes: read every sequence once, write every tree once
    qmin = sum(d[0] * d[2] for d in descs) + sum(tb - 256 for tb in tbytes)
    qmin_gbps = qmin / (ms_batch / 1e3) / 1e9
    out = {
        "metric": METRIC,
        "value": total / (ms_batch / 1e3),
        "unit": "symbols/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_batch,
        "instrumented_ms_per_step": ms_batch_instrumented,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8/u16",
        "data": "synthetic",
        "config": {"workload": "c4: " + WORKLOADS["c4"], "sequences": m, "total_symbols": total},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBPS, "traffic": load_batch_traffic(),
                     "kernel": "batched build kernels: one-workgroup builds of the short sequences and the "
                               "level phases (supsum + prep + level pass) of the long ones"},
        "compulsory_bytes": {"bytes": qmin, "gbps": qmin_gbps, "frac_of_peak": qmin_gbps / HBM_PEAK_GBPS},
        "one_call_per_sequence": None if ms_single is None else {
            "ms": ms_single, "symbols_per_s": total / (ms_single / 1e3), "batched_speedup": ms_single / ms_batch},
    }
    del dS, trees, work, work1
    return out


def bench_serve(args) -> int:
    print(json.dumps(serve_result(args)), flush=True)
    return 0


def serve_result(args) -> dict:
    """Serving loop: saturation throughput, then Poisson streams at 0.5 /
    0.8 / 0.95 of it, with p50/p99 request latency (arrival to answers)."""
    import torch

    from paper_1610_05994_amd import serve, wtree

    dev = torch.device("cuda:0")
    P = int(os.environ.get("WT_SERVE_POOL", "48"))
    print("bench: generating %d serving sequences" % P, file=sys.stderr, flush=True)
    specs = wtgen.serve_stream(P, 1.0, wtgen.SEED_BASE + 4)
    pool = serve.make_pool(specs, dev, workers=min(12, os.cpu_count() or 1))
    for p in pool:
        p["host"] = None          # only the device copies and counts are needed
    mean_n = float(np.mean([p["n"] for p in pool]))
    budget = int(float(os.environ.get("WT_SERVE_BUDGET_GIB", "64")) * (1 << 30))
    nstreams = int(os.environ.get("WT_SERVE_STREAMS", "4"))
    srv = serve.Server(budget_bytes=budget, streams=nstreams, max_inflight=8)
    torch.cuda.synchronize()

    def run(count, qps, seed, rid0):
        reqs = serve.requests_from(pool, wtgen.pool_stream(P, count, qps, seed), rid0)
        srv.run_stream(reqs, timeout=300)
        st = serve.summarize(reqs)
        for r in reqs:
            if r.state == serve.RESIDENT:
                srv.release(r.rid)
        return reqs, st

    print("bench: serving warmup", file=sys.stderr, flush=True)
    run(max(8, args.warmup * 8), 1e9, 1, 0)
    # saturation: every request present at t = 0
    nsat = int(os.environ.get("WT_SERVE_SAT", "256"))
    print("bench: serving saturation (%d requests)" % nsat, file=sys.stderr, flush=True)
    _, sat = run(nsat, 1e9, 2, 10_000)
    sustain = sat["symbols_per_s"]
    loads = {}
    rid = 20_000
    for f in (0.5, 0.8, 0.95):
        qps = f * sustain / mean_n
        count = int(max(100, min(2000, qps * 4.0)))
        print("bench: serving load %.2f (%.0f req/s, %d requests)" % (f, qps, count), file=sys.stderr, flush=True)
        _, st = run(count, qps, int(f * 100), rid)
        rid += 10_000
        st["qps"] = qps
        loads["%.2f" % f] = st
    # the same saturation requests, one wt_build call each, back to back
    print("bench: one build call per request", file=sys.stderr, flush=True)
    reqs = serve.requests_from(pool, wtgen.pool_stream(P, nsat, 1e9, 2), 0)
    t0 = time.perf_counter()
    for r in reqs:
        t = wtree.build(r.S, r.sigma)
        if len(r.rank_c):
            t.rank(r.rank_c, r.rank_i)
        if len(r.sel_c):
            t.select(r.sel_c, r.sel_j)
        torch.cuda.synchronize()
        t.close()
    one = sum(r.S.numel() for r in reqs) / (time.perf_counter() - t0)
    srv.close()
    mid = loads["0.80"]
    out = {
        "metric": METRIC,
        "value": sustain,
        "unit": "symbols/s",
        "n_gpus": 1,
        "steps": nsat,
        "warmup": args.warmup,
        "ms_per_step": sat["seconds"] * 1e3 / nsat,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8/u16/u32",
        "data": "synthetic",
        "config": {"workload": "c5: " + WORKLOADS["c5"], "pool_sequences": P, "mean_n": mean_n,
                   "budget_bytes": budget, "streams": nstreams},
        "latency_ms": {"p50": mid["p50_ms"], "p99": mid["p99_ms"], "at_load": 0.8},
        "serving": {"saturation": sat, "loads": loads, "arena_high_water": srv.arena.high_water},
        "one_call_per_request": {"symbols_per_s": one, "served_speedup": sustain / one},
    }
    del srv, pool
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    sys.exit(main())
