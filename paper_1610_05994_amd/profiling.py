"""Summaries of rocprofv3 output (``--output-format csv``).

``python -m paper_1610_05994_amd.profiling overlap TRACE.csv [PATTERN ...]``
reports, for the dispatches whose kernel name contains one of the patterns,
how long kernels of two or more different streams ran at the same time on
the device, against the time any of them ran: the evidence that batches
launched on different streams overlap.  Without patterns it takes the
serving loop's streams (those that ran a batched-build or multi-tree query
kernel) and every library kernel on them, the single builds of long
requests included.

``python -m paper_1610_05994_amd.profiling traffic --workload W --fetch DIR
--write DIR --bench-log LOG [--calib-mib 256] [--builds K] [--out JSON]``
turns two counter runs of ``bench.py --calib-copy-mib M`` (one with
``--pmc FETCH_SIZE``, one with ``--pmc WRITE_SIZE``) into HBM bytes: each
counter is scaled by what it reads for the plain device copy of M MiB that
the run starts with (bytes read, bytes written), and the result is given per
level-pass launch (the kernels the bench's roofline covers) and per build
(every kernel of the run but the copy, over the number of builds: one
ingest each, or ``--builds``), keyed by the hash of the kernel sources and
the tuning table (``kernel_source_hash``), so that the bench reports them
only while they describe the code that runs.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

_PKG = os.path.dirname(os.path.abspath(__file__))


def kernel_source_hash() -> str:
    """Hash of everything that decides what a build's kernels move: every
    source under csrc/ (kernels, launch sequences, layouts, the fold and
    narrowing decisions) and the tuning table (tile geometry)."""
    h = hashlib.sha256()
    csrc = os.path.join(_PKG, "csrc")
    paths = [os.path.join(csrc, f) for f in sorted(os.listdir(csrc))] + [os.path.join(_PKG, "tune_table.json")]
    for path in paths:
        if os.path.isfile(path):
            h.update(os.path.basename(path).encode())
            with open(path, "rb") as f:
                h.update(f.read())
    return h.hexdigest()[:16]


def read_counters(path: str):
    """{dispatch id: (kernel name, counter value)} from a counter run's CSV
    (a file, or the directory rocprofv3 wrote it under)."""
    if os.path.isdir(path):
        files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
        if not files:
            raise FileNotFoundError("no *counter_collection.csv under " + path)
        path = files[0]
    out = {}
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            d = int(row["Dispatch_Id"])
            name, val = row["Kernel_Name"], float(row["Counter_Value"])
            prev = out.get(d)
            out[d] = (name, (prev[1] if prev else 0.0) + val)
    return out


# the level passes of a single build (the bench's roofline kernel), and the
# batched build's kernels
LEVEL_KERNELS = ("k_level<", "k_level_narrow<")
BATCH_KERNELS = ("k_batch_", "k_small_batch")


def _bench_line(log: str):
    with open(log) as f:
        for line in f:
            if line.startswith("{"):
                return json.loads(line)
    raise ValueError("no JSON line in " + log)


def traffic(workload: str, fetch_dir: str, write_dir: str, bench_log: str, calib_mib: int = 256, builds: int = 0):
    fetch, write = read_counters(fetch_dir), read_counters(write_dir)
    calib = calib_mib << 10  # KiB the copy reads and writes
    # the calibration copy: the runtime's copy kernel with the largest reading
    cf = max((v for k, v in fetch.values() if "copyBuffer" in k), default=0.0)
    cw = max((v for k, v in write.values() if "copyBuffer" in k), default=0.0)
    if cf <= 0 or cw <= 0:
        raise ValueError("no calibration copy in the counter runs")
    fs, ws = calib / cf, calib / cw
    batched = workload == "c4"
    pats = BATCH_KERNELS if batched else LEVEL_KERNELS

    def kib(rows, match):
        vals = [v for k, v in rows.values() if match(k)]
        return sum(vals), len(vals)

    lf, nl = kib(fetch, lambda k: any(p in k for p in pats))
    lw, _ = kib(write, lambda k: any(p in k for p in pats))
    af, _ = kib(fetch, lambda k: "copyBuffer" not in k and (not batched or any(p in k for p in pats)))
    aw, _ = kib(write, lambda k: "copyBuffer" not in k and (not batched or any(p in k for p in pats)))
    nb = builds or sum(1 for k, _ in fetch.values() if "k_ingest<" in k)
    line = _bench_line(bench_log)
    ent = {"kernel_hash": kernel_source_hash(), "fetch_scale": fs, "write_scale": ws,
           "fetch_kib_copy": cf, "write_kib_copy": cw, "builds_in_run": nb}
    if batched:
        ent["bytes_per_batched_build"] = ((lf * fs + lw * ws) * 1024.0) / max(nb, 1)
        ent["launches"] = nl
    else:
        ent["bytes_per_level_launch"] = ((lf * fs + lw * ws) * 1024.0) / max(nl, 1)
        ent["algorithmic_bytes_per_level_launch"] = line["roofline"]["algorithmic_bytes_per_launch"]
        ent["level_launches"] = nl
        ent["bytes_per_build"] = ((af * fs + aw * ws) * 1024.0) / max(nb, 1)
    return ent

SERVE_KERNELS = ("k_batch_", "k_small_batch", "k_query_multi")


def read_dispatches(path: str, patterns=SERVE_KERNELS):
    out = []
    with open(path, newline="") as f:
        for row in csv.DictReader(f):
            name = row["Kernel_Name"]
            if patterns and not any(p in name for p in patterns):
                continue
            out.append((int(row["Start_Timestamp"]), int(row["End_Timestamp"]), int(row.get("Stream_Id") or 0),
                        int(row.get("Queue_Id") or 0), name))
    return out


def serving_dispatches(path: str):
    """Every library kernel (``wt::``) on the streams that ran a serving
    kernel (batched build or multi-tree query)."""
    rows = read_dispatches(path, ("wt::",))
    streams = {d[2] for d in rows if any(p in d[4] for p in SERVE_KERNELS)}
    return [d for d in rows if d[2] in streams]


def overlap(dispatches):
    """Sweep over start / end events: time with >= 1 kernel running, time
    with kernels of >= 2 distinct streams running, and the same per queue."""
    ev = []
    for s, e, stream, queue, _ in dispatches:
        if e > s:
            ev.append((s, 1, stream, queue))
            ev.append((e, -1, stream, queue))
    ev.sort(key=lambda x: (x[0], x[1]))
    active_s = defaultdict(int)
    active_q = defaultdict(int)
    busy = multi_stream = multi_queue = 0
    last = None
    for t, kind, stream, queue in ev:
        if last is not None and t > last:
            n_s = sum(1 for v in active_s.values() if v > 0)
            n_q = sum(1 for v in active_q.values() if v > 0)
            if n_s >= 1:
                busy += t - last
            if n_s >= 2:
                multi_stream += t - last
            if n_q >= 2:
                multi_queue += t - last
        active_s[stream] += kind
        active_q[queue] += kind
        last = t
    streams = sorted({d[2] for d in dispatches})
    queues = sorted({d[3] for d in dispatches})
    window = (max(d[1] for d in dispatches) - min(d[0] for d in dispatches)) if dispatches else 0
    return {"dispatches": len(dispatches), "streams": streams, "queues": queues,
            "window_ms": window / 1e6, "busy_ms": busy / 1e6,
            "busy_frac_of_window": (busy / window) if window else 0.0,
            "two_or_more_streams_ms": multi_stream / 1e6,
            "two_or_more_queues_ms": multi_queue / 1e6,
            "overlap_frac_of_busy": (multi_stream / busy) if busy else 0.0}


def main(argv):
    if len(argv) >= 2 and argv[0] == "overlap":
        pats = tuple(argv[2:])
        res = overlap(read_dispatches(argv[1], pats) if pats else serving_dispatches(argv[1]))
        for k, v in res.items():
            print("%s: %s" % (k, v))
        return 0
    if argv and argv[0] == "traffic":
        import argparse
        ap = argparse.ArgumentParser(prog="profiling traffic")
        ap.add_argument("--workload", required=True)
        ap.add_argument("--fetch", required=True)
        ap.add_argument("--write", required=True)
        ap.add_argument("--bench-log", required=True)
        ap.add_argument("--calib-mib", type=int, default=256)
        ap.add_argument("--builds", type=int, default=0)
        ap.add_argument("--out", default="")
        a = ap.parse_args(argv[1:])
        ent = traffic(a.workload, a.fetch, a.write, a.bench_log, a.calib_mib, a.builds)
        print(json.dumps({a.workload: ent}, indent=1))
        if a.out:
            data = {}
            if os.path.exists(a.out):
                with open(a.out) as f:
                    data = json.load(f)
            data[a.workload] = ent
            data["kernel_hash"] = ent["kernel_hash"]
            with open(a.out, "w") as f:
                json.dump(data, f, indent=1)
        return 0
    print(__doc__)
    return 2


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
