"""Summaries of rocprofv3 kernel traces (``--kernel-trace --output-format csv``).

``python -m paper_1610_05994_amd.profiling overlap TRACE.csv [PATTERN ...]``
reports, for the dispatches whose kernel name contains one of the patterns
(default: the batched-build and multi-tree query kernels of the serving
loop), how long kernels of two or more different streams ran at the same
time on the device, against the time any of them ran: the evidence that
batches launched on different streams overlap.
"""
from __future__ import annotations

import csv
import sys
from collections import defaultdict

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
    if len(argv) < 2 or argv[0] != "overlap":
        print(__doc__)
        return 2
    pats = tuple(argv[2:]) or SERVE_KERNELS
    res = overlap(read_dispatches(argv[1], pats))
    for k, v in res.items():
        print("%s: %s" % (k, v))
    return 0


if __name__ == "__main__":
    sys.exit(main(sys.argv[1:]))
