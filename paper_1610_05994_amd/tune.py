"""Autotuner for the tile geometry of the level pass.

The domain decomposition of the paper (Section 3.2) leaves the segment size
free.  Here a segment is the tile that one wavefront splits: 64 lanes x
``lane_bytes`` bytes of symbols (32, 64 or 128 bytes, at most 64 symbols per
lane).  Small tiles give short sequences more wavefronts; large tiles spread
the per-tile prefix, node-span and counter work over more symbols.  A short
sequence may instead be built whole by one workgroup in LDS (geometry 1:
64 KB, geometry 2: 160 KB).
Which wins depends on the width, the depth and the length, and differs
between a build on its own and a batched build of many sequences, so both
are tuned.

``tune()`` times the library's builds for every valid geometry over a grid
of (width, levels, lg n) -- mode 0 with ``wt_build``, mode 1 with
``wt_build_batch`` over a batch of same-shaped sequences -- and keeps the
fastest.  The table is written as JSON; ``apply_table`` expands it to every
key (nearest measured grid point) through ``wt_tune_set``.  The binding
applies ``tune_table.json`` next to this file when it loads the library
(``WT_TUNE_TABLE`` names another file; an empty value disables it).

    python -m paper_1610_05994_amd.tune [--quick] [--out PATH]
    python -m paper_1610_05994_amd.tune --modes 0 --widths 2 4 --merge

(``--merge`` measures only the given modes and widths and keeps the other
points of the existing table.)
"""
from __future__ import annotations

import argparse
import json
import os
import time

from . import wtree as wt

TABLE_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tune_table.json")

# representative depths per width (u8 text / byte alphabets, u16 mid-size
# alphabets, u32 large alphabets) and lengths from short to long
GRID_LEVELS = {1: (2, 5, 8), 2: (6, 12, 16), 4: (12, 20, 24)}
GRID_LG_N = (10, 12, 14, 16, 18, 20, 22, 24, 26, 28)
BATCH_SYMBOLS = 1 << 24   # symbols per timed batch in mode 1
BATCH_MAX = 2048
BATCH_WORK_CAP = 8 << 30  # workspace bytes of one timed batch


# one workgroup per sequence, every level in LDS: 512 threads in 64 KB,
# 1024 threads in 160 KB, with the longest sequence each takes
GEOM_SMALL, GEOM_MID = 1, 2
ONE_WG_CAP = {GEOM_SMALL: {1: 15360, 2: 10240, 4: 6144}, GEOM_MID: {1: 32768, 2: 26624, 4: 15360}}


def candidates(width: int, n: int | None = None):
    """Valid geometries for a width (and length): lane bytes of the tiled
    level passes, plus the one-workgroup builds where the length fits."""
    out = [lb for lb in (32, 64, 128) if lb // width <= 64]
    if n is not None:
        out = [g for g in (GEOM_SMALL, GEOM_MID) if n <= ONE_WG_CAP[g][width]] + out
    return out


def _input(torch, n: int, levels: int, width: int, gen):
    hi = 1 << levels
    x = torch.randint(0, hi, (n,), generator=gen, device="cuda", dtype=torch.int64)
    return x.to({1: torch.uint8, 2: torch.int16, 4: torch.int32}[width])


def _time_single(torch, S, sigma: int, width: int, reps: int) -> float:
    n = S.numel()
    rc, tb, wb = wt.wt_footprint(n, sigma, width)
    if rc != wt.WT_OK:
        raise wt.WtError(rc, "wt_footprint")
    tree = torch.empty(max(tb, 256), dtype=torch.uint8, device="cuda")
    work = torch.empty(max(wb, 256), dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream()
    sh = int(st.cuda_stream)

    def once():
        rc, h = wt.wt_build(S.data_ptr(), n, sigma, width, tree.data_ptr(), tree.numel(), work.data_ptr(),
                            work.numel(), sh)
        if rc != wt.WT_OK:
            raise wt.WtError(rc, "wt_build")
        return h

    wt.wt_free(once())
    torch.cuda.synchronize()
    hs = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        hs.append(once())
    e1.record(st)
    torch.cuda.synchronize()
    for h in hs:
        wt.wt_free(h)
    return e0.elapsed_time(e1) / reps


def _time_batch(torch, Ss, sigma: int, width: int, reps: int) -> float:
    import ctypes
    m = len(Ss)
    descs = [(S.numel(), sigma, width) for S in Ss]
    trees, tbytes = [], []
    for d in descs:
        rc, tb, _ = wt.wt_footprint(*d)
        if rc != wt.WT_OK:
            raise wt.WtError(rc, "wt_footprint")
        trees.append(torch.empty(max(tb, 256), dtype=torch.uint8, device="cuda"))
        tbytes.append(trees[-1].numel())
    rc, wb = wt.wt_batch_footprint(descs)
    if rc != wt.WT_OK:
        raise wt.WtError(rc, "wt_batch_footprint")
    work = torch.empty(max(wb, 256), dtype=torch.uint8, device="cuda")
    st = torch.cuda.current_stream()
    # marshal once, so that the timed region holds the library's own work
    c_S = (ctypes.c_void_p * m)(*[S.data_ptr() for S in Ss])
    c_d = (wt.wt_desc * m)(*[wt.wt_desc(*d) for d in descs])
    c_t = (ctypes.c_void_p * m)(*[t.data_ptr() for t in trees])
    c_tb = (ctypes.c_uint64 * m)(*tbytes)
    c_h = (ctypes.c_void_p * m)()
    L = wt.lib()

    def once():
        rc = L.wt_build_batch(m, c_S, c_d, c_t, c_tb, work.data_ptr(), work.numel(), int(st.cuda_stream), c_h)
        if rc != wt.WT_OK:
            raise wt.WtError(rc, "wt_build_batch")
        return list(c_h)

    for h in once():
        wt.wt_free(h)
    torch.cuda.synchronize()
    held = []
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        held.extend(once())   # handles are released after the timed region
    e1.record(st)
    torch.cuda.synchronize()
    for h in held:
        wt.wt_free(h)
    return e0.elapsed_time(e1) / reps


def _batch_count(n: int, sigma: int, width: int, levels: int, lg_n: int) -> int:
    """Sequences per timed batch: about BATCH_SYMBOLS symbols, with the
    workspace of the most demanding geometry under BATCH_WORK_CAP."""
    cnt = max(1, min(BATCH_MAX, BATCH_SYMBOLS // n))
    ws1 = 256
    for g in candidates(width, n):
        wt.wt_tune_set(1, width, levels, lg_n, g)
        rc, ws = wt.wt_batch_footprint([(n, sigma, width)])
        if rc != wt.WT_OK:
            raise wt.WtError(rc, "wt_batch_footprint")
        ws1 = max(ws1, ws)
    wt.wt_tune_set(1, width, levels, lg_n, 0)
    return max(1, min(cnt, BATCH_WORK_CAP // ws1))


def tune(quick: bool = False, reps: int = 5, seed: int = 1, log=print, modes=(0, 1), widths=(1, 2, 4)):
    """Measure every geometry over the grid (of the given modes and widths);
    returns the table dict."""
    import torch

    gen = torch.Generator(device="cuda")
    gen.manual_seed(seed)
    lg_ns = GRID_LG_N[::2] if quick else GRID_LG_N
    entries = []
    for mode in modes:
        for width, levels_list in GRID_LEVELS.items():
            if width not in widths:
                continue
            for levels in levels_list:
                sigma = 1 << levels
                for lg_n in lg_ns:
                    n = 1 << lg_n
                    if mode == 0:
                        inputs = _input(torch, n, levels, width, gen)
                    else:
                        if n > BATCH_SYMBOLS // 4:
                            continue   # long sequences are batched rarely; mode 0 covers them
                        cnt = _batch_count(n, sigma, width, levels, lg_n)
                        flat = _input(torch, cnt * n, levels, width, gen)
                        inputs = [flat[k * n:(k + 1) * n] for k in range(cnt)]
                    times = {}
                    for lb in candidates(width, n):
                        rc = wt.wt_tune_set(mode, width, levels, lg_n, lb)
                        if rc != wt.WT_OK:
                            raise wt.WtError(rc, "wt_tune_set")
                        if mode == 0:
                            times[lb] = _time_single(torch, inputs, sigma, width, reps)
                        else:
                            times[lb] = _time_batch(torch, inputs, sigma, width, reps)
                    wt.wt_tune_set(mode, width, levels, lg_n, 0)
                    best = min(times, key=times.get)
                    entries.append(dict(mode=mode, width=width, levels=levels, lg_n=lg_n, lane_bytes=best,
                                        ms={str(k): round(v, 5) for k, v in times.items()}))
                    log("mode %d w%d l%-2d lg%-2d  %s  -> %d" % (
                        mode, width, levels, lg_n, "  ".join("%d:%.4f" % kv for kv in times.items()), best),
                        flush=True)
                    del inputs
    return dict(device=torch.cuda.get_device_name(0), reps=reps, entries=entries)


def expand(entries):
    """Dense table {(mode, width, levels, lg_n): lane_bytes} from measured points.

    Each key takes the measured point of the same mode and width that is
    nearest in levels, then in lg n (mode 1 falls back to mode 0 for lengths
    it did not measure)."""
    out = {}
    by = {}
    for e in entries:
        by.setdefault((e["mode"], e["width"]), []).append(e)
    for mode in (0, 1):
        for width in (1, 2, 4):
            pts = by.get((mode, width), [])
            pts0 = by.get((0, width), [])
            for levels in range(1, min(24, 8 * width) + 1):
                for lg_n in range(0, 41):
                    cand = pts
                    if mode == 1 and pts and lg_n > max(p["lg_n"] for p in pts) + 1:
                        cand = pts0
                    if not cand:
                        continue
                    best = min(cand, key=lambda p: (abs(p["levels"] - levels), abs(p["lg_n"] - lg_n)))
                    out[(mode, width, levels, lg_n)] = int(best["lane_bytes"])
    return out


def apply_table(table) -> int:
    """wt_tune_set for every key of a table dict; returns the keys set."""
    dense = expand(table.get("entries", []))
    for (mode, width, levels, lg_n), lb in dense.items():
        rc = wt.wt_tune_set(mode, width, levels, lg_n, lb)
        if rc != wt.WT_OK:
            raise wt.WtError(rc, "wt_tune_set")
    return len(dense)


def load(path: str | None = None) -> int:
    """Apply a table file (default: tune_table.json beside this module)."""
    path = path or TABLE_PATH
    if not os.path.exists(path):
        return 0
    with open(path) as f:
        return apply_table(json.load(f))


def reset() -> None:
    """Back to the built-in default geometry for every key."""
    for mode in (0, 1):
        for width in (1, 2, 4):
            for levels in range(1, min(24, 8 * width) + 1):
                for lg_n in range(0, 41):
                    wt.wt_tune_set(mode, width, levels, lg_n, 0)


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--quick", action="store_true", help="every other length of the grid")
    ap.add_argument("--reps", type=int, default=5)
    ap.add_argument("--out", default=TABLE_PATH)
    ap.add_argument("--modes", type=int, nargs="+", default=[0, 1], choices=[0, 1])
    ap.add_argument("--widths", type=int, nargs="+", default=[1, 2, 4], choices=[1, 2, 4])
    ap.add_argument("--merge", action="store_true",
                    help="replace only the measured (mode, width) points of the table at --out")
    args = ap.parse_args()
    os.environ["WT_TUNE_TABLE"] = ""      # measure from the defaults
    table = tune(quick=args.quick, reps=args.reps, modes=tuple(args.modes), widths=tuple(args.widths))
    if args.merge and os.path.exists(args.out):
        with open(args.out) as f:
            old = json.load(f)
        done = {(e["mode"], e["width"]) for e in table["entries"]}
        table["entries"] = [e for e in old.get("entries", []) if (e["mode"], e["width"]) not in done] + \
            table["entries"]
    with open(args.out, "w") as f:
        json.dump(table, f, indent=1)
    print("wrote %s (%d points)" % (args.out, len(table["entries"])))


if __name__ == "__main__":
    main()
