"""Serving loop: continuous batching of wavelet-tree builds on one GPU.

Build requests arrive over time (each with its sequence already in device
memory).  The server

* admits a request when its HBM footprint -- tree memory from
  ``wt_footprint`` plus its share of the batch workspace from
  ``wt_batch_footprint`` -- fits in a fixed device arena, evicting resident
  trees (least recently used) when it must, and queues it otherwise; a
  request that could never fit is rejected;
* launches every request admitted in one scheduling pass as one
  ``wt_build_batch`` call, followed by that batch's rank/select queries, on
  the next of a few streams, so batches admitted while earlier ones still
  run overlap on the device (continuous batching: new work joins as slots
  and memory free up, it does not wait for a whole batch to drain);
* keeps every built tree resident in the arena for further queries until it
  is released, cancelled or evicted;
* records per request arrival, admission and completion times, from which
  p50/p99 latency and throughput follow.

Every build and query runs in the library's HIP kernels; the arena is one
torch allocation carved by offsets (PyTorch provides memory and streams
only).  The arena bookkeeping (``Arena``) is plain Python over offsets.
"""
from __future__ import annotations

import bisect
import time
from dataclasses import dataclass, field

import numpy as np

from . import wtree as wt

ALIGN = 256


class Arena:
    """First-fit allocator over [0, size) in ALIGN-byte units, coalescing
    free neighbours.  Pure bookkeeping: offsets only."""

    def __init__(self, size: int):
        self.size = size - size % ALIGN
        self.free_list = [(0, self.size)] if self.size else []   # sorted (offset, length)
        self.live = {}                                           # offset -> length
        self.used = 0
        self.high_water = 0

    @staticmethod
    def _round(n: int) -> int:
        return max(ALIGN, (n + ALIGN - 1) // ALIGN * ALIGN)

    def largest_free(self) -> int:
        return max((ln for _, ln in self.free_list), default=0)

    def alloc(self, nbytes: int):
        """Offset of a new block of at least nbytes, or None if none fits."""
        need = self._round(nbytes)
        for k, (off, ln) in enumerate(self.free_list):
            if ln >= need:
                if ln == need:
                    del self.free_list[k]
                else:
                    self.free_list[k] = (off + need, ln - need)
                self.live[off] = need
                self.used += need
                self.high_water = max(self.high_water, self.used)
                return off
        return None

    def free(self, off: int) -> None:
        ln = self.live.pop(off)
        self.used -= ln
        k = bisect.bisect_left(self.free_list, (off, 0))
        # merge with the following and the preceding free block
        if k < len(self.free_list) and self.free_list[k][0] == off + ln:
            ln += self.free_list[k][1]
            del self.free_list[k]
        if k > 0 and self.free_list[k - 1][0] + self.free_list[k - 1][1] == off:
            poff, pln = self.free_list[k - 1]
            self.free_list[k - 1] = (poff, pln + ln)
        else:
            self.free_list.insert(k, (off, ln))

    def check(self) -> None:
        """Invariants: blocks disjoint, sorted, coalesced, and covering the arena."""
        spans = sorted([(o, l, "free") for o, l in self.free_list] + [(o, l, "live") for o, l in self.live.items()])
        pos = 0
        for k, (o, l, kind) in enumerate(spans):
            assert o == pos, "gap or overlap at %d" % o
            assert l > 0 and l % ALIGN == 0
            if kind == "free" and k > 0:
                assert spans[k - 1][2] != "free", "uncoalesced free blocks"
            pos = o + l
        assert pos == self.size
        assert self.used == sum(self.live.values())


QUEUED, RUNNING, RESIDENT, RELEASED, CANCELLED, REJECTED = "queued", "running", "resident", "released", \
    "cancelled", "rejected"


@dataclass
class Request:
    """One build request: sequence S (device tensor of width-byte symbols),
    alphabet size sigma, and optional rank / select queries (host arrays)."""
    rid: int
    S: object
    sigma: int
    arrival: float = 0.0
    rank_c: np.ndarray | None = None
    rank_i: np.ndarray | None = None
    sel_c: np.ndarray | None = None
    sel_j: np.ndarray | None = None
    # filled by the server
    state: str = QUEUED
    width: int = 0
    n: int = 0
    t_admit: float = 0.0
    t_done: float = 0.0
    tree_off: int = -1
    tree_bytes: int = 0
    ws_solo: int = 0
    handle: int = 0
    status: int = -1
    rank_out: np.ndarray | None = None
    sel_out: np.ndarray | None = None
    last_use: float = 0.0
    error: str = ""

    @property
    def latency(self) -> float:
        return self.t_done - self.arrival


@dataclass
class _Batch:
    reqs: list
    stream: object
    event: object
    work_off: int
    host: object          # pinned answers + status words
    dev: object           # device answers (kept alive until done)
    nq: list = field(default_factory=list)


class Server:
    """Continuous-batching build server over one device arena."""

    def __init__(self, budget_bytes: int, streams: int = 4, max_batch: int = 512, max_inflight: int = 8,
                 device="cuda:0", clock=time.perf_counter):
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.arena = Arena(budget_bytes)
        self.mem = torch.empty(self.arena.size, dtype=torch.uint8, device=self.device)
        self.base = self.mem.data_ptr()
        self.streams = [torch.cuda.Stream(device=self.device) for _ in range(max(1, streams))]
        self.next_stream = 0
        self.max_batch = max_batch
        self.max_inflight = max_inflight
        self.clock = clock
        self.queue: list[Request] = []
        self.inflight: list[_Batch] = []
        self.resident: dict[int, Request] = {}
        self.all: dict[int, Request] = {}
        self.batches_launched = 0
        self.cancel_pending: set = set()

    # ------------------------------------------------------------ client --
    def submit(self, req: Request) -> None:
        req.width = req.S.element_size()
        req.n = req.S.numel()
        rc, tb, _ = wt.wt_footprint(req.n, req.sigma, req.width)
        if rc == wt.WT_OK:
            rc, ws = wt.wt_batch_footprint([(req.n, req.sigma, req.width)])
        self.all[req.rid] = req
        if rc != wt.WT_OK:
            req.state, req.error = REJECTED, wt.strerror(rc)
            req.t_done = self.clock()
            return
        if Arena._round(tb) + Arena._round(ws) > self.arena.size:
            # it would not fit even in an empty arena
            req.state, req.error = REJECTED, "footprint exceeds the arena"
            req.t_done = self.clock()
            return
        req.tree_bytes, req.ws_solo = tb, ws
        req.state = QUEUED
        self.all[req.rid] = req
        self.queue.append(req)

    def cancel(self, rid: int) -> None:
        """Queued: dropped.  Running: dropped when its batch completes.
        Resident: its tree memory is freed now."""
        req = self.all[rid]
        if req.state == QUEUED:
            self.queue.remove(req)
            req.state = CANCELLED
        elif req.state == RUNNING:
            self.cancel_pending.add(rid)
        elif req.state == RESIDENT:
            self._drop_resident(req, CANCELLED)

    def release(self, rid: int) -> None:
        req = self.all[rid]
        if req.state == RESIDENT:
            self._drop_resident(req, RELEASED)

    def tree_bitmaps(self, rid: int) -> np.ndarray:
        """Level bitmaps of a resident tree (host copy)."""
        req = self.all[rid]
        assert req.state == RESIDENT, req.state
        req.last_use = self.clock()
        rc, info = wt.wt_levels(req.handle)
        if rc != wt.WT_OK:
            raise wt.WtError(rc, "wt_levels")
        off = info["bitmaps"] - self.base
        cnt = info["levels"] * info["words_per_level"]
        return self.mem[off: off + 8 * cnt].cpu().numpy().view(np.uint64).reshape(info["levels"], -1)

    def query_rank(self, rid: int, c, i) -> np.ndarray:
        """Rank queries on a resident tree (synchronous helper)."""
        req = self.all[rid]
        assert req.state == RESIDENT, req.state
        req.last_use = self.clock()
        torch = self.torch
        c = torch.as_tensor(np.asarray(c, np.int32), device=self.device)
        i = torch.as_tensor(np.asarray(i, np.int64), device=self.device)
        out = torch.empty(c.numel(), dtype=torch.int64, device=self.device)
        st = torch.cuda.current_stream(self.device)
        rc = wt.wt_rank_batch(req.handle, c.data_ptr(), i.data_ptr(), out.data_ptr(), c.numel(), int(st.cuda_stream))
        if rc != wt.WT_OK:
            raise wt.WtError(rc, "wt_rank_batch")
        return out.cpu().numpy().view(np.uint64)

    # --------------------------------------------------------- scheduling --
    def _drop_resident(self, req: Request, state: str) -> None:
        self.resident.pop(req.rid, None)
        if req.handle:
            wt.wt_free(req.handle)
            req.handle = 0
        if req.tree_off >= 0:
            self.arena.free(req.tree_off)
            req.tree_off = -1
        req.state = state

    def _evict_one(self) -> bool:
        if not self.resident:
            return False
        victim = min(self.resident.values(), key=lambda r: r.last_use)
        self._drop_resident(victim, RELEASED)
        return True

    def poll(self) -> int:
        """Retire completed batches (in any order); returns how many."""
        done = 0
        keep = []
        for b in self.inflight:
            if b.event.query():
                self._complete(b)
                done += 1
            else:
                keep.append(b)
        self.inflight = keep
        return done

    def _complete(self, b: _Batch) -> None:
        now = self.clock()
        self.arena.free(b.work_off)
        host = b.host.numpy()
        m = len(b.reqs)
        k = m
        for q, req in enumerate(b.reqs):
            req.status = wt.WT_ERANGE if (int(host[q]) & 1) else wt.WT_OK
            nr, ns = b.nq[q]
            req.rank_out = host[k: k + nr].view(np.uint64).copy() if nr else np.zeros(0, np.uint64)
            k += nr
            req.sel_out = host[k: k + ns].view(np.uint64).copy() if ns else np.zeros(0, np.uint64)
            k += ns
            req.t_done = now
            req.last_use = now
            if req.rid in self.cancel_pending:
                self.cancel_pending.discard(req.rid)
                self._drop_resident(req, CANCELLED)
            else:
                req.state = RESIDENT
                self.resident[req.rid] = req

    def _admit(self):
        """Pick queued requests (FIFO) whose trees and workspace fit.

        The sum of the members' solo workspaces must stay free (contiguously)
        after the trees are placed.  A batch's workspace is usually less than
        that sum, but not always (which long sequences are built alone depends
        on the batch): if it does not fit, the last members go back to the
        head of the queue."""
        picked, descs, tree_offs = [], [], []
        ws_sum = 0
        while self.queue and len(picked) < self.max_batch:
            req = self.queue[0]
            off = self.arena.alloc(req.tree_bytes)
            if off is not None and self.arena.largest_free() >= ws_sum + req.ws_solo:
                picked.append(self.queue.pop(0))
                descs.append((req.n, req.sigma, req.width))
                tree_offs.append(off)
                ws_sum += req.ws_solo
                continue
            if off is not None:
                self.arena.free(off)
            if picked:
                break                  # launch these; the rest waits
            if self._evict_one():
                continue               # make room from resident trees (LRU)
            break                      # wait for running batches to free memory
        if not picked:
            return None
        while True:
            rc, ws = wt.wt_batch_footprint(descs)
            if rc != wt.WT_OK:
                raise wt.WtError(rc, "wt_batch_footprint")
            work_off = self.arena.alloc(ws)
            if work_off is not None:
                return picked, descs, tree_offs, work_off
            # (one request alone always fits: its solo workspace was checked)
            assert len(picked) > 1
            self.arena.free(tree_offs.pop())
            descs.pop()
            self.queue.insert(0, picked.pop())

    def _launch(self, picked, descs, tree_offs, work_off) -> None:
        torch = self.torch
        st = self.streams[self.next_stream]
        self.next_stream = (self.next_stream + 1) % len(self.streams)
        m = len(picked)
        now = self.clock()
        tbytes = [r.tree_bytes for r in picked]
        ptrs_S = [r.S.data_ptr() if r.n else 0 for r in picked]
        ptrs_T = [self.base + o for o in tree_offs]
        # the inputs were written on the client's stream: order after it
        st.wait_stream(torch.cuda.current_stream(self.device))
        rc, hs = wt.wt_build_batch(ptrs_S, descs, ptrs_T, tbytes, self.base + work_off,
                                   self.arena.live[work_off], int(st.cuda_stream))
        if rc != wt.WT_OK:
            for o in tree_offs:
                self.arena.free(o)
            self.arena.free(work_off)
            for r in picked:
                r.state, r.error, r.t_done = REJECTED, wt.strerror(rc), now
            return
        nq = []
        tot = 0
        for r in picked:
            nr = 0 if r.rank_c is None else len(r.rank_c)
            ns = 0 if r.sel_c is None else len(r.sel_c)
            nq.append((nr, ns))
            tot += nr + ns
        # every query of the batch in one launch: per query its tree, kind
        # (1 rank, 2 select), symbol and argument
        qt = np.repeat(np.arange(m, dtype=np.uint32), [a + b for a, b in nq]) if tot else np.zeros(0, np.uint32)
        qk = np.concatenate([np.concatenate([np.full(a, 1, np.uint8), np.full(b, 2, np.uint8)]) for a, b in nq]) \
            if tot else np.zeros(0, np.uint8)
        empty32, empty64 = np.zeros(0, np.int32), np.zeros(0, np.int64)
        qc = np.concatenate([np.concatenate([r.rank_c if r.rank_c is not None else empty32,
                                             r.sel_c if r.sel_c is not None else empty32]) for r in picked]) \
            .astype(np.int32) if tot else empty32
        qx = np.concatenate([np.concatenate([r.rank_i if r.rank_i is not None else empty64,
                                             r.sel_j if r.sel_j is not None else empty64]) for r in picked]) \
            .astype(np.int64) if tot else empty64
        with torch.cuda.stream(st):
            dev = torch.empty(m + tot, dtype=torch.int64, device=self.device)
            # status words of the trees (first 4 bytes of each tree)
            offs = torch.tensor([o // 4 for o in tree_offs], dtype=torch.int64, device=self.device)
            dev[:m] = self.mem.view(torch.int32).index_select(0, offs).to(torch.int64)
            packed = None
            if tot:
                # one host-to-device copy for all query arguments
                blob = np.concatenate([qx.view(np.uint8), qc.view(np.uint8), qt.view(np.uint8), qk])
                packed = torch.from_numpy(blob).to(self.device)
                rc_w, wb = wt.wt_query_multi_footprint(m)
                views = torch.empty(wb, dtype=torch.uint8, device=self.device)
                base = packed.data_ptr()
                rc = wt.wt_query_multi(hs, base + 12 * tot, base + 16 * tot, base + 8 * tot, base,
                                       dev.data_ptr() + 8 * m, tot, views.data_ptr(), wb, int(st.cuda_stream))
                if rc != wt.WT_OK:
                    raise wt.WtError(rc, "wt_query_multi")
                packed = (packed, views)
        for q, (r, h) in enumerate(zip(picked, hs)):
            r.handle, r.tree_off, r.t_admit, r.state = h, tree_offs[q], now, RUNNING
        host = torch.empty(m + tot, dtype=torch.int64, pin_memory=True)
        with torch.cuda.stream(st):
            host.copy_(dev, non_blocking=True)
            ev = torch.cuda.Event()
            ev.record(st)
        self.inflight.append(_Batch(picked, st, ev, work_off, host, (dev, packed, offs), nq))
        self.batches_launched += 1

    def step(self) -> bool:
        """One scheduling pass: retire finished batches, launch admissible
        queued requests.  Returns True if anything happened."""
        did = self.poll() > 0
        if self.queue and len(self.inflight) < self.max_inflight:
            adm = self._admit()
            if adm is not None:
                self._launch(*adm)
                did = True
        return did

    def drain(self, timeout: float = 120.0) -> None:
        t0 = self.clock()
        while self.queue or self.inflight:
            if not self.step():
                if self.inflight:
                    self.inflight[0].event.synchronize()
                elif self.queue:
                    raise RuntimeError("requests cannot be admitted: %d queued" % len(self.queue))
            if self.clock() - t0 > timeout:
                raise TimeoutError("drain")

    def run_stream(self, reqs, timeout: float = 600.0):
        """Serve requests whose .arrival are offsets (s) from now; returns
        when every one has completed or been rejected."""
        t0 = self.clock()
        pending = sorted(reqs, key=lambda r: r.arrival)
        for r in pending:
            r.arrival += t0
        k = 0
        while k < len(pending) or self.queue or self.inflight:
            now = self.clock()
            while k < len(pending) and pending[k].arrival <= now:
                self.submit(pending[k])
                k += 1
            if not self.step():
                if k < len(pending) and not self.inflight:
                    wait = pending[k].arrival - self.clock()
                    if wait > 2e-4:
                        time.sleep(wait - 1e-4)
            if self.clock() - t0 > timeout:
                raise TimeoutError("run_stream")
        return reqs

    def close(self) -> None:
        self.drain()
        for r in list(self.resident.values()):
            self._drop_resident(r, RELEASED)


# ------------------------------------------------------------ workloads --

def resolve_queries(draws, n: int, sigma: int, counts: np.ndarray):
    """Turn (kind, c, x) draws into rank (c, i) and select (c, j) arguments:
    rank takes i uniform in [0, n]; select takes j uniform in [1, occ(c)]
    when c occurs (j = 1 otherwise, whose answer is 'none')."""
    rc, ri, sc, sj = [], [], [], []
    for kind, c, x in draws:
        c = int(c) % sigma
        if kind == 0:
            rc.append(c)
            ri.append(min(n, int(x * (n + 1))))
        else:
            occ = int(counts[c]) if c < len(counts) else 0
            sc.append(c)
            sj.append(1 + min(occ - 1, int(x * occ)) if occ else 1)
    return (np.array(rc, np.int32), np.array(ri, np.int64), np.array(sc, np.int32), np.array(sj, np.int64))


def _gen_one(sp):
    import wtgen
    S = wtgen.serve_input(sp)
    counts = np.bincount(S, minlength=sp["sigma"]) if sp["n"] else np.zeros(sp["sigma"], np.int64)
    return S, counts


def make_pool(specs, device, workers: int = 1):
    """Device copies of the sequences of serving specs (wtgen.serve_stream
    entries), with their symbol counts for query resolution.  workers > 1
    draws the sequences in that many fresh worker processes (spawned, so no
    child inherits the parent's GPU state); the bytes are the same."""
    if workers > 1 and len(specs) > 1:
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
            made = list(ex.map(_gen_one, specs))
    else:
        made = [_gen_one(sp) for sp in specs]
    pool = []
    for sp, (S, counts) in zip(specs, made):
        pool.append(dict(S=wt.to_device(S, device), host=S, sigma=sp["sigma"], n=sp["n"], counts=counts))
    return pool


def requests_from(pool, arrivals, rid0: int = 0):
    """Requests for wtgen.pool_stream arrivals over a pool."""
    reqs = []
    for k, a in enumerate(arrivals):
        p = pool[a["pool"]]
        rc, ri, sc, sj = resolve_queries(a["queries"], p["n"], p["sigma"], p["counts"])
        reqs.append(Request(rid=rid0 + k, S=p["S"], sigma=p["sigma"], arrival=a["t"], rank_c=rc, rank_i=ri,
                            sel_c=sc, sel_j=sj))
    return reqs


def summarize(reqs, t_first=None, t_last=None) -> dict:
    """Latency percentiles (ms) and throughput over completed requests."""
    done = [r for r in reqs if r.state in (RESIDENT, RELEASED) and r.t_done > 0]
    if not done:
        return dict(completed=0)
    lat = np.array([r.latency for r in done]) * 1e3
    wait = np.array([r.t_admit - r.arrival for r in done]) * 1e3
    t0 = min(r.arrival for r in done) if t_first is None else t_first
    t1 = max(r.t_done for r in done) if t_last is None else t_last
    syms = sum(r.n for r in done)
    return dict(completed=len(done), rejected=sum(r.state == REJECTED for r in reqs),
                p50_ms=float(np.percentile(lat, 50)), p99_ms=float(np.percentile(lat, 99)),
                mean_ms=float(lat.mean()), max_ms=float(lat.max()),
                queue_p50_ms=float(np.percentile(wait, 50)), queue_p99_ms=float(np.percentile(wait, 99)),
                symbols=int(syms), seconds=float(t1 - t0), symbols_per_s=float(syms / max(t1 - t0, 1e-9)))

