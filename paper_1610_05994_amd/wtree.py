"""ctypes binding of libwtree.so (include/wtree.h).

The functions ``wt_*`` below carry the same names and arguments as the C
ABI and only marshal arguments; every step of a build or query runs in the
HIP kernels of the library.  ``Tree``/``build`` add torch-allocated device
memory and streams on top (PyTorch is used for memory and streams only).

Loading fails loudly if the library has not been built: there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
# WT_LIBRARY names another build of the library (e.g. the write-counting
# build, libwtree_check.so, beside this module)
LIB_PATH = os.environ.get("WT_LIBRARY") or os.path.join(_PKG, "libwtree.so")
CHECK_LIB_PATH = os.path.join(_PKG, "libwtree_check.so")

WT_OK, WT_EINVAL, WT_ERANGE, WT_ENOMEM, WT_ENOTFOUND, WT_EDEVICE = range(6)
WT_MAX_SIGMA = 1 << 24

EXPORTED = [
    "wt_footprint", "wt_build", "wt_build_matrix", "wt_matrix_zeros", "wt_batch_footprint", "wt_build_batch", "wt_tree_status",
    "wt_free", "wt_levels", "wt_access_batch", "wt_rank_batch", "wt_select_batch",
    "wt_access", "wt_rank", "wt_select", "wt_query_multi_footprint", "wt_query_multi", "wt_strerror",
    "wt_tune_set", "wt_tune_get", "wt_buffered_footprint", "wt_build_buffered",
    "wt_multiary_footprint", "wt_build_multiary", "wt_multiary_levels",
    "wt_prof_enable", "wt_prof_read", "wt_build_noalloc", "wt_debug_write_counters",
    "wt_histogram", "wt_huffman_footprint", "wt_build_huffman", "wt_huffman_levels",
]
HUFF_MAX_LEVELS = 24
WT_NOALLOC_WORK_BYTES = 64 << 20


class WtError(RuntimeError):
    def __init__(self, status: int, what: str = ""):
        self.status = status
        super().__init__("%s: %s (status %d)" % (what or "wtree", strerror(status), status))


class wt_desc(ctypes.Structure):
    _fields_ = [("n", ctypes.c_uint64), ("sigma", ctypes.c_uint32), ("width", ctypes.c_uint32)]


class wt_prof_rec(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_char * 32), ("level", ctypes.c_uint32), ("width", ctypes.c_uint32),
                ("n", ctypes.c_uint64), ("bytes", ctypes.c_uint64), ("ms", ctypes.c_float)]


_lib = None


def lib():
    """The loaded library; raises if libwtree.so is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libwtree.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    vp, u32, u64, i32 = ctypes.c_void_p, ctypes.c_uint32, ctypes.c_uint64, ctypes.c_int
    P = ctypes.POINTER
    sig = {
        "wt_footprint": ([P(wt_desc), P(u64), P(u64)], i32),
        "wt_build": ([vp, P(wt_desc), vp, u64, vp, u64, vp, P(vp)], i32),
        "wt_build_matrix": ([vp, P(wt_desc), vp, u64, vp, u64, vp, P(vp)], i32),
        "wt_build_noalloc": ([vp, P(wt_desc), vp, u64, vp], i32),
        "wt_debug_write_counters": ([vp, vp, u64], i32),
        "wt_histogram": ([vp, P(wt_desc), vp, vp], i32),
        "wt_huffman_footprint": ([vp, P(wt_desc), P(u64), P(u64)], i32),
        "wt_build_huffman": ([vp, P(wt_desc), vp, vp, u64, vp, u64, vp, P(vp)], i32),
        "wt_huffman_levels": ([vp, P(u32), vp, vp, vp, vp, vp], i32),
        "wt_matrix_zeros": ([vp, P(u64)], i32),
        "wt_buffered_footprint": ([P(wt_desc), u64, P(u64), P(u64)], i32),
        "wt_multiary_footprint": ([P(wt_desc), P(u64), P(u64)], i32),
        "wt_build_multiary": ([vp, P(wt_desc), vp, u64, vp, u64, vp, P(vp)], i32),
        "wt_multiary_levels": ([vp, P(u32), P(vp), P(u64), P(vp), P(u64)], i32),
        "wt_build_buffered": ([vp, P(wt_desc), u64, vp, u64, vp, u64, vp, P(vp)], i32),
        "wt_batch_footprint": ([u32, P(wt_desc), P(u64)], i32),
        "wt_build_batch": ([u32, P(vp), P(wt_desc), P(vp), P(u64), vp, u64, vp, P(vp)], i32),
        "wt_tree_status": ([vp], i32),
        "wt_free": ([vp], None),
        "wt_levels": ([vp, P(u32), P(vp), P(u64), P(vp), P(u64), P(u64)], i32),
        "wt_access_batch": ([vp, vp, vp, u64, vp], i32),
        "wt_rank_batch": ([vp, vp, vp, vp, u64, vp], i32),
        "wt_select_batch": ([vp, vp, vp, vp, u64, vp], i32),
        "wt_access": ([vp, u64, P(u32)], i32),
        "wt_rank": ([vp, u32, u64, P(u64)], i32),
        "wt_select": ([vp, u32, u64, P(u64)], i32),
        "wt_strerror": ([i32], ctypes.c_char_p),
        "wt_query_multi_footprint": ([u32, P(u64)], i32),
        "wt_query_multi": ([u32, P(vp), vp, vp, vp, vp, vp, u64, vp, u64, vp], i32),
        "wt_tune_set": ([u32, u32, u32, u32, u32], i32),
        "wt_tune_get": ([u32, u32, u32, u32, P(u32)], i32),
        "wt_prof_enable": ([i32], i32),
        "wt_prof_read": ([P(wt_prof_rec), u64, P(u64)], i32),
    }
    for name, (args, res) in sig.items():
        f = getattr(L, name)
        f.argtypes = args
        f.restype = res
    _lib = L
    # tile geometry chosen by the autotuner (tune.py), if a table is present
    table = os.environ.get("WT_TUNE_TABLE")
    if table is None:
        table = os.path.join(_PKG, "tune_table.json")
    if table:
        from . import tune
        tune.load(table)
    return L


# ------------------------------------------------------------ raw C ABI ---

def strerror(status: int) -> str:
    return lib().wt_strerror(status).decode()


def wt_tune_set(mode: int, width: int, levels: int, lg_n: int, lane_bytes: int) -> int:
    return lib().wt_tune_set(mode, width, levels, lg_n, lane_bytes)


def wt_tune_get(mode: int, width: int, levels: int, lg_n: int):
    v = ctypes.c_uint32()
    rc = lib().wt_tune_get(mode, width, levels, lg_n, ctypes.byref(v))
    return rc, v.value


def wt_footprint(n: int, sigma: int, width: int):
    d = wt_desc(n, sigma, width)
    tb, wb = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib().wt_footprint(ctypes.byref(d), ctypes.byref(tb), ctypes.byref(wb))
    return rc, tb.value, wb.value


def wt_build(d_S: int, n: int, sigma: int, width: int, d_tree: int, tree_bytes: int, d_work: int,
             work_bytes: int, stream: int):
    d = wt_desc(n, sigma, width)
    h = ctypes.c_void_p()
    rc = lib().wt_build(d_S, ctypes.byref(d), d_tree, tree_bytes, d_work, work_bytes, stream, ctypes.byref(h))
    return rc, h.value


def wt_build_noalloc(d_S: int, n: int, sigma: int, width: int, d_tree: int, tree_bytes: int, stream: int) -> int:
    d = wt_desc(n, sigma, width)
    return lib().wt_build_noalloc(d_S, ctypes.byref(d), d_tree, tree_bytes, stream)


def wt_debug_write_counters(d_counts: int, d_base: int, nbytes: int) -> int:
    return lib().wt_debug_write_counters(d_counts, d_base, nbytes)


def wt_histogram(d_S: int, n: int, sigma: int, width: int, d_counts: int, stream: int) -> int:
    d = wt_desc(n, sigma, width)
    return lib().wt_histogram(d_S, ctypes.byref(d), d_counts, stream)


def wt_huffman_footprint(counts: np.ndarray, n: int, sigma: int, width: int):
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    d = wt_desc(n, sigma, width)
    tb, wb = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib().wt_huffman_footprint(counts.ctypes.data_as(ctypes.c_void_p), ctypes.byref(d), ctypes.byref(tb),
                                    ctypes.byref(wb))
    return rc, tb.value, wb.value


def wt_build_huffman(d_S: int, n: int, sigma: int, width: int, counts: np.ndarray, d_tree: int, tree_bytes: int,
                     d_work: int, work_bytes: int, stream: int):
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    d = wt_desc(n, sigma, width)
    h = ctypes.c_void_p()
    rc = lib().wt_build_huffman(d_S, ctypes.byref(d), counts.ctypes.data_as(ctypes.c_void_p), d_tree, tree_bytes,
                                d_work, work_bytes, stream, ctypes.byref(h))
    return rc, h.value


def wt_huffman_levels(h: int, sigma: int):
    lv = ctypes.c_uint32()
    arrs = [np.zeros(HUFF_MAX_LEVELS, dtype=np.uint64) for _ in range(4)]
    code = np.zeros(max(1, sigma), dtype=np.uint32)
    vp = ctypes.c_void_p
    rc = lib().wt_huffman_levels(h, ctypes.byref(lv), *[a.ctypes.data_as(vp) for a in arrs],
                                 code.ctypes.data_as(vp))
    L = lv.value
    return rc, dict(levels=L, sizes=[int(x) for x in arrs[0][:L]], bits_off=[int(x) for x in arrs[1][:L]],
                    dir_off=[int(x) for x in arrs[2][:L]], dir_entries=[int(x) for x in arrs[3][:L]],
                    code_table=code[:sigma])


def wt_build_matrix(d_S: int, n: int, sigma: int, width: int, d_tree: int, tree_bytes: int, d_work: int,
                    work_bytes: int, stream: int):
    d = wt_desc(n, sigma, width)
    h = ctypes.c_void_p()
    rc = lib().wt_build_matrix(d_S, ctypes.byref(d), d_tree, tree_bytes, d_work, work_bytes, stream,
                               ctypes.byref(h))
    return rc, h.value


def wt_matrix_zeros(h: int, levels: int):
    z = (ctypes.c_uint64 * max(1, levels))()
    rc = lib().wt_matrix_zeros(h, z)
    return rc, np.array(z[:levels], dtype=np.uint64)


def wt_multiary_footprint(n: int, sigma: int, width: int):
    d = wt_desc(n, sigma, width)
    tb, wb = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib().wt_multiary_footprint(ctypes.byref(d), ctypes.byref(tb), ctypes.byref(wb))
    return rc, tb.value, wb.value


def wt_build_multiary(d_S: int, n: int, sigma: int, width: int, d_tree: int, tree_bytes: int, d_work: int,
                      work_bytes: int, stream: int):
    d = wt_desc(n, sigma, width)
    h = ctypes.c_void_p()
    rc = lib().wt_build_multiary(d_S, ctypes.byref(d), d_tree, tree_bytes, d_work, work_bytes, stream,
                                 ctypes.byref(h))
    return rc, h.value


def wt_multiary_levels(h: int):
    lv, wpl, ds = ctypes.c_uint32(), ctypes.c_uint64(), ctypes.c_uint64()
    dig, dr = ctypes.c_void_p(), ctypes.c_void_p()
    rc = lib().wt_multiary_levels(h, ctypes.byref(lv), ctypes.byref(dig), ctypes.byref(wpl), ctypes.byref(dr),
                                  ctypes.byref(ds))
    return rc, dict(levels=lv.value, digits=dig.value or 0, words=wpl.value, dir=dr.value or 0,
                    dir_stride=ds.value)


def wt_buffered_footprint(n: int, sigma: int, width: int, buffer_syms: int):
    d = wt_desc(n, sigma, width)
    tb, wb = ctypes.c_uint64(), ctypes.c_uint64()
    rc = lib().wt_buffered_footprint(ctypes.byref(d), buffer_syms, ctypes.byref(tb), ctypes.byref(wb))
    return rc, tb.value, wb.value


def wt_build_buffered(S: int, n: int, sigma: int, width: int, buffer_syms: int, d_tree: int, tree_bytes: int,
                      d_work: int, work_bytes: int, stream: int):
    d = wt_desc(n, sigma, width)
    h = ctypes.c_void_p()
    rc = lib().wt_build_buffered(S, ctypes.byref(d), buffer_syms, d_tree, tree_bytes, d_work, work_bytes, stream,
                                 ctypes.byref(h))
    return rc, h.value


def wt_batch_footprint(descs):
    arr = (wt_desc * len(descs))(*[wt_desc(*d) for d in descs])
    wb = ctypes.c_uint64()
    rc = lib().wt_batch_footprint(len(descs), arr, ctypes.byref(wb))
    return rc, wb.value


def wt_build_batch(d_S, descs, d_trees, tree_bytes, d_work: int, work_bytes: int, stream: int):
    m = len(descs)
    S = (ctypes.c_void_p * m)(*d_S)
    D = (wt_desc * m)(*[wt_desc(*d) for d in descs])
    T = (ctypes.c_void_p * m)(*d_trees)
    TB = (ctypes.c_uint64 * m)(*tree_bytes)
    out = (ctypes.c_void_p * m)()
    rc = lib().wt_build_batch(m, S, D, T, TB, d_work, work_bytes, stream, out)
    return rc, [out[q] for q in range(m)]


def wt_tree_status(h: int) -> int:
    return lib().wt_tree_status(h)


def wt_free(h: int) -> None:
    lib().wt_free(h)


def wt_levels(h: int):
    l, bp, wpl, rp, rs, re = (ctypes.c_uint32(), ctypes.c_void_p(), ctypes.c_uint64(), ctypes.c_void_p(),
                              ctypes.c_uint64(), ctypes.c_uint64())
    rc = lib().wt_levels(h, ctypes.byref(l), ctypes.byref(bp), ctypes.byref(wpl), ctypes.byref(rp),
                         ctypes.byref(rs), ctypes.byref(re))
    return rc, dict(levels=l.value, bitmaps=bp.value, words_per_level=wpl.value, ranks=rp.value,
                    rank_stride=rs.value, rank_entries=re.value)


def wt_access_batch(h: int, d_i: int, d_sym: int, m: int, stream: int) -> int:
    return lib().wt_access_batch(h, d_i, d_sym, m, stream)


def wt_rank_batch(h: int, d_c: int, d_i: int, d_r: int, m: int, stream: int) -> int:
    return lib().wt_rank_batch(h, d_c, d_i, d_r, m, stream)


def wt_select_batch(h: int, d_c: int, d_j: int, d_pos: int, m: int, stream: int) -> int:
    return lib().wt_select_batch(h, d_c, d_j, d_pos, m, stream)


def wt_query_multi_footprint(ntrees: int):
    wb = ctypes.c_uint64()
    rc = lib().wt_query_multi_footprint(ntrees, ctypes.byref(wb))
    return rc, wb.value


def wt_query_multi(handles, d_tree: int, d_kind: int, d_c: int, d_x: int, d_out: int, m: int, d_work: int,
                   work_bytes: int, stream: int) -> int:
    arr = (ctypes.c_void_p * max(1, len(handles)))(*handles)
    return lib().wt_query_multi(len(handles), arr, d_tree, d_kind, d_c, d_x, d_out, m, d_work, work_bytes, stream)


def wt_access(h: int, i: int):
    s = ctypes.c_uint32()
    rc = lib().wt_access(h, i, ctypes.byref(s))
    return rc, s.value


def wt_rank(h: int, c: int, i: int):
    r = ctypes.c_uint64()
    rc = lib().wt_rank(h, c, i, ctypes.byref(r))
    return rc, r.value


def wt_select(h: int, c: int, j: int):
    p = ctypes.c_uint64()
    rc = lib().wt_select(h, c, j, ctypes.byref(p))
    return rc, p.value


def wt_prof_enable(on: bool) -> int:
    return lib().wt_prof_enable(1 if on else 0)


def wt_prof_read():
    """Waits for the recorded events; returns a list of per-launch dicts."""
    cnt = ctypes.c_uint64()
    rc = lib().wt_prof_read(None, 0, ctypes.byref(cnt))
    if rc != WT_OK:
        raise WtError(rc, "wt_prof_read")
    arr = (wt_prof_rec * max(1, cnt.value))()
    rc = lib().wt_prof_read(arr, cnt.value, ctypes.byref(cnt))
    if rc != WT_OK:
        raise WtError(rc, "wt_prof_read")
    return [dict(kernel=r.kernel.decode(), level=r.level, width=r.width, n=r.n, bytes=r.bytes, ms=r.ms)
            for r in arr[: cnt.value]]


# ------------------------------------------------- torch-backed helpers ---

_TORCH_OF_WIDTH = {1: "uint8", 2: "int16", 4: "int32"}


def _torch():
    import torch
    return torch


def _stream_handle(stream) -> int:
    torch = _torch()
    s = stream if stream is not None else torch.cuda.current_stream()
    return int(s.cuda_stream)


def _alloc(nbytes: int, device):
    torch = _torch()
    return torch.empty(max(int(nbytes), 256), dtype=torch.uint8, device=device)


class Tree:
    """A built tree whose memory is a torch tensor; owns the C handle."""

    def __init__(self, handle: int, tree_mem, work_mem, S, n: int, sigma: int, width: int, stream,
                 matrix: bool = False, arity: int = 2):
        self.handle = handle
        self.matrix = matrix
        self.arity = arity
        self.tree_mem = tree_mem
        self.work_mem = work_mem   # kept alive until the build has finished
        self.S = S
        self.n, self.sigma, self.width = n, sigma, width
        self.stream = stream
        rc, info = wt_multiary_levels(handle) if arity == 4 else wt_levels(handle)
        if rc != WT_OK:
            raise WtError(rc, "wt_multiary_levels" if arity == 4 else "wt_levels")
        self.info = info

    @property
    def levels(self) -> int:
        return self.info["levels"]

    def status(self) -> int:
        return wt_tree_status(self.handle)

    def check(self) -> None:
        rc = self.status()
        if rc != WT_OK:
            raise WtError(rc, "build")

    def zeros(self) -> np.ndarray:
        """z_i of every level (wavelet matrix only)."""
        rc, z = wt_matrix_zeros(self.handle, self.levels)
        if rc != WT_OK:
            raise WtError(rc, "wt_matrix_zeros")
        return z

    def release_workspace(self) -> None:
        self.work_mem = None

    def _region(self, ptr: int, count: int):
        torch = _torch()
        base = self.tree_mem.data_ptr()
        off = ptr - base
        flat = self.tree_mem[off: off + count * 8]
        return flat.view(torch.int64)

    def bitmaps_device(self):
        """(levels, words_per_level) int64 view of the level bitmaps."""
        l, W = self.levels, self.info["words_per_level"]
        return self._region(self.info["bitmaps"], l * W).view(l, W)

    def ranks_device(self):
        l, K = self.levels, self.info["rank_stride"]
        return self._region(self.info["ranks"], l * K).view(l, K)

    def bitmaps(self) -> np.ndarray:
        self.check()
        return self.bitmaps_device().cpu().numpy().view(np.uint64)

    def digits(self) -> np.ndarray:
        """4-ary tree: (levels, words) uint64 digit levels, 32 two-bit digits per word."""
        self.check()
        l, W = self.levels, self.info["words"]
        return self._region(self.info["digits"], l * W).view(l, W).cpu().numpy().view(np.uint64)

    def digit_dir(self) -> np.ndarray:
        """4-ary tree: (levels, dir_stride, 4) uint64 counts of digits 0..3 before 512k."""
        self.check()
        l, K = self.levels, self.info["dir_stride"]
        return self._region(self.info["dir"], l * K * 4).view(l, K, 4).cpu().numpy().view(np.uint64)

    def ranks(self) -> np.ndarray:
        self.check()
        return self.ranks_device().cpu().numpy().view(np.uint64)

    def access(self, pos):
        torch = _torch()
        pos = torch.as_tensor(pos, dtype=torch.int64, device=self.tree_mem.device).contiguous()
        out = torch.empty(pos.numel(), dtype=torch.int32, device=pos.device)
        rc = wt_access_batch(self.handle, pos.data_ptr(), out.data_ptr(), pos.numel(), _stream_handle(self.stream))
        if rc != WT_OK:
            raise WtError(rc, "wt_access_batch")
        return out

    def rank(self, c, i):
        torch = _torch()
        dev = self.tree_mem.device
        c = torch.as_tensor(c, dtype=torch.int32, device=dev).contiguous()
        i = torch.as_tensor(i, dtype=torch.int64, device=dev).contiguous()
        out = torch.empty(c.numel(), dtype=torch.int64, device=dev)
        rc = wt_rank_batch(self.handle, c.data_ptr(), i.data_ptr(), out.data_ptr(), c.numel(),
                           _stream_handle(self.stream))
        if rc != WT_OK:
            raise WtError(rc, "wt_rank_batch")
        return out

    def select(self, c, j):
        torch = _torch()
        dev = self.tree_mem.device
        c = torch.as_tensor(c, dtype=torch.int32, device=dev).contiguous()
        j = torch.as_tensor(j, dtype=torch.int64, device=dev).contiguous()
        out = torch.empty(c.numel(), dtype=torch.int64, device=dev)
        rc = wt_select_batch(self.handle, c.data_ptr(), j.data_ptr(), out.data_ptr(), c.numel(),
                             _stream_handle(self.stream))
        if rc != WT_OK:
            raise WtError(rc, "wt_select_batch")
        return out

    def close(self) -> None:
        if self.handle:
            wt_free(self.handle)
            self.handle = 0

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def to_device(S: np.ndarray, device="cuda"):
    """Copy a numpy symbol array to the GPU (uint16/uint32 travel as int16/int32 views)."""
    torch = _torch()
    width = S.dtype.itemsize
    view = {1: np.uint8, 2: np.int16, 4: np.int32}[width]
    return torch.from_numpy(np.ascontiguousarray(S).view(view)).to(device)


def build(S, sigma: int, width: int | None = None, stream=None, tree_mem=None, work_mem=None,
          matrix: bool = False, arity: int = 2) -> Tree:
    """Build the tree (with matrix=True the wavelet matrix, with arity=4 the
    4-ary tree) of a device tensor S (uint8 / int16 / int32 storage)."""
    torch = _torch()
    width = width or S.element_size()
    n = S.numel()
    if arity not in (2, 4) or (arity == 4 and matrix):
        raise WtError(WT_EINVAL, "build")
    rc, tb, wb = (wt_multiary_footprint if arity == 4 else wt_footprint)(n, sigma, width)
    if rc != WT_OK:
        raise WtError(rc, "wt_footprint")
    dev = S.device
    tree_mem = tree_mem if tree_mem is not None else _alloc(tb, dev)
    work_mem = work_mem if work_mem is not None else _alloc(wb, dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    fn = wt_build_multiary if arity == 4 else (wt_build_matrix if matrix else wt_build)
    rc, h = fn(S.data_ptr() if n else 0, n, sigma, width, tree_mem.data_ptr(), tree_mem.numel(),
               work_mem.data_ptr(), work_mem.numel(), int(st.cuda_stream))
    if rc != WT_OK:
        raise WtError(rc, fn.__name__)
    return Tree(h, tree_mem, work_mem, S, n, sigma, width, st, matrix, arity)


def build_buffered(S, sigma: int, buffer_syms: int, width: int | None = None, device="cuda", stream=None,
                   tree_mem=None, work_mem=None) -> Tree:
    """Buffered build of S read in pieces of buffer_syms symbols.  S is a
    host numpy array or torch tensor (page-locked for overlapped copies) or
    a device tensor; it has been read completely when this returns."""
    torch = _torch()
    if isinstance(S, np.ndarray):
        S = torch.from_numpy(np.ascontiguousarray(S).view({1: np.uint8, 2: np.int16, 4: np.int32}[S.dtype.itemsize]))
    width = width or S.element_size()
    n = S.numel()
    rc, tb, wb = wt_buffered_footprint(n, sigma, width, buffer_syms)
    if rc != WT_OK:
        raise WtError(rc, "wt_buffered_footprint")
    dev = torch.device(device) if not S.is_cuda else S.device
    tree_mem = tree_mem if tree_mem is not None else _alloc(tb, dev)
    work_mem = work_mem if work_mem is not None else _alloc(wb, dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    rc, h = wt_build_buffered(S.data_ptr() if n else 0, n, sigma, width, buffer_syms, tree_mem.data_ptr(),
                              tree_mem.numel(), work_mem.data_ptr(), work_mem.numel(), int(st.cuda_stream))
    if rc != WT_OK:
        raise WtError(rc, "wt_build_buffered")
    return Tree(h, tree_mem, work_mem, S, n, sigma, width, st)


def build_batch(Ss, sigmas, widths=None, stream=None):
    """Build several trees with wt_build_batch; returns a list of Tree."""
    torch = _torch()
    m = len(Ss)
    widths = widths or [S.element_size() for S in Ss]
    descs = [(S.numel(), int(sg), int(w)) for S, sg, w in zip(Ss, sigmas, widths)]
    dev = Ss[0].device
    trees_mem, tbytes = [], []
    for (n, sg, w) in descs:
        rc, tb, _ = wt_footprint(n, sg, w)
        if rc != WT_OK:
            raise WtError(rc, "wt_footprint")
        trees_mem.append(_alloc(tb, dev))
        tbytes.append(trees_mem[-1].numel())
    rc, wb = wt_batch_footprint(descs)
    if rc != WT_OK:
        raise WtError(rc, "wt_batch_footprint")
    work = _alloc(wb, dev)
    st = stream if stream is not None else torch.cuda.current_stream(dev)
    rc, hs = wt_build_batch([S.data_ptr() if S.numel() else 0 for S in Ss], descs,
                            [t.data_ptr() for t in trees_mem], tbytes, work.data_ptr(), work.numel(),
                            int(st.cuda_stream))
    if rc != WT_OK:
        raise WtError(rc, "wt_build_batch")
    return [Tree(h, tm, work, S, d[0], d[1], d[2], st) for h, tm, S, d in zip(hs, trees_mem, Ss, descs)]


class HuffTree(Tree):
    """A Huffman-shaped tree: depth d holds n_d positions (its own size)."""

    def __init__(self, handle: int, tree_mem, work_mem, S, n: int, sigma: int, width: int, stream):
        self.handle = handle
        self.matrix = False
        self.arity = 2
        self.tree_mem = tree_mem
        self.work_mem = work_mem
        self.S = S
        self.n, self.sigma, self.width = n, sigma, width
        self.stream = stream
        rc, info = wt_huffman_levels(handle, sigma)
        if rc != WT_OK:
            raise WtError(rc, "wt_huffman_levels")
        self.info = info

    @property
    def sizes(self):
        return self.info["sizes"]

    def lengths(self) -> np.ndarray:
        return (self.info["code_table"] & 31).astype(np.uint8)

    def codes(self) -> np.ndarray:
        return (self.info["code_table"] >> 8).astype(np.uint32)

    def bitmaps(self):
        """Per depth: round_up(ceil(n_d/64), 8) uint64 words."""
        self.check()
        host = self.tree_mem.cpu().numpy()
        out = []
        for d in range(self.levels):
            words = ((self.sizes[d] + 63) // 64 + 7) // 8 * 8
            o = self.info["bits_off"][d]
            out.append(host[o:o + 8 * words].view(np.uint64).copy())
        return out

    def ranks(self):
        """Per depth: round_up(ceil(n_d/512) + 1, 8) uint64 directory entries."""
        self.check()
        host = self.tree_mem.cpu().numpy()
        out = []
        for d in range(self.levels):
            ent = (self.info["dir_entries"][d] + 7) // 8 * 8
            o = self.info["dir_off"][d]
            out.append(host[o:o + 8 * ent].view(np.uint64).copy())
        return out


def histogram(S, sigma: int, width: int | None = None, stream=None) -> np.ndarray:
    """Symbol counts of a device tensor S (wt_histogram), on the host."""
    torch = _torch()
    width = width or S.element_size()
    n = S.numel()
    counts = torch.empty(max(1, sigma), dtype=torch.int64, device=S.device)
    st = stream if stream is not None else torch.cuda.current_stream(S.device)
    rc = wt_histogram(S.data_ptr() if n else 0, n, sigma, width, counts.data_ptr(), int(st.cuda_stream))
    if rc != WT_OK:
        raise WtError(rc, "wt_histogram")
    st.synchronize()
    return counts[:sigma].cpu().numpy().view(np.uint64).copy()


def build_huffman(S, sigma: int, width: int | None = None, stream=None, counts=None, tree_mem=None,
                  work_mem=None) -> HuffTree:
    """Huffman-shaped tree of a device tensor S: its histogram on the GPU
    (unless the counts are given), then the build from those counts."""
    torch = _torch()
    width = width or S.element_size()
    n = S.numel()
    st = stream if stream is not None else torch.cuda.current_stream(S.device)
    if counts is None:
        counts = histogram(S, sigma, width, st)
    rc, tb, wb = wt_huffman_footprint(counts, n, sigma, width)
    if rc != WT_OK:
        raise WtError(rc, "wt_huffman_footprint")
    tree_mem = tree_mem if tree_mem is not None else _alloc(tb, S.device)
    work_mem = work_mem if work_mem is not None else _alloc(wb, S.device)
    rc, h = wt_build_huffman(S.data_ptr() if n else 0, n, sigma, width, counts, tree_mem.data_ptr(),
                             tree_mem.numel(), work_mem.data_ptr(), work_mem.numel(), int(st.cuda_stream))
    if rc != WT_OK:
        raise WtError(rc, "wt_build_huffman")
    return HuffTree(h, tree_mem, work_mem, S, n, sigma, width, st)
