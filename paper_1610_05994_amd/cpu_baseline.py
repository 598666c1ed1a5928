"""Multicore CPU construction (OpenMP) of the paper's parallel algorithms,
pwt (Section 3.1, one level per thread) and dd (Section 3.2, one segment per
thread), from libwtcpu.so.  A host-side comparator for the GPU library: same
output layout (level bitmaps and rank directories), no code shared with the
GPU kernels or the test oracle."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libwtcpu.so")
ALGOS = ("pwt", "dd")
_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libwtcpu.so is not built (%s); run __graft_entry__.build()" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        u64, u32, vp, i32 = ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p, ctypes.c_int
        for name in ("wtc_build_pwt", "wtc_build_dd"):
            f = getattr(L, name)
            f.argtypes = [vp, u64, u32, u32, vp, vp, i32]
            f.restype = i32
        for name in ("wtc_words", "wtc_rank_stride"):
            getattr(L, name).argtypes = [u64]
            getattr(L, name).restype = u64
        _lib = L
    return _lib


def levels(sigma: int) -> int:
    return max(0, (int(sigma) - 1).bit_length())


def build(S: np.ndarray, sigma: int, algo: str = "dd", threads: int = 0):
    """(status, bitmaps (levels, words), ranks (levels, stride)) of S."""
    if algo not in ALGOS:
        raise ValueError(algo)
    S = np.ascontiguousarray(S)
    n = int(S.shape[0])
    L = lib()
    l = levels(sigma)
    B = np.empty((l, int(L.wtc_words(n))), dtype=np.uint64)
    R = np.empty((l, int(L.wtc_rank_stride(n))), dtype=np.uint64)
    f = L.wtc_build_pwt if algo == "pwt" else L.wtc_build_dd
    rc = f(S.ctypes.data_as(ctypes.c_void_p), n, int(sigma), S.dtype.itemsize,
           B.ctypes.data_as(ctypes.c_void_p), R.ctypes.data_as(ctypes.c_void_p), int(threads))
    return rc, B, R
