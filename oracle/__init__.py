"""Python face of the sequential CPU oracle (``wt_oracle.c``).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
benchmark's ``cpu_baseline`` leg may import this package.  The GPU library
never calls it, and it never calls the GPU library: the two share no code.

The C source builds the tree from its recursive definition (Section 2.2:
every node hands its symbols, in order, to the child of their next bit;
each level is the concatenation of its nodes' bitmaps) and answers queries
by the walks of Section 2.2; see the header of ``wt_oracle.c`` for the
readings taken where the paper is loose.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "wt_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ERANGE, ENOMEM, ENOTFOUND = 0, 1, 2, 3, 4


def compile_oracle(force: bool = True) -> str:
    """Compile the oracle with gcc -O2 (the paper's optimisation level)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        compile_oracle(force=False)
        L = ctypes.CDLL(_LIB)
        u32, u64, vp = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p
        L.wto_levels.argtypes = [u32]
        L.wto_levels.restype = u32
        L.wto_words_per_level.argtypes = [u64]
        L.wto_words_per_level.restype = u64
        L.wto_rank_entries.argtypes = [u64]
        L.wto_rank_entries.restype = u64
        L.wto_rank_stride.argtypes = [u64]
        L.wto_rank_stride.restype = u64
        L.wto_build.argtypes = [vp, u64, u32, u32, vp, vp]
        L.wto_build.restype = ctypes.c_int
        L.wto_access.argtypes = [vp, u64, u32, u64, vp, vp, vp]
        L.wto_access.restype = ctypes.c_int
        L.wto_rank.argtypes = [vp, u64, u32, u32, u64, vp]
        L.wto_rank.restype = ctypes.c_int
        L.wto_select.argtypes = [vp, u64, u32, u32, u64, vp]
        L.wto_select.restype = ctypes.c_int
        L.wto_decode.argtypes = [vp, u64, u32, vp]
        L.wto_decode.restype = ctypes.c_int
        L.wto_build_matrix.argtypes = [vp, u64, u32, u32, vp, vp, vp]
        L.wto_build_matrix.restype = ctypes.c_int
        L.wto_matrix_access.argtypes = [vp, vp, u64, u32, u64, vp]
        L.wto_matrix_access.restype = ctypes.c_int
        L.wto_matrix_rank.argtypes = [vp, vp, u64, u32, u32, u64, vp]
        L.wto_matrix_rank.restype = ctypes.c_int
        L.wto_matrix_select.argtypes = [vp, vp, u64, u32, u32, u64, vp]
        L.wto_matrix_select.restype = ctypes.c_int
        L.wto_levels4.argtypes = [u32]
        L.wto_levels4.restype = u32
        L.wto_words4.argtypes = [u64]
        L.wto_words4.restype = u64
        L.wto_build4.argtypes = [vp, u64, u32, u32, vp, vp]
        L.wto_build4.restype = ctypes.c_int
        L.wto_access4.argtypes = [vp, u64, u32, u64, vp]
        L.wto_access4.restype = ctypes.c_int
        L.wto_rank4.argtypes = [vp, u64, u32, u32, u64, vp]
        L.wto_rank4.restype = ctypes.c_int
        L.wto_select4.argtypes = [vp, u64, u32, u32, u64, vp]
        L.wto_select4.restype = ctypes.c_int
        L.wto_huffman_lengths.argtypes = [vp, u32, vp, vp]
        L.wto_huffman_lengths.restype = ctypes.c_int
        L.wto_huffman_codes.argtypes = [vp, u32, u32, vp]
        L.wto_huffman_codes.restype = ctypes.c_int
        L.wto_build_huffman.argtypes = [vp, u64, u32, u32, vp, vp, u32, vp, vp, vp, vp]
        L.wto_build_huffman.restype = ctypes.c_int
        _lib = L
    return _lib


def levels(sigma: int) -> int:
    return int(lib().wto_levels(sigma))


def words_per_level(n: int) -> int:
    return int(lib().wto_words_per_level(n))


def rank_entries(n: int) -> int:
    return int(lib().wto_rank_entries(n))


def rank_stride(n: int) -> int:
    return int(lib().wto_rank_stride(n))


@dataclass
class OracleTree:
    n: int
    sigma: int
    levels: int
    bitmaps: np.ndarray        # (levels, words_per_level(n)) uint64
    ranks: np.ndarray | None   # (levels, rank_stride(n)) uint64, or None


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def build(S: np.ndarray, sigma: int, with_ranks: bool = True) -> OracleTree:
    """Sequential construction of every level (and rank directory)."""
    S = np.ascontiguousarray(S)
    width = S.dtype.itemsize
    n = int(S.shape[0])
    lv = levels(sigma)
    B = np.zeros((lv, words_per_level(n)), dtype=np.uint64)
    R = np.zeros((lv, rank_stride(n)), dtype=np.uint64) if with_ranks else None
    rc = lib().wto_build(_ptr(S), n, sigma, width, _ptr(B), _ptr(R) if R is not None else None)
    if rc != OK:
        raise ValueError("oracle build failed with status %d" % rc)
    return OracleTree(n, sigma, lv, B, R)


def build_status(S: np.ndarray, sigma: int, width: int | None = None) -> int:
    """Raw status of a build (for argument-validation tests)."""
    S = np.ascontiguousarray(S)
    n = int(S.shape[0])
    lv = levels(max(sigma, 1))
    B = np.zeros((max(lv, 1), words_per_level(n)), dtype=np.uint64)
    return int(lib().wto_build(_ptr(S), n, sigma, width or S.dtype.itemsize, _ptr(B), None))


def access(t: OracleTree, i: int):
    """Returns (symbol, bits per level, in-node index per level)."""
    sym = ctypes.c_uint32()
    bits = np.zeros(max(t.levels, 1), dtype=np.uint32)
    idx = np.zeros(max(t.levels, 1), dtype=np.uint64)
    rc = lib().wto_access(_ptr(t.bitmaps), t.n, t.sigma, i, ctypes.byref(sym), _ptr(bits), _ptr(idx))
    if rc != OK:
        raise ValueError("access status %d" % rc)
    return int(sym.value), bits[: t.levels].tolist(), [int(x) for x in idx[: t.levels]]


def rank(t: OracleTree, c: int, i: int) -> int:
    out = ctypes.c_uint64()
    rc = lib().wto_rank(_ptr(t.bitmaps), t.n, t.sigma, c, i, ctypes.byref(out))
    if rc != OK:
        raise ValueError("rank status %d" % rc)
    return int(out.value)


def select(t: OracleTree, c: int, j: int):
    """0-based position of the j-th (1-based) c, or None if there is none."""
    out = ctypes.c_uint64()
    rc = lib().wto_select(_ptr(t.bitmaps), t.n, t.sigma, c, j, ctypes.byref(out))
    if rc == ENOTFOUND:
        return None
    if rc != OK:
        raise ValueError("select status %d" % rc)
    return int(out.value)


def decode(t: OracleTree) -> np.ndarray:
    out = np.zeros(t.n, dtype=np.uint32)
    rc = lib().wto_decode(_ptr(t.bitmaps), t.n, t.sigma, _ptr(out))
    if rc != OK:
        raise ValueError("decode status %d" % rc)
    return out


# ------------------------------------------------------- wavelet matrix ---

@dataclass
class OracleMatrix:
    n: int
    sigma: int
    levels: int
    bitmaps: np.ndarray        # (levels, words_per_level(n)) uint64
    ranks: np.ndarray | None   # (levels, rank_stride(n)) uint64, or None
    zeros: np.ndarray          # (levels,) uint64: zeros of each level


def build_matrix(S: np.ndarray, sigma: int, with_ranks: bool = True) -> OracleMatrix:
    """Sequential wavelet-matrix construction from its definition."""
    S = np.ascontiguousarray(S)
    width = S.dtype.itemsize
    n = int(S.shape[0])
    lv = levels(sigma)
    B = np.zeros((lv, words_per_level(n)), dtype=np.uint64)
    R = np.zeros((lv, rank_stride(n)), dtype=np.uint64) if with_ranks else None
    Z = np.zeros(max(lv, 1), dtype=np.uint64)
    rc = lib().wto_build_matrix(_ptr(S), n, sigma, width, _ptr(B), _ptr(R) if R is not None else None, _ptr(Z))
    if rc != OK:
        raise ValueError("oracle wto_build_matrix status %d" % rc)
    return OracleMatrix(n, sigma, lv, B, R, Z[:lv])


def matrix_access(t: OracleMatrix, i: int) -> int:
    sym = ctypes.c_uint32()
    rc = lib().wto_matrix_access(_ptr(t.bitmaps), _ptr(t.zeros), t.n, t.sigma, i, ctypes.byref(sym))
    if rc != OK:
        raise ValueError("matrix access status %d" % rc)
    return int(sym.value)


def matrix_rank(t: OracleMatrix, c: int, i: int) -> int:
    out = ctypes.c_uint64()
    rc = lib().wto_matrix_rank(_ptr(t.bitmaps), _ptr(t.zeros), t.n, t.sigma, c, i, ctypes.byref(out))
    if rc != OK:
        raise ValueError("matrix rank status %d" % rc)
    return int(out.value)


def matrix_select(t: OracleMatrix, c: int, j: int):
    out = ctypes.c_uint64()
    rc = lib().wto_matrix_select(_ptr(t.bitmaps), _ptr(t.zeros), t.n, t.sigma, c, j, ctypes.byref(out))
    if rc == ENOTFOUND:
        return None
    if rc != OK:
        raise ValueError("matrix select status %d" % rc)
    return int(out.value)


# ------------------------------------------------------- 4-ary tree ---

def levels4(sigma: int) -> int:
    """Levels of the 4-ary tree: ceil(ceil(lg sigma) / 2)."""
    return int(lib().wto_levels4(sigma))


def words4(n: int) -> int:
    """64-bit words per 4-ary level (32 two-bit digits each, padded to 8)."""
    return int(lib().wto_words4(n))


@dataclass
class OracleTree4:
    n: int
    sigma: int
    levels: int
    digits: np.ndarray          # (levels, words4(n)) uint64, 2-bit digits
    dir: np.ndarray | None      # (levels, rank_stride(n), 4) uint64 counts of digits 0..3


def build4(S: np.ndarray, sigma: int, with_dir: bool = True) -> OracleTree4:
    """Sequential 4-ary wavelet-tree construction (pwt with four-way nodes)."""
    S = np.ascontiguousarray(S)
    width = S.dtype.itemsize
    n = int(S.shape[0])
    lv = levels4(sigma)
    D = np.zeros((lv, words4(n)), dtype=np.uint64)
    R = np.zeros((lv, rank_stride(n), 4), dtype=np.uint64) if with_dir else None
    rc = lib().wto_build4(_ptr(S), n, sigma, width, _ptr(D), _ptr(R) if R is not None else None)
    if rc != OK:
        raise ValueError("oracle wto_build4 status %d" % rc)
    return OracleTree4(n, sigma, lv, D, R)


def access4(t: OracleTree4, i: int) -> int:
    sym = ctypes.c_uint32()
    rc = lib().wto_access4(_ptr(t.digits), t.n, t.sigma, i, ctypes.byref(sym))
    if rc != OK:
        raise ValueError("access4 status %d" % rc)
    return int(sym.value)


def rank4(t: OracleTree4, c: int, i: int) -> int:
    out = ctypes.c_uint64()
    rc = lib().wto_rank4(_ptr(t.digits), t.n, t.sigma, c, i, ctypes.byref(out))
    if rc != OK:
        raise ValueError("rank4 status %d" % rc)
    return int(out.value)


def select4(t: OracleTree4, c: int, j: int):
    out = ctypes.c_uint64()
    rc = lib().wto_select4(_ptr(t.digits), t.n, t.sigma, c, j, ctypes.byref(out))
    if rc == ENOTFOUND:
        return None
    if rc != OK:
        raise ValueError("select4 status %d" % rc)
    return int(out.value)


# ------------------------------------------------- Huffman-shaped tree ---

def huffman_lengths(counts: np.ndarray):
    """Code lengths (uint8 per symbol, 0 for absent symbols) and the longest."""
    counts = np.ascontiguousarray(counts, dtype=np.uint64)
    sigma = int(counts.shape[0])
    ln = np.zeros(sigma, dtype=np.uint8)
    mx = ctypes.c_uint32()
    rc = lib().wto_huffman_lengths(_ptr(counts), sigma, _ptr(ln), ctypes.byref(mx))
    if rc != OK:
        raise ValueError("huffman lengths status %d" % rc)
    return ln, int(mx.value)


def huffman_codes(lengths: np.ndarray, maxlen: int) -> np.ndarray:
    """Canonical codes (right-aligned in each symbol's length)."""
    lengths = np.ascontiguousarray(lengths, dtype=np.uint8)
    code = np.zeros(lengths.shape[0], dtype=np.uint32)
    rc = lib().wto_huffman_codes(_ptr(lengths), lengths.shape[0], maxlen, _ptr(code))
    if rc != OK:
        raise ValueError("huffman codes status %d" % rc)
    return code


@dataclass
class OracleHuffman:
    n: int
    sigma: int
    levels: int                 # the longest code length
    lengths: np.ndarray         # (sigma,) uint8
    codes: np.ndarray           # (sigma,) uint32, right-aligned
    sizes: list                 # n_d: symbols whose code is longer than d
    bitmaps: list               # per depth: words_per_level(n_d) uint64
    ranks: list                 # per depth: rank_stride(n_d) uint64, or None
    only: int = -1              # with no levels and n > 0: the one symbol of S


def build_huffman(S: np.ndarray, sigma: int, with_ranks: bool = True) -> OracleHuffman:
    """Huffman-shaped wavelet tree of S from its definition (code lengths from
    the symbol counts of S, canonical codes, one bitmap per depth)."""
    S = np.ascontiguousarray(S)
    width = S.dtype.itemsize
    n = int(S.shape[0])
    if n and int(S.max()) >= sigma:
        raise ValueError("symbol out of range")
    counts = np.bincount(S.astype(np.int64), minlength=sigma).astype(np.uint64) if n else np.zeros(sigma, np.uint64)
    ln, L = huffman_lengths(counts)
    code = huffman_codes(ln, L)
    sizes = [int(counts[ln > d].sum()) for d in range(L)]
    bofs = np.zeros(max(L, 1), dtype=np.uint64)
    rofs = np.zeros(max(L, 1), dtype=np.uint64)
    tb = tr = 0
    for d in range(L):
        bofs[d], rofs[d] = tb, tr
        tb += words_per_level(sizes[d])
        tr += rank_stride(sizes[d])
    B = np.zeros(max(tb, 1), dtype=np.uint64)
    R = np.zeros(max(tr, 1), dtype=np.uint64) if with_ranks else None
    rc = lib().wto_build_huffman(_ptr(S), n, sigma, width, _ptr(ln), _ptr(code), L, _ptr(bofs), _ptr(rofs),
                                 _ptr(B), _ptr(R) if R is not None else None)
    if rc != OK:
        raise ValueError("oracle wto_build_huffman status %d" % rc)
    bm = [B[int(bofs[d]):int(bofs[d]) + words_per_level(sizes[d])].copy() for d in range(L)]
    rk = [R[int(rofs[d]):int(rofs[d]) + rank_stride(sizes[d])].copy() for d in range(L)] if with_ranks else None
    only = int(np.flatnonzero(counts)[0]) if (L == 0 and n > 0) else -1
    return OracleHuffman(n, sigma, L, ln, code, sizes, bm, rk, only)


def _bits(words: np.ndarray, size: int) -> np.ndarray:
    """A depth's bitmap as size 0/1 values (position p = word p/64, bit p%64)."""
    b = np.unpackbits(words.view(np.uint8), bitorder="little")
    return b[:size].astype(np.int64)


class HuffmanWalker:
    """Queries on an OracleHuffman by walking its bitmaps (Section 2.2's
    navigation by counting bits of a node's range), with the internal nodes
    of every depth laid out from left to right: a node's 0-child and 1-child
    take, in that order, the next places at the next depth when they are
    internal, and a child whose prefix is a code is that symbol's leaf."""

    def __init__(self, t: OracleHuffman):
        self.t = t
        self.bits = [_bits(t.bitmaps[d], t.sizes[d]) for d in range(t.levels)]
        self.leaf = {}
        for s in range(t.sigma):
            if t.lengths[s]:
                self.leaf[(int(t.lengths[s]), int(t.codes[s]))] = s
        # node table: depth -> {prefix: (start, size)}
        self.nodes = []
        if t.levels:
            self.nodes.append({0: (0, t.n)})
        for d in range(t.levels):
            nxt, pos = {}, 0
            for pre in sorted(self.nodes[d]):
                b, sz = self.nodes[d][pre]
                ones = int(self.bits[d][b:b + sz].sum())
                for bit, cnt in ((0, sz - ones), (1, ones)):
                    child = 2 * pre + bit
                    if (d + 1, child) not in self.leaf and cnt > 0:
                        nxt[child] = (pos, cnt)
                        pos += cnt
            self.nodes.append(nxt)

    def access(self, i: int) -> int:
        if self.t.levels == 0:
            return self.t.only
        pre, p = 0, i
        for d in range(self.t.levels):
            b, sz = self.nodes[d][pre]
            bit = int(self.bits[d][b + p])
            p = int((self.bits[d][b:b + p] == bit).sum())
            pre = 2 * pre + bit
            if (d + 1, pre) in self.leaf:
                return self.leaf[(d + 1, pre)]
        raise AssertionError("walk did not end at a leaf")

    def rank(self, c: int, i: int) -> int:
        L = int(self.t.lengths[c]) if c < self.t.sigma else 0
        if self.t.levels == 0:
            return i if c == self.t.only else 0
        if L == 0:
            return 0
        code = int(self.t.codes[c])
        pre, cnt = 0, i
        for d in range(L):
            b, sz = self.nodes[d][pre]
            bit = (code >> (L - 1 - d)) & 1
            cnt = int((self.bits[d][b:b + cnt] == bit).sum())
            pre = 2 * pre + bit
        return cnt

    def select(self, c: int, j: int):
        """0-based position of the j-th (1-based) c, or None."""
        if j < 1:
            return None
        if self.t.levels == 0:
            return j - 1 if (c == self.t.only and j <= self.t.n) else None
        L = int(self.t.lengths[c]) if c < self.t.sigma else 0
        if L == 0:
            return None
        code = int(self.t.codes[c])
        path, pre = [], 0
        for d in range(L):
            path.append(pre)
            pre = 2 * pre + ((code >> (L - 1 - d)) & 1)
        # leaf size: the count of its bit in the parent node
        d = L - 1
        b, sz = self.nodes[d][path[d]]
        bit = code & 1
        if j > int((self.bits[d][b:b + sz] == bit).sum()):
            return None
        k = j - 1                              # index among the leaf's symbols
        for d in range(L - 1, -1, -1):
            b, sz = self.nodes[d][path[d]]
            bit = (code >> (L - 1 - d)) & 1
            where = np.flatnonzero(self.bits[d][b:b + sz] == bit)
            k = int(where[k])                   # index inside the node at depth d
        return k
