"""Test helpers: independent characterisations and a tree comparator.

Nothing here is used by the library.  The functions restate facts about the
pointerless wavelet tree in forms different from the oracle's counting-sort
construction, so that they can pin it:

* ``levels_by_stable_sort``: level i's bitmap is the bit (l-1-i) plane of S
  after a *stable* sort by the top i bits (each node's symbols stay in input
  order, nodes in prefix order -- Section 2.2 and Proposition 1).  numpy's
  stable argsort does the sorting.
* ``ranks_by_cumsum``: the rank directory is a cumulative popcount.
* ``compare_levels``: reports the first differing (level, word) or (level,
  entry), used by every parity test.
"""
from __future__ import annotations

import numpy as np


def n_levels(sigma: int) -> int:
    return max(0, int(sigma - 1).bit_length())


def words_per_level(n: int) -> int:
    return ((n + 63) // 64 + 7) // 8 * 8


def rank_entries(n: int) -> int:
    return (n + 511) // 512 + 1


def rank_stride(n: int) -> int:
    return (rank_entries(n) + 7) // 8 * 8


def pack_bits(bits: np.ndarray, words: int) -> np.ndarray:
    """Pack a 0/1 vector LSB-first into ``words`` uint64 words (zero padded)."""
    by = np.packbits(bits.astype(np.uint8), bitorder="little")
    buf = np.zeros(words * 8, dtype=np.uint8)
    buf[: by.size] = by
    return buf.view("<u8").astype(np.uint64)


def unpack_bits(words: np.ndarray, n: int) -> np.ndarray:
    by = np.ascontiguousarray(words.astype("<u8")).view(np.uint8)
    return np.unpackbits(by, bitorder="little")[:n]


def levels_by_stable_sort(S: np.ndarray, sigma: int) -> np.ndarray:
    l = n_levels(sigma)
    n = S.shape[0]
    W = words_per_level(n)
    s = S.astype(np.int64)
    out = np.zeros((l, W), dtype=np.uint64)
    for i in range(l):
        order = np.argsort(s >> (l - i), kind="stable")
        bits = (s[order] >> (l - 1 - i)) & 1
        out[i] = pack_bits(bits, W)
    return out


def ranks_by_cumsum(bitmaps: np.ndarray, n: int) -> np.ndarray:
    l = bitmaps.shape[0]
    K = rank_entries(n)
    out = np.zeros((l, rank_stride(n)), dtype=np.uint64)
    for i in range(l):
        bits = unpack_bits(bitmaps[i], n).astype(np.int64)
        cs = np.concatenate([[0], np.cumsum(bits)])
        pos = np.minimum(np.arange(K, dtype=np.int64) * 512, n)
        out[i, :K] = cs[pos]
    return out


def compare_levels(got: np.ndarray, want: np.ndarray, what: str = "bitmap"):
    """None if equal, else a message naming the first differing level/index."""
    got = np.asarray(got)
    want = np.asarray(want)
    if got.shape != want.shape:
        return "%s shape %s != %s" % (what, got.shape, want.shape)
    diff = np.argwhere(got != want)
    if diff.size == 0:
        return None
    lv, k = (int(x) for x in diff[0])
    return "%s differs at level %d index %d: got %#x want %#x (%d differing entries)" % (
        what, lv, k, int(got[lv, k]), int(want[lv, k]), diff.shape[0])
