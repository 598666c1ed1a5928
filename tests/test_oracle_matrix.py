"""Pins of the wavelet-matrix oracle (the variant's standard definition:
A_0 = S, level i = bit (l-1-i) of A_i, A_{i+1} = A_i stably partitioned by
that bit over the whole level, z_i = zeros of level i).

Independent of the oracle's C code:
- library routine: A_i is S stably sorted (numpy, kind="stable") by its top
  i bits read in reverse order (the last partition bit is the most
  significant), so every level is a bit plane of a numpy argsort;
- closed forms: z_i counts the zeros of bit (l-1-i) over S; level 0 is the
  MSB plane of S in input order (the wavelet tree's level 0); sigma = 2 gives
  S itself; the rank directory is the cumulative popcount;
- brute force: access / rank / select through the matrix walk equal S,
  counts of S[:i] and positions of the j-th occurrence, for every argument
  on small inputs.
"""
import numpy as np
import pytest

import oracle
import wtgen
from tests import treecheck as tc


def _reverse_bits(x: np.ndarray, nbits: int) -> np.ndarray:
    out = np.zeros_like(x)
    for t in range(nbits):
        out |= ((x >> t) & 1) << (nbits - 1 - t)
    return out


def matrix_by_argsort(S, sigma):
    l = oracle.levels(sigma)
    S = S.astype(np.int64)
    levels = []
    for i in range(l):
        key = _reverse_bits(S >> (l - i), i) if i else np.zeros_like(S)
        A = S[np.argsort(key, kind="stable")]
        levels.append(((A >> (l - 1 - i)) & 1).astype(np.uint8))
    return levels


SIGMAS = [1, 2, 3, 5, 16, 20, 256, 1000, 1 << 16]
NS = [0, 1, 2, 63, 64, 65, 511, 512, 513, 3000]


@pytest.mark.parametrize("sigma", SIGMAS)
def test_levels_match_stable_sort_by_reversed_prefix(sigma):
    for k, n in enumerate(NS):
        S = wtgen.uniform(n, sigma, 4000 + 7 * k + sigma % 97)
        t = oracle.build_matrix(S, sigma)
        ref = matrix_by_argsort(S, sigma)
        assert t.levels == len(ref)
        for i, bits in enumerate(ref):
            assert np.array_equal(tc.unpack_bits(t.bitmaps[i], n), bits), (sigma, n, i)
            assert int(t.zeros[i]) == int(n - bits.sum())
        if t.levels:
            assert np.array_equal(t.ranks, tc.ranks_by_cumsum(t.bitmaps, n))


def test_closed_forms():
    S = wtgen.uniform(5000, 256, 11)
    m = oracle.build_matrix(S, 256)
    w = oracle.build(S, 256)
    assert np.array_equal(m.bitmaps[0], w.bitmaps[0])           # level 0: MSB plane in input order
    for i in range(8):
        assert int(m.zeros[i]) == int(np.sum(((S >> (7 - i)) & 1) == 0))
    S2 = wtgen.uniform(777, 2, 12)
    m2 = oracle.build_matrix(S2, 2)
    assert np.array_equal(tc.unpack_bits(m2.bitmaps[0], 777), S2.astype(np.uint8))
    m1 = oracle.build_matrix(S2 * 0, 1)
    assert m1.levels == 0


@pytest.mark.parametrize("sigma,n", [(4, 200), (20, 300), (256, 250), (1000, 120)])
def test_queries_brute_force(sigma, n):
    S = wtgen.zipf(n, sigma, 1.0, 900 + sigma)
    t = oracle.build_matrix(S, sigma)
    for i in range(n):
        assert oracle.matrix_access(t, i) == int(S[i])
    for c in sorted(set(S.tolist()) | {0, sigma - 1}):
        occ = np.flatnonzero(S == c)
        for i in range(0, n + 1, 7):
            assert oracle.matrix_rank(t, c, i) == int(np.sum(S[:i] == c))
        for j in range(1, len(occ) + 1):
            assert oracle.matrix_select(t, c, j) == int(occ[j - 1])
        assert oracle.matrix_select(t, c, len(occ) + 1) is None
        assert oracle.matrix_select(t, c, 0) is None


def test_out_of_range_rejected():
    S = wtgen.uniform(100, 10, 3).astype(np.uint8)
    S[5] = 12
    with pytest.raises(ValueError):
        oracle.build_matrix(S, 10)
