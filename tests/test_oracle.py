"""Pins of the CPU oracle against facts that do not come from the oracle.

* the paper's worked example (Section 2.2 figure and access walk; Section
  3.1 snapshot caption), stored in ``tests/golden/paper_example.json``;
* the stable-sort characterisation of every level (numpy stable argsort);
* brute-force access / rank / select computed directly on S;
* invariants: per-level popcounts, node boundaries from the histogram,
  children partitioning their parent;
* closed forms: sorted input (the paper's ``cont`` data, Section 4), sigma =
  2, constant input, level 0 being the most significant bit plane;
* the rank directory against a cumulative popcount;
* a full forward decode reproducing S.
"""
import json
import os

import numpy as np
import pytest

import oracle
import wtgen
from tests import treecheck as tc

HERE = os.path.dirname(os.path.abspath(__file__))


def _example():
    with open(os.path.join(HERE, "golden", "paper_example.json")) as f:
        g = json.load(f)
    alpha = g["alphabet"]
    S = np.array([alpha.index(ch) for ch in g["sequence"]], dtype=np.uint8)
    return g, alpha, S


def test_paper_example_access_walk():
    g, alpha, S = _example()
    t = oracle.build(S, len(alpha))
    assert t.levels == 4 and t.n == 30
    w = g["access_walk"]
    sym, bits, idx = oracle.access(t, w["position"])
    assert bits == w["bits"]
    assert idx[:3] == w["in_node_index_after_levels_0_1_2"]
    assert alpha[sym] == w["symbol"]
    # the symbol range halves along the walk exactly as printed
    lo, hi = 0, len(alpha) - 1
    ranges = [[lo, hi]]
    for b in bits:
        mid = (lo + hi + 1) // 2
        lo, hi = (mid, hi) if b else (lo, mid - 1)
        ranges.append([lo, hi])
    assert ranges == w["symbol_ranges"]


def test_paper_caption_positions():
    g, alpha, S = _example()
    t = oracle.build(S, len(alpha))
    for pos, ch in g["caption_positions"].items():
        assert alpha[oracle.access(t, int(pos))[0]] == ch


SIGMAS = [1, 2, 3, 4, 5, 16, 20, 27, 230, 256, 1 << 10, 1 << 16, 1 << 20]
NS = [0, 1, 2, 63, 64, 65, 511, 512, 513, 4095, 4096, 100_000]


@pytest.mark.parametrize("sigma", SIGMAS)
def test_levels_equal_stable_sort(sigma):
    for k, n in enumerate(NS):
        if sigma >= 1 << 16 and n == 100_000:
            n = 30_000
        S = wtgen.uniform(n, sigma, 1000 + k)
        t = oracle.build(S, sigma)
        want = tc.levels_by_stable_sort(S, sigma)
        msg = tc.compare_levels(t.bitmaps, want)
        assert msg is None, "sigma=%d n=%d: %s" % (sigma, n, msg)


@pytest.mark.parametrize("sigma", [2, 5, 16, 256, 1 << 12])
def test_levels_equal_stable_sort_skewed(sigma):
    S = wtgen.zipf(50_000, sigma, 1.1, 7)
    t = oracle.build(S, sigma)
    assert tc.compare_levels(t.bitmaps, tc.levels_by_stable_sort(S, sigma)) is None


def test_rank_directory_is_cumulative_popcount():
    for sigma, n in [(4, 0), (4, 1), (256, 511), (256, 512), (256, 513), (20, 70_001), (1 << 16, 4097)]:
        S = wtgen.uniform(n, sigma, n + sigma)
        t = oracle.build(S, sigma)
        assert tc.compare_levels(t.ranks, tc.ranks_by_cumsum(t.bitmaps, n), "rank") is None


@pytest.mark.parametrize("sigma,n", [(1, 17), (2, 100), (3, 64), (5, 130), (16, 300), (20, 257), (27, 90)])
def test_brute_force_queries(sigma, n):
    S = wtgen.uniform(n, sigma, sigma * 31 + n)
    t = oracle.build(S, sigma)
    for i in range(n):
        assert oracle.access(t, i)[0] == S[i]
    for c in range(sigma):
        occ = np.flatnonzero(S == c)
        for i in range(n + 1):
            assert oracle.rank(t, c, i) == int(np.count_nonzero(S[:i] == c))
        for j in range(0, occ.size + 2):
            want = int(occ[j - 1]) if 1 <= j <= occ.size else None
            assert oracle.select(t, c, j) == want


def test_brute_force_queries_skewed_large_alphabet():
    sigma, n = 1 << 10, 1500
    S = wtgen.zipf(n, sigma, 1.0, 5)
    t = oracle.build(S, sigma)
    for i in range(0, n, 7):
        assert oracle.access(t, i)[0] == S[i]
    for c in list(np.unique(S)[:40]) + [0, sigma - 1]:
        c = int(c)
        occ = np.flatnonzero(S == c)
        for i in range(0, n + 1, 13):
            assert oracle.rank(t, c, i) == int(np.count_nonzero(S[:i] == c))
        for j in range(0, occ.size + 2):
            want = int(occ[j - 1]) if 1 <= j <= occ.size else None
            assert oracle.select(t, c, j) == want


@pytest.mark.parametrize("sigma", [2, 20, 256, 1 << 14])
def test_invariants(sigma):
    n = 20_000
    S = wtgen.zipf(n, sigma, 1.0, 99)
    t = oracle.build(S, sigma)
    l = t.levels
    s = S.astype(np.int64)
    H = np.bincount(s, minlength=1 << l)
    P = np.concatenate([[0], np.cumsum(H)])
    for i in range(l):
        bits = tc.unpack_bits(t.bitmaps[i], n).astype(np.int64)
        # popcount of a level = symbols with that bit set
        assert bits.sum() == int(((s >> (l - 1 - i)) & 1).sum())
        # node v of level i spans [P[v << (l-i)], P[(v+1) << (l-i)]); its
        # zeros form its left child, whose size is the histogram's count
        for v in range(min(1 << i, 512)):
            b, e = P[v << (l - i)], P[(v + 1) << (l - i)]
            mid = P[(2 * v + 1) << (l - i - 1)]
            assert (e - b) - bits[b:e].sum() == mid - b
        # padding bits beyond n are zero
        assert not tc.unpack_bits(t.bitmaps[i], t.bitmaps.shape[1] * 64)[n:].any()


@pytest.mark.parametrize("sigma", [4, 16, 1 << 6, 1 << 10, 1 << 14])
def test_sorted_input_levels_are_bit_planes(sigma):
    # the paper's ``cont`` data: a sorted sequence keeps input order at every
    # level, so level i is simply bit plane (l-1-i) of S
    n = sigma * 37 + 11
    S = wtgen.cont(n, sigma)
    assert np.all(np.diff(S.astype(np.int64)) >= 0)
    t = oracle.build(S, sigma)
    l = t.levels
    for i in range(l):
        want = tc.pack_bits((S.astype(np.int64) >> (l - 1 - i)) & 1, t.bitmaps.shape[1])
        assert np.array_equal(t.bitmaps[i], want)


def test_level0_is_msb_plane_and_binary_alphabet_is_identity():
    S = wtgen.uniform(10_000, 2, 3)
    t = oracle.build(S, 2)
    assert np.array_equal(t.bitmaps[0], tc.pack_bits(S, t.bitmaps.shape[1]))
    S = wtgen.uniform(10_000, 300, 4)
    t = oracle.build(S, 300)
    assert np.array_equal(t.bitmaps[0], tc.pack_bits((S.astype(np.int64) >> 8) & 1, t.bitmaps.shape[1]))


def test_constant_input_gives_constant_levels():
    for c in [0, 5, 255]:
        S = np.full(3000, c, dtype=np.uint8)
        t = oracle.build(S, 256)
        for i in range(8):
            bits = tc.unpack_bits(t.bitmaps[i], 3000)
            assert np.all(bits == ((c >> (7 - i)) & 1))


@pytest.mark.parametrize("sigma", [1, 2, 7, 256, 1 << 16, 1 << 20])
def test_decode_roundtrip(sigma):
    for n in [0, 1, 77, 5000]:
        S = wtgen.uniform(n, sigma, n * 7 + sigma)
        t = oracle.build(S, sigma)
        assert np.array_equal(oracle.decode(t), S.astype(np.uint32))


def test_edge_cases_and_errors():
    t = oracle.build(np.zeros(0, np.uint8), 256)
    assert t.bitmaps.shape == (8, 0) and t.ranks.shape == (8, 8)
    assert not t.ranks.any()
    t = oracle.build(np.zeros(10, np.uint8), 1)
    assert t.levels == 0
    assert oracle.build_status(np.zeros(4, np.uint8), 0) == oracle.EINVAL
    assert oracle.build_status(np.array([0, 3, 4], np.uint8), 4) == oracle.ERANGE
    assert oracle.build_status(np.zeros(4, np.uint8), 300, 1) == oracle.EINVAL
    assert oracle.build_status(np.zeros(4, np.uint8), 4, 3) == oracle.EINVAL


def test_comparator_reports_a_flipped_bit():
    # tester self-test: a single corrupted bit or rank entry is located
    S = wtgen.uniform(5000, 256, 8)
    t = oracle.build(S, 256)
    bad = t.bitmaps.copy()
    bad[5, 17] ^= np.uint64(1 << 9)
    msg = tc.compare_levels(bad, t.bitmaps)
    assert msg is not None and "level 5 index 17" in msg
    badr = t.ranks.copy()
    badr[2, 3] += np.uint64(1)
    msg = tc.compare_levels(badr, t.ranks, "rank")
    assert msg is not None and "level 2 index 3" in msg
