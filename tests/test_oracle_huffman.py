"""Pins of the oracle's Huffman-shaped wavelet tree (CPU only).

The paper names Huffman-shaped trees as future work (Section 5) without a
definition or printed values, so the oracle is pinned to things outside it:

* a sequence worked by hand from the construction rules (tests/golden);
* optimality of the code lengths: the Kraft sum is exactly 1, and the cost
  sum(count * length) equals the minimum over every complete length vector
  (brute force on small alphabets) and the cost of a heap-based Huffman
  merge (a different procedure; ties may give other lengths, never another
  cost);
* equal counts over 2^k symbols: every code has length k, the canonical code
  of a symbol is the symbol itself, and the tree is the balanced one of
  Section 2.2 (the oracle's balanced tree, pinned elsewhere), bit for bit;
* every depth d equals the next code bit of the symbols whose code is longer
  than d, stably sorted by their first d code bits (numpy stable argsort);
* access / rank / select against S by brute force over all arguments;
* depth sizes and the directory as a cumulative popcount.
"""
import heapq
import itertools
import json
import os

import numpy as np
import pytest

import oracle
import wtgen

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "huffman_ties.json")


def _bits(words, size):
    return np.unpackbits(np.asarray(words, np.uint64).view(np.uint8), bitorder="little")[:size].astype(np.int64)


def _counts(S, sigma):
    return np.bincount(S.astype(np.int64), minlength=sigma).astype(np.uint64)


def test_worked_example_with_ties():
    g = json.load(open(GOLDEN))
    S = np.array(g["S"], dtype=np.uint8)
    t = oracle.build_huffman(S, g["sigma"])
    assert t.lengths.tolist() == g["lengths"]
    assert t.codes.tolist() == g["codes"]
    assert t.sizes == g["sizes"]
    for d, want in enumerate(g["levels"]):
        assert "".join(map(str, _bits(t.bitmaps[d], t.sizes[d]))) == want


def _cost(counts, lengths):
    return int(sum(int(c) * int(l) for c, l in zip(counts, lengths)))


@pytest.mark.parametrize("seed", range(40))
def test_lengths_are_optimal_brute_force(seed):
    rng = np.random.Generator(np.random.PCG64(seed))
    k = int(rng.integers(2, 7))
    counts = rng.integers(1, 20, k).astype(np.uint64)
    if seed % 5 == 0:
        counts[:] = counts[0]                     # all ties
    ln, L = oracle.huffman_lengths(counts)
    assert sum(2.0 ** -int(x) for x in ln) == 1.0  # complete code
    best = min(_cost(counts, v) for v in itertools.product(range(1, k), repeat=k)
               if sum(2.0 ** -x for x in v) == 1.0)
    assert _cost(counts, ln) == best
    assert L == int(ln.max())


def _heap_cost(counts):
    h = [int(c) for c in counts if c > 0]
    heapq.heapify(h)
    cost = 0
    while len(h) > 1:
        a, b = heapq.heappop(h), heapq.heappop(h)
        cost += a + b
        heapq.heappush(h, a + b)
    return cost


@pytest.mark.parametrize("sigma,s", [(256, 1.1), (1000, 1.0), (4096, 0.7), (37, 2.0)])
def test_cost_equals_heap_huffman(sigma, s):
    S = wtgen.zipf(200_000, sigma, s, 5 + sigma)
    counts = _counts(S, sigma)
    ln, L = oracle.huffman_lengths(counts)
    assert _cost(counts, ln) == _heap_cost(counts)
    assert all((ln[c] == 0) == (counts[c] == 0) for c in range(sigma))
    present = counts > 0
    assert sum(2.0 ** -int(x) for x in ln[present]) == pytest.approx(1.0, abs=0)


def test_canonical_codes_are_prefix_free_and_ordered():
    S = wtgen.zipf(100_000, 300, 1.2, 9)
    counts = _counts(S, 300)
    ln, L = oracle.huffman_lengths(counts)
    code = oracle.huffman_codes(ln, L)
    syms = sorted((int(ln[c]), c) for c in range(300) if ln[c])
    # consecutive in (length, symbol) order; left-aligned codes increase
    prev = None
    for l, c in syms:
        v = int(code[c]) << (L - l)
        if prev is not None:
            assert v > prev
        prev = v
    words = {format(int(code[c]), "0%db" % l) for l, c in syms}
    for a in words:
        for b in words:
            assert a == b or not b.startswith(a)


@pytest.mark.parametrize("k", [1, 2, 4, 8])
def test_equal_counts_give_the_balanced_tree(k):
    sigma = 1 << k
    rng = np.random.Generator(np.random.PCG64(k))
    S = rng.permutation(np.repeat(np.arange(sigma), 50)).astype(np.uint8 if k <= 8 else np.uint16)
    h = oracle.build_huffman(S, sigma)
    assert h.levels == k and set(h.lengths.tolist()) == {k}
    assert h.codes.tolist() == list(range(sigma))
    bal = oracle.build(S, sigma)
    for d in range(k):
        assert h.sizes[d] == S.shape[0]
        assert np.array_equal(h.bitmaps[d], bal.bitmaps[d])
        assert np.array_equal(h.ranks[d], bal.ranks[d])


@pytest.mark.parametrize("sigma,n,s", [(5, 1000, 1.0), (256, 5000, 1.1), (1 << 12, 20_000, 0.9),
                                       (3, 4097, 2.0), (300, 64, 1.0)])
def test_levels_equal_stable_sort_of_code_prefixes(sigma, n, s):
    S = wtgen.zipf(n, sigma, s, n + sigma)
    t = oracle.build_huffman(S, sigma)
    ln = t.lengths[S].astype(np.int64)
    code = t.codes[S].astype(np.int64)
    for d in range(t.levels):
        live = np.flatnonzero(ln > d)
        pre = code[live] >> (ln[live] - d)
        order = live[np.argsort(pre, kind="stable")]
        want = (code[order] >> (ln[order] - 1 - d)) & 1
        assert t.sizes[d] == live.shape[0]
        assert np.array_equal(_bits(t.bitmaps[d], t.sizes[d]), want), d
        # padding bits past n_d are zero, the directory is a cumulative popcount
        allb = _bits(t.bitmaps[d], t.bitmaps[d].shape[0] * 64)
        assert not allb[t.sizes[d]:].any()
        cum = np.concatenate([[0], np.cumsum(want)])
        K = (t.sizes[d] + 511) // 512 + 1
        assert t.ranks[d][:K - 1].tolist() == [int(cum[512 * k]) for k in range(K - 1)]
        assert int(t.ranks[d][K - 1]) == int(cum[-1])
        assert not t.ranks[d][K:].any()
    assert sum(t.sizes) == int((ln).sum())


@pytest.mark.parametrize("sigma,n,s", [(6, 300, 1.0), (64, 500, 1.3), (256, 300, 0.5), (2, 200, 1.0)])
def test_queries_brute_force(sigma, n, s):
    S = wtgen.zipf(n, sigma, s, 77 + sigma)
    t = oracle.build_huffman(S, sigma)
    w = oracle.HuffmanWalker(t)
    assert [w.access(i) for i in range(n)] == S.astype(int).tolist()
    for c in range(sigma):
        occ = np.flatnonzero(S == c)
        for i in range(n + 1):
            assert w.rank(c, i) == int((S[:i] == c).sum())
        for j in range(1, occ.shape[0] + 2):
            want = int(occ[j - 1]) if j <= occ.shape[0] else None
            assert w.select(c, j) == want


def test_one_symbol_and_empty_input():
    S = np.full(1000, 7, dtype=np.uint8)
    t = oracle.build_huffman(S, 10)
    assert t.levels == 0 and t.only == 7 and not t.lengths.any()
    w = oracle.HuffmanWalker(t)
    assert w.access(999) == 7 and w.rank(7, 500) == 500 and w.rank(3, 500) == 0
    assert w.select(7, 1000) == 999 and w.select(7, 1001) is None and w.select(3, 1) is None
    e = oracle.build_huffman(np.zeros(0, dtype=np.uint8), 4)
    assert e.levels == 0 and e.only == -1


def test_comparator_catches_a_planted_mistake():
    # a flipped code bit in one symbol's code must change some level
    S = wtgen.zipf(3000, 50, 1.0, 3)
    t = oracle.build_huffman(S, 50)
    bad = t.codes.copy()
    c = int(np.argmax(t.lengths))
    bad[c] ^= 1
    ln = t.lengths[S].astype(np.int64)
    d = int(t.lengths[c]) - 1
    live = np.flatnonzero(ln > d)
    code_bad = bad[S].astype(np.int64)
    pre = code_bad[live] >> (ln[live] - d)
    order = live[np.argsort(pre, kind="stable")]
    want_bad = (code_bad[order] >> (ln[order] - 1 - d)) & 1
    assert not np.array_equal(_bits(t.bitmaps[d], t.sizes[d]), want_bad)
