"""Pins of the 4-ary wavelet-tree oracle (fan-out 4: level i lists digit i
of every symbol's base-4 code, node after node, stable inside a node).

Independent of the oracle's C code:
- library routine: level i equals digit i of S stably sorted (numpy,
  kind="stable") by its top i digits;
- relation to the binary tree: with an even number of bits, the high bit of
  level i's digits is the binary tree's level 2i (both list the symbols in
  the order of their top 2i bits);
- closed forms: sigma <= 4 gives S itself; level 0 is the top digit of S in
  input order; a sorted input gives every digit plane in input order; the
  directory is the running count of each digit and its four counts add up to
  the position;
- brute force: access / rank / select through the digit walk equal S, counts
  of S[:i] and positions of the j-th occurrence, for every argument on small
  inputs.
"""
import numpy as np
import pytest

import oracle
import wtgen


def unpack_digits(words: np.ndarray, n: int) -> np.ndarray:
    w = words.astype(np.uint64)
    p = np.arange(n, dtype=np.uint64)
    return ((w[(p >> np.uint64(5)).astype(np.int64)] >> (np.uint64(2) * (p & np.uint64(31)))) & np.uint64(3)).astype(np.int64)


def digits_by_argsort(S, sigma):
    L4 = oracle.levels4(sigma)
    S = S.astype(np.int64)
    out = []
    for i in range(L4):
        A = S[np.argsort(S >> (2 * (L4 - i)), kind="stable")]
        out.append((A >> (2 * (L4 - 1 - i))) & 3)
    return out


SIGMAS = [2, 3, 4, 5, 16, 20, 64, 255, 256, 1000, 1 << 16, (1 << 20) + 7]


@pytest.mark.parametrize("sigma", SIGMAS)
def test_levels_match_stable_sort(sigma):
    for k, n in enumerate([0, 1, 2, 31, 32, 33, 511, 512, 513, 3000]):
        S = wtgen.uniform(n, sigma, 900 + 7 * k + sigma % 89)
        t = oracle.build4(S, sigma)
        want = digits_by_argsort(S, sigma)
        assert t.levels == len(want) == (max(0, (sigma - 1).bit_length()) + 1) // 2
        for i in range(t.levels):
            assert np.array_equal(unpack_digits(t.digits[i], n), want[i]), (sigma, n, i)
            # padding digits are zero
            total = t.digits.shape[1] * 32
            assert not unpack_digits(t.digits[i], total)[n:].any()


def test_skewed_and_sorted_inputs():
    for S, sigma in [(wtgen.zipf(20_000, 256, 1.1, 31), 256), (wtgen.gauss_mix(20_000, 1 << 20, 32), 1 << 20),
                     (wtgen.cont(5000, 1 << 12), 1 << 12)]:
        t = oracle.build4(S, sigma)
        for i, want in enumerate(digits_by_argsort(S, sigma)):
            assert np.array_equal(unpack_digits(t.digits[i], len(S)), want)


def test_high_bits_are_the_binary_levels():
    # sigma = 2^8 (l = 8, even): digit level i's high bits = binary level 2i
    for S, sigma in [(wtgen.uniform(5000, 256, 41), 256), (wtgen.zipf(7000, 1 << 12, 1.0, 42), 1 << 12)]:
        t4 = oracle.build4(S, sigma)
        t2 = oracle.build(S, sigma)
        n = len(S)
        for i in range(t4.levels):
            hi = unpack_digits(t4.digits[i], n) >> 1
            p = np.arange(n)
            b = (t2.bitmaps[2 * i][p >> 6] >> (p & 63).astype(np.uint64)) & np.uint64(1)
            assert np.array_equal(hi, b.astype(np.int64)), i


def test_closed_forms():
    # sigma <= 4: the one level is S itself
    for sigma in (2, 3, 4):
        S = wtgen.uniform(1000, sigma, 50 + sigma)
        t = oracle.build4(S, sigma)
        assert t.levels == 1 and np.array_equal(unpack_digits(t.digits[0], 1000), S.astype(np.int64))
    # level 0 is the top digit in input order; sorted input: every plane in order
    S = wtgen.uniform(4000, 1 << 10, 53).astype(np.uint16)
    t = oracle.build4(S, 1 << 10)
    assert np.array_equal(unpack_digits(t.digits[0], 4000), (S.astype(np.int64) >> 8) & 3)
    S = np.sort(S)
    t = oracle.build4(S, 1 << 10)
    for i in range(t.levels):
        assert np.array_equal(unpack_digits(t.digits[i], 4000), (S.astype(np.int64) >> (2 * (4 - i))) & 3)
    # directory: running counts per digit, summing to the position
    S = wtgen.uniform(2000, 300, 54).astype(np.uint16)
    t = oracle.build4(S, 300)
    for i in range(t.levels):
        d = unpack_digits(t.digits[i], 2000)
        K = (2000 + 511) // 512 + 1
        for k in range(K):
            upto = min(512 * k, 2000)
            assert [int(t.dir[i, k, x]) for x in range(4)] == [int((d[:upto] == x).sum()) for x in range(4)]
            assert int(t.dir[i, k].sum()) == upto
        assert not t.dir[i, K:].any()


@pytest.mark.parametrize("sigma,n", [(2, 50), (5, 120), (16, 200), (20, 257), (256, 300), (1 << 12, 150)])
def test_queries_brute_force(sigma, n):
    S = wtgen.uniform(n, sigma, 60 + n + sigma % 31)
    t = oracle.build4(S, sigma)
    for i in range(n):
        assert oracle.access4(t, i) == int(S[i])
    cs = sorted(set(int(x) for x in S))[:12] + [sigma - 1]
    for c in cs:
        occ = np.flatnonzero(S == c)
        for i in range(n + 1):
            assert oracle.rank4(t, c, i) == int((S[:i] == c).sum())
        for j in range(1, len(occ) + 2):
            got = oracle.select4(t, c, j)
            assert got == (int(occ[j - 1]) if j <= len(occ) else None)
        assert oracle.select4(t, c, 0) is None


def test_out_of_range_rejected():
    S = np.array([1, 2, 9], dtype=np.uint8)
    with pytest.raises(ValueError):
        oracle.build4(S, 9)
