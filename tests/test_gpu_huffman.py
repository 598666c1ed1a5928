"""GPU parity of the Huffman-shaped wavelet tree against the CPU oracle.

Integer work: the code table (every symbol's length and canonical code),
the depth sizes, every bitmap word and every directory entry (padding
included) must be equal to the oracle's, which builds the tree from its
definition; queries must answer for S.  Cases span alphabets from 2 to 2^20
symbols, skewed and uniform counts, lengths across several tiles with
ragged tails, n = 0, one distinct symbol, symbols out of range and absent
from the counts.
"""
import sys

import numpy as np
import pytest

import oracle
import wtgen
from tests import treecheck as tc

pytestmark = pytest.mark.gpu


def _wt():
    from paper_1610_05994_amd import wtree
    return wtree


def _dev():
    import torch
    return torch.device("cuda:0")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def build_and_compare(S, sigma, tag=""):
    wt = _wt()
    _say("case huffman %s: n=%d sigma=%d width=%d" % (tag, S.shape[0], sigma, S.dtype.itemsize))
    t = wt.build_huffman(wt.to_device(S, _dev()), sigma)
    assert t.status() == wt.WT_OK
    ref = oracle.build_huffman(S, sigma)
    assert t.levels == ref.levels
    assert np.array_equal(t.lengths(), ref.lengths), "code lengths"
    present = ref.lengths > 0
    assert np.array_equal(t.codes()[present], ref.codes[present]), "canonical codes"
    assert list(t.sizes) == list(ref.sizes)
    gb, gr = t.bitmaps(), t.ranks()
    for d in range(ref.levels):
        msg = tc.compare_levels(gb[d][None, :], ref.bitmaps[d][None, :])
        assert msg is None, "%s depth %d: %s" % (tag, d, msg)
        msg = tc.compare_levels(gr[d][None, :], ref.ranks[d][None, :], "rank")
        assert msg is None, "%s depth %d: %s" % (tag, d, msg)
    return t, ref


CASES = [
    (2, 1000, 1.0), (3, 70_001, 1.5), (4, 4097, 0.0), (20, 100_000, 1.0), (256, 300_007, 1.1),
    (256, 1 << 20, 0.0), (1 << 12, 500_000, 0.9), (1 << 16, 1_000_003, 1.0), (1 << 20, 600_000, 1.0),
    (1 << 20, 3 << 20, 1.0),
]


@pytest.mark.parametrize("sigma,n,s", CASES)
def test_huffman_matches_oracle(sigma, n, s):
    S = wtgen.uniform(n, sigma, 41 + n) if s == 0.0 else wtgen.zipf(n, sigma, s, 41 + n)
    t, _ = build_and_compare(S, sigma, tag="zipf%.1f" % s)
    t.close()


def test_huffman_c2_shaped_large():
    # the single-build workload's distribution at 2^24 symbols (u8, sigma 256, Zipf 1.1)
    S, sigma = wtgen.workload("c2@lg24")
    t, _ = build_and_compare(S, sigma, tag="c2@lg24")
    t.close()


@pytest.mark.parametrize("sigma,n,s", [(7, 3000, 1.0), (300, 20_000, 1.2), (1 << 16, 50_000, 0.8)])
def test_huffman_queries(sigma, n, s):
    import torch
    S = wtgen.zipf(n, sigma, s, 5 + sigma)
    t, ref = build_and_compare(S, sigma, tag="queries")
    dev = _dev()
    acc = t.access(torch.arange(n, device=dev)).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
    assert np.array_equal(acc, S.astype(np.int64))
    rng = np.random.Generator(np.random.PCG64(n))
    cs = np.concatenate([S[rng.integers(0, n, 300)].astype(np.int64), rng.integers(0, sigma, 100)])
    iq = rng.integers(0, n + 1, cs.shape[0])
    r = t.rank(cs, iq).cpu().numpy()
    # brute force over S, via per-symbol occurrence lists
    occ = {int(c): np.flatnonzero(S == c) for c in np.unique(cs)}
    want = np.array([np.searchsorted(occ[int(c)], i) for c, i in zip(cs, iq)])
    assert np.array_equal(r, want)
    js = np.array([rng.integers(1, occ[int(c)].shape[0] + 2) if occ[int(c)].shape[0] else 1 for c in cs])
    sel = t.select(cs, js).cpu().numpy().view(np.uint64)
    wsel = np.array([occ[int(c)][j - 1] if j <= occ[int(c)].shape[0] else np.iinfo(np.uint64).max
                     for c, j in zip(cs, js)], dtype=np.uint64)
    assert np.array_equal(sel, wsel)
    t.close()


def test_huffman_equal_counts_equal_the_balanced_tree():
    wt = _wt()
    rng = np.random.Generator(np.random.PCG64(8))
    S = rng.permutation(np.repeat(np.arange(256), 4099)).astype(np.uint8)
    h, _ = build_and_compare(S, 256, tag="equal-counts")
    b = wt.build(wt.to_device(S, _dev()), 256)
    bb, br = b.bitmaps(), b.ranks()
    hb, hr = h.bitmaps(), h.ranks()
    for d in range(8):
        assert np.array_equal(hb[d], bb[d]) and np.array_equal(hr[d], br[d])
    h.close()
    b.close()


def test_huffman_edge_cases():
    import torch
    wt = _wt()
    dev = _dev()
    # n = 0
    t = wt.build_huffman(torch.zeros(0, dtype=torch.uint8, device=dev), 5)
    assert t.status() == wt.WT_OK and t.levels == 0
    t.close()
    # one distinct symbol: no levels, queries still answer
    S = np.full(5000, 9, dtype=np.uint8)
    t = wt.build_huffman(wt.to_device(S, dev), 12)
    assert t.status() == wt.WT_OK and t.levels == 0
    assert int(t.access(torch.tensor([4999], device=dev)).item()) == 9
    assert t.rank([9, 3], [4000, 4000]).cpu().tolist() == [4000, 0]
    assert t.select([9], [5000]).cpu().tolist() == [4999]
    t.close()
    # two symbols
    S = np.array([1, 0, 1, 1, 0, 1] * 1000, dtype=np.uint8)
    t, _ = build_and_compare(S, 2, tag="two")
    t.close()
    # a symbol >= sigma, and one that the counts call absent: reported, not built on
    S = wtgen.zipf(10_000, 16, 1.0, 3)
    counts = np.bincount(S, minlength=16).astype(np.uint64)
    bad = S.copy()
    bad[777] = 16
    t = wt.build_huffman(wt.to_device(bad, dev), 16, counts=counts)
    assert t.status() == wt.WT_ERANGE
    t.close()
    S2 = (S % 15).astype(np.uint8)          # symbol 15 never occurs
    c2 = np.bincount(S2, minlength=16).astype(np.uint64)
    bad = S2.copy()
    bad[5] = 15
    t = wt.build_huffman(wt.to_device(bad, dev), 16, counts=c2)
    assert t.status() == wt.WT_ERANGE
    t.close()
    # counts that are not S's histogram (wrong total) are refused on the host
    rc, _, _ = wt.wt_huffman_footprint(c2 + 1, S2.shape[0], 16, 1)
    assert rc == wt.WT_EINVAL
    # the same build again on the same inputs is clean
    t, _ = build_and_compare(S, 16, tag="after-error")
    t.close()
