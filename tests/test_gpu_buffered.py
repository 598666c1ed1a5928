"""GPU parity of the buffered build (partial trees per buffer, offsets by
prefix sums over the buffers, then the merge of the partial bitmaps) against
the oracle's wavelet tree of the whole sequence: every bitmap word and rank
entry, padding included, bit-exact.  Covers ragged last buffers, buffers
shorter than a tile and than a 512-bit block, many buffers, alphabets up to
2^24 (far more nodes than symbols per buffer), sigma = 1 and 2, n = 0, a
single buffer, host pageable / page-locked / device sources, out-of-range
symbols in one buffer, and the workspace reused for a second build."""
import numpy as np
import pytest

import oracle
import wtgen
from tests import treecheck as tc

pytestmark = pytest.mark.gpu


def _wt():
    from paper_1610_05994_amd import wtree
    return wtree


def _check(S, sigma, buf, tag, source="host"):
    import torch
    wt = _wt()
    src = S
    if source == "pinned":
        src = wt._torch().from_numpy(np.ascontiguousarray(S).view({1: np.uint8, 2: np.int16, 4: np.int32}[S.dtype.itemsize])).pin_memory()
    elif source == "device":
        src = wt.to_device(S, torch.device("cuda:0"))
    print("buffered: n=%d sigma=%d buffer=%d source=%s" % (len(S), sigma, buf, source), flush=True)
    t = wt.build_buffered(src, sigma, buf, width=S.dtype.itemsize, device="cuda:0")
    ref = oracle.build(S, sigma)
    assert t.status() == wt.WT_OK, tag
    assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None, tag
    assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None, tag
    return t, ref


@pytest.mark.parametrize("sigma", [2, 3, 20, 256, 1000, 1 << 16, 1 << 20])
def test_buffered_parity(sigma):
    cases = [(100, 7), (1000, 64), (5000, 511), (40_000, 4096), (100_003, 30_000), (300_001, 65_536)]
    for k, (n, buf) in enumerate(cases):
        S = wtgen.uniform(n, sigma, 7100 + 17 * k + sigma % 97)
        t, _ = _check(S, sigma, buf, (n, sigma, buf))
        t.close()


def test_buffered_skewed_and_sparse():
    cases = [(wtgen.zipf(1 << 21, 256, 1.1, 71), 256, 300_000),
             (wtgen.gauss_mix(1 << 20, 1 << 20, 72), 1 << 20, 1 << 18),
             (wtgen.cont(200_000, 1 << 16), 1 << 16, 33_333),
             (np.full(70_000, 5, np.uint8), 8, 10_000),
             (wtgen.uniform(40_000, 10, 73).astype(np.uint32) * 1_000_000, 1 << 24, 9_000)]
    for S, sigma, buf in cases:
        t, _ = _check(S, sigma, buf, (len(S), sigma, buf))
        t.close()


@pytest.mark.parametrize("source", ["host", "pinned", "device"])
def test_buffered_sources(source):
    S = wtgen.zipf(1 << 20, 256, 1.1, 74)
    t, _ = _check(S, 256, 100_000, source, source)
    t.close()


def test_buffered_degenerate():
    wt = _wt()
    # sigma = 1: no levels, status only
    t, _ = _check(np.zeros(5000, np.uint8), 1, 1000, "sigma1")
    assert t.levels == 0
    t.close()
    # n = 0, and a single buffer (the ordinary build of a staged copy)
    t, _ = _check(np.zeros(0, np.uint8), 256, 1000, "empty")
    t.close()
    S = wtgen.uniform(12_345, 300, 75).astype(np.uint16)
    t, _ = _check(S, 300, 1 << 20, "single")
    t.close()
    # one symbol per buffer
    S = wtgen.uniform(600, 50, 76)
    t, _ = _check(S, 50, 1, "one per buffer")
    t.close()


def test_buffered_out_of_range_and_reuse():
    import torch
    wt = _wt()
    S = wtgen.uniform(50_000, 100, 77)
    bad = S.copy()
    bad[37_000] = 120                  # inside the fourth buffer of 10000
    rc, tb, wb = wt.wt_buffered_footprint(len(S), 100, 1, 10_000)
    assert rc == wt.WT_OK
    tree = torch.empty(tb, dtype=torch.uint8, device="cuda:0")
    work = torch.empty(wb, dtype=torch.uint8, device="cuda:0")
    t = wt.build_buffered(bad, 100, 10_000, device="cuda:0", tree_mem=tree, work_mem=work)
    assert t.status() == wt.WT_ERANGE
    t.close()
    # the same memory, a good input: status and tree are clean again
    t = wt.build_buffered(S, 100, 10_000, device="cuda:0", tree_mem=tree, work_mem=work)
    ref = oracle.build(S, 100)
    assert t.status() == wt.WT_OK
    assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None
    assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None
    t.close()


def test_buffered_queries_and_large():
    """2^25 u8 Zipf symbols in 2^22-symbol buffers; rank / select / access
    through the merged tree against the oracle."""
    wt = _wt()
    S = wtgen.zipf(1 << 25, 256, 1.1, 78)
    t, ref = _check(S, 256, 1 << 22, "large")
    rng = np.random.default_rng(79)
    pos = rng.integers(0, len(S), 200).astype(np.uint64)
    assert np.array_equal(t.access(pos).cpu().numpy().astype(np.int64), S[pos.astype(np.int64)].astype(np.int64))
    cs = rng.integers(0, 256, 200).astype(np.uint32)
    iv = rng.integers(0, len(S) + 1, 200).astype(np.uint64)
    got = t.rank(cs, iv).cpu().numpy().view(np.uint64)
    want = np.array([oracle.rank(ref, int(c), int(i)) for c, i in zip(cs, iv)], np.uint64)
    assert np.array_equal(got, want)
    t.close()
