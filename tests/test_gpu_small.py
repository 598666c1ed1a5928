"""GPU parity of the one-workgroup build of short sequences.

Short sequences (up to 15360 / 10240 / 6144 symbols of 1 / 2 / 4 bytes with
64 KB of LDS, up to 32768 / 26624 / 15360 with 160 KB) are built by one
workgroup with every level in LDS; node boundaries come from a
segmented scan instead of per-node tables.  Bit-exact against the oracle at
the chunk-size boundaries (4096, 8192 symbols), at the capacities, for every
alphabet size class (up to 2^24, i.e. far more nodes than symbols), for
sorted, constant and sparse inputs, out-of-range symbols, and inside
batches mixed with long sequences.
"""
import numpy as np
import pytest

import oracle
import wtgen
from tests import treecheck as tc

pytestmark = pytest.mark.gpu

CAP = {1: 15360, 2: 10240, 4: 6144}
CAP2 = {1: 32768, 2: 26624, 4: 15360}


def _wt():
    from paper_1610_05994_amd import wtree
    return wtree


def _check(t, S, sigma, tag):
    ref = oracle.build(S, sigma)
    assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None, tag
    assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None, tag


@pytest.mark.parametrize("width,sigmas", [(1, [1, 2, 3, 17, 256]), (2, [5, 1 << 12, 1 << 16]),
                                          (4, [2, 1000, 1 << 20, 1 << 24])])
def test_small_sizes_and_alphabets(width, sigmas):
    wt = _wt()
    import torch
    dev = torch.device("cuda:0")
    ns = [0, 1, 2, 63, 64, 65, 511, 512, 513, 4095, 4096, 4097, 8191, 8192, 8193, CAP[width] - 1, CAP[width],
          CAP[width] + 1, 16384, 16385, CAP2[width] - 1, CAP2[width]]
    for sigma in sigmas:
        for k, n in enumerate(sorted(set(x for x in ns if x <= CAP2[width]))):
            S = wtgen.uniform(n, sigma, 1300 + 17 * k + sigma % 1000).astype(wtgen.dtype_for(width))
            print("small: n=%d sigma=%d width=%d" % (n, sigma, width), flush=True)
            t = wt.build(wt.to_device(S, dev) if n else torch.zeros(0, dtype={1: torch.uint8, 2: torch.int16,
                                                                               4: torch.int32}[width], device=dev),
                         sigma)
            assert t.status() == wt.WT_OK
            _check(t, S, sigma, (n, sigma, width))
            t.close()


def test_small_structured_inputs():
    wt = _wt()
    import torch
    dev = torch.device("cuda:0")
    cases = [
        (np.sort(wtgen.uniform(9000, 1 << 12, 3)).astype(np.uint16), 1 << 12),
        (np.sort(wtgen.uniform(6000, 1 << 24, 4)).astype(np.uint32)[::-1].copy(), 1 << 24),
        (np.full(15000, 200, np.uint8), 256),
        ((wtgen.uniform(4000, 8, 5).astype(np.uint32) * 100_000), 1 << 20),   # 8 distinct, far apart
        (wtgen.zipf(15360, 256, 1.2, 6), 256),
    ]
    for S, sigma in cases:
        print("small structured: n=%d sigma=%d" % (len(S), sigma), flush=True)
        t = wt.build(wt.to_device(S, dev), sigma)
        _check(t, S, sigma, (len(S), sigma))
        t.close()


def test_small_out_of_range_and_status_reset():
    wt = _wt()
    import torch
    dev = torch.device("cuda:0")
    S = wtgen.uniform(3000, 100, 8).astype(np.uint8)
    S[1234] = 150
    t = wt.build(wt.to_device(S, dev), 100)
    assert t.status() == wt.WT_ERANGE
    # the same tree memory reused for a valid build reports OK again
    S2 = wtgen.uniform(3000, 100, 9).astype(np.uint8)
    t2 = wt.build(wt.to_device(S2, dev), 100, tree_mem=t.tree_mem)
    assert t2.status() == wt.WT_OK
    _check(t2, S2, 100, "reuse")


def test_small_and_tiled_sequences_in_one_batch():
    wt = _wt()
    import torch
    dev = torch.device("cuda:0")
    specs = [(100, 4, 1), (15360, 256, 1), (15361, 256, 1), (70_000, 20, 1), (10240, 1 << 16, 2),
             (10241, 1 << 16, 2), (6144, 1 << 24, 4), (6145, 1 << 20, 4), (0, 7, 1), (1, 1 << 20, 4), (300, 1, 1),
             (32768, 256, 1), (32769, 256, 1), (26624, 1 << 16, 2), (15360, 1 << 24, 4), (15361, 1 << 24, 4)]
    Ss = [wtgen.uniform(n, sg, 1400 + k).astype(wtgen.dtype_for(w)) for k, (n, sg, w) in enumerate(specs)]
    print("small+tiled batch: %d sequences" % len(Ss), flush=True)
    dS = [wt.to_device(S, dev) if len(S) else torch.zeros(0, dtype={1: torch.uint8, 2: torch.int16,
                                                                     4: torch.int32}[S.dtype.itemsize], device=dev)
          for S in Ss]
    trees = wt.build_batch(dS, [sg for _, sg, _ in specs])
    for t, S, (n, sg, w) in zip(trees, Ss, specs):
        assert t.status() == wt.WT_OK
        _check(t, S, sg, (n, sg, w))
        t.close()
