"""GPU parity of every tile geometry the autotuner may choose.

The geometry (one workgroup per sequence with 64 KB or 160 KB of LDS, or
tiled level passes with 32, 64 or 128 lane bytes) changes how the work is split, never the tree: for
every valid geometry, single and batched builds must equal the oracle bit
for bit.  Lengths straddle the tile sizes (512 .. 8192 symbols) with ragged
tails; lengths above the one-workgroup capacity fall back to tiles.
"""
import numpy as np
import pytest

import oracle
import wtgen
from tests import treecheck as tc

pytestmark = pytest.mark.gpu


def _mods():
    from paper_1610_05994_amd import tune, wtree
    return tune, wtree


def _force(lane_bytes):
    tune, wt = _mods()
    for mode in (0, 1):
        for width in (1, 2, 4):
            lb = lane_bytes if (lane_bytes in (1, 2) or lane_bytes in tune.candidates(width)) else 0
            for levels in range(1, min(24, 8 * width) + 1):
                for lg_n in range(0, 41):
                    assert wt.wt_tune_set(mode, width, levels, lg_n, lb) == wt.WT_OK


@pytest.fixture
def restore_table():
    yield
    tune, _ = _mods()
    tune.reset()
    tune.load()


CASES = [  # (n, sigma, width)
    (1, 2, 1), (511, 3, 1), (2049, 256, 1), (8191, 200, 1), (70_001, 256, 1),
    (513, 16, 2), (4097, 1 << 12, 2), (50_000, 1 << 16, 2),
    (1025, 1 << 20, 4), (8193, 5000, 4), (60_000, 1 << 20, 4),
]


@pytest.mark.parametrize("lane_bytes", [1, 2, 32, 64, 128])
def test_every_geometry_builds_the_oracle_tree(lane_bytes, restore_table):
    _, wt = _mods()
    import torch
    _force(lane_bytes)
    for k, (n, sigma, width) in enumerate(CASES):
        S = wtgen.uniform(n, sigma, 900 + k).astype(wtgen.dtype_for(width))
        print("geometry %d: n=%d sigma=%d width=%d" % (lane_bytes, n, sigma, width), flush=True)
        t = wt.build(wt.to_device(S, torch.device("cuda:0")), sigma)
        ref = oracle.build(S, sigma)
        assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None
        assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None
        t.close()


@pytest.mark.parametrize("lane_bytes", [32, 64, 128])
def test_every_geometry_clustered_large_alphabet(lane_bytes, restore_table):
    # Gaussian clusters over 2^20 symbols: deep levels hold tiles of many
    # small nodes next to a few large ones (the few-node and dense split
    # paths of the staged variant), with a ragged last tile; and the same
    # for bytes (clusters a few symbols wide over 256, and a steep Zipf),
    # where 128 lane bytes is no u8 geometry and the default one runs
    _, wt = _mods()
    import torch
    _force(lane_bytes)
    for k, (n, width) in enumerate([(300_001, 4), (200_003, 2), (400_003, 1), (600_011, 1)]):
        sigma = (1 << 20) if width == 4 else ((1 << 16) if width == 2 else 256)
        if width == 1 and k == 3:
            S = wtgen.zipf(n, sigma, 1.6, 950 + k)
        else:
            S = wtgen.gauss_mix(n, sigma, 950 + k, 16, max(1.0, sigma / 512), width)
        print("geometry %d clustered: n=%d sigma=%d width=%d" % (lane_bytes, n, sigma, width), flush=True)
        t = wt.build(wt.to_device(S, torch.device("cuda:0")), sigma)
        ref = oracle.build(S, sigma)
        assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None
        assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None
        t.close()


@pytest.mark.parametrize("lane_bytes", [1, 2, 32, 128])
def test_every_geometry_batched(lane_bytes, restore_table):
    _, wt = _mods()
    import torch
    _force(lane_bytes)
    Ss, sig = [], []
    for k, (n, sigma, width) in enumerate(CASES):
        Ss.append(wtgen.uniform(n, sigma, 950 + k).astype(wtgen.dtype_for(width)))
        sig.append(sigma)
    print("geometry %d batched: %d sequences" % (lane_bytes, len(Ss)), flush=True)
    dev = torch.device("cuda:0")
    trees = wt.build_batch([wt.to_device(S, dev) for S in Ss], sig)
    for t, S, sigma in zip(trees, Ss, sig):
        ref = oracle.build(S, sigma)
        assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None
        assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None
        t.close()


def test_mixed_geometries_in_one_batch(restore_table):
    """Sequences of one batch may carry different geometries (one class each)."""
    _, wt = _mods()
    import torch
    _force(0)
    # u16 at 12 levels: lane bytes 32 for lg n = 12, 128 for lg n = 13
    assert wt.wt_tune_set(1, 2, 12, 12, 32) == wt.WT_OK
    assert wt.wt_tune_set(1, 2, 12, 13, 128) == wt.WT_OK
    Ss = [wtgen.uniform(n, 1 << 12, 990 + k).astype(np.uint16) for k, n in enumerate([5000, 9000, 4100, 12000])]
    dev = torch.device("cuda:0")
    trees = wt.build_batch([wt.to_device(S, dev) for S in Ss], [1 << 12] * 4)
    for t, S in zip(trees, Ss):
        ref = oracle.build(S, 1 << 12)
        assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None
        assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None
        t.close()
