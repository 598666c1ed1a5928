"""GPU parity of builds whose symbol orders narrow as the levels go by.

A single build of 2- and 4-byte symbols (n >= 2^18) keeps in T_i only the
low bytes of each symbol that the remaining levels need; the node of a
symbol then takes its high bits from the anchor node holding its position.
The tree must not change: every case is compared with the oracle bit for
bit, for each lane geometry (which decides how far the orders narrow: none,
4 -> 2 bytes, or 4 -> 2 -> 1 and 2 -> 1).  The inputs put anchor
boundaries inside tiles and inside lanes (anchor nodes of a few symbols),
leave anchor nodes empty (sparse alphabets), and narrow at level 0 (small
alphabets in wide storage).
"""
import numpy as np
import pytest

import oracle
import wtgen
from tests import treecheck as tc

pytestmark = pytest.mark.gpu

N0 = (1 << 18) + 4099  # above the narrowing threshold, with a ragged last tile
# long enough for anchor levels of 256 and 512 nodes (at most one tile in 8
# may hold two anchors, or the order does not narrow that far)
N1 = (1 << 23) + 4099


def _mods():
    from paper_1610_05994_amd import tune, wtree
    return tune, wtree


@pytest.fixture
def restore_table():
    yield
    tune, _ = _mods()
    tune.reset()
    tune.load()


def _force(lane_bytes, widths=(2, 4)):
    _, wt = _mods()
    for width in widths:
        lb = lane_bytes if lane_bytes // width <= 64 else 0
        for levels in range(1, min(24, 8 * width) + 1):
            for lg_n in range(0, 41):
                assert wt.wt_tune_set(0, width, levels, lg_n, lb) == wt.WT_OK


def _check(S, sigma, tag):
    import torch
    _, wt = _mods()
    print("narrow %s: n=%d sigma=%d width=%d" % (tag, S.shape[0], sigma, S.dtype.itemsize), flush=True)
    t = wt.build(wt.to_device(S, torch.device("cuda:0")), sigma)
    assert t.status() == wt.WT_OK
    ref = oracle.build(S, sigma)
    msg = tc.compare_levels(t.bitmaps(), ref.bitmaps)
    assert msg is None, "%s: %s" % (tag, msg)
    msg = tc.compare_levels(t.ranks(), ref.ranks, "rank")
    assert msg is None, "%s: %s" % (tag, msg)
    t.close()


def _few_per_anchor(n, sigma, low_bits, seed, width):
    """Most symbols in one anchor node; every other anchor node holds 0 to 3
    symbols, so that anchor boundaries fall inside lanes."""
    rng = np.random.Generator(np.random.PCG64(seed))
    anchors = sigma >> low_bits
    extra = []
    for v in range(anchors):
        extra.extend((v << low_bits) + rng.integers(0, 1 << low_bits, int(rng.integers(0, 4))))
    extra = np.array(extra, dtype=np.int64)
    bulk = (int(rng.integers(0, anchors)) << low_bits) + rng.integers(0, 1 << low_bits, n - extra.shape[0])
    S = np.concatenate([bulk, extra])
    return rng.permutation(S).astype(wtgen.dtype_for(width))


def _sparse(n, sigma, seed, width, step=1021):
    """Symbols from a sparse subset (multiples of a prime): most anchor
    nodes are empty."""
    rng = np.random.Generator(np.random.PCG64(seed))
    vals = np.arange(0, sigma, step)
    return vals[rng.integers(0, vals.shape[0], n)].astype(wtgen.dtype_for(width))


CASES = [  # (tag, n, sigma, width, maker)
    # narrowing at level 0 / 1 with anchors of 2 nodes or none
    ("u32-uniform-300", N0, 300, 4, lambda n: wtgen.uniform(n, 300, 64, width=4)),
    ("u16-uniform-2^9", N0, 1 << 9, 2, lambda n: wtgen.uniform(n, 1 << 9, 68, width=2)),
    ("u16-uniform-4", N0, 4, 2, lambda n: wtgen.uniform(n, 4, 69, width=2)),
    ("u32-zipf-2^17-short", N0, 1 << 17, 4, lambda n: wtgen.zipf(n, 1 << 17, 1.2, 63, width=4)),
    # 1-byte orders under 256 / 512 anchors, 2-byte orders under 256
    ("u32-zipf-2^17", N1, 1 << 17, 4, lambda n: wtgen.zipf(n, 1 << 17, 1.2, 73, width=4)),
    ("u32-few-per-anchor", N1, 1 << 17, 4, lambda n: _few_per_anchor(n, 1 << 17, 8, 65, 4)),
    ("u32-uniform-2^24", N1, 1 << 24, 4, lambda n: wtgen.uniform(n, 1 << 24, 62, width=4)),
    ("u16-zipf-2^16", N1, 1 << 16, 2, lambda n: wtgen.zipf(n, 1 << 16, 1.0, 67, width=2)),
    ("u16-few-per-anchor", N1, 1 << 16, 2, lambda n: _few_per_anchor(n, 1 << 16, 8, 70, 2)),
    ("u16-sparse", N1, 1 << 16, 2, lambda n: _sparse(n, 1 << 16, 71, 2, step=97)),
    ("u32-sparse", N1, 1 << 17, 4, lambda n: _sparse(n, 1 << 17, 66, 4)),
]


@pytest.mark.parametrize("lane_bytes", [32, 64, 128])
def test_narrowed_orders_build_the_oracle_tree(lane_bytes, restore_table):
    _force(lane_bytes)
    for tag, n, sigma, width, make in CASES:
        S = make(n)
        assert S.dtype.itemsize == width
        _check(S, sigma, "%s@%d" % (tag, lane_bytes))


def test_narrowed_sorted_and_constant_inputs():
    # sorted: every tile single-node, anchors change only at tile-internal
    # boundaries; constant: one node per level, no anchor boundary at all
    S = np.sort(wtgen.zipf(N1, 1 << 16, 0.8, 72, width=4))
    _check(S, 1 << 16, "u32-sorted")
    S = np.full(N1, 40_000, dtype=np.uint16)
    _check(S, 1 << 16, "u16-constant")


def test_narrowed_large_clustered(restore_table):
    # 2^20 symbols, 20 levels: 4 -> 2 -> 1 bytes under anchors of 16 and
    # 4096 nodes (E = 32), at the large-alphabet workload's distribution
    _force(128)
    S = wtgen.gauss_mix((1 << 26) + 4099, 1 << 20, 74)
    _check(S, 1 << 20, "u32-gauss-2^26@128")


def test_narrowed_orders_with_doubled_tiles(restore_table):
    # 64 bytes per lane at every width: the narrowing passes that also double
    # the next level's symbols per lane run where most levels of the narrower
    # width keep nodes of many tiles (u32 -> u16 at 16 -> 32 symbols per
    # lane; u16 -> u8 at 32 -> 64 symbols per lane for a long sequence)
    _force(64, widths=(1, 2, 4))
    _check(wtgen.zipf(N1, 1 << 17, 1.2, 79, width=4), 1 << 17, "u32-zipf-2^17-doubled")
    _check(wtgen.zipf((1 << 26) + 4099, 1 << 16, 1.0, 80, width=2), 1 << 16, "u16-zipf-2^16-2^26-doubled")


@pytest.mark.parametrize("lane_bytes", [64, 128])
def test_narrowed_wavelet_matrix(lane_bytes, restore_table):
    # a wavelet matrix has one node per level: its orders narrow with no
    # anchors, at any length above the threshold (and, at 64 bytes per lane,
    # double their symbols per lane where they narrow to 1 byte)
    import torch
    _, wt = _mods()
    _force(lane_bytes, widths=(1, 2, 4))
    for tag, S, sigma in [("u32-gauss-2^20", wtgen.gauss_mix(N0, 1 << 20, 75), 1 << 20),
                          ("u32-uniform-2^24", wtgen.uniform(N0, 1 << 24, 76, width=4), 1 << 24),
                          ("u32-uniform-300", wtgen.uniform(N0, 300, 77, width=4), 300),
                          ("u16-zipf-2^16", wtgen.zipf(N1, 1 << 16, 1.0, 78, width=2), 1 << 16)]:
        print("narrow matrix %s@%d: n=%d" % (tag, lane_bytes, S.shape[0]), flush=True)
        t = wt.build(wt.to_device(S, torch.device("cuda:0")), sigma, matrix=True)
        assert t.status() == wt.WT_OK
        ref = oracle.build_matrix(S, sigma)
        assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None, tag
        assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None, tag
        assert np.array_equal(t.zeros(), ref.zeros), tag
        t.close()
