"""Seeded random cross-checks of every build path against the oracle: lengths
log-uniform over one workgroup's capacity to many tiles, alphabets from 2 to
2^24 (odd and even bit counts, non-powers of two), all widths, uniform /
Zipf / Gaussian-cluster / sorted / sparse inputs.  Each draw builds the
binary tree, the wavelet matrix, the 4-ary tree and a buffered tree (random
buffer size) and compares every word and directory entry bit-exactly; the
draws are also built together in one batch."""
import numpy as np
import pytest

import oracle
import wtgen
from tests import treecheck as tc

pytestmark = pytest.mark.gpu


def _wt():
    from paper_1610_05994_amd import wtree
    return wtree


def _draw(rng, k):
    lg = rng.uniform(4, 19)
    n = int(2 ** lg)
    lg_sigma = int(rng.integers(1, 25))
    sigma = int(rng.integers(2 ** (lg_sigma - 1) + 1, 2 ** lg_sigma + 1)) if lg_sigma > 1 else 2
    width = wtgen.width_for(sigma)
    if rng.random() < 0.25 and width < 4:
        width *= 2                            # wider storage than needed
    kind = int(rng.integers(0, 5))
    seed = 9000 + k
    if kind == 0:
        S = wtgen.uniform(n, sigma, seed, width)
    elif kind == 1:
        S = wtgen.zipf(n, sigma, 1.0 + rng.random(), seed, width)
    elif kind == 2:
        S = wtgen.gauss_mix(n, sigma, seed, 16, max(1.0, sigma / 512), width)
    elif kind == 3:
        S = wtgen.cont(n, sigma, width)
    else:                                     # a few distinct symbols far apart
        S = (wtgen.uniform(n, 7, seed, width).astype(np.uint64) * (sigma // 7)).astype(wtgen.dtype_for(width))
    return S, sigma, kind


def _digits_equal(t, ref):
    d, r = t.digits(), t.digit_dir()
    return all(np.array_equal(d[i], ref.digits[i]) and np.array_equal(r[i], ref.dir[i]) for i in range(ref.levels))


@pytest.mark.parametrize("block", range(4))
def test_random_builds(block):
    import torch
    wt = _wt()
    rng = np.random.default_rng(161 + block)
    draws = [_draw(rng, 100 * block + k) for k in range(25)]
    dev = torch.device("cuda:0")
    for S, sigma, kind in draws:
        tag = (len(S), sigma, S.dtype.itemsize, kind)
        print("random: n=%d sigma=%d width=%d kind=%d" % tag, flush=True)
        dS = wt.to_device(S, dev)
        ref = oracle.build(S, sigma)
        t = wt.build(dS, sigma)
        assert t.status() == wt.WT_OK, tag
        assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None, tag
        assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None, tag
        t.close()
        refm = oracle.build_matrix(S, sigma)
        t = wt.build(dS, sigma, matrix=True)
        assert tc.compare_levels(t.bitmaps(), refm.bitmaps) is None, ("matrix",) + tag
        assert tc.compare_levels(t.ranks(), refm.ranks, "rank") is None, ("matrix",) + tag
        assert np.array_equal(t.zeros(), refm.zeros), ("matrix",) + tag
        t.close()
        t = wt.build(dS, sigma, arity=4)
        assert _digits_equal(t, oracle.build4(S, sigma)), ("4-ary",) + tag
        t.close()
        buf = int(rng.integers(max(1, len(S) // 16), len(S) + 1))  # at most 16 buffers
        t = wt.build_buffered(S, sigma, buf, width=S.dtype.itemsize, device=dev)
        assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None, ("buffered", buf) + tag
        assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None, ("buffered", buf) + tag
        t.close()
    # the same draws in one batch
    trees = wt.build_batch([wt.to_device(S, dev) for S, _, _ in draws], [sg for _, sg, _ in draws],
                           [S.dtype.itemsize for S, _, _ in draws])
    for (S, sigma, kind), t in zip(draws, trees):
        ref = oracle.build(S, sigma)
        assert t.status() == wt.WT_OK
        assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None, ("batch", len(S), sigma, kind)
        assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None, ("batch", len(S), sigma, kind)
