"""wt_build_noalloc (workspace in a fixed device array of the library) against
wt_build (workspace from the caller) through the C ABI.

Integer work: the tree memory of both builds -- status word, every bitmap
word and every rank-directory entry, padding included -- must be equal byte
for byte, on two calls in a row with the second on a smaller input (the
array then still holds the first build's contents), and equal to the CPU
oracle.  Sizes whose workspace exceeds the array are rejected before any
work is enqueued.
"""
import sys

import numpy as np
import pytest

import oracle
import wtgen
from tests import treecheck as tc

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _build_both(S, sigma, stream):
    import torch
    from paper_1610_05994_amd import wtree as wt
    dev = torch.device("cuda:0")
    n, width = S.shape[0], S.dtype.itemsize
    rc, tb, wb = wt.wt_footprint(n, sigma, width)
    assert rc == wt.WT_OK and wb <= wt.WT_NOALLOC_WORK_BYTES
    dS = wt.to_device(S, dev)
    sh = int(stream.cuda_stream)
    ref_tree = torch.full((tb,), 0xA5, dtype=torch.uint8, device=dev)
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    rc, h = wt.wt_build(dS.data_ptr(), n, sigma, width, ref_tree.data_ptr(), tb, work.data_ptr(), wb, sh)
    assert rc == wt.WT_OK
    assert wt.wt_tree_status(h) == wt.WT_OK
    wt.wt_free(h)
    got_tree = torch.full((tb,), 0x5A, dtype=torch.uint8, device=dev)
    rc = wt.wt_build_noalloc(dS.data_ptr(), n, sigma, width, got_tree.data_ptr(), tb, sh)
    assert rc == wt.WT_OK, wt.strerror(rc)
    stream.synchronize()
    ref = ref_tree.cpu().numpy()
    got = got_tree.cpu().numpy()
    return ref, got, tb


def _levels(tree, n, sigma):
    l = max(0, (sigma - 1).bit_length())
    W = ((n + 63) // 64 + 7) // 8 * 8
    K = ((n + 511) // 512 + 1 + 7) // 8 * 8
    bits = tree[256:256 + 8 * l * W].view(np.uint64).reshape(l, W)
    ranks = tree[256 + 8 * l * W:256 + 8 * l * (W + K)].view(np.uint64).reshape(l, K)
    return bits, ranks


@pytest.mark.parametrize("cases", [
    # u8 with the last level folded, then a smaller u8 input
    [((1 << 24) + 1234, 256, 1, "zipf"), (70_001, 256, 1, "zipf")],
    # a large alphabet (u32), then a smaller one of another width
    [((1 << 21) - 5, 1 << 20, 4, "uniform"), ((3 << 16) + 9, 1 << 16, 2, "uniform")],
])
def test_noalloc_matches_wt_build_twice(cases):
    import torch
    stream = torch.cuda.Stream()
    for k, (n, sigma, width, kind) in enumerate(cases):
        _say("case noalloc call %d: n=%d sigma=%d width=%d %s" % (k, n, sigma, width, kind))
        S = (wtgen.zipf(n, sigma, 1.1, 900 + k) if kind == "zipf" else wtgen.uniform(n, sigma, 900 + k))
        S = S.astype(wtgen.dtype_for(width))
        ref, got, tb = _build_both(S, sigma, stream)
        assert np.array_equal(got[:4], ref[:4]), "status word"
        assert np.array_equal(got[256:], ref[256:]), "tree bytes differ from wt_build's (call %d)" % k
        rb, rr = _levels(got, n, sigma)
        o = oracle.build(S, sigma)
        msg = tc.compare_levels(rb, o.bitmaps)
        assert msg is None, msg
        msg = tc.compare_levels(rr, o.ranks, "rank")
        assert msg is None, msg


def test_noalloc_rejects_sizes_beyond_the_array():
    import torch
    from paper_1610_05994_amd import wtree as wt
    dev = torch.device("cuda:0")
    n, sigma = 1 << 25, 256
    rc, tb, wb = wt.wt_footprint(n, sigma, 1)
    assert wb > wt.WT_NOALLOC_WORK_BYTES
    S = torch.zeros(n, dtype=torch.uint8, device=dev)
    tree = torch.zeros(tb, dtype=torch.uint8, device=dev)
    stream = torch.cuda.Stream()
    assert wt.wt_build_noalloc(S.data_ptr(), n, sigma, 1, tree.data_ptr(), tb, int(stream.cuda_stream)) == wt.WT_ENOMEM
    # a tree smaller than the footprint, bad alignment, bad descriptors
    assert wt.wt_build_noalloc(S.data_ptr(), 1000, sigma, 1, tree.data_ptr(), 16, 0) == wt.WT_ENOMEM
    assert wt.wt_build_noalloc(S.data_ptr() + 1, 1000, sigma, 1, tree.data_ptr(), tb, 0) == wt.WT_EINVAL
    assert wt.wt_build_noalloc(S.data_ptr(), 1000, 0, 1, tree.data_ptr(), tb, 0) == wt.WT_EINVAL
    stream.synchronize()
    assert not tree.any().item(), "nothing may be written by a rejected call"
