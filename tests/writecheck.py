"""One writer per bitmap word, counted (run by tests/test_gpu_writes.py in
its own process with WT_LIBRARY naming the write-counting build).

For every kind of build the library has -- tiled single builds (plain,
staged, folded last level, narrowed orders with anchors), one-workgroup
builds, batched builds, the wavelet matrix, the 4-ary tree, the buffered
build and the Huffman-shaped tree -- the tree memory is counted per 16-bit
granule while the tree is built: every granule of the bitmaps (and digit
levels) must be stored exactly once, padding included, and nothing else in
the tree memory may be stored by a bitmap store.
"""
from __future__ import annotations

import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import wtgen  # noqa: E402


def _say(msg):
    print(msg, flush=True)


class Counter:
    """Counters over one span of device memory."""

    def __init__(self, wt, torch, mem):
        self.wt, self.torch, self.mem = wt, torch, mem
        self.cnt = torch.zeros(mem.numel() // 2, dtype=torch.int32, device=mem.device)
        assert wt.wt_debug_write_counters(self.cnt.data_ptr(), mem.data_ptr(), mem.numel()) == wt.WT_OK

    def finish(self, regions, tag):
        """regions: (byte offset, bytes) of the bitmaps inside the span."""
        self.torch.cuda.synchronize()
        assert self.wt.wt_debug_write_counters(0, 0, 0) == self.wt.WT_OK
        c = self.cnt.cpu().numpy()
        want = np.zeros_like(c)
        for off, nb in regions:
            assert off % 2 == 0 and nb % 2 == 0
            want[off // 2:(off + nb) // 2] += 1
        bad = np.flatnonzero(c != want)
        assert bad.size == 0, "%s: %d granules with a writer count other than expected, first at byte %d: %d " \
                              "stores, %d expected" % (tag, bad.size, 2 * bad[0], c[bad[0]], want[bad[0]])
        _say("write check %s: %d granules, each stored once" % (tag, int(want.sum())))


def level_regions(wt, tree, base):
    rc, info = wt.wt_levels(tree.handle)
    assert rc == wt.WT_OK
    return [(info["bitmaps"] - base, info["levels"] * info["words_per_level"] * 8)] if info["levels"] else []


def single(wt, torch, S, sigma, tag, matrix=False, arity=2, geometry=None):
    dev = torch.device("cuda:0")
    n, width = S.shape[0], S.dtype.itemsize
    levels = (sigma - 1).bit_length()
    if geometry is not None:
        assert wt.wt_tune_set(0, width, levels, max(0, n.bit_length() - 1), geometry) == wt.WT_OK
    fp = wt.wt_multiary_footprint if arity == 4 else wt.wt_footprint
    rc, tb, wb = fp(n, sigma, width)
    assert rc == wt.WT_OK
    tree_mem = torch.empty(tb, dtype=torch.uint8, device=dev)
    cnt = Counter(wt, torch, tree_mem)
    t = wt.build(wt.to_device(S, dev), sigma, tree_mem=tree_mem, matrix=matrix, arity=arity)
    assert t.status() == wt.WT_OK
    base = tree_mem.data_ptr()
    if arity == 4:
        rc, info = wt.wt_multiary_levels(t.handle)
        assert rc == wt.WT_OK
        regions = [(info["digits"] - base, info["levels"] * info["words"] * 8)]
    else:
        regions = level_regions(wt, t, base)
    cnt.finish(regions, tag)
    t.close()
    if geometry is not None:
        assert wt.wt_tune_set(0, width, levels, max(0, n.bit_length() - 1), 0) == wt.WT_OK


def batch(wt, torch, Ss, sigmas, tag):
    dev = torch.device("cuda:0")
    descs = [(S.shape[0], sg, S.dtype.itemsize) for S, sg in zip(Ss, sigmas)]
    offs, total = [], 0
    for d in descs:
        rc, tb, _ = wt.wt_footprint(*d)
        assert rc == wt.WT_OK
        offs.append((total, tb))
        total += (tb + 255) // 256 * 256
    mem = torch.empty(total, dtype=torch.uint8, device=dev)
    rc, wb = wt.wt_batch_footprint(descs)
    assert rc == wt.WT_OK
    work = torch.empty(max(wb, 256), dtype=torch.uint8, device=dev)
    dS = [wt.to_device(S, dev) for S in Ss]
    cnt = Counter(wt, torch, mem)
    base = mem.data_ptr()
    rc, hs = wt.wt_build_batch([x.data_ptr() for x in dS], descs, [base + o for o, _ in offs], [tb for _, tb in offs],
                               work.data_ptr(), work.numel(), int(torch.cuda.current_stream().cuda_stream))
    assert rc == wt.WT_OK
    regions = []
    for h in hs:
        assert wt.wt_tree_status(h) == wt.WT_OK
        rc, info = wt.wt_levels(h)
        if info["levels"]:
            regions.append((info["bitmaps"] - base, info["levels"] * info["words_per_level"] * 8))
    cnt.finish(regions, tag)
    for h in hs:
        wt.wt_free(h)


def buffered(wt, torch, S, sigma, bsyms, tag):
    dev = torch.device("cuda:0")
    n, width = S.shape[0], S.dtype.itemsize
    rc, tb, _ = wt.wt_footprint(n, sigma, width)
    assert rc == wt.WT_OK
    tree_mem = torch.empty(tb, dtype=torch.uint8, device=dev)
    cnt = Counter(wt, torch, tree_mem)
    t = wt.build_buffered(wt.to_device(S, dev), sigma, bsyms, tree_mem=tree_mem)
    assert t.status() == wt.WT_OK
    cnt.finish(level_regions(wt, t, tree_mem.data_ptr()), tag)
    t.close()


def huffman(wt, torch, S, sigma, tag):
    dev = torch.device("cuda:0")
    counts = np.bincount(S.astype(np.int64), minlength=sigma).astype(np.uint64)
    n, width = S.shape[0], S.dtype.itemsize
    rc, tb, wb = wt.wt_huffman_footprint(counts, n, sigma, width)
    assert rc == wt.WT_OK
    tree_mem = torch.empty(tb, dtype=torch.uint8, device=dev)
    work_mem = torch.empty(max(wb, 256), dtype=torch.uint8, device=dev)
    cnt = Counter(wt, torch, tree_mem)
    t = wt.build_huffman(wt.to_device(S, dev), sigma, counts=counts, tree_mem=tree_mem, work_mem=work_mem)
    assert t.status() == wt.WT_OK
    rc, info = wt.wt_huffman_levels(t.handle, sigma)
    assert rc == wt.WT_OK
    regions = [(off, ((size + 63) // 64 + 7) // 8 * 8 * 8) for off, size in zip(info["bits_off"], info["sizes"])]
    cnt.finish(regions, tag)
    t.close()


def main() -> int:
    import torch

    from paper_1610_05994_amd import tune
    from paper_1610_05994_amd import wtree as wt
    assert os.path.basename(wt.LIB_PATH) == "libwtree_check.so", "run with WT_LIBRARY naming the write-counting build"
    S = wtgen.zipf((1 << 21) + 4099, 256, 1.1, 11)
    single(wt, torch, S, 256, "u8 folded last level")
    single(wt, torch, wtgen.uniform(5000, 200, 12), 200, "u8 one workgroup")
    single(wt, torch, wtgen.gauss_mix((1 << 20) + 33, 1 << 20, 13), 1 << 20, "u32 staged deep levels")
    single(wt, torch, wtgen.zipf((1 << 22) + 77, 1 << 16, 1.0, 14, width=2), 1 << 16,
           "u16 narrowed to 1 byte under 256 anchors", geometry=64)
    single(wt, torch, wtgen.gauss_mix((1 << 20) + 5, 1 << 20, 15), 1 << 20, "u32 narrowed to 2 bytes", geometry=128)
    single(wt, torch, wtgen.gauss_mix((1 << 20) + 5, 1 << 20, 16), 1 << 20, "wavelet matrix, narrowed",
           matrix=True, geometry=128)
    single(wt, torch, wtgen.zipf(300_007, 1000, 1.0, 17), 1000, "4-ary tree", arity=4)
    specs = [(3000, 20, 1), (40_000, 1 << 16, 2), (200_003, 256, 1), (120_000, 1 << 20, 4), (1, 4, 1),
             ((1 << 23) + 9, 1 << 20, 4)]  # (the last one long enough to be built alone)
    batch(wt, torch, [wtgen.uniform(n, sg, 18 + n).astype(wtgen.dtype_for(w)) for n, sg, w in specs],
          [sg for _, sg, _ in specs], "batch of 6")
    buffered(wt, torch, wtgen.zipf(1 << 20, 256, 1.1, 19), 256, 1 << 18, "buffered, 4 buffers")
    huffman(wt, torch, wtgen.zipf(500_000, 300, 1.2, 20), 300, "Huffman-shaped")
    tune.load()
    print("write check: ok", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
