"""CPU-side checks of the C ABI: the library loads, exports every function
that include/wtree.h declares, and its host-only logic (footprints,
argument validation, status strings) behaves as documented.  No call here
reaches the GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _wt():
    from paper_1610_05994_amd import wtree
    return wtree


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in sorted(os.listdir(inc)):
        if fn.endswith(".h"):
            with open(os.path.join(inc, fn)) as f:
                names |= set(re.findall(r"\b(wt_[a-z_]+)\s*\(", f.read()))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    wt = _wt()
    L = wt.lib()
    names = _declared()
    assert len(names) >= 16
    for name in names:
        assert hasattr(L, name), name
    assert sorted(wt.EXPORTED) == names


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    wt = _wt()
    monkeypatch.setattr(wt, "_lib", None)
    monkeypatch.setattr(wt, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(ImportError):
        wt.lib()


def test_footprint_matches_layout_convention():
    wt = _wt()
    for n, sigma, width in [(0, 1, 1), (1, 2, 1), (1 << 20, 256, 1), (1000, 1 << 20, 4), (4097, 20, 2)]:
        rc, tb, wb = wt.wt_footprint(n, sigma, width)
        assert rc == wt.WT_OK
        l = max(0, (sigma - 1).bit_length())
        W = ((n + 63) // 64 + 7) // 8 * 8
        KS = ((n + 511) // 512 + 1 + 7) // 8 * 8
        assert tb == 256 + 8 * l * (W + KS)
        assert wb >= 256 and wb % 256 == 0


@pytest.mark.parametrize("n,sigma,width", [(10, 0, 1), (10, 257, 1), (10, 70000, 2), (10, 4, 3),
                                           (10, (1 << 24) + 1, 4), (1 << 40, 4, 1)])
def test_footprint_rejects_bad_descriptors(n, sigma, width):
    wt = _wt()
    assert wt.wt_footprint(n, sigma, width)[0] == wt.WT_EINVAL


def test_build_argument_checks_before_any_device_call():
    wt = _wt()
    rc, tb, wb = wt.wt_footprint(1000, 256, 1)
    fake = 1 << 40  # never dereferenced: every case fails validation first
    assert wt.wt_build(fake, 1000, 256, 1, 0, tb, fake, wb, 0)[0] == wt.WT_EINVAL
    assert wt.wt_build(fake + 3, 1000, 256, 1, fake, tb, fake, wb, 0)[0] == wt.WT_EINVAL
    assert wt.wt_build(fake, 1000, 256, 1, fake + 64, tb, fake, wb, 0)[0] == wt.WT_EINVAL
    assert wt.wt_build(fake, 1000, 256, 1, fake, tb - 1, fake, wb, 0)[0] == wt.WT_ENOMEM
    assert wt.wt_build(fake, 1000, 256, 1, fake, tb, fake, wb - 1, 0)[0] == wt.WT_ENOMEM
    assert wt.wt_build(fake, 1000, 0, 1, fake, tb, fake, wb, 0)[0] == wt.WT_EINVAL
    assert wt.wt_build(0, 1000, 256, 1, fake, tb, fake, wb, 0)[0] == wt.WT_EINVAL


def test_batch_footprint_and_checks():
    wt = _wt()
    descs = [(1000, 4, 1), (5000, 1 << 16, 2)]
    rc, wb = wt.wt_batch_footprint(descs)
    assert rc == wt.WT_OK
    singles = sum(wt.wt_footprint(*d)[2] for d in descs)
    assert wb >= singles
    assert wt.wt_batch_footprint([(10, 0, 1)])[0] == wt.WT_EINVAL
    fake = 1 << 40
    tbs = [wt.wt_footprint(*d)[1] for d in descs]
    rc, hs = wt.wt_build_batch([fake, fake], descs, [fake, fake], tbs, fake, wb - 1, 0)
    assert rc == wt.WT_ENOMEM and hs == [None, None]
    rc, hs = wt.wt_build_batch([fake, fake], descs, [fake, fake], [tbs[0], tbs[1] - 8], fake, wb, 0)
    assert rc == wt.WT_ENOMEM


def test_status_strings():
    wt = _wt()
    assert wt.strerror(wt.WT_OK) == "success"
    assert "sigma" in wt.strerror(wt.WT_ERANGE)
    assert wt.strerror(99) == "unknown status"
    assert wt.lib().wt_tree_status(None) == wt.WT_EINVAL
    wt.lib().wt_free(None)


def test_tune_table_set_get_and_validation():
    wt = _wt()
    # u16, sigma = 2^16 (16 levels, no folded last level, whose record area
    # grows with the tile): the workspace follows the per-tile counters
    rc, before = wt.wt_tune_get(0, 2, 16, 20)
    assert rc == wt.WT_OK and before in (32, 64, 128)
    try:
        assert wt.wt_tune_set(0, 2, 16, 20, 64) == wt.WT_OK
        _, _, wb64 = wt.wt_footprint(1 << 20, 1 << 16, 2)
        assert wt.wt_tune_set(0, 2, 16, 20, 32) == wt.WT_OK
        assert wt.wt_tune_get(0, 2, 16, 20) == (wt.WT_OK, 32)
        rc, tb32, wb32 = wt.wt_footprint(1 << 20, 1 << 16, 2)
        assert rc == wt.WT_OK
        # half the tile -> twice the per-tile counters; the tree is unchanged
        assert wb32 > wb64
        assert tb32 == wt.wt_footprint(1 << 20, 1 << 16, 2)[1]
        # the batched mode keeps its own entry
        assert wt.wt_tune_get(1, 2, 16, 20)[0] == wt.WT_OK
        assert wt.wt_tune_set(0, 2, 16, 20, 0) == wt.WT_OK
        assert wt.wt_tune_get(0, 2, 16, 20) == (wt.WT_OK, 64)
    finally:
        wt.wt_tune_set(0, 2, 16, 20, before)
    for bad in [(2, 1, 8, 20, 64), (0, 3, 8, 20, 64), (0, 1, 0, 20, 64), (0, 1, 9, 20, 64),
                (0, 4, 25, 20, 64), (0, 1, 8, 41, 64), (0, 1, 8, 20, 128), (0, 2, 8, 20, 48),
                (0, 2, 8, 20, 3)]:
        assert wt.wt_tune_set(*bad) == wt.WT_EINVAL, bad
    assert wt.wt_tune_get(0, 1, 8, 41)[0] == wt.WT_EINVAL


def test_tune_table_expansion_takes_nearest_point():
    from paper_1610_05994_amd import tune
    pts = [dict(mode=0, width=2, levels=6, lg_n=10, lane_bytes=32),
           dict(mode=0, width=2, levels=16, lg_n=26, lane_bytes=128),
           dict(mode=1, width=2, levels=6, lg_n=12, lane_bytes=64)]
    d = tune.expand(pts)
    assert d[(0, 2, 5, 0)] == 32 and d[(0, 2, 16, 40)] == 128 and d[(0, 2, 15, 12)] == 128
    assert d[(1, 2, 6, 12)] == 64 and d[(1, 2, 6, 13)] == 64
    assert d[(1, 2, 16, 30)] == 128          # past the batched grid: mode 0's point
    assert (0, 1, 8, 20) not in d            # no point for width 1: default kept
    assert all(lb in tune.candidates(w, 1) for (_, w, _, _), lb in d.items())
    assert tune.candidates(1, 15360)[:2] == [tune.GEOM_SMALL, tune.GEOM_MID]
    assert tune.candidates(1, 15361)[0] == tune.GEOM_MID and tune.GEOM_MID not in tune.candidates(1, 32769)


def test_short_sequences_need_no_workspace():
    wt = _wt()
    for width, cap, cap2 in [(1, 15360, 32768), (2, 10240, 26624), (4, 6144, 15360)]:
        assert wt.wt_footprint(cap, 200, width)[2] == 256
        assert wt.wt_footprint(cap + 1, 200, width)[2] == 256
        assert wt.wt_footprint(cap2, 200, width)[2] == 256
        assert wt.wt_footprint(cap2 + 1, 200, width)[2] > 256
        # forcing tiles on a short sequence brings the workspace back
        levels = 8
        lg = cap.bit_length() - 1
        rc, before = wt.wt_tune_get(0, width, levels, lg)
        try:
            assert wt.wt_tune_set(0, width, levels, lg, 64) == wt.WT_OK
            assert wt.wt_footprint(cap, 200, width)[2] > 256
            assert wt.wt_tune_set(0, width, levels, lg, 1) == wt.WT_OK
            assert wt.wt_footprint(cap, 200, width)[2] == 256
            assert wt.wt_tune_set(0, width, levels, lg, 2) == wt.WT_OK
            assert wt.wt_footprint(cap, 200, width)[2] == 256
            assert wt.wt_tune_get(0, width, levels, lg)[1] == 2
        finally:
            wt.wt_tune_set(0, width, levels, lg, 0)


def test_query_multi_argument_checks():
    wt = _wt()
    rc, wb = wt.wt_query_multi_footprint(10)
    assert rc == wt.WT_OK and wb >= 10 * 48 and wb % 256 == 0
    assert wt.wt_query_multi([], 0, 0, 0, 0, 0, 0, 0, 0, 0) == wt.WT_OK          # m = 0: nothing to do
    assert wt.wt_query_multi([], 1, 1, 1, 1, 1, 5, 256, 256, 0) == wt.WT_EINVAL  # no trees
    assert wt.lib().wt_query_multi_footprint(3, None) == wt.WT_EINVAL


def test_matrix_entry_points_argument_checks():
    wt = _wt()
    d = wt.wt_desc(10, 0, 1)
    h = ctypes.c_void_p()
    assert wt.lib().wt_build_matrix(None, ctypes.byref(d), None, 0, None, 0, None, ctypes.byref(h)) == wt.WT_EINVAL
    z = (ctypes.c_uint64 * 4)()
    assert wt.lib().wt_matrix_zeros(None, z) == wt.WT_EINVAL


def test_buffered_footprint_and_argument_checks():
    wt = _wt()
    # one buffer: the ordinary build of a staged copy
    rc, tb, wb = wt.wt_buffered_footprint(1000, 256, 1, 1 << 20)
    rc2, tb2, wb2 = wt.wt_footprint(1000, 256, 1)
    assert rc == rc2 == wt.WT_OK and tb == tb2 and wb >= wb2 + 1000
    # several buffers: the tree is the plain one; the workspace holds the
    # partial trees (at least the final bitmaps) and the (nbuf + 1) x (2^l + 1)
    # offset table, and shrinks with the buffer as long as 2^l is small
    n, sigma = 1 << 24, 256
    rc, tb, wb_small = wt.wt_buffered_footprint(n, sigma, 1, 1 << 20)
    _, tb2, wb_plain = wt.wt_footprint(n, sigma, 1)
    assert rc == wt.WT_OK and tb == tb2
    assert wb_small >= 16 * 257 * 8 + 8 * (n // 8) and wb_small < wb_plain + tb
    _, _, wb_big = wt.wt_buffered_footprint(n, sigma, 1, 1 << 22)
    assert wb_big > wb_small - 2 * (1 << 20)
    d = wt.wt_desc(n, sigma, 1)
    h = ctypes.c_void_p()
    tbv, wbv = ctypes.c_uint64(), ctypes.c_uint64()
    assert wt.lib().wt_buffered_footprint(ctypes.byref(d), 0, ctypes.byref(tbv), ctypes.byref(wbv)) == wt.WT_EINVAL
    assert wt.lib().wt_buffered_footprint(ctypes.byref(d), 8, ctypes.byref(tbv), ctypes.byref(wbv)) == wt.WT_EINVAL
    bad = wt.wt_desc(10, 0, 1)
    assert wt.lib().wt_build_buffered(None, ctypes.byref(bad), 4, None, 0, None, 0, None, ctypes.byref(h)) == wt.WT_EINVAL
    assert wt.lib().wt_build_buffered(None, ctypes.byref(d), 1 << 20, None, 0, None, 0, None, ctypes.byref(h)) == wt.WT_EINVAL


def test_multiary_footprint_and_argument_checks():
    wt = _wt()
    for n, sigma, width in [(0, 1, 1), (1, 2, 1), (1000, 256, 1), (5000, 1 << 20, 4), (777, 20, 2)]:
        rc, tb, wb = wt.wt_multiary_footprint(n, sigma, width)
        assert rc == wt.WT_OK
        l4 = (max(0, (sigma - 1).bit_length()) + 1) // 2
        Wd = ((n + 31) // 32 + 7) // 8 * 8
        KS = ((n + 511) // 512 + 1 + 7) // 8 * 8
        assert tb == 256 + l4 * (8 * Wd + 32 * KS)
        assert wb >= 256 and wb % 256 == 0
    d = wt.wt_desc(10, 0, 1)
    h = ctypes.c_void_p()
    assert wt.lib().wt_build_multiary(None, ctypes.byref(d), None, 0, None, 0, None, ctypes.byref(h)) == wt.WT_EINVAL
    lv = ctypes.c_uint32()
    assert wt.lib().wt_multiary_levels(None, ctypes.byref(lv), None, None, None, None) == wt.WT_EINVAL
