"""GPU parity: the HIP build (through the C ABI) against the CPU oracle.

Integer work, so the bar is bit-exact equality of every bitmap word
(padding included) and every rank-directory entry, on the same seeded
inputs.  Sizes span several 4096-symbol tiles with ragged tails; the edge
cases cover empty input, sigma = 1 and 2, non-power-of-two alphabets,
sorted and constant input, sparse alphabets (tiles spanning many empty
nodes), and symbols out of range.
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


def build_and_compare(S, sigma, width=None, tag=""):
    wt = _wt()
    if width is not None and width != S.dtype.itemsize:
        S = S.astype(wtgen.dtype_for(width))
    _say("case %s: n=%d sigma=%d width=%d" % (tag, S.shape[0], sigma, S.dtype.itemsize))
    t = wt.build(wt.to_device(S, _dev()), sigma)
    got_b, got_r = t.bitmaps(), t.ranks()
    ref = oracle.build(S, sigma)
    msg = tc.compare_levels(got_b, ref.bitmaps)
    assert msg is None, "%s: %s" % (tag, msg)
    msg = tc.compare_levels(got_r, ref.ranks, "rank")
    assert msg is None, "%s: %s" % (tag, msg)
    return t, ref


SIGMAS = [1, 2, 3, 4, 5, 16, 20, 27, 230, 256, 1 << 10, 1 << 12, 1 << 16, 1 << 20]
NS = [1, 2, 63, 64, 65, 511, 512, 513, 4095, 4096, 4097, 8192 + 17, 100_000]


@pytest.mark.parametrize("sigma", SIGMAS)
def test_parity_grid(sigma):
    for k, n in enumerate(NS):
        S = wtgen.uniform(n, sigma, 500 + 31 * k + sigma)
        t, _ = build_and_compare(S, sigma, tag="grid")
        t.close()


@pytest.mark.parametrize("sigma,width", [(4, 2), (256, 4), (1000, 4), (1 << 16, 4)])
def test_parity_wide_storage(sigma, width):
    S = wtgen.uniform(50_000, sigma, 77)
    t, _ = build_and_compare(S, sigma, width=width, tag="wide")
    t.close()


def test_parity_empty():
    wt = _wt()
    import torch
    for sigma in [1, 2, 256, 1 << 20]:
        S = torch.zeros(0, dtype=torch.uint8 if sigma <= 256 else torch.int32, device=_dev())
        t = wt.build(S, sigma)
        assert t.status() == wt.WT_OK
        l = oracle.levels(sigma)
        assert t.bitmaps().shape == (l, 0)
        assert t.ranks().shape == (l, 8) and not t.ranks().any()
        t.close()


def test_parity_c1():
    S, sigma = wtgen.workload("c1")
    t, _ = build_and_compare(S, sigma, tag="c1")
    t.close()


@pytest.mark.parametrize("sigma,lg", [(256, 22), (27, 21), (1 << 16, 21), (1 << 12, 20)])
def test_parity_zipf(sigma, lg):
    S = wtgen.zipf(1 << lg, sigma, 1.1, 11 + sigma)
    t, _ = build_and_compare(S, sigma, tag="zipf")
    t.close()


@pytest.mark.parametrize("sigma,lg", [(4, 15), (4, 17), (5, 16), (16, 17), (128, 20), (256, 21)])
def test_parity_last_level_from_previous_pass(sigma, lg):
    # u8 lengths around the point where the pass of level l-2 also writes the
    # last level's bitmap (its directory then comes from that bitmap); skewed
    # input puts node boundaries inside tiles
    for k, n in enumerate([(1 << lg) + 12345, (1 << lg) - 77]):
        S = wtgen.zipf(n, sigma, 1.2, 600 + 7 * k + sigma)
        t, _ = build_and_compare(S, sigma, tag="fold")
        t.close()


@pytest.mark.parametrize("n", [(1 << 21) + 4099, (1 << 22) - 13])
def test_parity_folded_level_tiles_over_many_nodes(n):
    # u8, sigma = 256: nine symbols in ten are 0, the rest spread over the
    # alphabet, so the level-6 nodes other than node 0 are small and some
    # tiles of the pass that also writes the last level span dozens of them
    # (its direct path then leaves many shared 16-position granules)
    rng = np.random.Generator(np.random.PCG64(n))
    S = np.where(rng.random(n) < 0.9, 0, rng.integers(0, 256, n)).astype(np.uint8)
    t, _ = build_and_compare(S, 256, tag="fold-many-nodes")
    t.close()
    # the same after a sort of the tail: runs of every symbol, nodes in order
    S[n // 2:] = np.sort(S[n // 2:])
    t, _ = build_and_compare(S, 256, tag="fold-sorted-tail")
    t.close()


def test_parity_gauss_mix_large_alphabet():
    S, sigma = wtgen.workload("c3@lg22")
    t, _ = build_and_compare(S, sigma, tag="c3@lg22")
    t.close()


@pytest.mark.parametrize("sigma,n", [(16, 100_000), (1 << 12, 1 << 18), (1 << 20, 1 << 18), (1 << 20, 3 << 20)])
def test_parity_sorted(sigma, n):
    S = wtgen.cont(n, sigma)
    t, _ = build_and_compare(S, sigma, tag="sorted")
    t.close()


def test_parity_constant_and_sparse_alphabet():
    S = np.full(70_000, 200, dtype=np.uint8)
    t, _ = build_and_compare(S, 256, tag="constant")
    t.close()
    # ten distinct symbols spread over a 2^24 alphabet: deep-level tiles
    # cover millions of empty nodes
    rng = np.random.Generator(np.random.PCG64(5))
    vals = rng.integers(0, 1 << 24, 10, dtype=np.uint32)
    S = vals[rng.integers(0, 10, 300_000)].astype(np.uint32)
    t, _ = build_and_compare(S, 1 << 24, tag="sparse")
    t.close()


def test_queries_against_brute_force():
    import torch
    S = wtgen.zipf(200_000, 1000, 1.0, 3)
    sigma = 1000
    t, ref = build_and_compare(S, sigma, tag="queries")
    n = S.shape[0]
    acc = t.access(torch.arange(n, device=_dev())).cpu().numpy().astype(np.int64)
    assert np.array_equal(acc, S.astype(np.int64))
    rng = np.random.Generator(np.random.PCG64(9))
    cs = rng.integers(0, sigma, 3000)
    cs[:20] = np.unique(S)[:20]
    iv = rng.integers(0, n + 1, 3000)
    iv[:5] = [0, n, n, 1, n - 1]
    got = t.rank(torch.from_numpy(cs), torch.from_numpy(iv)).cpu().numpy()
    pos_of = {int(c): np.flatnonzero(S == c) for c in np.unique(cs)}
    want = np.array([np.searchsorted(pos_of[int(c)], i) for c, i in zip(cs, iv)])
    assert np.array_equal(got, want)
    js = np.array([rng.integers(0, pos_of[int(c)].size + 2) for c in cs])
    got = t.select(torch.from_numpy(cs), torch.from_numpy(js)).cpu().numpy().view(np.uint64)
    want = np.array([pos_of[int(c)][j - 1] if 1 <= j <= pos_of[int(c)].size else 2**64 - 1
                     for c, j in zip(cs, js)], dtype=np.uint64)
    assert np.array_equal(got, want)
    # single-query C entry points agree with the oracle's walks
    wt = _wt()
    for i in [0, 17, n - 1]:
        assert wt.wt_access(t.handle, i) == (wt.WT_OK, int(S[i]))
    for c in [int(S[0]), 999]:
        assert wt.wt_rank(t.handle, c, n // 2) == (wt.WT_OK, oracle.rank(ref, c, n // 2))
        sel = oracle.select(ref, c, 1)
        assert wt.wt_select(t.handle, c, 1) == ((wt.WT_OK, sel) if sel is not None else (wt.WT_ENOTFOUND, 0))
    assert wt.wt_access(t.handle, n)[0] == wt.WT_EINVAL
    assert wt.wt_rank(t.handle, sigma, 0)[0] == wt.WT_EINVAL
    t.close()


def test_queries_small_alphabets():
    import torch
    for sigma in [1, 2, 3]:
        S = wtgen.uniform(9000, sigma, sigma)
        t, _ = build_and_compare(S, sigma, tag="qsmall")
        n = S.shape[0]
        acc = t.access(torch.arange(n, device=_dev())).cpu().numpy().astype(np.int64)
        assert np.array_equal(acc, S.astype(np.int64))
        for c in range(sigma):
            occ = np.flatnonzero(S == c)
            iv = np.array([0, 1, n // 3, n])
            got = t.rank(torch.full((4,), c), torch.from_numpy(iv)).cpu().numpy()
            assert np.array_equal(got, [np.searchsorted(occ, i) for i in iv])
            js = np.array([1, occ.size, occ.size + 1])
            got = t.select(torch.full((3,), c), torch.from_numpy(js)).cpu().numpy().view(np.uint64)
            assert got[0] == occ[0] and got[1] == occ[-1] and got[2] == 2**64 - 1
        t.close()


def test_out_of_range_symbol_is_reported():
    wt = _wt()
    S = wtgen.uniform(10_000, 20, 1)
    S[4321] = 20
    t = wt.build(wt.to_device(S, _dev()), 20)
    assert t.status() == wt.WT_ERANGE
    t.close()
    S[4321] = 19
    t = wt.build(wt.to_device(S, _dev()), 20)
    assert t.status() == wt.WT_OK
    t.close()


def test_workspace_reuse_and_side_stream():
    import torch
    wt = _wt()
    S1 = wtgen.zipf(300_000, 1 << 12, 1.1, 1)
    S2 = wtgen.uniform(123_457, 1 << 12, 2)
    rc, tb, wb = wt.wt_footprint(300_000, 1 << 12, 2)
    work = torch.empty(wb, dtype=torch.uint8, device=_dev())
    s = torch.cuda.Stream()
    for S in (S1, S2, S1):
        d = wt.to_device(S, _dev())
        torch.cuda.synchronize()
        t = wt.build(d, 1 << 12, stream=s, work_mem=work)
        ref = oracle.build(S, 1 << 12)
        assert np.array_equal(t.bitmaps(), ref.bitmaps)
        assert np.array_equal(t.ranks(), ref.ranks)
        t.close()


def test_batch_matches_oracle():
    specs = wtgen.batch_specs(24, 42, lg_min=6, lg_max=17)
    Ss = wtgen.batch_inputs(specs)
    wt = _wt()
    _say("case batch: %d sequences" % len(Ss))
    trees = wt.build_batch([wt.to_device(S, _dev()) for S in Ss], [d["sigma"] for d in specs],
                           [d["width"] for d in specs])
    for S, d, t in zip(Ss, specs, trees):
        ref = oracle.build(S, d["sigma"])
        assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None, d
        assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None, d
        t.close()


def test_batch_mixed_widths_and_edge_sequences():
    """Batched build of sequences that mix widths, empty and tiny inputs,
    sigma = 1, and alphabets whose deep levels exceed one node chunk; every
    tree equals the oracle and the single-sequence build."""
    import torch
    wt = _wt()
    rng = np.random.Generator(np.random.PCG64(77))
    cases = [(0, 4, 1), (1, 2, 1), (3000, 1, 1), (4095, 20, 1), (70_001, 256, 1), (5000, 1 << 16, 2),
             (40_000, 1 << 15, 2), (9, 3, 2), (70_000, 1 << 20, 4), (2049, 1000, 4), (0, 1 << 20, 4),
             (123_457, 27, 1), (64, 1 << 13, 2)]
    Ss = [wtgen.zipf(n, sg, 1.0, 1000 + k, w) if n else np.zeros(0, wtgen.dtype_for(w))
          for k, (n, sg, w) in enumerate(cases)]
    _say("case batch-mixed: %d sequences" % len(Ss))
    dev = [wt.to_device(S, _dev()) for S in Ss]
    trees = wt.build_batch(dev, [c[1] for c in cases], [c[2] for c in cases])
    for (n, sg, w), S, d, t in zip(cases, Ss, dev, trees):
        assert t.status() == wt.WT_OK, (n, sg, w)
        ref = oracle.build(S, sg)
        assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None, (n, sg, w)
        assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None, (n, sg, w)
        single = wt.build(d, sg, width=w)
        assert np.array_equal(single.bitmaps(), t.bitmaps()) and np.array_equal(single.ranks(), t.ranks())
        single.close()
        if n:
            pos = torch.from_numpy(rng.integers(0, n, 256)).to(_dev())
            acc = t.access(pos).cpu().numpy().astype(np.int64) & 0xFFFFFFFF
            assert np.array_equal(acc, S[pos.cpu().numpy()].astype(np.int64))
        t.close()


def _batch_alone_check(cases, tag):
    """Builds the cases as one batch; every tree must equal the oracle's and
    the single build's.  Returns the lengths of the sequences that were
    built alone (single-build launches in the library's launch records)."""
    wt = _wt()
    Ss = []
    for k, (n, sg, w, kind) in enumerate(cases):
        if kind == "gauss":
            Ss.append(wtgen.gauss_mix(n, sg, 2000 + k))
        else:
            Ss.append(wtgen.zipf(n, sg, 1.0, 2000 + k, w) if n else np.zeros(0, wtgen.dtype_for(w)))
    _say("case %s: %d sequences, largest n=%d" % (tag, len(Ss), max(c[0] for c in cases)))
    dev = [wt.to_device(S, _dev()) for S in Ss]
    assert wt.wt_prof_enable(True) == wt.WT_OK
    try:
        trees = wt.build_batch(dev, [c[1] for c in cases], [c[2] for c in cases])
        recs = wt.wt_prof_read()
    finally:
        wt.wt_prof_enable(False)
    alone = sorted(r["n"] for r in recs if r["kernel"] == "ingest")
    for (n, sg, w, _), S, d, t in zip(cases, Ss, dev, trees):
        _say("case %s: n=%d sigma=%d width=%d" % (tag, n, sg, w))
        assert t.status() == wt.WT_OK, (n, sg, w)
        ref = oracle.build(S, sg)
        assert tc.compare_levels(t.bitmaps(), ref.bitmaps) is None, (n, sg, w)
        assert tc.compare_levels(t.ranks(), ref.ranks, "rank") is None, (n, sg, w)
        single = wt.build(d, sg, width=w)
        assert np.array_equal(single.bitmaps(), t.bitmaps()) and np.array_equal(single.ranks(), t.ranks())
        single.close()
        t.close()
    return alone


def test_batch_long_sequences_built_alone():
    """Long sequences of a batch are built as single builds inside the
    batched call (narrowed orders, folded last level) when that is faster:
    4-byte symbols from 2^25 on, and 1-byte from 2^25 or 2- and 4-byte from
    2^23 when no other sequence of the batch shares their batched launches.
    Every tree equals the oracle's and the single build's, whichever way it
    was built, and the short sequences around them are unaffected."""
    # each long sequence alone in its width: all three built alone
    alone = _batch_alone_check([((1 << 25) + 3, 4, 1, "zipf"), ((1 << 23) + 4099, 1 << 16, 2, "zipf"),
                                ((1 << 23) + 4099, 1 << 20, 4, "gauss"), (5000, 256, 1, "zipf"),
                                (0, 1 << 16, 2, "zipf")], "batch-long-1")
    assert alone == sorted([(1 << 25) + 3, (1 << 23) + 4099, (1 << 23) + 4099]), alone
    # two equal u16 sequences share their launches (batched); the u32 one of
    # 2^25 symbols goes alone in any case, which leaves the 2^23 u32 one alone
    # in its launches; below 2^23 symbols nothing goes alone
    alone = _batch_alone_check([((1 << 25) + 5, 1 << 20, 4, "gauss"), ((1 << 23) + 4099, 1 << 16, 2, "zipf"),
                                ((1 << 23) + 4099, 1 << 16, 2, "zipf"), ((1 << 23) + 7, 1 << 20, 4, "gauss"),
                                ((1 << 23) - 1, 1 << 16, 2, "zipf"), (70_001, 300, 2, "zipf")], "batch-long-2")
    assert alone == sorted([(1 << 25) + 5, (1 << 23) + 7]), alone


def test_batch_reports_out_of_range_per_sequence():
    wt = _wt()
    A = wtgen.uniform(5000, 16, 1)
    B = wtgen.uniform(7000, 16, 2)
    B[6999] = 16
    C = wtgen.uniform((1 << 23) + 1, 300, 3, width=2)  # long: built alone inside the batch
    C[1 << 22] = 300
    trees = wt.build_batch([wt.to_device(A, _dev()), wt.to_device(B, _dev()), wt.to_device(C, _dev())],
                           [16, 16, 300], [1, 1, 2])
    assert trees[0].status() == wt.WT_OK
    assert trees[1].status() == wt.WT_ERANGE
    assert trees[2].status() == wt.WT_ERANGE
    for t in trees:
        t.close()


@pytest.mark.slow
def test_full_size_c2_against_oracle():
    S, sigma = wtgen.workload("c2")
    t, _ = build_and_compare(S, sigma, tag="c2 full")
    t.close()


def test_query_multi_matches_per_tree_queries():
    """Mixed access/rank/select over several trees in one launch equals the
    per-tree calls (and the oracle), including out-of-range arguments."""
    wt = _wt()
    import torch
    dev = _dev()
    specs = [(5000, 20, 1), (70_000, 1 << 16, 2), (30_000, 1 << 20, 4), (1, 3, 1)]
    Ss = [wtgen.uniform(n, sg, 2100 + k).astype(wtgen.dtype_for(w)) for k, (n, sg, w) in enumerate(specs)]
    trees = [wt.build(wt.to_device(S, dev), sg) for S, (_, sg, _) in zip(Ss, specs)]
    rng = np.random.default_rng(8)
    m = 3000
    ti = rng.integers(0, len(trees) + 1, m).astype(np.uint32)            # index len(trees) is invalid
    kind = rng.integers(0, 4, m).astype(np.uint8)                         # kind 3 is invalid
    c = np.zeros(m, np.int32)
    x = np.zeros(m, np.int64)
    for q in range(m):
        if ti[q] < len(trees):
            n, sg, _ = specs[ti[q]]
            c[q] = rng.integers(0, sg + 2)
            x[q] = rng.integers(0, n + 3)
    blob = [torch.from_numpy(a).to(dev) for a in (ti, kind, c, x)]
    out = torch.empty(m, dtype=torch.int64, device=dev)
    rc, wb = wt.wt_query_multi_footprint(len(trees))
    work = torch.empty(wb, dtype=torch.uint8, device=dev)
    st = torch.cuda.current_stream()
    rc = wt.wt_query_multi([t.handle for t in trees], blob[0].data_ptr(), blob[1].data_ptr(), blob[2].data_ptr(),
                           blob[3].data_ptr(), out.data_ptr(), m, work.data_ptr(), wb, int(st.cuda_stream))
    assert rc == wt.WT_OK
    got = out.cpu().numpy().view(np.uint64)
    refs = [oracle.build(S, sg, with_ranks=False) for S, (_, sg, _) in zip(Ss, specs)]
    umax = np.iinfo(np.uint64).max
    for q in range(m):
        if ti[q] >= len(trees) or kind[q] > 2:
            assert got[q] == umax, q
            continue
        t, ref, (n, sg, _) = trees[ti[q]], refs[ti[q]], specs[ti[q]]
        if kind[q] == 0:
            want = Ss[ti[q]][x[q]] if x[q] < n else umax
        elif kind[q] == 1:
            want = oracle.rank(ref, int(c[q]), int(x[q])) if (c[q] < sg and x[q] <= n) else umax
        else:
            v = oracle.select(ref, int(c[q]), int(x[q])) if c[q] < sg else None
            want = umax if v is None else v
        assert int(got[q]) == int(want), (q, ti[q], kind[q], c[q], x[q], got[q], want)
    for t in trees:
        t.close()
