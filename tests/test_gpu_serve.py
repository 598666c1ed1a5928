"""GPU tests of the serving loop (continuous batching over one arena).

* Every request served in a Poisson mix gets the same tree and the same
  rank/select answers as the same sequence built alone, and both match the
  oracle (bit-exact, integer work).
* Under a tight HBM budget requests queue instead of failing, resident
  trees are evicted, memory never exceeds the budget, and all complete.
* Cancelled requests free their memory; a request larger than the budget is
  rejected while the rest are served.
"""
import numpy as np
import pytest

import oracle
import wtgen

pytestmark = pytest.mark.gpu

SIGMAS = (4, 256, 1 << 16, 1 << 20)
WIDTHS = (1, 1, 2, 4)


def _mods():
    from paper_1610_05994_amd import serve, wtree
    return serve, wtree


def _pool(count, seed, lg_min=10.0, lg_max=17.0):
    import torch
    serve, _ = _mods()
    specs = wtgen.serve_stream(count, 1.0, seed, lg_min=lg_min, lg_max=lg_max, sigmas=SIGMAS, widths=WIDTHS)
    return serve.make_pool(specs, torch.device("cuda:0"))


def _oracle_answers(p, req):
    t = oracle.build(p["host"], p["sigma"], with_ranks=False)
    r = [oracle.rank(t, int(c), int(i)) for c, i in zip(req.rank_c, req.rank_i)]
    s = []
    for c, j in zip(req.sel_c, req.sel_j):
        v = oracle.select(t, int(c), int(j))
        s.append(np.iinfo(np.uint64).max if v is None else v)
    return t, np.array(r, np.uint64), np.array(s, np.uint64)


def test_served_results_equal_alone_and_oracle():
    serve, wt = _mods()
    pool = _pool(12, 2024)
    arrivals = wtgen.pool_stream(len(pool), 48, 20000.0, 77)
    reqs = serve.requests_from(pool, arrivals)
    srv = serve.Server(budget_bytes=1 << 30, streams=3, max_inflight=4)
    print("serve mix: %d requests over %d sequences" % (len(reqs), len(pool)), flush=True)
    srv.run_stream(reqs, timeout=120)
    assert all(r.state == serve.RESIDENT for r in reqs), [r.state for r in reqs]
    assert srv.batches_launched >= 2
    cache = {}
    for r, a in zip(reqs, arrivals):
        p = pool[a["pool"]]
        assert r.status == wt.WT_OK
        if a["pool"] not in cache:
            alone = wt.build(p["S"], p["sigma"])
            cache[a["pool"]] = (alone.bitmaps(), _oracle_answers(p, r)[0], alone)
        alone_bits, otree, alone = cache[a["pool"]]
        got = srv.tree_bitmaps(r.rid)
        assert np.array_equal(got, alone_bits), r.rid
        assert np.array_equal(got, otree.bitmaps), r.rid
        # answers in the mix == answers of the tree built alone == oracle
        _, orank, osel = _oracle_answers(p, r)
        assert np.array_equal(r.rank_out, orank), r.rid
        assert np.array_equal(r.sel_out, osel), r.rid
        if len(r.rank_c):
            assert np.array_equal(alone.rank(r.rank_c, r.rank_i).cpu().numpy().view(np.uint64), orank)
        if len(r.sel_c):
            assert np.array_equal(alone.select(r.sel_c, r.sel_j).cpu().numpy().view(np.uint64), osel)
    srv.arena.check()
    srv.close()
    assert srv.arena.used == 0


def test_tight_budget_queues_and_evicts():
    serve, wt = _mods()
    pool = _pool(8, 31, lg_min=14.0, lg_max=17.0)
    need = max(wt.wt_footprint(p["n"], p["sigma"], p["S"].element_size())[1] +
               wt.wt_batch_footprint([(p["n"], p["sigma"], p["S"].element_size())])[1] for p in pool)
    budget = 3 * need
    arrivals = wtgen.pool_stream(len(pool), 40, 50000.0, 5)
    reqs = serve.requests_from(pool, arrivals)
    srv = serve.Server(budget_bytes=budget, streams=2, max_inflight=4)
    print("serve tight budget: %d bytes" % budget, flush=True)
    srv.run_stream(reqs, timeout=120)
    assert srv.arena.high_water <= srv.arena.size
    done = [r for r in reqs if r.state in (serve.RESIDENT, serve.RELEASED)]
    assert len(done) == len(reqs)
    assert any(r.state == serve.RELEASED for r in reqs)      # evicted to make room
    for r, a in zip(reqs, arrivals):
        _, orank, osel = _oracle_answers(pool[a["pool"]], r)
        assert np.array_equal(r.rank_out, orank) and np.array_equal(r.sel_out, osel)
    srv.arena.check()
    srv.close()


def test_cancel_and_reject():
    serve, wt = _mods()
    import torch
    pool = _pool(4, 9, lg_min=12.0, lg_max=13.0)
    srv = serve.Server(budget_bytes=64 << 20, streams=2, max_inflight=2)
    big = torch.zeros(40 << 20, dtype=torch.uint8, device="cuda:0")   # tree alone is > 64 MB at sigma 256
    reqs = [serve.Request(rid=k, S=pool[k % 4]["S"], sigma=pool[k % 4]["sigma"]) for k in range(6)]
    reqs.append(serve.Request(rid=99, S=big, sigma=256))
    for r in reqs:
        srv.submit(r)
    assert reqs[-1].state == serve.REJECTED
    srv.cancel(3)                          # still queued: never built
    assert reqs[3].state == serve.CANCELLED
    srv.drain()
    assert [r.state for r in reqs[:6]] == [serve.RESIDENT] * 3 + [serve.CANCELLED] + [serve.RESIDENT] * 2
    used = srv.arena.used
    srv.cancel(0)                          # resident: its tree memory is freed
    assert reqs[0].state == serve.CANCELLED and srv.arena.used < used
    srv.release(1)
    assert reqs[1].state == serve.RELEASED
    srv.arena.check()
    srv.close()
    assert srv.arena.used == 0
