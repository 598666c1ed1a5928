"""CPU checks of the serving arena allocator (offset bookkeeping only):
first fit, alignment, coalescing of freed neighbours, exhaustion, and
invariants under a long random alloc/free sequence; and of admission when a
batch needs more workspace than its members' solo figures add up to."""
import numpy as np

from paper_1610_05994_amd.serve import ALIGN, Arena


def test_first_fit_alignment_and_coalescing():
    a = Arena(10 * ALIGN + 17)
    assert a.size == 10 * ALIGN
    x = a.alloc(1)
    y = a.alloc(ALIGN + 1)
    z = a.alloc(3 * ALIGN)
    assert (x, y, z) == (0, ALIGN, 3 * ALIGN)
    assert a.used == 6 * ALIGN and a.largest_free() == 4 * ALIGN
    assert a.alloc(5 * ALIGN) is None
    a.free(y)
    assert a.alloc(2 * ALIGN) == ALIGN            # the hole is reused first
    a.free(ALIGN)
    a.free(x)
    a.free(z)
    a.check()
    assert a.free_list == [(0, 10 * ALIGN)] and a.used == 0
    assert a.high_water == 6 * ALIGN


def test_random_alloc_free_keeps_invariants():
    rng = np.random.default_rng(3)
    a = Arena(1 << 20)
    live = []
    for step in range(4000):
        if live and (rng.random() < 0.45 or a.largest_free() < 4096):
            off = live.pop(int(rng.integers(0, len(live))))
            a.free(off)
        else:
            n = int(rng.integers(1, 20000))
            off = a.alloc(n)
            if off is not None:
                assert off % ALIGN == 0
                live.append(off)
        if step % 97 == 0:
            a.check()
    for off in live:
        a.free(off)
    a.check()
    assert a.free_list == [(0, 1 << 20)]


def test_admission_gives_back_members_when_the_batch_workspace_is_larger():
    """Two long 4-byte sequences each built alone need less workspace than
    the two batched together: admission, which reserves the sum of the solo
    workspaces, then launches the first alone and puts the second back at the
    head of the queue, with the arena consistent (library footprints only,
    no device)."""
    from paper_1610_05994_amd import serve, tune, wtree as wt
    tune.load()
    d = (1 << 23, 1 << 20, 4)
    rc, tb, _ = wt.wt_footprint(*d)
    assert rc == wt.WT_OK
    rc, solo = wt.wt_batch_footprint([d])
    assert rc == wt.WT_OK
    rc, pair = wt.wt_batch_footprint([d, d])
    assert rc == wt.WT_OK
    assert pair > 2 * solo  # built alone, each takes the single build's workspace
    srv = serve.Server.__new__(serve.Server)
    srv.arena = Arena(2 * Arena._round(tb) + 2 * Arena._round(solo))
    srv.queue, srv.resident, srv.max_batch = [], {}, 512
    reqs = []
    for k in range(2):
        r = serve.Request(rid=k, S=None, sigma=d[1])
        r.n, r.width, r.tree_bytes, r.ws_solo = d[0], d[2], tb, solo
        reqs.append(r)
    srv.queue.extend(reqs)
    picked, descs, tree_offs, work_off = srv._admit()
    assert picked == [reqs[0]] and descs == [d] and len(tree_offs) == 1
    assert srv.queue == [reqs[1]] and reqs[1].state == serve.QUEUED
    srv.arena.check()
    assert srv.arena.used == Arena._round(tb) + Arena._round(solo)
