"""CPU checks of the serving arena allocator (offset bookkeeping only):
first fit, alignment, coalescing of freed neighbours, exhaustion, and
invariants under a long random alloc/free sequence."""
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
