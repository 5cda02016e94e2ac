"""The serving slab's extent allocator (host logic, no GPU): first fit, exact reuse,
and merging of neighbouring free extents."""
import random

import pytest

serve = pytest.importorskip("paper_2506_04763_amd.serve")


def test_first_fit_and_merging():
    e = serve._Extents(100)
    a, b, c = e.take(30), e.take(30), e.take(30)
    assert (a, b, c) == (0, 30, 60) and e.take(20) is None and e.take(10) == 90
    e.give(b, 30)
    assert e.take(31) is None and e.take(30) == 30   # the hole is reused exactly
    e.give(a, 30)
    e.give(30, 30)                                   # merges with the hole before it
    assert e.free == [(0, 60)]
    e.give(c, 30)
    e.give(90, 10)
    assert e.free == [(0, 100)]


def test_random_take_give_never_overlaps():
    rng = random.Random(3)
    size = 1 << 20
    e = serve._Extents(size)
    live = {}
    for _ in range(5000):
        if live and rng.random() < 0.45:
            off = rng.choice(list(live))
            e.give(off, live.pop(off))
        else:
            n = rng.choice((1, 7, 64, 4096, 30000))
            off = e.take(n)
            if off is not None:
                live[off] = n
        spans = sorted(list(live.items()) + e.free)
        pos = 0
        for off, n in spans:      # live and free extents tile [0, size) exactly
            assert off == pos
            pos += n
        assert pos == size
        assert all(e.free[i][0] + e.free[i][1] < e.free[i + 1][0] for i in range(len(e.free) - 1))
