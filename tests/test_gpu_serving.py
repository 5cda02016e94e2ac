"""Continuous-batching server: results alone equal results in the mix (bitwise, since
every reduction runs in a fixed order), budget admission and eviction."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
serve = pytest.importorskip("paper_2506_04763_amd.serve")


def small_requests():
    reqs = []
    sizes = [17, 33, 17, 65, 33, 17, 33, 65, 17, 33]
    for r, n in enumerate(sizes):
        lv = {17: 3, 33: 4, 65: 5}[n]
        scn = W.cube_3d(n, 0.5 + 0.15 * r, 100 + r, corr_cells=4.0, rate=0.02 + 0.008 * r, levels=lv)
        reqs.append(serve.StageRequest(r, scn, arrival=0.0, rtol=1e-8))
    return reqs


def run(reqs, slots, budget=50e9):
    srv = serve.Server(budget_bytes=budget, slots=slots, precision="mixed")
    futs = [srv.submit(q) for q in reqs]
    res = [f.result(timeout=120) for f in futs]
    stats = dict(peak=srv.peak_used, evictions=srv.evictions)
    srv.shutdown()
    return res, stats


def test_alone_equals_mix():
    reqs = small_requests()
    print("[serving] alone", flush=True)
    alone, _ = run(reqs, slots=1)
    print("[serving] mix", flush=True)
    mix, _ = run(reqs, slots=6)
    for a, m in zip(alone, mix):
        assert a.rid == m.rid
        assert a.stats["status"] == "TPF_OK" and m.stats["status"] == "TPF_OK"
        assert a.stats["iters"] == m.stats["iters"]
        np.testing.assert_array_equal(a.x, m.x)


def test_budget_eviction_and_rejection():
    reqs = small_requests()
    need = max(serve.grid_bytes(q.scenario, precision="mixed") for q in reqs)
    budget = int(need * 1.5)  # at most one or two grids resident at once
    res, st = run(reqs, slots=4, budget=budget)
    assert all(r.stats["status"] == "TPF_OK" for r in res)
    assert st["evictions"] > 0
    assert st["peak"] <= budget
    srv = serve.Server(budget_bytes=1e6, slots=2)
    fut = srv.submit(reqs[0])
    with pytest.raises(MemoryError):
        fut.result(timeout=60)
    srv.shutdown()


def test_slab_extents_reused_give_identical_results():
    """Under a budget for about two grids, arenas are carved again and again from the
    server's slab (evicting idle grids); every result equals the one computed under an
    ample budget, bit for bit."""
    reqs = small_requests()
    need = max(serve.grid_bytes(q.scenario, precision="mixed") for q in reqs)
    tight, st = run(reqs, slots=2, budget=int(need * 2.2))
    ample, st2 = run(reqs, slots=2, budget=50e9)
    assert st["evictions"] > 0 and st2["evictions"] == 0
    assert st["peak"] <= int(need * 2.2)
    for a, b in zip(tight, ample):
        assert a.stats["iters"] == b.stats["iters"]
        np.testing.assert_array_equal(a.x, b.x)


def test_resident_grid_reused():
    reqs = small_requests()[:2]
    srv = serve.Server(budget_bytes=50e9, slots=2)
    r1 = srv.submit(reqs[0]).result(timeout=60)
    again = serve.StageRequest(reqs[0].rid, reqs[0].scenario, arrival=0.0, rtol=1e-8)
    r2 = srv.submit(again).result(timeout=60)
    srv.shutdown()
    assert not r1.cache_hit and r2.cache_hit
    np.testing.assert_array_equal(r1.x, r2.x)
