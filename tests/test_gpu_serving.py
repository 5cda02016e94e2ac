"""Continuous-batching server: results alone equal results in the mix (bitwise, since
every reduction runs in a fixed order), budget admission and eviction."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
serve = pytest.importorskip("paper_2506_04763_amd.serve")


SIZES = [17, 33, 17, 65, 33, 17, 33, 65, 17, 33]


def request_spec(r, n):
    """(n, sigma, seed, correlation, rate, levels) of request r."""
    return (n, 0.5 + 0.15 * r, 100 + r, 4.0, 0.02 + 0.008 * r, {17: 3, 33: 4, 65: 5}[n])


def small_requests():
    reqs = []
    for r, n in enumerate(SIZES):
        n, sigma, seed, corr, rate, lv = request_spec(r, n)
        scn = W.cube_3d(n, sigma, seed, corr_cells=corr, rate=rate, levels=lv)
        reqs.append(serve.StageRequest(r, scn, arrival=0.0, rtol=1e-8))
    return reqs


def run(reqs, slots, budget=50e9, solver=None):
    srv = serve.Server(budget_bytes=budget, slots=slots, precision="mixed", solver=solver)
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


def test_served_results_match_the_oracle_under_eviction():
    """Six slots under a budget for about two grids, so arenas are carved from the
    slab again and again and idle grids are evicted: every served 17^3 and 33^3 result
    and one 65^3 result against the oracle's FP64 solve of the same request (assembled
    at the request's initial state, solved to 1e-12), per field, at the mixed-precision
    bound of the parity suite (1e-5), once with point and once with line smoothing.
    The oracle solves run in worker processes while the GPU serves."""
    import concurrent.futures as cf
    import multiprocessing as mp

    from tests import _serving_oracle as SO
    check = [r for r, n in enumerate(SIZES) if n in (17, 33)] + [SIZES.index(65)]
    specs = [request_spec(r, SIZES[r]) for r in check]
    ex = cf.ProcessPoolExecutor(max_workers=min(8, len(specs)), mp_context=mp.get_context("spawn"))
    futs = {ex.submit(SO.oracle_stage_solution, sp): r for sp, r in zip(specs, check)}
    reqs = small_requests()
    served = {}
    for label, solver in (("point", None), ("line", dict(smoother="line", nu_pre=1, nu_post=1))):
        need = max(serve.grid_bytes(q.scenario, precision="mixed", **(solver or {})) for q in reqs)
        res, st = run(reqs, slots=6, budget=int(need * 2.2), solver=solver)
        print(f"[serving] {label}: served {len(res)} requests, evictions {st['evictions']}, peak {st['peak']}",
              flush=True)
        assert st["evictions"] > 0 and all(r.stats["status"] == "TPF_OK" for r in res)
        served[label] = res
    worst = 0.0
    try:
        for fut in cf.as_completed(futs, timeout=600):
            r = futs[fut]
            _, x_ref, info = fut.result()
            for label, res in served.items():
                x = res[r].x
                err = max(np.linalg.norm(x[c::2] - x_ref[c::2]) / np.linalg.norm(x_ref[c::2]) for c in (0, 1))
                worst = max(worst, err)
                print(f"[serving] {label} request {r} ({SIZES[r]}^3): iters {res[r].stats['iters']}, "
                      f"rel_res_true {res[r].stats['rel_res_true']:.2e}, error vs oracle {err:.2e}", flush=True)
                assert err < 1e-5, (label, r, err)
    finally:
        ex.shutdown(cancel_futures=True)
    print(f"[serving] worst error against the oracle: {worst:.2e}", flush=True)
