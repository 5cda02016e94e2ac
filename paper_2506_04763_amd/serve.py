"""Continuous-batching server for independent stage-solve requests on one GPU.

Requests (one reservoir scenario each, any grid size) arrive over time.  A dispatcher
admits the oldest waiting request as soon as a slot is free and its grid fits the
HBM budget; grids stay resident after their solve (so a follow-up stage of the same
scenario skips create_grid) and are evicted least-recently-used when a new grid
needs the room.  Each slot owns a HIP stream and a host worker thread, so solves of
different requests overlap on the device; the library's per-iteration host
synchronisation blocks only the worker that issued it.  Every kernel reduces in a
fixed order, so a request's result does not depend on what else runs beside it.

The server allocates no device memory while it runs.  At start-up it takes one slab
of its whole budget (one allocation, outside any timed region) and carves grid
arenas out of it with a first-fit extent list that merges neighbouring free extents;
an admission that finds no hole large enough evicts idle grids, least recently used
first, until one appears.  Device allocations in the middle of a run (a grid arena
of several GB on memory the driver has just taken back) were measured to stall every
stream for up to seconds.  At shutdown the slab returns to PyTorch's cache as one
block, which the next server of the same budget gets back without an allocation.

Latency is measured from a request's arrival time to its solution being back in
host memory.
"""
from __future__ import annotations

import collections
import concurrent.futures as cf
import dataclasses
import queue
import threading
import time
from typing import Dict, List, Optional

import numpy as np

from . import Grid, grid_bytes


@dataclasses.dataclass
class StageRequest:
    rid: int
    scenario: object            # workloads.Scenario (host arrays)
    arrival: float = 0.0        # seconds after the server clock started
    h: float = 32.0
    rtol: float = 1e-8
    maxit: int = 500
    key: Optional[object] = None  # residency key (defaults to rid)


@dataclasses.dataclass
class StageResult:
    rid: int
    x: np.ndarray
    stats: dict
    t_arrive: float
    t_admit: float
    t_done: float
    cache_hit: bool

    @property
    def latency(self) -> float:
        return self.t_done - self.t_arrive


class _Resident:
    __slots__ = ("grid", "nbytes", "busy", "last_used", "offset")

    def __init__(self, grid, nbytes, offset):
        self.grid, self.nbytes, self.busy, self.last_used = grid, nbytes, False, time.perf_counter()
        self.offset = offset  # where the grid's arena starts in the server's slab


_ALIGN = 1 << 20  # arenas start on MiB boundaries of the slab


class _Extents:
    """First-fit allocator of [0, size) with coalescing free extents (host side)."""

    def __init__(self, size: int):
        self.free = [(0, size)]  # sorted (offset, length), no two adjacent

    def take(self, n: int) -> Optional[int]:
        for k, (off, length) in enumerate(self.free):
            if length >= n:
                if length == n:
                    del self.free[k]
                else:
                    self.free[k] = (off + n, length - n)
                return off
        return None

    def give(self, off: int, n: int):
        import bisect
        k = bisect.bisect_left(self.free, (off, 0))
        self.free.insert(k, (off, n))
        if k + 1 < len(self.free) and off + n == self.free[k + 1][0]:  # merge with the next
            self.free[k] = (off, n + self.free[k + 1][1])
            del self.free[k + 1]
        if k > 0 and self.free[k - 1][0] + self.free[k - 1][1] == off:  # and with the previous
            self.free[k - 1] = (self.free[k - 1][0], self.free[k - 1][1] + self.free[k][1])
            del self.free[k]


class Server:
    def __init__(self, budget_bytes: float = 200e9, slots: int = 8, precision: str = "mixed",
                 device: str = "cuda:0", keep_resident: bool = True, levels_of=None, solver=None):
        """solver: multigrid settings of every grid (smoother, nu_pre, nu_post, omega);
        None keeps the library's defaults."""
        import torch
        self.torch = torch
        self.device = torch.device(device)
        self.budget = int(budget_bytes) // _ALIGN * _ALIGN
        with torch.cuda.device(self.device):
            self._slab = torch.empty(self.budget, dtype=torch.uint8, device=self.device)
        self._extents = _Extents(self.budget)
        self.precision = precision
        self.solver = dict(solver or {})
        self.keep_resident = keep_resident
        self.levels_of = levels_of
        self._lock = threading.Condition()
        self._waiting: collections.deque = collections.deque()
        self._resident: "collections.OrderedDict[object, _Resident]" = collections.OrderedDict()
        self._used = 0
        self._free_slots = list(range(slots))
        self._streams = [torch.cuda.Stream(device=self.device) for _ in range(slots)]
        self._work: List[queue.Queue] = [queue.Queue() for _ in range(slots)]
        self._stop = False
        self.t0 = time.perf_counter()
        self.peak_used = 0
        self.evictions = 0
        self._threads = [threading.Thread(target=self._worker, args=(k,), daemon=True) for k in range(slots)]
        self._threads.append(threading.Thread(target=self._dispatch, daemon=True))
        for t in self._threads:
            t.start()

    # -- public --------------------------------------------------------------------
    def now(self) -> float:
        return time.perf_counter() - self.t0

    def submit(self, req: StageRequest) -> cf.Future:
        fut: cf.Future = cf.Future()
        with self._lock:
            self._waiting.append((req, fut, self.now() if req.arrival is None else req.arrival))
            self._lock.notify_all()
        return fut

    def shutdown(self):
        with self._lock:
            self._stop = True
            self._lock.notify_all()
        for q in self._work:
            q.put(None)
        for t in self._threads:
            t.join(timeout=60)
        with self._lock:
            for r in self._resident.values():
                if r.grid is not None:
                    r.grid.close()
            self._resident.clear()
            self._used = 0
            self._extents = _Extents(self.budget)
            self._slab = None

    # -- scheduling ------------------------------------------------------------------
    def _levels(self, scn):
        return self.levels_of(scn) if self.levels_of else scn.levels

    def _bytes(self, req):
        n = grid_bytes(req.scenario, precision=self.precision, levels=self._levels(req.scenario), **self.solver)
        return (n + _ALIGN - 1) // _ALIGN * _ALIGN

    def _evict(self, key):
        """Close an idle resident grid and return its extent to the slab."""
        r = self._resident.pop(key)
        if r.grid is not None:
            r.grid.close()  # synchronises the grid's stream: the extent is idle afterwards
        self._extents.give(r.offset, r.nbytes)
        self._used -= r.nbytes
        self.evictions += 1

    def _place(self, need) -> Optional[int]:
        """An extent of `need` bytes in the slab, evicting idle grids (least recently
        used first) until a large enough hole appears; None if none can be made."""
        while True:
            off = self._extents.take(need)
            if off is not None:
                return off
            idle = [k for k, r in self._resident.items() if not r.busy]
            if not idle:
                return None
            self._evict(idle[0])

    def _dispatch(self):
        while True:
            with self._lock:
                while not self._stop and not (self._waiting and self._free_slots):
                    self._lock.wait()
                if self._stop:
                    return
                req, fut, t_arr = self._waiting[0]
                key = req.rid if req.key is None else req.key
                hit = key in self._resident and not self._resident[key].busy
                if not hit:
                    need = self._bytes(req)
                    if need > self.budget:
                        self._waiting.popleft()
                        fut.set_exception(MemoryError(f"request {req.rid} needs {need} bytes > budget {self.budget}"))
                        continue
                    if key in self._resident:  # busy with an earlier request: wait for it
                        self._lock.wait(timeout=0.01)
                        continue
                    off = self._place(need)
                    if off is None:
                        self._lock.wait(timeout=0.01)  # wait for a running request to release memory
                        continue
                    self._used += need
                    self.peak_used = max(self.peak_used, self._used)
                    self._resident[key] = _Resident(None, need, off)
                res = self._resident[key]
                res.busy = True
                self._resident.move_to_end(key)
                self._waiting.popleft()
                slot = self._free_slots.pop()
                t_admit = self.now()
            self._work[slot].put((req, fut, t_arr, t_admit, key, hit))

    def _worker(self, slot):
        torch = self.torch
        stream = self._streams[slot]
        while True:
            item = self._work[slot].get()
            if item is None:
                return
            req, fut, t_arr, t_admit, key, hit = item
            try:
                with torch.cuda.device(self.device), torch.cuda.stream(stream):
                    with self._lock:
                        res = self._resident[key]
                    if res.grid is None:
                        arena = self._slab[res.offset:res.offset + res.nbytes]
                        res.grid = Grid(req.scenario, precision=self.precision, levels=self._levels(req.scenario),
                                        device=self.device, stream=stream, arena=arena, **self.solver)
                    g = res.grid
                    g._stream = stream
                    u0 = g.initial_state()
                    f = g.empty()
                    g.assemble_stage(u0, req.h, f0_out=f)
                    x, st = g.solve_stage(f, rtol=req.rtol, maxit=req.maxit)
                    xh = x.cpu().numpy()  # synchronous copy on this stream
                t_done = self.now()
                fut.set_result(StageResult(req.rid, xh, st, t_arr, t_admit, t_done, hit))
            except Exception as e:  # report the failure on the request's future
                fut.set_exception(e)
            finally:
                with self._lock:
                    r = self._resident.get(key)
                    if r is not None:
                        r.busy = False
                        r.last_used = time.perf_counter()
                        if not self.keep_resident:
                            self._evict(key)
                            self.evictions -= 1  # a release, not an eviction
                    self._free_slots.append(slot)
                    self._lock.notify_all()


# ---------------------------------------------------------------------------------
# Benchmark driver: Poisson arrivals replayed in real time.
# ---------------------------------------------------------------------------------
def _make_scenario(args):
    import workloads as W
    req = args
    return W.request_scenario(req)


def prepare_requests(count=256, rate_per_s=40.0, seed=5, workers=8):
    """Builds the request list and their scenarios (random fields) on the host."""
    import multiprocessing as mp

    import workloads as W
    reqs = W.serving_requests(count, rate_per_s, seed)
    ctx = mp.get_context("spawn")
    with ctx.Pool(min(workers, len(reqs))) as pool:
        scns = pool.map(_make_scenario, reqs, chunksize=1)
    return reqs, scns


def run_benchmark(count=256, rate_per_s=40.0, seed=5, budget_bytes=200e9, slots=8, precision="mixed",
                  quiet=False, prepared=None, time_scale=1.0, solver=None):
    """Replays the requests' Poisson arrivals in real time (arrival times multiplied by
    time_scale: 0.5 replays the same requests at twice the rate) and reports latency
    percentiles and throughput."""
    import workloads as W
    reqs, scns = prepared if prepared is not None else prepare_requests(count, rate_per_s, seed)
    srv = Server(budget_bytes=budget_bytes, slots=slots, precision=precision,
                 levels_of=lambda s: W.SERVE_LEVELS.get(s.n[0], s.levels), solver=solver)
    # warm the code paths (module load, first launches) outside the clock
    warm = srv.submit(StageRequest(-1, W.request_scenario(W.Request(-1, 0.0, 33, 1.0, 0.05, 999)), arrival=0.0))
    warm.result()
    srv.t0 = time.perf_counter()
    futs = []
    for req, scn in zip(reqs, scns):
        arrival = req.arrival * time_scale
        delay = arrival - srv.now()
        if delay > 0:
            time.sleep(delay)
        futs.append(srv.submit(StageRequest(req.rid, scn, arrival=arrival)))
    results = [f.result() for f in futs]
    makespan = max(r.t_done for r in results) - min(r.t_arrive for r in results)
    srv.shutdown()
    lat = np.array([r.latency for r in results])
    by_n: Dict[int, list] = collections.defaultdict(list)
    for req, r in zip(reqs, results):
        by_n[req.n].append(r.latency)
    out = {
        "requests": len(results),
        "arrival_rate_per_s": round(rate_per_s / time_scale, 3),
        "throughput_per_s": round(len(results) / makespan, 3),
        "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 2),
        "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 2),
        "max_ms": round(1e3 * float(lat.max()), 2),
        "per_size_p50_ms": {int(n): round(1e3 * float(np.percentile(v, 50)), 2) for n, v in sorted(by_n.items())},
        "all_converged": bool(all(r.stats["status"] == "TPF_OK" for r in results)),
        "max_rel_res_true": float(max(r.stats["rel_res_true"] for r in results)),
        "slots": slots,
        "budget_gb": budget_bytes / 1e9,
        "peak_resident_gb": round(srv.peak_used / 1e9, 2),
        "evictions": srv.evictions,
        "precision": precision,
    }
    if not quiet:
        print(out, flush=True)
    return out


def capacity_sweep(rates=(40.0, 80.0, 160.0), count=256, base_rate=40.0, seed=5, prepared=None, **kw):
    """The serving workload replayed at several arrival rates (the same requests, arrival
    times compressed): throughput and latency percentiles per rate.  Throughput that
    stops following the arrival rate marks the device's capacity for this mix."""
    if prepared is None:
        prepared = prepare_requests(count, base_rate, seed)
    rows = []
    for rate in rates:
        out = run_benchmark(count=count, rate_per_s=base_rate, seed=seed, prepared=prepared, quiet=True,
                            time_scale=base_rate / rate, **kw)
        rows.append({k: out[k] for k in ("arrival_rate_per_s", "throughput_per_s", "p50_ms", "p99_ms", "max_ms",
                                         "all_converged", "evictions")})
    return {"rates": rows, "capacity_per_s": max(r["throughput_per_s"] for r in rows)}
