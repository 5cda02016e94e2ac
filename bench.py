#!/usr/bin/env python3
"""Stage-solve benchmark of the gfx950 two-phase solver.

One step = one LIMEX stage solve on the 129^3-vertex log-normal cube (sigma_lnK = 2,
correlation 8 cells, 4,293,378 DoF): assemble A = M(u0)/h - J(u0) and F(u0) in one
kernel, build the 6-level Galerkin hierarchy (FP32 copies + coarsest inverse), then
BiCGSTAB in FP64 preconditioned by the FP32 V(2,2) cycle to ||r|| <= 1e-8 ||F||.
The state is resident in HBM before the clock starts.

Prints one JSON line.  Options:
  --gpus N      only N = 1 is supported (the path runs on one GPU)
  --steps K     timed steps (default 10)      --warmup W  untimed steps (default 2)
  --no-cpu      skip the oracle CPU baseline  --no-fp64   skip the FP64 and FP16-coarse comparisons
  --no-serve    skip the continuous-batching serving workload (p50/p99 latency)
  --no-cases    skip the summaries of the paper's case 1 (Buckley-Leverett errors) and
                case 5 (257^3 layered run to 128 min) that the default line carries
  --limex-run K run the 257^3 LIMEX workload to K accepted steps (summary line only)
  --case5       Section 5's case 5 at the paper's mesh (257^3 vertices, 33,949,186 DoF)
                to 128 minutes of simulated time: total time, LIMEX steps and time per
                step, linear solves and time per solve beside the paper's Table
                case5_strong (summary line only)
  --case4       the same for Section 5's 2D case 4 at the mesh of Table case4_strong
                (4096 x 2048 cells, 16,789,506 DoF)
  --case1       the Buckley-Leverett validation (Section 5, Case 1) on 64 ... 512
                elements: error norms against the Welge solution, convergence rates,
                LIMEX step counts and run times beside the paper's Table error1
                (summary line only)
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
NST = 27


def algorithmic_bytes(cls: str, N: int, Nc_levels) -> float:
    """Bytes one launch of a kernel class must move (3D, per the data layout).

    smooth0 / resid0 (FP32): 27 blocks x 16 B of matrix + x, b, out (3 x 8 B) per vertex
    spmv64 (FP64): 27 x 32 B of matrix + x, y and the fused dot operand (3 x 16 B)
    assemble (mixed): FP64 + FP32 matrix writes (864 + 432 B), F write, state and
      per-vertex data reads (u, pv 32 B, p_dmin 8 B, Q 16 B, mask 1 B), cell data 32 B
    rap: per coarse level, the FP64 fine matrix read and FP64 + FP32 coarse writes.
    """
    if cls in ("smooth0", "resid0"):
        return N * (NST * 16 + 24)
    if cls == "smooth0_first":
        return N * (16 + 16)
    if cls == "spmv64":
        return N * (NST * 32 + 48)
    if cls == "assemble":
        return N * (NST * 48 + 16 + 32 + 8 + 16 + 1 + 32)
    if cls == "rap":
        return sum(nf * NST * 32 + nc * NST * 48 for nf, nc in Nc_levels) / max(len(Nc_levels), 1)
    return float("nan")


def cpu_baseline(iters_full, n_sample=49):
    """The FP64 oracle, as it stands, on a bounded sample: one full stage (residual,
    assembly by complex-step Jacobian, Galerkin hierarchy, BiCGSTAB to 1e-8) of the same
    recipe on a 33^3 grid, single-threaded.  Setup time and time per BiCGSTAB iteration
    are scaled linearly in DoF to 129^3, with the iteration count the 129^3 solve needs."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import stage as ST
    scn = W.cube_3d(n_sample, 2.0, 3, levels=4)
    with threadpool_limits(1):
        t0 = time.perf_counter()
        st = ST.Stage(scn)
        u = scn.u0.ravel()
        f = st.residual(u)
        st.assemble(u, 32.0)
        t1 = time.perf_counter()
        x, info = st.solve(f, rtol=1e-8)
        t2 = time.perf_counter()
    scale = (129 ** 3) / (n_sample ** 3)
    t_iter = (t2 - t1) / max(info["iters"], 1)
    t_full = scale * ((t1 - t0) + t_iter * iters_full)
    return {"value": 1.0 / t_full, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle stage on the {n_sample}^3 grid of the same recipe (sigma_lnK 2, seed 3): setup "
                      f"(residual + complex-step assembly + hierarchy) {t1 - t0:.2f} s, BiCGSTAB {t2 - t1:.2f} s for "
                      f"{info['iters']} iterations; scaled by the DoF ratio {scale:.1f} to 129^3 with the "
                      f"{iters_full} iterations the 129^3 solve takes: {t_full:.0f} s per stage"}


def run(args):
    import torch

    import paper_2506_04763_amd as tpf
    import workloads as W

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a ROCm GPU")
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    scn = W.cube_c3()
    N = scn.nverts
    h = 32.0
    rtol = 1e-8
    results = {}
    hot = ("smooth0", "resid0", "spmv64", "assemble")  # level-0 matrix kernels
    for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64", "mixed16"]):
        g = tpf.Grid(scn, precision=prec, levels=6)
        u0 = g.initial_state()
        f = g.empty()
        x = g.empty()
        stats = None
        for _ in range(args.warmup):
            g.assemble_stage(u0, h, f0_out=f)
            x, stats = g.solve_stage(f, rtol=rtol, maxit=500, out=x)
        torch.cuda.synchronize()
        prof = prec == "mixed"
        breakdown, dom = None, None
        if prof:
            # untimed breakdown step: every launch of every class timed with HIP events
            g.profile_begin(200000)
            g.assemble_stage(u0, h, f0_out=f)
            x, stats = g.solve_stage(f, rtol=rtol, maxit=500, out=x)
            torch.cuda.synchronize()
            breakdown = g.profile_end()
            dom = max((k for k in hot if breakdown[k][0]), key=lambda k: breakdown[k][1])
            # the timed steps record events around the dominant kernel class only
            g.profile_begin(200000, classes=[dom])
        t0 = time.perf_counter()
        iters = []
        for _ in range(args.steps):
            g.assemble_stage(u0, h, f0_out=f)
            x, stats = g.solve_stage(f, rtol=rtol, maxit=500, out=x)
            iters.append(stats["iters"])
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        kt = g.profile_end() if prof else None
        results[prec] = dict(ms=(t1 - t0) * 1e3 / args.steps, iters=iters, stats=stats, kt=kt, breakdown=breakdown,
                             dom=dom, levels=[g.level_dims(l) for l in range(g.levels)], bytes=g.nbytes)
        g.close()
        del g
        torch.cuda.empty_cache()

    mixed = results["mixed"]
    lv = mixed["levels"]
    nlev = [(lv[i][0] * lv[i][1] * lv[i][2], lv[i + 1][0] * lv[i + 1][1] * lv[i + 1][2]) for i in range(len(lv) - 1)]
    kernels = {}  # per-class breakdown of one stage (untimed step)
    for cls, (cnt, tot) in mixed["breakdown"].items():
        if cnt == 0:
            continue
        avg = tot / cnt
        b = algorithmic_bytes(cls, N, nlev)
        kernels[cls] = {"launches": cnt, "avg_ms": round(avg, 5), "ms_per_step": round(tot, 3),
                        "gbs": (round(b / (avg * 1e-3) / 1e9, 1) if b == b else None)}
    dom = mixed["dom"]
    cnt, tot = mixed["kt"][dom]  # live: every launch of the class inside the timed steps
    avg_ms = tot / cnt
    ach = algorithmic_bytes(dom, N, nlev) / (avg_ms * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            tj = json.load(open(tfile))
            if tj.get("kernel") == dom and tj.get("source_hash") == _source_hash(dom):
                traffic = tj.get("bytes_per_launch")
        except Exception:
            traffic = None
    line = {
        "metric": "LIMEX stage solves/sec + SpMV/smoother HBM GB/s at 129^3; p50/p99 latency",
        "value": round(1e3 / mixed["ms"], 4),
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(mixed["ms"], 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "cube129_lognormal_sigma2_seed3_mixed", "vertices": [129, 129, 129], "dof": 2 * N,
                   "levels": len(lv), "precision": "FP32 multigrid in FP64 BiCGSTAB", "rtol": rtol, "h_s": h,
                   "smoother": "V(2,2) block-Jacobi omega=2/3"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "launches_timed": cnt, "avg_us": round(avg_ms * 1e3, 2)},
        "iterations": mixed["iters"][-1],
        "rel_res_true": mixed["stats"]["rel_res_true"],
        "kernels": kernels,
        "arena_gb": round(mixed["bytes"] / 1e9, 3),
    }
    if "fp64" in results:
        r = results["fp64"]
        line["fp64"] = {"solves_per_s": round(1e3 / r["ms"], 4), "ms_per_step": round(r["ms"], 3),
                        "iterations": r["iters"][-1], "rel_res_true": r["stats"]["rel_res_true"]}
        line["mixed_over_fp64"] = round(r["ms"] / mixed["ms"], 3)
    if "mixed16" in results:  # coarse-level matrices in FP16 with row scales (optional mode)
        r = results["mixed16"]
        line["mixed16"] = {"solves_per_s": round(1e3 / r["ms"], 4), "ms_per_step": round(r["ms"], 3),
                           "iterations": r["iters"][-1], "rel_res_true": r["stats"]["rel_res_true"]}
    sm = [kernels[k]["gbs"] for k in ("smooth0", "resid0") if k in kernels]
    line["spmv_smoother_gbs"] = {"spmv64": kernels.get("spmv64", {}).get("gbs"),
                                 "smoother_fp32": kernels.get("smooth0", {}).get("gbs"),
                                 "resid_fp32": kernels.get("resid0", {}).get("gbs")}
    if not args.no_serve:
        from paper_2506_04763_amd import serve as SV
        prepared = SV.prepare_requests(args.serve_requests)
        sv = SV.run_benchmark(count=args.serve_requests, quiet=True, prepared=prepared)
        # the same requests replayed faster: where throughput stops following the rate
        sv["capacity"] = SV.capacity_sweep(rates=(80.0, 160.0, 320.0), count=args.serve_requests,
                                           prepared=prepared)
        line["serving"] = sv
        line["p50_ms"], line["p99_ms"] = sv["p50_ms"], sv["p99_ms"]
    if not args.no_cases:
        # the paper's own workloads, summarised (full records: --case1, --case5)
        try:
            c1 = case1_run()
            line["case1"] = {"L1": [r["L1"] for r in c1["rows"]], "L2": [r["L2"] for r in c1["rows"]],
                             "elements": [r["elements"] for r in c1["rows"]],
                             "steps": [r["steps"] for r in c1["rows"]], "rate_L1": c1["rate_L1"],
                             "rate_L2": c1["rate_L2"], "wall_s": [r["wall_s"] for r in c1["rows"]],
                             "paper_L1": [r["paper_limex"]["L1"] for r in c1["rows"]],
                             "paper_L2": [r["paper_limex"]["L2"] for r in c1["rows"]]}
        except Exception as e:  # reported, never fatal to the benchmark line
            line["case1"] = {"error": repr(e)}
        try:
            c5 = layered_run("case5")
            line["case5"] = {k: c5[k] for k in ("dof", "reached_t_end", "T_total_s", "N_limex", "t_limex_s",
                                                 "N_linear_solves", "t_linear_solve_s", "bicgstab_iterations",
                                                 "unconverged_solves")}
            line["case5"]["paper_256pe"] = c5["paper_table_case5_strong"]["256"]
        except Exception as e:
            line["case5"] = {"error": repr(e)}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(mixed["iters"][-1])
    return line


def limex_run(accepted_target=20, max_attempts=80):
    """The 257^3 layered-cube LIMEX run: adaptive steps with k = 3 extrapolation
    stages from tau0 = 32 s (TOL 5e-3, safety 0.75, tau_max 100 d), FP32 multigrid
    (6 levels) inside FP64 BiCGSTAB to 1e-8, until `accepted_target` steps are
    accepted.  Prints one progress line per attempted step (stderr) and returns a
    summary."""
    import torch

    import paper_2506_04763_amd as tpf
    import workloads as W
    scn = W.cube_c4()
    g = tpf.Grid(scn, precision="mixed", levels=6, limex_stages=3)
    u = g.initial_state()
    t, dt = 0.0, 32.0
    steps = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    while sum(1 for s in steps if s["accepted"]) < accepted_target and len(steps) < max_attempts:
        ts = time.perf_counter()
        acc, t, dt_next, st = g.limex_step(u, t, dt, stages=3, tol=5e-3, safety=0.75, dt_max=8.64e6, rtol=1e-8)
        torch.cuda.synchronize()
        rec = dict(accepted=bool(acc), dt=dt, eps=st["eps"], dt_next=dt_next, solves=st["solves"],
                   iters=st["iters_total"], unconverged=st["unconverged"], seconds=time.perf_counter() - ts)
        steps.append(rec)
        print(json.dumps({"limex_step": len(steps), "t": t, **rec}), file=sys.stderr, flush=True)
        dt = dt_next
    wall = time.perf_counter() - t0
    g.close()
    acc = [s for s in steps if s["accepted"]]
    return {"workload": "cube257_layered_sigma1.5_seed4_limex_k3", "vertices": list(scn.n), "dof": 2 * scn.nverts,
            "accepted": len(acc), "rejected": len(steps) - len(acc), "t_end_s": t, "wall_s": round(wall, 2),
            "s_per_attempted_step": round(wall / max(len(steps), 1), 3),
            "solves": sum(s["solves"] for s in steps), "bicgstab_iterations": sum(s["iters"] for s in steps),
            "unconverged_solves": sum(s["unconverged"] for s in steps),
            "dt_sequence": [round(s["dt"], 3) for s in steps]}


# Table case5_strong: PE -> (T_total s, LIMEX steps accepted + rejected, t_LIMEX s, N_linear, t_linear s)
PAPER_CASE5 = {256: (1182.3, "67+2", 17.13, 458, 0.335), 512: (640.0, "67+2", 9.28, 489, 0.194),
               1024: (372.2, "67+2", 5.39, 478, 0.146)}


# Table case4_strong, LIMEX rows: PE -> (T_total s, steps, t_LIMEX s (T_total / steps), N_linear, t_linear s)
PAPER_CASE4 = {64: (487.4, "47+1", 487.4 / 48, 307, 0.290), 128: (267.3, "47+1", 267.3 / 48, 307, 0.140),
               256: (130.7, "47+1", 130.7 / 48, 307, 0.067), 512: (65.0, "47+1", 65.0 / 48, 311, 0.033)}


def layered_run(case="case5", max_attempts=400, precision="mixed", rtol=1e-8, maxit=200):
    """Section 5, case 5 (257^3 layered cube) or case 4 (4096 x 2048 layered section)
    on one GPU: adaptive LIMEX (k = 3, TOL 5e-3, safety 0.75, tau0 32 s, tau_max
    100 d) from t = 0 to 128 min, FP32 multigrid inside FP64 BiCGSTAB to rtol with at
    most maxit iterations per stage solve (a stage solve that fails rejects the step),
    every step timed on the host around the device work (inputs resident; the state
    never leaves the GPU).  One progress line per attempted step on stderr."""
    import torch

    import paper_2506_04763_amd as tpf
    import workloads as W
    scn = W.case5(257) if case == "case5" else W.case4(4096)
    paper = PAPER_CASE5 if case == "case5" else PAPER_CASE4
    m = scn.meta
    t_setup = time.perf_counter()
    g = tpf.Grid(scn, precision=precision, limex_stages=m["stages"])
    u = g.initial_state()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    t, dt = 0.0, m["dt0"]
    steps = []
    t0 = time.perf_counter()
    while t < m["t_end"] * (1 - 1e-14) and len(steps) < max_attempts:
        dt = min(dt, m["t_end"] - t)
        ts = time.perf_counter()
        acc, t, dt_next, st = g.limex_step(u, t, dt, stages=m["stages"], tol=m["tol"], safety=m["safety"],
                                           dt_max=m["dt_max"], rtol=rtol, maxit=maxit)
        torch.cuda.synchronize()
        rec = dict(accepted=bool(acc), t=t, dt=dt, eps=st["eps"], solves=st["solves"], iters=st["iters_total"],
                   unconverged=st["unconverged"], seconds=time.perf_counter() - ts)
        steps.append(rec)
        print(json.dumps({f"{case}_step": len(steps), **rec}), file=sys.stderr, flush=True)
        dt = dt_next
    wall = time.perf_counter() - t0
    sn_max = float(u.reshape(-1, 2)[:, 1].max())
    g.close()
    acc = sum(1 for s in steps if s["accepted"])
    solves = sum(s["solves"] for s in steps)
    iters = sum(s["iters"] for s in steps)
    name = ("case5_257^3_layered_poly_kr_point_injection_128min" if case == "case5"
            else "case4_4097x2049_layered_poly_kr_point_injection_128min")
    return {"workload": name, "dof": 2 * scn.nverts,
            "levels": scn.levels, "precision": precision, "rtol": rtol, "maxit": maxit, "stages": m["stages"],
            "t_end_s": t, "reached_t_end": bool(t >= m["t_end"] * (1 - 1e-14)),
            "T_total_s": round(wall, 2), "setup_s": round(setup_s, 2),
            "N_limex": f"{acc}+{len(steps) - acc}", "t_limex_s": round(wall / max(len(steps), 1), 3),
            "N_linear_solves": solves, "t_linear_solve_s": round(wall / max(solves, 1), 4),
            "bicgstab_iterations": iters, "unconverged_solves": sum(s["unconverged"] for s in steps),
            "sn_max": sn_max,
            f"paper_table_{case}_strong": {str(k): {"T_total_s": v[0], "N_limex": v[1],
                                                    "t_limex_s": round(v[2], 3), "N_linear": v[3],
                                                    "t_linear_s": v[4]} for k, v in paper.items()},
            "dt_sequence": [round(s["dt"], 3) for s in steps]}


def case1_run(elements=(64, 128, 256, 512)):
    """Case 1 of Section 5: adaptive LIMEX (k = 2, TOL 5e-2, safety 0.25, tau0 1 s,
    tau_max 100 d) to 1500 days on the 300 m x 75 m strip, FP64 multigrid inside FP64
    BiCGSTAB to 1e-10, at each resolution; the L1 / L2 norms of S_w - S_wh against
    the analytic Welge solution and their rates, beside the paper's Table error1."""
    import torch

    import paper_2506_04763_amd as tpf
    import workloads as W
    from tests import buckley_leverett as BL
    rows, l1s, l2s = [], [], []
    for el in elements:
        scn = W.buckley_leverett(el)
        g = tpf.Grid(scn, precision="fp64", limex_stages=scn.meta["stages"])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        u, st = BL.run_gpu(g, scn)
        wall = time.perf_counter() - t0
        g.close()
        sw = 1.0 - u[:, 1].reshape(scn.n[1], scn.n[0])
        l1, l2 = BL.error_norms(sw, el)
        l1s.append(l1)
        l2s.append(l2)
        p = BL.PAPER_LIMEX[el]
        rows.append({"elements": el, "vertices": [scn.n[0], scn.n[1]], "dof": 2 * scn.nverts,
                     "levels": scn.levels, "steps": f"{st['accepted']}+{st['rejected']}",
                     "solves": st["solves"], "bicgstab_iterations": st["iterations"],
                     "unconverged": st["unconverged"], "wall_s": round(wall, 3),
                     "ms_per_step": round(1e3 * wall / max(st["accepted"] + st["rejected"], 1), 3),
                     "L1": round(l1, 4), "L2": round(l2, 4),
                     "paper_limex": {"steps": p[0], "L1": p[1], "L2": p[2]}})
        print(json.dumps({"case1": rows[-1]}), file=sys.stderr, flush=True)
    r1, r2 = BL.rates(l1s), BL.rates(l2s)
    pr1 = BL.rates([BL.PAPER_LIMEX[e][1] for e in elements])
    pr2 = BL.rates([BL.PAPER_LIMEX[e][2] for e in elements])
    return {"workload": "case1_buckley_leverett_300x75m_1500d", "precision": "fp64", "rtol": 1e-10,
            "rows": rows, "rate_L1": [round(r, 3) for r in r1], "rate_L2": [round(r, 3) for r in r2],
            "paper_rate_L1": [round(r, 3) for r in pr1], "paper_rate_L2": [round(r, 3) for r in pr2],
            "front_speed_m_per_s": BL.front_speed()}


def counters_driver(cycles=4, copy_bytes=1 << 30):
    """Short workload for hardware-counter runs: one 129^3 mixed-precision stage
    assembly, `cycles` V-cycles (4 fine-level smoother sweeps each), and a plain
    device-to-device copy of `copy_bytes` bytes whose FETCH_SIZE / WRITE_SIZE readings
    calibrate the counters against a known byte count."""
    import torch

    import paper_2506_04763_amd as tpf
    import workloads as W
    scn = W.cube_c3()
    g = tpf.Grid(scn, precision="mixed", levels=6)
    u0 = g.initial_state()
    f = g.empty()
    g.assemble_stage(u0, 32.0, f0_out=f)
    for _ in range(cycles):
        g.precondition(f)
    a = torch.empty(copy_bytes // 4, dtype=torch.float32, device="cuda")
    a.fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"counters_driver": "done", "vertices": scn.nverts, "copy_bytes": copy_bytes,
                      "source_hash": {k: _source_hash(k) for k in KERNEL_SOURCES}}), flush=True)


KERNEL_SOURCES = {  # files whose text defines each timed kernel class
    "smooth0": ["mg.hip", "stencil.h", "tpf_internal.h"],
    "resid0": ["mg.hip", "stencil.h", "tpf_internal.h"],
    "spmv64": ["mg.hip", "stencil.h", "tpf_internal.h"],
    "assemble": ["assemble.hip", "tpf_internal.h"],
}


def _source_hash(kernel="smooth0"):
    """Hash of the sources of a kernel class: hardware-counter figures recorded for
    one version of a kernel are not reported for another."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES.get(kernel, sorted(os.listdir(os.path.join(ROOT, "paper_2506_04763_amd", "csrc")))):
        h.update(open(os.path.join(ROOT, "paper_2506_04763_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cases", action="store_true",
                    help="leave out the case-1 and case-5 summaries of the default line")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--counters", action="store_true",
                    help="run the short hardware-counter workload instead of the benchmark")
    ap.add_argument("--limex-run", type=int, default=0, metavar="K",
                    help="run the 257^3 LIMEX workload until K steps are accepted instead of the benchmark")
    ap.add_argument("--case1", action="store_true",
                    help="run the Buckley-Leverett validation instead of the benchmark")
    ap.add_argument("--case5", action="store_true",
                    help="run Section 5's case 5 at 257^3 to 128 minutes instead of the benchmark")
    ap.add_argument("--case4", action="store_true",
                    help="run Section 5's case 4 at 4096 x 2048 cells to 128 minutes instead of the benchmark")
    args = ap.parse_args()
    if args.counters:
        counters_driver()
        return
    if args.case1:
        print(json.dumps(case1_run()), flush=True)
        return
    if args.case5 or args.case4:
        print(json.dumps(layered_run("case5" if args.case5 else "case4")), flush=True)
        return
    if args.limex_run:
        print(json.dumps(limex_run(args.limex_run)), flush=True)
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the stage solver has no multi-GPU "
                                   "path", "n_gpus": args.gpus}))
        sys.exit(2)
    print(json.dumps(run(args)), flush=True)


if __name__ == "__main__":
    main()
