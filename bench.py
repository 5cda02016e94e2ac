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
  --no-cases    skip the summaries the default line carries of the paper's case 1
                (Buckley-Leverett errors), case 5 (257^3 layered run to 128 min), case 4
                (4096 x 2048 cells to 128 min) and the 257^3 log-normal layered cube
                (20 accepted LIMEX steps)
  --limex-run K run the 257^3 LIMEX workload to K accepted steps (summary line only)
  --case5       Section 5's case 5 at the paper's mesh (257^3 vertices, 33,949,186 DoF)
                to 128 minutes of simulated time: total time, LIMEX steps and time per
                step, linear solves and time per solve beside the paper's Table
                case5_strong (summary line only)
  --case4       the same for Section 5's 2D case 4 at the mesh of Table case4_strong
                (4096 x 2048 cells, 16,789,506 DoF)
  --case4-compare  Table case4_2: case 4 on 256 x 128 cells for 10 years (injection for
                the first 2) with fixed implicit Euler steps of one day (Newton) against
                adaptive LIMEX: total time, steps, Newton and linear iterations
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



# Multigrid settings of every grid the benchmark builds: line-block Jacobi along the
# last axis, V(1, 1).  Damping per workload family: omega = 2/3 on the layered
# workloads (cases 4 and 5, the 257^3 layered cube, Table case4_2) and case 1, where
# stage systems captured from case-4 runs converge in 10-34 iterations against 22-37
# at 0.9 and fail at 1.0; omega = 0.9 on the log-normal cubes (the 129^3 stage and the
# serving requests): 62 iterations over six 129^3 cubes (sigma 1-2) against 67 at 2/3.
# --smoother point restores V(2, 2) point-block Jacobi with omega = 2/3 everywhere.
SOLVERS = {"line": {"smoother": "line", "nu_pre": 1, "nu_post": 1, "omega": 2.0 / 3.0},
           "point": {"smoother": "point", "nu_pre": 2, "nu_post": 2, "omega": 2.0 / 3.0}}
CUBE_OMEGA = {"line": 0.9, "point": 2.0 / 3.0}
SOLVER = dict(SOLVERS["line"])              # layered workloads and case 1
SOLVER_CUBE = dict(SOLVER, omega=CUBE_OMEGA["line"])  # log-normal cubes


def solver_label(sv=None):
    sv = SOLVER if sv is None else sv
    kind = "line-block Jacobi along the last axis" if sv["smoother"] == "line" else "point-block Jacobi"
    return f"V({sv['nu_pre']},{sv['nu_post']}) {kind}, omega={sv['omega']:.4g}"

def nonzero_blocks(n) -> int:
    """2x2 blocks of the 27-point stencil matrix that lie in the grid: prod(3 n_a - 2)."""
    out = 1
    for v in n:
        out *= 3 * v - 2
    return out


def algorithmic_bytes(cls: str, n, Nc_levels) -> float:
    """Bytes one launch of a kernel class must move (3D): the matrix blocks that exist
    (neighbours inside the grid; the stored zero blocks of out-of-grid neighbours are
    not counted) and the vectors.

    smooth0 / resid0 (FP32): blocks x 16 B + x, b, out (3 x 8 B per vertex); with line
      smoothing and one pre-sweep, every other residual (the one after the sweep from a
      zero guess) reads only the blocks off the lines, so resid0 averages the two
    spmv64 (FP64): blocks x 32 B + x, y and the fused dot operand (3 x 16 B per vertex)
    assemble (mixed): FP64 + FP32 matrix writes (48 B per block), F write, state and
      per-vertex data reads (u, pv 32 B, p_dmin 8 B, Q 16 B, mask 1 B), cell data 32 B
    rap: per coarse level, the FP64 fine matrix read and FP64 + FP32 coarse writes.
    line0 (FP32 line solve of a line sweep): the three line-LU blocks (48 B), the
      right-hand side or residual read (8 B), c written and read back (16 B), the
      result written (8 B; 16 B for the FP64 result of the cycle's last sweep) and the
      previous iterate read (8 B, not for the first sweep from zero): 80, 88 and 96 B
      per vertex for the first, middle and last sweep of a cycle, averaged over the
      cycle's sweeps.
    """
    N = n[0] * n[1] * n[2]
    B = nonzero_blocks(n)
    if cls == "resid0" and SOLVER_CUBE["smoother"] == "line" and SOLVER_CUBE["nu_pre"] == 1:
        B_line = n[0] * n[1] * (3 * n[2] - 2)  # the blocks along the last axis
        return (B - B_line / 2) * 16 + N * 24
    if cls in ("smooth0", "resid0"):
        return B * 16 + N * 24
    if cls == "smooth0_first":
        return N * (16 + 16)
    if cls == "spmv64":
        return B * 32 + N * 48
    if cls == "assemble":
        return B * 48 + N * (16 + 32 + 8 + 16 + 1 + 32)
    if cls == "line0":
        k = SOLVER_CUBE["nu_pre"] + SOLVER_CUBE["nu_post"]
        return N * (80 + 88 * max(k - 2, 0) + (96 if k >= 2 else 0)) / max(k, 1)
    if cls == "rap":
        return sum(nf * NST * 32 + nc * NST * 48 for nf, nc in Nc_levels) / max(len(Nc_levels), 1)
    return float("nan")


def cpu_baseline(iters_full, n_small=25):
    """The FP64 oracle, as it stands, on a bounded sample of the benchmark stage,
    single-threaded.  The oracle's stage is assembly by complex-step differentiation
    (54 complex residual passes at 129^3, one per colour and component) plus the
    Galerkin hierarchy and BiCGSTAB; its cost grows faster than the grid (large arrays).
    Measured on the 129^3 workload itself: one residual F(u0).  Measured on a
    n_small^3 grid of the same recipe: the ratio of a complex pass to a real residual,
    and the hierarchy and per-iteration times, which are scaled by the DoF ratio with
    the iteration count of the 129^3 solve."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import stage as ST
    big = W.cube_c3()
    small = W.cube_3d(n_small, 2.0, 3, levels=3)
    with threadpool_limits(1):
        st = ST.Stage(big)
        t0 = time.perf_counter()
        st.residual(big.u0.ravel())
        t_res = time.perf_counter() - t0
        sm = ST.Stage(small)
        u = small.u0.ravel()
        t0 = time.perf_counter()
        f = sm.residual(u)
        t1 = time.perf_counter()
        frozen = sm.fv.frozen_matrices(u.reshape(-1, 2))
        t2 = time.perf_counter()
        sm.assemble(u, 32.0, frozen=frozen)
        t3 = time.perf_counter()
        x, info = sm.solve(f, rtol=1e-8)
        t4 = time.perf_counter()
    passes = 2 * 27  # complex residual passes of the 3D Jacobian
    ratio = (t2 - t1) / passes / max(t1 - t0, 1e-9)  # one complex pass in units of one real residual
    scale = big.nverts / small.nverts
    t_setup = t_res * (1.0 + passes * ratio) + scale * (t3 - t2)
    t_iter = scale * (t4 - t3) / max(info["iters"], 1)
    t_full = t_setup + t_iter * iters_full
    return {"value": 1.0 / t_full, "unit": "solves/s", "cores": 1, "kind": "oracle",
            "sample": f"oracle (FP64 NumPy/SciPy, one thread) on the 129^3 stage: one residual F(u0) measured on "
                      f"the 129^3 workload ({t_res:.1f} s); the Jacobian as {passes} complex passes of "
                      f"{ratio:.2f} residuals each (ratio measured on {n_small}^3 of the same recipe); hierarchy "
                      f"{t3 - t2:.2f} s and BiCGSTAB {(t4 - t3) / max(info['iters'], 1):.3f} s per iteration at "
                      f"{n_small}^3 scaled by the DoF ratio {scale:.0f}, {iters_full} iterations: "
                      f"{t_full:.0f} s per stage"}


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
    hot = ("smooth0", "resid0", "spmv64", "assemble", "line0")  # level-0 kernels
    for prec in (["mixed"] if args.no_fp64 else ["mixed", "fp64", "mixed16"]):
        g = tpf.Grid(scn, precision=prec, levels=6, **SOLVER_CUBE)
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
        graph = None
        if prof:
            # the coarse levels as stream launches against one captured graph (identical
            # results), both without kernel timing; the timed steps use the faster
            graph = {}
            for mode in (False, True):
                g.set_coarse_graph(mode)
                g.assemble_stage(u0, h, f0_out=f)
                g.solve_stage(f, rtol=rtol, maxit=500, out=x)
                torch.cuda.synchronize()
                ta = time.perf_counter()
                for _ in range(args.steps):
                    g.assemble_stage(u0, h, f0_out=f)
                    x, st_ = g.solve_stage(f, rtol=rtol, maxit=500, out=x)
                torch.cuda.synchronize()
                graph["graph" if mode else "stream"] = round((time.perf_counter() - ta) * 1e3 / args.steps, 3)
            graph["timed_with"] = "graph" if graph["graph"] < graph["stream"] else "stream"
            g.set_coarse_graph(graph["timed_with"] == "graph")
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
                             dom=dom, levels=[g.level_dims(l) for l in range(g.levels)], bytes=g.nbytes,
                             graph=graph)
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
        b = algorithmic_bytes(cls, scn.n, nlev)
        kernels[cls] = {"launches": cnt, "avg_ms": round(avg, 5), "ms_per_step": round(tot, 3),
                        "gbs": (round(b / (avg * 1e-3) / 1e9, 1) if b == b else None)}
    dom = mixed["dom"]
    cnt, tot = mixed["kt"][dom]  # live: every launch of the class inside the timed steps
    avg_ms = tot / cnt
    ach = algorithmic_bytes(dom, scn.n, nlev) / (avg_ms * 1e-3) / 1e9
    traffic = None
    tfile = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tfile):
        try:
            tc = json.load(open(tfile)).get("classes", {}).get(dom, {})
            if tc.get("source_hash") == _source_hash(dom):
                traffic = tc.get("bytes_per_launch")
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
                   "smoother": solver_label(SOLVER_CUBE),
                   "coarse_levels": (mixed["graph"] or {}).get("timed_with", "stream")},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "launches_timed": cnt, "avg_us": round(avg_ms * 1e3, 2)},
        "iterations": mixed["iters"][-1],
        "rel_res_true": mixed["stats"]["rel_res_true"],
        "kernels": kernels,
        "arena_gb": round(mixed["bytes"] / 1e9, 3),
        "coarse_levels_ms_per_step": mixed["graph"],
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
                                 "resid_fp32": kernels.get("resid0", {}).get("gbs"),
                                 "line_fp32": kernels.get("line0", {}).get("gbs")}
    if not args.no_serve:
        from paper_2506_04763_amd import serve as SV
        prepared = SV.prepare_requests(args.serve_requests)
        sv = SV.run_benchmark(count=args.serve_requests, quiet=True, prepared=prepared, solver=SOLVER_CUBE)
        # the same requests replayed faster: where throughput stops following the rate
        sv["capacity"] = SV.capacity_sweep(rates=(80.0, 160.0, 320.0), count=args.serve_requests,
                                           prepared=prepared, solver=SOLVER_CUBE)
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
        keys = ("dof", "precision", "reached_t_end", "t_end_s", "T_total_s", "N_limex", "t_limex_s",
                "N_linear_solves", "t_linear_solve_s", "bicgstab_iterations", "unconverged_solves", "sn_max")
        for case, pe in (("case5", "256"), ("case4", "64")):
            try:
                c = layered_run(case)
                line[case] = {k: c[k] for k in keys}
                line[case][f"paper_{pe}pe"] = c[f"paper_table_{case}_strong"][pe]
            except Exception as e:
                line[case] = {"error": repr(e)}
        try:  # the 257^3 layered log-normal cube, 20 accepted k = 3 steps
            c4 = limex_run(20)
            line["cube257_limex"] = {k: c4[k] for k in c4 if k != "dt_sequence"}
            line["cube257_limex"]["dt_min_s"] = min(c4["dt_sequence"])
        except Exception as e:
            line["cube257_limex"] = {"error": repr(e)}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(mixed["iters"][-1])
    return line


def limex_run(accepted_target=20, max_attempts=80):
    """The 257^3 layered-cube LIMEX run: adaptive steps with k = 3 extrapolation
    stages from tau0 = 32 s (TOL 5e-3, safety 0.75, tau_max 100 d), FP32 multigrid
    (6 levels) inside FP64 BiCGSTAB to 1e-8, until `accepted_target` steps are
    accepted, with the consistency rule for the pressure (driver.limex_run).  Prints
    one progress line per attempted step (stderr) and returns a summary."""
    import torch

    import paper_2506_04763_amd as tpf
    import workloads as W
    from paper_2506_04763_amd import driver as DR
    scn = W.cube_c4()
    g = tpf.Grid(scn, precision="mixed", levels=6, limex_stages=3, **SOLVER)
    u = g.initial_state()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    def log(rec):
        print(json.dumps({"limex_step": rec["attempt"], **rec}), file=sys.stderr, flush=True)

    res = DR.limex_run(lambda t: (g, float("inf")), u, 0.0, float("inf"), 32.0, 3, 5e-3, 0.75, 8.64e6, 1e-8,
                       maxit=500, max_attempts=max_attempts, on_step=log, max_accepted=accepted_target)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    g.close()
    att = res["accepted"] + res["rejected"]
    return {"workload": "cube257_layered_sigma1.5_seed4_limex_k3", "vertices": list(scn.n), "dof": 2 * scn.nverts,
            "accepted": res["accepted"], "rejected": res["rejected"], "t_end_s": res["t"], "wall_s": round(wall, 2),
            "s_per_attempted_step": round(wall / max(att, 1), 3), "solves": res["solves"],
            "bicgstab_iterations": res["bicgstab_iterations"], "unconverged_solves": res["unconverged"],
            "projections": res["projections"], "dt_sequence": [round(x, 6) for x in res["dt_sequence"]]}


# Table case5_strong: PE -> (T_total s, LIMEX steps accepted + rejected, t_LIMEX s, N_linear, t_linear s)
PAPER_CASE5 = {256: (1182.3, "67+2", 17.13, 458, 0.335), 512: (640.0, "67+2", 9.28, 489, 0.194),
               1024: (372.2, "67+2", 5.39, 478, 0.146)}


# Table case4_strong, LIMEX rows: PE -> (T_total s, steps, t_LIMEX s (T_total / steps), N_linear, t_linear s)
PAPER_CASE4 = {64: (487.4, "47+1", 487.4 / 48, 307, 0.290), 128: (267.3, "47+1", 267.3 / 48, 307, 0.140),
               256: (130.7, "47+1", 130.7 / 48, 307, 0.067), 512: (65.0, "47+1", 65.0 / 48, 311, 0.033)}


# Multigrid precision per layered case: case 4's 2D section runs its multigrid in FP64.
# In FP32 its stage systems need 13-80 BiCGSTAB iterations where FP64 needs 6-19
# (systems captured at 256 x 128 cells), and at 4096 x 2048 cells solves fail at the
# 200-iteration cap (6-12 of about 460-1170 per run); each failure collapses the step
# size, so the run's length depends on where failures fall.  In FP64: 1 failure.
LAYERED_PRECISION = {"case5": "mixed", "case4": "fp64"}


def layered_run(case="case5", max_attempts=400, precision=None, rtol=1e-8, maxit=200):
    """Section 5, case 5 (257^3 layered cube) or case 4 (4096 x 2048 layered section)
    on one GPU: adaptive LIMEX (k = 3, TOL 5e-3, safety 0.75, tau0 32 s, tau_max
    100 d) from t = 0 to 128 min, the multigrid in LAYERED_PRECISION[case] (None) inside
    FP64 BiCGSTAB to rtol with at most maxit iterations per stage solve (a stage solve
    that fails rejects the step),
    every step timed on the host around the device work (inputs resident; the state
    never leaves the GPU).  One progress line per attempted step on stderr."""
    import torch

    import paper_2506_04763_amd as tpf
    import workloads as W
    scn = W.case5(257) if case == "case5" else W.case4(4096)
    paper = PAPER_CASE5 if case == "case5" else PAPER_CASE4
    precision = LAYERED_PRECISION[case] if precision is None else precision
    m = scn.meta
    t_setup = time.perf_counter()
    g = tpf.Grid(scn, precision=precision, limex_stages=m["stages"], **SOLVER)
    u = g.initial_state()
    torch.cuda.synchronize()
    setup_s = time.perf_counter() - t_setup
    from paper_2506_04763_amd import driver as DR

    def log(rec):
        print(json.dumps({f"{case}_step": rec["attempt"], **rec}), file=sys.stderr, flush=True)

    t0 = time.perf_counter()
    res = DR.limex_run(lambda t: (g, float("inf")), u, 0.0, m["t_end"], m["dt0"], m["stages"], m["tol"], m["safety"],
                       m["dt_max"], rtol, maxit=maxit, max_attempts=max_attempts, on_step=log)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    sn_max = float(u.reshape(-1, 2)[:, 1].max())
    g.close()
    t, acc = res["t"], res["accepted"]
    att = acc + res["rejected"]
    solves, iters = res["solves"], res["bicgstab_iterations"]
    name = ("case5_257^3_layered_poly_kr_point_injection_128min" if case == "case5"
            else "case4_4097x2049_layered_poly_kr_point_injection_128min")
    return {"workload": name, "dof": 2 * scn.nverts,
            "levels": scn.levels, "precision": precision, "rtol": rtol, "maxit": maxit, "stages": m["stages"],
            "t_end_s": t, "reached_t_end": bool(t >= m["t_end"] * (1 - 1e-14)),
            "T_total_s": round(wall, 2), "setup_s": round(setup_s, 2),
            "N_limex": f"{acc}+{res['rejected']}", "t_limex_s": round(wall / max(att, 1), 3),
            "N_linear_solves": solves, "t_linear_solve_s": round(wall / max(solves, 1), 4),
            "bicgstab_iterations": iters, "unconverged_solves": res["unconverged"],
            "projections": res["projections"], "sn_max": sn_max,
            f"paper_table_{case}_strong": {str(k): {"T_total_s": v[0], "N_limex": v[1],
                                                    "t_limex_s": round(v[2], 3), "N_linear": v[3],
                                                    "t_linear_s": v[4]} for k, v in paper.items()},
            "dt_sequence": [round(x, 3) for x in res["dt_sequence"]]}


# Table case4_2 (256 x 128 cells, T = 10 years): scheme -> (T_total s, time steps, N_nonlinear, N_linear)
PAPER_CASE4_2 = {"implicit_euler": (3938.76, "3650", 176596, 375093), "limex": (275.28, "6206+75", None, 58093)}


def case4_compare(cells_x=256, years=10.0, inj_years=2.0, ie_dt=86400.0, precision="fp64", lin_rtol=1e-6,
                  max_limex_attempts=40000, schemes=("limex", "implicit_euler"), wall_limit_s=1000.0,
                  max_newton=50, ie_lin_rtol=1e-6):
    """Table case4_2 of Section 5: case 4 on 256 x 128 cells for 10 years with the
    injection running for the first 2, once with fixed implicit Euler steps of one day
    (Newton, defect tolerances 1e-8 absolute / 1e-6 relative) and once with adaptive
    LIMEX (k = 3, TOL 5e-3, safety 0.75, tau0 32 s, tau_max 100 d); both solve their
    linear systems with BiCGSTAB + GMG to 1e-6 relative (the paper's relative linear
    tolerance).  The source switches off by moving the state to a second grid without
    it.  Reports total time, time steps, Newton iterations and linear iterations
    beside the paper's table.  The implicit-Euler Newton directions are solved to
    ie_lin_rtol (the paper's 1e-6 by default).  A scheme still running after wall_limit_s stops and
    reports the time it reached.  Each scheme's record is also printed to stdout as
    soon as it ends; progress lines go to stderr."""
    import copy

    import numpy as np
    import torch

    import paper_2506_04763_amd as tpf
    import workloads as W
    scn_on = W.case4(cells_x)
    scn_off = copy.deepcopy(scn_on)
    scn_off.vertex_source = np.zeros_like(scn_on.vertex_source)
    t_inj, t_end = inj_years * 365 * 86400.0, years * 365 * 86400.0
    m = scn_on.meta
    out = {"workload": f"case4_{cells_x}x{cells_x // 2}_10y_injection_2y", "dof": 2 * scn_on.nverts,
           "levels": scn_on.levels, "precision": precision, "linear_rtol": lin_rtol,
           "paper_table_case4_2": {k: {"T_total_s": v[0], "N_time_step": v[1], "N_nonlinear": v[2], "N_linear": v[3]}
                                   for k, v in PAPER_CASE4_2.items()}}
    grids = [tpf.Grid(s_, precision=precision, limex_stages=m["stages"], **SOLVER) for s_ in (scn_on, scn_off)]
    if "limex" in schemes:
        from paper_2506_04763_amd import driver as DR
        u = grids[0].initial_state()

        def grid_at(t):  # the injecting grid up to t_inj, then the one without the source
            return (grids[0], t_inj) if t < t_inj * (1 - 1e-14) else (grids[1], t_end)

        def log(rec):
            if rec["attempt"] % 500 == 0 or rec["projected"]:
                print(json.dumps({"case4_compare_limex": rec["attempt"], "t_days": rec["t"] / 86400,
                                  "dt": rec["dt"], "projected": rec["projected"]}), file=sys.stderr, flush=True)

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_wall = time.perf_counter() + wall_limit_s

        res = DR.limex_run(grid_at, u, 0.0, t_end, m["dt0"], m["stages"], m["tol"], m["safety"],
                           m["dt_max"], lin_rtol, maxit=200, max_attempts=max_limex_attempts, on_step=log,
                           stop=lambda: time.perf_counter() >= t_wall)
        torch.cuda.synchronize()
        out["limex"] = {"T_total_s": round(time.perf_counter() - t0, 2),
                        "N_time_step": f"{res['accepted']}+{res['rejected']}",
                        "reached_t_end": bool(res["t"] >= t_end * (1 - 1e-14)), "t_end_days": res["t"] / 86400.0,
                        "N_linear_solves": res["solves"], "N_linear": res["bicgstab_iterations"],
                        "unconverged_solves": res["unconverged"], "projections": res["projections"],
                        "projection_newton": res["projection_newton"],
                        "projection_linear": res["projection_linear_iters"],
                        "sn_max": float(u.reshape(-1, 2)[:, 1].max())}
        print(json.dumps({"case4_compare_record": "limex", **out["limex"]}), flush=True)
    if "implicit_euler" in schemes:
        u = grids[0].initial_state()
        t = 0.0
        steps = newton = lin = solves = fails = 0
        n_steps = int(round(t_end / ie_dt))
        todo = [ie_dt] * n_steps
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        t_wall = time.perf_counter() + wall_limit_s
        while todo and time.perf_counter() < t_wall:
            tau = todo.pop(0)
            g = grids[0] if t < t_inj * (1 - 1e-12) else grids[1]
            ok, st = g.ie_step(u, tau, atol=1e-8, rtol=1e-6, lin_rtol=ie_lin_rtol, maxit=200, max_newton=max_newton)
            newton += st["newton"]
            lin += st["linear_iters"]
            solves += st["linear_solves"]
            if not ok:  # repeated as two half steps
                fails += 1
                todo[:0] = [0.5 * tau, 0.5 * tau]
                continue
            t += tau
            steps += 1
            if steps % 250 == 0:
                print(json.dumps({"case4_compare_ie": steps, "t_days": t / 86400, "newton": newton}),
                      file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        out["implicit_euler"] = {"T_total_s": round(time.perf_counter() - t0, 2), "N_time_step": steps,
                                 "reached_t_end": not todo, "step_failures": fails, "N_nonlinear": newton,
                                 "N_linear": lin, "N_linear_solves": solves, "t_end_days": t / 86400.0,
                                 "max_newton": max_newton, "linear_rtol": ie_lin_rtol,
                                 "sn_max": float(u.reshape(-1, 2)[:, 1].max())}
        print(json.dumps({"case4_compare_record": "implicit_euler", **out["implicit_euler"]}), flush=True)
    for g in grids:
        g.close()
    if "limex" in out and "implicit_euler" in out:
        out["ie_over_limex_time"] = round(out["implicit_euler"]["T_total_s"] / max(out["limex"]["T_total_s"], 1e-9), 2)
        out["ie_over_limex_linear"] = round(out["implicit_euler"]["N_linear"] / max(out["limex"]["N_linear"], 1), 2)
    return out


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
        g = tpf.Grid(scn, precision="fp64", limex_stages=scn.meta["stages"], **SOLVER)
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
    assembly, `cycles` V-cycles and FP64 SpMVs on the finest level, and a plain
    device-to-device copy of `copy_bytes` bytes whose FETCH_SIZE / WRITE_SIZE readings
    calibrate the counters against a known byte count."""
    import torch

    import paper_2506_04763_amd as tpf
    import workloads as W
    scn = W.cube_c3()
    g = tpf.Grid(scn, precision="mixed", levels=6, **SOLVER_CUBE)
    u0 = g.initial_state()
    f = g.empty()
    g.assemble_stage(u0, 32.0, f0_out=f)
    for _ in range(cycles):
        g.precondition(f)
        g.spmv(f)
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
    "line0": ["mg.hip", "line.h", "stencil.h", "tpf_internal.h"],
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


def _csv_rows(directory, suffix):
    import csv
    import glob
    rows = []
    for f in sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True)):
        with open(f, newline="") as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def _short(name):
    """Kernel name without namespace, return type and argument list."""
    n = name.replace("void ", "", 1).replace("tpf::(anonymous namespace)::", "").replace("tpf::", "")
    return n.split("(")[0]


def summarise_trace(directory, steps):
    """Kernel-trace summary (rocprofv3 --kernel-trace CSV under `directory`): per kernel
    and grid size the launches, average/min/max duration and the time per step."""
    rows = _csv_rows(directory, "kernel_trace.csv")
    agg = {}
    for r in rows:
        if "Grid_Size_X" in r:
            grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        else:
            grid = int(r.get("Grid_Size", 0) or 0)
        key = (r["Kernel_Name"], grid)
        d = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3  # us
        agg.setdefault(key, []).append(d)
    total = sum(sum(v) for v in agg.values())
    out = ["| kernel | grid (threads) | launches | avg us | min us | max us | ms per step | % of kernel time |",
           "|---|---:|---:|---:|---:|---:|---:|---:|"]
    for (name, grid), v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        short = _short(name)
        out.append(f"| `{short}` | {grid} | {len(v)} | {sum(v) / len(v):.2f} | {min(v):.2f} | {max(v):.2f} | "
                   f"{sum(v) / 1e3 / steps:.3f} | {100 * sum(v) / total:.1f} |")
    out.append(f"\nTotal kernel time {total / 1e3:.1f} ms over {sum(len(v) for v in agg.values())} launches.")
    return "\n".join(out)


def summarise_counters(fetch_dir, write_dir, copy_bytes=1 << 30):
    """FETCH_SIZE / WRITE_SIZE per kernel and grid (one rocprofv3 --pmc pass per directory),
    calibrated by the device-to-device copy of copy_bytes bytes in the same workload."""
    def per_kernel(directory, counter):
        agg = {}
        for r in _csv_rows(directory, "counter_collection.csv"):
            if r.get("Counter_Name") != counter:
                continue
            key = (r["Kernel_Name"], int(r.get("Grid_Size", 0) or 0))
            agg.setdefault(key, []).append(float(r["Counter_Value"]))
        return {k: sum(v) / len(v) for k, v in agg.items()}
    fetch, write = per_kernel(fetch_dir, "FETCH_SIZE"), per_kernel(write_dir, "WRITE_SIZE")
    copy = [k for k in fetch if "copyBuffer" in k[0] or "copy" in k[0].lower()]
    cf = max((fetch[k] for k in copy), default=float("nan")) * 1024 / copy_bytes
    cw = max((write.get(k, 0.0) for k in copy), default=float("nan")) * 1024 / copy_bytes
    rows = {}
    for k in fetch:
        if k in copy:
            continue
        hb = fetch[k] * 1024 / cf + write.get(k, 0.0) * 1024 / cw
        rows[k] = dict(fetch_kib=fetch[k], write_kib=write.get(k, 0.0), bytes=hb)
    return rows, dict(fetch_factor=cf, write_factor=cw, copy_bytes=copy_bytes)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--smoother", choices=sorted(SOLVERS), default="line",
                    help="multigrid smoother of every grid: line (V(1,1) line-block Jacobi, the default) or point "
                         "(V(2,2) point-block Jacobi)")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cases", action="store_true",
                    help="leave out the case-1 and case-5 summaries of the default line")
    ap.add_argument("--serve-requests", type=int, default=256)
    ap.add_argument("--summarise-trace", metavar="DIR",
                    help="print the per-kernel table of a rocprofv3 kernel trace under DIR (uses --steps)")
    ap.add_argument("--summarise-counters", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "LOG"),
                    help="print FETCH_SIZE/WRITE_SIZE per kernel (calibrated by the 1 GiB copy of --counters) "
                         "and write profiles/traffic.json for the smoother; LOG is the stdout of one of the "
                         "--counters runs (its source hashes are the ones recorded)")
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
    ap.add_argument("--case4-compare", action="store_true",
                    help="Table case4_2: implicit Euler + Newton against LIMEX on case 4 (256 x 128 cells, 10 years)")
    ap.add_argument("--schemes", default="limex,implicit_euler", help="schemes of --case4-compare")
    ap.add_argument("--ie-lin-rtol", type=float, default=1e-6,
                    help="relative tolerance of the implicit-Euler Newton directions in --case4-compare")
    args = ap.parse_args()
    SOLVER.clear()
    SOLVER.update(SOLVERS[args.smoother])
    SOLVER_CUBE.clear()
    SOLVER_CUBE.update(SOLVERS[args.smoother], omega=CUBE_OMEGA[args.smoother])
    if args.summarise_trace:
        print(summarise_trace(args.summarise_trace, args.steps))
        return
    if args.summarise_counters:
        fetch_dir, write_dir, log = args.summarise_counters
        rows, cal = summarise_counters(fetch_dir, write_dir)
        run_hashes = None
        with open(log) as fh:
            for line in fh:
                if '"counters_driver"' in line:
                    run_hashes = json.loads(line)["source_hash"]
        if run_hashes is None:
            raise SystemExit(f"{log}: no counters_driver line (the stdout of a --counters run)")
        print(f"calibration: FETCH_SIZE factor {cal['fetch_factor']:.4f}, WRITE_SIZE factor {cal['write_factor']:.4f}\n")
        print("| kernel | grid | FETCH_SIZE KiB | WRITE_SIZE KiB | HBM bytes (calibrated) |")
        print("|---|---:|---:|---:|---:|")
        for (name, grid), r in sorted(rows.items(), key=lambda kv: -kv[1]["bytes"]):
            short = _short(name)
            print(f"| `{short}` | {grid} | {r['fetch_kib']:.0f} | {r['write_kib']:.0f} | {r['bytes'] / 1e6:.1f} MB |")
        # per kernel class, its finest-level launch (the largest grid of the class's kernel)
        pick = {"smooth0": lambda k: "k_jacobi_stream" in k and "float, float" in k,
                "resid0": lambda k: "k_resid_stream" in k and "float" in k,
                "line0": lambda k: k.startswith("void tpf::(anonymous namespace)::k_line<3, float"),
                "spmv64": lambda k: "k_spmv64<3" in k}
        out = {}
        for cls, match in pick.items():
            cand = [(k, r) for k, r in rows.items() if match(k[0])]
            if not cand:
                continue
            # the class's variants at its finest grid, averaged (they alternate launch for launch:
            # the residual with and without the line blocks, the line sweeps with FP32 and FP64 results)
            grid = max(k[1] for k, _ in cand)
            top = [(k, r) for k, r in cand if k[1] == grid]
            avg = {f: sum(r[f] for _, r in top) / len(top) for f in ("bytes", "fetch_kib", "write_kib")}
            out[cls] = {"kernel_name": " / ".join(sorted(_short(k[0]) for k, _ in top)), "grid": grid,
                        "source_hash": run_hashes.get(cls), "bytes_per_launch": round(avg["bytes"]),
                        "fetch_kib": avg["fetch_kib"], "write_kib": avg["write_kib"]}
        tj = {"calibration": cal, "source": "profiles/cube129_mixed_hbm_counters.md", "classes": out}
        with open(os.path.join(ROOT, "profiles", "traffic.json"), "w") as fh:
            json.dump(tj, fh, indent=1)
        return
    if args.counters:
        counters_driver()
        return
    if args.case1:
        print(json.dumps(case1_run()), flush=True)
        return
    if args.case4_compare:
        print(json.dumps(case4_compare(schemes=tuple(args.schemes.split(",")), ie_lin_rtol=args.ie_lin_rtol)),
              flush=True)
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
