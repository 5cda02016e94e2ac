"""Writes the oracle's solution of a full-size stage at sampled vertices.

    python tests/golden/make_fullsize_reference.py cube65    # ~5 min, ~3 GB
    python tests/golden/make_fullsize_reference.py cube129   # ~1 h, ~25 GB

The stage is the one the benchmark and the full-size GPU tests run: A = M(u0)/h -
J(u0) at the workload's initial state, h = 32 s, f = F(u0), solved by the oracle's
BiCGSTAB + V(2,2) to rtol 1e-10 (FP64).  Only the oracle and the seeded input
generator are called.  The output (JSON) holds the solution at sampled vertices and
the norms of both fields, for the per-field comparison with the GPU solution.
"""
from __future__ import annotations

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import workloads as W  # noqa: E402
from oracle import stage as ST  # noqa: E402
from tests._window import sample_vertices, vertex_index  # noqa: E402

WORKLOADS = {"cube65": (W.cube_c2, 5), "cube129": (W.cube_c3, 6)}


def main(name):
    make, levels = WORKLOADS[name]
    scn = make()
    t0 = time.time()
    st = ST.Stage(scn, levels=levels)
    u = scn.u0.ravel()
    f = st.residual(u)
    st.assemble(u, 32.0)
    x, info = st.solve(f, rtol=1e-10, maxit=400)
    r = f - st.A @ x
    samples = sample_vertices(scn, 200, seed=11)
    idx = [vertex_index(scn, v) for v in samples]
    xs = x.reshape(-1, 2)
    out = {
        "workload": name,
        "levels": levels,
        "h": 32.0,
        "rtol": 1e-10,
        "oracle_iters": int(info["iters"]),
        "oracle_rel_res_true": float(np.linalg.norm(r) / np.linalg.norm(f)),
        "norm_inf": [float(abs(xs[:, 0]).max()), float(abs(xs[:, 1]).max())],
        "norm_2": [float(np.linalg.norm(xs[:, 0])), float(np.linalg.norm(xs[:, 1]))],
        "f_norm_2": float(np.linalg.norm(f)),
        "samples": [[int(i), float(xs[i, 0]), float(xs[i, 1])] for i in idx],
        "seconds": round(time.time() - t0, 1),
    }
    with open(os.path.join(HERE, f"{name}_stage_solution.json"), "w") as fh:
        json.dump(out, fh, indent=0)
    print(name, out["oracle_iters"], out["oracle_rel_res_true"], out["seconds"], "s")


if __name__ == "__main__":
    main(sys.argv[1] if len(sys.argv) > 1 else "cube65")
