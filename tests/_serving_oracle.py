"""Oracle solves of serving requests, run in worker processes beside the GPU server
(test helper: the FP64 CPU oracle of the request's stage, assembled at its initial
state with h = 32 s and solved to 1e-12)."""
from __future__ import annotations


def oracle_stage_solution(spec):
    """spec: (n, sigma, seed, corr_cells, rate, levels) of a cube request -> (n, x)."""
    from threadpoolctl import threadpool_limits

    import workloads as W
    from oracle import stage as ST
    n, sigma, seed, corr, rate, levels = spec
    scn = W.cube_3d(n, sigma, seed, corr_cells=corr, rate=rate, levels=levels)
    with threadpool_limits(1):
        st = ST.Stage(scn)
        u = scn.u0.ravel()
        f = st.residual(u)
        st.assemble(u, 32.0)
        x, info = st.solve(f, rtol=1e-12, maxit=400)
    return spec, x, info
