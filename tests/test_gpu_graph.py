"""The V-cycle's coarse levels replayed as one captured HIP graph (tpf_set_coarse_graph)
against stream launches of the same kernels: bit for bit, on every replay, with the
program's own work and synchronisations between replays, after a re-assembly at a new
state (new values at the same addresses), and through whole solves."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
tpf = pytest.importorskip("paper_2506_04763_amd")


@pytest.mark.parametrize("prec", ["mixed", "fp64", "mixed16"])
def test_coarse_graph_equals_stream_launches(prec):
    scn = W.small_cube(17, sigma=1.5, seed=41, levels=4)   # 17^3 -> 9^3 -> 5^3 -> 3^3
    g = tpf.Grid(scn, precision=prec)
    ref = tpf.Grid(scn, precision=prec)
    g.set_coarse_graph(True)
    for seed in (3, 4):  # two assemblies: the captured graph must follow new matrix values
        u = torch.as_tensor(W.perturbed_state(scn, seed, sn_lo=0.05, sn_hi=0.5).ravel(), device="cuda")
        f = g.empty()
        g.assemble_stage(u, 32.0, f0_out=f)
        ref.assemble_stage(u, 32.0)
        x_ref = ref.precondition(f).cpu().numpy()
        for k in range(4):
            x = g.precondition(f)
            y = g.spmv(x)                       # eager work between replays
            torch.cuda.synchronize()
            _ = float(y.abs().max())
            print(f"[graph] {prec} assembly {seed} replay {k}", flush=True)
            np.testing.assert_array_equal(x.cpu().numpy(), x_ref)
        xs, st = g.solve_stage(f, rtol=1e-8 if prec != "fp64" else 1e-10)
        xr, sr = ref.solve_stage(f, rtol=1e-8 if prec != "fp64" else 1e-10)
        assert st["iters"] == sr["iters"]
        np.testing.assert_array_equal(xs.cpu().numpy(), xr.cpu().numpy())
    g.close()
    ref.close()
