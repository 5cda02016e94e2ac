"""tpf_solve_stage_static (the solve whose workspace is a fixed device array inside the
library) against tpf_solve_stage, through the C ABI: two calls in a row on the same
GPU, the second on a smaller grid, each bit for bit equal to the arena solve of the
same system (same kernels, same reduction order); an oversize grid is rejected."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
tpf = pytest.importorskip("paper_2506_04763_amd")
L = pytest.importorskip("paper_2506_04763_amd._lib")


def _static_solve(g, f, rtol, maxit=400):
    x = g.empty()
    st = L.SolveStats()
    status = g.lib.tpf_solve_stage_static(g.handle, C.c_void_p(f.data_ptr()), C.c_void_p(x.data_ptr()),
                                          float(rtol), int(maxit), C.byref(st), g._sptr())
    return status, x, st.as_dict()


def _system(scn, prec, seed, **solver):
    g = tpf.Grid(scn, precision=prec, **solver)
    u = torch.as_tensor(W.perturbed_state(scn, seed, sn_lo=0.05, sn_hi=0.5).ravel(), device="cuda")
    f = g.empty()
    g.assemble_stage(u, 32.0, f0_out=f)
    return g, f


def test_static_solve_equals_arena_solve_twice_then_smaller():
    cases = [(W.small_cube(17, sigma=2.0, seed=23, levels=3), "mixed", 1e-8),
             (W.lens_2d(17, 9), "fp64", 1e-10)]
    cases[1][0].levels = 3
    for scn, prec, rtol in cases:  # the second call is on the smaller grid
        g, f = _system(scn, prec, 5)
        x_ref, st_ref = g.solve_stage(f, rtol=rtol, maxit=400)
        status, x, st = _static_solve(g, f, rtol)
        torch.cuda.synchronize()
        print(f"[no-alloc] {scn.name} {prec}: arena {st_ref['iters']} its, static {st['iters']} its, "
              f"status {status}", flush=True)
        assert status == L.TPF_OK, L.last_error()
        assert st["iters"] == st_ref["iters"] and st["rel_res_true"] == st_ref["rel_res_true"]
        np.testing.assert_array_equal(x.cpu().numpy(), x_ref.cpu().numpy())
        # the grid's own solve is unaffected by the static call
        x_again, _ = g.solve_stage(f, rtol=rtol, maxit=400)
        np.testing.assert_array_equal(x_again.cpu().numpy(), x_ref.cpu().numpy())
        g.close()


def test_static_solve_with_the_line_smoother():
    """The benchmark's multigrid (V(1,1) line-block Jacobi): the static solve equals the
    arena solve bit for bit, on a mixed 3D grid and then a smaller FP64 2D grid."""
    cases = [(W.small_cube(17, sigma=2.0, seed=23, levels=3), "mixed", 1e-8), (W.lens_2d(17, 9), "fp64", 1e-10)]
    cases[1][0].levels = 3
    for scn, prec, rtol in cases:
        g, f = _system(scn, prec, 6, smoother="line", nu_pre=1, nu_post=1)
        x_ref, st_ref = g.solve_stage(f, rtol=rtol, maxit=400)
        status, x, st = _static_solve(g, f, rtol)
        torch.cuda.synchronize()
        print(f"[no-alloc] line {scn.name} {prec}: arena {st_ref['iters']} its, static {st['iters']} its", flush=True)
        assert status == L.TPF_OK, L.last_error()
        assert st["iters"] == st_ref["iters"] and st["rel_res_true"] == st_ref["rel_res_true"]
        np.testing.assert_array_equal(x.cpu().numpy(), x_ref.cpu().numpy())
        g.close()


def test_static_solve_with_the_coarse_graph_enabled():
    """With the coarse-level graph switched on before any V-cycle has captured it, the
    static solve runs the coarse levels as stream launches (capturing would allocate);
    after an arena solve has captured the graph, the static solve replays it.  Both equal
    the arena solve bit for bit."""
    scn = W.small_cube(17, sigma=1.5, seed=41, levels=4)
    g, f = _system(scn, "mixed", 8)
    g.set_coarse_graph(True)
    status, x0, st0 = _static_solve(g, f, 1e-8)  # no graph yet
    torch.cuda.synchronize()
    assert status == L.TPF_OK, L.last_error()
    x_ref, st_ref = g.solve_stage(f, rtol=1e-8, maxit=400)  # captures the graph
    status, x1, st1 = _static_solve(g, f, 1e-8)  # replays it
    torch.cuda.synchronize()
    assert status == L.TPF_OK, L.last_error()
    print(f"[no-alloc] coarse graph: static {st0['iters']} / {st1['iters']} its, arena {st_ref['iters']} its",
          flush=True)
    for x, st in ((x0, st0), (x1, st1)):
        assert st["iters"] == st_ref["iters"]
        np.testing.assert_array_equal(x.cpu().numpy(), x_ref.cpu().numpy())
    g.close()


def test_static_solve_rejects_an_oversize_grid():
    scn = W.small_cube(81, seed=3, levels=5)  # 531,441 vertices: 76 MB of Krylov vectors
    g, f = _system(scn, "mixed", 2)
    status, _, _ = _static_solve(g, f, 1e-8)
    msg = L.last_error()
    g.close()
    assert status == L.TPF_EINVAL and "static array" in msg, (status, msg)
