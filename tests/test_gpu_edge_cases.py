"""Edge and degenerate cases of the HIP path against the oracle (through the C ABI).

  * grids of one or a few cells, and a one-level hierarchy (the preconditioner is
    then the dense LU solve of the whole system, so BiCGSTAB converges at once);
  * one-level grids of 578 and 686 unknowns (the dense inverse's register kernel with
    up to 16 row blocks) and the largest coarsest level the dense solve takes (4096
    unknowns, a 64 x 32 grid);
  * a grid whose every vertex is Dirichlet (A = I, F = 0) and a zero right-hand side;
  * a stage step so long (1e12 s) that the storage part all but vanishes.
"""
import numpy as np
import pytest

import workloads as W
from oracle import stage as ST

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
tpf = pytest.importorskip("paper_2506_04763_amd")

from tests.test_gpu_parity import per_field, stencil_to_csr  # noqa: E402


def parity(scn, u, h, rtol_solve=1e-12):
    """Residual, stage matrix and a tight FP64 solve against the oracle; returns the
    GPU solve statistics."""
    ref = ST.Stage(scn)
    A = ref.assemble(u.ravel(), h).tocsr()
    F = ref.residual(u.ravel())
    g = tpf.Grid(scn, precision="fp64")
    ut = torch.as_tensor(u.ravel(), device="cuda")
    f = g.residual(ut).cpu().numpy()
    scale_f = max(np.abs(F).max(), 1e-300)
    assert np.abs(f - F).max() <= 1e-11 * scale_f
    g.assemble_stage(ut, h)
    Ag = stencil_to_csr(g.matrix(0).cpu().numpy(), g.level_dims(0), scn.dim)
    assert abs(Ag - A).max() <= 1e-11 * abs(A).max()
    x, st = g.solve_stage(torch.as_tensor(F, device="cuda"), rtol=rtol_solve, maxit=200)
    g.close()
    if np.abs(F).max() > 0:
        xd = np.linalg.solve(A.toarray(), F)
        assert per_field(x.cpu().numpy(), xd) < 1e-9
    return st


@pytest.mark.parametrize("name,make", [
    ("2d_3x2", lambda: W.lens_2d(3, 2)),
    ("2d_3x3", lambda: W.lens_2d(3, 3)),
    ("3d_3", lambda: W.small_cube(3, seed=41)),
    ("3d_3x3x3_case5", lambda: W.case5(5)),
])
def test_few_cell_grids_one_level(name, make):
    scn = make()
    scn.levels = 1
    print(f"[edge] {name} n={scn.n}", flush=True)
    u = W.perturbed_state(scn, 3, dp=2e4 if name.endswith("case5") else 50.0, sn_lo=0.12, sn_hi=0.5)
    st = parity(scn, u, 32.0)
    assert st["status"] == "TPF_OK" and st["iters"] <= 2


def test_one_level_hierarchy_is_the_exact_solve():
    """9^3 vertices on one level (1458 unknowns): one V-cycle is the dense LU solve."""
    scn = W.small_cube(9, seed=42, levels=1)
    u = W.perturbed_state(scn, 5, sn_lo=0.02, sn_hi=0.6)
    st = parity(scn, u, 32.0)
    assert st["status"] == "TPF_OK" and st["iters"] <= 2


def test_largest_coarsest_level():
    """A 64 x 32 grid on one level: 4096 unknowns, the dense solve's maximum (panel
    factorisation in global memory, the trailing updates over 64 x 64 tiles)."""
    scn = W.lens_2d(64, 32)
    scn.levels = 1
    assert 2 * scn.nverts == 4096
    u = W.perturbed_state(scn, 6, sn_lo=0.02, sn_hi=0.6)
    st = parity(scn, u, 32.0)
    assert st["status"] == "TPF_OK" and st["iters"] <= 2
    big = W.lens_2d(65, 32)
    big.levels = 1
    assert tpf.validate(big) != 0  # 4160 unknowns: rejected


def test_all_dirichlet_grid_and_zero_rhs():
    """2 x 2 x 2 vertices, all on the Dirichlet faces: A = I, F = 0.  The solve of a
    zero right-hand side returns x = 0 at once; a LIMEX step leaves u unchanged with
    eps = 0 and proposes tau_max."""
    scn = W.cube_3d(2, 1.0, 1)
    assert np.all(scn.dir_mask == 3)
    g = tpf.Grid(scn, precision="fp64", limex_stages=2)
    u = torch.as_tensor(scn.u0.ravel().copy(), device="cuda")
    f = g.residual(u)
    assert float(f.abs().max()) == 0.0
    g.assemble_stage(u, 32.0)
    A = stencil_to_csr(g.matrix(0).cpu().numpy(), g.level_dims(0), 3).toarray()
    np.testing.assert_array_equal(A, np.eye(2 * scn.nverts))
    x, st = g.solve_stage(torch.zeros_like(u), rtol=1e-10)
    assert st["status"] == "TPF_OK" and st["iters"] == 0 and float(x.abs().max()) == 0.0
    u0 = u.clone()
    acc, t, dt_next, ls = g.limex_step(u, 0.0, 32.0, stages=2, dt_max=1e6)
    assert acc and t == 32.0 and ls["eps"] == 0.0 and dt_next == 1e6
    assert bool(torch.equal(u, u0))
    g.close()


def test_zero_rhs_on_a_regular_grid():
    scn = W.lens_2d(17, 9)
    scn.levels = 3
    g = tpf.Grid(scn, precision="mixed")
    g.assemble_stage(torch.as_tensor(scn.u0.ravel(), device="cuda"), 32.0)
    x, st = g.solve_stage(torch.zeros(2 * scn.nverts, dtype=torch.float64, device="cuda"), rtol=1e-8)
    assert st["status"] == "TPF_OK" and st["iters"] == 0 and float(x.abs().max()) == 0.0
    g.close()


def test_very_long_stage_step():
    """h = 1e12 s: M/h is ~1e-10 of the flux part.  The stage matrix and every
    Galerkin level still match the oracle.  (No solve is compared: without storage
    the block-Jacobi multigrid meets pure upwind transport, and neither side's
    BiCGSTAB reaches a tight tolerance in a few hundred iterations.)"""
    scn = W.lens_2d(17, 9)
    scn.levels = 3
    u = W.perturbed_state(scn, 8, sn_lo=0.05, sn_hi=0.5)
    ref = ST.Stage(scn)
    ref.assemble(u.ravel(), 1e12)
    g = tpf.Grid(scn, precision="fp64")
    g.assemble_stage(torch.as_tensor(u.ravel(), device="cuda"), 1e12)
    for l in range(scn.levels):
        Ag = stencil_to_csr(g.matrix(l).cpu().numpy(), g.level_dims(l), scn.dim)
        Ar = ref.H.A[l]
        assert abs(Ag - Ar).max() <= 1e-11 * abs(Ar).max(), l
    g.close()


@pytest.mark.parametrize("name,make", [
    ("2d_17x17", lambda: W.lens_2d(17, 17)),  # 578 unknowns
    ("3d_7", lambda: W.small_cube(7, seed=43)),  # 686 unknowns
])
def test_dense_inverse_of_hundreds_of_unknowns(name, make):
    """One level of 257-1024 unknowns: the dense inverse is formed with the column in
    registers, 64-row blocks (up to 16 of them); the solve is then exact."""
    scn = make()
    scn.levels = 1
    assert 256 < 2 * scn.nverts <= 1024
    print(f"[edge] {name} n={2 * scn.nverts}", flush=True)
    u = W.perturbed_state(scn, 9, sn_lo=0.05, sn_hi=0.5)
    st = parity(scn, u, 32.0)
    assert st["status"] == "TPF_OK" and st["iters"] <= 2


@pytest.mark.parametrize("side_stream", [False, True], ids=["current_stream", "own_stream"])
def test_coarsest_factorisation_is_awaited_before_use(side_stream):
    """The coarsest LU runs on the grid's own stream, forked after the Galerkin products;
    the caller's stream waits for it before the first coarse solve.  With a coarsest
    level of 1122 unknowns (its LU takes far longer than the finest level's descent) a
    V-cycle issued right after the assembly must equal one issued after the device has
    gone idle, bit for bit, and also the V-cycle of a grid that held a different
    operator before (stale factors would show), on the current stream and on a stream
    of the caller's own."""
    scn = W.lens_2d(65, 33)
    scn.levels = 2
    u_old = torch.as_tensor(W.perturbed_state(scn, 4, sn_lo=0.05, sn_hi=0.5).ravel(), device="cuda")
    u = torch.as_tensor(W.perturbed_state(scn, 5, sn_lo=0.05, sn_hi=0.5).ravel(), device="cuda")
    stream = torch.cuda.Stream() if side_stream else None
    with torch.cuda.stream(stream):  # (None: the current stream)
        g = tpf.Grid(scn, precision="fp64", stream=stream)
        f = g.empty()
        g.assemble_stage(u_old, 32.0)
        torch.cuda.synchronize()
        g.assemble_stage(u, 32.0, f0_out=f)
        x_now = g.precondition(f).clone()      # queued right behind the assembly
        inv_now = g.coarse_inverse().clone()
        torch.cuda.synchronize()
        x_idle = g.precondition(f)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(x_now.cpu().numpy(), x_idle.cpu().numpy())
        np.testing.assert_array_equal(inv_now.cpu().numpy(), g.coarse_inverse().cpu().numpy())
        fresh = tpf.Grid(scn, precision="fp64", stream=stream)
        fresh.assemble_stage(u, 32.0)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(fresh.precondition(f).cpu().numpy(), x_idle.cpu().numpy())
        fresh.close()
        g.close()
