"""Per-class kernel timing of the library (the benchmark's live measurement), through
the C ABI: the launch counts of one stage follow the solver's structure, every timed
class has positive time, a class mask times only its classes, and timing changes no
result."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
tpf = pytest.importorskip("paper_2506_04763_amd")


def stage(g, u, h=32.0):
    f = g.empty()
    g.assemble_stage(u, h, f0_out=f)
    x, st = g.solve_stage(f, rtol=1e-8, maxit=200)
    return x.cpu().numpy(), st


@pytest.fixture(scope="module")
def cube():
    scn = W.small_cube(17, seed=31, levels=3)  # levels 17^3, 9^3 and the dense 5^3
    u = torch.as_tensor(W.perturbed_state(scn, 7, sn_lo=0.05, sn_hi=0.5).ravel(), device="cuda")
    return scn, u


def test_launch_counts_follow_the_solver(cube):
    scn, u = cube
    g = tpf.Grid(scn, precision="mixed")
    g.profile_begin(100000)
    x, st = stage(g, u)
    kt = g.profile_end()
    g.close()
    print(st, kt, flush=True)
    assert st["status"] == "TPF_OK" and st["restarts"] == 0
    it = st["iters"]
    cyc = 2 * it  # two V-cycles per BiCGSTAB iteration
    expect = {
        "assemble": 1,
        "rap": scn.levels - 1,
        "coarse_lu": 1,
        "spmv64": 2 * it + 1,  # two per iteration and the true residual that confirms convergence
        "smooth0": 3 * cyc,  # second pre-sweep and both post-sweeps of V(2,2)
        "smooth0_first": cyc,
        "resid0": cyc,
        "transfer0": 2 * cyc,  # restriction and prolongation
        # level 1: pre-sweep, residual, restriction with the coarsest, prolongation, two
        # post-sweeps (its first sweep runs inside the restriction from level 0); the
        # coarsest solve
        "coarse_levels": 7 * cyc,
    }
    for cls, n in expect.items():
        assert kt[cls][0] == n, (cls, kt[cls], n)
        assert kt[cls][1] > 0.0, cls


def test_launch_counts_follow_the_line_smoother(cube):
    """V(1, 1) line smoothing: a sweep from zero is one line solve; every other sweep is
    the level residual followed by a line solve."""
    scn, u = cube
    g = tpf.Grid(scn, precision="mixed", smoother="line", nu_pre=1, nu_post=1)
    g.profile_begin(100000)
    x, st = stage(g, u)
    kt = g.profile_end()
    g.close()
    print(st, kt, flush=True)
    assert st["status"] == "TPF_OK" and st["restarts"] == 0
    it = st["iters"]
    cyc = 2 * it
    expect = {
        "assemble": 1,
        "rap": scn.levels,  # the Galerkin products and the line LU of all smoothed levels
        "coarse_lu": 1,
        "spmv64": 2 * it + 1,
        "smooth0": 0,
        "smooth0_first": 0,
        "line0": 2 * cyc,  # the pre-sweep from zero and the post-sweep
        "resid0": 2 * cyc,  # the post-sweep's residual and the restricted one
        "transfer0": 2 * cyc,
        # level 1: line solve, residual, restriction, the coarsest solve, prolongation,
        # residual and line solve of the post-sweep
        "coarse_levels": 7 * cyc,
    }
    for cls, n in expect.items():
        assert kt[cls][0] == n, (cls, kt[cls], n)
        if n:
            assert kt[cls][1] > 0.0, cls


def test_class_mask_and_results_unchanged(cube):
    scn, u = cube
    g = tpf.Grid(scn, precision="mixed")
    x0, st0 = stage(g, u)
    g.profile_begin(100000, classes=["smooth0"])
    x1, st1 = stage(g, u)
    kt = g.profile_end()
    g.close()
    assert kt["smooth0"][0] == 6 * st1["iters"] and kt["smooth0"][1] > 0.0
    assert all(kt[c][0] == 0 for c in kt if c != "smooth0")
    assert st0["iters"] == st1["iters"]
    np.testing.assert_array_equal(x0, x1)
