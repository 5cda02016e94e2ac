"""Pins of the oracle's line-block Jacobi smoother (CPU).

The smoother is x <- x + omega A_L^{-1} (b - A x), A_L the couplings of A between
vertices of one line along the last axis.  Pinned here against what fixes it
independently of its code: the line structure written out by vertex coordinates, the
exact solve of operators that are their own line part, the closed-form inverse of a
constant tridiagonal line (sine eigenvectors), invariance under the block-diagonal
row transform of the coarse-grid correction, and the stall of point smoothing it
removes on the layered case.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import gmg as G
from oracle import stage as ST


def _coords(n, dim):
    nx, ny, nz = n
    out = []
    for v in range(nx * ny * nz):
        ix, t = v % nx, v // nx
        out.append((ix, t % ny, t // ny))
    return out


def _random_stencil_matrix(n, dim, seed):
    """2x2 blocks between every vertex and its 27 (3D) / 9 (2D) neighbours, random."""
    rng = np.random.default_rng(seed)
    xyz = _coords(n, dim)
    index = {c: v for v, c in enumerate(xyz)}
    rows, cols, vals = [], [], []
    for v, (ix, iy, iz) in enumerate(xyz):
        for dz in ((-1, 0, 1) if dim == 3 else (0,)):
            for dy in (-1, 0, 1):
                for dx in (-1, 0, 1):
                    w = index.get((ix + dx, iy + dy, iz + dz))
                    if w is None:
                        continue
                    for r in range(2):
                        for c in range(2):
                            rows.append(2 * v + r)
                            cols.append(2 * w + c)
                            vals.append(rng.standard_normal() + (20.0 if v == w and r == c else 0.0))
    N = len(xyz)
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * N, 2 * N)), xyz


@pytest.mark.parametrize("n,dim", [((5, 4, 1), 2), ((4, 3, 5), 3)])
def test_line_part_keeps_exactly_the_couplings_within_a_line(n, dim):
    A, xyz = _random_stencil_matrix(n, dim, 3)
    AL = G.line_part(A, n, dim).toarray()
    Ad = A.toarray()
    for i in range(Ad.shape[0]):
        for j in range(Ad.shape[1]):
            a, b = xyz[i // 2], xyz[j // 2]
            same = a[0] == b[0] and (dim == 2 or a[1] == b[1])
            assert AL[i, j] == (Ad[i, j] if same else 0.0)
    # a line couples a vertex with itself and its two neighbours along the last axis
    ax = 1 if dim == 2 else 2
    for i, j in zip(*np.nonzero(AL)):
        assert abs(xyz[i // 2][ax] - xyz[j // 2][ax]) <= 1


@pytest.mark.parametrize("n,dim", [((5, 4, 1), 2), ((4, 3, 5), 3)])
def test_one_undamped_sweep_solves_an_operator_that_is_its_own_line_part(n, dim):
    A, _ = _random_stencil_matrix(n, dim, 4)
    A = G.line_part(A, n, dim)
    H = G.Hierarchy(A, n, dim, 1, np.zeros(n[0] * n[1] * n[2], np.uint8), omega=1.0, smoother="line")
    rng = np.random.default_rng(5)
    b, x0 = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    x1 = H.smooth(0, x0, b, 1)
    assert np.linalg.norm(A @ x1 - b) <= 1e-12 * np.linalg.norm(b)
    # damping scales the correction
    H.omega = 0.5
    xh = H.smooth(0, x0, b, 1)
    np.testing.assert_allclose(xh, x0 + 0.5 * (x1 - x0), rtol=0, atol=1e-12 * np.abs(x1).max())


def test_line_solve_of_a_constant_tridiagonal_line_by_its_sine_eigenvectors():
    """Lines along y of a 3 x 7 grid, each component decoupled with the stencil
    (-1, 2 + e, -1) along the line: sin(k pi (j + 1) / 8), j = 0..6, is an
    eigenvector with eigenvalue 2 + e - 2 cos(k pi / 8), so one undamped sweep from
    zero returns b divided by it."""
    nx, ny, e = 3, 7, 0.3
    N = nx * ny
    rows, cols, vals = [], [], []
    for v in range(N):
        iy = v // nx
        for c in range(2):
            rows.append(2 * v + c); cols.append(2 * v + c); vals.append(2.0 + e)
            for dy in (-1, 1):
                if 0 <= iy + dy < ny:
                    rows.append(2 * v + c); cols.append(2 * (v + dy * nx) + c); vals.append(-1.0)
            # couplings across lines and between the components, which A_L drops
            if v % nx + 1 < nx:
                rows.append(2 * v + c); cols.append(2 * (v + 1) + c); vals.append(-0.7)
            rows.append(2 * v + c); cols.append(2 * v + 1 - c); vals.append(0.0)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(2 * N, 2 * N))
    H = G.Hierarchy(A, (nx, ny, 1), 2, 1, np.zeros(N, np.uint8), omega=1.0, smoother="line")
    b = np.zeros(2 * N)
    lam = np.zeros(2 * N)
    for v in range(N):
        ix, iy = v % nx, v // nx
        for c in range(2):
            k = 1 + ix + 3 * c  # a different eigenvector on every line and component
            b[2 * v + c] = np.sin(k * np.pi * (iy + 1) / (ny + 1))
            lam[2 * v + c] = 2.0 + e - 2.0 * np.cos(k * np.pi / (ny + 1))
    x = H.smooth(0, np.zeros(2 * N), b, 1)
    np.testing.assert_allclose(x, b / lam, rtol=1e-12, atol=1e-14)


def test_line_smoothing_is_invariant_under_the_volume_balance_transform():
    """T is block diagonal per vertex, so it maps A_L to T A_L:
    (T A_L)^{-1} (T b - T A x) = A_L^{-1} (b - A x); the finest level may be smoothed
    with A itself, as with point-block Jacobi."""
    scn = W.lens_2d(17, 9)
    scn.rho = (1000.0, 1460.0)
    st = ST.Stage(scn, levels=2, smoother="line")
    u = W.perturbed_state(scn, 5, sn_lo=0.05, sn_hi=0.5)
    A = st.assemble(u.ravel(), 32.0)
    T = st.H.T0
    rng = np.random.default_rng(1)
    x0, b = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    Ht = G.Hierarchy(T @ A, scn.n, scn.dim, 1, scn.dir_mask, smoother="line")
    H1 = G.Hierarchy(A, scn.n, scn.dim, 1, scn.dir_mask, smoother="line")
    xa = Ht.smooth(0, x0, T @ b, 3)
    xb = H1.smooth(0, x0, b, 3)
    assert np.linalg.norm(xa - xb) <= 1e-12 * np.linalg.norm(xb)


def test_line_smoothing_removes_the_stall_of_point_smoothing_on_layers():
    """Case 4 at 65 x 33 vertices, initial state, step 1e7 s: GMG-BiCGSTAB with point
    smoothing stalls above 1e-3 in 150 iterations, with line smoothing it converges
    to 1e-8 in at most 8."""
    scn = W.case4(64)
    u = scn.u0.ravel().astype(np.float64)
    res = {}
    for sm in ("jacobi", "line"):
        st = ST.Stage(scn, smoother=sm)
        st.assemble(u, 1e7)
        _, info = st.solve(st.residual(u), rtol=1e-8, maxit=150)
        res[sm] = info
    assert res["jacobi"]["rel_res_true"] > 1e-3
    assert res["line"]["rel_res_true"] <= 1e-8 and res["line"]["iters"] <= 8


def test_unknown_smoother_is_rejected():
    with pytest.raises(ValueError):
        G.Hierarchy(sp.identity(4, format="csr"), (2, 1, 1), 2, 1, np.zeros(2, np.uint8), smoother="gauss")


@pytest.mark.parametrize("n,dim", [((5, 4, 1), 2), ((4, 3, 5), 3)])
def test_residual_after_a_zero_guess_sweep_needs_no_line_blocks(n, dim):
    """After one damped line sweep from a zero guess, x = omega A_L^{-1} b, so
    b - A x = (1 - omega) b - (A - A_L) x: the identity the library's restriction
    residual uses to skip the line blocks of every row."""
    A, _ = _random_stencil_matrix(n, dim, 6)
    H = G.Hierarchy(A, n, dim, 1, np.zeros(n[0] * n[1] * n[2], np.uint8), omega=0.9, smoother="line")
    b = np.random.default_rng(7).standard_normal(A.shape[0])
    x = H.smooth(0, np.zeros_like(b), b, 1)
    AL = G.line_part(A, n, dim)
    direct = b - A @ x
    off = (1.0 - 0.9) * b - (A - AL) @ x
    np.testing.assert_allclose(off, direct, rtol=0, atol=1e-12 * np.abs(b).max())
