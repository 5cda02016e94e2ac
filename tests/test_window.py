"""The window construction used by the full-size parity tests reproduces the full
grid's oracle rows exactly (CPU only).

A window reaching two cells past a vertex gives that vertex's residual and stage-matrix
rows; a window reaching four fine cells past vertex 2I gives row I of the first
Galerkin coarse operator.  Checked here on grids small enough for the whole-grid oracle.
"""
import numpy as np
import pytest

import workloads as W
from oracle import stage as ST
from oracle.fv import FV
from tests._window import local_index, row_window, sample_vertices, vertex_index, window

CASES = [
    ("lens17x9", lambda: W.lens_2d(17, 9)),
    ("cube9", lambda: W.small_cube(9, sigma=1.5, seed=31)),
    ("cube9_patch", lambda: W.cube_3d(9, 1.0, 32, corr_cells=2.0, rate=0.05)),
    ("case5_9", lambda: W.case5(9)),
]


@pytest.fixture(scope="module", params=CASES, ids=[c[0] for c in CASES])
def full(request):
    scn = request.param[1]()
    scn.levels = 2
    u = W.perturbed_state(scn, 7, sn_lo=0.02, sn_hi=0.6)
    st = ST.Stage(scn, levels=2)
    A = st.assemble(u.ravel(), 32.0).tocsr()
    F = st.residual(u.ravel())
    return dict(scn=scn, u=u, A=A, A1=st.H.A[1].tocsr(), F=F)


def test_fine_rows_from_windows(full):
    scn, u = full["scn"], full["u"]
    for v in sample_vertices(scn, 6, seed=1):
        lo, hi = row_window(scn, v, 2)
        w = window(scn, lo, hi, u=u)
        fv = FV(w)
        Aw = fv.stage_matrix(w.u0, 32.0).tocsr()
        Fw = fv.residual(w.u0).ravel()
        gv, lv = vertex_index(scn, v), local_index(lo, hi, v)
        for r in (0, 1):
            np.testing.assert_allclose(Fw[2 * lv + r], full["F"][2 * gv + r], rtol=1e-13, atol=1e-13 * abs(full["F"]).max())
            row_full = full["A"][2 * gv + r]
            row_w = Aw[2 * lv + r]
            # map window columns to global columns
            cols_w = row_w.indices
            lvx = (cols_w // 2) % w.n[0]
            lvy = (cols_w // 2 // w.n[0]) % w.n[1]
            lvz = cols_w // 2 // (w.n[0] * w.n[1])
            gcol = 2 * ((lvx + lo[0]) + scn.n[0] * ((lvy + lo[1]) + scn.n[1] * (lvz + lo[2]))) + cols_w % 2
            dense_full = dict(zip(row_full.indices, row_full.data))
            scale = abs(row_full.data).max()
            for c, val in zip(gcol, row_w.data):
                assert abs(val - dense_full.get(c, 0.0)) <= 1e-13 * scale
            assert len(set(dense_full) - set(gcol)) == 0 or all(
                abs(dense_full[c]) <= 1e-13 * scale for c in set(dense_full) - set(gcol))


def test_coarse_rows_from_windows(full):
    scn, u = full["scn"], full["u"]
    nc = [(scn.n[a] - 1) // 2 + 1 if a < scn.dim else 1 for a in range(3)]
    rng = np.random.default_rng(2)
    picks = {(0, 0, 0), (nc[0] - 1, nc[1] - 1, nc[2] - 1), (nc[0] // 2, nc[1] // 2, nc[2] // 2)}
    for _ in range(4):
        picks.add(tuple(int(rng.integers(0, nc[a])) for a in range(3)))
    for I in sorted(picks):
        v = tuple(2 * I[a] for a in range(3))
        lo, hi = row_window(scn, v, 4)
        w = window(scn, lo, hi, u=u, levels=2)
        st = ST.Stage(w, levels=2)
        st.assemble(w.u0.ravel(), 32.0)
        A1w = st.H.A[1].tocsr()
        ncw = [(w.n[a] - 1) // 2 + 1 for a in range(3)]
        clo = [lo[a] // 2 for a in range(3)]
        li = (I[0] - clo[0]) + ncw[0] * ((I[1] - clo[1]) + ncw[1] * (I[2] - clo[2]))
        gi = I[0] + nc[0] * (I[1] + nc[1] * I[2])
        for r in (0, 1):
            row_full = full["A1"][2 * gi + r]
            row_w = A1w[2 * li + r]
            cols_w = row_w.indices
            cx = (cols_w // 2) % ncw[0]
            cy = (cols_w // 2 // ncw[0]) % ncw[1]
            cz = cols_w // 2 // (ncw[0] * ncw[1])
            gcol = 2 * ((cx + clo[0]) + nc[0] * ((cy + clo[1]) + nc[1] * (cz + clo[2]))) + cols_w % 2
            dense_full = dict(zip(row_full.indices, row_full.data))
            scale = abs(row_full.data).max()
            got = dict(zip(gcol, row_w.data))
            for c in set(dense_full) | set(got):
                assert abs(got.get(c, 0.0) - dense_full.get(c, 0.0)) <= 1e-12 * scale, (I, r, c)
