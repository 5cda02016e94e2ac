"""The library's per-thread kernel bodies built for the CPU (tests/cpu_harness/harness.hip,
AddressSanitizer on the host side) and checked without a GPU:

  * log_pos / exp_fin (the series logarithm and Taylor exponential of the constitutive
    powers) against 60-digit decimal arithmetic: within their stated 4e-16 relative;
  * residual and stage-matrix rows, with the laws evaluated inline, through the corner
    pass, and (3D) through the two-thread split of the row, against the FP64 oracle;
  * the two-pass Galerkin product over the exact thread mapping of its launches
    (XCD-aware block order included): every scratch and coarse block written exactly
    once, and the coarse operator equal to the oracle's;
  * the line-block Jacobi bodies (block LU of every line, one sweep per line in FP64
    and FP32, from a zero guess and in place) against the oracle's line solve.

Every launch's threads run over buffers of exactly the sizes the kernels get, so the
sanitizer reports any access outside them; the harness must exit cleanly."""
import decimal
import os
import subprocess

import numpy as np
import pytest
import scipy.sparse as sp

import workloads as W
from oracle import fv as FV
from oracle import gmg as G
from oracle import stage as ST

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SRC = os.path.join(HERE, "cpu_harness", "harness.hip")
CSRC = os.path.join(ROOT, "paper_2506_04763_amd", "csrc")
BUILD = os.path.join(HERE, "_build")
EXE = os.path.join(BUILD, "harness")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _sources():
    return [SRC] + [os.path.join(CSRC, f) for f in ("assemble.hip", "rap.hip", "line.h", "stencil.h", "tpf_internal.h")] + \
        [os.path.join(ROOT, "include", "tpf.h")]


@pytest.fixture(scope="module")
def harness():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    os.makedirs(BUILD, exist_ok=True)
    fresh = os.path.exists(EXE) and all(os.path.getmtime(EXE) > os.path.getmtime(f) for f in _sources())
    if not fresh:
        tmp = f"{EXE}.{os.getpid()}.tmp"  # parallel test workers each build, then rename atomically
        cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++20", "-Xclang", "-target-feature", "-Xclang",
               "-packed-fp32-ops", "-I", os.path.join(ROOT, "include"), "-I", CSRC,
               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fno-omit-frame-pointer", SRC, "-o", tmp]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr[-3000:]
        os.replace(tmp, EXE)
    return EXE


def run(exe, mode, values, tmp_path, nout):
    """Writes the flat list of float64 values, runs the harness, returns nout arrays of
    the sizes given (list of ints) from its output."""
    fin, fout = tmp_path / f"{mode}.in", tmp_path / f"{mode}.out"
    np.concatenate([np.atleast_1d(np.asarray(v, np.float64)).ravel() for v in values]).tofile(fin)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=0:halt_on_error=1")
    r = subprocess.run([exe, mode, str(fin), str(fout)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    data = np.fromfile(fout, np.float64)
    assert data.size == sum(nout), (data.size, nout)
    out, k = [], 0
    for n in nout:
        out.append(data[k:k + n])
        k += n
    return out


# ---------------------------------------------------------------------------------
def test_log_exp_within_stated_bound(harness, tmp_path):
    rng = np.random.default_rng(4)
    x = np.concatenate([10.0 ** rng.uniform(-300, 300, 4000), rng.uniform(1e-6, 1.0, 4000),
                        1.0 + rng.uniform(-1e-6, 1e-6, 500), 2.0 ** np.arange(-1000, 1000, 37.0),
                        np.array([0.70710678118654752, 0.7071067811865476, 1.4142135623730951, 2.0, 0.5])])
    y = np.concatenate([rng.uniform(-700, 700, 6000), rng.uniform(-1e-8, 1e-8, 500),
                        np.log(2.0) * (np.arange(-40, 40) + 0.5), rng.uniform(-30, 30, 2000)])
    n = min(x.size, y.size)
    x, y = x[:n], y[:n]
    lg, ex = run(harness, "math", [n, x, y], tmp_path, [n, n])
    decimal.getcontext().prec = 60
    worst_l = worst_e = 0.0
    for k in range(n):
        rl = decimal.Decimal(float(x[k])).ln()
        re = decimal.Decimal(float(y[k])).exp()
        if rl != 0:
            worst_l = max(worst_l, float(abs((decimal.Decimal(float(lg[k])) - rl) / rl)))
        worst_e = max(worst_e, float(abs((decimal.Decimal(float(ex[k])) - re) / re)))
    print(f"log_pos worst relative error {worst_l:.3e}, exp_fin {worst_e:.3e}")
    assert worst_l <= 4e-16 and worst_e <= 4e-16


# ---------------------------------------------------------------------------------
def stencil_to_csr(A, n, dim):
    A = np.asarray(A, np.float64)
    nx, ny, nz = n
    N = nx * ny * nz
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
    rows, cols, vals = [], [], []
    for o in range(A.shape[0]):
        dx, dy = o % 3 - 1, (o // 3) % 3 - 1
        dz = o // 9 - 1 if dim == 3 else 0
        jx, jy, jz = ix + dx, iy + dy, iz + dz
        ok = (jx >= 0) & (jx < nx) & (jy >= 0) & (jy < ny) & (jz >= 0) & (jz < nz)
        v = np.nonzero(ok)[0]
        j = (jx + nx * (jy + ny * jz))[ok]
        for e in range(4):
            rows.append(2 * v + e // 2)
            cols.append(2 * j + e % 2)
            vals.append(A[o, v, e])
        assert np.all(A[o, ~ok, :] == 0.0)  # out-of-grid neighbours stored as exact zeros
    return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(2 * N, 2 * N))


def csr_to_stencil(A, n, dim):
    nst = 27 if dim == 3 else 9
    nx, ny, nz = n
    N = nx * ny * nz
    out = np.zeros((nst, N, 4))
    A = A.tocoo()
    vi, vj = A.row // 2, A.col // 2
    e = 2 * (A.row % 2) + (A.col % 2)
    ix, iy, iz = vi % nx, (vi // nx) % ny, vi // (nx * ny)
    jx, jy, jz = vj % nx, (vj // nx) % ny, vj // (nx * ny)
    o = (jx - ix + 1) + 3 * (jy - iy + 1) + (9 * (jz - iz + 1) if dim == 3 else 0)
    np.add.at(out, (o, vi, e), A.data)
    return out


def row_rel(D, Ar):
    return max(abs(D[r::2]).max() / abs(Ar[r::2]).max() for r in (0, 1))


ASM_CASES = [
    ("lens17x9", lambda: W.lens_2d(17, 9), 50.0),
    ("cube9", lambda: W.small_cube(9, seed=22), 50.0),
    ("case5_9", lambda: W.case5(9), 2e4),
    ("case4_16x8", lambda: W.case4(16), 2e4),
]


@pytest.mark.parametrize("case", ASM_CASES, ids=[c[0] for c in ASM_CASES])
def test_assembly_rows_match_oracle(harness, tmp_path, case):
    name, mk, dp = case
    scn = mk()
    f = FV.FV(scn)
    u = W.perturbed_state(scn, 5, dp=dp, sn_lo=0.02, sn_hi=0.6)
    h = 32.0
    sx, sy, sz = scn.spacing
    kr = 1 if scn.kr_model == "poly" else 0
    vals = [scn.dim, *scn.n, sx, sy, sz, *scn.gravity, *scn.rho, *scn.mu, *scn.s_res, kr, *scn.kr_coef, 1.0 / h,
            scn.perm, scn.poro, scn.entry_p, scn.bc_lambda, f.pdmin, f.lam_ref, scn.dir_mask.astype(np.float64),
            f.Q, u]
    N, nst = scn.nverts, (27 if scn.dim == 3 else 9)
    sizes = [nst * N * 4, 2 * N, 2 * N, nst * N * 4, 2 * N] + ([nst * N * 4, 2 * N] if scn.dim == 3 else [])
    out = run(harness, "assemble", vals, tmp_path, sizes)
    Ar = f.stage_matrix(u, h)
    Fr = f.residual(u).ravel()
    Sr = f.storage_part(u, h)
    variants = [("inline", out[0], out[1]), ("corner pass", out[3], out[4])]
    if scn.dim == 3:
        variants.append(("split", out[5], out[6]))
    for label, A, F in variants:
        Ag = stencil_to_csr(A.reshape(nst, N, 4), scn.n, scn.dim)
        d = row_rel(abs(Ag - Ar).tocsr(), Ar)
        fe = max(np.abs(F[c::2] - Fr[c::2]).max() / np.abs(Fr[c::2]).max() for c in (0, 1))
        print(f"{name} {label}: matrix {d:.2e}, residual {fe:.2e}")
        assert d < 1e-11 and fe < 1e-11, (label, d, fe)
    mst = out[2].reshape(-1, 2)
    sw = np.asarray(Sr[2 * np.arange(N), 2 * np.arange(N) + 1]).ravel()
    sn = np.asarray(Sr[2 * np.arange(N) + 1, 2 * np.arange(N) + 1]).ravel()
    assert np.abs(mst[:, 0] - sw).max() <= 1e-12 * np.abs(sw).max() + 1e-300
    assert np.abs(mst[:, 1] - sn).max() <= 1e-12 * np.abs(sn).max() + 1e-300


RAP_CASES = [
    ("lens17x9", lambda: W.lens_2d(17, 9), 3, 50.0),
    ("cube9", lambda: W.small_cube(9, seed=22), 3, 50.0),
    ("cube5", lambda: W.small_cube(5, seed=21), 2, 50.0),   # the 5^3 two-level hierarchy
    ("case5_9", lambda: W.case5(9), 3, 2e4),
]


@pytest.mark.parametrize("case", RAP_CASES, ids=[c[0] for c in RAP_CASES])
def test_galerkin_product_coverage_and_values(harness, tmp_path, case):
    name, mk, levels, dp = case
    scn = mk()
    scn.levels = levels
    u = W.perturbed_state(scn, 5, dp=dp, sn_lo=0.02, sn_hi=0.6)
    st = ST.Stage(scn)
    st.assemble(u.ravel(), 32.0)
    H = st.H
    dim = scn.dim
    for l in range(levels - 1):
        nf, nc = H.sizes[l], H.sizes[l + 1]
        nf3 = tuple(nf) + (1,) * (3 - len(nf))
        nc3 = tuple(nc) + (1,) * (3 - len(nc))
        Nf, Nc = int(np.prod(nf3)), int(np.prod(nc3))
        Af = csr_to_stencil(H.A[l], nf3, dim)
        S = H.S[l].tocsr()
        mf = np.stack([np.asarray(S[2 * np.arange(Nf), 2 * np.arange(Nf) + 1]).ravel(),
                       np.asarray(S[2 * np.arange(Nf) + 1, 2 * np.arange(Nf) + 1]).ravel()], axis=1)
        mask = l == 0
        fmask = scn.dir_mask.astype(np.float64) if mask else np.zeros(Nf)
        nst = 27 if dim == 3 else 9
        vals = [dim, *nf3, *nc3, int(mask), scn.rho[0] / scn.rho[1], Af, mf, fmask]
        Ac, mc, cntB, cntA = run(harness, "rap", vals, tmp_path, [nst * Nc * 4, 2 * Nc, nst * Nf, nst * Nc])
        assert np.all(cntB == 1.0) and np.all(cntA == 1.0), (l, cntB.min(), cntB.max(), cntA.min(), cntA.max())
        Ag = stencil_to_csr(Ac.reshape(nst, Nc, 4), nc3, dim)
        d = row_rel(abs(Ag - H.A[l + 1]).tocsr(), H.A[l + 1])
        print(f"{name} level {l}->{l + 1}: coarse operator {d:.2e}")
        assert d < 1e-12, d
        Sc = H.S[l + 1].tocsr()
        np.testing.assert_allclose(mc.reshape(-1, 2)[:, 1], np.asarray(Sc[2 * np.arange(Nc) + 1,
                                                                           2 * np.arange(Nc) + 1]).ravel(),
                                   rtol=1e-12, atol=1e-300)


LINE_CASES = [
    ("lens9x5", lambda: W.lens_2d(9, 5), 3, 50.0),  # level 1: lines of 3 vertices
    ("lens17x9", lambda: W.lens_2d(17, 9), 3, 50.0),
    ("cube9", lambda: W.small_cube(9, seed=22), 3, 50.0),
    ("case4_64x32", lambda: W.case4(64), 3, 2e4),
    ("case5_9", lambda: W.case5(9), 3, 2e4),
]


@pytest.mark.parametrize("case", LINE_CASES, ids=[c[0] for c in LINE_CASES])
@pytest.mark.parametrize("single", [0, 1], ids=["fp64", "fp32"])
def test_line_smoother_bodies(harness, tmp_path, case, single):
    """The line LU and the per-line sweep over every line of every smoothed level
    (finest 9/27-point operators and Galerkin coarse levels), from a zero guess and in
    place on a residual, against the oracle's sparse LU of the line part:
    xo = xi + omega A_L^{-1} r, 1e-11 in FP64, 1e-4 in FP32 (factors and sweep in FP32)."""
    name, mk, levels, dp = case
    scn = mk()
    scn.levels = levels
    u = W.perturbed_state(scn, 5, dp=dp, sn_lo=0.02, sn_hi=0.6)
    st = ST.Stage(scn, smoother="line")
    st.assemble(u.ravel(), 32.0)
    H = st.H
    dim = scn.dim
    rng = np.random.default_rng(9)
    omega = 2.0 / 3.0
    for l in range(levels - 1):
        n3 = tuple(H.sizes[l]) + (1,) * (3 - len(H.sizes[l]))
        N = int(np.prod(n3))
        A = H.A[l]
        AL = G.line_part(A, n3, dim).tocsc()
        import scipy.sparse.linalg as ssl
        lu = ssl.splu(AL)
        r, xi = rng.standard_normal(2 * N), rng.standard_normal(2 * N)
        for first in (1, 0):
            vals = [dim, *n3, omega, first, single, csr_to_stencil(A, n3, dim), r, xi]
            xo, bad, lf = run(harness, "line", vals, tmp_path, [2 * N, 1, 12 * N])
            assert bad[0] == 0.0
            want = omega * lu.solve(r) + (0.0 if first else xi)
            err = max(np.abs(xo[c::2] - want[c::2]).max() / np.abs(want[c::2]).max() for c in (0, 1))
            print(f"{name} level {l} first={first} {'fp32' if single else 'fp64'}: {err:.2e}")
            assert err < (1e-4 if single else 1e-11), err
            # G_k is the inverse of the pivot block: G_k D'_k = I, D'_k = D_k - L_k W_{k-1}
            Gk = lf[:4 * N].reshape(N, 2, 2)
            assert np.all(np.isfinite(Gk))


def test_line_factor_reports_a_singular_pivot(harness, tmp_path):
    """A line whose pivot block is singular (a zero centre block with no couplings along
    the line) is counted, the way the library's factor kernel counts it before the
    next solve fails; the other lines are unaffected."""
    scn = W.lens_2d(9, 5)
    st = ST.Stage(scn, levels=2, smoother="line")
    u = W.perturbed_state(scn, 5, sn_lo=0.05, sn_hi=0.5)
    st.assemble(u.ravel(), 32.0)
    A = st.H.A[0].tolil()
    n3 = (9, 5, 1)
    v = 2 * 9 + 4  # line ix = 4, vertex iy = 2
    for r in (2 * v, 2 * v + 1):
        for c in list(A.rows[r]):
            if (c // 2) % 9 == v % 9:  # the vertex's own block and its line couplings
                A[r, c] = 0.0
    A = sp.csr_matrix(A)
    N = 45
    rng = np.random.default_rng(2)
    vals = [2, *n3, 2.0 / 3.0, 1, 0, csr_to_stencil(A, n3, 2), rng.standard_normal(2 * N), np.zeros(2 * N)]
    xo, bad, _ = run(harness, "line", vals, tmp_path, [2 * N, 1, 12 * N])
    assert bad[0] == 1.0
    ok_lines = [ix for ix in range(9) if ix != 4]
    assert all(np.isfinite(xo.reshape(5, 9, 2)[:, ix, :]).all() for ix in ok_lines)
