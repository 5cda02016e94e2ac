"""Pins of the FP64 oracle against what the paper prints and what mathematics fixes.

None of these tests re-types an oracle formula: each compares the oracle with a
printed value (tests/golden/paper_values.json), a closed form, a conservation law or
an independent library routine."""
import json
import os

import numpy as np
import pytest
import scipy.linalg as sla
import scipy.optimize as so
import scipy.sparse as sp

import workloads as W
from oracle import fv as FV
from oracle import gmg as G
from oracle import krylov as KR
from oracle import limex as LX
from oracle import stage as ST

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def make_scn(dim, n, extent, perm=1e-11, poro=0.3, pd=1000.0, lam=2.0, gravity=(0, 0, 0),
             rho=(1000.0, 1000.0), mu=(1e-3, 1e-3), s_res=(0.0, 0.0), u=None, levels=1):
    scn = W._empty("pin", dim, n, extent, gravity)
    scn.rho, scn.mu, scn.s_res = tuple(rho), tuple(mu), tuple(s_res)
    nc = scn.ncells
    scn.perm = np.broadcast_to(np.asarray(perm, float), (nc,)).copy()
    scn.poro = np.broadcast_to(np.asarray(poro, float), (nc,)).copy()
    scn.entry_p = np.broadcast_to(np.asarray(pd, float), (nc,)).copy()
    scn.bc_lambda = np.broadcast_to(np.asarray(lam, float), (nc,)).copy()
    if u is not None:
        scn.u0 = u
    scn.levels = levels
    return scn


# ---------------------------------------------------------------------------------
# Constitutive laws and the interface condition, pinned by printed numbers.
# ---------------------------------------------------------------------------------
def test_buckley_leverett_front_speed_matches_paper():
    """Welge tangent construction with the oracle's Burdine k_r (lambda = 2, p_c = 0)
    reproduces the front speed printed for Case-1."""
    g = GOLD["bl_front_speed"]
    p = g["params"]

    def fw(sw):
        sn = 1.0 - sw
        kw = FV.krw_bc(sn, p["lambda"], p["swr"], p["snr"]) / p["mu_w"]
        kn = FV.krn_bc(sn, p["lambda"], p["swr"], p["snr"]) / p["mu_n"]
        return kw / (kw + kn)

    def dfw(sw, h=1e-7):
        return (fw(sw + h) - fw(sw - h)) / (2 * h)

    # tangent from the initial state S_w = 0: f'(S_f) = f(S_f) / S_f
    sf = so.brentq(lambda s: dfw(s) - fw(s) / s, 0.3, 0.99)
    u_total = p["mass_flux"] / p["rho_w"]
    v = u_total / p["phi"] * dfw(sf)
    assert abs(v - g["value"]) / g["value"] < 0.5e-2
    assert round(v, 8) == pytest.approx(g["value"], rel=5e-3)


def test_barrier_threshold_matches_paper():
    """The case-2/case-3 switch of the hat saturation for a vertex on the interface
    of Case-4 layers 2 and 3 sits at the printed S_w* = 0.7778."""
    g = GOLD["barrier_threshold"]
    p = g["params"]
    pd2 = p["pd_coef"] * p["K2"] ** p["pd_exp"]
    pd3 = p["pd_coef"] * p["K3"] ** p["pd_exp"]
    assert pd3 > pd2
    swr, snr, lam = p["swr"], p["snr"], p["lambda"]

    def is_barrier(sw):
        sn = np.array([1.0 - sw])
        sh = FV.hat_sn(sn, pd2, lam, np.array([pd3]), lam, swr, snr)
        return sh[0] == snr

    lo, hi = 0.5, 0.9  # barrier below lo? no: high S_w (low p_c) is a barrier
    assert is_barrier(hi) and not is_barrier(lo)
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        if is_barrier(mid):
            hi = mid
        else:
            lo = mid
    assert round(hi, 4) == pytest.approx(g["value"], abs=1e-4)


def test_hat_cases_and_continuity():
    swr, snr, lam = 0.2, 0.1, 2.0
    sn = np.linspace(0.0, 0.69, 500)
    # case 1: the reference medium returns the vertex saturation
    np.testing.assert_array_equal(FV.hat_sn(sn, 1000.0, lam, 1000.0, lam, swr, snr), sn)
    # continuity of S^ across the case-2/case-3 boundary as p_d,e approaches P_i from below
    pdmin = 1000.0
    for s in (0.2, 0.4, 0.6):
        P = FV.pc_bc(np.array([s]), pdmin, lam, swr, snr)[0]
        below = FV.hat_sn(np.array([s]), pdmin, lam, np.array([P * (1 - 1e-9)]), lam, swr, snr)[0]
        at = FV.hat_sn(np.array([s]), pdmin, lam, np.array([P]), lam, swr, snr)[0]
        assert at == snr
        assert abs(below - snr) < 1e-7
    # case 3 preserves the capillary pressure: p_c,e(S^) = P_i
    pde = 1300.0
    s = np.array([0.5])
    sh = FV.hat_sn(s, pdmin, lam, np.array([pde]), lam, swr, snr)
    assert FV.pc_bc(sh, pde, lam, swr, snr)[0] == pytest.approx(FV.pc_bc(s, pdmin, lam, swr, snr)[0],
                                                               rel=1e-13)


def test_dof_counts_two_unknowns_per_vertex():
    for dim, cells, dof in GOLD["dof_counts"]["rows"]:
        assert 2 * int(np.prod([c + 1 for c in cells])) == dof


# ---------------------------------------------------------------------------------
# Discretisation: exactness, equilibrium and conservation.
# ---------------------------------------------------------------------------------
@pytest.mark.parametrize("dim", [2, 3])
def test_linear_pressure_single_phase_exact(dim):
    n = (9, 5, 1) if dim == 2 else (7, 5, 4)
    ext = (2.0, 1.0, 1.0) if dim == 2 else (1.2, 0.8, 0.6)
    scn = make_scn(dim, n, ext, perm=3e-11, pd=500.0)
    x, y, z = scn.vertex_coords()
    a = 250.0
    u = np.stack([1e5 + a * x, np.zeros_like(x)], axis=1)
    f = FV.FV(scn)
    F = f.residual_raw(u)
    scale = 1000.0 * 3e-11 / 1e-3 * a * np.prod(ext[1:dim])
    interior = (x > 1e-12) & (x < ext[0] - 1e-12)
    assert np.max(np.abs(F[interior])) < 1e-11 * scale
    # total inflow through x = 0 equals Darcy's law times the cross-section
    left = np.isclose(x, 0.0)
    assert F[left, 0].sum() == pytest.approx(1000.0 * 3e-11 * a / 1e-3 * np.prod(ext[1:dim]), rel=1e-12)
    assert np.max(np.abs(F[:, 1])) < 1e-14 * scale


@pytest.mark.parametrize("dim", [2, 3])
def test_hydrostatic_equilibrium(dim):
    n = (6, 7, 1) if dim == 2 else (5, 4, 6)
    ext = (1.0, 2.0, 1.0) if dim == 2 else (1.0, 1.0, 2.0)
    gvec = [0.0, 0.0, 0.0]
    gvec[dim - 1] = -9.81
    rng = np.random.default_rng(0)
    scn = make_scn(dim, n, ext, perm=np.exp(-25 + rng.standard_normal(W._empty("t", dim, n, ext, gvec).ncells)),
                   gravity=gvec, rho=(1000.0, 1000.0))
    coords = scn.vertex_coords()
    zz = coords[dim - 1]
    H = ext[dim - 1]
    p = 1e5 + 1000.0 * 9.81 * (H - zz)
    # single phase
    u = np.stack([p, np.zeros_like(p)], axis=1)
    F = FV.FV(scn).residual_raw(u)
    assert np.max(np.abs(F)) < 1e-10 * 1000.0 * np.exp(-25) / 1e-3 * 1000 * 9.81
    # equal densities, uniform S_n in one medium: both phases at rest
    scn2 = make_scn(dim, n, ext, perm=1e-11, gravity=gvec, rho=(1000.0, 1000.0))
    u2 = np.stack([p, np.full_like(p, 0.3)], axis=1)
    F2 = FV.FV(scn2).residual_raw(u2)
    assert np.max(np.abs(F2)) < 1e-9 * 1000.0 * 1e-11 / 1e-3 * 1000 * 9.81


@pytest.mark.parametrize("dim", [2, 3])
def test_discrete_conservation(dim):
    scn = W.lens_2d(17, 9) if dim == 2 else W.small_cube(7, sigma=1.5, seed=3)
    u = W.perturbed_state(scn, 7)
    f = FV.FV(scn)
    Fr = f.residual_raw(u)
    flux_scale = np.abs(f.flux_divergence(u)).sum(axis=0)
    for ph in range(2):
        assert abs(Fr[:, ph].sum() - f.Q[:, ph].sum()) <= 1e-12 * max(flux_scale[ph], f.Q[:, ph].sum(), 1e-300)
    # column sums of the flux Jacobian vanish
    J = f.jacobian(u, which="residual")
    keep = np.ones(2 * f.N)
    keep[f.dirichlet_dofs()] = 0
    Jr = sp.csr_matrix(J)
    # rebuild without Dirichlet clearing: J_raw = dF_raw/du via complex step of the raw residual
    fr = FV.FV(scn)
    fr.dir_mask = np.zeros_like(fr.dir_mask)
    Jraw = fr.jacobian(u)
    colsum = np.asarray(Jraw.sum(axis=0)).ravel()
    assert np.max(np.abs(colsum)) < 1e-12 * np.max(np.abs(Jraw).sum(axis=0))
    assert Jr.shape == Jraw.shape


def test_storage_total_mass_and_mass_matrix():
    scn = make_scn(3, (5, 4, 3), (1.0, 0.6, 0.4), poro=0.25, rho=(1000.0, 1460.0))
    f = FV.FV(scn)
    u = np.stack([np.full(scn.nverts, 1e5), np.full(scn.nverts, 0.35)], axis=1)
    m = f.storage(u)
    vol = 1.0 * 0.6 * 0.4
    assert m[:, 1].sum() == pytest.approx(0.25 * 1460.0 * 0.35 * vol, rel=1e-13)
    assert m[:, 0].sum() == pytest.approx(0.25 * 1000.0 * 0.65 * vol, rel=1e-13)
    M = f.mass_matrix(u).toarray()
    assert np.all(M[:, 0::2] == 0.0)
    # dm_n/dS_n = Phi rho_n |b_i| in one medium (case 1 everywhere)
    dual = LX.Norms(f).dual
    np.testing.assert_allclose(np.diag(M)[1::2], 0.25 * 1460.0 * dual, rtol=1e-13)


def _row_1d(n, ext):
    return make_scn(2, (n, 3, 1), (ext, 0.2, 1.0))


def test_capillary_flux_reduces_to_two_point_form():
    """S_n varying along x only, uniform p_w, no gravity: the non-wetting balance of an
    interior vertex is the textbook two-point capillary diffusion."""
    n, L = 9, 0.8
    scn = make_scn(2, (n, 3, 1), (L, 0.2, 1.0), perm=2e-11, pd=1500.0, lam=2.5, mu=(1e-3, 9e-4),
                   rho=(1000.0, 1460.0))
    x, y, _ = scn.vertex_coords()
    sn = 0.1 + 0.5 * (x / L) ** 2
    u = np.stack([np.full_like(x, 1e5), sn], axis=1)
    F = FV.FV(scn).residual_raw(u)
    dx = L / (n - 1)
    dy = 0.1

    def face(s0, s1):
        pc0 = 1500.0 * (1 - s0) ** (-1 / 2.5)
        pc1 = 1500.0 * (1 - s1) ** (-1 / 2.5)
        sm = 0.5 * (s0 + s1)
        se = 1 - sm
        krn = (1 - se) ** 2 * (1 - se ** ((2 + 2.5) / 2.5))
        return -1460.0 * krn * 2e-11 / 9e-4 * (pc1 - pc0) / dx * dy

    for i in range(1, n - 1):
        v = i + n * 1  # middle row: full dual face of height dy
        s_m, s_0, s_p = sn[v - 1], sn[v], sn[v + 1]
        expect = -(face(s_0, s_p) - face(s_m, s_0))
        assert F[v, 1] == pytest.approx(expect, rel=1e-12)
        assert abs(F[v, 0]) < 1e-25


def test_upwind_convective_flux_two_point_form():
    """Linear p_w along x, p_c = 0, S_n varying along x: each interior balance is the
    difference of fully upwinded two-point fluxes (upwind = the side the flow comes from)."""
    n, L = 9, 0.8
    a = -400.0  # pressure falls along +x: flow along +x, upwind = left vertex
    scn = make_scn(2, (n, 3, 1), (L, 0.2, 1.0), perm=2e-11, pd=0.0, lam=2.0, mu=(1e-3, 5e-3))
    x, y, _ = scn.vertex_coords()
    sn = 0.2 + 0.5 * np.sin(3 * x) ** 2
    u = np.stack([1e5 + a * x, sn], axis=1)
    F = FV.FV(scn).residual_raw(u)
    dy = 0.1
    qw = -2e-11 / 1e-3 * a * dy
    qn = -2e-11 / 5e-3 * a * dy
    for i in range(1, n - 1):
        v = i + n
        se_l, se_c = 1 - sn[v - 1], 1 - sn[v]
        fw_in, fw_out = 1000 * se_l ** 4 * qw, 1000 * se_c ** 4 * qw
        fn_in = 1000 * (1 - se_l) ** 2 * (1 - se_l ** 2) * qn
        fn_out = 1000 * (1 - se_c) ** 2 * (1 - se_c ** 2) * qn
        assert F[v, 0] == pytest.approx(fw_in - fw_out, rel=1e-12)
        assert F[v, 1] == pytest.approx(fn_in - fn_out, rel=1e-12)


def test_upwind_convective_flux_two_point_form_polynomial_law():
    """As above with the printed polynomial laws of Tables case4/case5 (k_rw = 0.9 S_e^2,
    k_rn = 0.5 (1 - S_e)) and residual saturations S_wr = 0.2, S_nr = 0.1."""
    n, L = 9, 0.8
    a = -400.0
    scn = make_scn(2, (n, 3, 1), (L, 0.2, 1.0), perm=2e-11, pd=0.0, lam=2.0, mu=(1e-3, 5e-3),
                   s_res=(0.2, 0.1))
    scn.kr_model, scn.kr_coef = "poly", (0.9, 0.5)
    x, y, _ = scn.vertex_coords()
    sn = 0.15 + 0.5 * np.sin(3 * x) ** 2
    u = np.stack([1e5 + a * x, sn], axis=1)
    F = FV.FV(scn).residual_raw(u)
    dy = 0.1
    qw = -2e-11 / 1e-3 * a * dy
    qn = -2e-11 / 5e-3 * a * dy
    for i in range(1, n - 1):
        v = i + n
        se_l, se_c = (1 - sn[v - 1] - 0.2) / 0.7, (1 - sn[v] - 0.2) / 0.7
        assert F[v, 0] == pytest.approx(1000 * 0.9 * (se_l ** 2 - se_c ** 2) * qw, rel=1e-12)
        assert F[v, 1] == pytest.approx(1000 * 0.5 * (se_c - se_l) * qn, rel=1e-12)


def test_point_source_enters_one_control_volume():
    """Case 5's injection: 0.05 pore volumes per year of the non-wetting phase, into the
    control volume whose dual box holds (100, 100, 30) m."""
    scn = W.case5(17)
    f = FV.FV(scn)
    rate = 0.05 * 200.0 ** 3 * 0.1 / (365 * 86400.0) * 700.0
    assert f.Q[:, 1].sum() == pytest.approx(rate, rel=1e-14) and f.Q[:, 0].sum() == 0.0
    v = int(np.argmax(f.Q[:, 1]))
    x, y, z = scn.vertex_coords()
    h = 200.0 / 16
    assert all(abs(c - p) <= h / 2 for c, p in zip((x[v], y[v], z[v]), (100.0, 100.0, 30.0)))
    # the initial state is in equilibrium away from the source: the residual vanishes
    # to rounding of the hydrostatic pressure differences
    F = f.residual(scn.u0)
    F[v] = 0.0
    assert np.abs(F).max() <= 1e-12 * rate


def test_neumann_patch_total():
    scn = W.small_cube(9)
    f = FV.FV(scn)
    assert f.Q[:, 1].sum() == pytest.approx(0.075 * 0.2 * 0.2, rel=1e-13)
    assert f.Q[:, 0].sum() == 0.0
    scn2 = W.lens_2d()
    f2 = FV.FV(scn2)
    assert f2.Q[:, 1].sum() == pytest.approx(0.075 * 0.2, rel=1e-13)


@pytest.mark.parametrize("dim", [2, 3, "case5", "case4"])
def test_jacobian_complex_step_vs_central_differences(dim):
    if dim in ("case5", "case4"):  # polynomial laws, residual saturations, layered p_d(K), point source
        scn = W.case5(5) if dim == "case5" else W.case4(16)
        u = W.perturbed_state(scn, 3, dp=2e4, sn_lo=0.12, sn_hi=0.6)
    else:
        scn = W.lens_2d(9, 5) if dim == 2 else W.small_cube(4, sigma=1.0, seed=5)
        u = W.perturbed_state(scn, 3, sn_lo=0.05, sn_hi=0.5)
    f = FV.FV(scn)
    J = f.jacobian(u).toarray()
    uf = u.ravel()
    rng = np.random.default_rng(1)
    cols = rng.choice(2 * f.N, size=min(24, 2 * f.N), replace=False)
    # S_n columns: second-order one-sided differences towards larger S_n, because the
    # Dirichlet vertices sit at S_n = 0, i.e. exactly on the S_e = 1 clamp, where the
    # derivative is the analytic (S_e <= 1) one-sided derivative.
    cols = np.concatenate([cols, 2 * np.nonzero(f.dir_mask)[0][:4] + 1])
    fmax = np.max(np.abs(f.residual(u)))
    for c in cols:
        hstep = 1e-2 if c % 2 == 0 else 1e-6

        def Fat(delta):
            uu = uf.copy()
            uu[c] += delta
            return f.residual(uu.reshape(-1, 2)).ravel()

        if c % 2 == 0:
            fd = (Fat(hstep) - Fat(-hstep)) / (2 * hstep)
        else:
            fd = (-3 * Fat(0.0) + 4 * Fat(hstep) - Fat(2 * hstep)) / (2 * hstep)
        scale = np.max(np.abs(J[:, c])) + 1e-300
        noise = 8 * np.finfo(float).eps * fmax / hstep
        assert np.max(np.abs(fd - J[:, c])) <= 1e-5 * scale + noise


# ---------------------------------------------------------------------------------
# Multigrid, Krylov and dense-LU checks.
# ---------------------------------------------------------------------------------
def test_prolongation_reproduces_linear_functions():
    n = (9, 5, 5)
    P = G.prolongation(n, 3)
    sizes = G.level_sizes(n, 3, 2)
    nc = sizes[1]
    zc, yc, xc = np.meshgrid(np.arange(nc[2]) * 2.0, np.arange(nc[1]) * 2.0, np.arange(nc[0]) * 2.0,
                             indexing="ij")
    zf, yf, xf = np.meshgrid(np.arange(n[2]) * 1.0, np.arange(n[1]) * 1.0, np.arange(n[0]) * 1.0,
                             indexing="ij")
    # pressure: (tri)linear interpolation reproduces linear functions; saturation:
    # aggregation reproduces constants and maps fine vertex i to coarse (i + 1) // 2
    lin_c = np.stack([3 * xc - yc + 2 * zc + 1, np.full_like(xc, 7.0)], axis=-1).ravel()
    lin_f = np.stack([3 * xf - yf + 2 * zf + 1, np.full_like(xf, 7.0)], axis=-1).ravel()
    np.testing.assert_allclose(P @ lin_c, lin_f, rtol=0, atol=1e-13)
    PS = P[1::2, 1::2]
    assert np.all(np.asarray(PS.sum(axis=1)).ravel() == 1.0)
    assert PS.sum() == np.prod(n)


def test_galerkin_and_two_grid_contraction():
    scn = W.lens_2d(17, 9)
    st = ST.Stage(scn, levels=2)
    u = W.perturbed_state(scn, 2, sn_lo=0.05, sn_hi=0.3)
    A = st.assemble(u.ravel(), 32.0)
    H = st.H
    P = H.P[0].toarray()
    S0 = H.S[0].toarray()
    # the row transform of the finest level, built here from its definition: the
    # wetting row of each vertex without Dirichlet components gains rho_w/rho_n times
    # the non-wetting row
    T = np.eye(A.shape[0])
    for v in np.nonzero(scn.dir_mask == 0)[0]:
        T[2 * v, 2 * v + 1] = scn.rho[0] / scn.rho[1]
    np.testing.assert_array_equal(H.T0.toarray(), T)
    # flux part: exact Galerkin product of the fine flux part, plus a unit diagonal on
    # coarse unknowns whose prolongation column is empty (all-Dirichlet aggregates)
    empty = np.abs(P).sum(axis=0) == 0
    assert empty.sum() > 0 and np.all(np.nonzero(empty)[0] % 2 == 1)
    np.testing.assert_allclose((H.A[1] - H.S[1]).toarray(), P.T @ T @ (A.toarray() - S0) @ P + np.diag(empty * 1.0),
                               rtol=0, atol=1e-12 * np.abs(A).max())
    S0 = T @ S0
    # lumped coarse storage: diagonal blocks, S_n column only, total storage conserved
    Sc = H.S[1].toarray()
    off = Sc.copy()
    for i in range(0, Sc.shape[0], 2):
        off[i:i + 2, i + 1] = 0.0
    assert np.all(off == 0.0)
    keep_cols = np.abs(P).sum(axis=1) > 0
    assert Sc.sum() == pytest.approx(S0[keep_cols][:, keep_cols].sum(), rel=1e-12)
    # two-grid iteration with exact coarse solve contracts the error
    xs = np.random.default_rng(0).standard_normal(A.shape[0])
    b = A @ xs
    x = np.zeros_like(b)
    errs = []
    for _ in range(10):
        x = x + H.vcycle(b - A @ x)
        errs.append(np.linalg.norm(x - xs))
    assert all(errs[i + 1] < errs[i] for i in range(9))
    assert errs[-1] < 1e-2 * errs[0]


@pytest.mark.parametrize("case", ["2d9x5", "2d9x9", "3d5"])
def test_bicgstab_gmg_matches_dense_lu(case):
    if case == "2d9x5":
        scn = W.lens_2d(9, 5); scn.levels = 2
    elif case == "2d9x9":
        scn = W.lens_2d(9, 9); scn.levels = 3
    else:
        scn = W.small_cube(5, seed=9); scn.levels = 2
    u = W.perturbed_state(scn, 4, sn_lo=0.05, sn_hi=0.4)
    st = ST.Stage(scn)
    A = st.assemble(u.ravel(), 10.0)
    F = st.residual(u.ravel())
    x, info = st.solve(F, rtol=1e-13, maxit=200)
    xd = np.linalg.solve(A.toarray(), F)
    for c in range(2):
        ref = xd[c::2]
        assert np.linalg.norm(x[c::2] - ref) <= 1e-10 * np.linalg.norm(ref)
    assert info["rel_res_true"] < 1e-12


def test_bicgstab_on_nonsymmetric_matrix_vs_lu():
    rng = np.random.default_rng(3)
    n = 60
    A = np.eye(n) * 4 + rng.standard_normal((n, n)) * 0.3
    b = rng.standard_normal(n)
    x, info = KR.bicgstab(A, b, lambda v: v, rtol=1e-14, maxit=400)
    np.testing.assert_allclose(x, sla.lu_solve(sla.lu_factor(A), b), rtol=1e-11, atol=1e-12)


# ---------------------------------------------------------------------------------
# LIMEX: closed forms on the scalar test equation, observed order, norms.
# ---------------------------------------------------------------------------------
def _scalar_limex(lam, H, k):
    return LX.limex_step(np.array([1.0]), H, k, lambda v: lam * v,
                         lambda h: (lambda f: f / (1.0 / h - lam)),
                         lambda a, b: float(abs(a - b)[0] / abs(a)[0]), 1e9, 1.0, 1e9)


def test_limex_scalar_closed_forms():
    lam, H = -3.0, 0.2
    out, acc, eps, dtn, kk = _scalar_limex(lam, H, 2)
    T11 = 1.0 / (1.0 - H * lam)
    T21 = (1.0 - H * lam / 2.0) ** -2
    assert kk[0] == pytest.approx(2 * T21 - T11, rel=1e-15)
    out3 = _scalar_limex(lam, H, 3)[4]
    T31 = (1.0 - H * lam / 3.0) ** -3
    T32 = T31 + (T31 - T21) / (3.0 / 2.0 - 1.0)
    T22 = 2 * T21 - T11
    T33 = T32 + (T32 - T22) / (3.0 - 1.0)
    assert out3[0] == pytest.approx(T33, rel=1e-14)


@pytest.mark.parametrize("k,order", [(2, 2), (3, 3)])
def test_limex_observed_order(k, order):
    lam = -2.0
    errs = []
    for H in (0.025, 0.0125, 0.00625):
        kk = _scalar_limex(lam, H, k)[4][0]
        errs.append(abs(kk - np.exp(lam * H)))
    rates = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    # local error of an order-k extrapolated linearly implicit Euler is O(H^(k+1))
    assert min(rates) > order + 0.75


def test_failed_stage_solve_rejects_the_step():
    """A stage solve that cannot reach rtol within maxit (forced: one iteration to
    1e-12) rejects the step: state returned unchanged, eps = inf, a quarter step next."""
    scn = W.lens_2d(17, 9)
    scn.levels = 2
    st = ST.Stage(scn)
    u = scn.u0.ravel().copy()
    out, info = st.limex_step(u, 32.0, stages=2, rtol=1e-12, maxit=1)
    assert not info["accepted"] and info["eps"] == float("inf")
    assert info["dt_next"] == 8.0 and info["solves"] == 1
    np.testing.assert_array_equal(out, u)


def test_step_size_rule_by_hand():
    assert LX.step_size(10.0, 0.001, 5e-3, 0.75, 1e9) == pytest.approx(10.0 * (3.75) ** (1 / 3), rel=1e-15)
    assert LX.step_size(10.0, 0.0, 5e-3, 0.75, 100.0) == 100.0


def test_norms_closed_forms():
    scn = make_scn(3, (5, 4, 6), (1.0, 0.5, 2.0))
    f = FV.FV(scn)
    nm = LX.Norms(f)
    x, y, z = scn.vertex_coords()
    assert nm.grad_sq(2 * x - 3 * y + 0.5 * z) == pytest.approx((4 + 9 + 0.25) * 1.0, rel=1e-13)
    # bilinear p = x*y on [0,1]x[0,0.5]x[0,2]: int (y^2 + x^2) = 2*(1/24 + 1/6)
    assert nm.grad_sq(x * y) == pytest.approx(2.0 * (0.5 ** 3 / 3 + 0.5 / 3), rel=1e-13)
    assert nm.sat_sq(np.full(scn.nverts, 0.7)) == pytest.approx(0.49 * 1.0, rel=1e-13)


def test_random_field_statistics():
    g = W.gaussian_field((64, 64, 64), 8.0, 1.5, seed=1)
    assert abs(g.var() / 1.5 ** 2 - 1) < 0.25
    c8 = np.mean(g[:, :, :-8] * g[:, :, 8:])
    assert abs(c8 / (1.5 ** 2 * np.exp(-1.0)) - 1) < 0.35
    g2 = W.gaussian_field((64, 64, 64), 8.0, 1.5, seed=1)
    np.testing.assert_array_equal(g, g2)


@pytest.mark.parametrize("dim", [2, 3])
def test_integration_point_exact_for_bilinear_pressure(dim):
    """For p = x*y the normal derivative is linear along each SCVF, so the midpoint
    (barycentre) rule is exact: the corner vertex balance equals the exact integral
    of the Darcy flux over its two (three) interior faces."""
    n = (5, 4, 1) if dim == 2 else (5, 4, 3)
    ext = (1.0, 0.6, 1.0) if dim == 2 else (1.0, 0.6, 0.5)
    scn = make_scn(dim, n, ext, perm=2e-11, pd=300.0)
    x, y, z = scn.vertex_coords()
    u = np.stack([1e5 + 1e3 * x * y, np.zeros_like(x)], axis=1)
    F = FV.FV(scn).residual_raw(u)
    dx, dy, dz = scn.spacing
    depth = dz / 2 if dim == 3 else 1.0
    # inflow into b_0 = K/mu rho * (int_{x-face} dp/dx + int_{y-face} dp/dy); z-face: dp/dz = 0
    expect = 1000.0 * 2e-11 / 1e-3 * 1e3 * (dy ** 2 / 8 + dx ** 2 / 8) * depth
    assert F[0, 0] == pytest.approx(expect, rel=1e-12)


def test_volume_balance_has_no_storage_and_leaves_block_jacobi_unchanged():
    """The transformed wetting row is rho_w times the pore-volume balance: its storage
    part vanishes for incompressible phases (to rounding), on every cell of a
    heterogeneous interface case.  A block-diagonal row transform T leaves damped
    block Jacobi unchanged, (TD)^{-1}(Tb - TAx) = D^{-1}(b - Ax), which is why the
    finest level may be smoothed with A itself."""
    scn = W.lens_2d(17, 9)
    scn.rho = (1000.0, 1460.0)
    st = ST.Stage(scn, levels=2)
    u = W.perturbed_state(scn, 5, sn_lo=0.05, sn_hi=0.5)
    A = st.assemble(u.ravel(), 32.0)
    T = st.H.T0
    S0 = st.fv.storage_part(u, 32.0)
    TS = (T @ S0).toarray()
    free = np.nonzero(scn.dir_mask == 0)[0]
    assert np.abs(TS[2 * free]).max() <= 1e-15 * np.abs(S0).max()
    np.testing.assert_array_equal(TS[1::2], S0.toarray()[1::2])
    assert np.abs(S0.toarray()[2 * free]).max() > 0.0
    rng = np.random.default_rng(1)
    x0, b = rng.standard_normal(A.shape[0]), rng.standard_normal(A.shape[0])
    Ht = G.Hierarchy(T @ A, scn.n, scn.dim, 1, scn.dir_mask)
    H1 = G.Hierarchy(A, scn.n, scn.dim, 1, scn.dir_mask)
    xa = Ht.smooth(0, x0, T @ b, 3)
    xb = H1.smooth(0, x0, b, 3)
    assert np.linalg.norm(xa - xb) <= 1e-12 * np.linalg.norm(xb)


def test_coarse_operators_regular_when_the_wetting_phase_is_immobile():
    """Case 1 of Section 5 at its initial state: ahead of the front S_w = 0, so only
    the non-wetting equation holds the pressure.  With the mass balances restricted as
    they stand, the aggregation restriction of that equation leaves the coarse
    operators singular; in volume-balance form they are regular, and GMG-BiCGSTAB
    reproduces the sparse direct solution."""
    import scipy.sparse.linalg as ssl
    scn = W.buckley_leverett(32)
    st = ST.Stage(scn)
    u = scn.u0.ravel()
    A = st.assemble(u, 1.0)
    f = st.residual(u)
    plain = G.Hierarchy(A, scn.n, scn.dim, st.levels, scn.dir_mask, S0=st.fv.storage_part(scn.u0, 1.0))
    assert np.linalg.cond(plain.A[-1].toarray()) > 1e14
    assert np.linalg.cond(st.H.A[-1].toarray()) < 1e10
    x, info = st.solve(f, rtol=1e-12, maxit=50)
    xd = ssl.spsolve(A.tocsc(), f)
    assert info["iters"] <= 10
    for c in range(2):
        assert np.linalg.norm(x[c::2] - xd[c::2]) <= 1e-9 * np.linalg.norm(xd[c::2])


def test_vcycle_is_a_contraction_on_a_heterogeneous_cube():
    """sigma_lnK = 2 on 33^3: the V(2,2) block-Jacobi cycle with lumped coarse storage
    is a convergent stationary iteration (the plain Galerkin product is not: its
    coarse storage blocks push the Jacobi spectrum past 2/omega)."""
    scn = W.cube_3d(33, 2.0, 3, levels=4)
    st = ST.Stage(scn)
    A = st.assemble(scn.u0.ravel(), 32.0)
    xs = np.random.default_rng(0).standard_normal(A.shape[0])
    b = A @ xs
    x = np.zeros_like(b)
    res = []
    for _ in range(6):
        x = x + st.H.vcycle(b - A @ x)
        res.append(np.linalg.norm(b - A @ x) / np.linalg.norm(b))
    assert all(res[i + 1] < res[i] for i in range(5))
    assert res[-1] < 1e-7


# ---------------------------------------------------------------------------------
# p_dmin and the reference medium (Section 3.3, Eq. pdmin), worked out by hand.
# ---------------------------------------------------------------------------------
def test_pdmin_and_reference_medium_by_hand_2d():
    """A 4 x 3-vertex grid of 3 x 2 cells (cell c = cx + 3 cy) with two media meeting
    at an equal entry pressure.  Expected p_dmin,i and m(i) for every vertex are written
    out from the cells around it (lowest cell index on a tie, reading R4): corner,
    edge and interior vertices, the lens-like high-p_d cells and the tie between
    cells 0 (lambda 2.5) and 1 (lambda 2.0)."""
    pd = [800.0, 800.0, 1500.0, 1500.0, 2000.0, 1200.0]
    lam = [2.5, 2.0, 2.0, 2.0, 3.0, 1.5]
    scn = make_scn(2, (4, 3, 1), (3.0, 2.0, 1.0), pd=pd, lam=lam)
    f = FV.FV(scn)
    # vertex v = ix + 4 iy: its cells, their minimum and the lowest minimiser
    want_pdmin = [800, 800, 800, 1500,    # iy = 0: {c0} {c0,c1} {c1,c2} {c2}
                  800, 800, 800, 1200,    # iy = 1: {c0,c3} {c0,c1,c3,c4} {c1,c2,c4,c5} {c2,c5}
                  1500, 1500, 1200, 1200]  # iy = 2: {c3} {c3,c4} {c4,c5} {c5}
    want_mref = [0, 0, 1, 2,
                 0, 0, 1, 5,
                 3, 3, 5, 5]
    np.testing.assert_array_equal(f.pdmin, np.array(want_pdmin, float))
    np.testing.assert_array_equal(f.mref, np.array(want_mref))
    np.testing.assert_array_equal(f.lam_ref, np.array(lam)[want_mref])
    # the tie at vertex 1 and 5 resolves to lambda 2.5 (cell 0), not 2.0 (cell 1)
    assert f.lam_ref[1] == 2.5 and f.lam_ref[5] == 2.5


def test_pdmin_and_reference_medium_by_hand_3d():
    """A 3^3-vertex grid of 2^3 cells (c = cx + 2 cy + 4 cz).  Vertices on each face
    centre, edge and the centre touch different cell sets, so a slip in the
    vertex-to-cell mapping of any axis moves one of these minima."""
    pd = [900.0, 700.0, 700.0, 1000.0, 1100.0, 650.0, 600.0, 1300.0]
    lam = [2.0, 2.0, 3.0, 2.0, 2.0, 4.0, 1.5, 2.0]
    scn = make_scn(3, (3, 3, 3), (1.0, 1.0, 1.0), pd=pd, lam=lam)
    f = FV.FV(scn)

    def v(ix, iy, iz):
        return ix + 3 * (iy + 3 * iz)
    cases = {  # vertex: (p_dmin, m) from the cells touching it
        (0, 0, 0): (900, 0),     # {c0}
        (2, 2, 2): (1300, 7),    # {c7}
        (1, 0, 0): (700, 1),     # {c0, c1}
        (1, 1, 0): (700, 1),     # {c0..c3}: tie c1 (lambda 2) / c2 (lambda 3) -> c1
        (1, 1, 1): (600, 6),     # all eight
        (0, 1, 1): (600, 6),     # x face: {c0, c2, c4, c6}
        (2, 1, 1): (650, 5),     # x face: {c1, c3, c5, c7}
        (1, 0, 1): (650, 5),     # y face: {c0, c1, c4, c5}
        (1, 2, 1): (600, 6),     # y face: {c2, c3, c6, c7}
        (1, 1, 2): (600, 6),     # z face: {c4..c7}
        (0, 0, 1): (900, 0),     # z edge: {c0, c4}
        (0, 1, 0): (700, 2),     # y edge: {c0, c2}
        (2, 0, 1): (650, 5),     # z edge: {c1, c5}
    }
    for (ix, iy, iz), (pdm, m) in cases.items():
        i = v(ix, iy, iz)
        assert f.pdmin[i] == pdm and f.mref[i] == m and f.lam_ref[i] == lam[m], ((ix, iy, iz), f.pdmin[i], f.mref[i])


# ---------------------------------------------------------------------------------
# The LIMEX error estimate (Section 4, Eq. norm_u), on states with closed forms.
# ---------------------------------------------------------------------------------
def test_error_estimate_closed_form_constant_saturation():
    """Linear pressures and spatially constant saturations: the Q1 interpolant of a
    linear function is exact, so ||grad p||^2 = |grad p|^2 |Omega| and the lumped
    ||S||^2 = S^2 |Omega| (the dual boxes tile Omega).  With p_c = 0 (p_d = 0) p_n = p_w,
    so eps = sqrt((|grad dp|^2 / |grad p|^2 + dS_w^2 / S_w^2) / 2) exactly.  A missing
    1/2, S_n in place of S_w (0.3 against 0.7) or a swapped normalisation fails."""
    scn = make_scn(3, (5, 4, 6), (1.0, 0.5, 2.0), pd=0.0)
    vol = 1.0 * 0.5 * 2.0
    x, y, z = scn.vertex_coords()
    nm = LX.Norms(FV.FV(scn))
    a = np.array([3.0e3, -1.0e3, 2.0e2])      # grad p_w of T_kk
    b = np.array([3.1e3, -0.9e3, 2.0e2])      # grad p_w of T_k,k-1
    kk = np.stack([a[0] * x + a[1] * y + a[2] * z + 1e5, np.full_like(x, 0.3)], axis=1)
    km = np.stack([b[0] * x + b[1] * y + b[2] * z + 1e5, np.full_like(x, 0.32)], axis=1)
    e_p2 = np.sum((a - b) ** 2) * vol / (np.sum(a ** 2) * vol)
    e_s2 = (0.02 ** 2 * vol) / (0.7 ** 2 * vol)
    assert nm.err_ratio(kk, km) == pytest.approx(np.sqrt(0.5 * (e_p2 + e_s2)), rel=1e-12)
    # the two halves separately: equal saturations, then equal pressures
    km_p = km.copy(); km_p[:, 1] = 0.3
    assert nm.err_ratio(kk, km_p) == pytest.approx(np.sqrt(0.5 * e_p2), rel=1e-12)
    km_s = km.copy(); km_s[:, 0] = kk[:, 0]
    assert nm.err_ratio(kk, km_s) == pytest.approx(np.sqrt(0.5 * e_s2), rel=1e-12)


def test_error_estimate_uses_the_convective_pressure():
    """Eqs. norm_uw/norm_un measure the pressure whose gradient drives the convective
    fluxes; with the unknowns (p_w, S_n) that is p_w, not p_n = p_w + p_c.  A
    homogeneous medium (p_d 1000 Pa, lambda 2) whose saturation is chosen per vertex so
    that p_c = p_d S_e^(-1/lambda) = 1500 + 750 x is linear: with the same saturation in
    both states only the pressure term is left, eps = sqrt(1/2) |grad dp_w| / |grad p_w|,
    while a p_n norm would give sqrt(1/2) |grad dp_w| / |grad p_w + grad p_c|."""
    scn = make_scn(2, (9, 5, 1), (2.0, 1.0, 1.0), pd=1000.0, lam=2.0, s_res=(0.1, 0.05))
    x, y, _ = scn.vertex_coords()
    pc = 1500.0 + 750.0 * x                        # 1500 ... 3000 Pa
    se = (pc / 1000.0) ** (-2.0)                   # S_e in (0.11, 0.44): no clamp
    sn = 1.0 - (0.1 + se * (1.0 - 0.1 - 0.05))
    nm = LX.Norms(FV.FV(scn))
    np.testing.assert_allclose(nm.fv.vertex_pc(np.stack([0 * x, sn], axis=1)), pc, rtol=1e-13)
    gw = np.array([-100.0, 50.0])
    dg = np.array([5.0, -2.0])
    kk = np.stack([2e5 + gw[0] * x + gw[1] * y, sn], axis=1)
    km = np.stack([2e5 + (gw[0] - dg[0]) * x + (gw[1] - dg[1]) * y, sn], axis=1)
    want = np.sqrt(0.5 * np.sum(dg ** 2) / np.sum(gw ** 2))
    assert nm.err_ratio(kk, km) == pytest.approx(want, rel=1e-12)
    gn = gw + np.array([750.0, 0.0])
    assert abs(nm.err_ratio(kk, km) / np.sqrt(0.5 * np.sum(dg ** 2) / np.sum(gn ** 2)) - 1) > 0.5


# ---------------------------------------------------------------------------------
# Consistency of the algebraic pressure (reading of the index-1 structure of
# M(u) u' = F(u), Section 4).
# ---------------------------------------------------------------------------------
def test_pressure_projection_satisfies_the_volume_balance():
    """After the projection the volume balance F_w/rho_w + F_n/rho_n vanishes at every
    vertex without a Dirichlet component (the incompressible constraint: the two
    storages cancel in it), the saturation is untouched bit for bit, and Newton
    converges fast (quadratically once close)."""
    scn = W.lens_2d(17, 9)
    scn.levels = 3
    st = ST.Stage(scn)
    u0 = W.perturbed_state(scn, 12, dp=80.0, sn_lo=0.05, sn_hi=0.5)
    F0 = st.residual(u0.ravel()).reshape(-1, 2)
    vol0 = F0[:, 0] / scn.rho[0] + F0[:, 1] / scn.rho[1]
    u, info = st.project_pressure(u0.ravel(), rtol=1e-12)
    u = u.reshape(-1, 2)
    assert info["converged"] and info["newton"] <= 8, info
    np.testing.assert_array_equal(u[:, 1], u0[:, 1])
    F = st.residual(u.ravel()).reshape(-1, 2)
    vol = F[:, 0] / scn.rho[0] + F[:, 1] / scn.rho[1]
    free = scn.dir_mask == 0
    print("volume balance before / after:", np.abs(vol0[free]).max(), np.abs(vol[free]).max(), info["history"])
    assert np.abs(vol[free]).max() <= 1e-8 * np.abs(vol0[free]).max()
    # what remains is the O(h_p) of the vanishing step: a 100 times smaller h_p leaves
    # a 100 times smaller volume balance
    u2, _ = st.project_pressure(u0.ravel(), h_p=1e-8, rtol=1e-13)
    F2 = st.residual(u2).reshape(-1, 2)
    vol2 = F2[:, 0] / scn.rho[0] + F2[:, 1] / scn.rho[1]
    assert 50.0 < np.abs(vol[free]).max() / np.abs(vol2[free]).max() < 200.0
    # the non-wetting balance itself is not zeroed: the saturation has its own dynamics
    assert np.abs(F[free, 1]).max() > 1e-3 * np.abs(F0[free, 1]).max()


def test_stall_rule_by_hand():
    r = ST.StallRule()
    assert not r.after_step(False, 80.0, 0.16)      # first rejection: the reference
    assert not r.after_step(False, 22.7, 0.017)     # tau/3.5, eps/9.6: falling, new reference
    assert not r.after_step(False, 13.8, 0.016)     # tau not yet halved
    assert r.after_step(False, 8.4, 0.0176)         # tau/2.7 but eps flat: project
    assert not r.after_step(False, 5.0, 0.001)      # the reference was cleared
    assert not r.after_step(False, 1.0, float("inf"))
    assert not r.after_step(True, 1.0, 1e-3)
    assert r.ref is None


@pytest.mark.parametrize("k,row,limit", [(3, 3, 1.0 / 3.0), (3, 2, 0.5), (2, 2, 0.5)])
def test_error_estimate_of_a_tableau_dominated_by_one_row(k, row, limit):
    """When the substeps of one tableau row diverge, that row dominates the extrapolation
    and eps tends to a ratio of the Aitken-Neville coefficients: for k = 3 a dominant
    T_31 gives T_32 ~ 3 T_31 and T_33 ~ 4.5 T_31, so both parts of Eq. norm_u tend to
    1.5 / 4.5 and eps to 1/3; a dominant T_21 gives T_kk - T_k,k-1 ~ T_kk / 2, eps 1/2."""
    scn = W.lens_2d(9, 5)
    f = FV.FV(scn)
    nm = LX.Norms(f)
    rng = np.random.default_rng(3)
    u = W.perturbed_state(scn, 2, sn_lo=0.1, sn_hi=0.3).ravel()
    w = rng.standard_normal(u.size)
    for scale in (1e6, 1e9):
        T1 = [u + 1e-3 * rng.standard_normal(u.size) for _ in range(k)]
        T1[row - 1] = T1[row - 1] + scale * w
        kk, km = LX.extrapolate(T1)
        assert nm.err_ratio(kk, km) == pytest.approx(limit, rel=1e-5 if scale == 1e9 else 1e-2)
