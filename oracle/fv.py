"""Vertex-centred finite volumes (box method) on structured Q1 quads / hexes for the
incompressible immiscible two-phase model with unknowns (p_w, S_n).

Paper passages followed (Section 2, Section 3):
  * mass balance per phase and the extended Darcy law (Eqs. m, u), saturation closure
    (Eq. S) and capillary pressure p_c = p_n - p_w (Eq. pc);
  * the box-method balance per control volume b_i: storage integrated over the
    sub-control volumes (SCV) b_i ∩ e_j, fluxes through the sub-control-volume faces
    (SCVF) evaluated at their integration points (Eqs. dsW, dpN);
  * upwinding of the relative permeabilities by the sign of the phase velocity
    without the capillary part, the capillary diffusion left central (Section 3.2,
    Eqs. up_krw, up_krn);
  * the p_dmin interface condition (Eqs. pdmin, hSw) applied to the non-wetting
    mobility and not to the wetting one (Eqs. krn_ip, krw_ip); p_dmin is a per-vertex
    constant computed once.

Readings taken where the paper is silent:
  * unknowns (p_w, S_n): the convective part of the non-wetting flux is upwinded with
    v_n' = -K/mu_n (grad p_w - rho_n g); the capillary part -k_rn K/mu_n grad p_c is
    central and sits in the non-wetting balance;
  * Brooks-Corey / Burdine laws in textbook form:
      S_e = (S_w - S_wr)/(1 - S_wr - S_nr),  p_c = p_d S_e^(-1/lam),
      k_rw = S_e^((2+3 lam)/lam),  k_rn = (1-S_e)^2 (1 - S_e^((2+lam)/lam));
    or, where a scenario selects the printed polynomial laws of Section 5 (cases 4
    and 5), k_rw = a_w S_e^2, k_rn = a_n (1 - S_e) with the same Brooks-Corey p_c;
    S_e is clamped to [1e-6, 1] inside p_c and k_r;
  * the Leverett J of a cell is J_e(S_e) = S_e^(-1/lam_e); the vertex capillary
    pressure P_i uses the reference medium m(i) = lowest-index adjacent cell with
    p_d = p_dmin,i;  hat cases are tested in the order equal / barrier / continuity;
  * storage of SCV (i, e) uses the hatted saturation of that SCV;
  * the capillary gradient is the Q1 gradient of the element-local nodal capillary
    pressures p_c,e(S^_{l,e}); k_rn in the capillary term is evaluated at the Q1
    interpolant of S^_{.,e} at the integration point;
  * each SCVF is oriented from its lower to its higher global vertex index; a zero
    upwind velocity picks the lower index;
  * integration point of an SCVF = barycentre of the face: (1/2, 1/4[, 1/4]) in the
    reference cell relative to its edge.
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.sparse as sp

SE_MIN = 1.0e-6


# ---------------------------------------------------------------------------------
# Constitutive laws (complex-step safe: every branch decision uses the real part).
# ---------------------------------------------------------------------------------
def _clamp_se(se):
    lo = np.where(np.real(se) < SE_MIN, True, False)
    hi = np.where(np.real(se) > 1.0, True, False)
    return np.where(lo, SE_MIN + 0 * se, np.where(hi, 1.0 + 0 * se, se))


def eff_sat(sn, swr, snr):
    """Effective wetting saturation S_e of a non-wetting saturation S_n (clamped)."""
    return _clamp_se(((1.0 - sn) - swr) / ((1.0 - swr) - snr))


def pc_bc(sn, pd, lam, swr, snr):
    """Brooks-Corey capillary pressure p_d S_e^(-1/lam)."""
    return pd * eff_sat(sn, swr, snr) ** (-1.0 / lam)


def krw_bc(sn, lam, swr, snr):
    """Burdine wetting relative permeability S_e^((2+3 lam)/lam)."""
    return eff_sat(sn, swr, snr) ** ((2.0 + 3.0 * lam) / lam)


def krn_bc(sn, lam, swr, snr):
    """Burdine non-wetting relative permeability (1-S_e)^2 (1 - S_e^((2+lam)/lam))."""
    se = eff_sat(sn, swr, snr)
    return (1.0 - se) ** 2 * (1.0 - se ** ((2.0 + lam) / lam))


def krw_poly(sn, a_w, swr, snr):
    """Polynomial wetting relative permeability a_w S_e^2 (Section 5, Tables case4 and
    case5: a_w = 0.9)."""
    return a_w * eff_sat(sn, swr, snr) ** 2


def krn_poly(sn, a_n, swr, snr):
    """Polynomial non-wetting relative permeability a_n (1 - S_e) (Tables case4 and
    case5: a_n = 0.5)."""
    return a_n * (1.0 - eff_sat(sn, swr, snr))


def hat_sn(sn, pdmin, lam_ref, pd_e, lam_e, swr, snr):
    """Saturation of the SCV (vertex i, element e) under the p_dmin interface
    condition (Eq. hSw), returned as a non-wetting saturation.

    sn: vertex S_n,i; pdmin, lam_ref: p_dmin,i and lambda of the reference medium;
    pd_e, lam_e: entry pressure and lambda of element e.
      case 1  p_d,e == p_dmin,i            -> S_n,i
      case 2  p_d,e >= P_i = p_dmin J(S_i) -> residual S_nr (S_w = 1 - S_nr)
      case 3  otherwise: S with p_d,e J_e(S) = P_i, i.e. S_e = (P_i/p_d,e)^(-lam_e)
    """
    dd = (1.0 - swr) - snr
    p_vert = pdmin * eff_sat(sn, swr, snr) ** (-1.0 / lam_ref)
    case1 = pd_e == pdmin
    case2 = pd_e >= np.real(p_vert)
    with np.errstate(divide="ignore", invalid="ignore"):  # case 3 is unused where p_d,e = 0
        se_star = (p_vert / pd_e) ** (-lam_e)
    sn3 = 1.0 - (swr + se_star * dd)
    return np.where(case1, sn, np.where(case2, snr + 0 * sn, sn3))


# ---------------------------------------------------------------------------------
# Discretisation
# ---------------------------------------------------------------------------------
class FV:
    """Box-method discretisation of one scenario (see workloads.Scenario)."""

    def __init__(self, scn):
        self.scn = scn
        d = scn.dim
        self.d = d
        self.n = tuple(scn.n)
        self.N = scn.nverts
        self.h = np.array(scn.spacing[:d], dtype=np.float64)
        self.vol = float(np.prod(self.h))
        self.scv = self.vol / 2 ** d
        self.g = np.array(scn.gravity[:d], dtype=np.float64)
        self.rho = np.array(scn.rho, dtype=np.float64)
        self.mu = np.array(scn.mu, dtype=np.float64)
        self.swr, self.snr = float(scn.s_res[0]), float(scn.s_res[1])
        self.K = np.asarray(scn.perm, np.float64)
        self.phi = np.asarray(scn.poro, np.float64)
        self.pd = np.asarray(scn.entry_p, np.float64)
        self.lam = np.asarray(scn.bc_lambda, np.float64)
        self.dir_mask = np.asarray(scn.dir_mask, np.uint8)
        self.kr_model = getattr(scn, "kr_model", "burdine")
        self.kr_coef = tuple(getattr(scn, "kr_coef", (1.0, 1.0)))
        if self.kr_model not in ("burdine", "poly"):
            raise ValueError(f"unknown relative-permeability law {self.kr_model!r}")
        nx, ny, nz = self.n
        ncz, ncy, ncx = scn.cell_shape
        cz, cy, cx = np.meshgrid(np.arange(ncz), np.arange(ncy), np.arange(ncx), indexing="ij")
        cx, cy, cz = cx.ravel(), cy.ravel(), cz.ravel()
        self.nc = 2 ** d
        self.bits = np.array([[(l >> a) & 1 for a in range(d)] for l in range(self.nc)])
        cols = []
        for l in range(self.nc):
            b = list(self.bits[l]) + [0] * (3 - d)
            cols.append((cx + b[0]) + nx * ((cy + b[1]) + ny * (cz + b[2])))
        self.cv = np.stack(cols, axis=1)  # (Ncells, 2^d) corner vertices
        self.ncells = self.cv.shape[0]
        # SCVFs of a cell: one per cell edge; normal along the edge, from l0 to l1
        self.scvf = []
        for a in range(d):
            others = [b for b in range(d) if b != a]
            for combo in itertools.product((0, 1), repeat=d - 1):
                l0 = 0
                xi = np.zeros(d)
                xi[a] = 0.5
                for b, bit in zip(others, combo):
                    l0 |= bit << b
                    xi[b] = 0.75 if bit else 0.25
                l1 = l0 | (1 << a)
                area = self.vol / (2 ** (d - 1) * self.h[a])
                self.scvf.append((a, l0, l1, self.shape(xi), self.grad(xi, a), area))
        self._pdmin_and_reference()
        self.Q = self.neumann_sources()

    # -- Q1 shape functions on the reference cell ---------------------------------
    def shape(self, xi):
        out = np.ones(self.nc)
        for l in range(self.nc):
            for a in range(self.d):
                out[l] *= xi[a] if self.bits[l, a] else 1.0 - xi[a]
        return out

    def grad(self, xi, a):
        """d N_l / d x_a at reference point xi (physical derivative)."""
        out = np.ones(self.nc)
        for l in range(self.nc):
            for b in range(self.d):
                if b == a:
                    out[l] *= (1.0 if self.bits[l, b] else -1.0) / self.h[a]
                else:
                    out[l] *= xi[b] if self.bits[l, b] else 1.0 - xi[b]
        return out

    # -- pre-processing: p_dmin,i and the reference medium (Eq. pdmin) ---------------
    def _pdmin_and_reference(self):
        pdmin = np.full(self.N, np.inf)
        for l in range(self.nc):
            np.minimum.at(pdmin, self.cv[:, l], self.pd)
        big = np.iinfo(np.int64).max
        mref = np.full(self.N, big, dtype=np.int64)
        cells = np.arange(self.ncells, dtype=np.int64)
        for l in range(self.nc):
            v = self.cv[:, l]
            cand = np.where(self.pd == pdmin[v], cells, big)
            np.minimum.at(mref, v, cand)
        self.pdmin = pdmin
        self.mref = mref
        self.lam_ref = self.lam[mref]

    def vertex_pc(self, u):
        """Vertex capillary pressure P_i = p_dmin,i J_m(i)(S_i) in the reference medium
        m(i) (the p_c that the interface condition of Eq. hSw compares with), so that
        p_n,i = p_w,i + P_i at every vertex.  u: (N, 2)."""
        se = eff_sat(u[:, 1], self.swr, self.snr)
        return self.pdmin * se ** (-1.0 / self.lam_ref)

    # -- Neumann sources: exact overlap of the dual-box face with each patch -------
    def neumann_sources(self):
        scn = self.scn
        Q = np.zeros((self.N, 2))
        coords = scn.vertex_coords()
        ext = scn.extent
        for p in scn.patches:
            a = p.axis
            on_face = np.isclose(coords[a], 0.0 if p.side == 0 else ext[a])
            measure = np.ones(self.N)
            others = [b for b in range(self.d) if b != a]
            for k, b in enumerate(others):
                lo = np.maximum(np.maximum(coords[b] - 0.5 * self.h[b], 0.0), p.lo[k])
                hi = np.minimum(np.minimum(coords[b] + 0.5 * self.h[b], ext[b]), p.hi[k])
                measure *= np.maximum(hi - lo, 0.0)
            Q[:, p.phase] += np.where(on_face, p.rate * measure, 0.0)
        src = getattr(scn, "vertex_source", None)
        if src is not None:  # mass rates into single control volumes (point sources)
            Q = Q + np.asarray(src, np.float64).reshape(self.N, 2)
        return Q

    # -- relative permeabilities of the scenario's law ------------------------------
    def krw(self, sn, lam):
        if self.kr_model == "poly":
            return krw_poly(sn, self.kr_coef[0], self.swr, self.snr)
        return krw_bc(sn, lam, self.swr, self.snr)

    def krn(self, sn, lam):
        if self.kr_model == "poly":
            return krn_poly(sn, self.kr_coef[1], self.swr, self.snr)
        return krn_bc(sn, lam, self.swr, self.snr)

    # -- per-cell evaluations -------------------------------------------------------
    def _cells(self, cells):
        return np.arange(self.ncells) if cells is None else np.asarray(cells)

    def hat(self, u, cells=None):
        c = self._cells(cells)
        cv = self.cv[c]
        sn = u[:, 1][cv]
        return hat_sn(sn, self.pdmin[cv], self.lam_ref[cv], self.pd[c][:, None],
                      self.lam[c][:, None], self.swr, self.snr)

    def storage(self, u, cells=None):
        """m_i = sum over the SCVs of b_i of Phi_e rho_alpha S^_alpha |SCV|, shape (N, 2)."""
        c = self._cells(cells)
        sh = self.hat(u, c)
        m = np.zeros((self.N, 2), dtype=np.result_type(u.dtype, np.float64))
        wphi = self.phi[c][:, None] * self.scv
        for l in range(self.nc):
            np.add.at(m[:, 0], self.cv[c, l], wphi[:, 0] * self.rho[0] * (1.0 - sh[:, l]))
            np.add.at(m[:, 1], self.cv[c, l], wphi[:, 0] * self.rho[1] * sh[:, l])
        return m

    def flux_divergence(self, u, cells=None):
        """-(sum of outward SCVF mass fluxes) per vertex and phase, shape (N, 2)."""
        c = self._cells(cells)
        cv = self.cv[c]
        p = u[:, 0][cv]
        sn = u[:, 1][cv]
        sh = self.hat(u, c)
        K = self.K[c]
        lam = self.lam[c]
        pd = self.pd[c]
        swr, snr = self.swr, self.snr
        pc = pc_bc(sh, pd[:, None], lam[:, None], swr, snr)
        out = np.zeros((self.N, 2), dtype=np.result_type(u.dtype, np.float64))
        rw, rn = self.rho
        mw, mn = self.mu
        for (a, l0, l1, Nsh, G, area) in self.scvf:
            ga = self.g[a]
            dp = p @ G
            # wetting phase: upwinded k_rw at the plain vertex saturation
            phi_w = -(K / mw) * (dp - rw * ga) * area
            up = np.real(phi_w) >= 0.0
            sn_up = np.where(up, sn[:, l0], sn[:, l1])
            fw = rw * self.krw(sn_up, lam) * phi_w
            # non-wetting phase: upwinded k_rn at the hatted SCV saturation
            phi_n = -(K / mn) * (dp - rn * ga) * area
            upn = np.real(phi_n) >= 0.0
            sh_up = np.where(upn, sh[:, l0], sh[:, l1])
            fn = rn * self.krn(sh_up, lam) * phi_n
            # capillary diffusion, central
            s_ip = sh @ Nsh
            dpc = pc @ G
            fc = -rn * self.krn(s_ip, lam) * (K / mn) * dpc * area
            np.add.at(out[:, 0], cv[:, l0], -fw)
            np.add.at(out[:, 0], cv[:, l1], fw)
            np.add.at(out[:, 1], cv[:, l0], -(fn + fc))
            np.add.at(out[:, 1], cv[:, l1], fn + fc)
        return out

    def residual_raw(self, u, cells=None):
        """F(u) = Q - outflow, before Dirichlet rows are cleared."""
        return self.Q + self.flux_divergence(u, cells)

    def residual(self, u, cells=None):
        """F(u) with the Dirichlet components set to zero (the stage RHS)."""
        F = self.residual_raw(u, cells)
        F[:, 0] = np.where(self.dir_mask & 1, 0.0, F[:, 0])
        F[:, 1] = np.where(self.dir_mask & 2, 0.0, F[:, 1])
        return F

    # -- Jacobians by complex-step differentiation --------------------------------
    def _colors(self):
        nx, ny, nz = self.n
        iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        ix, iy, iz = ix.ravel(), iy.ravel(), iz.ravel()
        return ix, iy, iz

    def jacobian(self, u, cells=None, step=1e-30, which="residual"):
        """J = dF/du (which='residual', Dirichlet rows zero) or dm/du ('storage') as a
        CSR matrix over interleaved DoFs 2*v + comp, by complex-step differentiation
        with a 3^d colouring of the vertices (each row's stencil sees every colour
        at most once)."""
        nx, ny, nz = self.n
        ix, iy, iz = self._colors()
        d = self.d
        color = (ix % 3) + 3 * (iy % 3) + (9 * (iz % 3) if d == 3 else 0)
        ncol = 3 ** d
        fun = self.residual if which == "residual" else self.storage
        rows, cols, vals = [], [], []
        for col in range(ncol):
            cxyz = [col % 3, (col // 3) % 3, col // 9]
            # neighbour of colour `col` for every vertex: offset per axis in {-1,0,1}
            offs = []
            for a, ii in enumerate((ix, iy, iz)):
                if a >= d:
                    offs.append(np.zeros_like(ii))
                    continue
                dlt = (cxyz[a] - ii) % 3
                offs.append(np.where(dlt == 2, -1, dlt))
            jx, jy, jz = ix + offs[0], iy + offs[1], iz + offs[2]
            ok = (jx >= 0) & (jx < nx) & (jy >= 0) & (jy < ny) & (jz >= 0) & (jz < nz)
            j = jx + nx * (jy + ny * jz)
            sel = color == col
            for comp in range(2):
                du = np.zeros((self.N, 2), dtype=np.complex128)
                du[sel, comp] = 1j * step
                Fc = fun(u.astype(np.complex128) + du, cells)
                D = Fc.imag / step
                for r in range(2):
                    rows.append(2 * np.nonzero(ok)[0] + r)
                    cols.append(2 * j[ok] + comp)
                    vals.append(D[ok, r])
        rows = np.concatenate(rows)
        cols = np.concatenate(cols)
        vals = np.concatenate(vals)
        return sp.csr_matrix((vals, (rows, cols)), shape=(2 * self.N, 2 * self.N))

    def mass_matrix(self, u):
        """M = dm/du (block diagonal; only the S_n column is non-zero)."""
        rows, cols, vals = [], [], []
        for comp in range(2):
            du = np.zeros((self.N, 2), dtype=np.complex128)
            du[:, comp] = 1e-30j
            D = self.storage(u.astype(np.complex128) + du).imag / 1e-30
            for r in range(2):
                rows.append(2 * np.arange(self.N) + r)
                cols.append(2 * np.arange(self.N) + comp)
                vals.append(D[:, r])
        return sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                             shape=(2 * self.N, 2 * self.N))

    def dirichlet_dofs(self):
        m = self.dir_mask
        dofs = np.concatenate([2 * np.nonzero(m & 1)[0], 2 * np.nonzero(m & 2)[0] + 1])
        return np.sort(dofs)

    def storage_part(self, u0, h):
        """M(u0)/h with the Dirichlet rows cleared: the storage part of the stage matrix."""
        keep = np.ones(2 * self.N)
        keep[self.dirichlet_dofs()] = 0.0
        return sp.csr_matrix(sp.diags(keep) @ self.mass_matrix(u0) / h)

    def stage_matrix(self, u0, h, cells=None, frozen=None):
        """A = M(u0)/h - J(u0) (Section 4: the linearly implicit Euler matrix divided
        by the step), with unit rows at the Dirichlet components.  frozen = (M, J) of
        u0 from an earlier call (the stages of one linearly implicit step share them)."""
        M, J = frozen if frozen is not None else self.frozen_matrices(u0, cells)
        keep = np.ones(2 * self.N)
        keep[self.dirichlet_dofs()] = 0.0
        A = sp.diags(keep) @ (M / h - J) + sp.diags(1.0 - keep)
        return sp.csr_matrix(A)

    def frozen_matrices(self, u0, cells=None):
        """(M(u0), J(u0)): the storage and flux Jacobians a linearly implicit step
        freezes at its initial state."""
        return self.mass_matrix(u0), self.jacobian(u0, cells)
