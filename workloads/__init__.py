"""Seeded synthetic scenarios for the two-phase (p_w, S_n) Darcy stage solver.

This module only *describes* inputs: grids, fluids, per-cell rock fields, Dirichlet
masks/values, injection patches and initial states.  It holds none of the method's
arithmetic (no constitutive law, no discretisation, no solver), so both the FP64 CPU
oracle and the HIP library can consume the same inputs without sharing any code of
the method itself.

Conventions (shared by every consumer):
  * vertex (ix, iy, iz) has coordinates (ix*dx, iy*dy, iz*dz), dx = Lx/(nx-1);
  * vertex arrays have shape (nz, ny, nx) (x fastest), cell arrays (ncz, ncy, ncx);
    in 2D nz = 1 and the cell arrays have shape (1, ny-1, nx-1);
  * the state u is (N, 2) float64, column 0 = p_w [Pa], column 1 = S_n [-];
  * dir_mask bit0 = p_w Dirichlet, bit1 = S_n Dirichlet; dir_value is (N, 2);
  * an injection patch is a rectangle on a boundary face with a mass rate per unit
    face measure (kg/(m^2 s) in 3D, kg/(m s) in 2D) of one phase into the domain;
  * a point source is a mass rate (kg/s) into the control volume (dual box) of the
    vertex whose box contains the point, held in vertex_source (N, 2).

Recipes follow the paper's parameter tables (Section 5: Case-4 step control values,
Case-5 geometry sizes) and synthetic layered / log-normal reservoirs standing in for
the paper's; the random field is a Gaussian field with exponential covariance drawn
by circulant embedding (Dietrich & Newsam 1997).
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import List, Optional, Tuple

import numpy as np

GRAV = 9.81


@dataclass
class Patch:
    axis: int          # face normal axis (0 x, 1 y, 2 z)
    side: int          # 0: coordinate 0, 1: coordinate = extent[axis]
    lo: Tuple[float, float]   # rectangle on the face, in the remaining axes (increasing order)
    hi: Tuple[float, float]
    rate: float        # kg/(m^{d-1} s) into the domain
    phase: int = 1     # 0 wetting, 1 non-wetting


@dataclass
class Scenario:
    name: str
    dim: int
    n: Tuple[int, int, int]          # vertices per axis (nz = 1 in 2D)
    extent: Tuple[float, float, float]
    gravity: Tuple[float, float, float]
    rho: Tuple[float, float]         # (w, n) kg/m^3
    mu: Tuple[float, float]          # (w, n) Pa s
    s_res: Tuple[float, float]       # (S_wr, S_nr)
    perm: np.ndarray                 # per cell, m^2
    poro: np.ndarray                 # per cell
    entry_p: np.ndarray              # per cell, Pa
    bc_lambda: np.ndarray            # per cell, Brooks-Corey lambda
    dir_mask: np.ndarray             # per vertex uint8
    dir_value: np.ndarray            # (N, 2)
    patches: List[Patch]
    u0: np.ndarray                   # (N, 2) initial state
    levels: int = 1
    h: float = 32.0                  # stage step for single-stage workloads [s]
    meta: dict = field(default_factory=dict)
    kr_model: str = "burdine"        # "burdine" (Brooks-Corey-Burdine) or "poly" (a_w S_e^2, a_n (1-S_e))
    kr_coef: Tuple[float, float] = (1.0, 1.0)   # (a_w, a_n) of the polynomial law
    vertex_source: Optional[np.ndarray] = None  # (N, 2) kg/s into single control volumes, or None

    @property
    def nverts(self) -> int:
        return int(self.n[0] * self.n[1] * self.n[2])

    @property
    def ncells(self) -> int:
        nz = self.n[2] - 1 if self.dim == 3 else 1
        return int((self.n[0] - 1) * (self.n[1] - 1) * nz)

    @property
    def cell_shape(self) -> Tuple[int, int, int]:
        nz = self.n[2] - 1 if self.dim == 3 else 1
        return (nz, self.n[1] - 1, self.n[0] - 1)

    @property
    def vert_shape(self) -> Tuple[int, int, int]:
        return (self.n[2], self.n[1], self.n[0])

    @property
    def spacing(self) -> Tuple[float, float, float]:
        dz = self.extent[2] / (self.n[2] - 1) if self.dim == 3 else 1.0
        return (self.extent[0] / (self.n[0] - 1), self.extent[1] / (self.n[1] - 1), dz)

    def vertex_coords(self):
        dx, dy, dz = self.spacing
        z, y, x = np.meshgrid(np.arange(self.n[2]) * dz, np.arange(self.n[1]) * dy,
                              np.arange(self.n[0]) * dx, indexing="ij")
        if self.dim == 2:
            z = np.zeros_like(z)
        return x.ravel(), y.ravel(), z.ravel()

    def cell_centres(self):
        dx, dy, dz = self.spacing
        ncz, ncy, ncx = self.cell_shape
        z, y, x = np.meshgrid((np.arange(ncz) + 0.5) * dz, (np.arange(ncy) + 0.5) * dy,
                              (np.arange(ncx) + 0.5) * dx, indexing="ij")
        return x.ravel(), y.ravel(), z.ravel()

    def with_state(self, u: np.ndarray) -> "Scenario":
        return replace(self, u0=np.ascontiguousarray(u, dtype=np.float64))


# ---------------------------------------------------------------------------------
# Gaussian random field, exponential covariance, circulant embedding.
# ---------------------------------------------------------------------------------
def gaussian_field(shape, corr_cells: float, sigma: float, seed: int, return_clip=False):
    """Stationary Gaussian field on a lattice of `shape` (cell units) with covariance
    C(r) = sigma^2 exp(-r / corr_cells), r the Euclidean lattice distance.

    The lattice is embedded in a periodic torus of twice its size per axis; the
    circulant covariance is diagonalised by the FFT, negative eigenvalues are clipped
    to zero (their relative weight is returned on request) and the field is the
    circulant square root applied to white noise from numpy's default_rng(seed).
    """
    shape = tuple(int(s) for s in shape)
    pad = tuple(2 * s if s > 1 else 1 for s in shape)
    grids = []
    for m in pad:
        k = np.arange(m, dtype=np.float64)
        grids.append(np.minimum(k, m - k))
    r2 = np.zeros(pad, dtype=np.float64)
    for ax, g in enumerate(grids):
        sh = [1] * len(pad)
        sh[ax] = pad[ax]
        r2 = r2 + (g.reshape(sh) ** 2)
    cov = (sigma ** 2) * np.exp(-np.sqrt(r2) / corr_cells)
    lam = np.fft.rfftn(cov).real
    del cov, r2
    neg = lam < 0
    clipped = float(-lam[neg].sum() / np.abs(lam).sum()) if neg.any() else 0.0
    lam[neg] = 0.0
    rng = np.random.default_rng(seed)
    w = rng.standard_normal(pad)
    z = np.fft.irfftn(np.sqrt(lam) * np.fft.rfftn(w), s=pad, axes=tuple(range(len(pad))))
    sl = tuple(slice(0, s) for s in shape)
    out = np.ascontiguousarray(z[sl])
    return (out, clipped) if return_clip else out


# ---------------------------------------------------------------------------------
# Fluids and rock shared by the lens and cube recipes.
# ---------------------------------------------------------------------------------
RHO = (1000.0, 1460.0)
MU = (1.0e-3, 9.0e-4)
PORO = 0.4
LAMBDA_BG = 2.5
PD_BG = 800.0
K_MEAN_LN = -25.0
P_TOP = 1.0e5


def _leverett_pd(perm):
    # entry pressure scaled with sqrt(K_ref / K), K_ref = exp(-25) m^2, p_d(K_ref) = 800 Pa
    return PD_BG * np.sqrt(np.exp(K_MEAN_LN) / perm)


def lens_2d(nx: int = 65, ny: int = 33) -> Scenario:
    """2D DNAPL-over-lens workload: 1.0 x 0.6 m, 65x33 vertices, gravity along -y,
    low-permeability lens over [0.3,0.7]x[0.25,0.4] (cell centres), injection of the
    non-wetting phase through the top-middle 0.2 m, hydrostatic Dirichlet sides."""
    Lx, Ly = 1.0, 0.6
    scn = _empty(f"lens2d_{nx}x{ny}", 2, (nx, ny, 1), (Lx, Ly, 1.0), (0.0, -GRAV, 0.0))
    cx, cy, _ = scn.cell_centres()
    lens = (cx >= 0.3) & (cx <= 0.7) & (cy >= 0.25) & (cy <= 0.4)
    scn.perm = np.where(lens, 5e-13, 5e-11)
    scn.poro = np.full(scn.ncells, PORO)
    scn.entry_p = np.where(lens, 1500.0, PD_BG)
    scn.bc_lambda = np.where(lens, 2.0, LAMBDA_BG)
    x, y, _ = scn.vertex_coords()
    p_hyd = P_TOP + RHO[0] * GRAV * (Ly - y)
    side = np.isclose(x, 0.0) | np.isclose(x, Lx)
    scn.dir_mask = np.where(side, 3, 0).astype(np.uint8)
    scn.dir_value = np.stack([p_hyd, np.zeros_like(p_hyd)], axis=1)
    scn.patches = [Patch(axis=1, side=1, lo=(0.4, 0.0), hi=(0.6, 0.0), rate=0.075, phase=1)]
    scn.u0 = np.stack([p_hyd, np.zeros_like(p_hyd)], axis=1)
    scn.levels = 4
    return scn


BL_LENGTH, BL_HEIGHT = 300.0, 75.0
BL_PORO, BL_PERM, BL_LAMBDA = 0.2, 1e-7, 2.0
BL_P_LEFT = 2e5          # Pa, Dirichlet p_n = p_w at x = 0
BL_OUTFLOW = 3e-4        # kg/(m^2 s) of the non-wetting phase leaving through x = 300 m
BL_T_END = 1500 * 86400.0


def buckley_leverett(elements: int = 64, levels: Optional[int] = None) -> Scenario:
    """Case 1 of Section 5 (Buckley-Leverett displacement, Table case1).

    A 300 m x 75 m strip of `elements` x elements/4 square cells; porosity 0.2,
    K = 1e-7 m^2; equal densities (1000 kg/m^3) and viscosities (1e-3 Pa s); no
    residual saturations; no capillary pressure (entry pressure 0); Brooks-Corey
    lambda = 2; no gravity (the two densities are equal and the displacement is
    horizontal).  x = 0: Dirichlet S_w = 1 (S_n = 0) and p_n = p_w = 2e5 Pa.
    x = 300 m: the non-wetting phase leaves at 3e-4 kg/(m^2 s) per unit depth.  Other
    faces are closed.  Initially S_w = 0; the initial p_w is the steady single-phase
    profile of that outflow (p_w is algebraic, so only its consistency matters)."""
    if elements % 4:
        raise ValueError("elements must be a multiple of 4")
    nx, ny = elements + 1, elements // 4 + 1
    scn = _empty(f"bl_{elements}", 2, (nx, ny, 1), (BL_LENGTH, BL_HEIGHT, 1.0), (0.0, 0.0, 0.0))
    scn.rho = (1000.0, 1000.0)
    scn.mu = (1e-3, 1e-3)
    nc = scn.ncells
    scn.perm = np.full(nc, BL_PERM)
    scn.poro = np.full(nc, BL_PORO)
    scn.entry_p = np.zeros(nc)
    scn.bc_lambda = np.full(nc, BL_LAMBDA)
    x, _, _ = scn.vertex_coords()
    darcy = BL_OUTFLOW / scn.rho[1]                      # m/s
    p = BL_P_LEFT - darcy * scn.mu[1] / BL_PERM * x
    left = np.isclose(x, 0.0)
    scn.dir_mask = np.where(left, 3, 0).astype(np.uint8)
    scn.dir_value = np.stack([np.full_like(x, BL_P_LEFT), np.zeros_like(x)], axis=1)
    scn.patches = [Patch(axis=0, side=1, lo=(0.0, 0.0), hi=(BL_HEIGHT, 0.0), rate=-BL_OUTFLOW, phase=1)]
    sn = np.where(left, 0.0, 1.0)
    scn.u0 = np.stack([np.where(left, BL_P_LEFT, p), sn], axis=1)
    scn.levels = default_levels(ny) if levels is None else levels
    scn.meta = dict(case="buckley_leverett", elements=elements, t_end=BL_T_END, dt0=1.0,
                    dt_max=100 * 86400.0, tol=5e-2, safety=0.25, stages=2)
    return scn


C5_EXTENT = 200.0
C5_LAYER_K = (1e-13, 1e-12, 8e-13, 7e-13)   # K_1 (bottom) ... K_4 (top), 50 m each
C5_P_BOTTOM = 5e7                            # Pa, Dirichlet p_n at z = 0
C5_INJECTION = (100.0, 100.0, 30.0)          # m, the injection point
C5_PV_PER_YEAR = 0.05
C5_T_END = 128 * 60.0


def case5_pd(perm):
    """Entry pressure law of Tables case4 and case5: p_d = 7.37 K^-0.43 Pa (K in m^2)."""
    return 7.37 * np.asarray(perm, np.float64) ** -0.43


def case5(n: int = 257, levels: Optional[int] = None) -> Scenario:
    """Case 5 of Section 5 (Table case5): 3D layer-wise heterogeneity.

    A 200 m cube of n^3 vertices (257^3 is the paper's 256^3-cell mesh) in four
    horizontal layers of 50 m with K_1 = 1e-13 (bottom), 1e-12, 8e-13, 7e-13 m^2;
    porosity 0.1; rho 1000 / 700 kg/m^3, mu 1e-3 / 5.654e-5 Pa s; S_wr 0.2, S_nr 0.1;
    Brooks-Corey lambda 2 with p_d = 7.37 K^-0.43; k_rw = 0.9 S_e^2, k_rn = 0.5 (1 - S_e);
    gravity along -z.  z = 0: Dirichlet S_w = 1 - S_nr and p_n = 5e7 Pa, i.e. p_w =
    5e7 - p_d(K_1) (S_e = 1 there); the other faces are closed.  Initially S_w = 1 - S_nr
    with hydrostatic p_w (the non-wetting phase is at its residual saturation, hence
    immobile, so this is an equilibrium).  The non-wetting phase is injected at
    0.05 pore volumes per year (year = 365 d) at the point (100, 100, 30) m, the 3D
    counterpart of Case 4's injection point, into the control volume containing it.
    Simulated time 128 min, tau0 = 32 s, tau_max = 100 d."""
    if (n - 1) % 4:
        raise ValueError("n - 1 must be a multiple of 4 (layer boundaries on vertices)")
    L = C5_EXTENT
    scn = _empty(f"case5_{n}", 3, (n, n, n), (L, L, L), (0.0, 0.0, -GRAV))
    scn.rho = (1000.0, 700.0)
    scn.mu = (1e-3, 5.654e-5)
    scn.s_res = (0.2, 0.1)
    scn.kr_model, scn.kr_coef = "poly", (0.9, 0.5)
    _, _, cz = scn.cell_centres()
    layer = np.minimum((cz // (L / 4)).astype(int), 3)
    scn.perm = np.asarray(C5_LAYER_K)[layer]
    scn.poro = np.full(scn.ncells, 0.1)
    scn.entry_p = case5_pd(scn.perm)
    scn.bc_lambda = np.full(scn.ncells, 2.0)
    x, y, z = scn.vertex_coords()
    p_bottom = C5_P_BOTTOM - float(case5_pd(C5_LAYER_K[0]))
    p = p_bottom - scn.rho[0] * GRAV * z
    sn0 = scn.s_res[1]
    bottom = np.isclose(z, 0.0)
    scn.dir_mask = np.where(bottom, 3, 0).astype(np.uint8)
    scn.dir_value = np.stack([np.full_like(z, p_bottom), np.full_like(z, sn0)], axis=1)
    scn.u0 = np.stack([p, np.full_like(z, sn0)], axis=1)
    h = L / (n - 1)
    idx = [int(np.floor(c / h + 0.5)) for c in C5_INJECTION]
    v = idx[0] + n * (idx[1] + n * idx[2])
    rate = C5_PV_PER_YEAR * L ** 3 * 0.1 / (365 * 86400.0) * scn.rho[1]   # kg/s
    src = np.zeros((scn.nverts, 2))
    src[v, 1] = rate
    scn.vertex_source = src
    scn.levels = default_levels(n) if levels is None else levels
    scn.meta = dict(case="case5", t_end=C5_T_END, dt0=32.0, dt_max=100 * 86400.0, tol=5e-3, safety=0.75,
                    stages=3, injection_vertex=v, injection_rate=rate)
    return scn


C4_EXTENT = (500.0, 200.0)
C4_INJECTION = (250.0, 30.0)


def case4(cells_x: int = 4096, levels: Optional[int] = None) -> Scenario:
    """Case 4 of Section 5 (Table case4, Fig. Ap): 2D layer-wise heterogeneity.

    A 500 m x 200 m section of cells_x x cells_x/2 cells (4096 x 2048 is the mesh of
    Table case4_strong, 16,789,506 DoF) in four horizontal layers of 50 m with the
    permeabilities, fluids, residual saturations, p_d(K) and polynomial k_r of case 5;
    gravity along -y.  y = 0: Dirichlet S_w = 1 - S_nr, p_n = 5e7 Pa; other sides
    closed.  Initially S_w = 1 - S_nr with hydrostatic p_w.  Non-wetting injection of
    0.05 pore volumes per year (per metre of depth) at the point (250, 30) m, into the
    control volume containing it.  The scaling runs simulate 128 min from tau0 = 32 s
    (tau_max 100 d, TOL 5e-3, safety 0.75)."""
    if cells_x % 8:
        raise ValueError("cells_x must be a multiple of 8 (layer boundaries on vertices)")
    Lx, Ly = C4_EXTENT
    nx, ny = cells_x + 1, cells_x // 2 + 1
    scn = _empty(f"case4_{cells_x}x{cells_x // 2}", 2, (nx, ny, 1), (Lx, Ly, 1.0), (0.0, -GRAV, 0.0))
    scn.rho = (1000.0, 700.0)
    scn.mu = (1e-3, 5.654e-5)
    scn.s_res = (0.2, 0.1)
    scn.kr_model, scn.kr_coef = "poly", (0.9, 0.5)
    _, cy, _ = scn.cell_centres()
    layer = np.minimum((cy // (Ly / 4)).astype(int), 3)
    scn.perm = np.asarray(C5_LAYER_K)[layer]
    scn.poro = np.full(scn.ncells, 0.1)
    scn.entry_p = case5_pd(scn.perm)
    scn.bc_lambda = np.full(scn.ncells, 2.0)
    x, y, _ = scn.vertex_coords()
    p_bottom = C5_P_BOTTOM - float(case5_pd(C5_LAYER_K[0]))
    p = p_bottom - scn.rho[0] * GRAV * y
    sn0 = scn.s_res[1]
    bottom = np.isclose(y, 0.0)
    scn.dir_mask = np.where(bottom, 3, 0).astype(np.uint8)
    scn.dir_value = np.stack([np.full_like(y, p_bottom), np.full_like(y, sn0)], axis=1)
    scn.u0 = np.stack([p, np.full_like(y, sn0)], axis=1)
    dx, dy, _ = scn.spacing
    ix, iy = int(np.floor(C4_INJECTION[0] / dx + 0.5)), int(np.floor(C4_INJECTION[1] / dy + 0.5))
    v = ix + nx * iy
    rate = C5_PV_PER_YEAR * Lx * Ly * 0.1 / (365 * 86400.0) * scn.rho[1]   # kg/s per metre of depth
    src = np.zeros((scn.nverts, 2))
    src[v, 1] = rate
    scn.vertex_source = src
    scn.levels = default_levels(ny) if levels is None else levels
    scn.meta = dict(case="case4", t_end=C5_T_END, dt0=32.0, dt_max=100 * 86400.0, tol=5e-3, safety=0.75,
                    stages=3, injection_vertex=v, injection_rate=rate)
    return scn


def _empty(name, dim, n, extent, gravity) -> Scenario:
    N = int(n[0] * n[1] * n[2])
    return Scenario(name=name, dim=dim, n=tuple(int(v) for v in n), extent=tuple(map(float, extent)),
                    gravity=tuple(map(float, gravity)), rho=RHO, mu=MU, s_res=(0.0, 0.0),
                    perm=np.zeros(0), poro=np.zeros(0), entry_p=np.zeros(0), bc_lambda=np.zeros(0),
                    dir_mask=np.zeros(N, np.uint8), dir_value=np.zeros((N, 2)), patches=[],
                    u0=np.zeros((N, 2)))


def default_levels(n: int) -> int:
    """Number of vertex-halving levels down to a coarsest grid of at most 9 vertices
    per axis (5 where the size allows), matching the workload table."""
    lv = 1
    m = n
    while (m - 1) % 2 == 0 and (m - 1) // 2 + 1 >= 5:
        m = (m - 1) // 2 + 1
        lv += 1
    return lv


def cube_3d(n: int, sigma: float, seed: int, corr_cells: float = 8.0, sn0: float = 0.05,
            rate: float = 0.075, layers: bool = False, levels: Optional[int] = None,
            h: float = 32.0, field_cache: Optional[np.ndarray] = None, layer_cells: float = 8.0) -> Scenario:
    """3D unit-cube workload with a log-normal permeability field.

    ln K = -25 + sigma * G, G a unit Gaussian field with exponential covariance and
    correlation length `corr_cells` cells; optional three low-permeability slabs
    (`layer_cells` cells thick, 8 by default, centred at z = 0.25, 0.5, 0.75, K x 1e-2).  Entry pressure scales
    with sqrt(K_ref/K); lambda = 2.5; porosity 0.4.  Gravity along -z, hydrostatic
    p_w from 1e5 Pa at the top, uniform initial S_n.  Dirichlet p_w (hydrostatic) and
    S_n = sn0 on the x = 0 and x = 1 faces; non-wetting injection over [0.4,0.6]^2 on
    the top face z = 1."""
    scn = _empty(f"cube{n}_s{sigma:g}_seed{seed}", 3, (n, n, n), (1.0, 1.0, 1.0), (0.0, 0.0, -GRAV))
    ncell = n - 1
    if field_cache is None:
        g = gaussian_field((ncell, ncell, ncell), corr_cells, 1.0, seed)
    else:
        g = field_cache
    lnk = K_MEAN_LN + sigma * g
    if layers:
        zc = (np.arange(ncell) + 0.5) / ncell
        slab = np.zeros(ncell, dtype=bool)
        thick = float(layer_cells) / ncell
        for zc0 in (0.25, 0.5, 0.75):
            slab |= np.abs(zc - zc0) < 0.5 * thick
        lnk = lnk + np.where(slab, np.log(1e-2), 0.0)[:, None, None]
    perm = np.exp(lnk).ravel()
    scn.perm = perm
    scn.poro = np.full(perm.size, PORO)
    scn.entry_p = _leverett_pd(perm)
    scn.bc_lambda = np.full(perm.size, LAMBDA_BG)
    x, y, z = scn.vertex_coords()
    p_hyd = P_TOP + RHO[0] * GRAV * (1.0 - z)
    side = np.isclose(x, 0.0) | np.isclose(x, 1.0)
    scn.dir_mask = np.where(side, 3, 0).astype(np.uint8)
    scn.dir_value = np.stack([p_hyd, np.full_like(p_hyd, sn0)], axis=1)
    scn.patches = [Patch(axis=2, side=1, lo=(0.4, 0.4), hi=(0.6, 0.6), rate=float(rate), phase=1)]
    scn.u0 = np.stack([p_hyd, np.full_like(p_hyd, sn0)], axis=1)
    scn.levels = default_levels(n) if levels is None else levels
    scn.h = h
    scn.meta = dict(sigma=sigma, seed=seed, corr_cells=corr_cells, layers=layers)
    return scn


def cube_c2() -> Scenario:
    """65^3 FP64 single-stage workload, sigma_lnK = 1.0, field seed 2, 5 levels."""
    return cube_3d(65, 1.0, 2, levels=5)


def cube_c3() -> Scenario:
    """129^3 mixed-precision single-stage workload, sigma_lnK = 2.0, field seed 3, 6 levels."""
    return cube_3d(129, 2.0, 3, levels=6)


def cube_c4() -> Scenario:
    """257^3 LIMEX workload, sigma_lnK = 1.5 plus three low-K slabs, field seed 4, 6 levels."""
    return cube_3d(257, 1.5, 4, layers=True, levels=6)


def cube_c4_scaled(n: int = 33, levels: Optional[int] = None) -> Scenario:
    """The 257^3 LIMEX recipe (sigma_lnK 1.5, field seed 4, three low-K slabs at
    z = 0.25, 0.5, 0.75, the same injection patch) on a smaller cube: slabs 2 cells
    thick, the correlation length the same 1/32 of the domain."""
    return cube_3d(n, 1.5, 4, corr_cells=(n - 1) / 32.0, layers=True, levels=levels, layer_cells=2.0)


# ---------------------------------------------------------------------------------
# Serving workload: Poisson arrivals of independent single-stage requests.
# ---------------------------------------------------------------------------------
SERVE_SIZES = (33, 65, 97, 129)
SERVE_WEIGHTS = (0.4, 0.3, 0.2, 0.1)
SERVE_LEVELS = {33: 4, 65: 5, 97: 5, 129: 6}


@dataclass
class Request:
    rid: int
    arrival: float     # seconds after the start of the run
    n: int
    sigma: float
    rate: float
    field_seed: int


def serving_requests(count: int = 256, rate_per_s: float = 40.0, seed: int = 5) -> List[Request]:
    """Poisson arrivals (exponential gaps) with grid sizes drawn from SERVE_SIZES with
    SERVE_WEIGHTS, sigma_lnK ~ U[0.5, 2], injection rate ~ U[0.02, 0.1]; request r
    uses field seed 1000 + r and parameter seed 2000 + r."""
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(1.0 / rate_per_s, size=count)
    t = np.cumsum(gaps) - gaps[0]
    out = []
    for r in range(count):
        prng = np.random.default_rng(2000 + r)
        n = int(prng.choice(SERVE_SIZES, p=SERVE_WEIGHTS))
        sigma = float(prng.uniform(0.5, 2.0))
        q = float(prng.uniform(0.02, 0.1))
        out.append(Request(r, float(t[r]), n, sigma, q, 1000 + r))
    return out


def request_scenario(req: Request, field_cache: Optional[np.ndarray] = None) -> Scenario:
    return cube_3d(req.n, req.sigma, req.field_seed, rate=req.rate,
                   levels=SERVE_LEVELS.get(req.n), field_cache=field_cache)


def small_cube(n: int = 9, sigma: float = 1.0, seed: int = 11, levels: Optional[int] = None,
               sn0: float = 0.05, corr_cells: float = 2.0) -> Scenario:
    """Small 3D case for parity tests (same recipe as cube_3d, shorter correlation)."""
    return cube_3d(n, sigma, seed, corr_cells=corr_cells, sn0=sn0, levels=levels)


def perturbed_state(scn: Scenario, seed: int, dp: float = 50.0, sn_lo: float = 0.02,
                    sn_hi: float = 0.6) -> np.ndarray:
    """A generic non-equilibrium state: hydrostatic-ish pressure plus noise and a
    random saturation in [sn_lo, sn_hi], Dirichlet DoFs kept at their values.  Used to
    exercise every branch of the discretisation in parity tests."""
    rng = np.random.default_rng(seed)
    u = scn.u0.copy()
    u[:, 0] = u[:, 0] + dp * rng.standard_normal(scn.nverts)
    u[:, 1] = rng.uniform(sn_lo, sn_hi, size=scn.nverts)
    m = scn.dir_mask
    u[:, 0] = np.where(m & 1, scn.dir_value[:, 0], u[:, 0])
    u[:, 1] = np.where(m & 2, scn.dir_value[:, 1], u[:, 1])
    return u
