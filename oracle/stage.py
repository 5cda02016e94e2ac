"""The stage solve and the LIMEX step of one scenario, composed from the oracle parts:
assemble A = M(u0)/h - J(u0) (fv), build the Galerkin hierarchy (gmg) and solve with
right-preconditioned BiCGSTAB (krylov); LIMEX (limex) drives stages of H/j."""
from __future__ import annotations

import numpy as np

from . import fv as _fv
from . import gmg as _gmg
from . import krylov as _kr
from . import limex as _lx


class Stage:
    def __init__(self, scn, levels=None, omega=2.0 / 3.0, nu1=2, nu2=2):
        self.scn = scn
        self.fv = _fv.FV(scn)
        self.levels = scn.levels if levels is None else levels
        self.omega, self.nu1, self.nu2 = omega, nu1, nu2
        self.A = None
        self.H = None

    def residual(self, u):
        return self.fv.residual(u.reshape(-1, 2)).ravel()

    def assemble(self, u0, h, frozen=None):
        """Stage matrix and hierarchy at u0 for the step h; frozen = (M(u0), J(u0))
        reuses the matrices of an earlier stage of the same step."""
        self.A = self.fv.stage_matrix(u0.reshape(-1, 2), h, frozen=frozen)
        S0 = self.fv.storage_part(u0.reshape(-1, 2), h)
        T0 = _gmg.volume_balance(self.fv.dir_mask, self.scn.rho)
        self.H = _gmg.Hierarchy(self.A, self.scn.n, self.scn.dim, self.levels, self.fv.dir_mask,
                                self.omega, self.nu1, self.nu2, S0=S0, T0=T0)
        return self.A

    def solve(self, f, rtol=1e-10, maxit=500):
        return _kr.bicgstab(self.A, f, self.H.vcycle, rtol, maxit)

    def limex_step(self, u, H, stages=2, tol=5e-3, safety=0.75, dt_max=8.64e6, rtol=1e-10,
                   maxit=500):
        norms = _lx.Norms(self.fv)
        info = dict(iters=[], solves=0)

        frozen = []  # M(u) and J(u), shared by the stages of this step

        def stage_solve(h):
            if not frozen:
                frozen.append(self.fv.frozen_matrices(u.reshape(-1, 2)))
            self.assemble(u, h, frozen=frozen[0])

            def solve(f):
                x, st = self.solve(f, rtol, maxit)
                info["iters"].append(st["iters"])
                info["solves"] += 1
                if not np.all(np.isfinite(x)) or not st["rel_res"] <= rtol:
                    raise _lx.StageSolveFailed()
                return x
            return solve

        out, acc, eps, dt_next, kk = _lx.limex_step(u.ravel(), H, stages, self.residual, stage_solve,
                                                     norms.err_ratio, tol, safety, dt_max)
        info.update(accepted=acc, eps=eps, dt_next=dt_next)
        return out, info
