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
    def __init__(self, scn, levels=None, omega=2.0 / 3.0, nu1=2, nu2=2, smoother="jacobi"):
        self.scn = scn
        self.smoother = smoother
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
                                self.omega, self.nu1, self.nu2, S0=S0, T0=T0, smoother=self.smoother)
        return self.A

    def solve(self, f, rtol=1e-10, maxit=500):
        return _kr.bicgstab(self.A, f, self.H.vcycle, rtol, maxit)

    def project_pressure(self, u, h_p=1e-6, rtol=1e-10, atol=0.0, max_newton=20, lin_rtol=1e-12, maxit=500):
        """Makes the pressure of u consistent with the saturation (reading of the
        index-1 structure of M(u) u' = F(u), Section 4: the pressure column has no
        storage, so p is algebraic).  Newton at fixed S on the stage system with a
        vanishing step h_p: A(u; h_p) delta = F(u), p += delta_p, S untouched; as h_p -> 0
        the pressure update is the Newton step of the volume balance
        F_w/rho_w + F_n/rho_n = 0 (the storage of the two phases cancels in it).  Stops
        when max|delta_p| <= max(atol, rtol max|p|).  Returns (u, info)."""
        v = np.asarray(u, np.float64).reshape(-1, 2).copy()
        hist = []
        for k in range(1, max_newton + 1):
            self.assemble(v.ravel(), h_p)
            x, st = self.solve(self.residual(v.ravel()), lin_rtol, maxit)
            dp = x.reshape(-1, 2)[:, 0]
            v[:, 0] += dp
            step = float(np.abs(dp).max())
            hist.append(step)
            if step <= max(atol, rtol * float(np.abs(v[:, 0]).max())):
                return v.ravel(), dict(newton=k, converged=True, history=hist)
        return np.asarray(u, np.float64).ravel().copy(), dict(newton=max_newton, converged=False, history=hist)

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


class StallRule:
    """When the error estimate stops falling with the step (the floor that an
    inconsistent algebraic pressure leaves, which no step size removes), the pressure
    is to be projected.  Within a run of rejections the first rejection is the
    reference (tau_r, eps_r); a later rejection at a step tau <= tau_r / 2 either
    confirms the decrease (eps <= eps_r / 2; it becomes the reference) or asks for a
    projection (eps > eps_r / 2; for a smooth error eps ~ tau^2 would have fallen about
    fourfold).  A failed stage solve (eps = inf) leaves the reference as it is; an
    accepted step clears it."""

    def __init__(self):
        self.ref = None

    def after_step(self, accepted, tau, eps):
        """True when the state's pressure should be projected before the next attempt."""
        if accepted:
            self.ref = None
            return False
        if not np.isfinite(eps):
            return False
        if self.ref is None:
            self.ref = (tau, eps)
            return False
        if tau <= 0.5 * self.ref[0]:
            if eps > 0.5 * self.ref[1]:
                self.ref = None
                return True
            self.ref = (tau, eps)
        return False
