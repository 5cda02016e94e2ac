"""Host-side time loop over tpf_limex_step (the adaptive LIMEX integration of Section 4)
with the consistency rule for the algebraic pressure.

With incompressible phases the pressure is the algebraic unknown of M(u) u' = F(u).
An accepted, extrapolated state can violate the discrete volume balance by more than
a linearised correction with the Jacobian frozen at that state restores (near upwind
switches the constraint is kinked); the stages of every later step then differ by an
amount that does not vanish with the step, the error estimate stalls above TOL and
the step size collapses.  The rule: within a run of rejected steps, the first is the
reference (tau_r, eps_r); a rejection at tau <= tau_r / 2 whose eps has not fallen below
eps_r / 2 (a smooth error, eps ~ tau^2, would have fallen about fourfold) triggers
tpf_project_pressure (Newton at fixed saturation onto the volume balance) before the
next attempt; a rejection whose eps did fall becomes the new reference; failed stage
solves (eps = inf) leave the reference alone; an accepted step clears it.
"""
from __future__ import annotations

import math


class StallDetector:
    """The trigger of the consistency rule (see the module docstring)."""

    def __init__(self):
        self.tau_ref = None
        self.eps_ref = None

    def project_next(self, accepted: bool, tau: float, eps: float) -> bool:
        if accepted:
            self.tau_ref = self.eps_ref = None
            return False
        if not math.isfinite(eps):
            return False
        if self.tau_ref is None:
            self.tau_ref, self.eps_ref = tau, eps
            return False
        if tau > 0.5 * self.tau_ref:
            return False
        if eps > 0.5 * self.eps_ref:
            self.tau_ref = self.eps_ref = None
            return True
        self.tau_ref, self.eps_ref = tau, eps
        return False


def limex_run(grid_at, u, t, t_end, dt, stages, tol, safety, dt_max, rtol, maxit=500, max_attempts=1_000_000,
              consistency=True, h_p=1e-6, on_step=None, max_accepted=None, stop=None):
    """Adaptive LIMEX steps on the device state u (in place) from t to t_end.

    grid_at(t) -> (grid, t_stop): the grid to step with at time t and the time up to
    which it applies (steps are shortened to land on t_stop; a scenario whose sources
    switch off takes a second grid from then on).  on_step(record) is called after
    every attempt; the run also ends after max_accepted accepted steps or when stop()
    returns True.  Returns a
    summary: steps accepted/rejected, stage solves, BiCGSTAB iterations, failed
    solves, projections, the time reached and the step sequence."""
    det = StallDetector()
    acc = rej = solves = iters = unconv = proj = proj_newton = proj_lin = 0
    dts = []
    while t < t_end * (1.0 - 1e-14) and acc + rej < max_attempts and (max_accepted is None or acc < max_accepted):
        if stop is not None and stop():
            break
        g, t_stop = grid_at(t)
        dt = min(dt, min(t_stop, t_end) - t)
        tau = dt
        ok, t, dt_next, st = g.limex_step(u, t, dt, stages=stages, tol=tol, safety=safety, dt_max=dt_max,
                                          rtol=rtol, maxit=maxit)
        acc += ok
        rej += not ok
        solves += st["solves"]
        iters += st["iters_total"]
        unconv += st["unconverged"]
        dts.append(tau)
        projected = None
        if consistency and det.project_next(ok, tau, st["eps"]):
            done, pst = g.project_pressure(u, h_p=h_p)
            proj += 1
            proj_newton += pst["newton"]
            proj_lin += pst["linear_iters"]
            projected = {"converged": bool(done), "newton": pst["newton"], "dp_max": pst["defect0"]}
        if on_step is not None:
            on_step(dict(attempt=acc + rej, accepted=bool(ok), t=t, dt=tau, eps=st["eps"], solves=st["solves"],
                         iters=st["iters_total"], unconverged=st["unconverged"], projected=projected))
        dt = dt_next
    return dict(accepted=acc, rejected=rej, t=t, solves=solves, bicgstab_iterations=iters, unconverged=unconv,
                projections=proj, projection_newton=proj_newton, projection_linear_iters=proj_lin,
                dt_sequence=dts)
