"""Fixed-step implicit Euler with Newton's method: the time-stepping baseline the paper
sets against LIMEX (Section 5: the solver settings that open the section, Case 1's
Table error1 and Case 4's Table case4_2).  TEST INFRASTRUCTURE ONLY, like the rest of
this package.

Paper passages followed:
  * the semi-discrete system M(u) u' = F(u) of Section 4, whose M(u) = dm/du is the
    derivative of the box-method storage m(u) (Section 3.1, Eqs. dsW/dpN);
  * the nonlinear iteration of the implicit Euler scheme stops at an absolute defect
    of 1e-8 or a relative one of 1e-6 (solver settings opening Section 5).
Readings taken where the paper is silent:
  * the discrete step is the conservative backward Euler step
        G(u) = m(u) - m(u_old) - tau F(u) = 0,
    whose Jacobian M(u) - tau J(u) is tau times the stage matrix A(u; h = tau) of the
    LIMEX stages, so a Newton step solves A(u_k; tau) delta = F(u_k) - (m(u_k) - m(u_old))/tau
    with unit rows (right-hand side 0) at the Dirichlet components;
  * the defect is ||G(u_k)||_2 in kg over the rows without a Dirichlet component,
    starting from u_0 = u_old (so G(u_0) = -tau F(u_old)); converged when
    ||G_k|| <= atol or ||G_k|| <= rtol ||G_0||, or when the accepted update is
    negligible, max|du_p| <= xtol max|p| and max|du_S| <= xtol (xtol = 1e-10): with
    pressures of 5e7 Pa every face flux carries ~5e-9 Pa of FP64 rounding in its
    pressure difference, which puts a floor of ~1e-7 kg under the defect of a one-day
    step on a 257 x 129 grid; once the iteration sits on that floor (a step that
    starts near equilibrium, G_0 ~ 0.1 kg) neither bar can be met and the update is
    at rounding level;
  * Newton is globalised by backtracking on the defect: a step whose defect is not
    smaller than its predecessor's is halved (at most max_halvings times in a row);
  * a step that has not converged after max_newton iterations is a failed step; the
    fixed-step driver then repeats it as two half steps (the paper does not say what
    its implicit Euler does on failure).
The linear systems are solved exactly (sparse LU): the oracle's Newton iterates are
those of the exact Newton method.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse.linalg as spla


class NewtonFailed(Exception):
    """Newton's method did not reach its tolerance within its iteration cap."""


def ie_step(fv, u_old, tau, atol=1e-8, rtol=1e-6, max_newton=30, max_halvings=8, linear_solve=None, xtol=1e-10):
    """One implicit Euler step of size tau from u_old ((N, 2) or flat) with Newton.

    fv: the oracle discretisation (oracle.fv.FV).  linear_solve(A, b) -> x, default
    sparse LU.  Returns (u_new (N, 2), info) with info = dict(newton, halvings,
    defect0, defect, converged, history, criterion = 'defect' or 'update'); raises
    NewtonFailed when max_newton is reached."""
    u_old = np.asarray(u_old, np.float64).reshape(-1, 2)
    keep = np.ones(2 * fv.N)
    keep[fv.dirichlet_dofs()] = 0.0
    m_old = fv.storage(u_old)
    solve = linear_solve or (lambda A, b: spla.spsolve(A.tocsc(), b))

    def rhs(u):
        # F(u) - (m(u) - m_old)/tau with the Dirichlet rows cleared; G = -tau * rhs
        r = fv.residual(u).ravel() - (fv.storage(u) - m_old).ravel() / tau
        return r * keep

    u = u_old.copy()
    r = rhs(u)
    d0 = tau * float(np.linalg.norm(r))
    hist = [d0]
    info = dict(newton=0, halvings=0, defect0=d0, defect=d0, converged=False, history=hist, criterion=None)
    if d0 <= atol:
        info["converged"] = True
        info["criterion"] = "defect"
        return u, info
    for k in range(1, max_newton + 1):
        A = fv.stage_matrix(u, tau)
        delta = solve(A, r).reshape(-1, 2)
        dprev = tau * float(np.linalg.norm(r))
        lam = 1.0
        for _ in range(max_halvings + 1):
            trial = u + lam * delta
            rt = rhs(trial)
            dt = tau * float(np.linalg.norm(rt))
            if dt < dprev or lam < 2.0 ** -max_halvings * 1.5:
                break
            lam *= 0.5
            info["halvings"] += 1
        step = lam * delta
        u, r = trial, rt
        hist.append(dt)
        info["newton"] = k
        info["defect"] = dt
        if dt <= atol or dt <= rtol * d0:
            info["converged"] = True
            info["criterion"] = "defect"
            return u, info
        if np.abs(step[:, 0]).max() <= xtol * np.abs(u[:, 0]).max() and np.abs(step[:, 1]).max() <= xtol:
            info["converged"] = True
            info["criterion"] = "update"
            return u, info
    raise NewtonFailed(f"Newton did not converge in {max_newton} iterations (defect {hist[-1]:.3e}, "
                       f"initial {d0:.3e})")


def ie_run(fv, u0, t_end, n_steps, **kw):
    """Fixed-step implicit Euler from t = 0 to t_end in n_steps equal steps (a step
    whose Newton iteration fails is repeated as two half steps).  Returns the final
    state and a summary (steps taken, Newton iterations, halvings, step failures)."""
    tau0 = t_end / n_steps
    u = np.asarray(u0, np.float64).reshape(-1, 2).copy()
    t = 0.0
    steps = newton = halvings = failures = 0
    todo = [tau0] * n_steps
    while todo:
        tau = todo.pop(0)
        try:
            u_new, info = ie_step(fv, u, tau, **kw)
        except NewtonFailed:
            failures += 1
            todo[:0] = [0.5 * tau, 0.5 * tau]
            continue
        u, t = u_new, t + tau
        steps += 1
        newton += info["newton"]
        halvings += info["halvings"]
    return u, dict(t=t, steps=steps, newton=newton, halvings=halvings, failures=failures)
