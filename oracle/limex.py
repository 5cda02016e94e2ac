"""LIMEX step: linearly implicit Euler substeps with a frozen matrix, extrapolation
tableau, scaled error norm and step-size rule (Section 4).

Paper passages followed:
  * semi-discrete form M(u) u' = F(u) and the linearly implicit Euler step
    (M(u_old) - tau J(u_old)) (u_new - u_old) = tau F(u_old), J = F_u exact;
  * step-size rule tau_new = (rho TOL / [[eps]])^(1/(q+1)) tau_old with q = 2;
  * error estimate [[eps]] = relative error in the scaled norm
    |||u|||^2 = alpha ||grad p||^2 + beta ||S_w||^2 (Eq. norm_u).  Eqs. norm_uw and norm_un
    derive it from the convective parts of both mass balances, which the pressure
    whose gradient drives them controls: p_n in the paper's (p_n, S_w) form, p_w in the
    (p_w, S_n) form used here (v_w and the convective v_n' both move with grad p_w).
Readings: harmonic stage sequence n_j = j, stage j takes j
substeps of H/j with M and J frozen at the step's initial state and F re-evaluated at
every substep; Aitken-Neville extrapolation
  T_{j,l+1} = T_{j,l} + (T_{j,l} - T_{j-1,l}) / (n_j / n_{j-l} - 1);
eps = |||T_kk - T_{k,k-1}||| / |||T_kk||| with alpha = 1/(2 ||grad p_w(T_kk)||^2),
beta = 1/(2 ||S_w(T_kk)||^2), so eps^2 = (e_p^2 + e_S^2)/2; accept iff eps <= TOL;
tau_new = min(tau_max, H (rho TOL / eps)^(1/3)).
"""
from __future__ import annotations

import numpy as np


def extrapolate(T1):
    """Aitken-Neville tableau from the first column T1[j-1] = T_{j,1}, n_j = j.
    Returns (T_kk, T_{k,k-1})."""
    k = len(T1)
    tab = [[t] for t in T1]
    for j in range(1, k):            # row index j (0-based) = stage j+1
        nj = j + 1
        for l in range(1, j + 1):     # build T_{j+1, l+1}
            njl = nj - l
            prev = tab[j][l - 1]
            tab[j].append(prev + (prev - tab[j - 1][l - 1]) / (nj / njl - 1.0))
    kk = tab[k - 1][k - 1]
    km = tab[k - 1][k - 2] if k > 1 else tab[k - 1][0]
    return kk, km


def step_size(H, eps, tol, safety, dt_max, q=2):
    return min(dt_max, H * (safety * tol / max(eps, 1e-300)) ** (1.0 / (q + 1)))


class StageSolveFailed(Exception):
    """A stage solve missed its tolerance within its iteration cap or broke down."""


def limex_step(u0, H, k, rhs, stage_solve, err_ratio, tol, safety, dt_max):
    """Generic LIMEX step.

    rhs(v)            -> F(v)
    stage_solve(h)    -> callable solving (M(u0)/h - J(u0)) x = f; raises
                         StageSolveFailed when the linear solve fails
    err_ratio(kk, km) -> eps
    Returns (u_new_or_u0, accepted, eps, dt_next, T_kk).

    A failed stage solve rejects the step (the paper gives no rule for it; a
    linearly implicit step that cannot be solved is treated as too long): eps = inf,
    the next step is a quarter of this one, and the remaining stages are skipped.
    """
    F0 = rhs(u0)
    T1 = []
    try:
        for j in range(1, k + 1):
            solve = stage_solve(H / j)
            v = u0.copy()
            for m in range(j):
                f = F0 if m == 0 else rhs(v)
                v = v + solve(f)
            T1.append(v)
    except StageSolveFailed:
        return u0, False, float("inf"), min(dt_max, 0.25 * H), None
    kk, km = extrapolate(T1)
    eps = err_ratio(kk, km)
    acc = eps <= tol
    dt_next = step_size(H, eps, tol, safety, dt_max)
    return (kk if acc else u0), acc, eps, dt_next, kk


class Norms:
    """H1-seminorm of the pressure (exact integral of the Q1 interpolant, 2-point
    Gauss rule per axis) and lumped L2 norm of S_w on the box-method grid."""

    def __init__(self, fv):
        self.fv = fv
        d = fv.d
        g = 0.5 / np.sqrt(3.0)
        self.qp = []
        import itertools
        for pt in itertools.product((0.5 - g, 0.5 + g), repeat=d):
            xi = np.array(pt)
            grads = np.stack([fv.grad(xi, a) for a in range(d)])  # (d, 2^d)
            self.qp.append(grads)
        self.w = fv.vol / len(self.qp)
        dual = np.zeros(fv.N)
        for l in range(fv.nc):
            np.add.at(dual, fv.cv[:, l], fv.scv)
        self.dual = dual

    def grad_sq(self, p):
        pc = p[self.fv.cv]
        tot = 0.0
        for G in self.qp:
            gv = pc @ G.T  # (Ncells, d)
            tot += float(np.sum(gv * gv)) * self.w
        return tot

    def sat_sq(self, sw):
        return float(np.sum(self.dual * sw * sw))

    def err_ratio(self, kk, km):
        """[[eps]] of Eq. norm_u between T_kk and T_{k,k-1} (flat or (N, 2) states):
        sqrt((||grad dp_w||^2 / ||grad p_w(kk)||^2 + ||dS_w||^2 / ||S_w(kk)||^2) / 2)."""
        kk = kk.reshape(-1, 2)
        km = km.reshape(-1, 2)
        dp = kk[:, 0] - km[:, 0]
        ds = -(kk[:, 1] - km[:, 1])
        gp = max(self.grad_sq(kk[:, 0]), 1e-300)
        gs = max(self.sat_sq(1.0 - kk[:, 1]), 1e-300)
        e2 = 0.5 * (self.grad_sq(dp) / gp + self.sat_sq(ds) / gs)
        return float(np.sqrt(e2))
