"""Right-preconditioned BiCGSTAB (van der Vorst 1992), FP64.

The paper solves every stage system with BiCGSTAB preconditioned by geometric
multigrid (Section 1; solver settings at the start of Section 5).  Variant used:
x0 = 0, shadow residual r^ = r0 = b, stop when
||r||_2 <= rtol ||b||_2 on the recursively updated residual, then report the true
residual ||b - A x|| / ||b|| recomputed from x.  A zero (t, t) gives omega = 0; a zero
rho restarts once with r^ = r.
"""
from __future__ import annotations

import numpy as np


def bicgstab(A, b, prec, rtol=1e-10, maxit=500):
    bnorm = float(np.linalg.norm(b))
    x = np.zeros_like(b)
    if bnorm == 0.0:
        return x, dict(iters=0, rel_res=0.0, rel_res_true=0.0)
    r = b.copy()
    rhat = r.copy()
    p = np.zeros_like(b)
    v = np.zeros_like(b)
    rho_old = alpha = omega = 1.0
    rho = float(rhat @ r)
    it = 0
    restarted = False
    rel = 1.0
    first = True
    for it in range(1, maxit + 1):
        if first:
            p = r.copy()
            first = False
        else:
            beta = (rho / rho_old) * (alpha / omega)
            p = r + beta * (p - omega * v)
        phat = prec(p)
        v = A @ phat
        alpha = rho / float(rhat @ v)
        s = r - alpha * v
        shat = prec(s)
        t = A @ shat
        tt = float(t @ t)
        omega = float(t @ s) / tt if tt > 0.0 else 0.0
        x = x + alpha * phat + omega * shat
        r = s - omega * t
        rho_old = rho
        rho = float(rhat @ r)
        rel = float(np.linalg.norm(r)) / bnorm
        if rel <= rtol:
            break
        if rho == 0.0 and not restarted:
            rhat = r.copy()
            rho = float(rhat @ r)
            restarted = True
            first = True
    true = float(np.linalg.norm(b - A @ x)) / bnorm
    return x, dict(iters=it, rel_res=rel, rel_res_true=true)
