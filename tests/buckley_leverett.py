"""Case 1 of Section 5 (Buckley-Leverett displacement): the analytic solution, the
error norms of Eq. Lp and the paper's printed values (Table error1).

The analytic solution is the Welge construction for the fractional-flow equation
S_t + (q/Phi) f(S)_x = 0, S(x, 0) = 0, S(0, t) = 1 (S the wetting saturation,
q = 3e-7 m/s the total Darcy velocity fixed by the outflow of 3e-4 kg/(m^2 s) at
1000 kg/m^3), with f = lambda_w / (lambda_w + lambda_n), lambda_a = k_ra / mu_a and the
Brooks-Corey-Burdine laws k_rw = S^((2+3L)/L), k_rn = (1-S)^2 (1 - S^((2+L)/L)), L = 2,
no residual saturations: behind the front each S >= S* travels at (q/Phi) f'(S);
the front S* solves f'(S*) S* = f(S*) (tangent from the initial state); ahead of it
S = 0.  This module is written from that textbook construction; it shares nothing
with the oracle or the GPU path.

The norms are those of Eq. Lp over the domain, per unit height of the strip:
||e||_p = (int_Omega |S_w - S_wh|^p / H)^(1/p) with S_wh the bilinear interpolant of
the vertex values; for the y-independent displacement this is the norm along x, the
magnitude Table error1 prints.
"""
from __future__ import annotations

import numpy as np
from scipy.optimize import brentq

# Table case1 and the Case-1 text
POROSITY = 0.2
Q_TOTAL = 3e-4 / 1000.0          # m/s
MU = (1e-3, 1e-3)
LAMBDA = 2.0
LENGTH, HEIGHT = 300.0, 75.0
T_END = 1500 * 86400.0
FRONT_SPEED_PAPER = 1.84e-6      # m/s, printed
# Table error1: elements -> (time steps, L1, L2) for the LIMEX scheme and implicit Euler
PAPER_LIMEX = {64: (483, 5.797, 1.425), 128: (654, 3.225, 1.060), 256: (860, 1.768, 0.777),
               512: (1055, 0.942, 0.561)}
PAPER_IE = {64: (65, 8.739, 1.663), 128: (130, 4.951, 1.250), 256: (260, 2.766, 0.931),
            512: (520, 1.521, 0.685)}


def frac(s):
    """Wetting fractional flow f(S); accepts complex S (complex-step derivative)."""
    krw = s ** ((2.0 + 3.0 * LAMBDA) / LAMBDA)
    krn = (1.0 - s) ** 2 * (1.0 - s ** ((2.0 + LAMBDA) / LAMBDA))
    lw, ln = krw / MU[0], krn / MU[1]
    return lw / (lw + ln)


def dfrac(s):
    h = 1e-30
    return np.imag(frac(np.asarray(s, dtype=complex) + 1j * h)) / h


def front_saturation():
    return brentq(lambda s: dfrac(s) * s - frac(s).real, 0.3, 0.999, xtol=1e-15)


def front_speed():
    s = front_saturation()
    return Q_TOTAL / POROSITY * frac(s).real / s


def profile(x, t):
    """Analytic wetting saturation at positions x (m) and time t (s)."""
    x = np.asarray(x, dtype=float)
    ss = front_saturation()
    c = Q_TOTAL * t / POROSITY
    xf = c * frac(ss).real / ss
    out = np.zeros_like(x)
    behind = x < xf
    # invert x = c f'(S) on [S*, 1] (f' decreasing there) by bisection, vectorised
    lo = np.full(behind.sum(), ss)
    hi = np.ones(behind.sum())
    xb = x[behind]
    for _ in range(60):
        mid = 0.5 * (lo + hi)
        right = c * dfrac(mid) > xb
        lo = np.where(right, mid, lo)
        hi = np.where(right, hi, mid)
    out[behind] = 0.5 * (lo + hi)
    return out


def error_norms(sw_vertices, elements, t=T_END, gauss=16):
    """L1 and L2 norms (Eq. Lp, per unit height) of S_w(t) - S_wh for vertex values
    sw_vertices of shape (ny, nx) on the elements x elements/4 grid.  Composite
    Gauss-Legendre quadrature on every element, with the element that holds the
    front split at the front."""
    ny, nx = sw_vertices.shape
    assert nx == elements + 1 and ny == elements // 4 + 1
    dx, dy = LENGTH / elements, HEIGHT / (ny - 1)
    ss = front_saturation()
    xf = Q_TOTAL * t / POROSITY * frac(ss).real / ss
    gx, gw = np.polynomial.legendre.leggauss(gauss)
    # x sub-intervals: element boundaries plus the front
    edges = np.union1d(np.linspace(0.0, LENGTH, nx), [xf] if 0 < xf < LENGTH else [])
    a, b = edges[:-1], edges[1:]
    xq = (0.5 * (b - a)[:, None] * (gx[None, :] + 1.0) + a[:, None]).ravel()
    wq = (0.5 * (b - a)[:, None] * gw[None, :]).ravel()
    exact = profile(xq, t)
    yq, yw = np.polynomial.legendre.leggauss(4)
    l1 = l2 = 0.0
    for j in range(ny - 1):
        for k in range(4):
            eta = 0.5 * (yq[k] + 1.0)
            row = (1.0 - eta) * sw_vertices[j] + eta * sw_vertices[j + 1]
            e = np.abs(exact - np.interp(xq, np.linspace(0.0, LENGTH, nx), row))
            w = 0.5 * yw[k] * dy / HEIGHT
            l1 += w * np.sum(wq * e)
            l2 += w * np.sum(wq * e * e)
    return float(l1), float(np.sqrt(l2))


def rates(norms):
    """r_Lp of Eq. r_Lp between consecutive resolutions (norms: list in refinement order)."""
    return [float(np.log2(norms[i] / norms[i + 1])) for i in range(len(norms) - 1)]


def run_gpu(grid, scn, rtol=1e-10, maxit=400, log=None, max_attempts=20000):
    """Adaptive LIMEX (Table case1 step control in scn.meta) from t = 0 to T_END on the
    GPU through the C ABI; the last step is shortened to end at T_END.  Returns the
    final state (host, (N, 2)) and a summary."""
    import torch

    m = scn.meta
    u = torch.as_tensor(scn.u0.ravel().copy(), device=grid.device)
    t, dt = 0.0, m["dt0"]
    acc = rej = solves = iters = unconv = 0
    while t < T_END * (1.0 - 1e-14) and acc + rej < max_attempts:
        dt = min(dt, T_END - t)
        ok, t, dt_next, st = grid.limex_step(u, t, dt, stages=m["stages"], tol=m["tol"], safety=m["safety"],
                                             dt_max=m["dt_max"], rtol=rtol, maxit=maxit)
        acc += ok
        rej += not ok
        solves += st["solves"]
        iters += st["iters_total"]
        unconv += st["unconverged"]
        if log is not None:
            log(acc + rej, ok, t, dt, st)
        dt = dt_next
    return u.cpu().numpy().reshape(-1, 2), dict(accepted=acc, rejected=rej, t_end=t, solves=solves,
                                                iterations=iters, unconverged=unconv)
