"""Geometric multigrid preconditioner on structured vertex grids (FP64, SciPy sparse).

The paper names a geometric multigrid preconditioner for BiCGSTAB (Section 1 and the
solver settings opening Section 5) without giving its components.  Reading used
here (listed in the design doc):
  * levels by vertex halving n -> (n-1)/2 + 1 along every active axis;
  * prolongation P = per-component (bi/tri)linear interpolation from level l+1 to l;
    on the finest level the rows of P at Dirichlet components are zero;
  * restriction R = P^T and Galerkin coarse operators A_{l+1} = P^T A_l P;
  * smoother: damped point-block Jacobi with the 2x2 diagonal blocks D,
    x <- x + omega D^{-1} (b - A x), zero initial guess on every level;
  * V(nu1, nu2) cycle; the coarsest level is solved with a dense LU factorisation
    with partial pivoting (scipy.linalg.lu_factor / lu_solve).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp


def coarse_size(n: int) -> int:
    return (n - 1) // 2 + 1


def interp_1d(nf: int) -> sp.csr_matrix:
    """Linear interpolation from (nf-1)/2+1 coarse to nf fine vertices on a line."""
    if nf == 1:
        return sp.csr_matrix(np.ones((1, 1)))
    nc = coarse_size(nf)
    rows, cols, vals = [], [], []
    for i in range(nf):
        if i % 2 == 0:
            rows.append(i); cols.append(i // 2); vals.append(1.0)
        else:
            rows += [i, i]; cols += [(i - 1) // 2, (i + 1) // 2]; vals += [0.5, 0.5]
    return sp.csr_matrix((vals, (rows, cols)), shape=(nf, nc))


def prolongation(n, dim, dir_mask=None) -> sp.csr_matrix:
    """P for interleaved DoFs (2*v + comp), vertices x-fastest."""
    nx, ny, nz = n
    Px, Py = interp_1d(nx), interp_1d(ny)
    Pz = interp_1d(nz) if dim == 3 else sp.csr_matrix(np.ones((1, 1)))
    Pv = sp.kron(Pz, sp.kron(Py, Px, format="csr"), format="csr")
    P = sp.kron(Pv, sp.identity(2, format="csr"), format="csr")
    if dir_mask is not None:
        keep = np.ones(P.shape[0])
        keep[2 * np.nonzero(dir_mask & 1)[0]] = 0.0
        keep[2 * np.nonzero(dir_mask & 2)[0] + 1] = 0.0
        P = sp.csr_matrix(sp.diags(keep) @ P)
    return P


def level_sizes(n, dim, levels):
    out = [tuple(n)]
    for _ in range(levels - 1):
        nx, ny, nz = out[-1]
        out.append((coarse_size(nx), coarse_size(ny), coarse_size(nz) if dim == 3 else 1))
    return out


def block_diag_inverse(A: sp.csr_matrix) -> np.ndarray:
    """Inverses of the 2x2 diagonal blocks of A, shape (N, 2, 2)."""
    d0 = A.diagonal(0)
    up = A.diagonal(1)[0::2]
    lo = A.diagonal(-1)[0::2]
    a, dd = d0[0::2], d0[1::2]
    b, c = up, lo
    det = a * dd - b * c
    inv = np.empty((a.size, 2, 2))
    inv[:, 0, 0] = dd / det
    inv[:, 0, 1] = -b / det
    inv[:, 1, 0] = -c / det
    inv[:, 1, 1] = a / det
    return inv


class Hierarchy:
    def __init__(self, A0, n, dim, levels, dir_mask, omega=2.0 / 3.0, nu1=2, nu2=2):
        self.sizes = level_sizes(n, dim, levels)
        self.A = [sp.csr_matrix(A0)]
        self.P = []
        for l in range(levels - 1):
            P = prolongation(self.sizes[l], dim, dir_mask if l == 0 else None)
            self.P.append(P)
            self.A.append(sp.csr_matrix(P.T @ self.A[-1] @ P))
        self.Dinv = [block_diag_inverse(A) for A in self.A]
        self.lu = sla.lu_factor(self.A[-1].toarray())
        self.omega, self.nu1, self.nu2 = omega, nu1, nu2

    def smooth(self, l, x, b, sweeps):
        A, Di = self.A[l], self.Dinv[l]
        for _ in range(sweeps):
            r = (b - A @ x).reshape(-1, 2)
            x = x + self.omega * np.einsum("nij,nj->ni", Di, r).ravel()
        return x

    def vcycle(self, b, l=0):
        """One V(nu1, nu2) cycle with zero initial guess: approximately A_l^{-1} b."""
        if l == len(self.A) - 1:
            return sla.lu_solve(self.lu, b)
        x = self.smooth(l, np.zeros_like(b), b, self.nu1)
        r = b - self.A[l] @ x
        e = self.vcycle(self.P[l].T @ r, l + 1)
        x = x + self.P[l] @ e
        return self.smooth(l, x, b, self.nu2)
