"""Geometric multigrid preconditioner on structured vertex grids (FP64, SciPy sparse).

The paper names a geometric multigrid preconditioner for BiCGSTAB (Section 1 and the
solver settings opening Section 5) without giving its components.  Reading used
here:
  * levels by vertex halving n -> (n-1)/2 + 1 along every active axis;
  * prolongation P = per-component (bi/tri)linear interpolation from level l+1 to l;
    on the finest level the rows of P at Dirichlet components are zero;
  * restriction R = P^T; coarse operators are Galerkin products of the flux part
    plus a lumped storage part:
        A_{l+1} = P^T (A'_l - S'_l) P + S_{l+1},
        S_{l+1} = row-sum lumping of P^T S'_l P placed on the S_n column,
    where S_0 = M(u0)/h (zero on Dirichlet rows) is the box method's diagonal storage,
    A'_l = A_l and S'_l = S_l on the coarse levels, and on the finest level
    A'_0 = T A_0, S'_0 = T S_0 with the volume-balance row transform T below;
  * volume-balance form of the coarse-grid correction: T is block diagonal; at each
    vertex without a Dirichlet component it replaces the wetting-phase mass balance
    by itself plus rho_w/rho_n times the non-wetting one (rho_w times the balance of
    pore volume, whose storage cancels for incompressible phases), other rows
    unchanged.  The restriction of the finest residual is P^T T r.  The pairing of the
    linear P with the wetting equation needs the equation that carries the pressure
    Laplacian: with the mass balances as they stand, a region where the wetting phase
    is immobile (k_rw = 0, e.g. ahead of a displacement front) leaves the pressure only
    in the non-wetting equation, restricted by aggregation, and the coarse operators
    become singular; the volume balance carries the total-mobility Laplacian wherever
    either phase moves.  Block Jacobi is invariant under a block-diagonal row
    transform ((TD)^{-1} T (b - A x) = D^{-1} (b - A x)), so the finest level is
    smoothed with A_0 itself;
    The plain product P^T A P turns the diagonal storage into a 27-point
    consistent-mass block whose Jacobi spectrum reaches 27/8 > 2/omega; keeping
    the coarse storage lumped, as the box method has it on the fine grid, keeps the
    block-Jacobi smoother stable on every level;
  * smoother: damped point-block Jacobi with the 2x2 diagonal blocks D,
    x <- x + omega D^{-1} (b - A x), zero initial guess on every level;
  * optional smoother for transport along the gravity axis (not in the paper; an
    option of this implementation): damped line-block Jacobi,
    x <- x + omega A_L^{-1} (b - A x), where A_L keeps the entries of A that couple two
    DoFs of the same vertex line along the last active axis (y in 2D, z in 3D) and
    drops all others: a block tridiagonal matrix with 2x2 blocks per line.  Like
    point-block Jacobi it is invariant under the block-diagonal row transform, so it
    also smooths with A_0 itself.  It is applied here by a sparse LU of A_L, the
    plain definition;
  * V(nu1, nu2) cycle; the coarsest level is solved with a dense LU factorisation
    with partial pivoting (scipy.linalg.lu_factor / lu_solve).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla


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


def aggregate_1d(nf: int) -> sp.csr_matrix:
    """Piecewise-constant interpolation on a line: fine vertex i takes the value of
    coarse vertex (i + 1) // 2 (coarse I aggregates fine 2I - 1 and 2I)."""
    if nf == 1:
        return sp.csr_matrix(np.ones((1, 1)))
    nc = coarse_size(nf)
    rows = np.arange(nf)
    return sp.csr_matrix((np.ones(nf), (rows, (rows + 1) // 2)), shape=(nf, nc))


def prolongation(n, dim, dir_mask=None, kinds=("linear", "constant")) -> sp.csr_matrix:
    """P for interleaved DoFs (2*v + comp), vertices x-fastest; kinds[c] is the
    interpolation of component c ('linear' or 'constant')."""
    nx, ny, nz = n
    blocks = []
    for kind in kinds:
        f1 = interp_1d if kind == "linear" else aggregate_1d
        Pz = f1(nz) if dim == 3 else sp.csr_matrix(np.ones((1, 1)))
        blocks.append(sp.kron(Pz, sp.kron(f1(ny), f1(nx), format="csr"), format="csr"))
    e = [sp.csr_matrix(([1.0], ([c], [c])), shape=(2, 2)) for c in range(2)]
    P = sp.csr_matrix(sp.kron(blocks[0], e[0]) + sp.kron(blocks[1], e[1]))
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


def line_part(A: sp.csr_matrix, n, dim) -> sp.csr_matrix:
    """A_L: the entries of A between DoFs of vertices on the same line along the last
    active axis (vertices x-fastest, so the line of vertex v is v mod nx in 2D and
    v mod nx*ny in 3D)."""
    nx, ny, _ = n
    stride = nx if dim == 2 else nx * ny
    C = sp.coo_matrix(A)
    keep = (C.row // 2) % stride == (C.col // 2) % stride
    return sp.csr_matrix((C.data[keep], (C.row[keep], C.col[keep])), shape=A.shape)


def lumped_storage(P, S):
    """Row sums of P^T S P placed on the S_n column of each 2x2 diagonal block."""
    d = np.asarray((P.T @ S @ P).sum(axis=1)).ravel()
    n2 = d.size
    rows = np.arange(n2)
    cols = 2 * (rows // 2) + 1
    return sp.csr_matrix((d, (rows, cols)), shape=(n2, n2))


def volume_balance(dir_mask, rho) -> sp.csr_matrix:
    """The row transform T of the coarse-grid correction (module docstring): identity,
    plus rho_w/rho_n in the (w, n) position of every vertex without a Dirichlet
    component."""
    N = dir_mask.size
    free = np.nonzero(dir_mask == 0)[0]
    rows = np.concatenate([np.arange(2 * N), 2 * free])
    cols = np.concatenate([np.arange(2 * N), 2 * free + 1])
    vals = np.concatenate([np.ones(2 * N), np.full(free.size, rho[0] / rho[1])])
    return sp.csr_matrix((vals, (rows, cols)), shape=(2 * N, 2 * N))


class Hierarchy:
    def __init__(self, A0, n, dim, levels, dir_mask, omega=2.0 / 3.0, nu1=2, nu2=2, S0=None, T0=None,
                 smoother="jacobi"):
        """S0: storage part of A0 (block diagonal, S_n column only); None means zero.
        T0: row transform of the finest level for the coarse-grid correction (None:
        identity).  smoother: 'jacobi' (point-block) or 'line' (line-block along the
        last active axis)."""
        if smoother not in ("jacobi", "line"):
            raise ValueError(f"unknown smoother {smoother!r}")
        self.smoother = smoother
        self.sizes = level_sizes(n, dim, levels)
        self.A = [sp.csr_matrix(A0)]
        S = sp.csr_matrix(A0.shape) if S0 is None else sp.csr_matrix(S0)
        self.S = [S]
        self.T0 = sp.identity(A0.shape[0], format="csr") if T0 is None else sp.csr_matrix(T0)
        self.P = []
        for l in range(levels - 1):
            P = prolongation(self.sizes[l], dim, dir_mask if l == 0 else None)
            self.P.append(P)
            Af, Sf = self.A[-1], self.S[-1]
            if l == 0:
                Af, Sf = self.T0 @ Af, self.T0 @ Sf
            Sc = lumped_storage(P, Sf)
            Ac = P.T @ (Af - Sf) @ P + Sc
            # coarse DoFs whose prolongation column is empty (an aggregate made only
            # of Dirichlet components) are decoupled: give them a unit diagonal
            empty = np.asarray(abs(P).sum(axis=0)).ravel() == 0.0
            if empty.any():
                Ac = Ac + sp.diags(empty.astype(np.float64))
            self.A.append(sp.csr_matrix(Ac))
            self.S.append(Sc)
        self.Dinv = [block_diag_inverse(A) for A in self.A]
        self.line_lu = ([spla.splu(sp.csc_matrix(line_part(A, nl, dim))) for A, nl in zip(self.A, self.sizes)]
                        if smoother == "line" else None)
        self.lu = sla.lu_factor(self.A[-1].toarray())
        self.omega, self.nu1, self.nu2 = omega, nu1, nu2

    def smooth(self, l, x, b, sweeps):
        A, Di = self.A[l], self.Dinv[l]
        for _ in range(sweeps):
            r = b - A @ x
            if self.line_lu is not None:
                x = x + self.omega * self.line_lu[l].solve(r)
            else:
                x = x + self.omega * np.einsum("nij,nj->ni", Di, r.reshape(-1, 2)).ravel()
        return x

    def vcycle(self, b, l=0):
        """One V(nu1, nu2) cycle with zero initial guess: approximately A_l^{-1} b."""
        if l == len(self.A) - 1:
            return sla.lu_solve(self.lu, b)
        x = self.smooth(l, np.zeros_like(b), b, self.nu1)
        r = b - self.A[l] @ x
        if l == 0:
            r = self.T0 @ r
        e = self.vcycle(self.P[l].T @ r, l + 1)
        x = x + self.P[l] @ e
        return self.smooth(l, x, b, self.nu2)
