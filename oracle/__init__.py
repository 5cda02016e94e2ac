"""FP64 CPU oracle for the two-phase (p_w, S_n) vertex-centred FV / LIMEX / BiCGSTAB+GMG
stage solver.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
`cpu_baseline` leg of `bench.py` may import this package.  The product path (the HIP
library and its Python binding) never imports, calls or links anything here, and this
package never imports the product path: the only code both sides share is the seeded
input description in `workloads/`, which holds none of the method's arithmetic.

It is written for clarity, not speed: NumPy/SciPy in float64, vectorised over cells,
with the Jacobian obtained from its definition J = dF/du by complex-step
differentiation (exact to rounding away from the branch points of the upwind and
interface rules; the branch taken at the evaluated state is frozen).

Modules
  fv      geometry of the box method on Q1 cells, Brooks-Corey-Burdine laws, the
          p_dmin interface condition, storage m(u), residual F(u), J, M, stage matrix
  gmg     per-component prolongation (linear p_w, aggregated S_n), Galerkin hierarchy
          with lumped coarse storage, damped 2x2 block Jacobi,
          V(nu1, nu2) cycle with a dense LU solve on the coarsest level
  krylov  right-preconditioned BiCGSTAB
  limex   linearly implicit Euler substeps, extrapolation tableau, scaled error norm
          and step-size rule

Parity status of each function is stated in its docstring; every function is pinned
by the `-m "not gpu"` tests in tests/test_oracle_*.py except where it says
"parity unpinned".
"""
