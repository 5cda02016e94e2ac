"""Fixed-step implicit Euler with Newton (the paper's comparison scheme, Section 5).

CPU (the oracle, pinned):
  * Case 1 at 64 elements with Table error1's 65 fixed steps: the error norms
    against the analytic Welge solution reproduce the table's implicit-Euler row;
  * Newton converges quadratically on a capillary lens step (defect history);
  * the non-wetting volume of Case 1 falls by exactly the outflow q H T (p_c = 0:
    the storage is linear in S_n, and a converged step balances m(u) - m(u_old)
    against tau F(u) row by row);
  * a vanishing step leaves the state unchanged, and the conservative form holds:
    m(u_new) - m(u_old) = tau F(u_new) to the Newton tolerance.
GPU (the C ABI, marked gpu): tpf_storage and tpf_ie_step against the oracle, and the
GPU run of Case 1 against Table error1.
"""
import numpy as np
import pytest

import workloads as W
from oracle import fv as FV
from oracle import ie as IE
from tests import buckley_leverett as BL


def sn_volume(scn, sn):
    dx, dy, _ = scn.spacing
    wx = np.full(scn.n[0], dx)
    wx[[0, -1]] = dx / 2
    wy = np.full(scn.n[1], dy)
    wy[[0, -1]] = dy / 2
    return float(np.sum((wy[:, None] * wx[None, :]).ravel() * scn.poro[0] * sn))


@pytest.fixture(scope="module")
def ie64():
    scn = W.buckley_leverett(64)
    f = FV.FV(scn)
    steps = BL.PAPER_IE[64][0]
    u, info = IE.ie_run(f, scn.u0, BL.T_END, steps)
    return scn, u, info


def test_oracle_ie_case1_matches_table_error1(ie64):
    """Table error1, implicit Euler at 64 elements: 65 steps, L1 8.739, L2 1.663."""
    scn, u, info = ie64
    sw = 1.0 - u[:, 1].reshape(scn.n[1], scn.n[0])
    l1, l2 = BL.error_norms(sw, 64)
    steps, p1, p2 = BL.PAPER_IE[64]
    print(f"oracle IE 64 elements: {info}, L1 {l1:.3f} (paper {p1}), L2 {l2:.3f} (paper {p2})")
    assert info["steps"] == steps and info["failures"] == 0
    assert abs(l1 / p1 - 1) < 0.02 and abs(l2 / p2 - 1) < 0.02
    # the implicit Euler front is more smeared than LIMEX's (Table error1: 8.739 > 5.797)
    assert l1 > BL.PAPER_LIMEX[64][1]


def test_oracle_ie_case1_conserves_nonwetting_volume(ie64):
    scn, u, info = ie64
    v0 = sn_volume(scn, scn.u0[:, 1])
    v1 = sn_volume(scn, u[:, 1])
    out = BL.Q_TOTAL * BL.HEIGHT * BL.T_END    # m^3 per unit depth leaving at x = 300 m
    assert (v0 - v1) == pytest.approx(out, rel=1e-8)


def test_newton_converges_quadratically_on_a_lens_step():
    scn = W.lens_2d(17, 9)
    f = FV.FV(scn)
    u0 = W.perturbed_state(scn, 3, dp=20.0, sn_lo=0.05, sn_hi=0.3)
    u, info = IE.ie_step(f, u0, 600.0, rtol=1e-12, atol=0.0)
    h = np.array(info["history"]) / info["defect0"]
    print("defect history", h)
    assert info["converged"] and h[-1] < 1e-12
    # quadratic convergence: once in the basin, each defect is at most ~ the square
    # of the previous one (relative to the first), down to the rounding floor
    k = int(np.argmax(h < 1e-2))
    assert k > 0 and len(h) - k >= 3
    for a, b in zip(h[k:-1], h[k + 1:]):
        if b > 1e-11:
            assert b <= 50.0 * a * a, (a, b)


def test_ie_step_is_conservative_and_consistent():
    """A converged step satisfies m(u_new) - m(u_old) = tau F(u_new) on every row
    without a Dirichlet component (the defect), and small steps move the saturation
    linearly in tau."""
    scn = W.small_cube(5, seed=21)
    f = FV.FV(scn)
    u0 = W.perturbed_state(scn, 4, dp=30.0, sn_lo=0.05, sn_hi=0.4)
    tau = 200.0
    u, info = IE.ie_step(f, u0, tau, rtol=1e-12, atol=0.0)
    G = f.storage(u) - f.storage(u0) - tau * f.residual(u)
    G = G.ravel()
    keep = np.ones(2 * f.N)
    keep[f.dirichlet_dofs()] = 0.0
    assert np.linalg.norm(G * keep) <= 1e-10 * info["defect0"]
    # consistency: for small steps the saturation moves by tau M^-1 F, linearly in tau
    # (the pressure is algebraic and jumps to the constraint at once)
    u1, _ = IE.ie_step(f, u0, 0.5, rtol=1e-10, atol=0.0)
    u2, _ = IE.ie_step(f, u0, 1.0, rtol=1e-10, atol=0.0)
    d1, d2 = u1[:, 1] - u0[:, 1], u2[:, 1] - u0[:, 1]
    assert np.linalg.norm(d1) > 0 and np.linalg.norm(d2 - 2 * d1) <= 2e-2 * np.linalg.norm(d2)
