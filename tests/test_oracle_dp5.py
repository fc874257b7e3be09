"""Pins of the oracle's fixed-step Dormand-Prince 5(4) stepper (CPU only).

The paper's solver is Diffrax's Dopri5 (section "Numerical approach"); the
oracle takes its tableau with a fixed step.  What fixes it independently of
the code that steps with it:

* the tableau satisfies Butcher's order conditions (all 17 up to order 5 for
  the solution weights, all 8 up to order 4 for the embedded ones) and
  c_i = sum_j a_ij; its first-same-as-last row b = a_7;
* it is the tableau scipy's RK45 (also Dormand-Prince) ships;
* stepping the SWF equation, the error at t_in falls at order 5 in dt, the
  BW amplitude integrated with the tableau's weights too, and the embedded
  estimate of one step falls at order 5.
"""
from fractions import Fraction as Fr

import numpy as np
import pytest
from scipy.integrate import RK45

import swf_workloads as W
from oracle import bw
from oracle.swf import DP5_A, DP5_B, DP5_BHAT, DP5_C, SWFSolve

pytestmark = pytest.mark.filterwarnings("ignore")


def _tableau():
    n = 7
    A = np.zeros((n, n))
    for i, row in enumerate(DP5_A):
        A[i, :len(row)] = row
    return A, np.array(DP5_B), np.array(DP5_BHAT), np.array(DP5_C)


def _order_conditions(A, b, c, order):
    """(value, exact) of Butcher's conditions up to `order` (rooted trees)."""
    Ac = A @ c
    Ac2 = A @ c ** 2
    AAc = A @ Ac
    conds = [(b.sum(), 1), (b @ c, Fr(1, 2)),
             (b @ c ** 2, Fr(1, 3)), (b @ Ac, Fr(1, 6))]
    if order >= 4:
        conds += [(b @ c ** 3, Fr(1, 4)), (b @ (c * Ac), Fr(1, 8)), (b @ Ac2, Fr(1, 12)), (b @ AAc, Fr(1, 24))]
    if order >= 5:
        conds += [(b @ c ** 4, Fr(1, 5)), (b @ (c ** 2 * Ac), Fr(1, 10)), (b @ Ac ** 2, Fr(1, 20)),
                  (b @ (c * Ac2), Fr(1, 15)), (b @ (A @ c ** 3), Fr(1, 20)), (b @ (c * AAc), Fr(1, 30)),
                  (b @ (A @ (c * Ac)), Fr(1, 40)), (b @ (A @ Ac2), Fr(1, 60)), (b @ (A @ AAc), Fr(1, 120))]
    return conds


def test_tableau_order_conditions():
    A, b, bh, c = _tableau()
    assert np.allclose(A.sum(axis=1), c, atol=1e-15)
    assert np.array_equal(A[6], b)                       # first same as last
    c5 = _order_conditions(A, b, c, 5)
    assert len(c5) == 17
    for val, exact in c5:
        assert val == pytest.approx(float(exact), abs=1e-14)
    for val, exact in _order_conditions(A, bh, c, 4):
        assert val == pytest.approx(float(exact), abs=1e-14)
    # the embedded weights are a different (fourth-order) solution
    assert any(abs(v - float(e)) > 1e-6 for v, e in _order_conditions(A, bh, c, 5)[8:])


def test_tableau_is_scipys_rk45():
    A, b, bh, c = _tableau()
    assert np.allclose(RK45.C, c[:6], rtol=0, atol=1e-15)
    assert np.allclose(RK45.A, A[:6, :5], rtol=0, atol=1e-15)
    assert np.allclose(RK45.B, b[:6], rtol=0, atol=1e-15)
    assert np.allclose(RK45.E, bh - b, rtol=0, atol=1e-15)   # scipy's error weights bhat - b


def _problem(dt, scheme="dp5", t_half=4.0):
    L = 30.0
    F = [W.Term(1, 0.9, W.gauss(1.5), [W.sech2(3.0), W.const(), W.const()]),
         W.Term(0, 0.4, W.sech2(1.2, c=0.3), [W.gauss(2.5, c=-0.5), W.const(), W.const()])]
    return W.Problem("dp5", [W.Grid(1, [64, 1, 1], [L, 1, 1])], [F],
                     [W.Solve(W.U_OUT, 1, [2 * np.pi * 3 / L, 0.2, 0.0])],
                     W.Window(-t_half, t_half, dt, scheme))


def test_solve_converges_at_order_5():
    ref = SWFSolve(_problem(0.0125), 0).run()
    errs = [np.abs(SWFSolve(_problem(dt), 0).run() - ref).max() for dt in (0.1, 0.05)]
    assert errs[1] < 1e-6 * np.abs(ref).max()
    assert 25.0 < errs[0] / errs[1] < 40.0, errs
    # the same window with RK4 at the larger step is less accurate
    rk4 = SWFSolve(_problem(0.1, "rk4"), 0).run()
    assert np.abs(rk4 - ref).max() > 5.0 * errs[0]


def test_embedded_estimate_order_5():
    sv = SWFSolve(_problem(0.1), 0)
    y = sv.run(count=30)                     # a state with the field on
    sizes = []
    for dt in (0.1, 0.05):
        s2 = SWFSolve(_problem(dt), 0)
        n = int(round((s2.window.t_out - sv.time(30)) / dt))
        assert abs(s2.time(n) - sv.time(30)) < 1e-12
        _, e = s2.dp5_error(n, y)
        sizes.append(np.abs(e).max())
    assert 20.0 < sizes[0] / sizes[1] < 45.0, sizes


def test_bw_amplitude_with_dp5_weights_converges_at_order_5():
    P = 2 * np.pi * 4 / 160.0

    def amp(dt):
        prob = W.config_bw_1d(P=P, n=128, L=160.0, dt=dt, t_half=25.0)
        prob.window = W.Window(prob.window.t_in, prob.window.t_out, dt, "dp5")
        return bw.Vertex(prob, 0).amplitude()["terms"]

    # (b,s) and (s,b) converge at order 5 (ratio ~30 when dt halves); the
    # (s,s) term, bilinear in the two stepped waves, converges faster here
    # (ratio ~65).  Weights of a lower-order rule would give ratios <= 16.
    ref = amp(0.025)
    e = [np.abs(amp(dt) - ref) / np.abs(ref) for dt in (0.2, 0.1)]
    assert np.all(e[1] < 1e-7)
    ratio = e[0] / e[1]
    assert np.all((ratio[1:] > 24.0) & (ratio[1:] < 40.0)) and 24.0 < ratio[0] < 80.0, ratio
