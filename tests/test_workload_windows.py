"""The workloads' time windows against the field's residual at their ends
(CPU, oracle only).

The pair marginal is read at t_in, where the field must be negligible (the
text around eq. (Nmn)): a field still on at t_in leaves a spurious pair
content of order |A(t_in)|^2 in the scattered wave.  One-dimensional analogues
(the same time profile, amplitude and spatial width along x, the transverse
momentum on trivial axes, 128 points over the same length, dt = 0.05) show
* the ragged batch's widest draw (Gaussian, tau = 15) has converged with the
  [-80, 80] window the workload uses: doubling the window moves P by < 1%;
* the (3+1)D Schwinger workload's stated window [-50, 50] (sech^2(t/8), still
  1.5e-5 of its peak at the ends) gives a P that is thousands of times the
  converged one, which [-100, 100] reaches to a few per cent.
"""
import numpy as np
import pytest

import swf_workloads as W
from oracle import observables as ob
from oracle.swf import SWFSolve


def marginal_1d(terms, L, p, t_half, n=128, dt=0.05):
    prob = W.Problem("window", [W.Grid(1, [n, 1, 1], [L, 1.0, 1.0])], [terms], [W.Solve(0, 1, list(p))],
                     W.Window(-t_half, t_half, dt))
    sv = SWFSolve(prob, 0)
    return ob.marginal(sv, sv.run())


def test_ragged_batch_widest_draw_window_has_converged():
    prob = W.config_ragged_2d()
    assert prob.window.t_out == 80.0 and prob.window.t_in == -80.0
    i = int(np.argmax([f[0].ft.w for f in prob.fields]))
    f = prob.fields[i][0]
    assert f.ft.w > 14.9
    terms = [W.Term(1, f.amp, W.gauss(f.ft.w), [W.gauss(f.fx[0].w), W.const(), W.const()])]
    p = prob.solves[i].p
    p1 = (p[0], 0.0, p[1])                       # the y momentum on a trivial axis
    P80 = marginal_1d(terms, 160.0, p1, 80.0)
    P160 = marginal_1d(terms, 160.0, p1, 160.0)
    P60 = marginal_1d(terms, 160.0, p1, 60.0)
    assert abs(P80 - P160) < 1e-2 * P160
    assert P60 > 100 * P160                      # the shorter window is dominated by the residual field


def test_3d_workload_stated_window_is_dominated_by_the_residual_field():
    prob = W.config_3d()
    assert prob.window.steps == 4000
    f = prob.fields[0][0]
    terms = [W.Term(3, f.amp, W.sech2(f.ft.w), [W.gauss(f.fx[0].w), W.const(), W.const()])]
    P50 = marginal_1d(terms, 120.0, (0.0, 0.0, 0.0), 50.0)
    P100 = marginal_1d(terms, 120.0, (0.0, 0.0, 0.0), 100.0)
    P120 = marginal_1d(terms, 120.0, (0.0, 0.0, 0.0), 120.0)
    assert P50 > 1000 * P100
    assert abs(P100 - P120) < 0.05 * P120
