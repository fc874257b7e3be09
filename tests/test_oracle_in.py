"""Pins of the oracle's in-states (CPU only).

U_in and V_in (section "Scattered wave functions": plane waves as t -> -inf)
are stepped forward from psi_scat(t_in) = 0 and read at t_out.  What fixes
them independently of the code that steps them:

* no field, no scattered wave; a pure gauge A = d Lambda gives the closed
  form psi_scat = (e^{-i Lambda} - 1) psi_back at every time;
* the overlap of two exact solutions is time independent, so an in-state
  read at t_out and an out-state read at t_in give the same Bogoliubov
  coefficient: (U_back|V_scat^in)(t_out) = (U_scat^out|V_back)(t_in) and
  (U_scat^in|V_back)(t_out) = (U_back|V_scat^out)(t_in), to RK4's order 4
  (lattice momenta: the background is an exact lattice solution, so the
  semi-discrete evolution is unitary);
* summed over a complete set of lattice modes the in- and out-state
  marginals balance: sum P_e^out = sum P_pos^in and sum P_e^in = sum P_pos^out;
* at first order in the field the in-state forms are minus the out-state
  amplitude Omega of eq. (Nmn), and form 1 = -form 2 for in-states too.
"""
import numpy as np
import pytest

import swf_workloads as W
from oracle import observables as ob
from oracle.swf import SWFSolve

pytestmark = pytest.mark.filterwarnings("ignore")


def test_in_state_without_field_stays_zero():
    prob = W.Problem("free", [W.Grid(1, [32, 1, 1], [20.0, 1, 1])], [[]], [W.Solve(W.U_IN, 1, [0.3, 0.2, 0.0])],
                     W.Window(-2.0, 2.0, 0.05))
    sv = SWFSolve(prob, 0)
    assert sv.forward and sv.t_end == 2.0
    assert np.abs(sv.run()).max() == 0.0


def test_in_state_pure_gauge_closed_form_2d():
    lam0, tau, w, n, L = 0.7, 2.0, 3.0, 40, 24.0
    p = [2 * np.pi * 2 / L, -2 * np.pi / L, 0.3]
    for kind in (W.U_IN, W.V_IN):
        prob = W.Problem("pg", [W.Grid(2, [n, n, 1], [L, L, 1])], [W.field_pure_gauge(lam0, tau, w, 2)],
                         [W.Solve(kind, 1, p)], W.Window(-12.0, 12.0, 0.02))
        sv = SWFSolve(prob, 0)
        half = prob.window.steps // 2
        y = None
        for start, count in ((0, half - 100), (half - 100, 100)):
            y = sv.run(y, start=start, count=count)
            t = sv.time(start + count)
            assert t < 0.0 if start == 0 else abs(t) < 1e-9   # forward in time
            Lam = lam0 * np.exp(-t ** 2 / tau ** 2 - (sv.lat.X[0] ** 2 + sv.lat.X[1] ** 2) / w ** 2)
            ref = (np.exp(-1j * Lam) - 1)[None] * sv.psi_back(t)
            assert np.abs(y - ref).max() < 1e-5 * np.abs(ref).max()
        y = sv.run(y, start=half)
        assert ob.marginal(sv, y) < 1e-12


def _field_1d():
    return [W.Term(1, 0.9, W.gauss(1.5), [W.sech2(3.0), W.const(), W.const()]),
            W.Term(0, 0.4, W.sech2(1.2, c=0.3), [W.gauss(2.5, c=-0.5), W.const(), W.const()])]


def _overlaps(dt, grid, field, p, q):
    """Both sides of the two in/out identities for U(1, p) and V(1, q) (the
    opposite spin pair does not couple in these fields)."""
    solves = [W.Solve(W.U_OUT, 1, p), W.Solve(W.V_OUT, 1, q), W.Solve(W.U_IN, 1, p), W.Solve(W.V_IN, 1, q)]
    prob = W.Problem("io", [grid], [field], solves, W.Window(-8.0, 8.0, dt))
    uo, vo, ui, vi = (SWFSolve(prob, i) for i in range(4))
    yuo, yvo, yui, yvi = uo.run(), vo.run(), ui.run(), vi.run()
    tin, tout = prob.window.t_in, prob.window.t_out
    dV = uo.lat.dV
    # the backgrounds of U and V are orthogonal at every time (p + q a non-zero lattice momentum)
    assert abs(ob.inner(uo.psi_back(tin), vo.psi_back(tin), dV)) < 1e-12
    i1 = (ob.inner(ui.psi_back(tout), yvi, dV), ob.inner(yuo, vo.psi_back(tin), dV))   # (U_out|V_in)
    i2 = (ob.inner(yui, vi.psi_back(tout), dV), ob.inner(uo.psi_back(tin), yvo, dV))   # (U_in|V_out)
    return i1, i2


@pytest.mark.parametrize("dim", [1, 2])
def test_in_out_overlaps_agree_at_order_4(dim):
    if dim == 1:
        L = 30.0
        grid = W.Grid(1, [64, 1, 1], [L, 1, 1])
        field = _field_1d()
        p = [2 * np.pi * 3 / L, 0.2, 0.0]
        q = [2 * np.pi * 1 / L, -0.2, 0.0]
    else:
        L = 24.0
        grid = W.Grid(2, [32, 32, 1], [L, L, 1])
        field = [W.Term(1, 0.8, W.gauss(1.5), [W.gauss(3.0), W.gauss(4.0), W.const()]),
                 W.Term(2, 0.5, W.sech2(1.0), [W.ugauss(3.0), W.gauss(3.0), W.const()])]
        p = [2 * np.pi * 2 / L, -2 * np.pi / L, 0.3]
        q = [0.0, 2 * np.pi * 2 / L, -0.3]
    errs = []
    for dt in (0.04, 0.02):
        i1, i2 = _overlaps(dt, grid, field, p, q)
        assert abs(i1[1]) > 1e-3 and abs(i2[1]) > 1e-3
        errs.append(np.array([abs(i1[0] - i1[1]) / abs(i1[1]), abs(i2[0] - i2[1]) / abs(i2[1])]))
    assert np.all(errs[1] < 2e-7), errs
    ratio = errs[0] / errs[1]
    assert np.all((ratio > 12.0) & (ratio < 20.0)), ratio


def test_in_out_marginals_balance_over_all_lattice_modes():
    # a 15-point line (no Nyquist mode), every lattice momentum and spin, with
    # q_perp = -p_perp: the four totals are |S_{+-}|^2 and |S_{-+}|^2 of the
    # one-particle evolution, equal by unitarity
    n, L, pperp = 15, 15.0, 0.3
    F = [W.Term(1, 1.3, W.sech2(1.0), [W.sech2(2.0), W.const(), W.const()]),
         W.Term(0, 0.5, W.gauss(0.8), [W.gauss(1.5, c=0.4), W.const(), W.const()])]
    solves = []
    for kx in range(-(n // 2), n // 2 + 1):
        px = 2 * np.pi * kx / L
        for s in (1, -1):
            for kind, perp in ((W.U_OUT, pperp), (W.V_OUT, -pperp), (W.U_IN, pperp), (W.V_IN, -pperp)):
                solves.append(W.Solve(kind, s, [px, perp, 0.0]))
    prob = W.Problem("cb", [W.Grid(1, [n, 1, 1], [L, 1, 1])], [F], solves, W.Window(-6.0, 6.0, 0.01))
    tot = {k: 0.0 for k in (W.U_OUT, W.V_OUT, W.U_IN, W.V_IN)}
    for i, sv in enumerate(prob.solves):
        s = SWFSolve(prob, i)
        tot[sv.kind] += ob.marginal(s, s.run())
    assert tot[W.U_OUT] > 1e-4
    assert tot[W.V_IN] == pytest.approx(tot[W.U_OUT], rel=1e-6)     # |S_{+-}|^2
    assert tot[W.U_IN] == pytest.approx(tot[W.V_OUT], rel=1e-6)     # |S_{-+}|^2
    assert tot[W.U_IN] == pytest.approx(tot[W.U_OUT], rel=1e-6)


def test_in_forms_first_order_and_opposite():
    L = 30.0
    weak = [W.Term(t.mu, 1e-4 * t.amp, t.ft, t.fx) for t in _field_1d()]
    p = [2 * np.pi * 3 / L, 0.2, 0.0]
    q = [2 * np.pi * 1 / L, -0.2, 0.0]
    solves = [W.Solve(W.U_OUT, 1, p), W.Solve(W.V_OUT, 1, q), W.Solve(W.U_IN, 1, p), W.Solve(W.V_IN, 1, q)]
    prob = W.Problem("weak", [W.Grid(1, [64, 1, 1], [L, 1, 1])], [weak], solves, W.Window(-8.0, 8.0, 0.02))
    uo, vo, ui, vi = (SWFSolve(prob, i) for i in range(4))
    yuo, yvo, yui, yvi = uo.run(), vo.run(), ui.run(), vi.run()
    om = ob.pair_amplitude(uo, yuo, vo, yvo, prob.window.t_in, 1)
    f1 = ob.pair_amplitude(ui, yui, vi, yvi, prob.window.t_out, 1)
    f2 = ob.pair_amplitude(ui, yui, vi, yvi, prob.window.t_out, 2)
    assert abs(om) > 1e-6
    assert abs(f1 + om) < 1e-3 * abs(om)       # second order is ~1e-4 of the first
    assert abs(f1 + f2) < 1e-6 * abs(f1)
    with pytest.raises(ValueError):
        ob.pair_amplitude(uo, yuo, vi, yvi, prob.window.t_in, 1)   # mixed directions
