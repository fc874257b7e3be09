"""Pins of the oracle's interaction-picture stepper (window.scheme "iprk4",
Lawson's integrating-factor RK4) on the CPU.

What fixes it independently of the code that steps with it:

* the free propagator's closed form cos(E tau) - i sin(E tau) H0(k)/E is
  scipy's matrix exponential of -i H0(k) tau;
* the free evolution is taken exactly: a positive-energy plane-wave spinor
  u(p) e^{ip.x} on the lattice comes back as e^{-i E_p h n} times itself
  after n steps of any size (the classical RK4 misses this at order h^5 per
  step);
* with the field on, the error falls at order 4 in dt, and the stepper and
  the classical RK4 converge to the same solution;
* BW amplitudes integrated with it converge to the classical stepper's.
"""
import dataclasses

import numpy as np
import pytest
from scipy.linalg import expm

import swf_workloads as W
from oracle import bw, dirac
from oracle.swf import SWFSolve


def _problem(dt, scheme="iprk4", t_half=4.0, dim=1):
    L = 30.0
    F = [W.Term(1, 0.9, W.gauss(1.5), [W.sech2(3.0), W.gauss(4.0) if dim == 2 else W.const(), W.const()]),
         W.Term(0, 0.4, W.sech2(1.2, c=0.3), [W.gauss(2.5, c=-0.5), W.const(), W.const()])]
    n = [64, 1, 1] if dim == 1 else [32, 16, 1]
    Ls = [L, 1, 1] if dim == 1 else [L, 20.0, 1]
    return W.Problem("ip", [W.Grid(dim, n, Ls)], [F],
                     [W.Solve(W.U_OUT, 1, [2 * np.pi * 3 / L, 0.2 if dim == 1 else 2 * np.pi / 20.0, 0.1])],
                     W.Window(-t_half, t_half, dt, scheme))


def test_free_propagator_is_the_matrix_exponential():
    sv = SWFSolve(_problem(0.1, dim=2), 0)
    rng = np.random.default_rng(3)
    for tau in (0.05, -0.37, 1.3):
        P = sv.free_propagator(tau)
        for _ in range(6):
            ix = tuple(rng.integers(0, s) for s in sv.lat.shape)
            H = sv.H0[(slice(None), slice(None)) + ix]
            assert np.allclose(P[(slice(None), slice(None)) + ix], expm(-1j * H * tau), rtol=0, atol=1e-13)


@pytest.mark.parametrize("scheme,exact", [("iprk4", True), ("rk4", False)])
def test_free_plane_wave_is_stepped_exactly(scheme, exact):
    # zero field: the scattered-wave equation is the free Dirac equation, and a
    # lattice plane wave of positive energy is an eigenstate of H0
    prob = _problem(0.25, scheme)
    prob.fields = [[W.Term(1, 0.0, W.gauss(1.0), [W.const(), W.const(), W.const()])]]
    sv = SWFSolve(prob, 0)
    L = prob.grids[0].L[0]
    p = np.array([2 * np.pi * 5 / L, 0.2, 0.1])
    u = dirac.u_spinor(1, p)
    x = sv.lat.X[0]
    y0 = u[:, None] * np.exp(1j * p[0] * x)[None]
    y = sv.run(y0.copy(), count=40)
    h = -prob.window.dt
    want = np.exp(-1j * dirac.energy(p) * h * 40) * y0
    err = np.abs(y - want).max()
    if exact:
        assert err < 1e-12
    else:
        assert err > 1e-6      # the classical stepper's phase error at this step


def test_converges_at_order_4_and_to_the_classical_solution():
    ref = SWFSolve(_problem(0.0125, "rk4"), 0).run()
    ip = {dt: SWFSolve(_problem(dt), 0).run() for dt in (0.2, 0.1, 0.0125)}
    assert np.abs(ip[0.0125] - ref).max() < 1e-7 * np.abs(ref).max()
    e = [np.abs(ip[dt] - ip[0.0125]).max() for dt in (0.2, 0.1)]
    assert 12.0 < e[0] / e[1] < 20.0, e


def test_two_dimensional_and_in_states():
    # a 2D lattice with a trivial axis, and an in-state stepped forward
    for kind in (W.U_OUT, W.U_IN):
        base = _problem(0.05, dim=2)
        base.solves = [W.Solve(kind, -1, [0.3, 2 * np.pi / 20.0, -0.2])]
        ref = SWFSolve(dataclasses.replace(base, window=W.Window(-4.0, 4.0, 0.0125, "rk4")), 0).run()
        got = SWFSolve(base, 0).run()
        assert np.abs(ref).max() > 1e-3
        assert np.abs(got - ref).max() < 1e-5 * np.abs(ref).max()


def test_bw_amplitude_with_the_interaction_picture():
    P = 2 * np.pi * 4 / 160.0

    def amp(dt, scheme):
        prob = W.config_bw_1d(P=P, n=128, L=160.0, dt=dt, t_half=25.0)
        prob.window = W.Window(prob.window.t_in, prob.window.t_out, dt, scheme)
        return bw.Vertex(prob, 0).amplitude()["terms"]

    ref = amp(0.025, "rk4")
    got = amp(0.1, "iprk4")
    assert np.all(np.abs(got - ref) <= 1e-5 * np.abs(ref))
