"""Weak-field (Born) limit of the oracle's pair amplitude and marginal.

To first order in the field, the scattered V wave seen by a free U wave at
t_in follows from d/dt (phi|psi) = -i (phi| gamma^0 J) for a free phi and
(i dslash - 1) psi = J, J = Aslash V_back, psi = 0 at t_out:

    Omega^(1)(p, q) = (U_b|V_s)(t_in) = i ubar_s(p) gamma^mu v_r(q) A~_mu(p + q),
    A~_mu(K) = int dt d^dx exp(i (K^0 t - K.x)) A_mu(t, x),

the projected term (U_s|Pi_+|V_s) being second order.  The electron marginal
(U_s|Pi_-|U_s) is then sum_r int d^dq / (2 pi)^d |Omega^(1)(p, q)|^2 at
q_perp = -p_perp.  Both pin the absolute normalisation of the pair path (the
(2 pi)^d, the spinors, the projector, dV) against closed forms written here
from the Fourier transforms of the field profiles, not from the oracle's field
code.  The field couples through A_0, A_1 and A_2 with three different
temporal/spatial shapes; a0 = 1e-4, so second-order terms are ~1e-4 of the
first-order ones.
"""
import numpy as np
import pytest
from scipy import integrate

import swf_workloads as W
from oracle import dirac
from oracle import observables as ob
from oracle.swf import SWFSolve

A0, A1, A2 = 1.0e-4, 1.5e-4, -0.8e-4     # amplitudes of the A_0, A_1, A_2 terms
TAU, TAU2, WX = 0.8, 0.7, 2.5


def field():
    return [W.Term(0, A0, W.gauss(TAU), [W.ugauss(WX), W.const(), W.const()]),   # A_0 ~ (x/w) e^{-(x/w)^2}
            W.Term(1, A1, W.gauss(TAU), [W.gauss(WX), W.const(), W.const()]),
            W.Term(2, A2, W.sech2(TAU2), [W.gauss(1.5 * WX), W.const(), W.const()])]


def ft_gauss(a, w):
    """int exp(-(s/w)^2) exp(i a s) ds."""
    return np.sqrt(np.pi) * w * np.exp(-(a * w) ** 2 / 4)


def ft_ugauss(a, w):
    """int (s/w) exp(-(s/w)^2) exp(i a s) ds."""
    return 1j * (a * w / 2) * np.sqrt(np.pi) * w * np.exp(-(a * w) ** 2 / 4)


def ft_sech2(a, tau):
    """int sech^2(s/tau) exp(i a s) ds."""
    if a == 0:
        return 2 * tau
    return np.pi * a * tau ** 2 / np.sinh(np.pi * a * tau / 2)


def a_tilde(K0, Kx):
    """A~_mu at K = (K0, Kx) for the field above (exp(i (K0 t - Kx x)))."""
    return np.array([A0 * ft_gauss(K0, TAU) * ft_ugauss(-Kx, WX),
                     A1 * ft_gauss(K0, TAU) * ft_gauss(-Kx, WX),
                     A2 * ft_sech2(K0, TAU2) * ft_gauss(-Kx, 1.5 * WX),
                     0.0])


def omega1(s, p, r, q):
    u = dirac.u_spinor(s, p)
    v = dirac.v_spinor(r, q)
    K0 = dirac.energy(p) + dirac.energy(q)
    At = a_tilde(K0, p[0] + q[0])
    aslash = sum(dirac.GAMMA[mu] * At[mu] for mu in range(4))
    return 1j * (np.conj(u) @ dirac.GAMMA0 @ aslash @ v)


def problem(solves):
    g = W.Grid(1, [256, 1, 1], [60.0, 1.0, 1.0])
    return W.Problem("born", [g], [field()], solves, W.Window(-6.0, 6.0, 0.02))


P = [0.3, 0.2, -0.1]
QX = [-0.5, 0.1, 0.63]


@pytest.fixture(scope="module")
def runs():
    solves = [W.Solve(0, 1, P)]
    for qx in QX:
        for r in (1, -1):
            solves.append(W.Solve(1, r, [qx, -P[1], -P[2]]))
    prob = problem(solves)
    out = []
    for i in range(len(solves)):
        sv = SWFSolve(prob, i)
        out.append((sv, sv.run()))
    return prob, out


def test_pair_amplitude_born_limit(runs):
    prob, out = runs
    su, yu = out[0]
    for i, (sv, yv) in enumerate(out[1:]):
        s, r, q = 1, prob.solves[i + 1].spin, prob.solves[i + 1].p
        want = omega1(s, P, r, q)
        assert abs(want) > 1e-6
        got1 = ob.pair_amplitude(su, yu, sv, yv, prob.window.t_in, 1)
        got2 = ob.pair_amplitude(su, yu, sv, yv, prob.window.t_in, 2)
        assert abs(got1 - want) < 1e-3 * abs(want), (q, r, got1, want)
        assert abs(got2 + want) < 1e-3 * abs(want), (q, r, got2, want)


def test_marginal_born_limit(runs):
    prob, out = runs
    su, yu = out[0]

    def dens(qx):
        q = [qx, -P[1], -P[2]]
        return sum(abs(omega1(1, P, r, q)) ** 2 for r in (1, -1)) / (2 * np.pi)

    want, _ = integrate.quad(dens, -12.0, 12.0, limit=400, epsabs=0, epsrel=1e-10)
    got = ob.marginal(su, yu)
    assert want > 1e-14
    assert abs(got - want) < 1e-3 * want, (got, want)
