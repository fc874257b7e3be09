"""GPU edge cases of the SWF path, through the C ABI, against the oracle or
against what holds exactly.

* No field (an empty term list, or every amplitude zero): the scattered wave
  has no source, so every component stays exactly zero, in both precisions,
  in 1D (whole-loop kernel), 2D and 3D; the marginal and the pair amplitude
  are exactly zero too.
* The largest supported field: eight separable terms touching every
  coupling, on the pass path, against the oracle.
* A window of a single RK4 step.
* The smallest FFT length on every axis (16^3).
* The weak-field (Born) limit: pair amplitude and marginal against their
  first-order closed forms.
FP64 to 1e-10 relative against the oracle, mixed to 2e-5.
"""
import numpy as np
import pytest

import swf_workloads as W
from oracle.swf import SWFSolve

from swf_cases import field_mix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2512_16889_amd import swf
    return swf


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def grid(dim, n, L):
    return W.Grid(dim, [n if j < dim else 1 for j in range(3)], [L if j < dim else 1.0 for j in range(3)])


@pytest.mark.parametrize("dim,n,L", [(1, 128, 60.0), (2, 32, 30.0), (3, 16, 18.0)])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
@pytest.mark.parametrize("empty", [True, False])
def test_no_field_gives_exactly_zero(S, dim, n, L, prec, empty):
    g = grid(dim, n, L)
    field = [] if empty else [W.Term(mu, 0.0, W.gauss(1.0), [W.gauss(3.0) if j < dim else W.const()
                                                            for j in range(3)]) for mu in range(4)]
    prob = W.Problem("zero", [g], [field], [W.Solve(0, 1, [0.2, -0.1, 0.3]), W.Solve(1, -1, [-0.2, 0.1, -0.3])],
                     W.Window(-1.0, 1.0, 0.05))
    with S.Context(prob, precision=prec) as ctx:
        ctx.step()
        ctx.sync()
        for i in range(2):
            assert np.all(ctx.get_psi(i) == 0)
            assert ctx.marginal(i) == 0.0
        assert ctx.pair(0, 1, 1) == 0


def test_eight_term_field_2d_vs_oracle(S):
    extra = [W.Term(2, 0.15, W.sech2(0.8, c=0.3), [W.gauss(2.5), W.sech2(3.0, c=0.5), W.const()]),
             W.Term(3, -0.2, W.gauss(1.1, k=0.6), [W.sech2(2.0, c=-0.3), W.gauss(2.8), W.const()]),
             W.Term(0, 0.1, W.sech2(1.4), [W.gauss(3.2, c=0.4), W.gauss(2.1), W.const()])]
    field = field_mix(2) + extra
    assert len(field) == 8
    prob = W.Problem("eight", [grid(2, 32, 30.0)], [field],
                     [W.Solve(0, 1, [0.3, -0.2, 0.1]), W.Solve(1, -1, [-0.1, 0.25, -0.1])],
                     W.Window(-2.0, 2.0, 0.05))
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        for i in range(2):
            y = SWFSolve(prob, i).run()
            assert np.abs(y).max() > 1e-3
            assert relerr(ctx.get_psi(i), y) < 1e-10


@pytest.mark.parametrize("dim,n,L", [(1, 64, 40.0), (2, 32, 30.0)])
def test_single_step_window(S, dim, n, L):
    prob = W.Problem("one", [grid(dim, n, L)], [field_mix(dim)], [W.Solve(0, 1, [0.3, -0.2, 0.1])],
                     W.Window(0.4, 0.45, 0.05))
    with S.Context(prob, precision="fp64") as ctx:
        total, _ = ctx.steps()
        assert total == 1
        assert ctx.step() == 0
        y = SWFSolve(prob, 0).run()
        assert np.abs(y).max() > 0
        assert relerr(ctx.get_psi(0), y) < 1e-12


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 2e-5)])
def test_smallest_lengths_3d(S, prec, tol):
    prob = W.Problem("small", [grid(3, 16, 16.0)], [field_mix(3)],
                     [W.Solve(0, 1, [0.2, -0.3, 0.1]), W.Solve(1, 1, [-0.2, 0.1, 0.3])], W.Window(-1.5, 1.5, 0.05))
    with S.Context(prob, precision=prec) as ctx:
        ctx.step()
        for i in range(2):
            assert relerr(ctx.get_psi(i), SWFSolve(prob, i).run()) < tol


def test_born_limit_vs_closed_form(S):
    # the weak-field pair amplitude and marginal on the GPU against the
    # first-order closed forms (independent of the oracle's stepping)
    from scipy import integrate
    import test_oracle_born as B
    solves = [W.Solve(0, 1, B.P)] + [W.Solve(1, r, [qx, -B.P[1], -B.P[2]]) for qx in B.QX for r in (1, -1)]
    prob = B.problem(solves)
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        for i in range(1, len(solves)):
            want = B.omega1(1, B.P, solves[i].spin, solves[i].p)
            assert abs(ctx.pair(0, i, 1) - want) < 1e-3 * abs(want)
            assert abs(ctx.pair(0, i, 2) + want) < 1e-3 * abs(want)
        got = ctx.marginal(0)

    def dens(qx):
        q = [qx, -B.P[1], -B.P[2]]
        return sum(abs(B.omega1(1, B.P, r, q)) ** 2 for r in (1, -1)) / (2 * np.pi)

    want, _ = integrate.quad(dens, -12.0, 12.0, limit=400, epsabs=0, epsrel=1e-10)
    assert abs(got - want) < 1e-3 * want
