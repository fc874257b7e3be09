"""GPU parity of the one-dimensional whole-loop kernel (options.persistent).

A (1+1)D solve runs every time step of a swf_step call inside one workgroup
with the state held on chip.  It is checked against:
* the FP64 oracle, element by element, for every line length it serves
  (64 ... 1024), both kinds, both spins, transverse momenta on the trivial
  axes, a field with A_0 and all alpha^j A_j couplings, and the absorber;
* the pass path (one launch per pass and stage) on the same inputs: step
  counts split over several calls, runs longer than one launch (1024 steps),
  batches of many solves (many workgroups), and observables at t_in;
* the fallback: a field with more profile tables than fit in LDS next to the
  exchange rows runs on the pass path (no whole-loop launch) with the same
  result.
FP64 to 1e-10 relative against the oracle; mixed precision to 2e-5 (FP32
state, about 100 steps).
"""
import numpy as np
import pytest

import swf_workloads as W
from oracle import observables as ob
from oracle.swf import SWFSolve

from swf_cases import field_mix, random_momenta

pytestmark = pytest.mark.gpu

LINE_KIND = 5


@pytest.fixture(scope="module")
def S():
    from paper_2512_16889_amd import swf
    return swf


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def line_problem(n, nterm=4, absorb=0, n_mom=1, t_half=2.0, dt=0.05, seed=0):
    L = 0.6 * n
    g = W.Grid(1, [n, 1, 1], [L, 1.0, 1.0], absorb_cells=absorb, absorb_strength=0.3 if absorb else 0.0)
    terms = field_mix(1)[:nterm]
    ps = random_momenta(n_mom, 1, g.L, g.n, seed)
    solves = [W.Solve(k, s, p) for p in ps for k in (0, 1) for s in (1, -1)]
    return W.Problem(f"line{n}", [g], [terms], solves, W.Window(-t_half, t_half, dt))


def whole_loop_launches(ctx):
    return ctx.kernel_stats(LINE_KIND)[0]


@pytest.mark.parametrize("n", [64, 128, 256, 512, 1024])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 2e-5)])
def test_line_kernel_full_solve_vs_oracle(S, n, prec, tol):
    prob = line_problem(n, nterm=4)
    with S.Context(prob, precision=prec, profile=True) as ctx:
        assert ctx.step() == 0
        ctx.sync()
        assert whole_loop_launches(ctx) > 0
        for i in range(len(prob.solves)):
            sv = SWFSolve(prob, i)
            y = sv.run()
            assert np.abs(y).max() > 1e-3
            assert relerr(ctx.get_psi(i), y) < tol, (n, prec, i)
            if prec == "fp64":
                assert ctx.marginal(i) == pytest.approx(ob.marginal(sv, y), rel=1e-8)


@pytest.mark.parametrize("n", [128, 1024])
def test_line_kernel_absorber_vs_oracle(S, n):
    prob = line_problem(n, nterm=2, absorb=n // 8)
    with S.Context(prob, precision="fp64", profile=True) as ctx:
        ctx.step()
        ctx.sync()
        assert whole_loop_launches(ctx) > 0
        for i in range(len(prob.solves)):
            assert relerr(ctx.get_psi(i), SWFSolve(prob, i).run()) < 1e-10


def test_line_kernel_single_step_from_random_state(S):
    prob = line_problem(256, nterm=3)
    k = 23
    with S.Context(prob, precision="fp64", profile=True) as ctx:
        states = {}
        for i in range(len(prob.solves)):
            states[i] = W.random_state((4, 256), seed=300 + i, scale=0.1)
            ctx.set_psi(i, states[i], k)
        ctx.step(1)
        ctx.sync()
        assert whole_loop_launches(ctx) == 1
        for i in range(len(prob.solves)):
            assert relerr(ctx.get_psi(i), SWFSolve(prob, i).step(k, states[i])) < 1e-12


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 1e-5)])
def test_line_kernel_matches_pass_path_split_calls(S, prec, tol):
    prob = line_problem(512, nterm=4, n_mom=2, t_half=3.0)
    steps = prob.window.steps
    with S.Context(prob, precision=prec, persistent=False) as ref:
        ref.step()
        ref.sync()
        want = [ref.get_psi(i) for i in range(len(prob.solves))]
        pw = [ref.marginal(i) for i in range(len(prob.solves))]
    with S.Context(prob, precision=prec, profile=True) as ctx:
        left = steps
        for c in (1, 7, 30):
            left = ctx.step(c)
        assert ctx.step(left) == 0
        ctx.sync()
        assert whole_loop_launches(ctx) == 4
        for i in range(len(prob.solves)):
            assert relerr(ctx.get_psi(i), want[i]) < tol
            if prec == "fp64":
                assert ctx.marginal(i) == pytest.approx(pw[i], rel=1e-9)


def test_line_kernel_longer_than_one_launch(S):
    # 1500 steps: two launches of the whole-loop kernel (at most 1024 steps each)
    prob = W.config_1d(t_half=15.0)   # the C1 line and field, 1500 steps
    assert prob.window.steps == 1500
    with S.Context(prob, precision="fp64", persistent=False) as ref:
        ref.step()
        ref.sync()
        want = ref.get_psi(0)
    with S.Context(prob, precision="fp64", profile=True) as ctx:
        ctx.step()
        ctx.sync()
        assert whole_loop_launches(ctx) == 2
        assert np.abs(want).max() > 1e-6
        assert relerr(ctx.get_psi(0), want) < 1e-11


def test_line_kernel_batch_many_solves(S):
    prob = line_problem(256, nterm=2, n_mom=12, t_half=1.0)   # 48 solves, one workgroup each
    with S.Context(prob, precision="fp64", persistent=False) as ref:
        ref.step()
        ref.sync()
        want = [ref.get_psi(i) for i in range(len(prob.solves))]
    with S.Context(prob, precision="fp64", profile=True) as ctx:
        ctx.step()
        ctx.sync()
        assert whole_loop_launches(ctx) == 1
        for i in range(len(prob.solves)):
            assert relerr(ctx.get_psi(i), want[i]) < 1e-12


def test_line_kernel_lds_fallback(S):
    # eight profile tables of 1024 doubles do not fit in LDS next to the FP64
    # exchange rows: the context runs the pass path instead, with the oracle's result
    prob = line_problem(1024, nterm=5, t_half=1.0)
    extra = [W.Term(0, 0.05 * (j + 1), W.gauss(1.0 + 0.2 * j), [W.sech2(8.0 + j), W.const(), W.const()])
             for j in range(3)]
    prob.fields = [list(prob.fields[0]) + extra]
    with S.Context(prob, precision="fp64", profile=True) as ctx:
        ctx.step()
        ctx.sync()
        assert whole_loop_launches(ctx) == 0
        for i in range(len(prob.solves)):
            assert relerr(ctx.get_psi(i), SWFSolve(prob, i).run()) < 1e-10


def test_line_kernel_not_used_when_a_grid_is_not_1d(S):
    # one 1D and one 2D grid in the same context: the whole-loop path needs
    # every grid to be 1D, so both run on the pass path, with the oracle's result
    g1 = W.Grid(1, [64, 1, 1], [38.4, 1.0, 1.0])
    g2 = W.Grid(2, [32, 32, 1], [30.0, 30.0, 1.0])
    prob = W.Problem("mixdim", [g1, g2], [field_mix(1)[:3], field_mix(2)],
                     [W.Solve(0, 1, [0.3, 0.2, -0.1], 0, 0), W.Solve(1, -1, [0.2, -0.3, 0.1], 1, 1)],
                     W.Window(-1.5, 1.5, 0.05))
    with S.Context(prob, precision="fp64", profile=True) as ctx:
        ctx.step()
        ctx.sync()
        assert whole_loop_launches(ctx) == 0
        for i in range(len(prob.solves)):
            assert relerr(ctx.get_psi(i), SWFSolve(prob, i).run()) < 1e-10


def test_line_kernel_with_graph_option(S):
    # use_graph captures the pass path's step; a 1D problem still runs the
    # whole-loop kernel and gives the same states
    prob = line_problem(128, nterm=3, n_mom=2)
    with S.Context(prob, precision="fp64", use_graph=True) as g, S.Context(prob, precision="fp64") as e:
        for c in (5, 17, 58):
            g.step(c)
            e.step(c)
            for i in range(len(prob.solves)):
                assert np.array_equal(g.get_psi(i), e.get_psi(i))


_C1_REF = {}


def c1_reference():
    """The (1+1)D Schwinger workload over its whole window (1024 points,
    6000 RK4 steps from t = 60 to -60) by the oracle, computed once."""
    if not _C1_REF:
        prob = W.config_1d()
        sv = SWFSolve(prob, 0)
        y = sv.run()
        _C1_REF.update(prob=prob, sv=sv, y=y, P=ob.marginal(sv, y))
    return _C1_REF


@pytest.mark.parametrize("persistent", [True, False])
def test_c1_full_window_vs_oracle(S, persistent):
    """The whole 6000-step (1+1)D workload, by the whole-loop kernel and by the
    pass path, against the oracle: psi element by element to 1e-10 of its
    largest value and the marginal P to 1e-9."""
    ref = c1_reference()
    prob = ref["prob"]
    with S.Context(prob, precision="fp64", persistent=persistent, profile=True) as ctx:
        assert ctx.step() == 0
        ctx.sync()
        assert (whole_loop_launches(ctx) > 0) == persistent
        psi = ctx.get_psi(0)
        assert np.abs(ref["y"]).max() > 1e-3
        assert relerr(psi, ref["y"]) < 1e-10
        assert ctx.marginal(0) == pytest.approx(ref["P"], rel=1e-9)
