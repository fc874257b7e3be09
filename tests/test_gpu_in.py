"""GPU parity of in-states U_in, V_in (stepped forward from t_in, read at
t_out) against the FP64 oracle, whose in-states are pinned on the CPU by the
pure-gauge closed form, the time independence of in/out overlaps and the
in/out balance of marginals.  Tolerances as for out-states: 1e-10 on psi
and 1e-9 on the observables in FP64, 2e-5 / 1e-4 in mixed precision.
"""
import numpy as np
import pytest

import swf_workloads as W
from oracle import observables as ob
from oracle.swf import SWFSolve

from swf_cases import field_mix, grid, lattice_p, problem

pytestmark = pytest.mark.gpu

IN = (W.U_IN, W.V_IN)
SHAPES = [(1, (64,), (40.0,)), (2, (32, 48), (30.0, 36.0)), (3, (16, 32, 16), (18.0, 24.0, 18.0))]


@pytest.fixture(scope="module")
def S():
    from paper_2512_16889_amd import swf
    return swf


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


@pytest.mark.parametrize("dim,n,L,persistent", [s + (True,) for s in SHAPES] + [SHAPES[0] + (False,)])
def test_in_states_full_solve_fp64(S, dim, n, L, persistent):
    # persistent: the 1D whole-loop kernel (False: the pass path for the 1D line)
    prob = problem(dim, n, L, kinds=IN, spins=(1, -1), n_mom=1, t_half=2.0)
    with S.Context(prob, precision="fp64", persistent=persistent) as ctx:
        d0 = ctx.diagnostics(0)
        assert d0[0] == 0.0
        assert ctx.step() == 0
        ctx.sync()
        for i in range(len(prob.solves)):
            sv = SWFSolve(prob, i)
            assert sv.forward
            y = sv.run()
            assert np.abs(y).max() > 1e-3
            assert relerr(ctx.get_psi(i), y) < 1e-10
            assert ctx.marginal(i) == pytest.approx(ob.marginal(sv, y), rel=1e-9)
            ss, bs = ob.diagnostics(sv, y, prob.window.t_out)
            d = ctx.diagnostics(i)
            assert d[0] == pytest.approx(ss, rel=1e-10)
            assert d[1] == pytest.approx(bs, rel=1e-8, abs=1e-10 * ss)


def test_in_states_halfway(S):
    # the time of every stage counts forward from t_in: compare after part of the window
    prob = problem(2, (32, 32), (30.0, 30.0), kinds=IN, spins=(1,), n_mom=1, t_half=2.0)
    half = prob.window.steps // 2 - 7
    with S.Context(prob, precision="fp64") as ctx:
        assert ctx.step(half) == prob.window.steps - half
        ctx.sync()
        for i in range(len(prob.solves)):
            sv = SWFSolve(prob, i)
            y = sv.run(count=half)
            assert relerr(ctx.get_psi(i), y) < 1e-10
            ss, _ = ob.diagnostics(sv, y, sv.time(half))
            assert ctx.diagnostics(i)[0] == pytest.approx(ss, rel=1e-10)


@pytest.mark.parametrize("dim,n,L", SHAPES)
def test_in_states_pair_forms(S, dim, n, L):
    g = grid(dim, n, L)
    p = lattice_p(dim, g.n, g.L, [2, -1, 1], trivial=(0.3, -0.2))
    q = lattice_p(dim, g.n, g.L, [-3, 2, 0], trivial=(-0.3, 0.2))
    prob = W.Problem("pair_in", [g], [field_mix(dim)], [W.Solve(W.U_IN, 1, p), W.Solve(W.V_IN, 1, q),
                                                       W.Solve(W.V_IN, -1, q)], W.Window(-2.0, 2.0, 0.05))
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        su = SWFSolve(prob, 0)
        yu = su.run()
        for j in (1, 2):
            sv = SWFSolve(prob, j)
            yv = sv.run()
            for form in (1, 2):
                ref = ob.pair_amplitude(su, yu, sv, yv, prob.window.t_out, form)
                assert abs(ctx.pair(0, j, form) - ref) <= 1e-9 * abs(ref) + 1e-13
        m = np.array(ctx.pair_matrix([0], [1, 2], 1)).reshape(1, 2)
        for jj, j in enumerate((1, 2)):
            assert abs(m[0, jj] - ctx.pair(0, j, 1)) <= 1e-12 * abs(ctx.pair(0, j, 1)) + 1e-14


@pytest.mark.parametrize("dim,n,L", SHAPES)
def test_in_states_mixed(S, dim, n, L):
    prob = problem(dim, n, L, kinds=IN, spins=(1,), n_mom=1, t_half=2.0)
    with S.Context(prob, precision="mixed") as ctx:
        ctx.step()
        ctx.sync()
        for i in range(len(prob.solves)):
            sv = SWFSolve(prob, i)
            y = sv.run()
            assert relerr(ctx.get_psi(i), y) < 2e-5
            assert ctx.marginal(i) == pytest.approx(ob.marginal(sv, y), rel=1e-4)


def test_in_states_errors(S):
    mixed = problem(1, (64,), (40.0,), kinds=(W.U_OUT, W.V_IN), spins=(1,))
    with pytest.raises(S.SwfError) as e:
        S.Context(mixed)
    assert e.value.code == S.SWF_E_UNSUPPORTED
    bw = W.config_bw_1d(n=64, L=100.0, steps=4)
    bw.solves = [W.Solve(s.kind + 2, s.spin, s.p, s.grid, s.field) for s in bw.solves]
    with pytest.raises(S.SwfError) as e:
        S.Context(bw)
    assert e.value.code == S.SWF_E_ARG and "U_out" in str(e.value)
