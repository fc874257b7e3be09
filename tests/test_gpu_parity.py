"""GPU parity: the HIP path through the C ABI against the FP64 CPU oracle.

FP64 path: every operator and every full solve agrees with the oracle to
1e-10 relative (rounding order differs; no bitwise claim).  Mixed path: FP32
state and transforms; agreement stated per test from the arithmetic
(about 1e-5 relative on psi after ~100 steps).
"""
import numpy as np
import pytest

import swf_workloads as W
from oracle import bw as obw
from oracle import observables as ob
from oracle.swf import SWFSolve

from swf_cases import field_mix, grid, lattice_p, problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2512_16889_amd import swf
    return swf


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


SHAPES = [(1, (64,), (40.0,)), (1, (48,), (36.0,)), (2, (32, 48), (30.0, 36.0)), (2, (16, 16), (20.0, 20.0)),
          (3, (16, 32, 16), (18.0, 24.0, 18.0)), (3, (40, 16, 48), (30.0, 18.0, 32.0))]


@pytest.mark.parametrize("dim,n,L", SHAPES)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 2e-6)])
def test_fft_and_kinetic_operators(S, dim, n, L, prec, tol):
    prob = problem(dim, n, L, kinds=(0, 1), spins=(1,))
    with S.Context(prob, precision=prec) as ctx:
        for i in range(len(prob.solves)):
            sv = SWFSolve(prob, i)
            psi = W.random_state((4,) + tuple(n), seed=10 + i)
            # op 0: forward transform over the non-trivial axes
            assert relerr(ctx.apply_op(0, i, psi), np.fft.fftn(psi, axes=tuple(range(1, dim + 1)))) < tol
            # op 1: the kinetic term IFFT(-i H0 FFT psi)
            assert relerr(ctx.apply_op(1, i, psi), sv.kinetic(psi)) < tol
            # op 2: the full right-hand side at time t
            for t in (-0.7, 0.3):
                assert relerr(ctx.apply_op(2, i, psi, t), sv.rhs(t, psi)) < 10 * tol


@pytest.mark.parametrize("dim,n,L", SHAPES)
def test_single_step_from_random_state(S, dim, n, L):
    prob = problem(dim, n, L, kinds=(0, 1), spins=(1, -1))
    with S.Context(prob, precision="fp64") as ctx:
        k = 17
        states = {}
        for i in range(len(prob.solves)):
            states[i] = W.random_state((4,) + tuple(n), seed=100 + i, scale=0.1)
            ctx.set_psi(i, states[i], k)
        ctx.step(1)
        ctx.sync()
        for i in range(len(prob.solves)):
            ref = SWFSolve(prob, i).step(k, states[i])
            assert relerr(ctx.get_psi(i), ref) < 1e-12


@pytest.mark.parametrize("dim,n,L", SHAPES)
def test_full_solve_fp64(S, dim, n, L):
    prob = problem(dim, n, L, kinds=(0, 1), spins=(1, -1), n_mom=1, t_half=2.0)
    with S.Context(prob, precision="fp64") as ctx:
        assert ctx.step() == 0
        ctx.sync()
        for i, s in enumerate(prob.solves):
            sv = SWFSolve(prob, i)
            y = sv.run()
            assert np.abs(y).max() > 1e-3
            assert relerr(ctx.get_psi(i), y) < 1e-10
            assert ctx.marginal(i) == pytest.approx(ob.marginal(sv, y), rel=1e-9)
            ss, bs = ob.diagnostics(sv, y, prob.window.t_in)
            d = ctx.diagnostics(i)
            assert d[0] == pytest.approx(ss, rel=1e-10)
            assert d[1] == pytest.approx(bs, rel=1e-8, abs=1e-10 * ss)
            assert d[3] == 1.0


@pytest.mark.parametrize("dim,n,L", [(1, (64,), (40.0,)), (2, (32, 48), (30.0, 36.0)), (3, (16, 32, 16), (18.0, 24.0, 18.0))])
def test_pair_amplitude_both_forms(S, dim, n, L):
    g = grid(dim, n, L)
    p = lattice_p(dim, g.n, g.L, [2, -1, 1], trivial=(0.3, -0.2))
    q = [v for v in lattice_p(dim, g.n, g.L, [-3, 2, 0], trivial=(-0.3, 0.2))]
    prob = W.Problem("pair", [g], [field_mix(dim)], [W.Solve(0, 1, p), W.Solve(1, 1, q), W.Solve(1, -1, q)],
                     W.Window(-2.0, 2.0, 0.05))
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        su = SWFSolve(prob, 0)
        yu = su.run()
        for j in (1, 2):
            sv = SWFSolve(prob, j)
            yv = sv.run()
            for form in (1, 2):
                ref = ob.pair_amplitude(su, yu, sv, yv, prob.window.t_in, form)
                got = ctx.pair(0, j, form)
                assert abs(got - ref) <= 1e-9 * abs(ref) + 1e-13
            assert ctx.probability(S.P_PAIR, 0, j) == pytest.approx(abs(ob.pair_amplitude(su, yu, sv, yv, prob.window.t_in, 1)) ** 2, rel=1e-8, abs=1e-24)


def test_bw_amplitude_1d_fig7_kinematics(S):
    P = 2 * np.pi * 4 / 160.0
    spins = ((1, 1), (1, -1))
    prob = W.config_bw_1d(P=P, n=128, L=160.0, dt=0.1, t_half=25.0, spins=spins)
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        for v in range(len(prob.vertices)):
            ref = obw.Vertex(prob, v).amplitude()
            for term in range(3):
                got = ctx.bw(v, term)
                want = ref["terms"][term]
                assert abs(got - want) <= 1e-9 * abs(want), (v, term, got, want)
            tot = ctx.bw(v)
            assert abs(tot - ref["total"]) <= 1e-7 * abs(ref["total"])
        # exact spin structure (eq. (MparaE)) holds on the GPU too
        assert ctx.bw(1) / ctx.bw(0) == pytest.approx(-0.6j, abs=1e-8)


def test_bw_amplitude_2d(S):
    g = grid(2, (32, 32), (40.0, 40.0))
    F = [W.Term(1, 0.8, W.gauss(2.0, k=0.5), [W.gauss(5.0), W.gauss(6.0), W.const()]),
         W.Term(0, 0.2, W.sech2(2.0), [W.ugauss(4.0), W.gauss(5.0), W.const()])]
    k = [2 * np.pi * 2 / 40.0, 0.0, 1.1]
    p = [2 * np.pi * 3 / 40.0, -2 * np.pi / 40.0, 0.4]
    q = [0.2, 0.3, 0.7]
    prob = W.Problem("bw2", [g], [F], [W.Solve(0, 1, p), W.Solve(1, -1, q)], W.Window(-6.0, 6.0, 0.05),
                     [W.Vertex(0, 1, k, [0.0, 0.6, 0.8])])
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        ref = obw.Vertex(prob, 0).amplitude()
        for term in range(3):
            want = ref["terms"][term]
            assert abs(ctx.bw(0, term) - want) <= 1e-9 * abs(want) + 1e-14


@pytest.mark.parametrize("dim,n,L", [(1, (64,), (40.0,)), (2, (32, 48), (30.0, 36.0)), (3, (16, 16, 32), (18.0, 18.0, 24.0))])
def test_mixed_precision_full_solve(S, dim, n, L):
    prob = problem(dim, n, L, kinds=(0, 1), spins=(1,), t_half=2.0)
    with S.Context(prob, precision="mixed") as ctx:
        ctx.step()
        ctx.sync()
        for i in range(len(prob.solves)):
            sv = SWFSolve(prob, i)
            y = sv.run()
            assert relerr(ctx.get_psi(i), y) < 2e-5
            assert ctx.marginal(i) == pytest.approx(ob.marginal(sv, y), rel=1e-4)


def test_absorber_matches_oracle(S):
    g = W.Grid(2, [32, 32, 1], [30.0, 30.0, 1.0], absorb_cells=5, absorb_strength=0.3)
    prob = W.Problem("abs", [g], [field_mix(2)], [W.Solve(0, 1, [0.3, -0.2, 0.1])], W.Window(-3.0, 3.0, 0.05))
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        y = SWFSolve(prob, 0).run()
        assert relerr(ctx.get_psi(0), y) < 1e-10


def test_ragged_batch_matches_per_instance_and_oracle(S):
    grids = [grid(2, (32, 32), (30.0, 30.0)), grid(2, (48, 48), (30.0, 30.0)), grid(2, (16, 64), (30.0, 40.0))]
    fields = [field_mix(2), W.field_gauss_2d(0.7, 1.5, 6.0)]
    solves = [W.Solve(0, 1, [0.2, 0.1, 0.0], 0, 0), W.Solve(0, -1, [-0.3, 0.2, 0.1], 1, 1),
              W.Solve(1, 1, [0.1, -0.4, 0.0], 2, 0), W.Solve(0, 1, [0.5, 0.0, 0.0], 1, 0),
              W.Solve(0, 1, [0.0, 0.3, 0.2], 0, 1)]
    prob = W.Problem("ragged", grids, fields, solves, W.Window(-2.0, 2.0, 0.05))
    with S.Context(prob, precision="fp64", batched=True) as a, S.Context(prob, precision="fp64", batched=False) as b:
        a.step()
        b.step()
        for i in range(len(solves)):
            pa, pb = a.get_psi(i), b.get_psi(i)
            assert np.array_equal(pa, pb)          # same kernels, same tiles: bitwise
            assert relerr(pa, SWFSolve(prob, i).run()) < 1e-10


def test_graph_replay_bitwise_equals_eager(S):
    prob = problem(2, (32, 32), (30.0, 30.0), kinds=(0, 1), spins=(1,), t_half=1.5)
    with S.Context(prob, precision="mixed", use_graph=True) as g, S.Context(prob, precision="mixed") as e:
        for chunk in (7, 13, 40):
            g.step(chunk)
            e.step(chunk)
            for i in range(len(prob.solves)):
                assert np.array_equal(g.get_psi(i), e.get_psi(i))
        for i in range(len(prob.solves)):
            assert g.marginal(i) == e.marginal(i)


@pytest.mark.parametrize("graph_steps", [5, 16])
def test_multi_step_graph_bitwise_equals_eager(S, graph_steps):
    # graph_steps consecutive steps per graph, the one-step graph for the rest;
    # a BW problem so the vertex integrals ride along, and a run with the
    # in-loop check (every step then replays the one-step graph)
    P = 2 * np.pi * 4 / 160.0
    prob = W.config_bw_1d(P=P, n=128, L=160.0, dt=0.1, t_half=5.0)
    with S.Context(prob, precision="fp64", use_graph=True, graph_steps=graph_steps) as g, \
            S.Context(prob, precision="fp64") as e:
        for chunk in (7, 23, 1, 69):
            g.step(chunk)
            e.step(chunk)
            for i in range(len(prob.solves)):
                assert np.array_equal(g.get_psi(i), e.get_psi(i))
        assert g.steps() == e.steps()
        want = e.bw(0)
        assert g.bw(0) == want
    with S.Context(prob, precision="fp64", use_graph=True, graph_steps=graph_steps, check_every=3) as c:
        c.step()
        assert c.bw(0) == want
        for i in range(2):
            assert relerr(c.get_psi(i), SWFSolve(prob, i).run()) < 1e-10


def test_repeatable_bitwise(S):
    prob = problem(3, (16, 16, 16), (18.0, 18.0, 18.0), kinds=(0,), spins=(1,), t_half=1.0)
    res = []
    for _ in range(2):
        with S.Context(prob, precision="fp64") as c:
            c.step()
            res.append((c.get_psi(0), c.marginal(0)))
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1] == res[1][1]


def test_checkpoint_resume_bitwise(S):
    P = 2 * np.pi * 4 / 160.0
    prob = W.config_bw_1d(P=P, n=128, L=160.0, dt=0.1, t_half=10.0)
    with S.Context(prob, precision="fp64") as full:
        full.step()
        want = full.bw(0)
        psi_want = [full.get_psi(i) for i in range(2)]
    with S.Context(prob, precision="fp64") as a:
        a.step(77)
        snap = [a.get_psi(i) for i in range(2)]
        m = a.get_bw_state(0)
    with S.Context(prob, precision="fp64") as b:
        for i in range(2):
            b.set_psi(i, snap[i], 77)
        b.set_bw_state(0, m)
        b.step()
        for i in range(2):
            assert np.array_equal(b.get_psi(i), psi_want[i])
        assert b.bw(0) == want


def test_order_errors(S):
    prob = problem(1, (64,), (40.0,), kinds=(0,), spins=(1,))
    with S.Context(prob, precision="fp64") as c:
        with pytest.raises(S.SwfError) as e:
            c.marginal(0)
        assert e.value.code == S.SWF_E_ORDER
        total, _ = c.steps()
        with pytest.raises(S.SwfError) as e:
            c.step(total + 1)
        assert e.value.code == S.SWF_E_ORDER
        c.step()
        with pytest.raises(S.SwfError) as e:
            c.probability(S.P_MARGINAL_POS, 0)
        assert e.value.code == S.SWF_E_ARG


def test_nonfinite_detected(S):
    prob = problem(1, (64,), (40.0,), kinds=(0,), spins=(1,))
    with S.Context(prob, precision="fp64") as c:
        psi = np.zeros((4, 64), dtype=complex)
        psi[2, 5] = np.nan
        c.set_psi(0, psi, 0)
        with pytest.raises(S.SwfError) as e:
            c.diagnostics(0)
        assert e.value.code == S.SWF_E_NONFINITE


@pytest.mark.parametrize("dim,persistent", [(1, True), (1, False), (2, False)])
def test_in_loop_nonfinite_check(S, dim, persistent):
    """options.check_every: a NaN planted in one solve at step 3 is reported by
    swf_step at the first check after it (step 4 with checks every 2 steps),
    naming that solve; a clean run of the same context passes every check."""
    n, L = ((64,), (40.0,)) if dim == 1 else ((32, 32), (20.0, 20.0))
    prob = problem(dim, n, L, kinds=(0,), spins=(1, -1))
    shape = (4,) + n
    with S.Context(prob, precision="fp64", check_every=2, persistent=persistent) as c:
        assert c.step(6) == prob.window.steps - 6          # clean: every check passes
        c.reset()
        psi = np.zeros(shape, dtype=complex)
        psi[(2,) + (5,) * dim] = np.inf
        c.set_psi(1, psi, 3)
        c.set_psi(0, np.zeros(shape, dtype=complex), 3)
        with pytest.raises(S.SwfError) as e:
            c.step(4)
        assert e.value.code == S.SWF_E_NONFINITE
        assert "solve 1" in str(e.value) and "after step 4" in str(e.value)
        assert c.steps()[1] == 7                            # the steps were still taken
