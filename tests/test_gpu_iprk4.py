"""GPU parity of the interaction-picture stepper (options.stepper = SWF_IPRK4,
Lawson's integrating-factor RK4) against the FP64 oracle's, which is pinned on
the CPU by scipy's matrix exponential, exact free plane waves and order-4
convergence to the classical solution.  Same tolerances as the RK4 path:
1e-10 on psi and 1e-9 on observables in FP64, 2e-5 on psi in mixed precision.
"""
import dataclasses

import numpy as np
import pytest

import swf_workloads as W
from oracle import bw as obw
from oracle import observables as ob
from oracle.swf import SWFSolve

from swf_cases import field_mix, grid, problem

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2512_16889_amd import swf
    return swf


def relerr(a, b):
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def ip(prob, dt=None):
    w = prob.window
    return dataclasses.replace(prob, window=W.Window(w.t_in, w.t_out, dt or w.dt, "iprk4"))


SHAPES = [(1, (64,), (40.0,)), (2, (32, 48), (30.0, 36.0)), (3, (16, 32, 16), (18.0, 24.0, 18.0))]


@pytest.mark.parametrize("dim,n,L", SHAPES)
@pytest.mark.parametrize("kinds", [(W.U_OUT, W.V_OUT), (W.U_IN, W.V_IN)])
def test_iprk4_full_solve_fp64(S, dim, n, L, kinds):
    prob = ip(problem(dim, n, L, kinds=kinds, spins=(1, -1), n_mom=1, t_half=2.0))
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        ctx.sync()
        for i in range(len(prob.solves)):
            sv = SWFSolve(prob, i)
            assert sv.scheme == "iprk4"
            y = sv.run()
            assert np.abs(y).max() > 1e-3
            assert relerr(ctx.get_psi(i), y) < 1e-10
            assert ctx.marginal(i) == pytest.approx(ob.marginal(sv, y), rel=1e-9)


def test_iprk4_differs_from_rk4(S):
    # the stepper really switches: at dt = 0.2 the two schemes differ far above rounding
    base = problem(2, (32, 32), (30.0, 30.0), kinds=(W.U_OUT,), spins=(1,), n_mom=1, dt=0.2, t_half=2.0)
    out = {}
    for prob in (base, ip(base)):
        with S.Context(prob, precision="fp64") as ctx:
            ctx.step()
            out[prob.window.scheme] = ctx.get_psi(0)
        assert relerr(out[prob.window.scheme], SWFSolve(prob, 0).run()) < 1e-10
    assert relerr(out["iprk4"], out["rk4"]) > 1e-6


def test_iprk4_ragged_batch(S):
    # two grid sizes in one context (two launch groups), batched and per instance
    g0, g1 = grid(2, (32, 32), (30.0, 30.0)), grid(2, (48, 16), (36.0, 20.0))
    F = field_mix(2)
    solves = [W.Solve(0, 1, [0.3, -0.2, 0.1], 0), W.Solve(1, -1, [0.1, 0.4, -0.3], 1), W.Solve(0, -1, [-0.2, 0.1, 0.2], 1)]
    prob = W.Problem("rag", [g0, g1], [F], solves, W.Window(-2.0, 2.0, 0.05, "iprk4"))
    for batched in (True, False):
        with S.Context(prob, precision="fp64", batched=batched) as ctx:
            ctx.step()
            for i in range(len(solves)):
                assert relerr(ctx.get_psi(i), SWFSolve(prob, i).run()) < 1e-10


def test_iprk4_absorber(S):
    g = W.Grid(2, [32, 32, 1], [30.0, 30.0, 1.0], absorb_cells=5, absorb_strength=0.3)
    prob = ip(W.Problem("abs", [g], [field_mix(2)], [W.Solve(0, 1, [0.3, -0.2, 0.1])], W.Window(-3.0, 3.0, 0.05)))
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        assert relerr(ctx.get_psi(0), SWFSolve(prob, 0).run()) < 1e-10


@pytest.mark.parametrize("dim,n,L", SHAPES)
def test_iprk4_mixed(S, dim, n, L):
    prob = ip(problem(dim, n, L, kinds=(W.U_OUT, W.V_OUT), spins=(1,), n_mom=1, t_half=2.0))
    with S.Context(prob, precision="mixed") as ctx:
        ctx.step()
        for i in range(len(prob.solves)):
            sv = SWFSolve(prob, i)
            y = sv.run()
            assert relerr(ctx.get_psi(i), y) < 2e-5
            assert ctx.marginal(i) == pytest.approx(ob.marginal(sv, y), rel=1e-4)


def test_iprk4_bw_1d_fig7(S):
    P = 2 * np.pi * 4 / 160.0
    prob = ip(W.config_bw_1d(P=P, n=128, L=160.0, dt=0.1, t_half=25.0, spins=((1, 1), (1, -1))))
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        for v in range(len(prob.vertices)):
            ref = obw.Vertex(prob, v).amplitude()
            for term in range(3):
                want = ref["terms"][term]
                assert abs(ctx.bw(v, term) - want) <= 1e-9 * abs(want), (v, term)
        assert ctx.bw(1) / ctx.bw(0) == pytest.approx(-0.6j, abs=1e-8)


def test_iprk4_bw_2d_packet_and_plane(S):
    g = grid(2, (32, 32), (40.0, 40.0))
    F = [W.Term(1, 0.8, W.gauss(2.0, k=0.5), [W.gauss(5.0), W.gauss(6.0), W.const()]),
         W.Term(0, 0.2, W.sech2(2.0), [W.ugauss(4.0), W.gauss(5.0), W.const()])]
    k = [2 * np.pi * 2 / 40.0, 0.0, 1.1]
    p = [2 * np.pi * 3 / 40.0, -2 * np.pi / 40.0, 0.4]
    q = [0.2, 0.3, 0.7]
    modes = [([0.5, 0.1, 1.1], [0.0, 0.6, 0.8], 0.7 - 0.1j), (k, [0.8, 0.0, 0.6], 0.2 + 0.5j)]
    prob = ip(W.Problem("bw2", [g], [F], [W.Solve(0, 1, p), W.Solve(1, -1, q)], W.Window(-6.0, 6.0, 0.05),
                        [W.Vertex(0, 1, k, [0.0, 0.6, 0.8]), W.Vertex(0, 1, k, [0.0, 0.6, 0.8], modes)]))
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        for v, Vx in ((0, obw.Vertex), (1, obw.PacketVertex)):
            ref = Vx(prob, v).amplitude()
            for term in range(3):
                want = ref["terms"][term]
                assert abs(ctx.bw(v, term) - want) <= 1e-9 * abs(want) + 1e-14, (v, term)


def test_iprk4_graph_replay_bitwise(S):
    prob = ip(problem(2, (32, 32), (30.0, 30.0), kinds=(W.U_OUT, W.V_OUT), spins=(1,), n_mom=1, t_half=1.0))
    out = []
    for use_graph in (False, True):
        with S.Context(prob, precision="fp64", use_graph=use_graph) as ctx:
            ctx.step(7)
            ctx.sync()
            ctx.step()
            out.append([ctx.get_psi(i) for i in range(len(prob.solves))])
    for a, b in zip(*out):
        assert np.array_equal(a, b)


def test_iprk4_errors(S):
    prob = ip(W.config_bw_1d(n=64, L=100.0, steps=4))
    with pytest.raises(S.SwfError) as e:
        S.Context(prob, precision="fp64", bw_partial=True)
    assert e.value.code == S.SWF_E_UNSUPPORTED


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_iprk4_launch_config_2d_512_x64_pure_gauge(S, prec):
    # the 2D workload's launch configuration (64 solves on 512^2) stepped by the
    # interaction picture through a pure-gauge pulse: the scattered wave is
    # (exp(-i Lambda) - 1) psi_back at every site, checked at sampled sites
    from test_gpu_fullsize import pure_gauge_check
    lam0, tau, w = 0.8, 4.0, 10.0
    prob = W.config_2d(n_solves=64, t_half=60.0)
    prob.fields = [W.field_pure_gauge(lam0, tau, w, 2)]
    prob.window = W.Window(0.0, 24.0, 0.02, "iprk4")
    pure_gauge_check(S, prob, lam0, tau, w, prec, prob.window.steps)
