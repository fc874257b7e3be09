"""GPU parity of the pair-amplitude matrix (swf_pair_matrix, eq. (Nmn)).

Omega(m, n) for every pair of U and V solves, computed as two dense complex
contractions on the FP64 matrix cores, against
* the FP64 oracle's pair amplitude, element by element, for every pair of a
  small 2D batch (both forms) and a 1D batch;
* the per-pair path (swf_amplitude, itself checked against the oracle) for
  a 3D batch of 70 U x 67 V solves: two 64 x 64 output tiles in each
  direction with ragged edges, and more sites than one split covers;
* the same in mixed precision (FP32 states, FP64 products and sums);
and the error paths (order, form, trivial-axis momentum, solve kinds).
FP64: 1e-10 of the largest |Omega| (the orderings of the sums differ);
mixed: 1e-6 against the per-pair path on the same FP32 states.
"""
import numpy as np
import pytest

import swf_workloads as W
from oracle import observables as ob
from oracle.swf import SWFSolve

from swf_cases import field_mix, grid, lattice_p

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2512_16889_amd import swf
    return swf


def close(got, ref, tol):
    scale = np.abs(ref).max()
    assert scale > 0
    err = float(np.abs(got - ref).max() / scale)
    assert err < tol, err


def batch(dim, n, L, nu, nv, seed, t_half=2.0, dt=0.05, trivial=(0.3, -0.2)):
    g = grid(dim, n, L)
    rng = np.random.default_rng(seed)
    solves = []
    for kind, count, sgn in ((0, nu, 1.0), (1, nv, -1.0)):
        for i in range(count):
            m = [int(rng.integers(-3, 4)) for _ in range(3)]
            p = lattice_p(dim, g.n, g.L, m, trivial=tuple(sgn * t for t in trivial))
            # off-lattice momenta too: the direct term is a continuum Fourier coefficient
            p = [p[j] + (0.37 * (2 * np.pi / g.L[j]) if (j < dim and i % 2) else 0.0) for j in range(3)]
            solves.append(W.Solve(kind, 1 if i % 3 else -1, p))
    prob = W.Problem("pairs", [g], [field_mix(dim)], solves, W.Window(-t_half, t_half, dt))
    return prob, list(range(nu)), list(range(nu, nu + nv))


@pytest.mark.parametrize("form", [1, 2])
def test_pair_matrix_2d_vs_oracle(S, form):
    prob, us, vs = batch(2, (32, 48), (30.0, 36.0), 3, 4, seed=1)
    tin = prob.window.t_in
    runs = {i: (SWFSolve(prob, i), None) for i in us + vs}
    runs = {i: (sv, sv.run()) for i, (sv, _) in runs.items()}
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        got = ctx.pair_matrix(us, vs, form)
    ref = np.array([[ob.pair_amplitude(runs[u][0], runs[u][1], runs[v][0], runs[v][1], tin, form) for v in vs]
                    for u in us])
    close(got, ref, 1e-10)


def test_pair_matrix_1d_vs_oracle(S):
    prob, us, vs = batch(1, (64,), (40.0,), 4, 3, seed=2)
    tin = prob.window.t_in
    runs = {i: SWFSolve(prob, i) for i in us + vs}
    ys = {i: runs[i].run() for i in runs}
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        got = ctx.pair_matrix(us, vs, 1)
    ref = np.array([[ob.pair_amplitude(runs[u], ys[u], runs[v], ys[v], tin, 1) for v in vs] for u in us])
    close(got, ref, 1e-10)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-10), ("mixed", 1e-6)])
def test_pair_matrix_3d_tiles_vs_per_pair(S, prec, tol):
    prob, us, vs = batch(3, (16, 16, 16), (18.0, 18.0, 18.0), 70, 67, seed=3, t_half=1.0)
    with S.Context(prob, precision=prec) as ctx:
        ctx.step()
        got1 = ctx.pair_matrix(us, vs, 1)
        got2 = ctx.pair_matrix(us, vs, 2)
        # the per-pair path on a sample that covers every tile and the ragged edges
        rows = [0, 5, 33, 63, 64, 69]
        cols = [0, 17, 40, 63, 64, 66]
        ref1 = np.array([[ctx.pair(us[m], vs[n], 1) for n in cols] for m in rows])
        ref2 = np.array([[ctx.pair(us[m], vs[n], 2) for n in cols] for m in rows])
    close(got1[np.ix_(rows, cols)], ref1, tol)
    close(got2[np.ix_(rows, cols)], ref2, tol)


def test_pair_matrix_subsets_and_repeat(S):
    prob, us, vs = batch(2, (16, 16), (20.0, 20.0), 5, 6, seed=4)
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        full = ctx.pair_matrix(us, vs, 1)
        again = ctx.pair_matrix(us, vs, 1)
        sub = ctx.pair_matrix([us[3], us[1]], [vs[5]], 1)
    assert np.array_equal(full, again)                       # fixed-order sums: bitwise repeatable
    close(sub, full[np.ix_([3, 1], [5])], 1e-12)


def test_pair_matrix_errors(S):
    prob, us, vs = batch(2, (16, 16), (20.0, 20.0), 2, 2, seed=5)
    with S.Context(prob, precision="fp64") as ctx:
        with pytest.raises(S.SwfError) as e:
            ctx.pair_matrix(us, vs, 1)
        assert e.value.code == S.SWF_E_ORDER
        ctx.step()
        with pytest.raises(S.SwfError) as e:
            ctx.pair_matrix(us, vs, 3)
        assert e.value.code == S.SWF_E_ARG
        with pytest.raises(S.SwfError) as e:
            ctx.pair_matrix(vs, us, 1)                       # kinds swapped
        assert e.value.code == S.SWF_E_ARG
    # a V solve whose trivial-axis momentum does not balance the U solves'
    g = grid(2, (16, 16), (20.0, 20.0))
    bad = W.Problem("bad", [g], [field_mix(2)],
                    [W.Solve(0, 1, [0.1, 0.2, 0.3]), W.Solve(1, 1, [0.0, 0.1, -0.3]), W.Solve(1, 1, [0.0, 0.1, 0.2])],
                    W.Window(-1.0, 1.0, 0.05))
    with S.Context(bad, precision="fp64") as ctx:
        ctx.step()
        assert ctx.pair_matrix([0], [1], 1).shape == (1, 1)
        with pytest.raises(S.SwfError) as e:
            ctx.pair_matrix([0], [1, 2], 1)
        assert e.value.code == S.SWF_E_ARG
