"""GPU test of swf_pair_matrix_noalloc: the pair-amplitude matrix of eq. (Nmn)
with its device scratch in the library's static array instead of context
memory.

Two calls in a row through the C ABI on one context, the second on a smaller
matrix (so stale partial tiles of the first call would show), each against
swf_pair_matrix on the same states.  Both runs split the site sums over
different numbers of ranges (the static array holds fewer partial tiles), so
they agree to FP64 rounding of the sums: 1e-12 of the largest |Omega|.  A
matrix beyond the array's size is rejected before any work is queued.
"""
import ctypes as C

import numpy as np
import pytest

import swf_workloads as W

from swf_cases import field_mix, grid, lattice_p

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def S():
    from paper_2512_16889_amd import swf
    return swf


def batch(nu, nv, seed):
    # 96 x 96 sites: more site ranges than the static array leaves room for,
    # so the no-allocation call runs with fewer splits than swf_pair_matrix
    g = grid(2, (96, 96), (40.0, 40.0))
    rng = np.random.default_rng(seed)
    solves = []
    for kind, count, sgn in ((0, nu, 1.0), (1, nv, -1.0)):
        for i in range(count):
            m = [int(rng.integers(-3, 4)) for _ in range(3)]
            p = lattice_p(2, g.n, g.L, m, trivial=(0.3 * sgn, 0.0))
            p = [p[j] + (0.37 * (2 * np.pi / g.L[j]) if (j < 2 and i % 2) else 0.0) for j in range(3)]
            solves.append(W.Solve(kind, 1 if i % 3 else -1, p))
    prob = W.Problem("pairs", [g], [field_mix(2)], solves, W.Window(-1.0, 1.0, 0.05))
    return prob, list(range(nu)), list(range(nu, nu + nv))


def call(S, ctx, fn, us, vs, form):
    a = (C.c_int * len(us))(*us)
    b = (C.c_int * len(vs))(*vs)
    out = np.zeros(2 * len(us) * len(vs))
    code = fn(ctx._ctx, form, a, len(us), b, len(vs), out.ctypes.data_as(C.POINTER(C.c_double)))
    return code, (out[0::2] + 1j * out[1::2]).reshape(len(us), len(vs))


def test_noalloc_pair_matrix_matches_allocating_call(S):
    prob, us, vs = batch(70, 67, seed=5)
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        ctx.sync()
        for form, (mu, mv) in ((1, (70, 67)), (2, (5, 9))):
            u, v = us[:mu], vs[:mv]
            print(f"noalloc pair matrix: form {form}, {mu} x {mv} on 96x96", flush=True)
            code, got = call(S, ctx, S._lib.swf_pair_matrix_noalloc, u, v, form)
            assert code == S.SWF_OK, S._lib.swf_last_error(ctx._ctx).decode()
            code, ref = call(S, ctx, S._lib.swf_pair_matrix, u, v, form)
            assert code == S.SWF_OK, S._lib.swf_last_error(ctx._ctx).decode()
            scale = np.abs(ref).max()
            assert scale > 0
            err = float(np.abs(got - ref).max() / scale)
            assert err < 1e-12, err


def test_noalloc_pair_matrix_rejects_oversize(S):
    prob, us, vs = batch(1, 1, seed=6)
    with S.Context(prob, precision="fp64") as ctx:
        ctx.step()
        ctx.sync()
        assert S.noalloc_scratch_bytes() == 32 << 20
        big = 1025
        code, _ = call(S, ctx, S._lib.swf_pair_matrix_noalloc, [us[0]] * big, [vs[0]] * big, 1)
        assert code == S.SWF_E_ARG
        assert "static" in S._lib.swf_last_error(ctx._ctx).decode()
        # the context still works after the rejection
        code, got = call(S, ctx, S._lib.swf_pair_matrix_noalloc, us, vs, 1)
        assert code == S.SWF_OK
        assert np.isfinite(got).all()
