"""GPU parity at the workloads' full grid sizes, for every tile variant.

* 2D grids of every benchmark length (256 ... 1024): one RK4 step from a
  random state, element by element against the oracle's step, for each tile
  variant forced in turn (every kernel the autotuner can pick) and both
  precisions; and narrow grids of 768 and 1024 points along y with enough
  solves that the persistent y pass steps several tiles per workgroup.
* 3D: the lengths 256 and 320 on each axis in turn (the other axes short), so
  the row pass and both column passes of those lengths are checked against
  the oracle.
* The (1+1)D line of 1024 points: one step through every pass-path tile
  variant and through the whole-loop kernel, against the oracle.
* The benchmark launch configurations themselves (64 x 512^2, 8 x 256^3,
  320^3) are too large for the oracle; there a pure-gauge field is stepped
  through the same kernels and tiles and the scattered wave is compared at
  sampled sites with its closed form (exp(-i Lambda) - 1) psi_back, which
  holds at any grid size.  At 320^3 the BW vertex integrals are checked the
  same way: with that closed form every integrand is a plane-wave factor
  times lattice sums that reduce to one-dimensional sums.
FP64 to 1e-12 (one step) or 1e-5 (closed form, limited by the RK4 and
spectral discretisation); mixed precision to 2e-6 (one step) or 3e-4
(closed form).
"""
import numpy as np
import pytest

import swf_workloads as W
from oracle.swf import SWFSolve

pytestmark = pytest.mark.gpu

_REF = {}


@pytest.fixture(scope="module")
def S():
    from paper_2512_16889_amd import swf
    return swf


def relerr(a, b):
    return float(np.abs(a - b).max() / np.abs(b).max())


def reference_step(key, prob, k0):
    """Random states and the oracle's one-step results, cached per problem."""
    if key not in _REF:
        states, refs = [], []
        for i, sv in enumerate(prob.solves):
            g = prob.grids[sv.grid]
            psi = W.random_state((4,) + tuple(g.n[:g.dim]), seed=17 + i, scale=0.05)
            states.append(psi)
            refs.append(SWFSolve(prob, i).step(k0, psi))
        _REF[key] = (states, refs)
    return _REF[key]


def one_step_case(S, key, prob, prec, variant, persistent=True):
    k0 = prob.window.steps // 2
    states, refs = reference_step(key, prob, k0)
    tol = 1e-12 if prec == "fp64" else 2e-6
    with S.Context(prob, precision=prec, variant=variant, persistent=persistent) as ctx:
        for i, psi in enumerate(states):
            ctx.set_psi(i, psi, k0)
        ctx.step(1)
        ctx.sync()
        for i in range(len(states)):
            err = relerr(ctx.get_psi(i), refs[i])
            assert err < tol, (prec, variant, i, err)


@pytest.mark.parametrize("n", [256, 384, 512, 768, 1024])
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_2d_full_length_one_step(S, n, variant, prec):
    prob = W.config_2d(n=n, n_solves=1, seed=n)
    one_step_case(S, ("2d", n), prob, prec, variant)


@pytest.mark.parametrize("n", [768, 1024])
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_2d_persistent_column_loop(S, n, variant):
    # FP64 y passes of 768 and 1024 points whose tiles fill the LDS run as one
    # persistent workgroup per compute unit: 72 solves of 64 x n give 576
    # tiles, so each workgroup steps two or three of them (the last round
    # ragged), loading the next while it transforms the current one
    prob = W.config_2d(n=n, n_solves=72, seed=n + 1)
    prob.grids = [W.Grid(2, [64, n, 1], [20.0, 160.0, 1.0])]
    one_step_case(S, ("2d_narrow", n), prob, "fp64", variant)


@pytest.mark.parametrize("axis", [0, 1, 2])
@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("n", [256, 320])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_3d_full_length_each_axis(S, axis, n, variant, prec):
    shape = [16, 16, 16]
    shape[axis] = n
    L = [12.0, 12.0, 12.0]
    L[axis] = 60.0 * n / 256
    F = [W.Term(3, 0.8, W.sech2(8.0), [W.gauss(4.0), W.gauss(4.0), W.gauss(4.0)]),
         W.Term(1, 0.3, W.gauss(6.0), [W.gauss(3.0), W.sech2(3.0), W.gauss(3.5)])]
    prob = W.Problem("3d_axis", [W.Grid(3, shape, L)], [F], [W.Solve(0, 1, [0.2, -0.1, 0.5])],
                     W.Window(-50.0, 50.0, 0.025))
    one_step_case(S, ("3d", axis, n), prob, prec, variant)


def pure_gauge_check(S, prob, lam0, tau, w, prec, steps, nsample=2048, variant=None):
    """Step a pure-gauge problem and compare sampled sites with the closed form."""
    from oracle import dirac
    rng = np.random.default_rng(5)
    tol = 1e-5 if prec == "fp64" else 3e-4
    with S.Context(prob, precision=prec, tune=variant is None, variant=variant) as ctx:
        ctx.step(steps)
        ctx.sync()
        t = prob.window.t_out - steps * prob.window.dt
        for i, sv in enumerate(prob.solves):
            g = prob.grids[sv.grid]
            psi = ctx.get_psi(i)
            n = g.n[:g.dim]
            idx = [rng.integers(0, n[j], nsample) for j in range(g.dim)]
            x = [-g.L[j] / 2 + idx[j] * g.L[j] / n[j] for j in range(g.dim)]
            lam = lam0 * np.exp(-t ** 2 / tau ** 2 - sum(xj ** 2 for xj in x) / w ** 2)
            wsp, E, K = dirac.background_spinor(sv.kind, sv.spin, sv.p)
            back = wsp[:, None] * np.exp(-1j * E * t + 1j * sum(K[j] * x[j] for j in range(g.dim)))[None]
            ref = (np.exp(-1j * lam) - 1.0)[None] * back
            got = psi[(slice(None),) + tuple(idx)]
            assert np.abs(ref).max() > 0.1
            err = float(np.abs(got - ref).max() / np.abs(ref).max())
            assert err < tol, (prec, i, err)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_launch_config_2d_512_x64_pure_gauge(S, prec):
    lam0, tau, w = 0.8, 4.0, 10.0
    prob = W.config_2d(n_solves=64, t_half=60.0)
    prob.fields = [W.field_pure_gauge(lam0, tau, w, 2)]
    prob.window = W.Window(0.0, 24.0, 0.02)            # Lambda(t_out) ~ 1e-16; ends at the pulse maximum
    pure_gauge_check(S, prob, lam0, tau, w, prec, prob.window.steps)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_launch_config_3d_256_x8_pure_gauge(S, prec):
    lam0, tau, w = 0.8, 2.0, 8.0
    prob = W.config_3d()
    prob.fields = [W.field_pure_gauge(lam0, tau, w, 3)]
    prob.window = W.Window(0.0, 12.0, 0.025)
    pure_gauge_check(S, prob, lam0, tau, w, prec, prob.window.steps)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_launch_config_ragged_256_pure_gauge(S, prec):
    # the ragged batch's own launch configuration: 256 solves on the five grid
    # sizes of the seed-0 draw (one launch group per size, the 1024^2 group
    # with its XCD-grouped column tiles), one pure-gauge field for all
    lam0, tau, w = 0.8, 2.0, 10.0
    prob = W.config_ragged_2d()
    sizes = sorted(set(g.n[0] for g in prob.grids))
    assert sizes == [256, 384, 512, 768, 1024] and len(prob.solves) == 256
    prob.fields = [W.field_pure_gauge(lam0, tau, w, 2)]
    for s in prob.solves:
        s.field = 0
    prob.window = W.Window(0.0, 12.0, 0.02)            # Lambda(t_out) ~ 1e-16; ends at the pulse maximum
    pure_gauge_check(S, prob, lam0, tau, w, prec, prob.window.steps, nsample=512)


def test_launch_config_3d_320_pure_gauge(S):
    lam0, tau, w = 0.8, 2.0, 8.0
    prob = W.config_bw_3d(n_p=1)
    prob.fields = [W.field_pure_gauge(lam0, tau, w, 3)]
    prob.vertices = []
    prob.window = W.Window(0.0, 12.0, 0.025)
    pure_gauge_check(S, prob, lam0, tau, w, "mixed", prob.window.steps)


def pure_gauge_bw_reference(prob, lam0, tau, w, nsteps):
    """Accumulated vertex integrals M_ab after nsteps for a pure-gauge field,
    where every scattered wave is (exp(-i Lambda) - 1) psi_back.  The three
    integrands are then plane-wave factors times lattice sums of
    2 - 2 cos Lambda, exp(-i Lambda) - 1 and exp(i Lambda) - 1 with
    Lambda = c(t) g(x) g(y) g(z); their power series in c reduce every sum to
    products of one-dimensional sums (exact to rounding at any grid size).
    Integrated with the RK4 weights at the stage times (Simpson), which agrees
    with the augmented RK4 to O(dt^4)."""
    from math import factorial
    from oracle import dirac
    from oracle.bw import gamma_eps
    g = prob.grids[0]
    win = prob.window
    x = [-g.L[j] / 2 + np.arange(g.n[j]) * g.L[j] / g.n[j] for j in range(3)]
    dV = np.prod([g.L[j] / g.n[j] for j in range(3)])
    J = 48
    out = []
    for vx in prob.vertices:
        wu, Eu, Ku = dirac.background_spinor(0, prob.solves[vx.u_solve].spin, prob.solves[vx.u_solve].p)
        wv, Ev, Kv = dirac.background_spinor(1, prob.solves[vx.v_solve].spin, prob.solves[vx.v_solve].p)
        k3 = np.asarray(vx.k, dtype=float)
        k0 = float(np.linalg.norm(k3))
        amp = np.conj(wu) @ (gamma_eps(vx.eps) @ wv)
        Q = Kv - Ku + k3
        # S_j = prod over axes of sum_i g(x_i)^j e^{i Q_a x_i}
        Sj = np.array([np.prod([np.sum(np.exp(-j * x[a] ** 2 / w ** 2 + 1j * Q[a] * x[a])) for a in range(3)])
                       for j in range(J + 1)])

        def mdot(t):
            c = lam0 * np.exp(-t ** 2 / tau ** 2)
            s_e = sum((-1j * c) ** j * Sj[j] / factorial(j) for j in range(1, J + 1))        # exp(-i L) - 1
            s_ec = sum((1j * c) ** j * Sj[j] / factorial(j) for j in range(1, J + 1))        # exp(+i L) - 1
            s_cos = -(s_e + s_ec)                                                              # 2 - 2 cos L
            ph = dV * amp * np.exp(1j * (Eu - Ev - k0) * t)
            return ph * np.array([s_cos, s_e, s_ec])

        h = -win.dt
        M = np.zeros(3, dtype=complex)
        for n in range(nsteps):
            t = win.t_out - n * win.dt
            M += h / 6.0 * (mdot(t) + 4.0 * mdot(t + h / 2) + mdot(t + h))
        out.append(M)
    return out


@pytest.mark.parametrize("photons", ["one", "four"])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-5), ("mixed", 3e-4)])
def test_launch_config_bw_320_pure_gauge(S, prec, tol, photons):
    # the BW vertex reduction in the 320^3 launch configuration (one momentum,
    # four spin pairs: 2 U + 2 V solves, 4 vertices) against the closed form:
    # with the workload's one photon the four vertices are reduced as one
    # group (each solve read once); with four photons, one group each
    lam0, tau, w = 0.8, 2.0, 8.0
    prob = W.config_bw_3d(n_p=1)
    prob.fields = [W.field_pure_gauge(lam0, tau, w, 3)]
    if photons == "four":
        ks = [([0.0, 0.0, 2.0], [-1.0, 0.0, 0.0]), ([0.3, 0.0, 1.9], [0.0, 1.0, 0.0]),
              ([0.0, -0.4, 1.8], [0.6, 0.0, 0.8]), ([0.2, 0.25, 2.2], [0.0, 0.8, -0.6])]
        prob.vertices = [W.Vertex(vx.u_solve, vx.v_solve, k, e) for vx, (k, e) in zip(prob.vertices, ks)]
    prob.window = W.Window(0.0, 8.0, 0.05)             # Lambda(t_out) ~ 1e-7, ends at the pulse maximum
    nsteps = prob.window.steps
    ref = pure_gauge_bw_reference(prob, lam0, tau, w, nsteps)
    with S.Context(prob, precision=prec) as ctx:
        ctx.step(nsteps)
        ctx.sync()
        for v in range(len(prob.vertices)):
            got = ctx.get_bw_state(v)
            assert np.abs(ref[v]).min() > 1.0
            err = float(np.abs(got - ref[v]).max() / np.abs(ref[v]).max())
            assert err < tol, (prec, v, err, got, ref[v])


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
def test_1d_1024_one_step(S, variant):
    # the pass path's tile variants (the whole-loop kernel switched off)
    prob = W.config_1d()
    one_step_case(S, ("1d",), prob, "fp64", variant, persistent=False)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_1d_1024_one_step_whole_loop(S, prec):
    prob = W.config_1d()
    one_step_case(S, ("1d",), prob, prec, None)


@pytest.mark.parametrize("variant", [0, 1, 2, 3])
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("mixed", 5e-6)])
def test_row_pass_variants_with_absorber(S, variant, prec, tol):
    """Every row-pass tile variant finishes the RK4 step with the boundary
    mask: three steps from a random state on a 320 x 16 lattice with the mask
    on and trivial-axis momenta, against the oracle."""
    g = W.Grid(2, [320, 16, 1], [90.0, 12.0, 1.0], absorb_cells=6, absorb_strength=0.3)
    F = [W.Term(1, 0.6, W.gauss(3.0), [W.gauss(8.0), W.gauss(3.0), W.const()]),
         W.Term(0, 0.2, W.sech2(2.0), [W.ugauss(6.0), W.const(), W.const()])]
    prob = W.Problem("cs_abs", [g], [F], [W.Solve(0, 1, [0.3, -0.2, 0.1]), W.Solve(1, -1, [0.1, 0.2, -0.1])],
                     W.Window(-2.0, 2.0, 0.025))
    k0 = 40
    states = [W.random_state((4, 320, 16), seed=70 + i, scale=0.1) for i in range(2)]
    with S.Context(prob, precision=prec, variant=variant) as ctx:
        for i, psi in enumerate(states):
            ctx.set_psi(i, psi, k0)
        ctx.step(3)
        ctx.sync()
        for i in range(2):
            ref = SWFSolve(prob, i).run(states[i], start=k0, count=3)
            err = relerr(ctx.get_psi(i), ref)
            assert err < tol, (prec, variant, i, err)


def test_bw_320_shape_mixed_against_fp64_full_window(S):
    """The Breit-Wheeler workload's shape over its whole 3000-step window on a
    48^3 lattice over the same box (32 solves, 32 vertices): the mixed path's
    |M|^2 of every vertex against the FP64 path's, to the 1e-4 the benchmark
    states for the mixed path."""
    import dataclasses
    prob = W.config_bw_3d()
    prob = dataclasses.replace(prob, grids=[dataclasses.replace(prob.grids[0], n=[48, 48, 48])])
    vals = {}
    for prec in ("fp64", "mixed"):
        with S.Context(prob, precision=prec) as ctx:
            ctx.step()
            vals[prec] = np.array([abs(ctx.bw(v)) ** 2 for v in range(len(prob.vertices))])
    assert vals["fp64"].min() > 0
    err = np.abs(vals["mixed"] - vals["fp64"]) / vals["fp64"]
    print(f"48^3 full window: max rel |M|^2 error mixed vs fp64 {err.max():.3e}")
    assert err.max() < 1e-4
