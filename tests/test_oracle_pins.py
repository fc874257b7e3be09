"""Physics pins of the oracle's SWF solver and observables (CPU only).

Each test ties the oracle to an independent statement:
* A = 0 gives psi_scat = 0 exactly (eq. (scatDirac) has no source);
* a pure-gauge potential A = dLambda has the closed-form scattered wave
  (exp(-i Lambda) - 1) psi_back (from D_mu = d_mu + i A_mu, eq. (DiracEq));
* the full psi = psi_b + psi_s keeps its norm: 2Re(psi_b|psi_s) + (psi_s|psi_s) = 0;
* (U_out|V_out) = 0 (appendix "Exact spin dependence"), hence form 1 = -form 2
  of eq. (Nmn);
* Sauter pulse: Narozhny-Nikishov closed-form pair number per mode;
* brute force: the full wave function evolved with scipy's DOP853 (an
  independent integrator and an independently written Hamiltonian) gives the
  same marginal and pair amplitude;
* charge-conjugation + reflection symmetry of the spectrum;
* RK4 converges at order 4 in dt;
* a 90-degree rotation of field and momentum on a square lattice leaves the
  spin-summed marginal unchanged;
* summed over every lattice mode, electrons and positrons balance.
"""
import numpy as np
import pytest
from scipy.integrate import solve_ivp

import swf_workloads as W
from oracle import dirac
from oracle import observables as ob
from oracle.swf import SWFSolve

pytestmark = pytest.mark.filterwarnings("ignore")


def one_d_problem(solves, n=96, L=80.0, dt=0.025, t_half=20.0, a=1.2, tau=3.0, w=6.0):
    F = [W.Term(1, a, W.sech2(tau), [W.sech2(w), W.const(), W.const()])]
    return W.Problem("p", [W.Grid(1, [n, 1, 1], [L, 1, 1])], [F], solves, W.Window(-t_half, t_half, dt))


def test_zero_field_gives_zero_scattered_wave():
    prob = W.Problem("z", [W.Grid(2, [16, 16, 1], [10.0, 10.0, 1])], [[]],
                     [W.Solve(0, 1, [0.3, -0.2, 0.1])], W.Window(-1.0, 1.0, 0.1))
    sv = SWFSolve(prob, 0)
    assert np.all(sv.run() == 0)


def test_pure_gauge_closed_form_2d():
    lam0, tau, w, n, L = 0.7, 2.0, 3.0, 40, 24.0
    p = [2 * np.pi * 2 / L, -2 * np.pi / L, 0.3]
    prob = W.Problem("pg", [W.Grid(2, [n, n, 1], [L, L, 1])], [W.field_pure_gauge(lam0, tau, w, 2)],
                     [W.Solve(0, 1, p)], W.Window(-12.0, 12.0, 0.02))
    sv = SWFSolve(prob, 0)
    half = prob.window.steps // 2
    for start, count in ((0, half - 100), (half - 100, 100)):
        y = sv.run(None if start == 0 else y, start=start, count=count)
        t = sv.time(start + count)
        Lam = lam0 * np.exp(-t ** 2 / tau ** 2 - (sv.lat.X[0] ** 2 + sv.lat.X[1] ** 2) / w ** 2)
        ref = (np.exp(-1j * Lam) - 1)[None] * sv.psi_back(t)
        assert np.abs(y - ref).max() < 1e-5 * np.abs(ref).max()
    y = sv.run(y, start=half)
    assert ob.marginal(sv, y) < 1e-12


def test_norm_identity_and_orthogonality():
    L = 80.0
    px = 2 * np.pi * 5 / L
    qx = -2 * np.pi * 3 / L
    prob = one_d_problem([W.Solve(0, 1, [px, 0.2, 0.0]), W.Solve(1, 1, [qx, -0.2, 0.0])], L=L)
    su, sv = SWFSolve(prob, 0), SWFSolve(prob, 1)
    yu, yv = su.run(), sv.run()
    tin = prob.window.t_in
    for s, y in ((su, yu), (sv, yv)):
        ss, bs = ob.diagnostics(s, y, tin)
        assert ss > 1.0 and abs(ss + bs) < 1e-7 * ss
    dV = su.lat.dV
    orth = ob.inner(su.psi_back(tin), yv, dV) + ob.inner(yu, sv.psi_back(tin), dV) + ob.inner(yu, yv, dV)
    f1 = ob.pair_amplitude(su, yu, sv, yv, tin, 1)
    f2 = ob.pair_amplitude(su, yu, sv, yv, tin, 2)
    assert abs(f1) > 1e-3
    assert abs(orth) < 1e-7 * abs(f1)
    assert abs(f1 + f2) < 1e-6 * abs(f1)


def sauter_closed_form(E0, tau, px, pperp):
    """Pair number per mode for E(t) = E0 sech^2(t/tau) (Narozhny-Nikishov),
    with px the final (t -> +inf) momentum along the field."""
    pt = px - E0 * tau
    ep = np.sqrt(1 + pperp ** 2 + (pt + E0 * tau) ** 2)
    em = np.sqrt(1 + pperp ** 2 + (pt - E0 * tau) ** 2)
    num = np.sinh(np.pi * tau / 2 * (2 * E0 * tau + em - ep)) * np.sinh(np.pi * tau / 2 * (2 * E0 * tau - em + ep))
    return num / (np.sinh(np.pi * tau * ep) * np.sinh(np.pi * tau * em))


@pytest.mark.parametrize("E0,tau,px,pperp", [(0.5, 2.0, 0.3, 0.2), (1.0, 1.0, -0.5, 0.5), (0.4, 1.5, 0.8, 0.0)])
@pytest.mark.parametrize("spin", [1, -1])
def test_sauter_pulse_closed_form(E0, tau, px, pperp, spin):
    L = 2 * np.pi / abs(px)          # the momentum sits on the lattice
    T = 16.0 * tau
    prob = W.Problem("s", [W.Grid(1, [4, 1, 1], [L, 1, 1])], [W.field_sauter_time(E0, tau)],
                     [W.Solve(0, spin, [px, pperp, 0.0])], W.Window(-T, T, 0.005 * tau))
    sv = SWFSolve(prob, 0)
    y = sv.run()
    A_in = [0.0, E0 * tau * (np.tanh(-T / tau) - 1.0), 0.0, 0.0]
    P = ob.marginal_in_uniform_field(sv, y + sv.psi_back(prob.window.t_in), A_in)
    assert P / L == pytest.approx(sauter_closed_form(E0, tau, px, pperp), rel=2e-6)


def _brute_force_full(sv, problem, a, tau, w):
    """Evolve the full psi from psi_back(t_out) to t_in with DOP853; the
    Hamiltonian is written out here independently of the oracle."""
    lat = sv.lat
    k = [lat.k1d[0], np.full(lat.shape, sv.K[1]), np.full(lat.shape, sv.K[2])]
    H0 = sum(dirac.ALPHA[j][:, :, None] * k[j][None, None] for j in range(3)) + dirac.BETA[:, :, None]
    x = lat.x1d[0]

    def f(t, yf):
        psi = yf.view(complex).reshape(4, -1)
        pk = np.fft.fft(psi, axis=1)
        kin = np.fft.ifft(np.einsum("abk,bk->ak", H0, pk), axis=1)
        A1 = a / np.cosh(t / tau) ** 2 / np.cosh(x / w) ** 2
        pot = dirac.ALPHA[0] @ psi * A1[None]
        return (-1j * (kin + pot)).reshape(-1).view(float)

    y0 = sv.psi_back(problem.window.t_out).astype(complex).reshape(-1).view(float)
    sol = solve_ivp(f, (problem.window.t_out, problem.window.t_in), y0, method="DOP853", rtol=1e-12, atol=1e-13)
    return sol.y[:, -1].view(complex).reshape(4, -1)


def test_brute_force_full_evolution():
    L, a, tau, w = 80.0, 1.2, 3.0, 6.0
    p = [2 * np.pi * 5 / L, 0.2, 0.0]
    q = [-2 * np.pi * 3 / L, -0.2, 0.0]
    prob = one_d_problem([W.Solve(0, 1, p), W.Solve(1, 1, q)], L=L, dt=0.0125, a=a, tau=tau, w=w)
    su, sv = SWFSolve(prob, 0), SWFSolve(prob, 1)
    yu, yv = su.run(), sv.run()
    fu = _brute_force_full(su, prob, a, tau, w)
    fv = _brute_force_full(sv, prob, a, tau, w)
    tin = prob.window.t_in
    Pbf = float(np.real(ob.projected_overlap(su, fu, fu, -1)))
    assert ob.marginal(su, yu) == pytest.approx(Pbf, rel=1e-8)
    Pbf_v = float(np.real(ob.projected_overlap(sv, fv, fv, +1)))
    assert ob.marginal(sv, yv) == pytest.approx(Pbf_v, rel=1e-8)
    Obf = ob.projected_overlap(su, fu, fv, -1)      # (U_out|Pi_-|V_out) = form 2
    f2 = ob.pair_amplitude(su, yu, sv, yv, tin, 2)
    assert abs(Obf - f2) < 1e-7 * abs(f2)


def test_charge_conjugation_reflection_symmetry():
    # A_1 even in x: spin-summed P_e(p) equals spin-summed P_pos(R p), R: x -> -x
    L = 80.0
    p = [2 * np.pi * 4 / L, 0.3, 0.0]
    q = [-p[0], 0.3, 0.0]
    prob = one_d_problem([W.Solve(0, 1, p), W.Solve(0, -1, p), W.Solve(1, 1, q), W.Solve(1, -1, q)], L=L)
    P = [ob.marginal(SWFSolve(prob, i), SWFSolve(prob, i).run()) for i in range(4)]
    assert P[0] + P[1] == pytest.approx(P[2] + P[3], rel=1e-9)
    assert P[0] > 1e-6


def test_rk4_order_four():
    L = 80.0
    p = [2 * np.pi * 5 / L, 0.2, 0.0]
    vals = []
    for dt in (0.1, 0.05, 0.025):
        prob = one_d_problem([W.Solve(0, 1, p)], L=L, dt=dt, t_half=12.0)
        sv = SWFSolve(prob, 0)
        vals.append(sv.run())
    e1 = np.abs(vals[0] - vals[2]).max()
    e2 = np.abs(vals[1] - vals[2]).max()
    # Richardson: e(dt)/e(dt/2) = (2^4 - 1) * 2^4 / (2^4 - 1) ... for order 4 the ratio of
    # differences against the finest run is (1 - 2^-8)/(1 - 2^-4)*2^4 ~ 17
    ratio = e1 / e2
    assert 14.0 < ratio < 20.0


def test_spatial_refinement_converges_spectrally():
    # P12: at fixed box and dt, the marginal converges exponentially in the
    # number of grid points (pseudo-spectral derivative, smooth field): the
    # error against n = 96 drops by more than 20x for every 8 points added,
    # which no fixed-order difference scheme does (order k gives 1.25^k at
    # 32 -> 40), and is at rounding level from n = 64 on
    L = 40.0
    F = [W.Term(1, 0.6, W.gauss(1.0), [W.gauss(3.0), W.const(), W.const()]),
         W.Term(0, 0.4, W.sech2(1.2), [W.ugauss(2.5), W.const(), W.const()])]
    p = [2 * np.pi * 2 / L, 0.2, 0.0]
    P = {}
    for n in (32, 40, 48, 64, 96):
        prob = W.Problem("c", [W.Grid(1, [n, 1, 1], [L, 1, 1])], [F], [W.Solve(0, 1, p)],
                         W.Window(-6.0, 6.0, 0.01))
        sv = SWFSolve(prob, 0)
        P[n] = ob.marginal(sv, sv.run())
    e = {n: abs(P[n] - P[96]) for n in (32, 40, 48, 64)}
    assert e[32] > 20 * e[40] > 400 * e[48]
    assert e[64] < 1e-12 * P[96]


def test_time_only_mode_matches_dop853():
    # A_1(t) = a sech^2(t/tau) -> 0 at both ends: one lattice mode, 4x4 ODE
    a, tau, px, pp = 0.9, 1.5, 0.4, 0.3
    L = 2 * np.pi / px
    F = [W.Term(1, a, W.sech2(tau))]
    prob = W.Problem("t", [W.Grid(1, [4, 1, 1], [L, 1, 1])], [F], [W.Solve(0, 1, [px, pp, 0.0])],
                     W.Window(-20.0, 20.0, 0.005))
    sv = SWFSolve(prob, 0)
    y = sv.run()
    P = ob.marginal(sv, y) / L

    def f(t, c):
        c = c.view(complex)
        K = np.array([px + a / np.cosh(t / tau) ** 2, pp, 0.0])   # k^j + A_j
        return (-1j * dirac.hamiltonian0(K) @ c).view(float)

    E = dirac.energy([px, pp, 0.0])
    u = dirac.u_spinor(1, [px, pp, 0.0])
    c0 = (u * np.exp(-1j * E * 20.0)).astype(complex).view(float)
    sol = solve_ivp(f, (20.0, -20.0), c0, method="DOP853", rtol=1e-12, atol=1e-14)
    c = sol.y[:, -1].view(complex)
    n_ref = float(np.real(c.conj() @ dirac.projector([px, pp, 0.0], -1) @ c))
    assert P == pytest.approx(n_ref, rel=1e-7)


def test_marginal_resolves_tiny_negative_energy_content():
    # psi~(k) = a(k) u(k) + b(k) v(k) with |b|^2 / |a|^2 ~ 1e-12: the electron
    # marginal must return dV/N sum |b|^2 (orthonormal eigenvectors) to high
    # relative accuracy although (psi|psi) is 1e12 times larger.
    n, L = 32, 40.0
    prob = W.Problem("t", [W.Grid(1, [n, 1, 1], [L, 1, 1])], [[]], [W.Solve(0, 1, [0.0, 0.3, 0.0])],
                     W.Window(-1.0, 1.0, 0.1))
    sv = SWFSolve(prob, 0)
    rng = np.random.default_rng(9)
    a = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    b = 1e-6 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    psik = np.zeros((4, n), dtype=complex)
    for i in range(n):
        K = [sv.kfull[0][i], sv.kfull[1][i], sv.kfull[2][i]]
        w, V = np.linalg.eigh(dirac.hamiltonian0(K))      # ascending: two negative, two positive
        psik[:, i] = a[i] * V[:, 3] + b[i] * V[:, 0]
    psi = np.fft.ifft(psik, axis=1)
    want = sv.lat.dV / n * np.sum(np.abs(b) ** 2)
    total = sv.lat.dV / n * np.sum(np.abs(a) ** 2 + np.abs(b) ** 2)
    assert total / want > 1e11
    assert ob.marginal(sv, psi) == pytest.approx(want, rel=1e-6)


def _reflected(pr):
    """The profile of s -> f(-s) for an even envelope (gauss, sech2, const)."""
    assert pr.type in (W.PROF_CONST, W.PROF_GAUSS, W.PROF_SECH2)
    return W.Profile(pr.type, -pr.c, pr.w, pr.k, -pr.phi)


def _rotated_field(terms):
    """R A for the 90-degree rotation R (x, y) -> (-y, x) about z: A_0 and A_3
    are scalars under R, (A_1, A_2) -> (-A_2, A_1), all at the point R^-1 x =
    (y, -x)."""
    out = []
    for tm in terms:
        fx = [_reflected(tm.fx[1]), tm.fx[0], tm.fx[2]]          # f(R^-1 x) = f_x(y) f_y(-x) f_z(z)
        mu, amp = {0: (0, tm.amp), 1: (2, tm.amp), 2: (1, -tm.amp), 3: (3, tm.amp)}[tm.mu]
        out.append(W.Term(mu, amp, tm.ft, fx))
    return out


def test_rotation_by_90_degrees_maps_the_spectrum():
    # square periodic lattice: the rotation maps lattice points to lattice
    # points, so the spin-summed marginal obeys P(p; A) = P(R p; R A).  What
    # can break it on the lattice: the Nyquist mode (wavenumber -pi/dx, not
    # +pi/dx) and the box edge (-L/2 is a lattice point, +L/2 is not), so the
    # grid is fine enough and every profile negligible at the edge.  Every
    # coupling is on (A_0, A_1, A_2, A_3), with off-centre profiles and
    # carriers, so a swapped axis or a wrong sign in alpha^j breaks it.
    n, L = 64, 24.0
    F = [W.Term(1, 0.9, W.sech2(1.2), [W.gauss(2.5, c=0.7), W.sech2(1.2, c=-0.4), W.const()]),
         W.Term(2, 0.6, W.gauss(1.0, c=0.2), [W.sech2(1.5, c=0.3, k=0.5, phi=0.2), W.gauss(2.0), W.const()]),
         W.Term(0, 0.4, W.gauss(1.3, k=0.7), [W.gauss(2.2, c=-0.6), W.gauss(2.4, c=0.5), W.const()]),
         W.Term(3, 0.3, W.sech2(0.9), [W.gauss(2.5), W.sech2(1.0, c=0.9), W.const()])]
    p = [0.45, -0.3, 0.2]
    Rp = [-p[1], p[0], p[2]]
    g = W.Grid(2, [n, n, 1], [L, L, 1])
    win = W.Window(-2.5, 2.5, 0.05)
    P = []
    for field, mom in ((F, p), (_rotated_field(F), Rp)):
        prob = W.Problem("rot", [g], [field], [W.Solve(0, 1, mom), W.Solve(0, -1, mom)], win)
        P.append(sum(ob.marginal(SWFSolve(prob, i), SWFSolve(prob, i).run()) for i in range(2)))
    assert P[0] > 1e-6
    assert P[1] == pytest.approx(P[0], rel=1e-8)
    # and a rotation that is not a symmetry of the field changes it
    prob = W.Problem("rot", [g], [F], [W.Solve(0, 1, Rp), W.Solve(0, -1, Rp)], win)
    Pwrong = sum(ob.marginal(SWFSolve(prob, i), SWFSolve(prob, i).run()) for i in range(2))
    assert abs(Pwrong - P[0]) > 1e-3 * P[0]


def test_charge_balance_over_all_lattice_modes():
    # every created electron has a positron partner: summed over all lattice
    # momenta and spins, sum P_e(s, p) = sum P_pos(r, q) with q_perp = -p_perp
    # (exact for unitary evolution; RK4 is unitary to O(dt^4)).  An odd
    # number of points has no Nyquist mode, whose wavenumber the lattice
    # derivative takes as -pi/dx for both signs of the background momentum.
    n, L, pperp = 15, 15.0, 0.3
    solves = []
    for kx in range(-(n // 2), n // 2 + 1):
        px = 2 * np.pi * kx / L
        for s in (1, -1):
            solves.append(W.Solve(0, s, [px, pperp, 0.0]))
            solves.append(W.Solve(1, s, [px, -pperp, 0.0]))
    F = [W.Term(1, 1.3, W.sech2(1.0), [W.sech2(2.0), W.const(), W.const()]),
         W.Term(0, 0.5, W.gauss(0.8), [W.gauss(1.5, c=0.4), W.const(), W.const()])]
    prob = W.Problem("cb", [W.Grid(1, [n, 1, 1], [L, 1, 1])], [F], solves, W.Window(-6.0, 6.0, 0.01))
    Pe = Pp = 0.0
    for i, sv in enumerate(prob.solves):
        svv = SWFSolve(prob, i)
        P = ob.marginal(svv, svv.run())
        if sv.kind == 0:
            Pe += P
        else:
            Pp += P
    assert Pe > 1e-4
    assert Pp == pytest.approx(Pe, rel=1e-6)


def _free_packet_run(n, L, cells, strength, checkpoints, k0=2.0, sigma=4.0, dt=0.05):
    """A positive-energy Gaussian packet u(k0) e^{i k0 x - x^2/sigma^2}
    evolved freely (A = 0, so psi_s obeys the free Dirac equation) on a 1D
    box, with the boundary mask on or off; returns (x, psi) at the given step
    counts."""
    t_half = 0.5 * dt * checkpoints[-1]
    g = W.Grid(1, [n, 1, 1], [L, 1.0, 1.0], cells, strength)
    prob = W.Problem("absorb", [g], [[]], [W.Solve(0, 1, [0.4, 0.0, 0.0])], W.Window(-t_half, t_half, dt))
    sv = SWFSolve(prob, 0)
    x = sv.lat.X[0]
    y = dirac.u_spinor(1, np.array([k0, 0.0, 0.0]))[:, None] * \
        np.exp(1j * k0 * x - x ** 2 / sigma ** 2)[None]
    out, done = [], 0
    for c in checkpoints:
        y = sv.run(y, start=done, count=c - done)
        done = c
        out.append(y.copy())
    return x, out


def test_absorbing_mask_matches_a_larger_periodic_box():
    """The boundary mask (not part of the paper) is meant to make a periodic box
    act like an unbounded one for waves leaving it.  Pin: a packet moving at
    v = 0.89 on a box of length L = 80 with the mask (24 cells, strength 0.05)
    gives, inside the unmasked interior, the same wave as on a box of 2L without
    mask, both while it is still inside (the mask must not touch it) and after
    it has left (it must be absorbed, not reflected): 1e-4 of the packet's
    height.  Without the mask it wraps round the box L and comes back into the
    interior at O(1)."""
    n, L, cells = 128, 80.0, 24
    steps = [200, 2000]           # t = 10: packet inside; t = 100: it crossed an edge (and, on L, would wrap)
    x1, masked = _free_packet_run(n, L, cells, 0.05, steps)
    x2, big = _free_packet_run(2 * n, 2 * L, 0, 0.0, steps)
    _, bare = _free_packet_run(n, L, 0, 0.0, steps)
    inner = L / 2 - cells * L / n
    s1, s2 = np.abs(x1) < inner, np.abs(x2) < inner
    assert np.allclose(x1[s1], x2[s2])
    for k in range(2):
        err = np.abs(masked[k][:, s1] - big[k][:, s2]).max()
        assert err < 1e-4, (k, err)
    # at the end the packet has left the interior of the large box ...
    assert np.abs(big[1][:, s2]).max() < 1e-5
    # ... while without the mask it has wrapped back into that of the small one
    assert np.abs(bare[1][:, s1] - big[1][:, s2]).max() > 0.1
