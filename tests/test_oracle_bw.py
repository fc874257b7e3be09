"""Pins of the oracle's nonlinear Breit-Wheeler amplitude (CPU only).

* Exact spin structure for E(t,x) fields, eq. (MparaE):
  M(r,s) = [delta_rs - delta_{r,-s} i p2] M, for the Fig. 7 kinematics
  (golden fixture tests/golden/bw_exact_spin_fig7.json).
* M_past + M_finite is independent of t_in (stated below eq. (MScatScatPast)):
  moving t_in further into the field-free past moves weight from the past
  term (analytic) to the finite term (stepped), and the difference shrinks
  at RK4's order 4 in dt.
* The section's second route (partial integration in t, only the source
  term in the integrand, no past term) gives the same three terms as finite
  + past, converging at order 4.
"""
import json
import os

import numpy as np
import pytest

import swf_workloads as W
from oracle import bw

GOLD = os.path.join(os.path.dirname(__file__), "golden")
pytestmark = pytest.mark.filterwarnings("ignore")


def test_exact_spin_structure_fig7():
    with open(os.path.join(GOLD, "bw_exact_spin_fig7.json")) as f:
        g = json.load(f)
    P = 2 * np.pi * 4 / 160.0
    spins = ((1, 1), (1, -1), (-1, 1), (-1, -1))
    prob = W.config_bw_1d(P=P, n=128, L=160.0, dt=0.1, t_half=25.0, spins=spins)
    assert prob.vertices[0].k == g["photon_k"]
    M = {sr: bw.Vertex(prob, i).amplitude()["total"] for i, sr in enumerate(spins)}
    assert abs(M[(1, 1)]) > 1e-4
    exp = g["expected"]
    assert M[(1, -1)] / M[(1, 1)] == pytest.approx(complex(*exp["M(+,-)/M(+,+)"]), abs=1e-8)
    assert M[(-1, 1)] / M[(1, 1)] == pytest.approx(complex(*exp["M(-,+)/M(+,+)"]), abs=1e-8)
    assert M[(-1, -1)] / M[(1, 1)] == pytest.approx(complex(*exp["M(-,-)/M(+,+)"]), abs=1e-8)


def test_t_in_independence_converges():
    P = 2 * np.pi * 4 / 160.0
    diffs = []
    for dt in (0.05, 0.025):
        tot = []
        for th in (30.0, 40.0):
            prob = W.config_bw_1d(P=P, n=256, L=160.0, dt=dt, t_half=th)
            tot.append(bw.Vertex(prob, 0).amplitude()["total"])
        diffs.append(abs(tot[0] - tot[1]) / abs(tot[0]))
    assert diffs[1] < 2e-4
    assert 10.0 < diffs[0] / diffs[1] < 24.0


def test_partial_integration_route_matches():
    # the second route of the section (partial integration in t: only the
    # source term survives, no past term) against finite + past, per term;
    # Fig. 7 kinematics with lattice momenta, where both are exact on the
    # lattice.  The terms are ~2000x the total (they cancel), so each is
    # compared against its own size, and the difference shrinks at order 4.
    P = 2 * np.pi * 4 / 160.0
    diffs = []
    for dt in (0.1, 0.05):
        v = bw.Vertex(W.config_bw_1d(P=P, n=128, L=160.0, dt=dt, t_half=25.0), 0)
        r1, r2 = v.amplitude()["terms"], v.amplitude_partial()["terms"]
        assert np.all(np.abs(r1) > 1.0)
        diffs.append(np.abs(r1 - r2) / np.abs(r1))
    assert np.all(diffs[0] < 3e-6) and np.all(diffs[1] < 2e-7)
    ratio = diffs[0] / diffs[1]
    assert np.all((ratio > 12.0) & (ratio < 20.0)), ratio


# ---------------------------------------------------------------- wave packets
def _fig7_problem(modes, P=2 * np.pi * 4 / 160.0):
    prob = W.config_bw_1d(P=P, n=128, L=160.0, dt=0.1, t_half=25.0)
    vx = prob.vertices[0]
    prob.vertices = [W.Vertex(vx.u_solve, vx.v_solve, vx.k, vx.eps, modes)]
    return prob


def _plane(prob, k, eps):
    vx = prob.vertices[0]
    import dataclasses
    pw = dataclasses.replace(prob, vertices=[W.Vertex(vx.u_solve, vx.v_solve, list(k), list(eps))])
    return bw.Vertex(pw, 0).amplitude()


def test_packet_of_one_mode_is_the_plane_wave():
    k, eps = [0.0, 1.2, 0.0], [-1.0, 0.0, 0.0]
    prob = _fig7_problem([(k, eps, 1.0)])
    a = bw.PacketVertex(prob, 0).amplitude()
    b = _plane(prob, k, eps)
    for part in ("finite", "past"):
        assert np.abs(a[part] - b[part]).max() <= 1e-12 * np.abs(b[part]).max()


def test_packet_is_the_weighted_sum_of_its_plane_waves():
    # three components with off-lattice momenta along x (the non-trivial axis;
    # k_y = p_y + q_y is fixed by the trivial axis), two polarisations and
    # complex weights: the packet's finite part (one integrand with the field
    # E(t,x)) and past part equal the weighted sums of separate plane-wave runs
    modes = [([-0.11, 1.2, 0.0], [-1.0, 0.0, 0.0], 0.5 + 0.2j),
             ([0.0, 1.2, 0.0], [0.0, 0.0, 1.0], -0.3 + 0.4j),
             ([0.17, 1.2, 0.0], [-0.6, 0.0, 0.8], 0.25 - 0.1j)]
    prob = _fig7_problem(modes)
    a = bw.PacketVertex(prob, 0).amplitude()
    ref = {"finite": 0, "past": 0}
    for k, e, c in modes:
        b = _plane(prob, k, e)
        for part in ref:
            ref[part] = ref[part] + c * b[part]
    for part in ref:
        scale = np.abs(ref[part]).max()
        assert scale > 1e-3
        assert np.abs(a[part] - ref[part]).max() <= 1e-10 * scale, part
    # a wrong time phase of one component is seen
    bad = [(k, e, c) for k, e, c in modes]
    bad[2] = ([0.17, 1.2, 0.0], [-0.6, 0.0, 0.8], -(0.25 - 0.1j))
    a_bad = bw.PacketVertex(_fig7_problem(bad), 0).amplitude()
    assert np.abs(a_bad["finite"] - ref["finite"]).max() > 1e-3 * np.abs(ref["finite"]).max()


def test_packet_plane_wave_limit():
    # a packet Gaussian in k_x about the Fig. 7 photon, weights summing to 1:
    # as its momentum width sigma shrinks (the packet grows in x) its
    # amplitude tends to the plane wave's, the difference falling as sigma^2
    # (M(k) turns on a scale of ~0.01 in k_x here: the three terms are each
    # ~2000x the total they cancel to)
    k, eps = [0.0, 1.2, 0.0], [-1.0, 0.0, 0.0]
    prob = _fig7_problem([(k, eps, 1.0)])
    M0 = _plane(prob, k, eps)["total"]
    errs = []
    for sigma in (0.004, 0.002):
        modes = W.gaussian_packet(k, eps, 0, sigma, 9, sigma / 2)
        a = bw.PacketVertex(_fig7_problem(modes), 0).amplitude()["total"]
        errs.append(abs(a - M0) / abs(M0))
    assert errs[0] < 0.02
    assert 3.0 < errs[0] / errs[1] < 5.0, errs
