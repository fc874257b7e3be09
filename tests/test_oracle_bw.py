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
