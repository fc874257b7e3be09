"""Pins for the oracle's algebra, lattice and field pieces (CPU only).

Every check compares the oracle with something it does not compute itself:
the Clifford algebra, the defining relations of R_s (eq. (Reqs)), the free
Dirac equation for u_s, v_s (eq. (uv)), the polarisation basis printed in
eq. (epsParaPerp), closed-form field values of eq. (singleE)/(doubleE).
"""
import json
import os

import numpy as np
import pytest

import swf_workloads as W
from oracle import dirac
from oracle.field import potential, profile
from oracle.lattice import Lattice

GOLD = os.path.join(os.path.dirname(__file__), "golden")
pytestmark = pytest.mark.filterwarnings("ignore")


def test_clifford_algebra():
    for m in range(4):
        for n in range(4):
            ac = dirac.GAMMA[m] @ dirac.GAMMA[n] + dirac.GAMMA[n] @ dirac.GAMMA[m]
            assert np.allclose(ac, 2 * dirac.ETA[m, n] * np.eye(4))
    for j in range(3):
        assert np.allclose(dirac.ALPHA[j], dirac.ALPHA[j].conj().T)
        assert np.allclose(dirac.ALPHA[j] @ dirac.BETA + dirac.BETA @ dirac.ALPHA[j], 0)


@pytest.mark.parametrize("s", [1, -1])
def test_R_relations(s):
    R = dirac.R_spinor(s)
    g = dirac.GAMMA
    assert np.allclose(g[0] @ g[1] @ R, R)
    assert np.allclose(1j * g[2] @ g[3] @ R, s * R)
    assert np.allclose(R.conj() @ dirac.R_spinor(s), 1)
    assert abs(R.conj() @ dirac.R_spinor(-s)) < 1e-15


def test_spinors_free_dirac_equation():
    rng = np.random.default_rng(3)
    for _ in range(20):
        p = rng.normal(size=3) * 1.5
        E = dirac.energy(p)
        pv = np.concatenate([[E], p])
        for s in (1, -1):
            u = dirac.u_spinor(s, p)
            v = dirac.v_spinor(s, p)
            # (pslash - 1) u = 0, (pslash + 1) v = 0
            assert np.abs((dirac.slash(pv) - np.eye(4)) @ u).max() < 1e-13
            assert np.abs((dirac.slash(pv) + np.eye(4)) @ v).max() < 1e-13
            # unit density (the covariant-p_1 reading of eq. (uv))
            assert abs(u.conj() @ u - 1) < 1e-13 and abs(v.conj() @ v - 1) < 1e-13
            # ubar u = 1/p0, vbar v = -1/p0
            assert abs(u.conj() @ dirac.GAMMA0 @ u - 1 / E) < 1e-13
            assert abs(v.conj() @ dirac.GAMMA0 @ v + 1 / E) < 1e-13
        for r in (1, -1):
            for s in (1, -1):
                assert abs(dirac.u_spinor(r, p).conj() @ dirac.u_spinor(s, p) - (r == s)) < 1e-13
                # u(p) and v(-p) are eigenvectors of H0(p) with opposite energies
                assert abs(dirac.u_spinor(r, p).conj() @ dirac.v_spinor(s, -p)) < 1e-13


def test_covariant_p1_reading_is_the_normalised_one():
    # with the contravariant component in the normalisation u^dag u != 1
    p = np.array([0.7, -0.3, 0.4])
    E = dirac.energy(p)
    u_alt = (np.eye(4) + dirac.slash(np.concatenate([[E], p]))) @ dirac.R_spinor(1) / np.sqrt(
        2 * E * (E + p[0]))
    assert abs(u_alt.conj() @ u_alt - 1) > 0.1


def test_projectors():
    rng = np.random.default_rng(4)
    for _ in range(10):
        K = rng.normal(size=3)
        Pp, Pm = dirac.projector(K, 1), dirac.projector(K, -1)
        assert np.allclose(Pp @ Pp, Pp) and np.allclose(Pm @ Pm, Pm)
        assert np.allclose(Pp + Pm, np.eye(4)) and np.allclose(Pp @ Pm, 0)
        H = dirac.hamiltonian0(K)
        assert np.allclose(H @ H, dirac.energy(K) ** 2 * np.eye(4))
        for s in (1, -1):
            assert np.allclose(Pp @ dirac.u_spinor(s, K), dirac.u_spinor(s, K))
            assert np.allclose(Pm @ dirac.v_spinor(s, -K), dirac.v_spinor(s, -K))


def test_polarization_basis_golden():
    with open(os.path.join(GOLD, "polarization_basis.json")) as f:
        g = json.load(f)
    for c in g["cases"]:
        par, perp = dirac.polarization_basis(c["e"], c["k"])
        assert np.allclose(par, c["eps_par"]) and np.allclose(perp, c["eps_perp"])
        khat = np.asarray(c["k"]) / np.linalg.norm(c["k"])
        assert np.isclose(np.dot(np.cross(par, perp), khat), 1.0)


def test_profiles_closed_form():
    s = np.linspace(-3, 3, 13)
    assert np.allclose(profile(W.gauss(2.0, c=0.5), s), np.exp(-((s - 0.5) / 2) ** 2))
    assert np.allclose(profile(W.sech2(1.5), s), 1 / np.cosh(s / 1.5) ** 2)
    assert np.allclose(profile(W.tanh(0.7), s), np.tanh(s / 0.7))
    assert np.allclose(profile(W.ugauss(2.0), s), (s / 2) * np.exp(-(s / 2) ** 2))
    assert np.allclose(profile(W.gauss(1.0, k=0.3, phi=0.2), s), np.exp(-s ** 2) * np.cos(0.3 * s + 0.2))
    assert np.allclose(profile(W.const(), s), 1.0)


def test_single_and_double_e_fields():
    # eq. (singleE) and (doubleE) written out directly
    E0, om, kx, ky, dxs = 0.25, 0.25, 0.125, 0.125, 1.75 / 0.125
    g = W.Grid(2, [16, 12, 1], [80.0, 60.0, 1.0])
    lat = Lattice(g)
    t = 0.7

    def one(x, y):
        return -(E0 / kx) * np.sin(kx * x) * np.exp(-(om * t) ** 2 - (kx * x) ** 2 - (ky * y) ** 2)

    A = potential(W.field_single_e(E0, om, kx, ky, dim=2), t, lat)
    assert np.allclose(A[0], one(lat.X[0], lat.X[1]), atol=1e-14)
    assert np.allclose(A[1], 0) and np.allclose(A[2], 0) and np.allclose(A[3], 0)
    A2 = potential(W.field_double_e(E0, om, kx, ky, dxs), t, lat)
    ref = one(lat.X[0] + dxs, lat.X[1]) + one(lat.X[0] - dxs, lat.X[1])
    assert np.allclose(A2[0], ref, atol=1e-14)


def test_field_rejects_trivial_axis_dependence():
    lat = Lattice(W.Grid(1, [8, 1, 1], [10.0, 1, 1]))
    with pytest.raises(ValueError):
        potential([W.Term(1, 1.0, W.const(), [W.const(), W.gauss(1.0), W.const()])], 0.0, lat)


def test_lattice_spectral_derivative():
    g = W.Grid(2, [24, 16, 1], [12.0, 8.0, 1.0])
    lat = Lattice(g)
    f = np.sin(2 * np.pi * 3 * lat.X[0] / 12.0) * np.cos(2 * np.pi * 2 * lat.X[1] / 8.0)
    dfx = np.real(np.fft.ifftn(1j * lat.K[0] * np.fft.fftn(f)))
    ref = (2 * np.pi * 3 / 12.0) * np.cos(2 * np.pi * 3 * lat.X[0] / 12.0) * np.cos(
        2 * np.pi * 2 * lat.X[1] / 8.0)
    assert np.abs(dfx - ref).max() < 1e-12
    assert lat.k1d[0][12] == pytest.approx(-np.pi / lat.dx[0])   # Nyquist kept negative
    assert lat.dV == pytest.approx(0.5 * 0.5)


def test_absorber_mask_shape():
    lat = Lattice(W.Grid(1, [32, 1, 1], [32.0, 1, 1]))
    m = lat.absorber(4, 0.5)
    assert m[0] == pytest.approx(0.5) and m[-1] == pytest.approx(0.5)
    assert np.all(m[4:-4] == 1.0) and np.all(np.diff(m[:5]) > 0)
