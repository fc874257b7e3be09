"""Pins of the oracle's finite-difference derivative variant (SWFSolve(...,
fd_order=2p)), the scope table's stencil derivative judged against the
spectral one (CPU only).

* the stencil's Fourier symbol is what the stencil does: applied in Fourier
  space it equals the periodic stencil applied with np.roll;
* the weights give order 2p: the symbol's relative error falls as (k dx)^2p;
* the background built from the symbol solves the stencil's free Dirac
  equation: (alpha.K(p) + beta) u(K(p)) = E(K(p)) u(K(p));
* the stencil solution converges to the spectral one as dx shrinks, at the
  stencil's order.
"""
import numpy as np
import pytest

import swf_workloads as W
from oracle import dirac, observables as ob
from oracle.lattice import fd_coefficients, fd_symbol
from oracle.swf import SWFSolve


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_symbol_is_the_periodic_stencil(order):
    n, L = 48, 12.0
    dx = L / n
    rng = np.random.default_rng(order)
    f = rng.normal(size=n) + 1j * rng.normal(size=n)
    direct = sum(a * (np.roll(f, -m) - np.roll(f, m)) for m, a in enumerate(fd_coefficients(order), start=1)) / dx
    k = 2 * np.pi * np.fft.fftfreq(n, dx)
    spectral = np.fft.ifft(1j * fd_symbol(k, dx, order) * np.fft.fft(f))
    assert np.allclose(spectral, direct, rtol=0, atol=1e-12)


@pytest.mark.parametrize("order", [2, 4, 6, 8])
def test_symbol_order(order):
    dx = 0.1
    err = [abs(fd_symbol(k, dx, order) - k) / k for k in (0.8, 0.4)]
    assert err[0] / err[1] == pytest.approx(2.0 ** order, rel=0.05)


def test_background_solves_the_stencil_dirac_equation():
    p = np.array([0.7, -0.3, 0.2])
    for order in (2, 8):
        K = np.array([fd_symbol(p[0], 0.25, order), fd_symbol(p[1], 0.25, order), p[2]])
        for kind, spin in ((0, 1), (1, -1)):
            w, E, _ = dirac.background_spinor(kind, spin, K)
            H = dirac.hamiltonian0(K if kind % 2 == 0 else -K)
            assert np.allclose(H @ w, E * w, atol=1e-13)


def _prob(n):
    # (1+1)D Schwinger on the workload's box (L = 200: the field vanishes at the
    # edge), a short window around the pulse
    return W.config_1d(n=n, L=200.0, dt=0.02, t_half=6.0, p=(0.4, 0.1, 0.0))


def test_stencil_converges_to_the_spectral_solution_at_its_order():
    ref_sv = SWFSolve(_prob(1024), 0)
    ref = ob.marginal(ref_sv, ref_sv.run())
    sv = SWFSolve(_prob(256), 0)
    assert abs(ob.marginal(sv, sv.run()) - ref) < 1e-13 * ref      # spectral: converged at 256 points
    for order, lo, hi in ((2, 3.2, 5.0), (4, 12.0, 20.0), (8, 150.0, 400.0)):
        err = []
        for n in (256, 512):
            s = SWFSolve(_prob(n), 0, fd_order=order)
            err.append(abs(ob.marginal(s, s.run()) - ref) / ref)
        assert lo < err[0] / err[1] < hi, (order, err)
