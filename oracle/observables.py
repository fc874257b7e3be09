"""Inner products at t_in: pair amplitude, marginals and diagnostics.

The pair number of eq. (Nmn) is built from inner products
(psi|phi) = int d^3x psi^dagger phi taken at t_in, and a sum over a complete
set of free states i.  Reading of the garbled display (the two |...|^2
blocks are printed side by side): they are two equivalent expressions of the
same amplitude, here

    form 1:  Omega = (U_back|V_scat) + (U_scat|Pi_+|V_scat)
    form 2:  Omega = (U_scat|V_back) + (U_scat|Pi_-|V_scat)

where the sum over free positive- (negative-) energy states i becomes the
projector Pi_+ (Pi_-) in Fourier space.  Orthogonality of U_out and V_out
makes form 1 = -form 2, so both give the same N = |Omega|^2.

Electron marginal (sum over all positron states): P_e(s,p) =
(U_scat|Pi_-|U_scat); positron marginal: P_pos(r,q) = (V_scat|Pi_+|V_scat).

In-states (stepped forward from t_in) are read the same way at t_out, where
the field is off again: the marginal of U_in is its negative-energy content
there, and the two forms become (U_in|Pi_+|V_in) = -(U_in|Pi_-|V_in), the
time-reversed counterpart of Omega (equal to -Omega at first order in the
field; not the same amplitude beyond it).  The overlap of an in- and an
out-state is time independent, which ties the two directions together:
(U_back|V_scat^in)(t_out) = (U_scat^out|V_back)(t_in) = (U_out|V_in) and
(U_scat^in|V_back)(t_out) = (U_back|V_scat^out)(t_in) = (U_in|V_out).
Normalisation: dN = P d^d p / (2 pi)^d with d the number of non-trivial axes,
per unit transverse volume.  On the lattice (psi|phi) = dV sum_x psi^dagger
phi = dV/N sum_k psi~^dagger phi~ with psi~ = FFT(psi).
"""
from __future__ import annotations

import numpy as np

from . import dirac
from .swf import apply


def inner(a, b, dV):
    return dV * np.sum(np.conj(a) * b)


def projector_field(sv, sign: int):
    """Per-k energy projector 1/2 (1 + sign H0(k)/E_k) on the solve's lattice."""
    lat = sv.lat
    return 0.5 * (dirac.I4.reshape((4, 4) + (1,) * lat.dim) + sign * sv.H0 / sv.Ek[None, None])


def projected_overlap(sa, psi_a, psi_b, sign: int):
    """dV/N sum_k FFT(psi_a)^dagger Pi_sign(k) FFT(psi_b), Pi on sa's lattice.

    Pi is an orthogonal projector (Hermitian, Pi^2 = Pi), so the quadratic form
    equals (Pi a)^dagger (Pi b); that form is used because the probabilities of
    interest are exponentially small next to (psi|psi): the expanded form
    1/2 (|a|^2 - a^dag H0 a / E) would cancel to a relative error of order
    eps (psi|psi)/P, the projected form keeps it at eps sqrt((psi|psi)/P)."""
    lat = sa.lat
    P = projector_field(sa, sign)
    pa = apply(P, lat.fft(psi_a))
    pb = pa if psi_b is psi_a else apply(P, lat.fft(psi_b))
    return lat.dV / lat.N * np.sum(np.conj(pa) * pb)


def marginal(sv, psi_s):
    """Electron marginal for a U solve, positron marginal for a V solve."""
    sign = -1 if sv.solve.kind % 2 == 0 else +1
    return float(np.real(projected_overlap(sv, psi_s, psi_s, sign)))


def _check_pair(su, sv):
    if su.solve.kind % 2 != 0 or sv.solve.kind % 2 != 1 or su.forward != sv.forward:
        raise ValueError("pair amplitude needs a U solve and a V solve, both out- or both in-states")
    if su.lat.shape != sv.lat.shape or su.lat.L != sv.lat.L:
        raise ValueError("U and V must share a lattice")
    for j in range(su.lat.dim, 3):
        # trivial axes: transverse momentum conservation q_perp = -p_perp
        if abs(su.K[j] - sv.K[j]) > 1e-12:
            raise ValueError("pair amplitude needs q_perp = -p_perp on trivial axes")


def pair_amplitude(su, psi_u, sv, psi_v, t: float, form: int = 1):
    """Omega(m, n) of eq. (Nmn) (form 1 or form 2) from out-states at t = t_in,
    per (2 pi)^(3-d) delta(p_perp + q_perp); for in-states at t = t_out the
    same forms give their time-reversed counterpart."""
    _check_pair(su, sv)
    dV = su.lat.dV
    if form == 1:
        return inner(su.psi_back(t), psi_v, dV) + projected_overlap(su, psi_u, psi_v, +1)
    return inner(psi_u, sv.psi_back(t), dV) + projected_overlap(su, psi_u, psi_v, -1)


def pair_number(su, psi_u, sv, psi_v, t_in: float) -> float:
    return float(abs(pair_amplitude(su, psi_u, sv, psi_v, t_in, 1)) ** 2)


def diagnostics(sv, psi_s, t: float):
    """((psi_s|psi_s), 2 Re(psi_b|psi_s)).  For the homogeneous evolution of
    the full psi = psi_b + psi_s their sum stays 0 (norm conservation)."""
    dV = sv.lat.dV
    ss = float(np.real(inner(psi_s, psi_s, dV)))
    bs = float(2.0 * np.real(inner(sv.psi_back(t), psi_s, dV)))
    return ss, bs


def marginal_in_uniform_field(sv, psi_full, A_cov):
    """Negative-energy (U) / positive-energy (V) content of a full wave
    function at a time where a spatially uniform potential A_cov = (A_0, A_1,
    A_2, A_3) is still on: project with H(k) = alpha^j (k^j + A_j) + beta.
    Used for fields such as the Sauter pulse whose A does not vanish at t_in."""
    lat = sv.lat
    sign = -1 if sv.solve.kind % 2 == 0 else +1
    kin = [sv.kfull[j] + A_cov[j + 1] for j in range(3)]
    H = sum(dirac.ALPHA[j][:, :, None] * kin[j].reshape(1, 1, -1) for j in range(3)).reshape(
        (4, 4) + lat.shape) + dirac.BETA.reshape((4, 4) + (1,) * lat.dim)
    E = np.sqrt(1.0 + sum(k ** 2 for k in kin))
    P = 0.5 * (dirac.I4.reshape((4, 4) + (1,) * lat.dim) + sign * H / E[None, None])
    pk = apply(P, lat.fft(psi_full))
    return float(np.real(lat.dV / lat.N * np.sum(np.conj(pk) * pk)))
