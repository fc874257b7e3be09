"""Dirac algebra in the Dirac representation, metric (+,-,-,-).

Follows the paper's conventions: D_mu = d_mu + i A_mu with the charge absorbed
into A (eq. (DiracEq)); alpha^k = gamma^0 gamma^k and beta = gamma^0 (below
eq. (LambdaDef)); the free spinors of eq. (uv) built from the R_s of
eq. (Reqs).  Reading taken here: the p_1 in the normalisation of eq. (uv) is
the covariant component, p_1 = -p^1 (the only reading with u^dagger u = 1).
"""
from __future__ import annotations

import numpy as np

SIGMA = [
    np.array([[0, 1], [1, 0]], dtype=complex),
    np.array([[0, -1j], [1j, 0]], dtype=complex),
    np.array([[1, 0], [0, -1]], dtype=complex),
]
I2 = np.eye(2, dtype=complex)
Z2 = np.zeros((2, 2), dtype=complex)
I4 = np.eye(4, dtype=complex)

GAMMA0 = np.block([[I2, Z2], [Z2, -I2]])
GAMMA = [GAMMA0] + [np.block([[Z2, s], [-s, Z2]]) for s in SIGMA]
ETA = np.diag([1.0, -1.0, -1.0, -1.0])
BETA = GAMMA0
ALPHA = [GAMMA0 @ GAMMA[j] for j in (1, 2, 3)]


def slash(p_contra) -> np.ndarray:
    """gamma^mu p_mu for a contravariant 4-vector p^mu."""
    p_cov = ETA @ np.asarray(p_contra, dtype=float)
    return sum(GAMMA[m] * p_cov[m] for m in range(4))


def energy(p3) -> float:
    p3 = np.asarray(p3, dtype=float)
    return float(np.sqrt(1.0 + p3 @ p3))


def R_spinor(s: int) -> np.ndarray:
    """The R_s of eq. (Reqs): gamma^0 gamma^1 R = R, i gamma^2 gamma^3 R = s R,
    unit norm; the real representative 1/2 (1, s, s, 1)."""
    return 0.5 * np.array([1.0, s, s, 1.0], dtype=complex)


def u_spinor(s: int, p3) -> np.ndarray:
    """u_s(p) = (1 + pslash) R_s / sqrt(2 p^0 (p_0 + p_1)), p_1 = -p^1 (eq. (uv))."""
    p3 = np.asarray(p3, dtype=float)
    p0 = energy(p3)
    pv = np.concatenate([[p0], p3])
    return (I4 + slash(pv)) @ R_spinor(s) / np.sqrt(2.0 * p0 * (p0 - p3[0]))


def v_spinor(s: int, p3) -> np.ndarray:
    """v_s(p) = (1 - pslash) R_s / sqrt(2 p^0 (p_0 + p_1)), p_1 = -p^1 (eq. (uv))."""
    p3 = np.asarray(p3, dtype=float)
    p0 = energy(p3)
    pv = np.concatenate([[p0], p3])
    return (I4 - slash(pv)) @ R_spinor(s) / np.sqrt(2.0 * p0 * (p0 - p3[0]))


def hamiltonian0(K) -> np.ndarray:
    """Free Dirac Hamiltonian alpha.K + beta for a plane wave exp(+i K.x)."""
    K = np.asarray(K, dtype=float)
    return sum(ALPHA[j] * K[j] for j in range(3)) + BETA


def projector(K, sign: int) -> np.ndarray:
    """Energy projector 1/2 (1 + sign H0(K)/E_K).  sign=+1 keeps the
    positive-energy part (time dependence exp(-i E t)), sign=-1 the negative
    one.  The paper's Lambda_(+-) of eq. (LambdaDef) are labelled by the sign
    of the exponent exp(+-i Q_0 t), so its Lambda_+ is projector(., -1)."""
    return 0.5 * (I4 + sign * hamiltonian0(K) / energy(K))


def polarization_basis(e, k):
    """Photon polarisation vectors of eq. (epsParaPerp):
    eps_perp = e x k / |e x k|, eps_par = eps_perp x k / |eps_perp x k|."""
    e = np.asarray(e, dtype=float)
    k = np.asarray(k, dtype=float)
    perp = np.cross(e, k)
    perp /= np.linalg.norm(perp)
    par = np.cross(perp, k)
    par /= np.linalg.norm(par)
    return par, perp


def background_spinor(kind: int, spin: int, p3):
    """(spinor, E, K) of the background wave w exp(-i E t + i K.x):
    U: u_s(p) exp(-i p.x) -> (u, +p^0, +p);  V: v_s(p) exp(+i p.x) -> (v, -p^0, -p).
    In- and out-states share their backgrounds (kinds 0, 2: U; 1, 3: V)."""
    p3 = np.asarray(p3, dtype=float)
    if kind % 2 == 0:
        return u_spinor(spin, p3), energy(p3), p3.copy()
    return v_spinor(spin, p3), -energy(p3), -p3
