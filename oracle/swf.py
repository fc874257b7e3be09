"""The scattered-wave-function equation, stepped from t_out back to t_in
(out-states) or from t_in forward to t_out (in-states).

Paper, section "Scattered wave functions": psi = psi_back + psi_scat with the
plane-wave background psi_back = u e^{-ipx} (U) or v e^{ipx} (V), the same for
in- and out-states, and the scattered part solving the inhomogeneous equation
(i Dslash - 1) psi_scat = Aslash psi_back, eq. (scatDirac), with
psi_scat -> 0 as t -> +infinity for out-states and as t -> -infinity for
in-states; with the field negligible outside [t_in, t_out] these are
psi_scat(t_out) = 0 and psi_scat(t_in) = 0.  Multiplying by gamma^0 gives the
evolution form used here,

    d_t psi_s = -alpha^j d_j psi_s - i beta psi_s - i (A_0 + alpha^j A_j)(psi_s + psi_b),

whose kinetic part is evaluated spectrally (derivative through FFT, section
"Numerical approach"): -i H0(k) in Fourier space with H0(k) = alpha.k + beta,
where trivial axes contribute their conserved momentum (p_perp for U, -q_perp
for V).  Time integration: classical RK4 (reading of the paper's adaptive
Dopri5 for the fixed-dt workloads) with step h = -dt from t_out, t_n = t_out -
n dt, for out-states, and h = +dt from t_in, t_n = t_in + n dt, for in-states,
the times evaluated from the step index.
"""
from __future__ import annotations

import numpy as np

from . import dirac
from .field import potential
from .lattice import Lattice


def apply(M, psi):
    """Per-site 4x4 matrix times spinor: out[a] = sum_b M[a, b] psi[b]."""
    return np.einsum("ab...,b...->a...", M, psi)


class SWFSolve:
    """One solve (U_out, V_out, U_in or V_in of (s, p)) on its lattice."""

    def __init__(self, problem, index: int):
        sv = problem.solves[index]
        self.solve = sv
        self.forward = sv.kind >= 2     # in-states run forward from t_in
        self.grid = problem.grids[sv.grid]
        self.terms = problem.fields[sv.field]
        self.window = problem.window
        self.lat = Lattice(self.grid)
        self.w, self.E, self.K = dirac.background_spinor(sv.kind, sv.spin, sv.p)
        lat = self.lat
        self.kfull = lat.full_momentum(self.K)
        self.H0 = sum(dirac.ALPHA[j][:, :, None] * self.kfull[j].reshape(1, 1, -1)
                      for j in range(3)).reshape((4, 4) + lat.shape) + \
            dirac.BETA.reshape((4, 4) + (1,) * lat.dim)
        self.Ek = np.sqrt(1.0 + sum(kj ** 2 for kj in self.kfull))
        self.mask = lat.absorber(self.grid.absorb_cells, self.grid.absorb_strength) \
            if self.grid.absorb_cells > 0 else None
        self.phase_x = np.exp(1j * sum(self.K[j] * lat.X[j] for j in range(lat.dim))) \
            if lat.dim > 0 else np.ones(lat.shape)

    # -- background plane wave, eq. (scatDirac)'s source ------------------
    def psi_back(self, t: float):
        return self.w.reshape((4,) + (1,) * self.lat.dim) * \
            (np.exp(-1j * self.E * t) * self.phase_x)[None]

    # -- right-hand side --------------------------------------------------
    def potential_matrix(self, t: float):
        A = potential(self.terms, t, self.lat)
        V = A[0][None, None] * dirac.I4.reshape((4, 4) + (1,) * self.lat.dim)
        for j in range(3):
            V = V + A[j + 1][None, None] * dirac.ALPHA[j].reshape((4, 4) + (1,) * self.lat.dim)
        return V

    def kinetic(self, psi):
        return self.lat.ifft(-1j * apply(self.H0, self.lat.fft(psi)))

    def rhs(self, t: float, psi):
        return self.kinetic(psi) - 1j * apply(self.potential_matrix(t), psi + self.psi_back(t))

    # -- classical RK4, h = -dt (out) or +dt (in) -------------------------
    def time(self, n: int) -> float:
        if self.forward:
            return self.window.t_in + n * self.window.dt
        return self.window.t_out - n * self.window.dt

    @property
    def t_end(self) -> float:
        """Where a full run ends and the observables are read: t_in for
        out-states, t_out for in-states."""
        return self.window.t_out if self.forward else self.window.t_in

    def step_stages(self, n: int, y):
        """One RK4 step from t_n; returns y_{n+1} and the four stage inputs
        with their times (the augmented BW integral needs them)."""
        h = self.window.dt if self.forward else -self.window.dt
        t = self.time(n)
        y1 = y
        k1 = self.rhs(t, y1)
        y2 = y + 0.5 * h * k1
        k2 = self.rhs(t + 0.5 * h, y2)
        y3 = y + 0.5 * h * k2
        k3 = self.rhs(t + 0.5 * h, y3)
        y4 = y + h * k3
        k4 = self.rhs(t + h, y4)
        ynew = y + (h / 6.0) * (k1 + 2.0 * k2 + 2.0 * k3 + k4)
        if self.mask is not None:
            ynew = ynew * self.mask[None]
        return ynew, (y1, y2, y3, y4), (t, t + 0.5 * h, t + 0.5 * h, t + h)

    def step(self, n: int, y):
        return self.step_stages(n, y)[0]

    def zero_state(self):
        return np.zeros((4,) + self.lat.shape, dtype=complex)

    def run(self, y=None, start: int = 0, count: int | None = None):
        """Advance ``count`` steps from step index ``start`` (default: the
        whole window from psi_scat = 0 at its start)."""
        if y is None:
            y = self.zero_state()
        if count is None:
            count = self.window.steps - start
        for n in range(start, start + count):
            y = self.step(n, y)
        return y


def solve_all(problem):
    """Run every solve of the problem over the window; returns list of
    (SWFSolve, psi_s at the end of its run)."""
    out = []
    for i in range(len(problem.solves)):
        s = SWFSolve(problem, i)
        out.append((s, s.run()))
    return out
