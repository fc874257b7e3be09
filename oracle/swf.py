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
the times evaluated from the step index; or the paper's Dopri5 (the
Dormand-Prince 5(4) tableau) with the same fixed step (window.scheme "dp5");
or, as a variant stepper, the interaction picture (window.scheme "iprk4"):
Lawson's integrating-factor RK4 (J. D. Lawson, SIAM J. Numer. Anal. 4 (1967)
372), which takes the free evolution exp(-i H0(k) tau) exactly in Fourier
space and integrates only the field terms with the classical RK4 tableau.
"""
from __future__ import annotations

import numpy as np

from . import dirac
from .field import potential
from .lattice import Lattice


# Dormand-Prince 5(4) tableau (Dormand and Prince, J. Comput. Appl. Math. 6
# (1980) 19), the Dopri5 solver of the paper's listing in section "Numerical
# approach", here taken with a fixed step: c, the rows of A, the fifth-order
# weights b (b = the last row of A, so the last stage is the next step's
# first) and the embedded fourth-order weights bhat of its error estimate.
DP5_C = (0.0, 1 / 5, 3 / 10, 4 / 5, 8 / 9, 1.0, 1.0)
DP5_A = ((),
         (1 / 5,),
         (3 / 40, 9 / 40),
         (44 / 45, -56 / 15, 32 / 9),
         (19372 / 6561, -25360 / 2187, 64448 / 6561, -212 / 729),
         (9017 / 3168, -355 / 33, 46732 / 5247, 49 / 176, -5103 / 18656),
         (35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84))
DP5_B = (35 / 384, 0.0, 500 / 1113, 125 / 192, -2187 / 6784, 11 / 84, 0.0)
DP5_BHAT = (5179 / 57600, 0.0, 7571 / 16695, 393 / 640, -92097 / 339200, 187 / 2100, 1 / 40)


def apply(M, psi):
    """Per-site 4x4 matrix times spinor: out[a] = sum_b M[a, b] psi[b]."""
    return np.einsum("ab...,b...->a...", M, psi)


class SWFSolve:
    """One solve (U_out, V_out, U_in or V_in of (s, p)) on its lattice."""

    def __init__(self, problem, index: int, fd_order: int = 0):
        """fd_order > 0: the spatial derivative is the periodic central finite
        difference of that (even) order instead of the spectral one, a variant
        for judging a stencil against the paper's spectral derivative: the free
        Hamiltonian becomes H0(K(k)) with K the stencil's symbol, and the
        background is that Hamiltonian's plane-wave solution, the spinor and
        energy of momentum K(p) on the lattice axes (the phase keeps p)."""
        sv = problem.solves[index]
        self.solve = sv
        self.forward = sv.kind >= 2     # in-states run forward from t_in
        self.scheme = getattr(problem.window, "scheme", "rk4")
        if self.scheme not in ("rk4", "dp5", "iprk4"):
            raise ValueError(f"unknown time stepper {self.scheme!r}")
        self.grid = problem.grids[sv.grid]
        self.terms = problem.fields[sv.field]
        self.window = problem.window
        self.lat = Lattice(self.grid, fd_order)
        self.w, self.E, self.K = dirac.background_spinor(sv.kind, sv.spin, sv.p)
        if fd_order:
            from .lattice import fd_symbol
            dim = self.grid.dim
            p_eff = [float(fd_symbol(sv.p[j], self.lat.dx[j], fd_order)) if j < dim else sv.p[j] for j in range(3)]
            self.w, self.E, _ = dirac.background_spinor(sv.kind, sv.spin, p_eff)
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

    def field_terms(self, t: float, psi):
        """The right-hand side without the kinetic term: -i V(t) (psi + psi_b)."""
        return -1j * apply(self.potential_matrix(t), psi + self.psi_back(t))

    def rhs(self, t: float, psi):
        return self.kinetic(psi) + self.field_terms(t, psi)

    # -- the free evolution, exactly ----------------------------------------
    def free_propagator(self, tau: float):
        """exp(-i H0(k) tau) per Fourier mode: H0(k)^2 = E_k^2, so the
        exponential series sums to cos(E_k tau) - i sin(E_k tau) H0(k) / E_k."""
        I = dirac.I4.reshape((4, 4) + (1,) * self.lat.dim)
        return np.cos(self.Ek * tau)[None, None] * I - \
            1j * (np.sin(self.Ek * tau) / self.Ek)[None, None] * self.H0

    def free_evolve(self, psi, tau: float):
        """psi evolved by the free Dirac equation d_t psi = -i H0 psi over tau."""
        return self.lat.ifft(apply(self.free_propagator(tau), self.lat.fft(psi)))

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
        """One step from t_n; returns y_{n+1}, the stage inputs with their
        times (the augmented BW integral needs them) and the scheme's weights
        of the stages."""
        if self.scheme == "dp5":
            return self._dp5_stages(n, y)[:4]
        if self.scheme == "iprk4":
            return self._iprk4_stages(n, y)
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
        return ynew, (y1, y2, y3, y4), (t, t + 0.5 * h, t + 0.5 * h, t + h), (1 / 6, 1 / 3, 1 / 3, 1 / 6)

    # -- interaction picture: Lawson's integrating-factor RK4 ------------------
    def _iprk4_stages(self, n: int, y):
        """One step of d_t y = L y + N(t, y), L = -i H0 taken exactly: with
        phi = exp(-L (t - t_n)) y the classical RK4 tableau is applied to
        d_t phi = exp(-L (t - t_n)) N(t, exp(L (t - t_n)) phi) and the result
        mapped back.  With P(tau) = exp(L tau):
            k1 = N(t, y)
            k2 = N(t + h/2, P(h/2) (y + h/2 k1))
            k3 = N(t + h/2, P(h/2) y + h/2 k2)
            k4 = N(t + h, P(h) y + h P(h/2) k3)
            y_{n+1} = P(h) y + h/6 (P(h) k1 + 2 P(h/2) k2 + 2 P(h/2) k3 + k4).
        The stage inputs (the arguments of N) are approximations of psi at
        the stage times in the original picture, so the augmented BW integral
        takes them with the RK4 weights, as for the classical stepper."""
        h = self.window.dt if self.forward else -self.window.dt
        t = self.time(n)
        P = lambda v, tau: self.free_evolve(v, tau)  # noqa: E731
        N = self.field_terms
        y1 = y
        k1 = N(t, y1)
        y2 = P(y + 0.5 * h * k1, 0.5 * h)
        k2 = N(t + 0.5 * h, y2)
        y3 = P(y, 0.5 * h) + 0.5 * h * k2
        k3 = N(t + 0.5 * h, y3)
        y4 = P(y, h) + h * P(k3, 0.5 * h)
        k4 = N(t + h, y4)
        ynew = P(y, h) + (h / 6.0) * (P(k1, h) + 2.0 * P(k2, 0.5 * h) + 2.0 * P(k3, 0.5 * h) + k4)
        if self.mask is not None:
            ynew = ynew * self.mask[None]
        return ynew, (y1, y2, y3, y4), (t, t + 0.5 * h, t + 0.5 * h, t + h), (1 / 6, 1 / 3, 1 / 3, 1 / 6)

    # -- Dormand-Prince 5(4), fixed step ------------------------------------
    def _dp5_stages(self, n: int, y):
        """One Dormand-Prince step: the six stages of the fifth-order solution
        (the seventh, at t + h with weight 0, only serves the error estimate)."""
        h = self.window.dt if self.forward else -self.window.dt
        t = self.time(n)
        ys, ts, ks = [], [], []
        for i in range(6):
            yi = y
            for a, k in zip(DP5_A[i], ks):
                if a != 0.0:
                    yi = yi + (h * a) * k
            ti = t + DP5_C[i] * h
            ys.append(yi)
            ts.append(ti)
            ks.append(self.rhs(ti, yi))
        ynew = y
        for b, k in zip(DP5_B, ks):
            if b != 0.0:
                ynew = ynew + (h * b) * k
        if self.mask is not None:
            ynew = ynew * self.mask[None]
        return ynew, tuple(ys), tuple(ts), DP5_B[:6], ks, h, t

    def dp5_error(self, n: int, y):
        """(y_{n+1}, e): the step and the embedded estimate e = y5 - y4 =
        h sum_i (b_i - bhat_i) k_i, with k_7 = F(t + h, y_{n+1}) (no mask)."""
        if self.mask is not None:
            raise ValueError("the error estimate is defined without the absorber")
        ynew, _, _, _, ks, h, t = self._dp5_stages(n, y)
        ks = ks + [self.rhs(t + h, ynew)]
        e = sum((h * (b - bh)) * k for b, bh, k in zip(DP5_B, DP5_BHAT, ks))
        return ynew, e

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
