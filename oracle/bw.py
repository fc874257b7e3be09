"""Nonlinear Breit-Wheeler amplitude from scattered waves.

Section "Nonlinear Breit-Wheeler pair production": with out-solutions U, V
and an absorbed plane-wave photon eps_mu e^{-ikx}, M = int d^4x Ubar epsslash
e^{-ikx} V splits into (scat,scat) + (back,scat) + (scat,back) terms, the
(back,back) term being a vanishing delta^4(p+q-k).  Each term is split at
t_in into a finite-time part, eq. (Mabfinite), and an asymptotic-past part
done analytically after decomposing the free scattered waves into positive-
and negative-energy plane waves, eq. (MScatScatPast) and its two single-mode
partners.  The future part vanishes because psi_scat = 0 after t_out.

Finite part: the paper appends M_ab(t) to the stepped state (the
Y = (psi, M) construction), so the same RK4 integrates
dM_ab/dt = int d^dx Ubar_a epsslash e^{-ikx} V_b from t_out to t_in; with
epsilon_mu = (0, eps) one has gamma^0 epsslash = alpha.eps.  Then
M_finite = int_{t_in}^{t_out} = -M(t_in).

Past part, on the lattice: U~ = FFT(U_scat(t_in)), V~' = FFT(V_scat(t_in)
e^{i k.x}) so that V~'(kappa) is V~(kappa - k); with Pi_sigma the energy
projectors (sigma = +1: e^{-iEt}),

  M_past^{ss} = e^{-i k0 t_in} dV/N sum_kappa sum_{sigma,sigma'}
        (Pi_sigma U~)^dag (alpha.eps) (Pi_sigma' V~') / (i(sigma E_kappa - sigma' E_{kappa-k} - k0)),
  M_past^{bs} = e^{i(p0-k0) t_in} sum_sigma' u^dag (alpha.eps) Pi_sigma'(p-k) V_c(p-k)
                / (i(p0 - sigma' E_{p-k} - k0)),
  M_past^{sb} = e^{i(q0-k0) t_in} sum_sigma (Pi_sigma(k-q) U_c(k-q))^dag (alpha.eps) v
                / (i(sigma E_{k-q} + q0 - k0)),

with V_c(kappa) = dV sum_x V_scat(x) e^{-i kappa.x} (continuum Fourier
coefficient at an off-lattice kappa).  The paper's Lambda_(+-) carry the sign
of the exponent e^{+-iQ_0 t}, i.e. Lambda_+ = Pi_-; the three formulas above
are its (MScatScatPast) family rewritten in that reading, including the
typo reading v_scat(q) -> v(q) in the (scat,back) term.

Returned normalisation: M per (2 pi)^(3-d) delta_perp(q + p - k), no
phase-space or e^2 factors (the Fig. 7 convention).
"""
from __future__ import annotations

import numpy as np

from . import dirac
from .swf import SWFSolve, apply


def gamma_eps(eps):
    """gamma^0 epsslash for epsilon_mu = (0, eps): alpha.eps."""
    return sum(dirac.ALPHA[j] * float(eps[j]) for j in range(3))


class Vertex:
    def __init__(self, problem, index: int):
        vx = problem.vertices[index]
        self.vx = vx
        self.U = SWFSolve(problem, vx.u_solve)
        self.V = SWFSolve(problem, vx.v_solve)
        if self.U.solve.kind != 0 or self.V.solve.kind != 1:
            raise ValueError("vertex needs a U solve and a V solve")
        if self.U.lat.shape != self.V.lat.shape:
            raise ValueError("vertex solves must share the lattice")
        self.k3 = np.asarray(vx.k, dtype=float)
        self.k0 = float(np.linalg.norm(self.k3))
        self.G = gamma_eps(vx.eps)
        lat = self.U.lat
        for j in range(lat.dim, 3):
            if abs(self.U.K[j] - self.k3[j] - self.V.K[j]) > 1e-12:
                raise ValueError("trivial-axis momentum conservation p + q = k violated")
        self.photon_x = np.exp(1j * sum(self.k3[j] * lat.X[j] for j in range(lat.dim))) \
            if lat.dim > 0 else np.ones(lat.shape)

    def mdot(self, t, yU, yV):
        """dM_ab/dt for (scat,scat), (back,scat), (scat,back) at time t."""
        lat = self.U.lat
        ph = np.exp(-1j * self.k0 * t) * self.photon_x
        bU = self.U.psi_back(t)
        bV = self.V.psi_back(t)

        def f(a, b):
            return lat.dV * np.sum(ph[None] * np.conj(a) * apply(self.G, b))

        return np.array([f(yU, yV), f(bU, yV), f(yU, bV)])

    def run(self):
        """Step U and V in lock-step with the augmented M; returns
        (psi_U(t_in), psi_V(t_in), M(t_in)) with M(t_out) = 0."""
        win = self.U.window
        h = -win.dt
        yU = self.U.zero_state()
        yV = self.V.zero_state()
        M = np.zeros(3, dtype=complex)
        for n in range(win.steps):
            yU_new, sU, tt, wts = self.U.step_stages(n, yU)
            yV_new, sV, _, _ = self.V.step_stages(n, yV)
            d = [self.mdot(tt[i], sU[i], sV[i]) for i in range(len(tt))]
            if self.U.scheme == "rk4":
                M = M + (h / 6.0) * (d[0] + 2.0 * d[1] + 2.0 * d[2] + d[3])
            else:
                for w, di in zip(wts, d):
                    M = M + (h * w) * di
            yU, yV = yU_new, yV_new
        return yU, yV, M

    def past(self, psiU, psiV, t_in):
        """M_past for (scat,scat), (back,scat), (scat,back)."""
        return self.past_for(psiU, psiV, t_in, self.k3, self.vx.eps)

    def past_for(self, psiU, psiV, t_in, k3, eps):
        """M_past of a plane-wave photon of 3-momentum k3 and polarisation eps."""
        U, V, lat = self.U, self.V, self.U.lat
        k3 = np.asarray(k3, dtype=float)
        k0 = float(np.linalg.norm(k3))
        G = gamma_eps(eps)
        photon_x = np.exp(1j * sum(k3[j] * lat.X[j] for j in range(lat.dim))) if lat.dim > 0 else np.ones(lat.shape)
        # (scat, scat)
        Uk = lat.fft(psiU)
        Vk = lat.fft(psiV * photon_x[None])
        kU = U.kfull
        kV = [kU[j] - k3[j] for j in range(3)]
        EU = np.sqrt(1.0 + sum(a ** 2 for a in kU))
        EV = np.sqrt(1.0 + sum(a ** 2 for a in kV))
        I4 = dirac.I4.reshape((4, 4) + (1,) * lat.dim)

        def proj(kk, E, sign):
            H = sum(dirac.ALPHA[j].reshape((4, 4) + (1,) * lat.dim) * kk[j][None, None]
                    for j in range(3)) + dirac.BETA.reshape((4, 4) + (1,) * lat.dim)
            return 0.5 * (I4 + sign * H / E[None, None])

        acc = 0.0 + 0.0j
        for sg in (1, -1):
            PU = apply(proj(kU, EU, sg), Uk)
            for sgp in (1, -1):
                PV = apply(proj(kV, EV, sgp), Vk)
                den = 1j * (sg * EU - sgp * EV - k0)
                acc += np.sum(np.conj(PU) * apply(G, PV) / den[None])
        m_ss = np.exp(-1j * k0 * t_in) * lat.dV / lat.N * acc

        def cont_ft(psi, kappa):
            ph = np.exp(-1j * sum(kappa[j] * lat.X[j] for j in range(lat.dim)))
            return lat.dV * np.sum(psi * ph[None], axis=tuple(range(1, lat.dim + 1)))

        # (back, scat): U_back = u e^{-i p0 t + i p.x}
        p3 = U.K
        p0 = U.E
        kap = p3 - k3
        Ek = dirac.energy(kap)
        Vc = cont_ft(psiV, kap)
        m_bs = 0.0 + 0.0j
        for sgp in (1, -1):
            PV = dirac.projector(kap, sgp) @ Vc
            m_bs += np.conj(U.w) @ (G @ PV) / (1j * (p0 - sgp * Ek - k0))
        m_bs *= np.exp(1j * (p0 - k0) * t_in)

        # (scat, back): V_back = v e^{+i q0 t - i q.x}; V.K = -q, V.E = -q0
        q3 = -V.K
        q0 = -V.E
        kap = k3 - q3
        Ek = dirac.energy(kap)
        Uc = cont_ft(psiU, kap)
        m_sb = 0.0 + 0.0j
        for sg in (1, -1):
            PU = dirac.projector(kap, sg) @ Uc
            m_sb += np.conj(PU) @ (G @ V.w) / (1j * (sg * Ek + q0 - k0))
        m_sb *= np.exp(1j * (q0 - k0) * t_in)
        return np.array([m_ss, m_bs, m_sb])

    # -- second route: partial integration in t -----------------------------
    # Section "Nonlinear Breit-Wheeler": with the scattered waves split into
    # projected, phase-removed components, integrating by parts in t turns
    # every term into an integral over d/dt of those components; the free
    # (H0) part of the evolution drops out mode by mode (Pi_sigma H0 = sigma E
    # Pi_sigma on the lattice), so only the source S = -i V (psi_s + psi_b)
    # remains and the integrand vanishes outside the field: no past term, the
    # window [t_in, t_out] holds the whole integral.  In the reading of the
    # first route (Lambda_+ = Pi_-, e^{-ikx} photon, alpha.eps):
    #   ss: i e^{-i k0 t} dV/N sum_kappa sum_{s,s'} [(Pi_s S~_U)^dag G Pi_s' V~'
    #       + (Pi_s U~)^dag G Pi_s' S~'_V] / Om_ss',  Om = s E - s' E' - k0,
    #       V~' = FFT(V e^{ik.x}) (E' and Pi_s' at kappa - k);
    #   bs: sum_s' i e^{i(p0-k0)t} u^dag G Pi_s'(p-k) S_V,c(p-k) / (p0 - s' E - k0);
    #   sb: sum_s  i e^{i(q0-k0)t} (Pi_s(k-q) S_U,c(k-q))^dag G v / (s E + q0 - k0).
    # Exact on the lattice when p, q and k are lattice momenta on the
    # non-trivial axes (the shift theorem and the mode-wise identity hold).
    def mdot_partial(self, t, yU, yV):
        U, V, lat = self.U, self.V, self.U.lat
        k3, k0, G = self.k3, self.k0, self.G
        SU = U.rhs(t, yU) - U.kinetic(yU)
        SV = V.rhs(t, yV) - V.kinetic(yV)
        Uk, SUk = lat.fft(yU), lat.fft(SU)
        Vk, SVk = lat.fft(yV * self.photon_x[None]), lat.fft(SV * self.photon_x[None])
        kU = U.kfull
        kV = [kU[j] - k3[j] for j in range(3)]
        EU = np.sqrt(1.0 + sum(a ** 2 for a in kU))
        EV = np.sqrt(1.0 + sum(a ** 2 for a in kV))
        I4 = dirac.I4.reshape((4, 4) + (1,) * lat.dim)

        def proj(kk, E, sign):
            H = sum(dirac.ALPHA[j].reshape((4, 4) + (1,) * lat.dim) * kk[j][None, None]
                    for j in range(3)) + dirac.BETA.reshape((4, 4) + (1,) * lat.dim)
            return 0.5 * (I4 + sign * H / E[None, None])

        acc = 0.0 + 0.0j
        for sg in (1, -1):
            PU, PSU = apply(proj(kU, EU, sg), Uk), apply(proj(kU, EU, sg), SUk)
            for sgp in (1, -1):
                PV, PSV = apply(proj(kV, EV, sgp), Vk), apply(proj(kV, EV, sgp), SVk)
                om = sg * EU - sgp * EV - k0
                acc += np.sum((np.conj(PSU) * apply(G, PV) + np.conj(PU) * apply(G, PSV)) / om[None])
        m_ss = 1j * np.exp(-1j * k0 * t) * lat.dV / lat.N * acc

        def cont_ft(psi, kappa):
            ph = np.exp(-1j * sum(kappa[j] * lat.X[j] for j in range(lat.dim)))
            return lat.dV * np.sum(psi * ph[None], axis=tuple(range(1, lat.dim + 1)))

        p3, p0 = U.K, U.E
        kap = p3 - k3
        Ek = dirac.energy(kap)
        Sc = cont_ft(SV, kap)
        m_bs = sum(np.conj(U.w) @ (G @ (dirac.projector(kap, sgp) @ Sc)) / (p0 - sgp * Ek - k0) for sgp in (1, -1))
        m_bs *= 1j * np.exp(1j * (p0 - k0) * t)

        q3, q0 = -V.K, -V.E
        kap = k3 - q3
        Ek = dirac.energy(kap)
        Sc = cont_ft(SU, kap)
        m_sb = sum(np.conj(dirac.projector(kap, sg) @ Sc) @ (G @ V.w) / (sg * Ek + q0 - k0) for sg in (1, -1))
        m_sb *= 1j * np.exp(1j * (q0 - k0) * t)
        return np.array([m_ss, m_bs, m_sb])

    def amplitude_partial(self):
        """M by the partial-integration route: the three terms integrated over
        [t_in, t_out] with the same augmented RK4 as the first route."""
        win = self.U.window
        h = -win.dt
        yU = self.U.zero_state()
        yV = self.V.zero_state()
        M = np.zeros(3, dtype=complex)
        for n in range(win.steps):
            yU_new, sU, tt, wts = self.U.step_stages(n, yU)
            yV_new, sV, _, _ = self.V.step_stages(n, yV)
            d = [self.mdot_partial(tt[i], sU[i], sV[i]) for i in range(len(tt))]
            if self.U.scheme == "rk4":
                M = M + (h / 6.0) * (d[0] + 2.0 * d[1] + 2.0 * d[2] + d[3])
            else:
                for w, di in zip(wts, d):
                    M = M + (h * w) * di
            yU, yV = yU_new, yV_new
        terms = -M
        return {"terms": terms, "total": complex(np.sum(terms))}

    def amplitude(self):
        """Returns dict with per-term finite and past parts and the total M."""
        psiU, psiV, Mt = self.run()
        t_in = self.U.window.t_in
        finite = -Mt
        past = self.past(psiU, psiV, t_in)
        return {"finite": finite, "past": past, "terms": finite + past,
                "total": complex(np.sum(finite + past)), "psiU": psiU, "psiV": psiV}


class PacketVertex(Vertex):
    """Breit-Wheeler amplitude for a photon wave packet (the BW section's
    numerical approach, on wave packets): f_mu(x) = sum_m c_m eps_m,mu e^{-i k_m x}
    takes the place of eps_mu e^{-ikx} in the finite-time integrand of
    eq. (Mabfinite), so with epsilon_mu = (0, eps) the integrand is
    Ubar_a gamma^0 (alpha.E(t,x)) V_b with E = sum_m c_m eps_m e^{-i(k0_m t - k_m.x)};
    the past terms, eq. (MScatScatPast) and its partners, are evaluated on the
    packet's momentum grid and summed with the weights c_m."""

    def __init__(self, problem, index: int):
        vx = problem.vertices[index]
        if not vx.modes:
            raise ValueError("PacketVertex needs a vertex with modes")
        self.modes = [(np.asarray(k, dtype=float), np.asarray(e, dtype=float), complex(c)) for k, e, c in vx.modes]
        # the base class checks the solves and trivial-axis conservation with the first mode
        import dataclasses
        first = dataclasses.replace(vx, k=list(self.modes[0][0]), eps=list(self.modes[0][1]), modes=[])
        probe = dataclasses.replace(problem, vertices=[first])
        super().__init__(probe, 0)
        self.vx = vx
        lat = self.U.lat
        for k3, _, _ in self.modes:
            for j in range(lat.dim, 3):
                if abs(self.U.K[j] - k3[j] - self.V.K[j]) > 1e-12:
                    raise ValueError("trivial-axis momentum conservation p + q = k violated by a mode")
        self.mode_x = [np.exp(1j * sum(k3[j] * lat.X[j] for j in range(lat.dim))) if lat.dim > 0
                       else np.ones(lat.shape) for k3, _, _ in self.modes]

    def packet_field(self, t):
        """E(t, x): complex polarisation 3-vector field of the packet (3, *lattice)."""
        E = np.zeros((3,) + self.U.lat.shape, dtype=complex)
        for (k3, e, c), ph in zip(self.modes, self.mode_x):
            a = c * np.exp(-1j * float(np.linalg.norm(k3)) * t) * ph
            for j in range(3):
                E[j] = E[j] + a * e[j]
        return E

    def mdot(self, t, yU, yV):
        lat = self.U.lat
        E = self.packet_field(t)
        bU = self.U.psi_back(t)
        bV = self.V.psi_back(t)

        def alpha_E(b):
            return sum(apply(dirac.ALPHA[j].reshape((4, 4) + (1,) * lat.dim) * E[j][None, None], b)
                       for j in range(3))

        def f(a, b):
            return lat.dV * np.sum(np.conj(a) * alpha_E(b))

        return np.array([f(yU, yV), f(bU, yV), f(yU, bV)])

    def past(self, psiU, psiV, t_in):
        return sum(c * self.past_for(psiU, psiV, t_in, k3, e) for k3, e, c in self.modes)
