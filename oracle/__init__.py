"""Plain FP64 CPU oracle for the scattered-wave-function (SWF) hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product library imports, links or
runs this package; only the tests, the smoke check and the benchmark's CPU
baseline leg do.  It shares no code with the HIP path: the only thing both
sides consume is the data-only input module ``swf_workloads``.

What it computes (arXiv 2512.16889, "Solving the Dirac equation on a GPU for
strong-field processes in multidimensional background fields"):

* ``dirac``       gamma matrices, free spinors u_s / v_s of eq. (uv) with the
                  R_s of eq. (Reqs), free Hamiltonian and energy projectors
                  (the Lambda matrices of eq. (LambdaDef)), photon
                  polarisation basis of eq. (epsParaPerp).
* ``lattice``     periodic grid, FFT wavenumbers (section "Numerical approach").
* ``field``       separable background potentials A_mu(t, x), including the
                  paper's single/double-peak examples, eqs. (singleE), (doubleE).
* ``swf``         the inhomogeneous Dirac equation for the scattered wave,
                  eq. (scatDirac), discretised pseudo-spectrally in space and
                  integrated with classical RK4 from t_out back to t_in
                  (out-states U_out, V_out) or from t_in forward to t_out
                  (in-states U_in, V_in); or with the paper's Dopri5
                  tableau at a fixed step; or in the interaction picture
                  (Lawson's integrating-factor RK4: the free evolution
                  exp(-i H0(k) tau) exact in Fourier space).  A variant
                  derivative, the periodic central finite difference of
                  order 2, 4 or 8 (``fd_order``), judges a stencil against
                  the spectral derivative.
* ``observables`` inner products at the end of a run: the pair amplitude of
                  eq. (Nmn) in both of its forms, electron/positron marginals,
                  norm/orthogonality diagnostics.
* ``bw``          nonlinear Breit-Wheeler amplitude: the finite-time vertex
                  overlap of eq. (Mabfinite) integrated as an augmented
                  state (the Y = (psi, M) construction of the BW numerical
                  section) plus the analytic asymptotic-past terms
                  (eq. (MScatScatPast) and its two single-mode partners);
                  and the section's second route, eq. (MScatScat2) and its
                  partners (partial integration in t), as an independent
                  check of the first; and a photon wave packet f_mu(x) =
                  sum_m c_m eps_m e^{-i k_m x} in place of the plane wave
                  (finite part with f in the integrand, past part summed
                  over the packet's momentum grid), as the section's
                  numerical approach describes.

Pins (tests/test_oracle_*.py, all ``-m "not gpu"``) tie every function to
something other than itself: Clifford algebra and spinor identities, the
closed-form pure-gauge scattered wave, the Sauter-pulse pair spectrum,
brute-force full-wave-function evolution with scipy's DOP853, unitarity and
orthogonality identities, charge-conjugation symmetry, RK4 convergence
order; for the interaction picture, scipy's matrix exponential of H0(k),
a free plane wave stepped exactly at any step size, order-4 convergence to
the classical stepper's solution; for in-states, the pure-gauge closed form, the time independence of
in/out overlaps (an in-state read at t_out against an out-state read at
t_in) and the in/out balance of marginals over a complete lattice; the
exact spin structure of the BW amplitude for E(t,x) fields and
the t_in independence of past + finite BW terms; for wave packets, a packet
of one plane wave is that wave, a packet is the weighted sum of its plane
waves, and a Gaussian packet tends to the plane wave as its momentum width
shrinks (at order sigma^2).

The absorbing-boundary mask (not part of the paper; off for every other pin
and parity case) is pinned by a wave packet leaving the box: inside the
unmasked interior the masked box gives the wave of a periodic box twice as
long, before and after the packet crosses the edge.
"""
