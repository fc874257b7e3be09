"""Background potential A_mu(t, x) as a sum of separable terms.

The paper assumes A_mu -> 0 as |x^mu| -> infinity (section "Scattered wave
functions") and works with analytic fields such as eqs. (singleE) and
(doubleE).  A term adds amp * f_t(t) * f_x(x) * f_y(y) * f_z(z) to the
covariant component A_mu; a profile is env((s - c)/w) * cos(k s + phi).
"""
from __future__ import annotations

import numpy as np

from swf_workloads import PROF_CONST, PROF_GAUSS, PROF_SECH2, PROF_TANH, PROF_UGAUSS


def profile(pr, s):
    s = np.asarray(s, dtype=float)
    if pr.type == PROF_CONST:
        env = np.ones_like(s)
    else:
        u = (s - pr.c) / pr.w
        if pr.type == PROF_GAUSS:
            env = np.exp(-u * u)
        elif pr.type == PROF_SECH2:
            env = 1.0 / np.cosh(u) ** 2
        elif pr.type == PROF_TANH:
            env = np.tanh(u)
        elif pr.type == PROF_UGAUSS:
            env = u * np.exp(-u * u)
        else:
            raise ValueError(f"unknown profile type {pr.type}")
    if pr.k != 0.0 or pr.phi != 0.0:
        env = env * np.cos(pr.k * s + pr.phi)
    return env


def potential(terms, t, lat):
    """A_mu(t, x) on the lattice: list of 4 real arrays (mu = 0..3)."""
    A = [np.zeros(lat.shape) for _ in range(4)]
    for term in terms:
        val = term.amp * float(profile(term.ft, t))
        f = np.full(lat.shape, val)
        for j in range(lat.dim):
            f = f * profile(term.fx[j], lat.X[j])
        for j in range(lat.dim, 3):
            # trivial axes: the field must not depend on them
            if term.fx[j].type != PROF_CONST or term.fx[j].k != 0.0 or term.fx[j].phi != 0.0:
                raise ValueError("field depends on a trivial axis")
        A[term.mu] = A[term.mu] + f
    return A
