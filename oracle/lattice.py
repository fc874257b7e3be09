"""Periodic spatial lattice for the pseudo-spectral discretisation.

The paper stores psi(t) as an array of shape (g, n_x, n_y, n_z) and takes
spatial derivatives through FFTs (section "Numerical approach").  Here the
non-trivial axes are the first ``dim`` of (x, y, z); x_j[i] = -L_j/2 + i L_j/n_j
and k_j = 2 pi fftfreq(n_j, L_j/n_j) (numpy's convention, Nyquist kept at
-pi/dx).  A plane wave exp(i k.x) then has d_j -> i k_j.
"""
from __future__ import annotations

import numpy as np


class Lattice:
    def __init__(self, grid, fd_order: int = 0):
        self.dim = int(grid.dim)
        self.n = [int(grid.n[j]) for j in range(self.dim)]
        self.L = [float(grid.L[j]) for j in range(self.dim)]
        self.dx = [self.L[j] / self.n[j] for j in range(self.dim)]
        self.x1d = [-self.L[j] / 2 + np.arange(self.n[j]) * self.dx[j] for j in range(self.dim)]
        self.k1d = [2 * np.pi * np.fft.fftfreq(self.n[j], self.dx[j]) for j in range(self.dim)]
        self.fd_order = fd_order
        if fd_order:
            # a periodic central finite-difference derivative is diagonal in Fourier
            # space with the stencil's symbol in place of k
            self.k1d = [fd_symbol(k, self.dx[j], fd_order) for j, k in enumerate(self.k1d)]
        self.X = np.meshgrid(*self.x1d, indexing="ij")
        self.K = np.meshgrid(*self.k1d, indexing="ij")
        self.dV = float(np.prod(self.dx))
        self.N = int(np.prod(self.n))
        self.shape = tuple(self.n)
        self.axes = tuple(range(1, self.dim + 1))   # spatial axes of a (4, ...) spinor array

    def fft(self, psi):
        return np.fft.fftn(psi, axes=self.axes)

    def ifft(self, psik):
        return np.fft.ifftn(psik, axes=self.axes)

    def full_momentum(self, trivial):
        """Per-site 3-momentum: lattice k on non-trivial axes, the conserved
        constant ``trivial[j]`` on the others.  Returns a list of 3 arrays."""
        out = []
        for j in range(3):
            if j < self.dim:
                out.append(self.K[j])
            else:
                out.append(np.full(self.shape, float(trivial[j])))
        return out

    def absorber(self, cells: int, strength: float):
        """Mask m(x) = prod_j m_j(x_j) applied after every step when enabled:
        m_j = 1 - strength * sin^2(pi/2 * (cells - d)/cells) within ``cells``
        of either edge (d = distance in cells to the nearest edge), 1 inside.
        Not part of the paper (its scattered waves are simply kept inside a
        periodic box); off whenever cells == 0.  Pinned as an absorbing layer:
        an outgoing packet leaves the interior as it would on a periodic box
        twice as long (no reflection, no wrap-around)."""
        m = np.ones(self.shape)
        if cells <= 0:
            return m
        for j in range(self.dim):
            i = np.arange(self.n[j])
            d = np.minimum(i, self.n[j] - 1 - i).astype(float)
            mj = np.where(d < cells, 1.0 - strength * np.sin(0.5 * np.pi * (cells - d) / cells) ** 2, 1.0)
            shp = [1] * self.dim
            shp[j] = self.n[j]
            m = m * mj.reshape(shp)
        return m


def fd_coefficients(order: int):
    """Weights a_1..a_p of the central first-derivative stencil of even order
    2p, f'(x) ~ sum_m a_m (f(x + m dx) - f(x - m dx)) / dx: the unique
    weights that make it exact for polynomials of degree 2p, in closed form
    a_m = (-1)^(m+1) (p!)^2 / (m (p-m)! (p+m)!)."""
    from math import factorial
    if order < 2 or order % 2:
        raise ValueError("the central stencil has an even order >= 2")
    p = order // 2
    return [(-1) ** (m + 1) * factorial(p) ** 2 / (m * factorial(p - m) * factorial(p + m)) for m in range(1, p + 1)]


def fd_symbol(k, dx: float, order: int):
    """The stencil's Fourier symbol: it maps exp(ikx) to i K(k) exp(ikx) with
    K(k) = sum_m 2 a_m sin(m k dx) / dx (for any k, on or off the lattice)."""
    k = np.asarray(k, dtype=float)
    return sum(2.0 * a * np.sin(m * k * dx) for m, a in enumerate(fd_coefficients(order), start=1)) / dx

