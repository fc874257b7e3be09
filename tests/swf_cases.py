"""Small SWF problems shared by the parity tests (descriptors only).

Fields switch on every coupling (A_0 and all three alpha^j A_j, several
profile shapes and carriers) and grids mix power-of-two and mixed-radix
lengths, so a wrong sign, index or axis in any pass shows up.
"""
import numpy as np

import swf_workloads as W


def field_mix(dim):
    """A_0, A_1, A_2, A_3 all non-zero, every profile type, carriers on."""
    g = [W.gauss(4.0), W.sech2(5.0, c=0.5), W.gauss(3.5, k=0.4, phi=0.3)]
    fx = [g[j] if j < dim else W.const() for j in range(3)]

    def with_axis(j, prof):
        f = list(fx)
        if j < dim:
            f[j] = prof
        return f

    return [
        W.Term(1, 0.9, W.sech2(1.5), list(fx)),
        W.Term(0, 0.35, W.ugauss(1.2, c=0.2), with_axis(0, W.ugauss(3.0))),
        W.Term(2, 0.25, W.gauss(1.3, k=0.8, phi=0.1), with_axis(min(1, dim - 1), W.sech2(3.0))),
        W.Term(3, 0.2, W.gauss(1.1), with_axis(dim - 1, W.gauss(2.5, c=-0.4))),
        W.Term(1, 0.1, W.tanh(0.9), list(fx)),
    ]


def grid(dim, n, L):
    nn = list(n) + [1] * (3 - len(n))
    LL = list(L) + [1.0] * (3 - len(L))
    return W.Grid(dim, nn, LL)


def random_momenta(k, dim, L, n, seed):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(k):
        p = []
        for j in range(3):
            if j < dim:
                kny = np.pi * n[j] / L[j]
                p.append(float(rng.uniform(-0.5, 0.5) * kny))
            else:
                p.append(float(rng.uniform(-0.6, 0.6)))
        out.append(p)
    return out


def problem(dim, n, L, kinds=(0, 1), spins=(1, -1), n_mom=1, dt=0.05, t_half=2.0, seed=0,
            field=None):
    g = grid(dim, n, L)
    ps = random_momenta(n_mom, dim, g.L, g.n, seed)
    solves = [W.Solve(k, s, p) for p in ps for k in kinds for s in spins]
    return W.Problem(f"mix{dim}d", [g], [field or field_mix(dim)], solves, W.Window(-t_half, t_half, dt))


def lattice_p(dim, n, L, m, trivial=(0.3, -0.2)):
    """A momentum on the lattice: m[j] grid units on non-trivial axes."""
    p = []
    for j in range(3):
        if j < dim:
            p.append(2 * np.pi * m[j] / L[j])
        else:
            p.append(trivial[j - dim] if j - dim < len(trivial) else 0.0)
    return p
