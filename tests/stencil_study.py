"""Finite-difference stencil against the spectral derivative at matched P
error, on the CPU oracle: the (1+1)D Schwinger workload (sech^2 pulse,
L = 200, dt = 0.02, the whole 6000-step window), the electron marginal
P(s, p) of its solve.  Reference: spectral on 2048 points.  Prints one row
per derivative: the relative P error at each lattice size.

    python tests/stencil_study.py
"""
import os
import sys

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

import swf_workloads as W  # noqa: E402
from oracle import observables as ob  # noqa: E402
from oracle.swf import SWFSolve  # noqa: E402


def marginal(n, order=0):
    sv = SWFSolve(W.config_1d(n=n), 0, fd_order=order)
    return ob.marginal(sv, sv.run())


def main():
    ref = marginal(2048)
    sizes = (256, 512, 1024, 2048)
    print(f"reference P = {ref:.12e} (spectral, 2048 points)")
    print("| derivative | " + " | ".join(f"{n} points" for n in sizes) + " |")
    print("|---|" + "---|" * len(sizes))
    for order in (0, 2, 4, 8):
        cells = []
        for n in sizes:
            if order == 0 and n == 2048:
                cells.append("(reference)")
                continue
            cells.append(f"{abs(marginal(n, order) - ref) / ref:.1e}")
        name = "spectral" if order == 0 else f"central, order {order}"
        print(f"| {name} | " + " | ".join(cells) + " |", flush=True)


if __name__ == "__main__":
    main()
