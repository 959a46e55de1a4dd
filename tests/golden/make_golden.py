"""Writes the stored expected values under tests/golden/ by calling only the
CPU oracle and the seeded input generator.

The paper prints no worked example, so these are regression anchors for the
4-index-free factored oracle on the 8-fragment lattice workload (2x2x2,
3.1 A spacing, all 28 pairs): E2_xy after 0 and 3 effective-field iterations.
Run:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import fefgen  # noqa: E402
from oracle import fef  # noqa: E402


def main():
    s = fefgen.make_system(0)
    lines = ["# E2_xy (Eh) for the 8-fragment lattice workload; columns:",
             "# x y niter0 niter3   (oracle FP64, written by make_golden.py)"]
    E0, t0 = fef.pair_energies(s)
    C, e, hist = fef.run_scf(s, 3)
    E3, t3 = fef.pair_energies(s, C, e)
    for k in range(s.npair):
        lines.append(f"{s.pair_x[k]} {s.pair_y[k]} {E0[k]:.17e} {E3[k]:.17e}")
    lines.append(f"# total {t0:.17e} {t3:.17e}")
    with open(os.path.join(HERE, "config0_e2.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
