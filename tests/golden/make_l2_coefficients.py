"""Writes l2_coefficients.txt: the exact minimisers of the L2 polynomial cost
(eq:l2cost, Section 2.5) for degrees 0..8, as computed by the oracle.

    python tests/golden/make_l2_coefficients.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as orc  # noqa: E402


def main():
    lines = ["# exact coefficients c_0 .. c_d (ascending powers) of the L2-optimal polynomial",
             "# (eq:l2cost, Section 2.5), degrees 0..8; written by make_l2_coefficients.py from oracle/"]
    for d in range(9):
        lines.append(f"{d} " + " ".join(str(c) for c in orc.l2_poly_coefficients(d)))
    with open(os.path.join(HERE, "l2_coefficients.txt"), "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
