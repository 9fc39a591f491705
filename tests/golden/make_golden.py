"""Writes the stored expected values under tests/golden/ (calls only the oracle).

    python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle  # noqa: E402


def main():
    c = oracle.cheby_coeffs(10, 1.0, 64.0)
    with open(os.path.join(HERE, "cheby_order10_1_64.txt"), "w") as f:
        f.write("# Chebyshev interpolation coefficients c_j of 1/y on [1.0, 64.0], 10 terms:\n")
        f.write("# the smoother polynomial of Sec. 4 (order 10 approximation to 1/x on [1, 64]).\n")
        f.write("# p(y) = sum_j c_j T_j((2y - 65)/63) - c_0/2.  Written by tests/golden/make_golden.py.\n")
        for j, v in enumerate(c):
            f.write(f"{j} {v:.17e}\n")


if __name__ == "__main__":
    main()
