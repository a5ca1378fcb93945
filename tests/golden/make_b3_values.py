"""Writes b3_spline_values.txt: the B3 spline of Sec. 4.2 in exact rationals.

Run from the repository root:  python tests/golden/make_b3_values.py
It evaluates the paper's printed cubic B-spline with fractions.Fraction, so
every stored value is exact; it imports nothing from the library or oracle.
"""
import os
from fractions import Fraction as F


def phi(x):
    x = F(x)
    return F(1, 12) * (abs(x - 2) ** 3 - 4 * abs(x - 1) ** 3 + 6 * abs(x) ** 3
                       - 4 * abs(x + 1) ** 3 + abs(x + 2) ** 3)


def main():
    lines = ["# B3-spline scaling function of the starlet, Sec. 4.2 (the cubic",
             "# B-spline phi(x) = (|x-2|^3 - 4|x-1|^3 + 6|x|^3 - 4|x+1|^3 + |x+2|^3)/12),",
             "# evaluated in exact rational arithmetic at x = m/8, m = -20..20.",
             "# columns: numerator_of_x denominator_of_x numerator_of_phi denominator_of_phi"]
    for m in range(-20, 21):
        x = F(m, 8)
        v = phi(x)
        lines.append("%d %d %d %d" % (x.numerator, x.denominator, v.numerator, v.denominator))
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "b3_spline_values.txt")
    with open(out, "w") as f:
        f.write("\n".join(lines) + "\n")


if __name__ == "__main__":
    main()
