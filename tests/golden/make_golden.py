"""Writes the stored template values under tests/golden/ (calls only oracle/).

templates_mpmath.txt: G_z(q) = int_{-1/2}^{1/2} exp(i pi (z s^2 - 2 q s)) ds,
the response whose closed form the oracle uses (Section 1, the predicted
normalised response named before eq. 2), evaluated by 30-digit mpmath
quadrature of the defining integral. Columns: z q Re(G) Im(G).

Run from the repository root:  python tests/golden/make_golden.py
"""
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle.templates import response_g_mpmath  # noqa: E402

CASES = [(z, q) for z in (2.0, 7.0, 16.0, 100.0, -7.0, 200.0)
         for q in (0.0, 1.0, -3.0, 0.3, 12.5, -40.0, 128.0)]


def main():
    path = os.path.join(HERE, "templates_mpmath.txt")
    with open(path, "w") as f:
        f.write("# z q re im  (mpmath quadrature of the defining integral, 30 digits)\n")
        for z, q in CASES:
            g = response_g_mpmath(z, q, dps=30)
            f.write(f"{z:.1f} {q:.1f} {g.real:.17e} {g.imag:.17e}\n")


if __name__ == "__main__":
    main()
