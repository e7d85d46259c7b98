"""Write tests/golden/*.txt from the oracle only (exact rational Gram-Schmidt basis).

Each file lists: dim k, then one line per point: the point's coordinates followed by the
values of the orthonormal basis there, from ExactBasis (exact rationals, normalised in FP64).
Run: python tests/golden/make_golden.py
"""
import os
import sys
from fractions import Fraction

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import sympy as sp  # noqa: E402

from oracle.bruteforce import ExactBasis  # noqa: E402

CASES = {(2, 3): [(Fraction(1, 7), Fraction(2, 5)), (Fraction(1, 3), Fraction(1, 3)),
                  (Fraction(3, 4), Fraction(1, 8))],
         (3, 2): [(Fraction(1, 7), Fraction(2, 9), Fraction(1, 5)),
                  (Fraction(1, 4), Fraction(1, 4), Fraction(1, 4))]}

for (dim, k), pts in CASES.items():
    B = ExactBasis(dim, k)
    lines = ["%d %d" % (dim, k)]
    for p in pts:
        sub = {g: sp.Rational(v.numerator, v.denominator) for g, v in zip(B.gens, p)}
        vals = [float(sp.Rational(psi.subs(sub))) / float(n) ** 0.5 for psi, n in zip(B.psi, B.norm2)]
        lines.append(" ".join(["%s" % (str(v)) for v in p] + ["%.17g" % v for v in vals]))
    with open(os.path.join(HERE, "dubiner_%dd_k%d.txt" % (dim, k)), "w") as f:
        f.write("\n".join(lines) + "\n")
print("written")
