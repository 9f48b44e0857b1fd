"""Writes tests/golden/tiny_lp.json: exact optima of tiny rational l1-QR instances.

Calls only the oracle (the exact rational simplex); the stored optimum is then
re-derived in the tests by vertex enumeration and by the float FS-QRPPA oracle.
Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys
from fractions import Fraction

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__)))))
from oracle import lp  # noqa: E402

CASES = [
    # (X1 rows with the intercept first, y, tau, lam), all small rationals
    ([[1, 0], [1, 1], [1, 2], [1, 3], [1, 4]], [1, 3, 2, 5, 4], "1/2", [0, 0]),
    ([[1, 0], [1, 1], [1, 2], [1, 3], [1, 4], [1, 5]], [0, 2, 1, 4, 3, 7], "3/10", [0, "1/4"]),
    ([[1, 1, 0], [1, 0, 1], [1, 1, 1], [1, 2, -1], [1, -1, 2], [1, 0, 0]],
     [2, 1, 3, 1, 2, "1/2"], "9/10", [0, "1/10", "1/10"]),
    ([[1, 2, -1], [1, -1, 1], [1, 0, 2], [1, 1, 1], [1, -2, 0], [1, 3, 1]],
     [1, -1, 2, "3/2", -2, 4], "1/4", [0, "1/2", "1/5"]),
]


def main():
    out = []
    for X1, y, tau, lam in CASES:
        Xf = [[Fraction(v) for v in r] for r in X1]
        yf = [Fraction(v) for v in y]
        lf = [Fraction(v) for v in lam]
        c, A, b = lp.lp_data(Xf, yf, Fraction(tau), lf)
        val, _ = lp.simplex_exact(c, A, b)
        out.append(dict(X1=[[str(v) for v in r] for r in Xf], y=[str(v) for v in yf],
                        tau=tau, lam=[str(v) for v in lf], optimum=str(val),
                        source="exact rational simplex (oracle/lp.py)"))
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "tiny_lp.json")
    with open(path, "w") as f:
        json.dump(out, f, indent=1)
    print("wrote", path)


if __name__ == "__main__":
    main()
