"""Writes maxwell_oracle.json: the Maxwell limit (kappa = inf) of the
approximation, from the approximation-quality oracle only.

* optimum_c: the c minimising D(f_M||g; c) (eq:relative_entropy with the
  Maxwell density 2/sqrt(pi) x^(1/2) e^-x, a = (4/(3 sqrt(pi)))^(2/3),
  b/c = 1), the criterion of the grid search of Sec. 3;
* D and dE/E at a few c, for the GPU parity tests.

Run from the repository root:  python tests/golden/make_maxwell_golden.py
"""
import json
import math
import os
import sys

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))
from oracle import quality  # noqa: E402


def main():
    c_opt = quality.optimum_c(math.inf, 0.05, 0.11, tol=1e-9)
    points = []
    for c in (0.0, 0.02, 0.05, float(quality.C_MAXWELL), 0.123, 0.3, 1.0):
        d, e = quality.quality(math.inf, c)
        points.append({"c": c, "D": d, "dE_over_E": e})
    out = {"_about": "Maxwell limit of the approximation from oracle/quality.py (mpmath, 30 digits); "
                     "written by tests/golden/make_maxwell_golden.py.",
           "optimum_c": c_opt, "D_at_optimum": quality.quality(math.inf, c_opt)[0], "points": points}
    path = os.path.join(os.path.dirname(__file__), "maxwell_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
