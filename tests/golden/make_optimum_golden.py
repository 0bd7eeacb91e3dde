"""Writes optimum_c_oracle.json: the c that minimises the relative entropy
D(f||g; kappa, c) (eq:relative_entropy) at a few kappa where the minimum lies
inside the paper's range c in [0, 1.5] (Sec. 3, Fig. fig:map), by the
approximation-quality oracle's golden-section search at 30 digits.

Run from the repository root:  python tests/golden/make_optimum_golden.py
"""
import json
import os
import sys
from multiprocessing import Pool

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))
from oracle import quality  # noqa: E402

KAPPAS = [1.6, 2.0, 2.6, 3.0, 3.3, 5.0, 6.0, 8.0, 10.0]


def one(k):
    ca = float(quality.c_approx(k))
    lo, hi = max(0.0, ca - 0.1), ca + 0.1
    c = quality.optimum_c(k, lo, hi, tol=1e-10)
    return {"kappa": k, "bracket": [lo, hi], "optimum_c": c, "D_at_optimum": float(quality.relative_entropy(k, c)),
            "c_from_eq_c": ca}


def main():
    with Pool(6) as pool:
        rows = pool.map(one, KAPPAS)
    out = {"_about": "Minimiser of D(f||g; kappa, c) over c from oracle/quality.py (mpmath, 30 digits, "
                     "golden-section search); written by tests/golden/make_optimum_golden.py.",
           "points": rows}
    path = os.path.join(os.path.dirname(__file__), "optimum_c_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(json.dumps(out, indent=1))


if __name__ == "__main__":
    main()
