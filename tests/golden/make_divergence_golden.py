"""Writes divergence_oracle.json: the approximation-quality oracle's relative
entropy D(f||g; kappa, c) (eq:relative_entropy) and energy error (Fig.
fig:DE(b)) at a fixed set of (kappa, c) points, for the GPU parity tests.

Calls only oracle/quality.py.  Run from the repository root:
    python tests/golden/make_divergence_golden.py
"""
import json
import os
import sys
from multiprocessing import Pool

sys.path.insert(0, os.path.abspath(os.path.join(os.path.dirname(__file__), "..", "..")))
from oracle import quality  # noqa: E402

KAPPAS = [1.51, 1.6, 2.0, 2.6, 3.0, 3.9, 4.1, 4.2, 5.0, 7.5, 10.0, 15.0, 30.0]
CS = [0.0, 0.02, 0.3, 1.0, 1.5, 4.0, None]  # None: c from eq:c


def one(point):
    k, c = point
    d = float(quality.relative_entropy(k, c))
    # With c = 0 the tails of f and g differ by a constant factor, so the energy
    # integrand decays like x^(1/2 - kappa); next to kappa = 3/2 its integral is
    # not settled below x = 1e300 and no value is stored.
    e = None if (c == 0.0 and k < 1.55) else float(quality.energy_error(k, c))
    cval = float(quality.c_approx(k)) if c is None else c
    return {"kappa": k, "c": cval, "c_from_eq_c": c is None, "D": d, "dE_over_E": e}


def main():
    points = [(k, c) for k in KAPPAS for c in CS]
    with Pool(6) as pool:
        rows = pool.map(one, points)
    out = {
        "_about": "Relative entropy D(f||g; kappa, c) of eq:relative_entropy and energy error "
                  "(E_approx - E_kappa)/E_kappa (Fig. fig:DE(b), eq:kappaE) from oracle/quality.py "
                  "(mpmath, 30 digits). Written by tests/golden/make_divergence_golden.py.",
        "points": rows,
    }
    path = os.path.join(os.path.dirname(__file__), "divergence_oracle.json")
    with open(path, "w") as fh:
        json.dump(out, fh, indent=1)
    print(f"wrote {len(rows)} points to {path}")


if __name__ == "__main__":
    main()
