"""The SIMT cost model of Sec. 6 as the benchmark evaluates it (bench.py):
acceptance rates eq:mt_eff and eq:pareto_eff against the ranges the paper
prints, and Ridley's loop counts eq:ridley1 / eq:ridley2 against brute-force
statistics of the largest of t geometric loop counts."""
import json
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

GOLD = json.load(open(os.path.join(ROOT, "tests", "golden", "paper_statements.json")))


def test_acceptance_ranges():
    ks = np.concatenate([[1.5 + 1e-6], np.linspace(1.6, 200, 400)])
    p1 = np.array([bench.mt_acceptance(k) for k in ks])
    p2 = np.array([bench.pareto_acceptance(k) for k in ks])
    r1, r2 = GOLD["mt_acceptance_range"], GOLD["pareto_acceptance_range"]
    assert abs(p1[0] - r1["low"]) < 0.005 and abs(p1[-1] - r1["high"]) < 0.005
    assert np.all(np.diff(p1) > 0)
    assert abs(p2[0] - r2["high"]) < 0.005 and abs(p2[-1] - r2["low"]) < 0.005
    assert np.all(np.diff(p2) < 0)
    # the rejection rate 1 - p2 spans the range Sec. 6 prints
    r3 = GOLD["pareto_rejection_range"]
    assert abs((1 - p2[0]) - r3["low"]) < 0.005 and abs((1 - p2[-1]) - r3["high"]) < 0.005


def _max_of_geometric(rho, t, kmax=400):
    """Mean and mode of the largest of t i.i.d. loop counts with P(count > k) = rho^k."""
    k = np.arange(0, kmax)
    mean = np.sum(1 - (1 - rho ** k) ** t)
    m = np.arange(1, kmax)
    pm = np.diff(np.concatenate([[0.0], (1 - rho ** m) ** t]))
    return mean, int(m[np.argmax(pm)])


def test_threshold_t32():
    assert abs((2 ** (1 / 32) - 1) - GOLD["ridley_threshold_t32"]["approx"]) < 0.0005


@pytest.mark.parametrize("t", [32, 64])
def test_mu1_is_the_head_of_the_mean(t):
    for rho in (0.005, 0.02, 0.05):
        mean, _ = _max_of_geometric(rho, t)
        # eq:ridley1 keeps the k = 0, 1, 2 terms of sum_k P(max > k)
        assert 0 <= mean - bench.ridley_mu1(rho, t) < t * rho ** 3 / (1 - rho)


@pytest.mark.parametrize("t", [32, 64])
def test_mu2_tracks_the_largest_count(t):
    for rho in (0.19, 0.23, 0.27):
        mean, mode = _max_of_geometric(rho, t)
        mu = bench.ridley_mu2(rho, t)
        assert abs(mu - mean) < 0.2
        assert abs(mu - mode) < 1.3
