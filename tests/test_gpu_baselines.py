"""The same-GPU exact Kappa generators used as comparators (Sec. 5, Sec. 6).

They sample eq:kappa exactly, so their speeds pass a KS test against the exact
CDF of eq:CDF at any size; their mean loop counts match the acceptance rates
the paper prints: p1 of eq:mt_eff (Marsaglia-Tsang gamma inside the t form)
and p2 of eq:pareto_eff (Type II Pareto rejection), which pins the Pareto
proposal and acceptance test reconstructed from the paper's description.
"""
import json
import math
import os

import numpy as np
import pytest
import torch
from scipy import special, stats

import paper_2602_05606_amd as kp

pytestmark = pytest.mark.gpu

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_statements.json")))


def exact_cdf(x, k):
    return special.betainc(1.5, k - 0.5, x / (x + k))


def p1(k):
    """eq:mt_eff with shape k = kappa - 1/2."""
    return math.exp(k - 1 / 3 + special.gammaln(k) - 0.5 * math.log(2 * math.pi) - (k - 0.5) * math.log(k - 1 / 3))


def p2(kappa):
    """eq:pareto_eff."""
    return math.exp((1 + kappa / 2) * math.log(kappa) - math.log(2) - 0.5 * (kappa - 1) * math.log(kappa - 1)
                    + special.betaln(1.5, kappa - 0.5))


def test_acceptance_formulas_match_the_papers_ranges():
    g1, g2 = GOLD["mt_acceptance_range"], GOLD["pareto_acceptance_range"]
    assert abs(p1(1.5 + 1e-9 - 0.5) - g1["low"]) < 0.01 and abs(p1(1e4) - g1["high"]) < 0.01
    assert abs(p2(1.5 + 1e-9) - g2["high"]) < 0.01 and abs(p2(1e4) - g2["low"]) < 0.01


@pytest.mark.parametrize("which", ["t", "pareto"])
@pytest.mark.parametrize("kappa", [1.6, 3.0, 10.0])
@pytest.mark.parametrize("precision", [kp.FP32, kp.FP64])
def test_exact_generators(which, kappa, precision):
    n = 1_000_000
    fn = kp.sample_exact_t if which == "t" else kp.sample_exact_pareto
    vx, vy, vz, iters = fn(kappa, 1.3, n, 17, precision=precision, with_iters=True)
    torch.cuda.synchronize()
    v = np.stack([t.cpu().numpy().astype(np.float64) for t in (vx, vy, vz)])
    it = iters.cpu().numpy()
    x = (v ** 2).sum(0) / 1.3 ** 2
    p = stats.kstest(x, lambda t: exact_cdf(t, kappa)).pvalue
    cos_t = v[0] / np.sqrt((v ** 2).sum(0))
    pc = stats.kstest(cos_t, stats.uniform(loc=-1, scale=2).cdf).pvalue
    acc = p1(kappa - 0.5) if which == "t" else p2(kappa)
    mean_it = it.mean()
    sd = math.sqrt((1 - acc) / acc ** 2 / n)
    print(f"{which} kappa {kappa} prec {precision}: KS p {p:.3f}, iters {mean_it:.5f} vs 1/p {1 / acc:.5f}")
    assert p > 1e-4 and pc > 1e-4
    assert it.min() >= 1 and it.max() < 64
    assert abs(mean_it - 1 / acc) < 6 * sd


@pytest.mark.parametrize("which", ["t", "pareto"])
def test_wave_loop_counts_follow_the_geometric_model(which):
    """Sec. 6: a SIMT group waits for its slowest lane.  With independent
    Philox draws per iteration the loop counts are geometric with rejection
    rate rho = 1 - p, so the largest of t of them has mean
    sum_k 1 - (1 - rho^k)^t; checked for t = 64 (the wave) and 32."""
    kappa, n = 3.0, 1 << 22
    fn = kp.sample_exact_t if which == "t" else kp.sample_exact_pareto
    *_, it = fn(kappa, 1.0, n, 23, precision=kp.FP32, with_iters=True)
    it = it.to(torch.float64)
    rho = 1 - (p1(kappa - 0.5) if which == "t" else p2(kappa))
    k = np.arange(0, 400)
    for t in (32, 64):
        expect = float(np.sum(1 - (1 - rho ** k) ** t))
        got = it.view(-1, t).max(dim=1).values.mean().item()
        print(f"{which} t={t}: mean of group max {got:.4f}, geometric model {expect:.4f}")
        assert abs(got - expect) < 0.03
