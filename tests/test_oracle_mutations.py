"""The oracle's pins catch plausible mistakes.

Each case copies oracle/kappa_oracle.c, plants one mistake (a wrong sign, a
dropped or altered term, a swapped operand, a wrong index or constant),
builds the copy, and runs the oracle pin tests against it.  The pins must
fail for every mutant.  Mistakes are planted only in the copy, on the CPU.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "kappa_oracle.c")
PIN_TESTS = ["tests/test_oracle_philox.py", "tests/test_oracle_setup.py", "tests/test_oracle_sampler.py"]

MUTANTS = {
    "root_sign": ("(D - A) / (2.0 * b)", "(D + A) / (2.0 * b)"),
    "discriminant_term": ("A * A - 4.0 * b * L", "A * A - 2.0 * b * L"),
    "power_two_thirds": ("exp((2.0 / 3.0) * log(u))", "exp((3.0 / 2.0) * log(u))"),
    "c_denominator_constant": ("7.89 * kappa", "7.98 * kappa"),
    "kappa_star": ("double ks = kappa - 0.5;", "double ks = kappa - 0.45;"),
    "beta_argument": ("lgamma(kappa + 1.0)", "lgamma(kappa + 0.5)"),
    "b_exponent": ("exp(ln_inner / ks)", "exp(ln_inner / kappa)"),
    "direction_swap": ("v[1] = V * sin_t * cos(phi)", "v[1] = V * sin_t * sin(phi)"),
    "philox_key_word": ("hi_b ^ x1 ^ k0", "hi_b ^ x1 ^ k1"),
    "philox_weyl": ("k1 += PHILOX_WEYL_B;", "k1 += PHILOX_WEYL_A;"),
    "uniform_scale": ("*u = ldexp((double)(2 * m53 + 1), -54);", "*u = ldexp((double)(2 * m53 + 1), -53);"),
    "azimuth_word": ("double phi = 2.0 * M_PI * azimuth_uniform(r[2]);\n    v[0]", "double phi = 2.0 * M_PI * azimuth_uniform(r[1]);\n    v[0]"),
    "tail_threshold": ("return mode == MODE_FP32 && r0 >= 0xFFFFF000u;", "return mode == MODE_FP32 && r0 >= 0xFFFFE000u;"),
    "fp64_word_order": ("((((uint64_t)r0) << 32) | (uint64_t)r3)", "((((uint64_t)r3) << 32) | (uint64_t)r0)"),
    "adjoint_L_term": ("(da + dc * L + c * dL)", "(da + dc * L + dc * dL)"),
    "adjoint_a_derivative": ("a * (-1.0 / kappa - (2.0 / 3.0) * dlnB)", "a * (-1.0 / kappa + (2.0 / 3.0) * dlnB)"),
    "G_power": ("*G = exp(1.5 * log(inner));", "*G = exp(1.25 * log(inner));"),
    "high_side_log": ("lT = log(-expm1((2.0 / 3.0) * lnU1));", "lT = log(-expm1((2.0 / 3.0) * lnU1)) * 1.0000001;"),
}


@pytest.mark.slow
@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_fail_on_mutant(tmp_path, name):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not unique"
    mutant_c = tmp_path / "mutant.c"
    mutant_c.write_text(src.replace(old, new))
    lib = tmp_path / "libmutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-ffp-contract=off", "-fopenmp", "-fPIC",
                    "-shared", "-o", str(lib), str(mutant_c), "-lm"], check=True)
    env = dict(os.environ, KAPPA_ORACLE_LIB=str(lib), OMP_NUM_THREADS="4")
    res = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *PIN_TESTS],
                         cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert res.returncode != 0, f"mutant {name} passed every pin:\n{res.stdout[-2000:]}"
