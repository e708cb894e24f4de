"""Correctly rounded elementary functions (reading R33), on the CPU.

The oracle's cr_log / cr_exp / cr_pow (Python decimal at 60 digits) are
pinned against facts outside them: exact special values, the libm results
they may differ from by at most one unit in the last place, the identities
ln(2^k) = k ln 2 and x^1 = x, and their monotonicity. The library's
double-double versions (csrc/crmath.h, the code both the host table and
the kernels run) are compiled here with g++ and must give the same bits as
the oracle's on every sampled argument, including every step-rule factor
(j+1)^-0.3 and (j+1)^-0.6 for j up to 8192.
"""

import math
import os
import random
import subprocess

import numpy as np
import pytest

from oracle.crmath import cr_exp, cr_log, cr_pow

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2506_17650_amd", "csrc")


def ulps(a, b):
    return abs(int(np.float64(a).view(np.int64)) - int(np.float64(b).view(np.int64)))


def test_oracle_special_values():
    assert cr_log(1.0) == 0.0 and cr_exp(0.0) == 1.0
    assert cr_pow(7.0, 1.0) == 7.0 and cr_pow(2.0, 10.0) == 1024.0 and cr_pow(9.0, 0.5) == 3.0
    assert cr_pow(5.0, 0.0) == 1.0
    # ln 2 to 21 digits (a mathematical constant): the double nearest it
    assert cr_log(2.0) == 0.6931471805599453
    assert cr_exp(1.0) == 2.718281828459045


def test_oracle_within_one_ulp_of_libm_and_monotone():
    rng = random.Random(7)
    xs = sorted(math.exp(rng.uniform(-40, 40)) for _ in range(500))
    logs = [cr_log(x) for x in xs]
    assert all(ulps(cr, math.log(x)) <= 1 for cr, x in zip(logs, xs))
    assert all(a <= b for a, b in zip(logs, logs[1:]))
    es = sorted(rng.uniform(-60, 60) for _ in range(500))
    exps = [cr_exp(a) for a in es]
    assert all(ulps(cr, math.exp(a)) <= 1 for cr, a in zip(exps, es))
    assert all(a <= b for a, b in zip(exps, exps[1:]))
    for j in range(1, 400):
        assert ulps(cr_pow(j + 1.0, -0.3), (j + 1.0) ** -0.3) <= 1


def test_oracle_log_of_powers_of_two():
    # ln(2^k) = k ln 2: the double nearest k times a 40-digit ln 2
    from decimal import Decimal, localcontext
    with localcontext() as ctx:
        ctx.prec = 50
        ln2 = Decimal("0.6931471805599453094172321214581765680755001343602552")
        for k in list(range(-60, 61)) + [-1000, 1000]:
            assert cr_log(2.0 ** k) == float(ln2 * k), k


@pytest.fixture(scope="module")
def lib_driver(tmp_path_factory):
    src = tmp_path_factory.mktemp("crm") / "drv.cpp"
    src.write_text(
        '#include <cstdio>\n#include "crmath.h"\nusing namespace opdhg::crm;\n'
        'int main() { char op; double a, b;\n'
        '  while (scanf(" %c %la %la", &op, &a, &b) == 3)\n'
        "    printf(\"%a\\n\", op == 'l' ? cr_log(a) : op == 'e' ? cr_exp(a) : cr_pow(a, b));\n"
        "}\n")
    exe = src.parent / "drv"
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-I", CSRC, str(src), "-o",
                    str(exe)], check=True)
    return str(exe)


def test_library_double_double_matches_oracle(lib_driver):
    rng = random.Random(11)
    cases = [("l", math.exp(rng.uniform(-30, 30)), 0.0) for _ in range(3000)]
    cases += [("e", rng.uniform(-50, 50), 0.0) for _ in range(3000)]
    cases += [("p", j + 1.0, e) for j in range(1, 8193) for e in (-0.3, -0.6)]
    cases += [("p", math.exp(rng.uniform(-5, 5)), rng.uniform(-2, 2)) for _ in range(1000)]
    # the primal-weight update's arguments: ratios of norms and weights near 1
    cases += [("l", rng.uniform(0.01, 100.0), 0.0) for _ in range(1000)]
    inp = "".join(f"{o} {a.hex()} {b.hex()}\n" for o, a, b in cases)
    out = subprocess.run([lib_driver], input=inp, capture_output=True, text=True,
                         check=True).stdout.split()
    assert len(out) == len(cases)
    bad = []
    for (o, a, b), r in zip(cases, out):
        want = cr_log(a) if o == "l" else cr_exp(a) if o == "e" else cr_pow(a, b)
        if float.fromhex(r) != want:
            bad.append((o, a, b, r, want))
    assert not bad, bad[:5]
