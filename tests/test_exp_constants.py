"""The FP64 exponential of the Gaussian-sum march (a host check of its
formula; the kernel itself is held to the oracle by the FP64 parity tests).

e^x on [-32, 0] is taken by Cody-Waite reduction x = n ln2 + r with ln2 split
into a 32-bit head and a tail, and a degree-12 Taylor polynomial of e^r by
Horner.  The constants are read from the kernel source; every fused
multiply-add is emulated with one exact rounding, and the result is compared
with a 50-digit exponential."""
import math
import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction

import pytest

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2301_03814_amd", "csrc", "march.hip")


def constants():
    s = open(SRC).read()
    body = s[s.index("__device__ inline double bump_exp<double>(double x) {"):]
    body = body[:body.index("return ldexp")]
    num = r"([0-9.eE+-]+)"
    inv = float(re.search(r"kInvLn2 = " + num, body).group(1))
    head = float(re.search(r"kLn2Head = " + num, body).group(1))
    tail = float(re.search(r"kLn2Tail = " + num, body).group(1))
    arr = re.search(r"kC\[13\] = \{([^}]*)\}", body).group(1)
    coef = [float(t) for t in arr.replace("\n", " ").split(",") if t.strip()]
    return inv, head, tail, coef


def fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def exp_kernel(x, inv, head, tail, coef):
    n = float(round(x * inv))
    r = fma(-n, head, x)
    r = fma(-n, tail, r)
    p = coef[0]
    for c in coef[1:]:
        p = fma(p, r, c)
    return math.ldexp(p, int(n))


def test_constants_are_the_exact_expansions():
    getcontext().prec = 60
    inv, head, tail, coef = constants()
    ln2 = Decimal(2).ln()
    assert inv == float(1 / ln2)
    # head: at most 32 significant bits, so n * head is exact for |n| < 2^21
    m, _ = math.frexp(head)
    assert (Fraction(m) * 2 ** 32).denominator == 1
    assert tail == float(ln2 - Decimal(head))
    assert coef == [float(Fraction(1, math.factorial(k))) for k in range(12, -1, -1)]


@pytest.mark.parametrize("seed", [0, 1])
def test_relative_error_on_the_cutoff_range(seed):
    import random
    getcontext().prec = 50
    inv, head, tail, coef = constants()
    rng = random.Random(seed)
    xs = [rng.uniform(-32.0, 0.0) for _ in range(1500)]
    xs += [0.0, -32.0, -0.5 * math.log(2.0), 0.5 * math.log(2.0) - 32.0, -1e-300]
    worst = 0.0
    for x in xs:
        e = Decimal(x).exp()
        worst = max(worst, float(abs((Decimal(exp_kernel(x, inv, head, tail, coef)) - e) / e)))
    assert worst <= 3.5e-16
