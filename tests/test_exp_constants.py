"""The FP64 exponential of the Gaussian-sum march (a host check of its
formula; the kernel itself is held to the oracle by the FP64 parity tests).

e^x on [-32, 0] is taken by Cody-Waite reduction x = k ln2/64 + r with ln2/64
split into a 32-bit head and a tail, a degree-5 Taylor polynomial of e^r by
Horner, and the factor 2^(k >> 6) 2^((k & 63)/64) from a 64-entry table.
The constants are read from the kernel source; every fused multiply-add is
emulated with one exact rounding, the table entries are taken correctly
rounded (the kernel fills them with the device exp2, which adds its own
rounding), and the result is compared with a 50-digit exponential."""
import math
import os
import re
from decimal import Decimal, getcontext
from fractions import Fraction

import pytest

SRC = os.path.join(os.path.dirname(__file__), "..", "paper_2301_03814_amd", "csrc", "march.hip")


def constants():
    s = open(SRC).read()
    body = s[s.index("__device__ inline double exp_gauss(double x,"):]
    body = body[:body.index("return ldexp")]
    num = r"([0-9.eE+-]+)"
    inv = float(re.search(r"k64InvLn2 = " + num, body).group(1))
    head = float(re.search(r"kLn2Head = " + num, body).group(1))
    tail = float(re.search(r"kLn2Tail = " + num, body).group(1))
    arr = re.search(r"kC\[6\] = \{([^}]*)\}", body).group(1)
    coef = [float(t) for t in arr.replace("\n", " ").split(",") if t.strip()]
    return inv, head, tail, coef


def fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))


def exp_kernel(x, inv, head, tail, coef, table):
    kf = float(round(x * inv))  # rint: ties to even, as Python's round
    r = fma(-kf, head, x)
    r = fma(-kf, tail, r)
    p = coef[0]
    for c in coef[1:]:
        p = fma(p, r, c)
    k = int(kf)
    return math.ldexp(float(Fraction(table[k & 63]) * Fraction(p)), k >> 6)


def test_constants_are_the_exact_expansions():
    getcontext().prec = 60
    inv, head, tail, coef = constants()
    ln2_64 = Decimal(2).ln() / 64
    assert inv == float(1 / ln2_64)
    # head: at most 32 significant bits, so k * head is exact for |k| < 2^21
    m, _ = math.frexp(head)
    assert (Fraction(m) * 2 ** 32).denominator == 1
    assert tail == float(ln2_64 - Decimal(head))
    assert coef == [float(Fraction(1, math.factorial(k))) for k in range(5, -1, -1)]


@pytest.mark.parametrize("seed", [0, 1])
def test_relative_error_on_the_cutoff_range(seed):
    import random
    getcontext().prec = 50
    inv, head, tail, coef = constants()
    table = [float(Decimal(2) ** (Decimal(j) / 64)) for j in range(64)]
    rng = random.Random(seed)
    xs = [rng.uniform(-32.0, 0.0) for _ in range(1500)]
    xs += [0.0, -32.0, -math.log(2.0) / 128, -math.log(2.0) / 128 - 31.0, -1e-300]
    worst = 0.0
    for x in xs:
        e = Decimal(x).exp()
        worst = max(worst, float(abs((Decimal(exp_kernel(x, inv, head, tail, coef, table)) - e) / e)))
    assert worst <= 3.5e-16
