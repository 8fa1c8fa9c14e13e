"""The binary64 weight exp of the pair kernels (exp_tab in rwpt_pairstep.h):
its constants are checked against high-precision values, and the algorithm,
emulated with correctly rounded binary64 operations, against exp."""
import math
import os
import random
import re
from decimal import Decimal, getcontext
from fractions import Fraction

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "paper_1811_05474_amd", "csrc", "rwpt_pairstep.h")

getcontext().prec = 60


def _source():
    return open(HEADER).read()


def _table():
    body = re.search(r"kExp2Frac\[64\]\s*=\s*\{(.*?)\};", _source(), re.S).group(1)
    vals = [float.fromhex(v) for v in re.findall(r"0x[0-9a-fA-F.]+p[+-]\d+", body)]
    assert len(vals) == 64
    return vals


def _const(name):
    return float.fromhex(re.search(name + r"\s*=\s*(0x[0-9a-fA-F.]+p[+-]\d+)", _source()).group(1))


def _fma(a, b, c):
    return float(Fraction(a) * Fraction(b) + Fraction(c))  # one rounding, like the hardware FMA


def test_table_is_correctly_rounded_powers_of_two():
    for j, v in enumerate(_table()):
        exact = Decimal(2) ** (Decimal(j) / Decimal(64))
        assert v == float(Fraction(exact)), j


def test_reduction_constants():
    ln2 = Decimal(2).ln()
    hi, lo, inv = _const("kLn2_64Hi"), _const("kLn2_64Lo"), _const("kInvLn2_64")
    assert inv == float(Fraction(Decimal(64) / ln2))
    # the head has at most 32 significant bits, so t * head is exact for |t| < 2^21
    m, e = math.frexp(hi)
    assert (Fraction(m) * 2 ** 32).denominator == 1
    # head + tail = ln2/64 to within half an ulp of the tail
    assert abs(Fraction(hi) + Fraction(lo) - Fraction(ln2 / 64)) <= Fraction(math.ulp(lo)) / 2


def _exp_tab(x, tbl, hi, lo, inv):
    x = max(x, -1000.0)
    t = float(round(x * inv))  # round half to even, as rint
    r = _fma(-t, hi, x)
    r = _fma(-t, lo, r)
    k = int(t)
    p = 1.0 / 120.0
    for c in (1.0 / 24.0, 1.0 / 6.0, 0.5, 1.0):
        p = _fma(p, r, c)
    q = p * r
    f = tbl[k & 63]
    return math.ldexp(_fma(f, q, f), k >> 6)


def test_exp_tab_error_at_most_1p2_ulp():
    tbl, hi, lo, inv = _table(), _const("kLn2_64Hi"), _const("kLn2_64Lo"), _const("kInvLn2_64")
    rng = random.Random(5)
    # the weights' range (s^2 / sigma^2 <= kappa^2 = 9) and far below it
    xs = [-9.0 * rng.random() for _ in range(800)] + [-700.0 * rng.random() for _ in range(400)]
    xs += [0.0, -0.0, -9.0, -1e-300, -math.log(2) / 128, -700.0]
    worst = 0.0
    for x in xs:
        exact = Decimal(x).exp()
        got = _exp_tab(x, tbl, hi, lo, inv)
        err = abs(Decimal(got) - exact) / Decimal(math.ulp(float(exact)))
        worst = max(worst, float(err))
    assert worst <= 1.2, worst
    assert _exp_tab(0.0, tbl, hi, lo, inv) == 1.0
    assert _exp_tab(-2000.0, tbl, hi, lo, inv) == 0.0
