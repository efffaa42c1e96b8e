"""Compile-time constants of the device numerics that are not written as
expressions, checked against their definitions: the Cody-Waite split of ln 2
used by the FP64 exponential (head with at most 42 significant bits, so that
k ln2_hi is exact for |k| < 2^11; head + tail = ln 2 to far below an ulp)."""
import decimal
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _constant(name):
    with open(os.path.join(ROOT, "paper_2207_01173_amd", "csrc", "hgks_numerics.hpp")) as f:
        text = f.read()
    m = re.search(rf"constexpr double {name} = (0x[0-9a-fA-Fp.+-]+);", text)
    assert m, name
    return float.fromhex(m.group(1))


def test_ln2_split():
    hi, lo = _constant("kLn2Hi"), _constant("kLn2Lo")
    decimal.getcontext().prec = 60
    ln2 = decimal.Decimal(2).ln()
    # the head's significand has at most 42 bits
    m = decimal.Decimal(hi) * (2 ** 42)
    assert m == m.to_integral_value() and 2 ** 41 <= m < 2 ** 42
    err = abs(decimal.Decimal(hi) + decimal.Decimal(lo) - ln2)
    assert err < decimal.Decimal(2) ** -100
    # the tail is the remainder rounded to double
    assert lo == float(ln2 - decimal.Decimal(hi))
