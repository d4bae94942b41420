"""Pins of the oracle's multiple-double arithmetic (paper Section 1.1, Table 1) against
exact rational arithmetic (``fractions.Fraction`` on the dyadic limbs) and mpmath at
high precision.  A dropped limb, a sign slip or a wrong carry makes these fail."""
import math
from fractions import Fraction

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import mdgen

PS = (1, 2, 4, 8, 16)


def F(x):
    return sum((Fraction(float(v)) for v in x), Fraction(0))


def bound(P):
    # each limb is within one ulp of the remaining value: relative error < 2^(1-52P)
    return Fraction(2) ** (1 - 52 * P)


def rel(got, exact):
    if exact == 0:
        return abs(got)
    return abs(got - exact) / abs(exact)


def md_sample(P, seed, stream, scale_exp=0):
    a = mdgen.md_vector(P, 1, seed, stream)[:, 0]
    return a * 2.0 ** scale_exp


def check_normal(x):
    """Limbs decrease: |x_{k+1}| <= ulp(x_k) (zeros only at the tail)."""
    seen_zero = False
    for k in range(len(x) - 1):
        if x[k] == 0.0:
            seen_zero = True
        if seen_zero:
            assert x[k + 1] == 0.0
        else:
            assert abs(x[k + 1]) <= math.ulp(x[k])


@pytest.mark.parametrize("P", PS)
def test_ops_exact_rational(orc, P):
    for t in range(40):
        a = md_sample(P, t, 1)
        b = md_sample(P, t, 2, scale_exp=(t % 11) * 9 - 45)
        fa, fb = F(a), F(b)
        cases = [
            (orc.md_add(a, b), fa + fb),
            (orc.md_sub(a, b), fa - fb),
            (orc.md_mul(a, b), fa * fb),
            (orc.md_div(a, b), fa / fb),
        ]
        for got, exact in cases:
            assert rel(F(got), exact) < bound(P)
            check_normal(got)


@pytest.mark.parametrize("P", PS)
def test_sqrt_mpmath(orc, P):
    import mpmath

    with mpmath.workprec(60 * P + 200):
        for t in range(15):
            a = md_sample(P, t, 3, scale_exp=(t % 5) * 40 - 80)
            if a[0] < 0:
                a = -a
            r = orc.md_sqrt(a)
            exact = mpmath.sqrt(mpmath.mpf(F(a).numerator) / F(a).denominator)
            got = mpmath.mpf(F(r).numerator) / F(r).denominator
            assert abs(got - exact) / exact < mpmath.mpf(2) ** (1 - 52 * P)
            check_normal(r)


@pytest.mark.parametrize("P", (2, 4, 8))
def test_catastrophic_cancellation(orc, P):
    # a - b where the leading limbs cancel exactly: the result is the (exact) lower part
    a = md_sample(P, 7, 1)
    b = a.copy()
    b[-1] = b[-1] * 0.5 if b[-1] != 0 else 2.0 ** -300
    got = orc.md_sub(a, b)
    assert F(got) == F(a) - F(b)
    # x + (-x) is exactly zero
    assert np.all(orc.md_add(a, -a) == 0.0)


@pytest.mark.parametrize("P", (2, 4, 8))
def test_special_values(orc, P):
    one = np.zeros(P); one[0] = 1.0
    two = np.zeros(P); two[0] = 2.0
    z = np.zeros(P)
    assert F(orc.md_add(one, one)) == 2
    assert F(orc.md_mul(two, two)) == 4
    assert F(orc.md_div(one, two)) == Fraction(1, 2)
    assert np.all(orc.md_mul(z, two) == 0.0)
    assert np.all(orc.md_sqrt(z) == 0.0)
    four = np.zeros(P); four[0] = 4.0
    assert F(orc.md_sqrt(four)) == 2
    # 1/3 to P limbs: error below the bound, and 3 * (1/3) rounds back close to 1
    three = np.zeros(P); three[0] = 3.0
    third = orc.md_div(one, three)
    assert rel(F(third), Fraction(1, 3)) < bound(P)
    # exponent extremes (far from under/overflow of the lowest limb)
    big = one * 2.0 ** 600
    small = one * 2.0 ** -600
    assert F(orc.md_mul(big, small)) == 1
    # gap: 1 + 2^-200 is representable in P >= 4 limbs exactly
    gap = orc.md_round(P, [1.0, 2.0 ** -200])
    if P >= 4:
        assert F(gap) == 1 + Fraction(2) ** -200


@settings(max_examples=150, deadline=None)
@given(
    st.integers(min_value=0, max_value=2**31),
    st.sampled_from((2, 4, 8)),
    st.integers(min_value=-300, max_value=300),
    st.sampled_from(("add", "sub", "mul", "div")),
)
def test_ops_hypothesis(orc, seed, P, e, op):
    a = md_sample(P, seed, 1)
    b = md_sample(P, seed, 2, scale_exp=e)
    if b[0] == 0.0:
        return
    fn = {"add": orc.md_add, "sub": orc.md_sub, "mul": orc.md_mul, "div": orc.md_div}[op]
    exact = {"add": F(a) + F(b), "sub": F(a) - F(b), "mul": F(a) * F(b), "div": F(a) / F(b)}[op]
    assert rel(F(fn(a, b)), exact) < bound(P)


@settings(max_examples=60, deadline=None)
@given(st.lists(st.floats(min_value=-1e30, max_value=1e30, allow_nan=False), min_size=1, max_size=40),
       st.sampled_from((1, 2, 4, 8)))
def test_round_exact_sum(orc, terms, P):
    r = orc.md_round(P, terms)
    exact = sum((Fraction(t) for t in terms), Fraction(0))
    assert rel(F(r), exact) < bound(P)


def test_precision_levels(orc):
    """Section 1.1: P doubles give about 16P decimal places; 1/3 in dd/qd/od shows it."""
    for P, digits in ((2, 31), (4, 62), (8, 125)):
        one = np.zeros(P); one[0] = 1.0
        three = np.zeros(P); three[0] = 3.0
        err = abs(F(orc.md_div(one, three)) - Fraction(1, 3))
        assert err < Fraction(1, 10 ** digits)
