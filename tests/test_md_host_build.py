"""The GPU library's multiple-double header (csrc/md.hpp), compiled for the host, against the
oracle and exact rationals: the arithmetic the kernels run meets its accuracy contract
(normwise error a small multiple of 2^(-53P)) and normalises its outputs."""
import ctypes
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import mdgen


@pytest.fixture(scope="module")
def H():
    from paper_2110_08375_amd import build

    if not os.path.exists(build.HOSTLIB) or os.path.getmtime(build.HOSTLIB) < os.path.getmtime(
            os.path.join(build.CSRC, "md.hpp")):
        build.build_host_shim()
    L = ctypes.CDLL(build.HOSTLIB)
    dp = ctypes.POINTER(ctypes.c_double)
    L.mdh_op.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
    L.mdh_dot.argtypes = [ctypes.c_int, ctypes.c_int, dp, dp, dp, dp]
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def op(H, P, code, a, b, c=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    c = np.zeros(P) if c is None else np.ascontiguousarray(c, dtype=np.float64)
    r = np.zeros(P)
    assert H.mdh_op(P, code, _p(a), _p(b), _p(c), _p(r)) == 0
    return r


def F(x):
    return sum((Fraction(float(v)) for v in x), Fraction(0))


ADD, SUB, MUL, DIV, SQRT, FMA, RECIP, MULD = range(8)


def normalised(x):
    for k in range(len(x) - 1):
        if x[k] == 0.0:
            if x[k + 1] != 0.0:
                return False
        elif abs(x[k + 1]) > math.ulp(x[k]):
            return False
    return True


@pytest.mark.parametrize("P", (1, 2, 4, 8))
def test_ops_against_exact(H, P):
    eps = Fraction(2) ** (-53 * P)
    for t in range(60):
        a = mdgen.md_vector(P, 1, t, 1)[:, 0]
        b = mdgen.md_vector(P, 1, t, 2)[:, 0] * 2.0 ** ((t % 13) * 7 - 42)
        c = mdgen.md_vector(P, 1, t, 3)[:, 0]
        fa, fb, fc = F(a), F(b), F(c)
        checks = [
            (ADD, fa + fb, abs(fa) + abs(fb), 8),
            (SUB, fa - fb, abs(fa) + abs(fb), 8),
            (MUL, fa * fb, abs(fa * fb), 32),
            (DIV, fa / fb, abs(fa / fb), 128),
            (RECIP, 1 / fb, abs(1 / fb), 128),
            (FMA, fc + fa * fb, abs(fc) + abs(fa * fb), 64),
        ]
        for code, exact, scale, k in checks:
            r = op(H, P, code, a, b, c)
            assert abs(F(r) - exact) <= k * eps * scale, (P, code)
            assert normalised(r)
        r = op(H, P, MULD, a, np.array([b[0]] + [0.0] * (P - 1)))
        assert abs(F(r) - fa * Fraction(b[0])) <= 16 * eps * abs(fa * Fraction(b[0]))


@pytest.mark.parametrize("P", (2, 4, 8))
def test_sqrt_against_oracle(H, orc, P):
    for t in range(30):
        a = mdgen.md_vector(P, 1, t, 4)[:, 0] * 2.0 ** (t % 9 - 4)
        if a[0] < 0:
            a = -a
        g = op(H, P, SQRT, a, a)
        o = orc.md_sqrt(a)
        assert abs(F(g) - F(o)) <= Fraction(2) ** (8 - 53 * P) * F(o)
    assert np.all(op(H, P, SQRT, np.zeros(P), np.zeros(P)) == 0.0)


@pytest.mark.parametrize("P", (2, 4, 8))
def test_exact_cancellation(H, P):
    a = mdgen.md_vector(P, 1, 5, 1)[:, 0]
    b = a.copy()
    b[-1] *= 0.5
    r = op(H, P, SUB, a, b)
    assert F(r) == F(a) - F(b)
    assert np.all(op(H, P, ADD, a, -a) == 0.0)


@pytest.mark.parametrize("P", (2, 4, 8))
def test_lazy_dot_product_against_oracle(H, orc, P):
    """A long dot product accumulated as in the kernels (lazy level sums, periodic renormalisation)."""
    n = 300
    a = mdgen.md_vector(P, n, 9, 1)
    b = mdgen.md_vector(P, n, 9, 2)
    c = mdgen.md_vector(P, 1, 9, 3)[:, 0]
    r = np.zeros(P)
    aa = np.ascontiguousarray(a.T)
    bb = np.ascontiguousarray(b.T)
    assert H.mdh_dot(P, n, _p(aa), _p(bb), _p(np.ascontiguousarray(c)), _p(r)) == 0
    exact = F(c) + sum(F(a[:, i]) * F(b[:, i]) for i in range(n))
    scale = abs(F(c)) + sum(abs(F(a[:, i]) * F(b[:, i])) for i in range(n))
    assert abs(F(r) - exact) <= 64 * n * Fraction(2) ** (-53 * P) * scale
    assert normalised(r)


@pytest.mark.parametrize("P", (4, 8))
def test_newton_residual_after_exact_cancellation(H, P):
    """Regression: 1 - b y cancels its top levels exactly; the renormalised residual used to
    keep a zero limb between nonzero ones (or two overlapping limbs), and truncating it to
    P/2 limbs lost ~50 bits of the reciprocal.  Inputs found by sweeping seeds."""
    eps = Fraction(2) ** (-53 * P)
    worst = Fraction(0)
    for t in range(200):
        b = mdgen.md_vector(P, 1, t, 2)[:, 0] * 2.0 ** ((t % 13) * 7 - 42)
        r = op(H, P, RECIP, b, b)
        worst = max(worst, abs(F(r) * F(b) - 1))
        a = mdgen.md_vector(P, 1, t, 4)[:, 0]
        a = a if a[0] > 0 else -a
        s = op(H, P, SQRT, a, a)
        worst = max(worst, abs(F(s) ** 2 - F(a)) / F(a))
    assert worst <= 2 ** 12 * eps
    # the seed that exposed it (quad double)
    if P == 4:
        b = np.array([47.41589486320882, 2.6195326442484756e-15, -3.3598135411187007e-32, 1.1778734330149813e-48])
        assert abs(F(op(H, P, RECIP, b, b)) * F(b) - 1) <= 64 * eps
