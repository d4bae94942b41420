"""The seeded input generator: vectorised backends agree bit for bit with the scalar
definition, limbs are non-overlapping by construction, and the recipes have the stated
structure."""
import math

import numpy as np
import pytest

import mdgen


def test_uniform_matches_scalar_definition():
    v = mdgen.uniform(12345, 3, 50, k0=7)
    for i in range(50):
        assert v[i] == mdgen.uniform_scalar(12345, 3, 7 + i)
    assert np.all(v >= -1.0) and np.all(v < 1.0)


def test_torch_backend_bit_identical():
    torch = pytest.importorskip("torch")
    for P in (1, 2, 4, 8):
        a = mdgen.md_uniform(P, 33, 17, 99, mdgen.STREAM_A)
        t = mdgen.md_uniform(P, 33, 17, 99, mdgen.STREAM_A, device="cpu").numpy()
        assert np.array_equal(a, t)
    U = mdgen.upper_triangular(4, 20, 5, well_conditioned=True)
    Ut = mdgen.upper_triangular(4, 20, 5, well_conditioned=True, device="cpu").numpy()
    assert np.array_equal(U, Ut)


@pytest.mark.parametrize("P", (2, 4, 8))
def test_limbs_nonoverlapping(P):
    a = mdgen.md_uniform(P, 64, 64, 1, mdgen.STREAM_A).reshape(P, -1)
    for k in range(1, P):
        hi, lo = a[k - 1], a[k]
        nz = hi != 0
        ulp = np.array([math.ulp(x) for x in hi[nz]])
        assert np.all(np.abs(lo[nz]) <= ulp / 2)
        assert np.all(lo[~nz] == 0.0)


def test_upper_triangular_structure():
    n = 40
    U = mdgen.upper_triangular(2, n, 3)
    lead = U[0].T  # rows x cols
    assert np.all(np.tril(lead, -1) == 0.0)
    d = np.diag(lead)
    assert np.all((d >= 1.0) & (d <= 2.0))
    W = mdgen.upper_triangular(2, n, 3, well_conditioned=True)
    off = np.triu(W[0].T, 1)
    assert np.max(np.abs(off)) <= 2.0 ** -math.ceil(math.log2(n))


def test_batch_shapes_ranges():
    sh = mdgen.batch_shapes(512, 4)
    assert len(sh) == 512
    for m, n in sh:
        assert 32 <= m <= 512 and 16 <= n <= m


def test_upper_triangular_exact_rhs_is_exact():
    """b = R * ones holds exactly (rational check), with the numpy and torch backends equal."""
    from fractions import Fraction

    import torch

    for n in (5, 40, 129):
        R, b = mdgen.upper_triangular_exact(4, n, 7)
        assert np.all(R[1:] == 0.0) and np.all(b[1:] == 0.0)
        for row in range(n):
            exact = sum(Fraction(float(R[0, col, row])) for col in range(n))
            assert Fraction(float(b[0, row])) == exact
        assert np.all(np.diag(R[0]) >= 1.0) and np.all(np.diag(R[0]) <= 2.0)
        assert np.all(np.tril(R[0].T, -1) == 0.0)
        Rt, bt = mdgen.upper_triangular_exact(4, n, 7, device="cpu")
        assert np.array_equal(Rt.numpy(), R) and np.array_equal(bt.numpy(), b)


def test_conditioned_matrix_has_requested_kappa():
    A = mdgen.conditioned(2, 120, 80, 3, kappa=1e6)
    assert A.shape == (2, 80, 120)
    s = np.linalg.svd(A[0].T, compute_uv=False)
    assert abs(s[0] - 1.0) < 1e-9 and abs(s[-1] / 1e-6 - 1.0) < 1e-6
    assert np.all(np.abs(A[1]) <= np.spacing(np.abs(A[0])))


def test_conditioned_exact_rhs_is_exact():
    """b = A x_true of the exact-rhs precision-form input, checked in exact rationals; kappa
    stays at the requested 1e8 after the rounding of A."""
    from fractions import Fraction

    m, n = 96, 64
    A, x, b = mdgen.conditioned_exact(4, m, n, 5)
    assert np.all(A[1:] == 0) and np.all(x[1:] == 0) and np.all(b[2:] == 0)
    for i in range(m):
        S = sum(Fraction(float(A[0, j, i])) * Fraction(float(x[0, j])) for j in range(n))
        assert S == Fraction(float(b[0, i])) + Fraction(float(b[1, i])), i
        assert abs(b[1, i]) <= abs(np.spacing(b[0, i]))  # two non-overlapping limbs
    k = np.linalg.cond(A[0].T)
    assert 0.9e8 < k < 1.1e8
