"""Pins of the oracle's complex least-squares path (paper Section 3: on complex data the
transpose of Algorithm 2 becomes the Hermitian transpose; Section 2, end: real and imaginary
parts in separate arrays; Section 4, Table 5: complex double double QR).  Every check is
against something the mathematics fixes: exact complex rational arithmetic, the exact
normal-equation solution, unitarity of Q and Q R = A, the modulus and phase of R(0,0), the
real oracle on real data, exact equivariance under multiplication by i, and LAPACK at P = 1.
"""
from fractions import Fraction

import numpy as np
import pytest

import mdgen


def F(x):
    return sum((Fraction(float(v)) for v in x), Fraction(0))


def u(P):
    return 2.0 ** (-(52 * P + 1))


def cf(Z, *idx):
    """Exact complex value of entry idx of a complex md array (2, P, ...)."""
    return (F(Z[(0, slice(None)) + idx]), F(Z[(1, slice(None)) + idx]))


def cmul(a, b):
    return (a[0] * b[0] - a[1] * b[1], a[0] * b[1] + a[1] * b[0])


def cconj(a):
    return (a[0], -a[1])


def cadd(a, b):
    return (a[0] + b[0], a[1] + b[1])


def csub(a, b):
    return (a[0] - b[0], a[1] - b[1])


def cdiv(a, b):
    d = b[0] * b[0] + b[1] * b[1]
    n = cmul(a, cconj(b))
    return (n[0] / d, n[1] / d)


def cabs(a):
    return abs(complex(float(a[0]), float(a[1])))


def cmat(A):
    """(2, P, n, m) -> m x n list of exact complex pairs."""
    _, P, n, m = A.shape
    return [[cf(A, j, i) for j in range(n)] for i in range(m)]


def cvec(x):
    return [cf(x, i) for i in range(x.shape[2])]


def to_np(A):
    """Leading limbs as a numpy complex matrix (m x n)."""
    return A[0, 0].T + 1j * A[1, 0].T


def kappa(A):
    return float(np.linalg.cond(to_np(A)))


def solve_exact(M, r):
    """Gaussian elimination in exact complex rationals (M Hermitian positive definite)."""
    n = len(M)
    M = [row[:] + [r[i]] for i, row in enumerate(M)]
    for k in range(n):
        piv = M[k][k]
        for i in range(k + 1, n):
            f = cdiv(M[i][k], piv)
            for j in range(k, n + 1):
                M[i][j] = csub(M[i][j], cmul(f, M[k][j]))
    x = [(Fraction(0), Fraction(0))] * n
    for i in range(n - 1, -1, -1):
        s = M[i][n]
        for j in range(i + 1, n):
            s = csub(s, cmul(M[i][j], x[j]))
        x[i] = cdiv(s, M[i][i])
    return x


def cnorm(v):
    return float(np.sqrt(sum(float(a[0]) ** 2 + float(a[1]) ** 2 for a in v)))


# ------------------------------------------------------------------------------ scalars
@pytest.mark.parametrize("P", (1, 2, 4, 8))
def test_complex_mul_div_exact(orc, P):
    """Complex product and quotient against exact rational arithmetic."""
    a_all = mdgen.cmd_uniform(P, 40, 1, 3 + P, mdgen.STREAM_A)
    b_all = mdgen.cmd_uniform(P, 40, 1, 3 + P, mdgen.STREAM_B)
    for i in range(40):
        a = np.ascontiguousarray(a_all[:, :, 0, i])
        b = np.ascontiguousarray(b_all[:, :, 0, i])
        ea, eb = cf(a_all, 0, i), cf(b_all, 0, i)
        p = orc.cmd_mul(a, b)
        want = cmul(ea, eb)
        got = (F(p[0]), F(p[1]))
        scale = cabs(ea) * cabs(eb)
        for k in range(2):
            assert abs(float(got[k] - want[k])) <= 4 * u(P) * scale
        q = orc.cmd_div(a, b)
        want = cdiv(ea, eb)
        got = (F(q[0]), F(q[1]))
        scale = cabs(ea) / cabs(eb)
        for k in range(2):
            assert abs(float(got[k] - want[k])) <= 16 * u(P) * scale


# ------------------------------------------------------------------------------ least squares
@pytest.mark.parametrize("P,m,n", [(2, 6, 4), (2, 5, 5), (4, 7, 5), (8, 5, 3)])
def test_x_matches_exact_rational_lstsq(orc, P, m, n):
    """x equals the exact solution of A^H A x = A^H b within kappa * u."""
    A, _ = mdgen.cls_problem(P, m, n, 21 + m)
    b = mdgen.cmd_vector(P, m, 21 + m, mdgen.STREAM_B)
    r = orc.clstsq(A, b)
    assert r["info"] == 0
    Ae, be = cmat(A), cvec(b)
    G = [[(Fraction(0), Fraction(0))] * n for _ in range(n)]
    for i in range(n):
        for j in range(n):
            s = (Fraction(0), Fraction(0))
            for k in range(m):
                s = cadd(s, cmul(cconj(Ae[k][i]), Ae[k][j]))
            G[i][j] = s
    rhs = []
    for i in range(n):
        s = (Fraction(0), Fraction(0))
        for k in range(m):
            s = cadd(s, cmul(cconj(Ae[k][i]), be[k]))
        rhs.append(s)
    xs = solve_exact(G, rhs)
    got = cvec(r["x"])
    err = cnorm([csub(g, w) for g, w in zip(got, xs)])
    k = kappa(A)
    assert err <= 200 * n * k * k * u(P) * max(1.0, cnorm(xs))


@pytest.mark.parametrize("P,m,n", [(2, 7, 5), (4, 6, 6), (8, 5, 3)])
def test_q_unitary_and_qr_is_a(orc, P, m, n):
    """Q^H Q = I and Q R = A, exactly evaluated on the computed factors."""
    A = mdgen.cmd_uniform(P, m, n, 31 + m, mdgen.STREAM_A)
    Fq, beta = orc.cqr(A)
    Q = orc.cexplicit_q(Fq, beta)
    Qe = cmat(Q)
    for i in range(m):
        for j in range(m):
            s = (Fraction(0), Fraction(0))
            for k in range(m):
                s = cadd(s, cmul(cconj(Qe[k][i]), Qe[k][j]))
            want = (Fraction(1 if i == j else 0), Fraction(0))
            assert cabs(csub(s, want)) <= 40 * m * u(P)
    Fe, Ae = cmat(Fq), cmat(A)
    anorm = float(np.linalg.norm(to_np(A), 2))
    for i in range(m):
        for j in range(n):
            s = (Fraction(0), Fraction(0))
            for k in range(min(j, m - 1) + 1):  # R is upper triangular
                s = cadd(s, cmul(Qe[i][k], Fe[k][j]))
            assert cabs(csub(s, Ae[i][j])) <= 40 * m * n * u(P) * anorm


@pytest.mark.parametrize("P,m,n", [(2, 9, 4), (4, 6, 3), (8, 5, 2)])
def test_first_diagonal_modulus_and_phase(orc, P, m, n):
    """R(0,0) = e^{i theta} ||A(:,0)|| with theta the phase of A(0,0) (the reflector
    maps x to e^{i theta} mu e_1: Golub-Van Loan 5.1.1 on |x1|, rotated by x1's phase)."""
    import mpmath

    A = mdgen.cmd_uniform(P, m, n, 41 + m, mdgen.STREAM_A)
    Fq, _ = orc.cqr(A)
    with mpmath.workprec(60 * P + 200):
        col = [cf(A, 0, i) for i in range(m)]
        nrm2 = sum(a[0] * a[0] + a[1] * a[1] for a in col)
        mu = mpmath.sqrt(mpmath.mpf(nrm2.numerator) / nrm2.denominator)
        a0 = col[0]
        r0 = mpmath.sqrt(mpmath.mpf((a0[0] ** 2 + a0[1] ** 2).numerator) / (a0[0] ** 2 + a0[1] ** 2).denominator)
        want_re = mpmath.mpf(a0[0].numerator) / a0[0].denominator / r0 * mu
        want_im = mpmath.mpf(a0[1].numerator) / a0[1].denominator / r0 * mu
        got = cf(Fq, 0, 0)
        gr = mpmath.mpf(got[0].numerator) / got[0].denominator
        gi = mpmath.mpf(got[1].numerator) / got[1].denominator
        assert abs(gr - want_re) <= 20 * m * u(P) * mu
        assert abs(gi - want_im) <= 20 * m * u(P) * mu


@pytest.mark.parametrize("P,m,n", [(2, 8, 5), (4, 7, 7), (8, 6, 4)])
def test_real_data_matches_real_oracle(orc, P, m, n):
    """On real data (zero imaginary parts) x is the real least-squares solution and |R|
    equals the real |R| (the diagonal phases may differ by a sign)."""
    A, _ = mdgen.ls_problem(P, m, n, 51 + m)
    b = mdgen.md_vector(P, m, 51 + m, mdgen.STREAM_B)
    rr = orc.lstsq(A, b)
    Ac = np.stack([A, np.zeros_like(A)])
    bc = np.stack([b, np.zeros_like(b)])
    rc = orc.clstsq(Ac, bc)
    k = kappa(Ac)
    xr = [F(rr["x"][:, i]) for i in range(n)]
    xc = cvec(rc["x"])
    scale = max(1.0, float(np.abs(rr["x"][0]).max()))
    for a, c in zip(xr, xc):
        assert abs(float(c[0] - a)) <= 100 * n * k * u(P) * scale
        assert abs(float(c[1])) <= 100 * n * k * u(P) * scale
    for j in range(n):
        for i in range(j + 1):
            re, im = cf(rc["F"], j, i)
            assert abs(abs(complex(float(re), float(im))) - abs(float(F(rr["F"][:, j, i])))) <= 100 * n * u(P) * 4


@pytest.mark.parametrize("P", (2, 4))
def test_times_i_equivariance(orc, P):
    """A -> iA, b -> ib (exact) leaves x, beta and v unchanged and maps R to iR."""
    m, n = 9, 6
    A = mdgen.cmd_uniform(P, m, n, 61, mdgen.STREAM_A)
    b = mdgen.cmd_vector(P, m, 61, mdgen.STREAM_B)
    iA = np.stack([-A[1], A[0]])
    ib = np.stack([-b[1], b[0]])
    r0 = orc.clstsq(A, b)
    r1 = orc.clstsq(iA, ib)
    k = kappa(A)
    tol = 100 * n * k * u(P)
    assert np.max(np.abs(r1["x"][:, 0] - r0["x"][:, 0])) <= tol * max(1.0, np.abs(r0["x"][:, 0]).max())
    assert np.max(np.abs(r1["beta"][0] - r0["beta"][0])) <= tol
    for j in range(n):
        for i in range(m):
            g0, g1 = cf(r0["F"], j, i), cf(r1["F"], j, i)
            want = cmul((Fraction(0), Fraction(1)), g0) if i <= j else g0  # R -> iR, v unchanged
            assert cabs(csub(g1, want)) <= tol * max(1.0, cabs(g0))


@pytest.mark.parametrize("P,m,n", [(2, 40, 24), (4, 30, 20), (8, 20, 12)])
def test_recovers_x_true_and_residual_orthogonal(orc, P, m, n):
    A, xt = mdgen.cls_problem(P, m, n, 71 + m)
    b = orc.cmatvec(A, xt, P)  # b = A x_true rounded to P limbs
    r = orc.clstsq(A, b)
    k = kappa(A)
    err = float(np.linalg.norm((r["x"][0, 0] - xt[0, 0]) + 1j * (r["x"][1, 0] - xt[1, 0])))
    assert err <= 100 * n * k * u(P) * float(np.linalg.norm(xt[0, 0] + 1j * xt[1, 0]))
    # A^H (b - A x) = 0 for a general right-hand side
    b2 = mdgen.cmd_vector(P, m, 71 + m, mdgen.STREAM_B)
    r2 = orc.clstsq(A, b2)
    res = orc.cmatvec(A, r2["x"], P, c=b2)
    g = orc.cmatvec(A, res, P, trans=True)
    gn = float(np.abs(g[0, 0] + 1j * g[1, 0]).max())
    anorm = float(np.linalg.norm(to_np(A), 2))
    assert gn <= 100 * m * k * u(P) * anorm * anorm * max(1.0, float(np.abs(r2["x"][:, 0]).max()))


@pytest.mark.parametrize("P", (2, 4))
def test_capply_qh_equals_explicit_qh(orc, P):
    m, n, nrhs = 8, 5, 3
    A = mdgen.cmd_uniform(P, m, n, 81, mdgen.STREAM_A)
    B = mdgen.cmd_uniform(P, m, nrhs, 81, mdgen.STREAM_B)
    Fq, beta = orc.cqr(A)
    QhB = orc.capply_qh(Fq, beta, B)
    Qe, Be = cmat(orc.cexplicit_q(Fq, beta)), cmat(B)
    for c in range(nrhs):
        for i in range(m):
            s = (Fraction(0), Fraction(0))
            for k in range(m):
                s = cadd(s, cmul(cconj(Qe[k][i]), Be[k][c]))
            assert cabs(csub(cf(QhB, c, i), s)) <= 40 * m * u(P)


def test_sigma_zero_columns(orc):
    """Upper-triangular complex input: every sigma is 0, beta = 0 and A is untouched; for a
    square matrix the last column always has sigma = 0 and keeps R(n-1, n-1)."""
    P, n = 2, 5
    A = mdgen.cmd_uniform(P, n, n, 91, mdgen.STREAM_A)
    for j in range(n):
        A[:, :, j, j + 1:] = 0.0
    Fq, beta = orc.cqr(A)
    assert np.all(beta == 0.0)
    assert np.array_equal(Fq, A)
    B = mdgen.cmd_uniform(P, n, n, 92, mdgen.STREAM_A)
    Fb, bb = orc.cqr(B)
    assert np.all(bb[:, n - 1] == 0.0)
    assert bb[0, 0] > 0.0


@pytest.mark.parametrize("P", (2, 4, 8))
def test_cbacksub_exact_rational(orc, P):
    n = 6
    R = mdgen.cmd_uniform(P, n, n, 101, mdgen.STREAM_A)
    for j in range(n):
        R[:, :, j, j + 1:] = 0.0
        R[0, 0, j, j] += 4.0  # keep it well conditioned
    y = mdgen.cmd_vector(P, n, 101, mdgen.STREAM_B)
    x, info = orc.cbacksub(R, y)
    assert info == 0
    Re, ye = cmat(R), cvec(y)
    xs = [None] * n
    for i in range(n - 1, -1, -1):
        s = ye[i]
        for k in range(i + 1, n):
            s = csub(s, cmul(Re[i][k], xs[k]))
        xs[i] = cdiv(s, Re[i][i])
    for i in range(n):
        assert cabs(csub(cf(x, i), xs[i])) <= 50 * n * u(P) * max(1.0, cabs(xs[i]))


def test_cbacksub_zero_diagonal_info(orc):
    P, n = 2, 4
    R = mdgen.cmd_uniform(P, n, n, 111, mdgen.STREAM_A)
    R[:, :, 2, 2] = 0.0
    _, info = orc.cbacksub(R, mdgen.cmd_vector(P, n, 111, mdgen.STREAM_B))
    assert info == 3


def test_thread_count_independent(orc):
    A = mdgen.cmd_uniform(2, 30, 20, 121, mdgen.STREAM_A)
    b = mdgen.cmd_vector(2, 30, 121, mdgen.STREAM_B)
    r1 = orc.clstsq(A, b, nthreads=1)
    r4 = orc.clstsq(A, b, nthreads=4)
    assert np.array_equal(r1["x"], r4["x"]) and np.array_equal(r1["F"], r4["F"])


@pytest.mark.parametrize("m,n", [(20, 20), (50, 30)])
def test_p1_matches_lapack(orc, m, n):
    A = mdgen.cmd_uniform(1, m, n, 131 + m, mdgen.STREAM_A)
    b = mdgen.cmd_vector(1, m, 131 + m, mdgen.STREAM_B)
    r = orc.clstsq(A, b)
    want = np.linalg.lstsq(to_np(A), b[0, 0] + 1j * b[1, 0], rcond=None)[0]
    got = r["x"][0, 0] + 1j * r["x"][1, 0]
    assert np.linalg.norm(got - want) <= 1e-12 * kappa(A) * np.linalg.norm(want)
