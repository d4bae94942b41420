"""Pins of the oracle's least-squares path (paper Section 1: A = QR reduces A x = b to
R x = Q^T b; Section 3: Householder vectors with the Golub-Van Loan 5.1.1 sign choice;
Section 2: back substitution) against facts fixed by the mathematics: the Cholesky factor
of the exact A^T A, the exact rational normal-equation solution, orthogonality of Q,
orthogonality of the residual, special cases and LAPACK at P = 1."""
from fractions import Fraction

import numpy as np
import pytest

import mdgen


def F(x):
    return sum((Fraction(float(v)) for v in x), Fraction(0))


def u(P):
    return 2.0 ** (-(52 * P + 1))


def fmat(A):
    """(P, n, m) md matrix -> m x n list of Fractions."""
    P, n, m = A.shape
    return [[F(A[:, j, i]) for j in range(n)] for i in range(m)]


def fvec(x):
    return [F(x[:, i]) for i in range(x.shape[1])]


def solve_fraction(M, r):
    """Gaussian elimination with exact rationals (no pivoting needed for SPD M)."""
    n = len(M)
    M = [row[:] + [r[i]] for i, row in enumerate(M)]
    for k in range(n):
        piv = M[k][k]
        for i in range(k + 1, n):
            f = M[i][k] / piv
            for j in range(k, n + 1):
                M[i][j] -= f * M[k][j]
    x = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        s = M[i][n] - sum(M[i][j] * x[j] for j in range(i + 1, n))
        x[i] = s / M[i][i]
    return x


def kappa(A):
    return float(np.linalg.cond(A[0].T))


@pytest.mark.parametrize("P,m,n", [(2, 6, 4), (2, 5, 5), (4, 7, 5), (8, 4, 3)])
def test_R_is_cholesky_of_exact_gram(orc, P, m, n):
    import mpmath

    A = mdgen.md_uniform(P, m, n, 11 + m, mdgen.STREAM_A)
    Fq, beta = orc.qr(A)
    Af = fmat(A)
    with mpmath.workprec(60 * P + 300):
        G = [[sum(Af[k][i] * Af[k][j] for k in range(m)) for j in range(n)] for i in range(n)]
        Gm = mpmath.matrix([[mpmath.mpf(g.numerator) / g.denominator for g in row] for row in G])
        L = mpmath.cholesky(Gm)  # G = L L^T, R = L^T with positive diagonal
        scale = mpmath.sqrt(max(abs(Gm[i, i]) for i in range(n)))
        for i in range(n):
            for j in range(i, n):
                r = F(Fq[:, j, i])
                got = mpmath.mpf(r.numerator) / r.denominator
                want = L[j, i]
                if m == n and i == n - 1:
                    # the last column has sigma = 0: its reflector is the identity and R_nn
                    # keeps the sign it has after the previous reflectors
                    want = abs(want) * (1 if got >= 0 else -1)
                assert abs(got - want) <= 50 * n * kappa(A) * u(P) * scale
        # GVL sign: R_jj = mu > 0 whenever sigma != 0 (every column except the last if m == n)
        for j in range(n - (1 if m == n else 0)):
            assert Fq[0, j, j] > 0


@pytest.mark.parametrize("P,m,n", [(2, 8, 5), (4, 6, 6), (8, 5, 4), (2, 12, 12)])
def test_x_matches_exact_rational_lstsq(orc, P, m, n):
    A = mdgen.md_uniform(P, m, n, 31 + n, mdgen.STREAM_A)
    b = mdgen.md_vector(P, m, 31 + n, mdgen.STREAM_B)
    out = orc.lstsq(A, b)
    assert out["info"] == 0
    Af, bf = fmat(A), fvec(b)
    G = [[sum(Af[k][i] * Af[k][j] for k in range(m)) for j in range(n)] for i in range(n)]
    r = [sum(Af[k][i] * bf[k] for k in range(m)) for i in range(n)]
    xs = solve_fraction(G, r)
    nx = max(abs(v) for v in xs)
    err = max(abs(F(out["x"][:, i]) - xs[i]) for i in range(n))
    assert float(err / nx) <= 100 * n * kappa(A) ** 2 * u(P) + 100 * n * kappa(A) * u(P)


@pytest.mark.parametrize("P,m,n", [(2, 7, 5), (4, 6, 6), (8, 5, 3)])
def test_q_orthogonal_and_qta_is_r(orc, P, m, n):
    A = mdgen.md_uniform(P, m, n, 5, mdgen.STREAM_A)
    Fq, beta = orc.qr(A)
    Q = orc.explicit_q(Fq, beta)
    Qf = fmat(Q)
    Af = fmat(A)
    tol = Fraction(50 * m) * Fraction(u(P))
    for i in range(m):
        for j in range(m):
            d = sum(Qf[k][i] * Qf[k][j] for k in range(m)) - (1 if i == j else 0)
            assert abs(d) <= tol
    # Q^T A = R (zero below the diagonal, R above)
    for i in range(m):
        for j in range(n):
            v = sum(Qf[k][i] * Af[k][j] for k in range(m))
            want = F(Fq[:, j, i]) if i <= j else Fraction(0)
            assert abs(v - want) <= tol * 4


@pytest.mark.parametrize("P", (2, 4))
def test_apply_qt_equals_explicit_qt(orc, P):
    m, n = 9, 6
    A = mdgen.md_uniform(P, m, n, 8, mdgen.STREAM_A)
    b = mdgen.md_vector(P, m, 8, mdgen.STREAM_B)
    Fq, beta = orc.qr(A)
    Q = orc.explicit_q(Fq, beta)
    qtb = orc.apply_qt(Fq, beta, b)
    ref = orc.matvec(Q, b, P, trans=True)
    for i in range(m):
        assert abs(F(qtb[:, i]) - F(ref[:, i])) <= Fraction(40 * m) * Fraction(u(P))
    # ||Q^T b||_2 = ||b||_2
    nb = sum(F(b[:, i]) ** 2 for i in range(m))
    nq = sum(F(qtb[:, i]) ** 2 for i in range(m))
    assert abs(nq - nb) / nb <= Fraction(80 * m) * Fraction(u(P))


@pytest.mark.parametrize("P,m,n", [(2, 40, 24), (4, 30, 20), (8, 20, 12)])
def test_residual_orthogonal_to_range(orc, P, m, n):
    A = mdgen.md_uniform(P, m, n, 17, mdgen.STREAM_A)
    b = mdgen.md_vector(P, m, 17, mdgen.STREAM_B)
    out = orc.lstsq(A, b)
    r = orc.matvec(A, out["x"], P, c=b)  # b - A x, exact then rounded
    atr = orc.matvec(A, r, P, trans=True)
    nA = np.linalg.norm(A[0].T, 2)
    nx = np.linalg.norm(out["x"][0])
    nb = np.linalg.norm(b[0])
    assert np.max(np.abs(atr[0])) <= 50 * m * u(P) * nA * (nA * nx + nb)
    # and the residual norm equals ||(Q^T b)(n:m)||
    rn = np.sqrt(sum(float(F(r[:, i])) ** 2 for i in range(m)))
    tail = np.sqrt(sum(float(F(out["qtb"][:, i])) ** 2 for i in range(n, m)))
    assert abs(rn - tail) <= 1e-12 * max(rn, 1e-300)


@pytest.mark.parametrize("P,m,n", [(2, 64, 48), (4, 32, 32), (8, 24, 16)])
def test_recovers_x_true(orc, P, m, n):
    A, xt = mdgen.ls_problem(P, m, n, 3)
    b = orc.rhs_for(A, xt)
    out = orc.lstsq(A, b)
    k = kappa(A)
    err = max(abs(F(out["x"][:, i]) - F(xt[:, i])) for i in range(n))
    nx = max(abs(F(xt[:, i])) for i in range(n))
    assert float(err / nx) <= 100 * n * k * u(P)


@pytest.mark.parametrize("P", (1, 2, 4))
def test_upper_triangular_input_is_untouched(orc, P):
    n = 7
    R = mdgen.upper_triangular(P, n, 4)
    R[0, 2, 2] = -R[0, 2, 2]  # negative diagonal entries keep their sign
    R[1:, 2, 2] = -R[1:, 2, 2]
    Fq, beta = orc.qr(R)
    assert np.array_equal(Fq, R)  # sigma = 0 in every column: bit-exact R = A
    assert np.all(beta == 0.0)
    y = mdgen.md_vector(P, n, 4, mdgen.STREAM_B)
    out = orc.lstsq(R, y)
    x, info = orc.backsub(R, y)
    assert info == 0 and np.array_equal(out["x"], x)


def test_three_four(orc):
    P = 2
    A = np.zeros((P, 1, 2))
    A[0, 0, 0], A[0, 0, 1] = 3.0, 4.0
    b = np.zeros((P, 2))
    b[0] = [6.0, 8.0]
    out = orc.lstsq(A, b)
    assert out["F"][0, 0, 0] == 5.0 and out["F"][1, 0, 0] == 0.0
    assert abs(F(out["x"][:, 0]) - 2) <= Fraction(2) ** -100
    # v = x / v1 with v1 = -sigma/(a11 + mu) = -16/8 = -2: v2 = 4 / -2 = -2
    assert out["F"][0, 0, 1] == -2.0
    # beta = 2 v1^2/(sigma + v1^2) = 8/20
    assert abs(F(out["beta"][:, 0]) - Fraction(2, 5)) <= Fraction(2) ** -100


def test_diagonal_matrix(orc):
    P, n = 4, 5
    A = np.zeros((P, n, n))
    for i in range(n):
        A[0, i, i] = (-1) ** i * (i + 1.5)
    b = mdgen.md_vector(P, n, 2, mdgen.STREAM_B)
    out = orc.lstsq(A, b)
    for i in range(n):
        want = F(b[:, i]) / Fraction(A[0, i, i])
        assert abs(F(out["x"][:, i]) - want) <= abs(want) * Fraction(2) ** -200


@pytest.mark.parametrize("m,n", [(20, 20), (50, 30)])
def test_p1_matches_lapack(orc, m, n):
    A = mdgen.md_uniform(1, m, n, 9, mdgen.STREAM_A)
    b = mdgen.md_vector(1, m, 9, mdgen.STREAM_B)
    out = orc.lstsq(A, b)
    An = A[0].T.copy()
    x_np = np.linalg.lstsq(An, b[0], rcond=None)[0]
    k = np.linalg.cond(An)
    assert np.max(np.abs(out["x"][0] - x_np)) <= 1e-14 * k * max(1, np.max(np.abs(x_np)))
    Rn = np.linalg.qr(An, mode="r")
    Ro = np.triu(out["F"][0].T[:n, :])
    s = np.sign(np.diag(Rn)) * np.sign(np.diag(Ro))
    assert np.allclose(Ro, s[:, None] * Rn, atol=1e-13 * np.abs(Rn).max())


@pytest.mark.parametrize("P", (2, 4, 8))
def test_backsub_exact_rational(orc, P):
    n = 6
    R = mdgen.upper_triangular(P, n, 21)
    y = mdgen.md_vector(P, n, 21, mdgen.STREAM_B)
    x, info = orc.backsub(R, y)
    assert info == 0
    Rf = fmat(R)
    yf = fvec(y)
    xs = [Fraction(0)] * n
    for i in range(n - 1, -1, -1):
        xs[i] = (yf[i] - sum(Rf[i][k] * xs[k] for k in range(i + 1, n))) / Rf[i][i]
    for i in range(n):
        assert abs(F(x[:, i]) - xs[i]) <= abs(xs[i]) * Fraction(1000) * Fraction(u(P)) + Fraction(u(P))


def test_zero_diagonal_info(orc):
    P, n = 2, 5
    R = mdgen.upper_triangular(P, n, 2)
    R[:, 3, 3] = 0.0
    R[:, 1, 1] = 0.0
    y = mdgen.md_vector(P, n, 2, mdgen.STREAM_B)
    _, info = orc.backsub(R, y)
    assert info == 2  # smallest 1-based index with R_ii == 0
    # a zero column in A gives an exactly zero R_jj
    A = mdgen.md_uniform(P, 8, 5, 3, mdgen.STREAM_A)
    A[:, 2, :] = 0.0
    out = orc.lstsq(A, mdgen.md_vector(P, 8, 3, mdgen.STREAM_B))
    assert out["info"] == 3


def test_thread_count_independent(orc):
    A = mdgen.md_uniform(2, 40, 30, 1, mdgen.STREAM_A)
    b = mdgen.md_vector(2, 40, 1, mdgen.STREAM_B)
    o1 = orc.lstsq(A, b, nthreads=1)
    o4 = orc.lstsq(A, b, nthreads=4)
    assert np.array_equal(o1["x"], o4["x"]) and np.array_equal(o1["F"], o4["F"])


def tally_closed_form(m, n, npos):
    """Exact md operation counts of the unblocked least-squares solve (Golub-Van Loan 5.1.1 and
    5.2.1 applied to A and b, then back substitution), as closed-form polynomials in m and n.

    Column j (L = m - j rows from the diagonal) of the QR costs: sigma, L-1 multiplications and
    additions; mu = sqrt(a_jj^2 + sigma), 1 multiplication, 1 addition, 1 square root; v1,
    1 addition (x1 <= 0) or 1 addition and 1 division (x1 > 0); beta = 2 v1^2 / (sigma + v1^2),
    1 multiplication, 1 addition, 1 division; v = x / v1, L-1 divisions; and for each of the
    n-j-1 columns to its right 2(L-1)+1 multiplications and as many additions.  With m = n the
    last column has sigma = 0 and stops after its sigma.  Q^T b costs 2L-1 of each per column
    with beta != 0; back substitution n(n-1)/2 of each and n divisions.  npos is the number of
    columns with x1 > 0."""
    sq = n if m > n else n - 1          # columns with sigma != 0
    s_l1 = n * (m - 1) - n * (n - 1) // 2                        # sum_j (L - 1)
    s_upd = (2 * (m - n) + 1) * n * (n - 1) // 2 + (n - 1) * n * (2 * n - 1) // 3  # sum_j (n-j-1)(2L-1)
    s_qtb = 2 * n * m - n * n - (1 if m == n else 0)               # sum_{j: sigma != 0} (2L - 1)
    tri = n * (n - 1) // 2
    add = s_l1 + 3 * sq + s_upd + s_qtb + tri
    mul = s_l1 + 2 * sq + s_upd + s_qtb + tri
    div = npos + sq + s_l1 + n
    return add, mul, div, sq


def test_closed_form_polynomials_match_their_loop_sums():
    """The closed forms above against the plain loop sums they summarise (pins the algebra)."""
    for m, n in ((60, 40), (33, 7), (100, 1), (17, 16), (16, 16), (5, 5), (2, 1)):
        add = mul = div = sq = 0
        for j in range(n):
            L = m - j
            add += L - 1
            mul += L - 1
            if L == 1:  # sigma = 0 (m = n, last column)
                continue
            add += 3
            mul += 2
            div += 1 + (L - 1)
            sq += 1
            add += (n - j - 1) * (2 * L - 1)
            mul += (n - j - 1) * (2 * L - 1)
            add += 2 * L - 1  # Q^T b
            mul += 2 * L - 1
        add += n * (n - 1) // 2
        mul += n * (n - 1) // 2
        div += n
        assert (add, mul, div, sq) == tally_closed_form(m, n, 0), (m, n)


@pytest.mark.parametrize("P,m,n", [(2, 60, 40), (1, 33, 7), (4, 100, 1), (2, 17, 16), (2, 16, 16), (8, 9, 9)])
def test_tally_exact(orc, P, m, n):
    """The oracle's operation tally equals the closed-form polynomials exactly, every term.
    The only data-dependent term is the number of columns with x1 > 0 (one extra division):
    by Golub-Van Loan 5.1.1, x1 <= 0 gives v1^2 >= sigma and so beta >= 1, x1 > 0 gives
    v1^2 < sigma and beta < 1, so it is read off the returned betas."""
    A = mdgen.md_uniform(P, m, n, 11 + m + n, mdgen.STREAM_A)
    out = orc.lstsq(A, mdgen.md_vector(P, m, 11, mdgen.STREAM_B), tally=True)
    beta = out["beta"][0]
    sig_nonzero = n if m > n else n - 1
    npos = int(np.sum(beta[:sig_nonzero] < 1.0))
    assert 0 < npos < sig_nonzero or sig_nonzero <= 2
    assert tuple(out["tally"]) == tally_closed_form(m, n, npos)
    # the QR alone: the same polynomials without the Q^T b and back-substitution terms
    F, bt, t = orc.qr(A, tally=True)
    add, mul, div, sq = tally_closed_form(m, n, npos)
    s_qtb = 2 * n * m - n * n - (1 if m == n else 0)
    tri = n * (n - 1) // 2
    assert tuple(t) == (add - s_qtb - tri, mul - s_qtb - tri, div - n, sq)
