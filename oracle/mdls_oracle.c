/*
 * mdls_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, CPU-only reference for multiple-double least squares: the arithmetic
 * of multiple-double numbers (unevaluated sums of P doubles, limb 0 most significant;
 * paper Section 1.1 and Table 1) and the unblocked Householder least-squares solve that
 * the paper's blocked Algorithm 2 and tiled Algorithm 1 accelerate (Section 1: A = QR
 * reduces A x = b to R x = Q^T b, solved by back substitution).
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg may load this
 * library.  It shares no code, header, table or helper with the GPU library.
 *
 * Arithmetic: every multiple-double operation is computed EXACTLY as a floating-point
 * expansion (Shewchuk, "Adaptive precision floating-point arithmetic and fast robust
 * geometric predicates", 1997: TwoSum, Grow-Expansion with zero elimination, Compress)
 * and then truncated to P limbs, limb k being the largest component of the compressed
 * exact remainder after limbs 0..k-1.  Division is long division with an exact
 * remainder; square root is a Newton iteration with an exact residual.  Relative error of
 * each operation is below 2^(1-52P) (truncation after P limbs, each within one ulp of the
 * remaining value).
 *
 * Least squares: Householder vectors and beta as in Golub and Van Loan, Matrix
 * Computations (3rd ed., 1996) Algorithm 5.1.1, which the paper cites for the sign choice
 * (Section 3, text before Algorithm 2): sigma = x(2:L)^T x(2:L); if sigma = 0 then beta = 0
 * (the reflector is the identity and R_jj keeps its sign); otherwise mu = sqrt(x1^2 +
 * sigma), v1 = x1 - mu if x1 <= 0 else -sigma/(x1 + mu), beta = 2 v1^2/(sigma + v1^2),
 * v = x / v1.  The reflector I - beta v v^T is applied column by column (unblocked QR,
 * Golub and Van Loan Algorithm 5.2.1); R_jj is set to mu.  Back substitution solves
 * R x = (Q^T b)(0:n) from the last row up.  All sums run in ascending index order.
 *
 * Storage (the paper's staging after Algorithm 1): a matrix of multiple doubles is P
 * planes of doubles, most significant first; each plane is column-major with leading
 * dimension ld; plane k starts ps doubles after plane k-1.  Vectors: P planes of stride vs.
 *
 * Complex data (the paper's complex double double QR, Section 4 Table 5): the same unblocked
 * QR, Q^H b and back substitution with complex multiple doubles (real and imaginary parts in
 * separate limb planes) and the Hermitian transpose in place of the transpose (Section 3);
 * the complex Householder vector is described above orc_cqr.
 *
 * Threading: OpenMP over independent columns (trailing columns, right-hand sides, rows
 * of a matrix-vector product).  Results do not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_MAXP 16
#define XCAP 512          /* capacity of one exact accumulator (components) */
#define XCOMPRESS_EVERY 8 /* compress after this many insertions */

/* ------------------------------------------------------------------ error-free transforms */

/* Knuth's TwoSum: s + e == a + b exactly, s = fl(a + b). */
static inline void two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    double bv = x - a;
    double av = x - bv;
    *e = (a - av) + (b - bv);
    *s = x;
}

/* Dekker's FastTwoSum, valid when |a| >= |b| (or a == 0): s + e == a + b exactly. */
static inline void fast_two_sum(double a, double b, double *s, double *e)
{
    double x = a + b;
    *e = b - (x - a);
    *s = x;
}

/* TwoProd with a fused multiply-add: p + e == a * b exactly. */
static inline void two_prod(double a, double b, double *p, double *e)
{
    double x = a * b;
    *e = fma(a, b, -x);
    *p = x;
}

/* ------------------------------------------------------------------ exact accumulator */
/* A nonoverlapping expansion, components in increasing magnitude, no zero components. */
typedef struct {
    int len;
    int since;
    double h[XCAP];
} xacc;

static void xacc_init(xacc *a)
{
    a->len = 0;
    a->since = 0;
}

/* Shewchuk's Compress, in place: same value, nonoverlapping, increasing, no zeros, and the
 * largest component approximates the whole sum with an error below one of its ulps. */
static int compress(int len, double *e)
{
    double g[XCAP];
    if (len <= 1)
        return len;
    int bottom = len - 1;
    double Q = e[len - 1], q;
    for (int i = len - 2; i >= 0; i--) {
        double Qn;
        fast_two_sum(Q, e[i], &Qn, &q);
        if (q != 0.0) {
            g[bottom--] = Qn;
            Q = q;
        } else {
            Q = Qn;
        }
    }
    g[bottom] = Q;
    int top = 0;
    for (int i = bottom + 1; i < len; i++) {
        double Qn;
        fast_two_sum(g[i], Q, &Qn, &q);
        if (q != 0.0)
            e[top++] = q;
        Q = Qn;
    }
    e[top++] = Q;
    if (top == 1 && e[0] == 0.0)
        return 0;
    return top;
}

/* Shewchuk's Grow-Expansion with zero elimination: add one double exactly. */
static void xacc_add(xacc *a, double b)
{
    if (b == 0.0)
        return;
    double Q = b, hh;
    int k = 0;
    for (int i = 0; i < a->len; i++) {
        two_sum(Q, a->h[i], &Q, &hh);
        if (hh != 0.0)
            a->h[k++] = hh;
    }
    if (Q != 0.0)
        a->h[k++] = Q;
    a->len = k;
    if (++a->since >= XCOMPRESS_EVERY || a->len > XCAP - 8) {
        a->len = compress(a->len, a->h);
        a->since = 0;
        if (a->len > XCAP - 8) {
            /* unreachable for values that span fewer than ~20000 bits; keep the largest
             * components rather than overrun the buffer */
            int drop = a->len - (XCAP - 8);
            memmove(a->h, a->h + drop, sizeof(double) * (size_t)(XCAP - 8));
            a->len = XCAP - 8;
        }
    }
}

static void xacc_add_md(xacc *a, int P, const double *x, double sign)
{
    for (int k = P - 1; k >= 0; k--)
        xacc_add(a, sign * x[k]);
}

/* add sign * x * y exactly (all P*Q partial products, both halves of each TwoProd) */
static void xacc_add_prod(xacc *a, int P, const double *x, int Q, const double *y, double sign)
{
    for (int i = P - 1; i >= 0; i--)
        for (int j = Q - 1; j >= 0; j--) {
            double p, e;
            two_prod(x[i], y[j], &p, &e);
            xacc_add(a, sign * e);
            xacc_add(a, sign * p);
        }
}

/* best double approximation of the accumulated value (largest compressed component) */
static double xacc_top(xacc *a)
{
    a->len = compress(a->len, a->h);
    a->since = 0;
    return a->len ? a->h[a->len - 1] : 0.0;
}

/* truncate the exact value to P limbs: limb k = largest component of the compressed
 * remainder left by limbs 0..k-1. */
static void xacc_round(xacc *a, int P, double *out)
{
    double t[XCAP];
    int len = a->len;
    memcpy(t, a->h, sizeof(double) * (size_t)len);
    len = compress(len, t);
    for (int k = 0; k < P; k++) {
        if (len == 0) {
            out[k] = 0.0;
            continue;
        }
        out[k] = t[len - 1];
        len--;
        len = compress(len, t);
    }
}

static int md_is_zero(int P, const double *x)
{
    for (int k = 0; k < P; k++)
        if (x[k] != 0.0)
            return 0;
    return 1;
}

/* ------------------------------------------------------------------ md operations */

void orc_md_add(int P, const double *a, const double *b, double *r)
{
    xacc x;
    xacc_init(&x);
    xacc_add_md(&x, P, a, 1.0);
    xacc_add_md(&x, P, b, 1.0);
    xacc_round(&x, P, r);
}

void orc_md_sub(int P, const double *a, const double *b, double *r)
{
    xacc x;
    xacc_init(&x);
    xacc_add_md(&x, P, a, 1.0);
    xacc_add_md(&x, P, b, -1.0);
    xacc_round(&x, P, r);
}

void orc_md_mul(int P, const double *a, const double *b, double *r)
{
    xacc x;
    xacc_init(&x);
    xacc_add_prod(&x, P, a, P, b, 1.0);
    xacc_round(&x, P, r);
}

/* a / b by long division: quotient digits q_k = top(remainder) / b_0, remainder updated
 * exactly; P + 2 digits, then the exact digit sum is truncated to P limbs. */
void orc_md_div(int P, const double *a, const double *b, double *r)
{
    xacc rem, quo;
    xacc_init(&rem);
    xacc_init(&quo);
    xacc_add_md(&rem, P, a, 1.0);
    for (int k = 0; k < P + 2; k++) {
        double top = xacc_top(&rem);
        if (top == 0.0)
            break;
        double q = top / b[0];
        xacc_add(&quo, q);
        xacc_add_prod(&rem, 1, &q, P, b, -1.0);
    }
    xacc_round(&quo, P, r);
}

/* sqrt(a), a >= 0: s <- s + top(a - s^2) / (2 s_0) with the residual exact and s kept to
 * P + 2 limbs; P + 3 steps from the double square root. */
void orc_md_sqrt(int P, const double *a, double *r)
{
    double s[ORC_MAXP + 2];
    int W = P + 2;
    if (a[0] <= 0.0) {
        for (int k = 0; k < P; k++)
            r[k] = (a[0] == 0.0) ? 0.0 : NAN;
        return;
    }
    memset(s, 0, sizeof(s));
    s[0] = sqrt(a[0]);
    for (int it = 0; it < P + 3; it++) {
        xacc res;
        xacc_init(&res);
        xacc_add_md(&res, P, a, 1.0);
        xacc_add_prod(&res, W, s, W, s, -1.0);
        double c = xacc_top(&res) / (2.0 * s[0]);
        if (c == 0.0)
            break;
        xacc sum;
        xacc_init(&sum);
        xacc_add_md(&sum, W, s, 1.0);
        xacc_add(&sum, c);
        xacc_round(&sum, W, s);
    }
    for (int k = 0; k < P; k++)
        r[k] = s[k];
}

/* exact sum of nterms doubles, truncated to P limbs */
void orc_md_round(int P, int nterms, const double *terms, double *r)
{
    xacc x;
    xacc_init(&x);
    for (int i = 0; i < nterms; i++)
        xacc_add(&x, terms[i]);
    xacc_round(&x, P, r);
}

static void md_neg(int P, const double *a, double *r)
{
    for (int k = 0; k < P; k++)
        r[k] = -a[k];
}

/* ------------------------------------------------------------------ SoA access */
static inline void ldm(int P, const double *X, long ps, long off, double *v)
{
    for (int k = 0; k < P; k++)
        v[k] = X[(long)k * ps + off];
}

static inline void stm(int P, double *X, long ps, long off, const double *v)
{
    for (int k = 0; k < P; k++)
        X[(long)k * ps + off] = v[k];
}

#define AT(i, j, ld) ((long)(j) * (long)(ld) + (long)(i))

static int valid_p(int P) { return P >= 1 && P <= ORC_MAXP; }

static void set_threads(int nthreads)
{
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#else
    (void)nthreads;
#endif
}

/* tally slots: 0 add (incl. sub), 1 mul, 2 div, 3 sqrt */
static void tally_add(long *t, long add, long mul, long div, long sq)
{
    if (!t)
        return;
    t[0] += add;
    t[1] += mul;
    t[2] += div;
    t[3] += sq;
}

/* ------------------------------------------------------------------ Householder QR */

/*
 * Unblocked Householder QR of the m x n matrix A (m >= n), in place: on return R is in the
 * upper triangle and the Householder vector of column j (unit first entry implicit) is in
 * A(j+1:m, j); beta (P planes of stride n) holds the n beta values.
 */
int orc_qr(int P, int m, int n, double *A, int lda, long ps, double *beta, long *tally,
           int nthreads)
{
    if (!valid_p(P) || m < n || n < 0 || lda < m)
        return -1;
    set_threads(nthreads);
    for (int j = 0; j < n; j++) {
        double sig[ORC_MAXP], ajj[ORC_MAXP], t1[ORC_MAXP], t2[ORC_MAXP];
        double mu[ORC_MAXP], v1[ORC_MAXP], bt[ORC_MAXP], rv[ORC_MAXP];
        long L = m - j;
        memset(sig, 0, sizeof(sig));
        for (int i = j + 1; i < m; i++) {
            ldm(P, A, ps, AT(i, j, lda), t1);
            orc_md_mul(P, t1, t1, t2);
            orc_md_add(P, sig, t2, sig);
        }
        tally_add(tally, L - 1, L - 1, 0, 0);
        ldm(P, A, ps, AT(j, j, lda), ajj);
        if (md_is_zero(P, sig)) {
            /* the reflector is the identity: beta = 0, R_jj = a_jj with its sign */
            memset(bt, 0, sizeof(bt));
            stm(P, beta, n, j, bt);
            continue;
        }
        orc_md_mul(P, ajj, ajj, t1);
        orc_md_add(P, t1, sig, t2);
        orc_md_sqrt(P, t2, mu);
        tally_add(tally, 1, 1, 0, 1);
        if (ajj[0] <= 0.0) {
            orc_md_sub(P, ajj, mu, v1);
            tally_add(tally, 1, 0, 0, 0);
        } else {
            orc_md_add(P, ajj, mu, t1);
            orc_md_div(P, sig, t1, t2);
            md_neg(P, t2, v1);
            tally_add(tally, 1, 0, 1, 0);
        }
        orc_md_mul(P, v1, v1, t1);           /* v1^2 */
        orc_md_add(P, sig, t1, t2);          /* sigma + v1^2 */
        for (int k = 0; k < P; k++)
            t1[k] *= 2.0;                    /* 2 v1^2, exact */
        orc_md_div(P, t1, t2, bt);
        tally_add(tally, 1, 1, 1, 0);
        stm(P, beta, n, j, bt);
        for (int i = j + 1; i < m; i++) {    /* v = x / v1, unit first entry implicit */
            ldm(P, A, ps, AT(i, j, lda), t1);
            orc_md_div(P, t1, v1, rv);
            stm(P, A, ps, AT(i, j, lda), rv);
        }
        tally_add(tally, 0, 0, L - 1, 0);
        stm(P, A, ps, AT(j, j, lda), mu);

        /* apply I - beta v v^T to columns j+1..n-1 */
#pragma omp parallel for schedule(dynamic, 1)
        for (int c = j + 1; c < n; c++) {
            double w[ORC_MAXP], a[ORC_MAXP], v[ORC_MAXP], p[ORC_MAXP], t[ORC_MAXP];
            ldm(P, A, ps, AT(j, c, lda), w);  /* v_j = 1 */
            for (int i = j + 1; i < m; i++) {
                ldm(P, A, ps, AT(i, j, lda), v);
                ldm(P, A, ps, AT(i, c, lda), a);
                orc_md_mul(P, v, a, p);
                orc_md_add(P, w, p, w);
            }
            orc_md_mul(P, bt, w, t);          /* t = beta w */
            ldm(P, A, ps, AT(j, c, lda), a);
            orc_md_sub(P, a, t, a);
            stm(P, A, ps, AT(j, c, lda), a);
            for (int i = j + 1; i < m; i++) {
                ldm(P, A, ps, AT(i, j, lda), v);
                ldm(P, A, ps, AT(i, c, lda), a);
                orc_md_mul(P, t, v, p);
                orc_md_sub(P, a, p, a);
                stm(P, A, ps, AT(i, c, lda), a);
            }
        }
        tally_add(tally, (long)(n - j - 1) * (2 * (L - 1) + 1), (long)(n - j - 1) * (2 * (L - 1) + 1), 0,
                  0);
    }
    return 0;
}

/* B := Q^T B for the m x nrhs matrix B, with Q the product of the reflectors stored by
 * orc_qr (H_0 first): apply H_0, H_1, ..., H_{n-1} in turn. */
int orc_apply_qt(int P, int m, int n, const double *A, int lda, long psa, const double *beta,
                 double *B, int ldb, long psb, int nrhs, long *tally, int nthreads)
{
    if (!valid_p(P) || m < n || lda < m || ldb < m || nrhs < 0)
        return -1;
    set_threads(nthreads);
    for (int j = 0; j < n; j++) {
        double bt[ORC_MAXP];
        ldm(P, beta, n, j, bt);
        if (md_is_zero(P, bt))
            continue;
#pragma omp parallel for schedule(dynamic, 1)
        for (int c = 0; c < nrhs; c++) {
            double w[ORC_MAXP], a[ORC_MAXP], v[ORC_MAXP], p[ORC_MAXP], t[ORC_MAXP];
            ldm(P, B, psb, AT(j, c, ldb), w);
            for (int i = j + 1; i < m; i++) {
                ldm(P, A, psa, AT(i, j, lda), v);
                ldm(P, B, psb, AT(i, c, ldb), a);
                orc_md_mul(P, v, a, p);
                orc_md_add(P, w, p, w);
            }
            orc_md_mul(P, bt, w, t);
            ldm(P, B, psb, AT(j, c, ldb), a);
            orc_md_sub(P, a, t, a);
            stm(P, B, psb, AT(j, c, ldb), a);
            for (int i = j + 1; i < m; i++) {
                ldm(P, A, psa, AT(i, j, lda), v);
                ldm(P, B, psb, AT(i, c, ldb), a);
                orc_md_mul(P, t, v, p);
                orc_md_sub(P, a, p, a);
                stm(P, B, psb, AT(i, c, ldb), a);
            }
        }
        tally_add(tally, (long)nrhs * (2 * (m - j - 1) + 1), (long)nrhs * (2 * (m - j - 1) + 1), 0, 0);
    }
    return 0;
}

/* Solve R x = y for the leading n x n upper triangle of R (rows n-1 down to 0, ascending k
 * in each row sum).  info = smallest 1-based i with R_ii == 0 (then x is not computed). */
int orc_backsub(int P, int n, const double *R, int ldr, long psr, const double *y, long ys,
                double *x, long xs, int *info, long *tally)
{
    double d[ORC_MAXP], s[ORC_MAXP], r[ORC_MAXP], xk[ORC_MAXP], p[ORC_MAXP];
    if (!valid_p(P) || n < 0 || ldr < n)
        return -1;
    *info = 0;
    for (int i = 0; i < n; i++) {
        ldm(P, R, psr, AT(i, i, ldr), d);
        if (md_is_zero(P, d)) {
            *info = i + 1;
            return 0;
        }
    }
    for (int i = n - 1; i >= 0; i--) {
        ldm(P, y, ys, i, s);
        for (int k = i + 1; k < n; k++) {
            ldm(P, R, psr, AT(i, k, ldr), r);
            ldm(P, x, xs, k, xk);
            orc_md_mul(P, r, xk, p);
            orc_md_sub(P, s, p, s);
        }
        ldm(P, R, psr, AT(i, i, ldr), d);
        orc_md_div(P, s, d, p);
        stm(P, x, xs, i, p);
    }
    tally_add(tally, (long)n * (n - 1) / 2, (long)n * (n - 1) / 2, n, 0);
    return 0;
}

/* Least squares: QR of A (in place), b := Q^T b (in place), x from R x = b(0:n). */
int orc_lstsq(int P, int m, int n, double *A, int lda, long psa, double *b, long bs, double *x,
              long xs, double *beta, int *info, long *tally, int nthreads)
{
    int rc = orc_qr(P, m, n, A, lda, psa, beta, tally, nthreads);
    if (rc)
        return rc;
    rc = orc_apply_qt(P, m, n, A, lda, psa, beta, b, m, bs, 1, tally, nthreads);
    if (rc)
        return rc;
    return orc_backsub(P, n, A, lda, psa, b, bs, x, xs, info, tally);
}

/* Explicit m x m orthogonal Q = H_0 H_1 ... H_{n-1}, by backward accumulation onto I. */
int orc_explicit_q(int P, int m, int n, const double *A, int lda, long psa, const double *beta,
                   double *Q, int ldq, long psq, int nthreads)
{
    if (!valid_p(P) || m < n || lda < m || ldq < m)
        return -1;
    set_threads(nthreads);
    for (int c = 0; c < m; c++)
        for (int i = 0; i < m; i++) {
            double z[ORC_MAXP];
            memset(z, 0, sizeof(z));
            if (i == c)
                z[0] = 1.0;
            stm(P, Q, psq, AT(i, c, ldq), z);
        }
    for (int j = n - 1; j >= 0; j--) {
        double bt[ORC_MAXP];
        ldm(P, beta, n, j, bt);
        if (md_is_zero(P, bt))
            continue;
#pragma omp parallel for schedule(dynamic, 1)
        for (int c = j; c < m; c++) {
            double w[ORC_MAXP], a[ORC_MAXP], v[ORC_MAXP], p[ORC_MAXP], t[ORC_MAXP];
            ldm(P, Q, psq, AT(j, c, ldq), w);
            for (int i = j + 1; i < m; i++) {
                ldm(P, A, psa, AT(i, j, lda), v);
                ldm(P, Q, psq, AT(i, c, ldq), a);
                orc_md_mul(P, v, a, p);
                orc_md_add(P, w, p, w);
            }
            orc_md_mul(P, bt, w, t);
            ldm(P, Q, psq, AT(j, c, ldq), a);
            orc_md_sub(P, a, t, a);
            stm(P, Q, psq, AT(j, c, ldq), a);
            for (int i = j + 1; i < m; i++) {
                ldm(P, A, psa, AT(i, j, lda), v);
                ldm(P, Q, psq, AT(i, c, ldq), a);
                orc_md_mul(P, t, v, p);
                orc_md_sub(P, a, p, a);
                stm(P, Q, psq, AT(i, c, ldq), a);
            }
        }
    }
    return 0;
}

/*
 * y := op(A) x  or  y := c - op(A) x  (when c != NULL), each output computed EXACTLY
 * (all partial products accumulated in one expansion) and truncated to Py limbs.
 * op(A) = A (trans == 0, A is rows x cols, x has cols entries) or A^T (trans != 0).
 * A has Pa limbs, x has Px limbs, c has Pc limbs.  Used to form right-hand sides
 * b = A x_true above the working precision, and residuals.
 */
int orc_matvec(int trans, int Pa, int Px, int Pc, int Py, int rows, int cols, const double *A,
               int lda, long psa, const double *x, long xs, const double *c, long cs, double *y,
               long ys, int nthreads)
{
    if (!valid_p(Pa) || !valid_p(Px) || !valid_p(Py) || (c && !valid_p(Pc)) || lda < rows)
        return -1;
    set_threads(nthreads);
    int nout = trans ? cols : rows;
    int nin = trans ? rows : cols;
#pragma omp parallel for schedule(dynamic, 4)
    for (int o = 0; o < nout; o++) {
        double a[ORC_MAXP], xv[ORC_MAXP], out[ORC_MAXP];
        xacc *acc = (xacc *)malloc(sizeof(xacc));
        xacc_init(acc);
        double sign = 1.0;
        if (c) {
            double cv[ORC_MAXP];
            ldm(Pc, c, cs, o, cv);
            xacc_add_md(acc, Pc, cv, 1.0);
            sign = -1.0;
        }
        for (int k = 0; k < nin; k++) {
            long off = trans ? AT(k, o, lda) : AT(o, k, lda);
            ldm(Pa, A, psa, off, a);
            ldm(Px, x, xs, k, xv);
            xacc_add_prod(acc, Pa, a, Px, xv, sign);
        }
        xacc_round(acc, Py, out);
        stm(Py, y, ys, o, out);
        free(acc);
    }
    return 0;
}

/* ------------------------------------------------------------------ complex multiple doubles */
/*
 * A complex multiple double is a pair (re, im) of P-limb numbers.  A complex matrix is 2P
 * planes: the P limb planes of the real parts, then the P limb planes of the imaginary parts,
 * every plane with the same stride ps (the paper keeps real and imaginary parts in separate
 * arrays, end of Section 2).  On complex data the transpose of Algorithm 2 becomes the
 * Hermitian transpose (Section 3).
 *
 * Householder vector of a complex column x (length L, x1 = |x1| e^{i theta}; theta = 0 when
 * x1 = 0): sigma = sum_{i>1} |x_i|^2; if sigma = 0 the reflector is the identity (beta = 0,
 * R_jj = x1 kept).  Otherwise mu = sqrt(|x1|^2 + sigma), and Golub-Van Loan 5.1.1 is applied
 * to the modulus |x1| and rotated by the phase of x1: nu = |x1| - mu computed as
 * -sigma/(|x1| + mu) when |x1| > 0 (else nu = -mu), v1 = e^{i theta} nu, beta = 2 nu^2 /
 * (sigma + nu^2), v = x / v1.  Then H = I - beta v v^H is Hermitian and unitary and
 * H x = e^{i theta} mu e_1, so R_jj = e^{i theta} mu; on real data with x1 > 0 this is the real
 * reflector.
 */
typedef struct {
    double re[ORC_MAXP], im[ORC_MAXP];
} cmd;

static inline void cld(int P, const double *X, long ps, long off, cmd *v)
{
    ldm(P, X, ps, off, v->re);
    ldm(P, X + (long)P * ps, ps, off, v->im);
}

static inline void cst(int P, double *X, long ps, long off, const cmd *v)
{
    stm(P, X, ps, off, v->re);
    stm(P, X + (long)P * ps, ps, off, v->im);
}

static int cmd_is_zero(int P, const cmd *a) { return md_is_zero(P, a->re) && md_is_zero(P, a->im); }

/* r = op(a) * b with op(a) = a or conj(a); each part summed exactly, then truncated */
static void cmd_mul_x(int P, const cmd *a, int conj_a, const cmd *b, cmd *r)
{
    const double sa = conj_a ? -1.0 : 1.0;
    cmd t;
    xacc x;
    xacc_init(&x);
    xacc_add_prod(&x, P, a->re, P, b->re, 1.0);
    xacc_add_prod(&x, P, a->im, P, b->im, -sa);
    xacc_round(&x, P, t.re);
    xacc_init(&x);
    xacc_add_prod(&x, P, a->re, P, b->im, 1.0);
    xacc_add_prod(&x, P, a->im, P, b->re, sa);
    xacc_round(&x, P, t.im);
    *r = t;
}

static void cmd_add(int P, const cmd *a, const cmd *b, cmd *r)
{
    orc_md_add(P, a->re, b->re, r->re);
    orc_md_add(P, a->im, b->im, r->im);
}

static void cmd_sub(int P, const cmd *a, const cmd *b, cmd *r)
{
    orc_md_sub(P, a->re, b->re, r->re);
    orc_md_sub(P, a->im, b->im, r->im);
}

/* |a|^2, summed exactly, then truncated */
static void cmd_abs2(int P, const cmd *a, double *r)
{
    xacc x;
    xacc_init(&x);
    xacc_add_prod(&x, P, a->re, P, a->re, 1.0);
    xacc_add_prod(&x, P, a->im, P, a->im, 1.0);
    xacc_round(&x, P, r);
}

/* a * s for a real multiple double s */
static void cmd_scale(int P, const cmd *a, const double *s, cmd *r)
{
    cmd t;
    orc_md_mul(P, a->re, s, t.re);
    orc_md_mul(P, a->im, s, t.im);
    *r = t;
}

/* a / b = (a conj(b)) / |b|^2 */
static void cmd_div(int P, const cmd *a, const cmd *b, cmd *r)
{
    double d[ORC_MAXP];
    cmd n;
    cmd_abs2(P, b, d);
    cmd_mul_x(P, b, 1, a, &n);  /* conj(b) a */
    orc_md_div(P, n.re, d, r->re);
    orc_md_div(P, n.im, d, r->im);
}

/* scalar entry points for tests: a, b, r hold 2P doubles (P real limbs, then P imaginary) */
void orc_cmd_mul(int P, const double *a, const double *b, double *r)
{
    cmd x, y, z;
    memcpy(x.re, a, sizeof(double) * P);
    memcpy(x.im, a + P, sizeof(double) * P);
    memcpy(y.re, b, sizeof(double) * P);
    memcpy(y.im, b + P, sizeof(double) * P);
    cmd_mul_x(P, &x, 0, &y, &z);
    memcpy(r, z.re, sizeof(double) * P);
    memcpy(r + P, z.im, sizeof(double) * P);
}

void orc_cmd_div(int P, const double *a, const double *b, double *r)
{
    cmd x, y, z;
    memcpy(x.re, a, sizeof(double) * P);
    memcpy(x.im, a + P, sizeof(double) * P);
    memcpy(y.re, b, sizeof(double) * P);
    memcpy(y.im, b + P, sizeof(double) * P);
    cmd_div(P, &x, &y, &z);
    memcpy(r, z.re, sizeof(double) * P);
    memcpy(r + P, z.im, sizeof(double) * P);
}

/* B(j:m, c) := H B(j:m, c) for c in [c0, c1), H = I - beta v v^H with v = (1, A(j+1:m, j)) */
static void capply_reflector(int P, int m, int j, const double *A, int lda, long psa, const double *bt, double *B,
                             int ldb, long psb, int c0, int c1)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int c = c0; c < c1; c++) {
        cmd w, a, v, p, t;
        cld(P, B, psb, AT(j, c, ldb), &w); /* v_j = 1 */
        for (int i = j + 1; i < m; i++) {
            cld(P, A, psa, AT(i, j, lda), &v);
            cld(P, B, psb, AT(i, c, ldb), &a);
            cmd_mul_x(P, &v, 1, &a, &p); /* conj(v_i) a_i */
            cmd_add(P, &w, &p, &w);
        }
        cmd_scale(P, &w, bt, &t); /* t = beta v^H b */
        cld(P, B, psb, AT(j, c, ldb), &a);
        cmd_sub(P, &a, &t, &a);
        cst(P, B, psb, AT(j, c, ldb), &a);
        for (int i = j + 1; i < m; i++) {
            cld(P, A, psa, AT(i, j, lda), &v);
            cld(P, B, psb, AT(i, c, ldb), &a);
            cmd_mul_x(P, &v, 0, &t, &p);
            cmd_sub(P, &a, &p, &a);
            cst(P, B, psb, AT(i, c, ldb), &a);
        }
    }
}

/*
 * Unblocked complex Householder QR of the m x n matrix A (m >= n), in place: R in the upper
 * triangle, v_j below the diagonal of column j (unit first entry implicit), beta (P planes of
 * stride n, real).  tally counts real multiple-double operations (a complex product is 4
 * multiplications and 2 additions, a complex sum 2 additions, |z|^2 2 multiplications and
 * 1 addition, a complex quotient 6 multiplications, 3 additions and 2 divisions).
 */
int orc_cqr(int P, int m, int n, double *A, int lda, long ps, double *beta, long *tally, int nthreads)
{
    if (!valid_p(P) || m < n || n < 0 || lda < m)
        return -1;
    set_threads(nthreads);
    for (int j = 0; j < n; j++) {
        double sig[ORC_MAXP], t1[ORC_MAXP], t2[ORC_MAXP], a2[ORC_MAXP], mu[ORC_MAXP], rho[ORC_MAXP];
        double nu[ORC_MAXP], bt[ORC_MAXP];
        cmd alpha, ph, v1, x, r;
        long L = m - j;
        memset(sig, 0, sizeof(sig));
        for (int i = j + 1; i < m; i++) {
            cld(P, A, ps, AT(i, j, lda), &x);
            cmd_abs2(P, &x, t1);
            orc_md_add(P, sig, t1, sig);
        }
        tally_add(tally, 2 * (L - 1), 2 * (L - 1), 0, 0);
        cld(P, A, ps, AT(j, j, lda), &alpha);
        if (md_is_zero(P, sig)) {
            memset(bt, 0, sizeof(bt));
            stm(P, beta, n, j, bt);
            continue;
        }
        cmd_abs2(P, &alpha, a2);
        orc_md_add(P, a2, sig, t1);
        orc_md_sqrt(P, t1, mu);
        orc_md_sqrt(P, a2, rho);
        tally_add(tally, 2, 2, 0, 2);
        memset(&ph, 0, sizeof(ph));
        if (md_is_zero(P, rho)) {
            ph.re[0] = 1.0;
            md_neg(P, mu, nu);
        } else {
            orc_md_div(P, alpha.re, rho, ph.re);
            orc_md_div(P, alpha.im, rho, ph.im);
            orc_md_add(P, rho, mu, t1);
            orc_md_div(P, sig, t1, t2);
            md_neg(P, t2, nu);
            tally_add(tally, 1, 0, 3, 0);
        }
        cmd_scale(P, &ph, nu, &v1);
        orc_md_mul(P, nu, nu, t1);  /* nu^2 */
        orc_md_add(P, sig, t1, t2); /* sigma + nu^2 */
        for (int k = 0; k < P; k++)
            t1[k] *= 2.0; /* exact */
        orc_md_div(P, t1, t2, bt);
        tally_add(tally, 1, 3, 1, 0);
        stm(P, beta, n, j, bt);
        for (int i = j + 1; i < m; i++) {
            cld(P, A, ps, AT(i, j, lda), &x);
            cmd_div(P, &x, &v1, &r);
            cst(P, A, ps, AT(i, j, lda), &r);
        }
        tally_add(tally, 3 * (L - 1), 6 * (L - 1), 2 * (L - 1), 0);
        cmd_scale(P, &ph, mu, &r);
        cst(P, A, ps, AT(j, j, lda), &r);
        tally_add(tally, 0, 2, 0, 0);
        capply_reflector(P, m, j, A, lda, ps, bt, A, lda, ps, j + 1, n);
        /* per column: L-1 conj products and sums, 1 scale, 1 sum, L-1 products and sums */
        tally_add(tally, (long)(n - j - 1) * (8 * (L - 1) + 2), (long)(n - j - 1) * (8 * (L - 1) + 2), 0, 0);
    }
    return 0;
}

/* B := Q^H B = H_{n-1} ... H_0 B for the m x nrhs complex matrix B */
int orc_capply_qh(int P, int m, int n, const double *A, int lda, long psa, const double *beta, double *B, int ldb,
                  long psb, int nrhs, long *tally, int nthreads)
{
    if (!valid_p(P) || m < n || lda < m || ldb < m || nrhs < 0)
        return -1;
    set_threads(nthreads);
    for (int j = 0; j < n; j++) {
        double bt[ORC_MAXP];
        ldm(P, beta, n, j, bt);
        if (md_is_zero(P, bt))
            continue;
        capply_reflector(P, m, j, A, lda, psa, bt, B, ldb, psb, 0, nrhs);
        tally_add(tally, (long)nrhs * (8 * (m - j - 1) + 2), (long)nrhs * (8 * (m - j - 1) + 2), 0, 0);
    }
    return 0;
}

/* Solve R x = y (complex, leading n x n upper triangle), rows n-1 down to 0, ascending k in
 * each row sum.  info = smallest 1-based i with R_ii == 0 (then x is not computed). */
int orc_cbacksub(int P, int n, const double *R, int ldr, long psr, const double *y, long ys, double *x, long xs,
                 int *info, long *tally)
{
    cmd d, s, r, xk, p;
    if (!valid_p(P) || n < 0 || ldr < n)
        return -1;
    *info = 0;
    for (int i = 0; i < n; i++) {
        cld(P, R, psr, AT(i, i, ldr), &d);
        if (cmd_is_zero(P, &d)) {
            *info = i + 1;
            return 0;
        }
    }
    for (int i = n - 1; i >= 0; i--) {
        cld(P, y, ys, i, &s);
        for (int k = i + 1; k < n; k++) {
            cld(P, R, psr, AT(i, k, ldr), &r);
            cld(P, x, xs, k, &xk);
            cmd_mul_x(P, &r, 0, &xk, &p);
            cmd_sub(P, &s, &p, &s);
        }
        cld(P, R, psr, AT(i, i, ldr), &d);
        cmd_div(P, &s, &d, &p);
        cst(P, x, xs, i, &p);
    }
    tally_add(tally, (long)n * (n - 1) / 2 * 4 + 3L * n, (long)n * (n - 1) / 2 * 4 + 6L * n, 2L * n, 0);
    return 0;
}

/* Complex least squares: QR of A (in place), b := Q^H b (in place), x from R x = b(0:n). */
int orc_clstsq(int P, int m, int n, double *A, int lda, long psa, double *b, long bs, double *x, long xs,
               double *beta, int *info, long *tally, int nthreads)
{
    int rc = orc_cqr(P, m, n, A, lda, psa, beta, tally, nthreads);
    if (rc)
        return rc;
    rc = orc_capply_qh(P, m, n, A, lda, psa, beta, b, m, bs, 1, tally, nthreads);
    if (rc)
        return rc;
    return orc_cbacksub(P, n, A, lda, psa, b, bs, x, xs, info, tally);
}

/* Explicit m x m unitary Q = H_0 H_1 ... H_{n-1}, by backward accumulation onto I. */
int orc_cexplicit_q(int P, int m, int n, const double *A, int lda, long psa, const double *beta, double *Q, int ldq,
                    long psq, int nthreads)
{
    if (!valid_p(P) || m < n || lda < m || ldq < m)
        return -1;
    set_threads(nthreads);
    for (int k = 0; k < 2 * P; k++)
        for (int c = 0; c < m; c++)
            for (int i = 0; i < m; i++)
                Q[(long)k * psq + AT(i, c, ldq)] = (k == 0 && i == c) ? 1.0 : 0.0;
    for (int j = n - 1; j >= 0; j--) {
        double bt[ORC_MAXP];
        ldm(P, beta, n, j, bt);
        if (md_is_zero(P, bt))
            continue;
        capply_reflector(P, m, j, A, lda, psa, bt, Q, ldq, psq, j, m);
    }
    return 0;
}

/*
 * Complex y := op(A) x  or  y := c - op(A) x  (when c != NULL), op(A) = A (trans == 0) or
 * A^H (trans != 0); each part of each output accumulated EXACTLY and truncated to Py limbs.
 */
int orc_cmatvec(int trans, int Pa, int Px, int Pc, int Py, int rows, int cols, const double *A, int lda, long psa,
                const double *x, long xs, const double *c, long cs, double *y, long ys, int nthreads)
{
    if (!valid_p(Pa) || !valid_p(Px) || !valid_p(Py) || (c && !valid_p(Pc)) || lda < rows)
        return -1;
    set_threads(nthreads);
    int nout = trans ? cols : rows;
    int nin = trans ? rows : cols;
    const double sa = trans ? -1.0 : 1.0; /* sign of Im(A) in op(A) */
#pragma omp parallel for schedule(dynamic, 4)
    for (int o = 0; o < nout; o++) {
        double ar[ORC_MAXP], ai[ORC_MAXP], xr[ORC_MAXP], xi[ORC_MAXP], out[ORC_MAXP];
        xacc *re = (xacc *)malloc(sizeof(xacc));
        xacc *im = (xacc *)malloc(sizeof(xacc));
        xacc_init(re);
        xacc_init(im);
        double sign = 1.0;
        if (c) {
            double cv[ORC_MAXP];
            ldm(Pc, c, cs, o, cv);
            xacc_add_md(re, Pc, cv, 1.0);
            ldm(Pc, c + (long)Pc * cs, cs, o, cv);
            xacc_add_md(im, Pc, cv, 1.0);
            sign = -1.0;
        }
        for (int k = 0; k < nin; k++) {
            long off = trans ? AT(k, o, lda) : AT(o, k, lda);
            ldm(Pa, A, psa, off, ar);
            ldm(Pa, A + (long)Pa * psa, psa, off, ai);
            ldm(Px, x, xs, k, xr);
            ldm(Px, x + (long)Px * xs, xs, k, xi);
            xacc_add_prod(re, Pa, ar, Px, xr, sign);
            xacc_add_prod(re, Pa, ai, Px, xi, -sa * sign);
            xacc_add_prod(im, Pa, ar, Px, xi, sign);
            xacc_add_prod(im, Pa, ai, Px, xr, sa * sign);
        }
        xacc_round(re, Py, out);
        stm(Py, y, ys, o, out);
        xacc_round(im, Py, out);
        stm(Py, y + (long)Py * ys, ys, o, out);
        free(re);
        free(im);
    }
    return 0;
}

/* Table-1-free bookkeeping helper for tests: number of compiled-in limbs supported. */
int orc_max_limbs(void) { return ORC_MAXP; }
