// md.hpp -- multiple-double arithmetic for the GPU library (gfx950).
//
// A multiple double of P limbs is an unevaluated sum x[0] + x[1] + ... + x[P-1] of doubles,
// limb 0 most significant (paper Section 1.1; P = 2, 4, 8 give double double, quad double
// and octo double, about 32, 64 and 128 decimal places).  Limbs are stored as P separate
// doubles, never as an array indexed at run time, so every limb lives in a register.
//
// Building blocks are the error-free transforms TwoSum (Knuth), FastTwoSum (Dekker) and
// TwoProd with a fused multiply-add.  On top of them sits a "level cascade": the exact
// terms of c + a*b are grouped by significance level l (a_i*b_j with i + j = l, the TwoProd
// errors of level l-1, limb c_l and the rounding errors carried up from level l-1), each
// level is summed with a TwoSum chain whose errors move down one level, and the last level
// is summed with plain additions and FMAs.  The P level sums form a lazy accumulator that
// a dot product keeps across many terms; one renormalisation (two bottom-up VecSum passes
// and a top-down TwoSum pass) turns it back into P limbs.  Reciprocal and reciprocal square
// root use Newton iterations that double the number of limbs at each step (one step per
// doubling), so their cost is dominated by the last, full-precision step.
//
// Accuracy contract (normwise): for add/fma the error is a small multiple of
// 2^(-53P) * (|c| + |a*b|); for mul, recip, div and sqrt it is a small multiple of
// 2^(-53P) relative.  Outputs are normalised to |x[k+1]| <= ulp(x[k]).
//
// Everything is __host__ __device__ so the same code can be compiled for the host and
// checked against the CPU oracle.  Compile with -ffp-contract=off: the transforms rely on
// every + and * being rounded separately.
#pragma once

#ifdef __HIPCC__
#include <hip/hip_runtime.h>
#define MDQ __host__ __device__ __forceinline__
#else
#include <cmath>
#define MDQ inline
#endif

namespace mdk {

template <int P>
struct V {
    double x[P];
};

template <int P>
struct Acc {  // lazy level sums, not normalised
    double s[P];
};

// ------------------------------------------------------------------ error-free transforms
MDQ void two_sum(double a, double b, double &s, double &e)
{
    double t = a + b;
    double bb = t - a;
    e = (a - (t - bb)) + (b - bb);
    s = t;
}

MDQ void fast_two_sum(double a, double b, double &s, double &e)
{
    double t = a + b;
    e = b - (t - a);
    s = t;
}

MDQ void two_prod(double a, double b, double &p, double &e)
{
    double t = a * b;
    e = __builtin_fma(a, b, -t);
    p = t;
}

// ------------------------------------------------------------------ constructors
template <int P>
MDQ V<P> zero()
{
    V<P> r;
#pragma unroll
    for (int k = 0; k < P; ++k) r.x[k] = 0.0;
    return r;
}

template <int P>
MDQ V<P> from_double(double d)
{
    V<P> r = zero<P>();
    r.x[0] = d;
    return r;
}

template <int P>
MDQ V<P> neg(const V<P> &a)
{
    V<P> r;
#pragma unroll
    for (int k = 0; k < P; ++k) r.x[k] = -a.x[k];
    return r;
}

// multiply by a power of two (exact unless a limb under/overflows)
template <int P>
MDQ V<P> scale(const V<P> &a, double pow2)
{
    V<P> r;
#pragma unroll
    for (int k = 0; k < P; ++k) r.x[k] = a.x[k] * pow2;
    return r;
}

template <int Q, int P>
MDQ V<Q> resize(const V<P> &a)
{
    V<Q> r;
#pragma unroll
    for (int k = 0; k < Q; ++k) r.x[k] = (k < P) ? a.x[k] : 0.0;
    return r;
}

template <int P>
MDQ bool is_zero(const V<P> &a)
{
    bool z = true;
#pragma unroll
    for (int k = 0; k < P; ++k) z = z && (a.x[k] == 0.0);
    return z;
}

// ------------------------------------------------------------------ renormalisation
// N doubles of roughly decreasing magnitude (possibly overlapping, possibly cancelling at
// the top) -> P normalised limbs with the same sum up to the dropped tail.
template <int N, int P>
MDQ V<P> renorm(double (&x)[N])
{
    static_assert(N >= P, "renorm needs at least P inputs");
    V<P> r;
    if constexpr (P == 1) {
        double s = x[N - 1];
#pragma unroll
        for (int i = N - 2; i >= 0; --i) s = x[i] + s;
        r.x[0] = s;
    } else if constexpr (N == 2) {
        two_sum(x[0], x[1], r.x[0], r.x[1]);
    } else {
#pragma unroll
        for (int pass = 0; pass < 2; ++pass) {
            double s = x[N - 1];
#pragma unroll
            for (int i = N - 2; i >= 0; --i) two_sum(x[i], s, s, x[i + 1]);
            x[0] = s;
        }
        double eps = x[0];
#pragma unroll
        for (int i = 1; i < P; ++i) two_sum(eps, x[i], r.x[i - 1], eps);
#pragma unroll
        for (int i = P; i < N; ++i) eps += x[i];
        r.x[P - 1] = eps;
    }
    return r;
}

template <int P>
MDQ V<P> acc_get(const Acc<P> &a)
{
    double t[P];
#pragma unroll
    for (int k = 0; k < P; ++k) t[k] = a.s[k];
    return renorm<P, P>(t);
}

template <int P>
MDQ Acc<P> acc_from(const V<P> &c)
{
    Acc<P> a;
#pragma unroll
    for (int k = 0; k < P; ++k) a.s[k] = c.x[k];
    return a;
}

template <int P>
MDQ Acc<P> acc_zero()
{
    Acc<P> a;
#pragma unroll
    for (int k = 0; k < P; ++k) a.s[k] = 0.0;
    return a;
}

// ------------------------------------------------------------------ level cascades
// s += a*b.  HAS_S = false means s is zero on entry (plain product).
template <int P, int L, int NC, bool HAS_S>
MDQ void casc_fma(double (&s)[P], const double (&a)[P], const double (&b)[P], const double *carry)
{
    if constexpr (L == P - 1) {
        double t;
        if constexpr (HAS_S) {
            t = s[L];
#pragma unroll
            for (int k = 0; k < NC; ++k) t += carry[k];
        } else {
            t = (NC > 0) ? carry[0] : 0.0;
#pragma unroll
            for (int k = 1; k < NC; ++k) t += carry[k];
        }
#pragma unroll
        for (int i = 0; i <= L; ++i) t = __builtin_fma(a[i], b[L - i], t);
        s[L] = t;
    } else {
        constexpr int NP = L + 1;
        constexpr int NOUT = NC + 2 * NP - (HAS_S ? 0 : 1);
        double out[NOUT];
        double t;
        int o = 0;
        double pe0;
        two_prod(a[0], b[L], t, pe0);
        if constexpr (HAS_S) {
            two_sum(s[L], t, t, out[o]);
            ++o;
        }
        out[o++] = pe0;
#pragma unroll
        for (int i = 1; i <= L; ++i) {
            double p, pe;
            two_prod(a[i], b[L - i], p, pe);
            two_sum(t, p, t, out[o]);
            ++o;
            out[o++] = pe;
        }
#pragma unroll
        for (int k = 0; k < NC; ++k) {
            two_sum(t, carry[k], t, out[o]);
            ++o;
        }
        s[L] = t;
        casc_fma<P, L + 1, NOUT, HAS_S>(s, a, b, out);
    }
}

// s += b
template <int P, int L, int NC>
MDQ void casc_add(double (&s)[P], const double (&b)[P], const double *carry)
{
    if constexpr (L == P - 1) {
        double t = s[L] + b[L];
#pragma unroll
        for (int k = 0; k < NC; ++k) t += carry[k];
        s[L] = t;
    } else {
        constexpr int NOUT = NC + 1;
        double out[NOUT];
        double t;
        two_sum(s[L], b[L], t, out[0]);
#pragma unroll
        for (int k = 0; k < NC; ++k) two_sum(t, carry[k], t, out[k + 1]);
        s[L] = t;
        casc_add<P, L + 1, NOUT>(s, b, out);
    }
}

// s += q*b with q a double
template <int P, int L, int NC>
MDQ void casc_fma_d(double (&s)[P], double q, const double (&b)[P], const double *carry)
{
    if constexpr (L == P - 1) {
        double t = s[L];
#pragma unroll
        for (int k = 0; k < NC; ++k) t += carry[k];
        s[L] = __builtin_fma(q, b[L], t);
    } else {
        constexpr int NOUT = NC + 2;
        double out[NOUT];
        double t, p;
        two_prod(q, b[L], p, out[0]);
        two_sum(s[L], p, t, out[1]);
#pragma unroll
        for (int k = 0; k < NC; ++k) two_sum(t, carry[k], t, out[k + 2]);
        s[L] = t;
        casc_fma_d<P, L + 1, NOUT>(s, q, b, out);
    }
}

template <int P>
MDQ void acc_fma(Acc<P> &acc, const V<P> &a, const V<P> &b)
{
    casc_fma<P, 0, 0, true>(acc.s, a.x, b.x, nullptr);
}

template <int P>
MDQ void acc_add(Acc<P> &acc, const V<P> &b)
{
    casc_add<P, 0, 0>(acc.s, b.x, nullptr);
}

template <int P>
MDQ void acc_fma_d(Acc<P> &acc, double q, const V<P> &b)
{
    casc_fma_d<P, 0, 0>(acc.s, q, b.x, nullptr);
}

// Long accumulations renormalise the level sums every kLazy<P> terms: left alone, the lower
// levels grow with the term count and the plain additions of the last level lose bits
// (measured on a 300-term octo-double dot product: 2^-408 relative without, 2^-425 with a
// renormalisation every 4 terms; double double needs none).
template <int P>
constexpr int kLazy = (P <= 2) ? 64 : (P == 4 ? 16 : 4);

// acc += a*b as term number i of a long accumulation
template <int P>
MDQ void acc_fma_step(Acc<P> &acc, const V<P> &a, const V<P> &b, int i)
{
    acc_fma(acc, a, b);
    if (((i + 1) % kLazy<P>) == 0) acc = acc_from(acc_get(acc));
}

// ------------------------------------------------------------------ basic operations
template <int P>
MDQ V<P> add(const V<P> &a, const V<P> &b)
{
    Acc<P> t = acc_from(a);
    acc_add(t, b);
    return acc_get(t);
}

template <int P>
MDQ V<P> sub(const V<P> &a, const V<P> &b)
{
    return add(a, neg(b));
}

template <int P>
MDQ V<P> mul(const V<P> &a, const V<P> &b)
{
    Acc<P> t;
    casc_fma<P, 0, 0, false>(t.s, a.x, b.x, nullptr);
    return acc_get(t);
}

// c + a*b
template <int P>
MDQ V<P> fma(const V<P> &c, const V<P> &a, const V<P> &b)
{
    Acc<P> t = acc_from(c);
    acc_fma(t, a, b);
    return acc_get(t);
}

// a * q, q a double
template <int P>
MDQ V<P> mul_d(const V<P> &a, double q)
{
    Acc<P> t = acc_zero<P>();
    acc_fma_d(t, q, a);
    return acc_get(t);
}

// 1/b: Newton y <- y + y (1 - b y), one step per doubling of the limb count.
template <int P>
MDQ V<P> recip(const V<P> &b)
{
    if constexpr (P == 1) {
        V<1> r;
        r.x[0] = 1.0 / b.x[0];
        return r;
    } else {
        V<P> y = resize<P>(recip<P / 2>(resize<P / 2>(b)));
        Acc<P> e = acc_from(from_double<P>(1.0));
        acc_fma(e, neg(b), y);
        V<P> ev = acc_get(e);  // 1 - b y, about 2^(-26P) relative
        return fma(y, y, ev);
    }
}

template <int P>
MDQ V<P> div(const V<P> &a, const V<P> &b)
{
    return mul(a, recip(b));
}

// 1/sqrt(a), a > 0: Newton y <- y + y (1 - a y^2) / 2, one step per doubling.
template <int P>
MDQ V<P> rsqrt(const V<P> &a)
{
    if constexpr (P == 1) {
        V<1> r;
        r.x[0] = 1.0 / sqrt(a.x[0]);
        return r;
    } else {
        V<P> y = resize<P>(rsqrt<P / 2>(resize<P / 2>(a)));
        V<P> y2 = mul(y, y);
        Acc<P> e = acc_from(from_double<P>(1.0));
        acc_fma(e, neg(a), y2);
        V<P> ev = scale(acc_get(e), 0.5);
        return fma(y, y, ev);
    }
}

// sqrt(a), a >= 0 (zero maps to zero)
template <int P>
MDQ V<P> sqrt_md(const V<P> &a)
{
    if (a.x[0] <= 0.0) return zero<P>();
    if constexpr (P == 1) {
        V<1> r;
        r.x[0] = sqrt(a.x[0]);
        return r;
    } else {
        return mul(a, rsqrt(a));
    }
}

}  // namespace mdk
