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
// and a top-down TwoSum pass) turns it back into P limbs.  Reciprocal, square root and
// reciprocal square root use Newton steps that double the number of limbs (1 -> 2 -> 4 -> 8),
// each with its residual formed to full length and its correction to half length.
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
        // Exact cancellation at the top leaves zero limbs between nonzero ones (e.g.
        // [s, 0, e, 0]); move them to the end (odd-even transposition, branch-free) so that
        // limb 0 always leads and truncation keeps the significant limbs.
#pragma unroll
        for (int pass = 0; pass < P; ++pass) {
#pragma unroll
            for (int i = pass & 1; i + 1 < P; i += 2) {
                const bool z = (r.x[i] == 0.0);
                const double hi = z ? r.x[i + 1] : r.x[i];
                const double lo = z ? 0.0 : r.x[i + 1];
                r.x[i] = hi;
                r.x[i + 1] = lo;
            }
        }
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

// Renormalise twice: merges the overlapping limbs a first pass can leave after cancellation
// (e.g. [e, -4e', e', 0] with e' ~ ulp(e)); used where a value is truncated afterwards.
template <int P>
MDQ V<P> acc_get_strict(const Acc<P> &a)
{
    const V<P> v = acc_get(a);
    double t[P];
#pragma unroll
    for (int k = 0; k < P; ++k) t[k] = v.x[k];
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
// s += a*b with a of NA limbs and b of NB limbs (NA, NB <= P); only the products
// a_i b_j with i + j <= P - 1 are formed, as TwoProd pairs up to level P - 2 and as plain
// FMAs at level P - 1.  HAS_S = false means s is zero on entry (a plain product).  Level L
// sums, in this order, s_L, the products of level L and the NC terms carried from level
// L - 1 with a TwoSum chain; the chain's rounding errors and the TwoProd errors of level L
// are carried to level L + 1.
template <int P, int NA, int NB, int L, int NC, bool HAS_S>
MDQ void casc_fma(double (&s)[P], const double *a, const double *b, const double *carry)
{
    constexpr int ILO = (L - NB + 1 > 0) ? (L - NB + 1) : 0;
    constexpr int IHI = (L < NA - 1) ? L : (NA - 1);
    constexpr int NP = (IHI >= ILO) ? (IHI - ILO + 1) : 0;
    if constexpr (L == P - 1) {
        double t;
        if constexpr (HAS_S)
            t = s[L];
        else if constexpr (NC > 0)
            t = carry[0];
        else
            t = 0.0;
        constexpr int K0 = (!HAS_S && NC > 0) ? 1 : 0;
#pragma unroll
        for (int k = K0; k < NC; ++k) t += carry[k];
#pragma unroll
        for (int i = ILO; i <= IHI; ++i) t = __builtin_fma(a[i], b[L - i], t);
        s[L] = t;
    } else {
        constexpr int NT = (HAS_S ? 1 : 0) + NP + NC;
        constexpr int NSE = (NT > 0) ? NT - 1 : 0;  // TwoSum errors
        constexpr int NOUT = NSE + NP;
        double out[NOUT > 0 ? NOUT : 1];
        double tm[NT > 0 ? NT : 1];
        constexpr int Q0 = HAS_S ? 1 : 0;
        if constexpr (HAS_S) tm[0] = s[L];
#pragma unroll
        for (int i = ILO; i <= IHI; ++i) two_prod(a[i], b[L - i], tm[Q0 + i - ILO], out[NSE + i - ILO]);
#pragma unroll
        for (int k = 0; k < NC; ++k) tm[Q0 + NP + k] = carry[k];
        double t = (NT > 0) ? tm[0] : 0.0;
#pragma unroll
        for (int k = 1; k < NT; ++k) two_sum(t, tm[k], t, out[k - 1]);
        s[L] = t;
        casc_fma<P, NA, NB, L + 1, NOUT, HAS_S>(s, a, b, out);
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

template <int P>
MDQ void acc_fma(Acc<P> &acc, const V<P> &a, const V<P> &b)
{
    casc_fma<P, P, P, 0, 0, true>(acc.s, a.x, b.x, nullptr);
}

template <int P>
MDQ void acc_add(Acc<P> &acc, const V<P> &b)
{
    casc_add<P, 0, 0>(acc.s, b.x, nullptr);
}

template <int P>
MDQ void acc_fma_d(Acc<P> &acc, double q, const V<P> &b)
{
    casc_fma<P, 1, P, 0, 0, true>(acc.s, &q, b.x, nullptr);
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
    casc_fma<P, P, P, 0, 0, false>(t.s, a.x, b.x, nullptr);
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

// Concatenate a P/2-limb value and a P/2-limb correction lying just below it, renormalise.
template <int P>
MDQ V<P> join_halves(const V<P / 2> &hi, const V<P / 2> &lo)
{
    double t[P];
#pragma unroll
    for (int k = 0; k < P / 2; ++k) {
        t[k] = hi.x[k];
        t[P / 2 + k] = lo.x[k];
    }
    return renorm<P, P>(t);
}

// 1/b.  Limb-doubling Newton step (Karp and Markstein, "High-precision division and square
// root", ACM TOMS 1997): with y ~ 1/b to P/2 limbs, the residual e = 1 - b y is formed to P
// limbs (it is about 2^(-26P) relative, so only its top P/2 limbs matter) and the correction
// y e is a P/2-limb product: y + y e is 1/b to P limbs.
template <int P>
MDQ V<P> recip(const V<P> &b)
{
    if constexpr (P == 1) {
        V<1> r;
        r.x[0] = 1.0 / b.x[0];
        return r;
    } else {
        constexpr int H = P / 2;
        const V<H> y = recip<H>(resize<H>(b));
        Acc<P> e = acc_from(from_double<P>(1.0));
        const V<P> nb = neg(b);
        casc_fma<P, P, H, 0, 0, true>(e.s, nb.x, y.x, nullptr);
        const V<H> eh = resize<H>(acc_get_strict(e));
        return join_halves<P>(y, mul(y, eh));
    }
}

template <int P>
MDQ V<P> div(const V<P> &a, const V<P> &b)
{
    return mul(a, recip(b));
}

// 1/sqrt(a), a > 0: y + y (1 - a y^2) / 2 with y to P/2 limbs, the residual to P limbs and
// the correction as a P/2-limb product.
template <int P>
MDQ V<P> rsqrt(const V<P> &a)
{
    if constexpr (P == 1) {
        V<1> r;
        r.x[0] = 1.0 / sqrt(a.x[0]);
        return r;
    } else {
        constexpr int H = P / 2;
        const V<H> y = rsqrt<H>(resize<H>(a));
        Acc<P> y2a;
        casc_fma<P, H, H, 0, 0, false>(y2a.s, y.x, y.x, nullptr);
        const V<P> y2 = acc_get_strict(y2a);  // y^2 to P limbs
        Acc<P> e = acc_from(from_double<P>(1.0));
        const V<P> na = neg(a);
        casc_fma<P, P, P, 0, 0, true>(e.s, na.x, y2.x, nullptr);
        const V<H> eh = scale(resize<H>(acc_get_strict(e)), 0.5);
        return join_halves<P>(y, mul(y, eh));
    }
}

// sqrt(a), a >= 0 (zero maps to zero).  Karp-Markstein: s = a y to P/2 limbs with
// y = 1/sqrt(a) to P/2 limbs, the residual a - s^2 to P limbs, and the correction
// (a - s^2) y / 2 as a P/2-limb product.
template <int P>
MDQ V<P> sqrt_md(const V<P> &a)
{
    if (a.x[0] <= 0.0) return zero<P>();
    if constexpr (P == 1) {
        V<1> r;
        r.x[0] = sqrt(a.x[0]);
        return r;
    } else {
        constexpr int H = P / 2;
        const V<H> ah = resize<H>(a);
        const V<H> y = rsqrt<H>(ah);
        const V<H> sh = mul(ah, y);
        Acc<P> r = acc_from(a);
        const V<H> nsh = neg(sh);
        casc_fma<P, H, H, 0, 0, true>(r.s, nsh.x, sh.x, nullptr);
        const V<H> rh = resize<H>(acc_get_strict(r));
        return join_halves<P>(sh, mul(rh, scale(y, 0.5)));
    }
}

}  // namespace mdk
