// mdls_cplx.hpp -- complex multiple-double least squares on gfx950: Householder QR with the
// Hermitian transpose in place of the transpose (paper Section 3, text after the W
// recurrence), Q^H b and the tiled back substitution (Section 2, Algorithm 1) on complex
// numbers; the paper's complex workload is the double double QR of Section 4, Table 5.
//
// Storage: a complex matrix is 2P planes, the P limb planes of the real parts followed by
// the P limb planes of the imaginary parts (the paper keeps real and imaginary parts in
// separate arrays, end of Section 2); every plane has the same stride ps and is column-major
// with leading dimension ld.  A complex vector of length L is 2P planes of L doubles.
//
// Householder vector of a column x (x1 = |x1| e^{i theta}, theta = 0 when x1 = 0): with
// sigma = sum_{i>1} |x_i|^2 and mu = sqrt(|x1|^2 + sigma), the Golub-Van Loan 5.1.1 choice is
// made on the modulus and rotated by the phase: nu = -sigma/(|x1| + mu) (nu = -mu when
// x1 = 0), v1 = e^{i theta} nu, beta = 2 nu^2/(sigma + nu^2), v = x/v1, and R_jj =
// e^{i theta} mu; sigma = 0 gives beta = 0 and R_jj = x1.  H = I - beta v v^H is Hermitian.
//
// Kernels (one QR panel of b = tile columns at a time):
//   k_cpanel  -- the whole panel in one persistent launch, one workgroup per column, each
//                column handed to the later ones through device memory behind a counter;
//   k_crefl   -- (the panel a launch per column instead) the reflector of its first column;
//   k_cstep   -- for panel column j: H_j applied to the panel columns right of j, one
//                workgroup per column; workgroup 0 then forms the reflector of column j+1
//                from the column it has just updated, so one launch per column carries the
//                panel's serial chain (k_cstep_r: the same with the rows in registers, for
//                columns of up to 4 x 256 rows in dd and qd);
//   k_cgram   -- G = Y^H Y (strictly upper part) of the panel;
//   k_cinvert -- T = (diag(1/beta) + triu(G, 1))^{-1} column-parallel, with the diagonal of
//                the inverse supplied as beta (so beta_j = 0 gives a zero row and column, the
//                identity reflector); also the diagonal tiles of R for the back substitution;
//                for tiles of 64 columns or more only their 32 x 32 diagonal blocks, and
//   k_cinv_blocks -- the blocks above those diagonal blocks, by block rows;
//   k_ctn, k_ctrmm_h, k_cnn_sub -- the trailing update C := (I - Y T^H Y^H) C, which is the
//                paper's C + Y W^H C with W = -Y T, and the same for Q^H B;
//   k_cbs_xi, k_cbs_upd -- x_i := U_i^{-1} b_i and b_j -= A_{j,i} x_i;
//   k_ctrmm_n, k_cidentity -- Q B and the explicit unitary factor (the blocks in reverse).
#pragma once
#include <atomic>

#include "mdls_impl.hpp"

namespace mdls_impl {

// ============================================================================ complex md values
template <int P>
struct CV {
    V<P> re, im;
};

template <int P>
struct CAcc {
    Acc<P> re, im;
};

// each complex multiply-add puts two terms into each part's accumulator
template <int P>
constexpr int kCLazy = (kLazy<P> / 2 > 0) ? kLazy<P> / 2 : 1;

template <int P>
__device__ __forceinline__ CV<P> czero()
{
    return CV<P>{zero<P>(), zero<P>()};
}

template <int P>
__device__ __forceinline__ CV<P> cone()
{
    return CV<P>{from_double<P>(1.0), zero<P>()};
}

template <int P>
__device__ __forceinline__ CV<P> cneg(const CV<P> &a)
{
    return CV<P>{neg(a.re), neg(a.im)};
}

template <int P>
__device__ __forceinline__ CV<P> cldm(const double *X, long ps, long off)
{
    return CV<P>{ldm<P>(X, ps, off), ldm<P>(X + (long)P * ps, ps, off)};
}

template <int P>
__device__ __forceinline__ void cstm(double *X, long ps, long off, const CV<P> &v)
{
    stm(X, ps, off, v.re);
    stm(X + (long)P * ps, ps, off, v.im);
}

template <int P>
__device__ __forceinline__ CV<P> clds_ld(const double *s)
{
    return CV<P>{lds_ld<P>(s), lds_ld<P>(s + P)};
}

template <int P>
__device__ __forceinline__ void clds_st(double *s, const CV<P> &v)
{
    lds_st(s, v.re);
    lds_st(s + P, v.im);
}

template <int P>
__device__ __forceinline__ CAcc<P> cacc_zero()
{
    return CAcc<P>{acc_zero<P>(), acc_zero<P>()};
}

template <int P>
__device__ __forceinline__ CAcc<P> cacc_from(const CV<P> &c)
{
    return CAcc<P>{acc_from(c.re), acc_from(c.im)};
}

template <int P>
__device__ __forceinline__ CV<P> cacc_get(const CAcc<P> &a)
{
    return CV<P>{acc_get(a.re), acc_get(a.im)};
}

// acc += op(a) b with op(a) = conj(a) when CONJ, else a
template <int P, bool CONJ>
__device__ __forceinline__ void cacc_fma(CAcc<P> &acc, const CV<P> &a, const CV<P> &b)
{
    const V<P> nai = neg(a.im);
    acc_fma(acc.re, a.re, b.re);
    acc_fma(acc.re, CONJ ? a.im : nai, b.im);
    acc_fma(acc.im, a.re, b.im);
    acc_fma(acc.im, CONJ ? nai : a.im, b.re);
}

// the same as term number i of a long accumulation
template <int P, bool CONJ>
__device__ __forceinline__ void cacc_fma_step(CAcc<P> &acc, const CV<P> &a, const CV<P> &b, int i)
{
    cacc_fma<P, CONJ>(acc, a, b);
    if (((i + 1) % kCLazy<P>) == 0) {
        acc.re = acc_from(acc_get(acc.re));
        acc.im = acc_from(acc_get(acc.im));
    }
}

template <int P>
__device__ __forceinline__ CV<P> cmul(const CV<P> &a, const CV<P> &b)
{
    CAcc<P> t = cacc_zero<P>();
    cacc_fma<P, false>(t, a, b);
    return cacc_get(t);
}

// c - a b
template <int P>
__device__ __forceinline__ CV<P> cfms(const CV<P> &c, const CV<P> &a, const CV<P> &b)
{
    CAcc<P> t = cacc_from(c);
    cacc_fma<P, false>(t, cneg(a), b);
    return cacc_get(t);
}

template <int P>
__device__ __forceinline__ CV<P> cadd(const CV<P> &a, const CV<P> &b)
{
    return CV<P>{add(a.re, b.re), add(a.im, b.im)};
}

// a s for a real s
template <int P>
__device__ __forceinline__ CV<P> cscale(const CV<P> &a, const V<P> &s)
{
    return CV<P>{mul(a.re, s), mul(a.im, s)};
}

template <int P>
__device__ __forceinline__ V<P> cabs2(const CV<P> &a)
{
    Acc<P> t = acc_zero<P>();
    acc_fma(t, a.re, a.re);
    acc_fma(t, a.im, a.im);
    return acc_get(t);
}

// 1/b = conj(b) / |b|^2
template <int P>
__device__ __forceinline__ CV<P> crecip(const CV<P> &b)
{
    const V<P> d = recip(cabs2(b));
    return CV<P>{mul(b.re, d), neg(mul(b.im, d))};
}

template <int P>
__device__ __forceinline__ CV<P> cwave_sum(const CV<P> &v)
{
    return CV<P>{wave_sum(v.re), wave_sum(v.im)};
}

// Sum over the workgroup, the same bits in every thread (waves combined in a fixed order).
// sred holds (kThreads / 64) * 2P doubles; called by all threads.
template <int P>
__device__ __forceinline__ CV<P> cblock_sum(const CV<P> &v, double *sred)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const CV<P> w = cwave_sum(v);
    if (lane == 0) clds_st(&sred[wid * 2 * P], w);
    __syncthreads();
    CV<P> s = clds_ld<P>(&sred[0]);
    for (int k = 1; k < kThreads / 64; ++k) s = cadd(s, clds_ld<P>(&sred[k * 2 * P]));
    __syncthreads();
    return s;
}

template <int P>
__device__ __forceinline__ V<P> rblock_sum(const V<P> &v, double *sred)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const V<P> w = wave_sum(v);
    if (lane == 0) lds_st(&sred[wid * P], w);
    __syncthreads();
    V<P> s = lds_ld<P>(&sred[0]);
    for (int k = 1; k < kThreads / 64; ++k) s = add(s, lds_ld<P>(&sred[k * P]));
    __syncthreads();
    return s;
}

// Entry (r, c) of the unit lower trapezoidal block Y (h rows, w columns) stored below the
// diagonal of A: 1 on the diagonal, 0 above it.
template <int P>
__device__ __forceinline__ CV<P> cy_entry(const double *Y, long ldy, long psy, long r, int c, int h, int w)
{
    if (r >= h || c >= w || r < c) return czero<P>();
    if (r == c) return cone<P>();
    return cldm<P>(Y, psy, (long)c * ldy + r);
}

// ============================================================================ QR panel
struct CPanelArgs {
    double *A;  // whole matrix, 2P planes of stride ps, leading dimension lda
    long lda, ps;
    int m;
    int j;     // k_cstep: the column whose reflector is applied; k_crefl: the column to reduce
    int jend;  // one past the panel's last column
    double *beta;  // P planes of stride bps
    long bps;
};

// The reflector of column c (rows c..m-1), formed by one whole workgroup: beta_c, v below the
// diagonal, R_cc on it.
template <int P>
__device__ __forceinline__ void c_reflector(double *A, long lda, long ps, int m, int c, double *beta, long bps, double *sred)
{
    const int tid = threadIdx.x;
    const long off = (long)c * lda;
    // every thread reads x1 before the barriers of the reduction; thread 0 overwrites it last
    const CV<P> alpha = cldm<P>(A, ps, off + c);
    Acc<P> acc = acc_zero<P>();
    int nt = 0;
    for (long r = c + 1 + tid; r < m; r += kThreads) {
        const CV<P> x = cldm<P>(A, ps, off + r);
        acc_fma(acc, x.re, x.re);
        acc_fma(acc, x.im, x.im);
        if (((++nt) % kCLazy<P>) == 0) acc = acc_from(acc_get(acc));
    }
    const V<P> sig = rblock_sum(acc_get(acc), sred);
    if (is_zero(sig)) {  // identity reflector, R_cc = x1
        if (tid == 0) stm(beta, bps, c, zero<P>());
        return;
    }
    const V<P> a2 = cabs2(alpha);
    const V<P> mu = sqrt_md(add(a2, sig));
    const V<P> rho = sqrt_md(a2);
    CV<P> ph;
    V<P> nu;
    if (is_zero(rho)) {
        ph = cone<P>();
        nu = neg(mu);
    } else {
        const V<P> ir = recip(rho);
        ph = CV<P>{mul(alpha.re, ir), mul(alpha.im, ir)};
        nu = neg(div(sig, add(rho, mu)));
    }
    const V<P> nu2 = mul(nu, nu);
    const V<P> bt = div(scale(nu2, 2.0), add(sig, nu2));
    const CV<P> iv = crecip(cscale(ph, nu));  // 1 / v1
    for (long r = c + 1 + tid; r < m; r += kThreads) cstm(A, ps, off + r, cmul(cldm<P>(A, ps, off + r), iv));
    if (tid == 0) {
        stm(beta, bps, c, bt);
        cstm(A, ps, off + c, cscale(ph, mu));
    }
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_crefl(CPanelArgs g)
{
    __shared__ double sred[(kThreads / 64) * 2 * P];
    c_reflector<P>(g.A, g.lda, g.ps, g.m, g.j, g.beta, g.bps, sred);
}

// Workgroup b: column c = j + 1 + b of the panel := H_j column (rows j..m-1, v_j = 1
// implicit); workgroup 0 then forms the reflector of column j + 1.  Each row is read and
// written by the same thread, so the only cross-thread hand-off is the barrier before
// c_reflector.
template <int P>
__global__ __launch_bounds__(kThreads) void k_cstep(CPanelArgs g)
{
    __shared__ double sred[(kThreads / 64) * 2 * P];
    const int c = g.j + 1 + blockIdx.x;
    const int tid = threadIdx.x;
    const long offj = (long)g.j * g.lda, offc = (long)c * g.lda;
    const V<P> bt = ldm<P>(g.beta, g.bps, g.j);
    if (!is_zero(bt)) {
        CAcc<P> acc = cacc_zero<P>();
        int nt = 0;
        for (long r = g.j + tid; r < g.m; r += kThreads) {
            const CV<P> v = (r == g.j) ? cone<P>() : cldm<P>(g.A, g.ps, offj + r);
            cacc_fma_step<P, true>(acc, v, cldm<P>(g.A, g.ps, offc + r), nt++);
        }
        const CV<P> w = cblock_sum(cacc_get(acc), sred);  // v^H a_c
        const CV<P> nt_ = cneg(cscale(w, bt));              // -beta v^H a_c
        for (long r = g.j + tid; r < g.m; r += kThreads) {
            const CV<P> v = (r == g.j) ? cone<P>() : cldm<P>(g.A, g.ps, offj + r);
            CAcc<P> a = cacc_from(cldm<P>(g.A, g.ps, offc + r));
            cacc_fma<P, false>(a, v, nt_);
            cstm(g.A, g.ps, offc + r, cacc_get(a));
        }
    }
    if (blockIdx.x == 0) {
        __syncthreads();
        c_reflector<P>(g.A, g.lda, g.ps, g.m, c, g.beta, g.bps, sred);
    }
}

// k_cstep with the rows in registers: thread t holds rows j + t + q * kThreads (q < QM) of
// columns j and c, so each is read once; the reflector of column j + 1 (workgroup 0) comes
// from the updated registers, x1 passing through LDS with the reduction's barriers.
// Requires m - j <= QM * kThreads.
template <int P, int QM>
__global__ __launch_bounds__(kThreads) void k_cstep_r(CPanelArgs g)
{
    __shared__ double sred[(kThreads / 64) * 2 * P];
    __shared__ double sx1[2 * P];
    const int c = g.j + 1 + blockIdx.x;
    const int tid = threadIdx.x;
    const long offj = (long)g.j * g.lda, offc = (long)c * g.lda;
    const V<P> bt = ldm<P>(g.beta, g.bps, g.j);
    CV<P> a[QM], v[QM];
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const long r = g.j + tid + (long)q * kThreads;
        const bool in = r < g.m;
        a[q] = in ? cldm<P>(g.A, g.ps, offc + r) : czero<P>();
        v[q] = (in && r > g.j) ? cldm<P>(g.A, g.ps, offj + r) : ((r == g.j) ? cone<P>() : czero<P>());
    }
    if (!is_zero(bt)) {
        CAcc<P> acc = cacc_zero<P>();
#pragma unroll
        for (int q = 0; q < QM; ++q) cacc_fma_step<P, true>(acc, v[q], a[q], q);
        const CV<P> w = cblock_sum(cacc_get(acc), sred);  // v^H a_c
        const CV<P> nt_ = cneg(cscale(w, bt));
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const long r = g.j + tid + (long)q * kThreads;
            CAcc<P> t = cacc_from(a[q]);
            cacc_fma<P, false>(t, v[q], nt_);
            a[q] = cacc_get(t);
            if (r < g.m) cstm(g.A, g.ps, offc + r, a[q]);
        }
    }
    if (blockIdx.x != 0) return;  // uniform per workgroup
    // the reflector of column c = j + 1: x1 is row c (thread 1, q = 0), x below it
    if (tid == 1) clds_st(sx1, a[0]);
    Acc<P> sacc = acc_zero<P>();
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const long r = g.j + tid + (long)q * kThreads;
        if (r > c && r < g.m) {
            acc_fma(sacc, a[q].re, a[q].re);
            acc_fma(sacc, a[q].im, a[q].im);
            if (((q + 1) % kCLazy<P>) == 0) sacc = acc_from(acc_get(sacc));
        }
    }
    const V<P> sig = rblock_sum(acc_get(sacc), sred);  // its barriers publish sx1
    if (is_zero(sig)) {
        if (tid == 0) stm(g.beta, g.bps, c, zero<P>());
        return;
    }
    const CV<P> alpha = clds_ld<P>(sx1);
    const V<P> a2 = cabs2(alpha);
    const V<P> mu = sqrt_md(add(a2, sig));
    const V<P> rho = sqrt_md(a2);
    CV<P> ph;
    V<P> nu;
    if (is_zero(rho)) {
        ph = cone<P>();
        nu = neg(mu);
    } else {
        const V<P> ir = recip(rho);
        ph = CV<P>{mul(alpha.re, ir), mul(alpha.im, ir)};
        nu = neg(div(sig, add(rho, mu)));
    }
    const V<P> nu2 = mul(nu, nu);
    const V<P> btc = div(scale(nu2, 2.0), add(sig, nu2));
    const CV<P> iv = crecip(cscale(ph, nu));  // 1 / v1
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const long r = g.j + tid + (long)q * kThreads;
        if (r > c && r < g.m) cstm(g.A, g.ps, offc + r, cmul(a[q], iv));
    }
    if (tid == 1) {
        stm(g.beta, g.bps, c, btc);
        cstm(g.A, g.ps, offc + c, cscale(ph, mu));
    }
}

// ============================================================================ persistent panel
// One launch per tile panel (columns kt .. kt + tile - 1, rows kt .. m - 1): workgroup b owns
// column c = kt + b for the whole launch, its h = m - kt rows held in LDS (2P planes of h
// doubles).  For j = kt .. c - 1 it waits until column j is published and applies H_j to its
// column; then it publishes its own column and last writes the column's final values.
//
// What is published for column j is the column x itself (rows below the diagonal, staged in
// a workspace buffer) and three scalars, not v = x/v1: with iv = 1/v1 and D = sum_{i>j}
// conj(x_i) a_i, H_j a has w = v^H a = a_j + conj(iv) D, row j becomes a_j - beta w =
// (1 - beta) a_j + conj(p1) D and the rows below a_i + x_i (p1 a_j + p2 D), where p1 =
// -beta iv and p2 = -beta |iv|^2.  The owner stages x before its reflector's chain (the stores
// overlap it), then stores p1, p2, beta, fences (release) and sets *count = c + 1; scaling its
// rows to v waits until the end, and so does the update of row j by H_j (D is kept in the
// unused head of the column's own staging slot), so neither is on the chain.  A workgroup
// waits only for lower-numbered ones and each wait is a bounded poll (a time-out raises *err,
// after which no wait polls), so the grid always drains.
//
// The reflector (the same vector as c_reflector's) is formed with a short chain: the four long
// md operations sqrt(q), 1/q, 1/sqrt(|x1|^2) and 1/sigma (q = |x1|^2 + sigma) run side by side,
// one per wave, and the rest are products: with rho = |x1|, mu = sqrt(q), nu = -sigma/(rho + mu)
// and v1 = e^{i theta} nu, 1/v1 = -conj(x1) (rho + mu)/(rho sigma), R_cc = x1 mu/rho, and
// beta = 2 nu^2/(sigma + nu^2) = sigma/(mu (mu + rho)) = 1 - rho/mu; the last form is used while
// sigma >= |x1|^2 (then rho/mu <= 1/sqrt 2, no cancellation), the one before it otherwise.
// x1 = 0 gives v1 = -mu, beta = 1, R_cc = mu.
struct CPersistArgs {
    double *A;  // whole matrix, 2P planes of stride ps, leading dimension lda
    long lda, ps;
    int m, kt;
    double *beta;  // P planes of stride bps
    long bps;
    double *xs;    // staged columns: 2P planes of stride xps, panel column b at b * m
    long xps;
    double *rec;   // per column c: p1 (2P doubles), p2, beta (P each) at rec + 4P c
    unsigned *count;  // columns published in this factorisation; zero before its first panel
    int *err;         // set to 1 if a wait times out
    unsigned spin;    // polls before a wait gives up
};

// Largest panel height of k_cpanel<P>: the column's 2P planes fit in 64 KiB of LDS.
template <int P>
constexpr int kCPanelRows = 4096 / P;

// Butterfly sum of a lazy accumulator over the 64 lanes, renormalised every kLazy<P> terms;
// both operands of each addition enter symmetrically, so every lane ends with the same bits.
template <int P>
__device__ __forceinline__ V<P> acc_wave_total(Acc<P> t)
{
    constexpr int RL = (kLazy<P> >= 64) ? 6 : (kLazy<P> >= 16 ? 4 : 2);  // levels per renormalisation
#pragma unroll
    for (int lv = 0; lv < 6; ++lv) {
        acc_add_acc(t, shfl_xor_acc(t, 32 >> lv));
        if ((lv + 1) % RL == 0 && lv < 5) t = acc_from(acc_get(t));
    }
    return acc_get(t);
}

// Workgroup totals, the same bits in every thread (the wave totals added in a fixed order);
// sred holds (kThreads / 64) * 2P doubles.  Called by all threads.
template <int P>
__device__ __forceinline__ CV<P> cacc_block_total(const CAcc<P> &a, double *sred)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const CV<P> w{acc_wave_total(a.re), acc_wave_total(a.im)};
    if (lane == 0) clds_st(&sred[wid * 2 * P], w);
    __syncthreads();
    CAcc<P> t = cacc_zero<P>();
    for (int k = 0; k < kThreads / 64; ++k) {
        const CV<P> o = clds_ld<P>(&sred[k * 2 * P]);
        acc_add(t.re, o.re);
        acc_add(t.im, o.im);
    }
    __syncthreads();
    return cacc_get(t);
}

template <int P>
__device__ __forceinline__ V<P> acc_block_total(const Acc<P> &a, double *sred)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const V<P> w = acc_wave_total(a);
    if (lane == 0) lds_st(&sred[wid * P], w);
    __syncthreads();
    Acc<P> t = acc_zero<P>();
    for (int k = 0; k < kThreads / 64; ++k) acc_add(t, lds_ld<P>(&sred[k * P]));
    __syncthreads();
    return acc_get(t);
}

template <int P>
__device__ __forceinline__ CV<P> cld_coherent(const double *X, long ps, long off)
{
    CV<P> v;
#pragma unroll
    for (int k = 0; k < P; ++k) {
        v.re.x[k] = ld_coherent(X + k * ps + off);
        v.im.x[k] = ld_coherent(X + (P + k) * ps + off);
    }
    return v;
}

template <int P>
__device__ __forceinline__ void cst_coherent(double *X, long ps, long off, const CV<P> &v)
{
#pragma unroll
    for (int k = 0; k < P; ++k) {
        st_coherent(X + k * ps + off, v.re.x[k]);
        st_coherent(X + (P + k) * ps + off, v.im.x[k]);
    }
}

// Wait until *count >= target: thread 0 polls (each poll after a short sleep), giving up after
// spin polls or once *err is set, then acquires; the barrier passes that on to the other
// threads, whose reads of published data are coherent loads.  Called by all threads.
__device__ inline void wait_count(unsigned *count, unsigned target, int *err, unsigned spin)
{
    if (threadIdx.x == 0) {
        unsigned spins = 0;
        while (__hip_atomic_load(count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            if ((spins & 255u) == 255u && __hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0) break;
            __builtin_amdgcn_s_sleep(1);
            if (++spins > spin) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    }
    __syncthreads();
}

template <int P>
__global__ __launch_bounds__(kThreads) void k_cpanel(CPersistArgs g)
{
    constexpr int QM = kCPanelRows<P> / kThreads;  // rows per thread
    extern __shared__ double sCol[];              // plane p of the column at sCol + p h
    __shared__ double sred[(kThreads / 64) * 2 * P];
    __shared__ double sch[4 * P];                 // sqrt(q), 1/q, 1/rho, 1/sigma
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int h = g.m - g.kt;
    const int jc = blockIdx.x;  // the column's diagonal row, counted from row kt
    const int c = g.kt + jc;
    const long offc = (long)c * g.lda + g.kt;
    double *const xc = g.xs + (long)jc * g.m;  // the column's staging slot
    // thread t holds rows t + q kThreads of the column (in LDS; other threads read only row
    // jj of step j and row jc, after the reductions that follow their last writes)
    auto sld = [&](int i) __attribute__((always_inline)) {
        CV<P> v;
#pragma unroll
        for (int e = 0; e < P; ++e) {
            v.re.x[e] = sCol[(long)e * h + i];
            v.im.x[e] = sCol[(long)(P + e) * h + i];
        }
        return v;
    };
    auto sst = [&](int i, const CV<P> &v) __attribute__((always_inline)) {
#pragma unroll
        for (int e = 0; e < P; ++e) {
            sCol[(long)e * h + i] = v.re.x[e];
            sCol[(long)(P + e) * h + i] = v.im.x[e];
        }
    };
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int i = tid + q * kThreads;
        if (i < h) sst(i, cldm<P>(g.A, g.ps, offc + i));
    }

    // ---- H_j for the columns before c; row jj keeps its value, D goes to the staging slot
    for (int j = g.kt; j < c; ++j) {
        const int jj = j - g.kt;
        wait_count(g.count, (unsigned)(j + 1), g.err, g.spin);
        const double *rj = g.rec + (long)4 * P * j;
        const double *xj = g.xs + (long)jj * g.m;
        // the staged column and the scalars together (one round trip)
        CV<P> x[QM];
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int i = tid + q * kThreads;
            x[q] = (i > jj && i < h) ? cld_coherent<P>(xj, g.xps, i) : czero<P>();
        }
        CV<P> p1;
        V<P> p2, bt;
#pragma unroll
        for (int e = 0; e < P; ++e) {
            p1.re.x[e] = ld_coherent(rj + e);
            p1.im.x[e] = ld_coherent(rj + P + e);
            p2.x[e] = ld_coherent(rj + 2 * P + e);
            bt.x[e] = ld_coherent(rj + 3 * P + e);
        }
        if (is_zero(bt)) continue;  // identity reflector (uniform)
        const CV<P> st1 = cmul(p1, sld(jj));  // p1 a_j, beside the dot
        // D: at most 2 QM = 32/P products per part, within kLazy<P>, renormalised at the end
        CAcc<P> acc = cacc_zero<P>();
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int i = tid + q * kThreads;
            if (i > jj && i < h) cacc_fma<P, true>(acc, x[q], sld(i));
        }
        const CV<P> D = cacc_block_total(cacc_from(cacc_get(acc)), sred);
        CAcc<P> t = cacc_from(st1);
        acc_fma(t.re, p2, D.re);
        acc_fma(t.im, p2, D.im);
        const CV<P> sc = cacc_get(t);  // p1 a_j + p2 D
#pragma unroll
        for (int q = 0; q < QM; ++q) {
            const int i = tid + q * kThreads;
            if (i > jj && i < h) {
                CAcc<P> u = cacc_from(sld(i));
                cacc_fma<P, false>(u, x[q], sc);
                sst(i, cacc_get(u));
            }
        }
        if (tid == (jj & (kThreads - 1))) cstm(xc, g.xps, jj, D);
    }

    // ---- stage the column below the diagonal, form the reflector, publish
    Acc<P> sacc = acc_zero<P>();
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int i = tid + q * kThreads;
        if (i > jc && i < h) {
            const CV<P> x = sld(i);
            cst_coherent(xc, g.xps, i, x);
            acc_fma(sacc, x.re, x.re);
            acc_fma(sacc, x.im, x.im);
        }
    }
    const V<P> sig = acc_block_total(acc_from(acc_get(sacc)), sred);  // its barriers publish row jc
    const CV<P> x1 = sld(jc);
    const bool ident = is_zero(sig);  // identity reflector: beta = 0, R_cc = x1
    CV<P> iv = cone<P>(), rjj = x1, p1 = czero<P>();  // iv: the factor of the rows below
    V<P> bt = zero<P>(), p2 = zero<P>();
    if (!ident) {
        const V<P> a2 = cabs2(x1);
        const V<P> q = add(a2, sig);
        const bool x1z = is_zero(a2);
        {
            V<P> r;
            if (wid == 0)
                r = sqrt_md(q);
            else if (wid == 1)
                r = recip(q);
            else if (wid == 2)
                r = x1z ? zero<P>() : rsqrt(a2);
            else
                r = recip(sig);
            if (lane == 0) lds_st(&sch[(wid & 3) * P], r);
        }
        __syncthreads();
        const V<P> mu = lds_ld<P>(&sch[0]), iq = lds_ld<P>(&sch[P]), ir = lds_ld<P>(&sch[2 * P]),
                   is = lds_ld<P>(&sch[3 * P]);
        if (x1z) {
            const V<P> imu = mul(mu, iq);
            iv = CV<P>{neg(imu), zero<P>()};
            bt = from_double<P>(1.0);
            rjj = CV<P>{mu, zero<P>()};
            p1 = CV<P>{imu, zero<P>()};
            p2 = neg(iq);
        } else {
            const V<P> rho = mul(a2, ir);
            const V<P> u = mul(add(rho, mu), mul(ir, is));  // (rho + mu)/(rho sigma)
            iv = CV<P>{neg(mul(x1.re, u)), mul(x1.im, u)};
            const V<P> mir = mul(mu, ir);
            rjj = CV<P>{mul(x1.re, mir), mul(x1.im, mir)};
            if (sub(sig, a2).x[0] >= 0.0)
                bt = fma(from_double<P>(1.0), neg(rho), mul(mu, iq));
            else
                bt = mul(sig, recip(mul(mu, add(mu, rho))));
            const V<P> nb = neg(bt);
            p1 = cscale(iv, nb);
            p2 = mul(nb, cabs2(iv));
        }
    }
    if (tid == 0) {
        double *rc = g.rec + (long)4 * P * c;
#pragma unroll
        for (int e = 0; e < P; ++e) {
            st_coherent(rc + e, p1.re.x[e]);
            st_coherent(rc + P + e, p1.im.x[e]);
            st_coherent(rc + 2 * P + e, p2.x[e]);
            st_coherent(rc + 3 * P + e, bt.x[e]);
        }
        stm(g.beta, g.bps, c, bt);
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __syncthreads();
    if (tid == 0) __hip_atomic_store(g.count, (unsigned)(c + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);

    // ---- final values (read only by later launches): row j of step j, R_cc, v = x/v1 below
#pragma unroll
    for (int q = 0; q < QM; ++q) {
        const int i = tid + q * kThreads;
        if (i < jc) {  // (1 - beta) a_j + conj(p1) D of step j = kt + i
            const double *rj = g.rec + (long)4 * P * (g.kt + i);
            CV<P> pj;
            V<P> bj;
#pragma unroll
            for (int e = 0; e < P; ++e) {
                pj.re.x[e] = ld_coherent(rj + e);
                pj.im.x[e] = ld_coherent(rj + P + e);
                bj.x[e] = ld_coherent(rj + 3 * P + e);
            }
            CV<P> a = sld(i);
            if (!is_zero(bj)) {
                CAcc<P> t = cacc_from(a);
                const V<P> nb = neg(bj);
                acc_fma(t.re, nb, a.re);
                acc_fma(t.im, nb, a.im);
                cacc_fma<P, true>(t, pj, cldm<P>(xc, g.xps, i));
                a = cacc_get(t);
            }
            cstm(g.A, g.ps, offc + i, a);
        } else if (i == jc) {
            cstm(g.A, g.ps, offc + i, rjj);
        } else if (i < h) {
            cstm(g.A, g.ps, offc + i, cmul(sld(i), iv));
        }
    }
}

namespace {
// A wait of the persistent panel timed out: R(0, 0) := NaN, so that the failure shows.
__global__ void k_cpoison(const int *err, double *A)
{
    if (threadIdx.x == 0 && *err != 0) A[0] = __builtin_nan("");
}
}  // namespace

// Workgroups of k_cpanel<P> one device can hold at once (with the largest column, 64 KiB of
// LDS), cached per device; 0 if the device cannot be queried.
template <int P>
int cpanel_capacity()
{
    static std::atomic<int> cache[64];
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 0;
    int c = cache[dev].load(std::memory_order_relaxed);
    if (c > 0) return c;
    int cus = 0, per_cu = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cpanel<P>, kThreads,
                                                     (size_t)kCPanelRows<P> * 2 * P * sizeof(double)) != hipSuccess)
        return 0;
    c = cus * per_cu;
    if (c > 0) cache[dev].store(c, std::memory_order_relaxed);
    return c;
}

// G(l, j) = y_l^H y_j for l < j (zero for l >= j) of the block Y (h rows, tile columns);
// one wave per (l, j): workgroup (lb, j) holds l = lb * 4 .. lb * 4 + 3.
template <int P>
__global__ __launch_bounds__(kThreads) void k_cgram(const double *Y, long lda, long ps, int h, int tile, double *G,
                                                   long gps)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int l = blockIdx.x * (kThreads / 64) + wid, j = blockIdx.y;
    if (l >= tile) return;
    if (l >= j) {
        if (lane == 0) cstm(G, gps, (long)j * tile + l, czero<P>());
        return;
    }
    CAcc<P> acc = cacc_zero<P>();
    int nt = 0;
    for (int r = j + lane; r < h; r += 64)  // y_j is zero above row j
        cacc_fma_step<P, true>(acc, cy_entry<P>(Y, lda, ps, r, l, h, tile), cy_entry<P>(Y, lda, ps, r, j, h, tile), nt++);
    const CV<P> s = cwave_sum(cacc_get(acc));
    if (lane == 0) cstm(G, gps, (long)j * tile + l, s);
}

// ============================================================================ triangular inverse
// X = U^{-1} for complex upper-triangular tiles, NC columns per workgroup, all advancing one
// row at a time from the bottom (paper Algorithm 1, stage 1): x_i = r_i d_i, then
// r_k -= U(k, i) x_i for k < i.  d_i = 1/U(i, i), or the real dsup_i when supplied (the T
// factor, whose inverse diagonal is beta).  Same InvArgs as the real kernel; the imaginary
// planes follow the real ones at P plane strides.
template <int P, int NC, int RPT>
__global__ __launch_bounds__(kThreads) void k_cinvert(InvArgs g)
{
    constexpr int RG = kThreads / NC;
    constexpr int Q = 2 * P;
    __shared__ double sD[256 * Q];
    __shared__ double sX[2][NC * Q];
    __shared__ double sU[2][256 * Q];
    const int t = blockIdx.y;
    const int c0 = blockIdx.x * NC;
    const int tid = threadIdx.x;
    const int jl = tid % NC, rg = tid / NC;
    const int j = c0 + jl;
    const double *U = g.U + (long)t * g.ustride;
    double *X = g.X + (long)t * g.xstride;
    const int c1 = min(c0 + NC, g.tile);

    for (int i = tid; i < c1; i += kThreads) {
        CV<P> d;
        if (g.dsup)
            d = CV<P>{ldm<P>(g.dsup + (long)t * g.tile, g.dps, i), zero<P>()};
        else
            d = crecip(cldm<P>(U, g.psu, (long)i * g.ldu + i));
        clds_st(&sD[i * Q], d);
    }
    CV<P> r[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int k = rg + q * RG;
        r[q] = (k == j) ? cone<P>() : czero<P>();
        if (j < g.tile && k < g.tile && k > j) cstm(X, g.psx, (long)j * g.ldx + k, czero<P>());
    }
    if (c1 > 0 && tid < c1 - 1) clds_st(&sU[(c1 - 1) & 1][tid * Q], cldm<P>(U, g.psu, (long)(c1 - 1) * g.ldu + tid));
    __syncthreads();
    for (int i = c1 - 1; i >= 0; --i) {
        const int buf = i & 1;
        CV<P> unext = czero<P>();
        const bool pre = i > 0 && tid < i - 1;
        if (pre) unext = cldm<P>(U, g.psu, (long)(i - 1) * g.ldu + tid);
        if (j < c1 && j >= i && (i % RG) == rg) {
            const int qi = i / RG;
            CV<P> xv = czero<P>();
#pragma unroll
            for (int q = 0; q < RPT; ++q)
                if (q == qi) {
                    const CV<P> d = clds_ld<P>(&sD[i * Q]);
                    xv = g.dsup ? cscale(r[q], d.re) : cmul(r[q], d);  // a supplied diagonal is real
                }
            clds_st(&sX[buf][jl * Q], xv);
            cstm(X, g.psx, (long)j * g.ldx + i, xv);
        }
        __syncthreads();
        if (j < c1 && j >= i) {
            const CV<P> xv = clds_ld<P>(&sX[buf][jl * Q]);
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int k = rg + q * RG;
                if (k < i) r[q] = cfms(r[q], clds_ld<P>(&sU[buf][k * Q]), xv);
            }
        }
        // sU[buf ^ 1] was last read in step i + 1, before this step's barrier
        if (pre) clds_st(&sU[buf ^ 1][tid * Q], unext);
    }
}

// Blocked complex inversion (tiles of 64 columns or more, a multiple of kInvNB = 32), as the
// real k_inv_blocks: with the 32 x 32 diagonal blocks X_II = U_II^{-1} of every tile formed
// first (k_cinvert on 32-column tiles: 32 dependent row steps instead of one per row of the
// tile), the blocks above them follow by block rows from the bottom, X_IK = -X_II sum_{I < J <=
// K} U_IJ X_JK.  Workgroup (slice, K - 1, tile) forms block column K for NCB of its columns;
// thread (r, c, p) holds row r and column c of the block row being formed and sums every NPART-th
// term of its two sums (the NPART partials then added in a fixed order), so a single tile still
// keeps every wave busy.  The block column is kept in LDS.  The workgroups also write the zeros
// below the diagonal blocks (the K == 1 ones block column 0 too), so X is the whole
// upper-triangular inverse.
template <int P>
constexpr int cinv_blk_cols()
{
    return P >= 8 ? 1 : (P == 4 ? 2 : (P == 2 ? 4 : 8));
}

struct CInvBlkArgs {
    const double *U;  // tile t at U + t ustride, ld ldu, plane stride psu
    long ldu, psu, ustride;
    const double *Xd;  // diagonal-block inverses: tile t's block I at Xd + (t nbt + I) 32^2, ld 32
    long dps;
    double *X;  // tile t at X + t xstride, ld ldx, plane stride psx
    long ldx, psx, xstride;
    int tile;
};

template <int P>
__global__ __launch_bounds__(kThreads) void k_cinv_blocks(CInvBlkArgs g)
{
    constexpr int NB = kInvNB, NCB = cinv_blk_cols<P>(), Q = 2 * P;
    constexpr int NPART = kThreads / (NB * NCB);
    static_assert(NPART >= 1 && NB * NCB * NPART == kThreads, "k_cinv_blocks layout");
    __shared__ double sX[256 * NCB * Q];         // rows 0 .. (K+1) NB - 1 of this workgroup's columns
    __shared__ double sP[NPART * NB * NCB * Q];  // partial sums
    __shared__ double sR[NB * NCB * Q];
    const int tid = threadIdx.x;
    const int r = tid % NB, c = (tid / NB) % NCB, part = tid / (NB * NCB);
    const int K = blockIdx.y + 1, t = blockIdx.z;
    const int cl = blockIdx.x * NCB + c;  // column inside block column K
    const int col = K * NB + cl;
    const double *U = g.U + (long)t * g.ustride;
    double *X = g.X + (long)t * g.xstride;
    const int nbt = g.tile / NB;
    auto xd = [&](int I, int row, int k) __attribute__((always_inline)) {
        return cldm<P>(g.Xd, g.dps, ((long)t * nbt + I) * NB * NB + (long)k * NB + row);
    };
    // sum of the NPART partials of entry (r, c), in part order
    auto combine = [&]() __attribute__((always_inline)) {
        CAcc<P> a = cacc_zero<P>();
        for (int q = 0; q < NPART; ++q) {
            const CV<P> o = clds_ld<P>(&sP[((q * NB + r) * NCB + c) * Q]);
            acc_add(a.re, o.re);
            acc_add(a.im, o.im);
        }
        return cacc_get(a);
    };
    if (part == 0) {
        const CV<P> v = xd(K, r, cl);
        clds_st(&sX[((K * NB + r) * NCB + c) * Q], v);
        cstm(X, g.psx, (long)col * g.ldx + K * NB + r, v);
        for (int I = K + 1; I < nbt; ++I) cstm(X, g.psx, (long)col * g.ldx + I * NB + r, czero<P>());
        if (K == 1) {
            cstm(X, g.psx, (long)cl * g.ldx + r, xd(0, r, cl));
            for (int I = 1; I < nbt; ++I) cstm(X, g.psx, (long)cl * g.ldx + I * NB + r, czero<P>());
        }
    }
    __syncthreads();
    for (int I = K - 1; I >= 0; --I) {
        // R(r, c) = sum over the rows k of block rows I+1 .. K of U(I NB + r, k) X(k, c)
        {
            CAcc<P> a = cacc_zero<P>();
            int nt = 0;
            for (int k = (I + 1) * NB + part; k < (K + 1) * NB; k += NPART)
                cacc_fma_step<P, false>(a, cldm<P>(U, g.psu, (long)k * g.ldu + I * NB + r),
                                        clds_ld<P>(&sX[(k * NCB + c) * Q]), nt++);
            clds_st(&sP[((part * NB + r) * NCB + c) * Q], cacc_get(a));
        }
        __syncthreads();
        if (part == 0) clds_st(&sR[(r * NCB + c) * Q], combine());
        __syncthreads();
        // X_IK(r, c) = -sum_{k >= r} X_II(r, k) R(k, c)
        {
            CAcc<P> a = cacc_zero<P>();
            int nt = 0;
            for (int k = r + part; k < NB; k += NPART)
                cacc_fma_step<P, false>(a, xd(I, r, k), clds_ld<P>(&sR[(k * NCB + c) * Q]), nt++);
            clds_st(&sP[((part * NB + r) * NCB + c) * Q], cacc_get(a));
        }
        __syncthreads();
        if (part == 0) {
            const CV<P> v = cneg(combine());
            clds_st(&sX[((I * NB + r) * NCB + c) * Q], v);
            cstm(X, g.psx, (long)col * g.ldx + I * NB + r, v);
        }
        __syncthreads();
    }
}

// ============================================================================ block reflector
// S(l, c) = y_l^H B(:, c): one wave per (l, c)
template <int P>
__global__ __launch_bounds__(kThreads) void k_ctn(const double *Y, long lda, long ps, int h, int tile, const double *B,
                                                 long ldb, long bps, int nrhs, double *S, long sps)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int l = blockIdx.x * (kThreads / 64) + wid, c = blockIdx.y;
    if (l >= tile || c >= nrhs) return;
    CAcc<P> acc = cacc_zero<P>();
    int nt = 0;
    for (int r = l + lane; r < h; r += 64)
        cacc_fma_step<P, true>(acc, cy_entry<P>(Y, lda, ps, r, l, h, tile), cldm<P>(B, bps, (long)c * ldb + r), nt++);
    const CV<P> s = cwave_sum(cacc_get(acc));
    if (lane == 0) cstm(S, sps, (long)c * tile + l, s);
}

// U(i, c) = sum_{l <= i} conj(T(l, i)) S(l, c), i.e. U = T^H S
template <int P>
__global__ __launch_bounds__(kThreads) void k_ctrmm_h(const double *T, long ldt, long tps, const double *S, long sps,
                                                     double *U, int tile, int nrhs)
{
    const int i = blockIdx.x * kThreads + threadIdx.x, c = blockIdx.y;
    if (i >= tile || c >= nrhs) return;
    CAcc<P> acc = cacc_zero<P>();
    for (int l = 0; l <= i; ++l)
        cacc_fma_step<P, true>(acc, cldm<P>(T, tps, (long)i * ldt + l), cldm<P>(S, sps, (long)c * tile + l), l);
    cstm(U, sps, (long)c * tile + i, cacc_get(acc));
}

// U(i, c) = sum_{l >= i} T(i, l) S(l, c), i.e. U = T S (the block reflector without the
// Hermitian transpose, for Q B)
template <int P>
__global__ __launch_bounds__(kThreads) void k_ctrmm_n(const double *T, long ldt, long tps, const double *S, long sps,
                                                     double *U, int tile, int nrhs)
{
    const int i = blockIdx.x * kThreads + threadIdx.x, c = blockIdx.y;
    if (i >= tile || c >= nrhs) return;
    CAcc<P> acc = cacc_zero<P>();
    for (int l = i; l < tile; ++l)
        cacc_fma_step<P, false>(acc, cldm<P>(T, tps, (long)l * ldt + i), cldm<P>(S, sps, (long)c * tile + l), l - i);
    cstm(U, sps, (long)c * tile + i, cacc_get(acc));
}

namespace {
// B(i, c) = 1 if i == c else 0 (2P planes)
__global__ void k_cidentity(double *B, long ldb, long bps, int rows, int cols, int P)
{
    const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (r >= rows || c >= cols) return;
    for (int k = 0; k < 2 * P; ++k) B[k * bps + (long)c * ldb + r] = (k == 0 && r == c) ? 1.0 : 0.0;
}
}  // namespace

// B(r, c) -= sum_l Y(r, l) U(l, c), r < h
template <int P>
__global__ __launch_bounds__(kThreads) void k_cnn_sub(const double *Y, long lda, long ps, int h, int tile, const double *U,
                                                     long ups, double *B, long ldb, long bps)
{
    const long r = (long)blockIdx.x * kThreads + threadIdx.x;
    const int c = blockIdx.y;
    if (r >= h) return;
    CAcc<P> acc = cacc_from(cldm<P>(B, bps, (long)c * ldb + r));
    const int lmax = (r < tile - 1) ? (int)r : tile - 1;
    for (int l = 0; l <= lmax; ++l)
        cacc_fma_step<P, false>(acc, cneg(cy_entry<P>(Y, lda, ps, r, l, h, tile)), cldm<P>(U, ups, (long)c * tile + l), l);
    cstm(B, bps, (long)c * ldb + r, cacc_get(acc));
}

// ============================================================================ back substitution
// x_i := Xinv_i y_i, one wave per output row
template <int P>
__global__ __launch_bounds__(kThreads) void k_cbs_xi(const double *Xi, long ldx, long psx, const double *y, long yps,
                                                    double *x, long xps, int tile)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int row = blockIdx.x * (kThreads / 64) + wid;
    if (row >= tile) return;
    CAcc<P> acc = cacc_zero<P>();
    int nt = 0;
    for (int c = row + lane; c < tile; c += 64)
        cacc_fma_step<P, false>(acc, cldm<P>(Xi, psx, (long)c * ldx + row), cldm<P>(y, yps, c), nt++);
    const CV<P> s = cwave_sum(cacc_get(acc));
    if (lane == 0) cstm(x, xps, row, s);
}

// y(0:rows) -= R(0:rows, columns of tile i) x_i; 64 rows per workgroup, the tile's columns
// split over the waves and combined in a fixed order
template <int P>
__global__ __launch_bounds__(kThreads) void k_cbs_upd(const double *Rc, long ldr, long psr, const double *xi, long xps,
                                                     double *y, long yps, int rows, int tile)
{
    constexpr int Q = 2 * P, NW = kThreads / 64;
    __shared__ double sx[256 * Q];
    __shared__ double sp[NW][64 * Q];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c = threadIdx.x; c < tile; c += kThreads) clds_st(&sx[c * Q], cldm<P>(xi, xps, c));
    __syncthreads();
    const long row = (long)blockIdx.x * 64 + lane;
    const int q = (tile + NW - 1) / NW;
    const int cb = wid * q, ce = min(tile, cb + q);
    CAcc<P> acc = cacc_zero<P>();
    if (row < rows)
        for (int c = cb; c < ce; ++c)
            cacc_fma_step<P, false>(acc, cldm<P>(Rc, psr, (long)c * ldr + row), clds_ld<P>(&sx[c * Q]), c - cb);
    clds_st(&sp[wid][lane * Q], cacc_get(acc));
    __syncthreads();
    if (wid == 0 && row < rows) {
        CV<P> s = clds_ld<P>(&sp[0][lane * Q]);
        for (int w = 1; w < NW; ++w) s = cadd(s, clds_ld<P>(&sp[w][lane * Q]));
        cstm(y, yps, row, cadd(cldm<P>(y, yps, row), cneg(s)));
    }
}

// ============================================================================ host side
// columns per workgroup of k_cinvert: each step of the serial row sweep costs a thread RPT
// complex multiply-adds (RPT = columns per workgroup), so one column per workgroup keeps the
// chain shortest and spreads a tile over tile workgroups
template <int P>
constexpr int kCInvCols = 1;

struct CLayout {
    size_t beta, T, G, S, U, y, ctr, px, pr, total;  // ctr, px, pr: the persistent panel's count and
                                                     // error flag, staged columns, scalars
    int sc;  // columns of S and U
};

inline CLayout clayout(int P, int m, int n, int tile)
{
    CLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += align256(bytes);
        return at;
    };
    L.sc = n > 64 ? n : 64;
    const size_t blk = sizeof(double) * 2 * (size_t)P * tile * n;  // 2P planes of tile x n
    L.beta = take(sizeof(double) * (size_t)P * n);
    L.T = take(blk);
    L.G = take(blk);
    L.S = take(sizeof(double) * 2 * (size_t)P * tile * L.sc);
    L.U = take(sizeof(double) * 2 * (size_t)P * tile * L.sc);
    L.y = take(sizeof(double) * 2 * (size_t)P * (m > n ? m : n));
    L.ctr = take(sizeof(unsigned) * 2);
    L.px = take(sizeof(double) * 2 * (size_t)P * m * tile);
    L.pr = take(sizeof(double) * 4 * (size_t)P * n);
    L.total = off;
    return L;
}

template <int P>
void cinvert_tiles(const InvArgs &ia, int ntiles, hipStream_t s)
{
    constexpr int NC = kCInvCols<P>;
    constexpr int RPT = 256 / (kThreads / NC);
    dim3 grid((ia.tile + NC - 1) / NC, ntiles);
    MDLS_LAUNCH("k_cinvert", P, 4.0 * ntiles * ia.tile * ia.tile * ia.tile / 6.0, (k_cinvert<P, NC, RPT>), grid,
                dim3(kThreads), s, ia);
}


// X = U^{-1} for ntiles tiles (diagonal from ia.dsup when given): blocked for tiles of 64 columns
// or more that are a multiple of 32, with Xd (2P planes of 32 * tile * ntiles doubles) for the
// diagonal blocks' inverses; the tiles must lie on the diagonal of one matrix (tile t at
// U + t tile (ldu + 1)) or be a single tile.
template <int P>
void cinvert_any(const InvArgs &ia, int ntiles, double *Xd, hipStream_t s)
{
    if (ia.tile < 64 || ia.tile % kInvNB != 0) {
        cinvert_tiles<P>(ia, ntiles, s);
        return;
    }
    const int nbt = ia.tile / kInvNB;
    const long dps = (long)kInvNB * ia.tile * ntiles;
    InvArgs id = ia;
    id.ustride = (long)kInvNB * (ia.ldu + 1);
    id.X = Xd;
    id.ldx = kInvNB;
    id.psx = dps;
    id.xstride = (long)kInvNB * kInvNB;
    id.tile = kInvNB;
    cinvert_tiles<P>(id, ntiles * nbt, s);
    const CInvBlkArgs ib{ia.U, ia.ldu, ia.psu, ia.ustride, Xd, dps, ia.X, ia.ldx, ia.psx, ia.xstride, ia.tile};
    constexpr int NCB = cinv_blk_cols<P>();
    double work = 0.0;  // complex md multiply-adds, 4 real ones each
    for (int K = 1; K < nbt; ++K) work += 4.0 * (K * (K + 1) / 2 + K) * kInvNB * kInvNB * kInvNB;
    MDLS_LAUNCH("k_cinv_blocks", P, work * ntiles, (k_cinv_blocks<P>), dim3(kInvNB / NCB, nbt - 1, ntiles),
                dim3(kThreads), s, ib);
}

// B(kt:m, cols) := (I - Y_k op(T_k) Y_k^H) B(kt:m, cols) for nc columns: S = Y^H B, U = op(T) S,
// B -= Y U, with op(T) = T^H (the product Q^H and the QR's trailing update)
template <int P>
void cblock_apply_h(const double *Y, long lda, long psa, int h, int tile, const double *Tk, long ldt, long tps, double *B,
                    long ldb, long bps, int nc, double *S, double *U, long sps, hipStream_t s)
{
    MDLS_LAUNCH("k_ctn", P, 4.0 * h * tile * nc, (k_ctn<P>), dim3((tile + 3) / 4, nc), dim3(kThreads), s, Y, lda, psa, h,
                tile, B, ldb, bps, nc, S, sps);
    MDLS_LAUNCH("k_ctrmm_h", P, 2.0 * tile * tile * nc, (k_ctrmm_h<P>), dim3((tile + kThreads - 1) / kThreads, nc),
                dim3(kThreads), s, Tk, ldt, tps, S, sps, U, tile, nc);
    MDLS_LAUNCH("k_cnn_sub", P, 4.0 * h * tile * nc, (k_cnn_sub<P>), dim3((h + kThreads - 1) / kThreads, nc),
                dim3(kThreads), s, Y, lda, psa, h, tile, U, sps, B, ldb, bps);
}

// The panel's columns kt .. jend - 1 a launch at a time: the first column's reflector, then per
// column j the update of the columns right of it and the next column's reflector.
template <int P>
void cpanel_columns(CPanelArgs pa, int kt, int jend, hipStream_t s)
{
    const int m = pa.m;
    pa.j = kt;
    pa.jend = jend;
    MDLS_LAUNCH("k_crefl", P, 6.0 * (m - kt), (k_crefl<P>), dim3(1), dim3(kThreads), s, pa);
    for (int j = kt; j < jend - 1; ++j) {
        pa.j = j;
        const int hj = m - j;
        const double work = 8.0 * hj * (jend - j - 1) + 6.0 * (hj - 1);
        const dim3 grid(jend - j - 1);
        // register-resident rows where they fit without spilling (P <= 4)
        bool done = false;
        if constexpr (P <= 4) {
            done = true;
            if (hj <= kThreads)
                MDLS_LAUNCH("k_cstep", P, work, (k_cstep_r<P, 1>), grid, dim3(kThreads), s, pa);
            else if (hj <= 2 * kThreads)
                MDLS_LAUNCH("k_cstep", P, work, (k_cstep_r<P, 2>), grid, dim3(kThreads), s, pa);
            else if (hj <= 4 * kThreads)
                MDLS_LAUNCH("k_cstep", P, work, (k_cstep_r<P, 4>), grid, dim3(kThreads), s, pa);
            else
                done = false;
        }
        if (!done) MDLS_LAUNCH("k_cstep", P, work, (k_cstep<P>), grid, dim3(kThreads), s, pa);
    }
}

// Blocked complex Householder QR; T (2P planes of ldt x n) receives T_k for every tile block.
template <int P>
int cqr_t(int m, int n, int tile, double *A, int lda, double *T, int ldt, void *ws, hipStream_t s)
{
    const CLayout L = clayout(P, m, n, tile);
    char *w = (char *)ws;
    double *beta = (double *)(w + L.beta);
    double *G = (double *)(w + L.G);
    double *S = (double *)(w + L.S);
    double *U = (double *)(w + L.U);
    if (!T) {
        T = (double *)(w + L.T);
        ldt = tile;
    }
    const long psa = (long)lda * n, tps = (long)ldt * n, gps = (long)tile * tile, sps = (long)tile * L.sc;
    const int N = n / tile;
    const CPanelArgs pa{A, (long)lda, psa, m, 0, 0, beta, (long)n};
    unsigned *count = (unsigned *)(w + L.ctr);
    int *err = (int *)(count + 1);
    // each panel as one persistent launch (the default for qd and od, where it is the faster
    // form; measured on MI355X: dd and double are faster a launch per column) while its column
    // fits and its workgroups can all be resident, else a launch per column
    const Tuning tu = tuning();
    const bool use = tu.cpanel == 1 || (tu.cpanel == 2 && P >= 4);
    const bool fits = use && cpanel_capacity<P>() >= tile;
    MDLS_LAUNCH("k_zero", P, 0, k_zero_u32, dim3(1), dim3(64), s, count, 2);
    bool persisted = false;
    for (int k = 0; k < N; ++k) {
        const int kt = k * tile, jend = kt + tile;
        const int h = m - kt;
        const bool done = fits && h <= kCPanelRows<P>;
        if (done) {
            const CPersistArgs ca{A, (long)lda, psa, m, kt, beta, (long)n, (double *)(w + L.px), (long)m * tile,
                                  (double *)(w + L.pr), count, err, tu.spin_limit};
            double work = 0;
            for (int j = 0; j < tile; ++j) work += 8.0 * (h - j) * (tile - j - 1) + 6.0 * (h - j);
            MDLS_LAUNCH_SHM("k_cpanel", P, work, (k_cpanel<P>), dim3(tile), dim3(kThreads),
                            (size_t)h * 2 * P * sizeof(double), s, ca);
        }
        if (!done) cpanel_columns<P>(pa, kt, jend, s);
        persisted = persisted || done;
        const double *Y = A + (long)kt * lda + kt;
        MDLS_LAUNCH("k_cgram", P, 2.0 * h * tile * tile, (k_cgram<P>), dim3((tile + 3) / 4, tile), dim3(kThreads), s, Y,
                    (long)lda, psa, h, tile, G, gps);
        InvArgs ia;
        ia.U = G;
        ia.ldu = tile;
        ia.psu = gps;
        ia.ustride = 0;
        ia.dsup = beta + kt;
        ia.dps = n;
        ia.X = T + (long)kt * ldt;
        ia.ldx = ldt;
        ia.psx = tps;
        ia.xstride = 0;
        ia.tile = tile;
        cinvert_any<P>(ia, 1, S, s);  // S is free until the update below
        if (jend < n)
            cblock_apply_h<P>(Y, (long)lda, psa, h, tile, T + (long)kt * ldt, (long)ldt, tps, A + (long)jend * lda + kt,
                              (long)lda, psa, n - jend, S, U, sps, s);
    }
    if (persisted) MDLS_LAUNCH("k_cpoison", P, 0, k_cpoison, dim3(1), dim3(64), s, err, A);
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

// B := Q^H B (m x nrhs, 2P planes of ldb x nrhs)
template <int P>
int capply_qh_t(int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *B, int ldb, int nrhs,
                void *ws, hipStream_t s)
{
    const CLayout L = clayout(P, m, n, tile);
    char *w = (char *)ws;
    double *S = (double *)(w + L.S);
    double *U = (double *)(w + L.U);
    const long psa = (long)lda * n, tps = (long)ldt * n, bps = (long)ldb * nrhs, sps = (long)tile * L.sc;
    const int N = n / tile;
    for (int c0 = 0; c0 < nrhs; c0 += L.sc) {
        const int nc = (nrhs - c0 < L.sc) ? nrhs - c0 : L.sc;
        double *Bc = B + (long)c0 * ldb;
        for (int k = 0; k < N; ++k) {
            const long kt = (long)k * tile;
            cblock_apply_h<P>(A + kt * lda + kt, (long)lda, psa, m - (int)kt, tile, T + kt * ldt, (long)ldt, tps, Bc + kt,
                              (long)ldb, bps, nc, S, U, sps, s);
        }
    }
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

// B := Q B (the tile blocks in reverse order, B := (I - Y_k T_k Y_k^H) B); with B = I this forms
// the unitary factor the paper's Algorithm 2 builds (Section 3)
template <int P>
int capply_q_t(int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *B, int ldb, int nrhs,
               void *ws, hipStream_t s)
{
    const CLayout L = clayout(P, m, n, tile);
    char *w = (char *)ws;
    double *S = (double *)(w + L.S);
    double *U = (double *)(w + L.U);
    const long psa = (long)lda * n, tps = (long)ldt * n, bps = (long)ldb * nrhs, sps = (long)tile * L.sc;
    const int N = n / tile;
    for (int c0 = 0; c0 < nrhs; c0 += L.sc) {
        const int nc = (nrhs - c0 < L.sc) ? nrhs - c0 : L.sc;
        double *Bc = B + (long)c0 * ldb;
        for (int k = N - 1; k >= 0; --k) {
            const long kt = (long)k * tile;
            const double *Y = A + kt * lda + kt;
            const int h = m - (int)kt;
            MDLS_LAUNCH("k_ctn", P, 4.0 * h * tile * nc, (k_ctn<P>), dim3((tile + 3) / 4, nc), dim3(kThreads), s, Y,
                        (long)lda, psa, h, tile, Bc + kt, (long)ldb, bps, nc, S, sps);
            MDLS_LAUNCH("k_ctrmm_n", P, 2.0 * tile * tile * nc, (k_ctrmm_n<P>), dim3((tile + kThreads - 1) / kThreads, nc),
                        dim3(kThreads), s, T + kt * ldt, (long)ldt, tps, S, sps, U, tile, nc);
            MDLS_LAUNCH("k_cnn_sub", P, 4.0 * h * tile * nc, (k_cnn_sub<P>), dim3((h + kThreads - 1) / kThreads, nc),
                        dim3(kThreads), s, Y, (long)lda, psa, h, tile, U, sps, Bc + kt, (long)ldb, bps);
        }
    }
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

// Q(:, 0:ncols) := the first ncols columns of the m x m unitary factor
template <int P>
int cform_q_t(int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *Q, int ldq, int ncols,
              void *ws, hipStream_t s)
{
    MDLS_LAUNCH("k_cidentity", P, 0, k_cidentity, dim3((m + 255) / 256, ncols), dim3(256), s, Q, (long)ldq,
                (long)ldq * ncols, m, ncols, P);
    return capply_q_t<P>(m, n, tile, A, lda, T, ldt, Q, ldq, ncols, ws, s);
}

// tiled back substitution on y (2P planes of n); x receives the solution
template <int P>
void cbacksub_tiles(const CLayout &L, char *w, int n, int tile, const double *R, long ldr, long psr, double *y, double *x,
                    long xps, int *d_info, hipStream_t s)
{
    const int N = n / tile;
    MDLS_LAUNCH("k_diag_check", P, 0, k_diag_check, dim3(1), dim3(kThreads), s, R, ldr, psr, n, 2 * P, d_info);
    double *Xinv = (double *)(w + L.G);
    const long xips = (long)tile * n;
    InvArgs ia;
    ia.U = R;
    ia.ldu = ldr;
    ia.psu = psr;
    ia.ustride = (long)tile * (ldr + 1);
    ia.dsup = nullptr;
    ia.dps = 0;
    ia.X = Xinv;
    ia.ldx = tile;
    ia.psx = xips;
    ia.xstride = (long)tile * tile;
    ia.tile = tile;
    cinvert_any<P>(ia, N, (double *)(w + L.S), s);
    const long yps = n;
    for (int i = N - 1; i >= 0; --i) {
        const long it = (long)i * tile;
        MDLS_LAUNCH("k_cbs_xi", P, 2.0 * tile * tile, (k_cbs_xi<P>), dim3((tile + 3) / 4), dim3(kThreads), s,
                    Xinv + (long)i * tile * tile, (long)tile, xips, y + it, yps, x + it, xps, tile);
        if (i > 0) {
            const int rows = i * tile;
            MDLS_LAUNCH("k_cbs_upd", P, 4.0 * rows * tile, (k_cbs_upd<P>), dim3((rows + 63) / 64), dim3(kThreads), s,
                        R + it * ldr, ldr, psr, x + it, xps, y, yps, rows, tile);
        }
    }
}

template <int P>
int cbacksub_t(int n, int tile, const double *R, int ldr, double *x, void *ws, int *d_info, hipStream_t s)
{
    const CLayout L = clayout(P, n, n, tile);
    char *w = (char *)ws;
    double *y = (double *)(w + L.y);
    MDLS_LAUNCH("k_copy", P, 0, k_copy, dim3((n + 255) / 256), dim3(256), s, x, (long)n, y, (long)n, n, 2 * P);
    cbacksub_tiles<P>(L, w, n, tile, R, ldr, (long)ldr * n, y, x, n, d_info, s);
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

// Complex least squares: A and b overwritten by the factors and Q^H b; x gets the solution.
template <int P>
int csolve_t(int m, int n, int tile, double *A, int lda, double *b, double *x, void *ws, int *d_info, hipStream_t s)
{
    const CLayout L = clayout(P, m, n, tile);
    char *w = (char *)ws;
    double *T = (double *)(w + L.T);
    int rc = cqr_t<P>(m, n, tile, A, lda, T, tile, ws, s);
    if (rc) return rc;
    rc = capply_qh_t<P>(m, n, tile, A, lda, T, tile, b, m, 1, ws, s);
    if (rc) return rc;
    double *y = (double *)(w + L.y);
    MDLS_LAUNCH("k_copy", P, 0, k_copy, dim3((n + 255) / 256), dim3(256), s, b, (long)m, y, (long)n, n, 2 * P);
    cbacksub_tiles<P>(L, w, n, tile, A, lda, (long)lda * n, y, x, n, d_info, s);
    // a timed-out wait of a persistent panel (cqr_t clears the flag first)
    MDLS_LAUNCH("k_fold_err", P, 0, k_fold_err, dim3(1), dim3(64), s, (const int *)(w + L.ctr) + 1, d_info);
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

#define MDLS_CPLX_FOR_PRECISION(X, P)                                                                               \
    X template int cqr_t<P>(int, int, int, double *, int, double *, int, void *, hipStream_t);                      \
    X template int capply_qh_t<P>(int, int, int, const double *, int, const double *, int, double *, int, int,      \
                                  void *, hipStream_t);                                                            \
    X template int cbacksub_t<P>(int, int, const double *, int, double *, void *, int *, hipStream_t);             \
    X template int capply_q_t<P>(int, int, int, const double *, int, const double *, int, double *, int, int,       \
                                 void *, hipStream_t);                                                             \
    X template int cform_q_t<P>(int, int, int, const double *, int, const double *, int, double *, int, int,        \
                                void *, hipStream_t);                                                              \
    X template int csolve_t<P>(int, int, int, double *, int, double *, double *, void *, int *, hipStream_t);

}  // namespace mdls_impl
