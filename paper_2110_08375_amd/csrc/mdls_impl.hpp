// mdls_impl.hpp -- MI355X (gfx950) kernels and host drivers of the multiple-double least-squares
// path; instantiated once per precision (mdls_p<P>.hip) and called by the C ABI (mdls_capi.hip).
//
// Hot path of a solve (paper Section 1: A = QR turns A x = b into R x = Q^T b):
//   QR (Section 3, Algorithm 2) as a sequence of narrow Householder panels.  For each panel of
//   W columns:
//     k_panel  -- Householder vectors and betas column by column (Golub-Van Loan 5.1.1 sign
//                 choice), the in-panel reflector updates, and the panel's compact-WY factor T
//                 (H_0 ... H_{W-1} = I - Y T Y^T, so the paper's W = -Y T).  The panel's rows
//                 stay in registers across all its columns; one workgroup reduction (and, when
//                 the panel spans several workgroups, one grid barrier) per column.
//     k_apply_s, k_apply_t, k_apply_u -- the trailing update C := C + Y (W^T C) =
//                 C - Y T^T (Y^T C) (paper's "YWT*C" and "R + YWTC" fused), applied to every
//                 column right of the panel and to the right-hand side, so Q^T b comes out of
//                 the factorisation.
//   Back substitution (Section 2, Algorithm 1):
//     k_invert -- invert the diagonal tiles (all columns of a tile in parallel, one row step at
//                 a time);
//     k_bs_xi  -- x_i := U_i^{-1} b_i;
//     k_bs_upd -- b_j -= A_{j,i} x_i for every j < i at once.
//
// Multiple-double numbers are P limb planes (limb 0 most significant); see md.hpp for the
// arithmetic.
#include <algorithm>
#include <climits>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <vector>

#pragma once
#include "mdls.h"
#include "mdls_kernels.hpp"
#include "mdls_split_kernels.hpp"

namespace mdls_impl {
using namespace mdk;

// ============================================================================ panel kernel
struct PanelArgs {
    double *A;  // panel column 0 at row (diagonal - off); the panel's diagonal is row off
    long lda, ps;
    int h, wact;   // rows from the diagonal down, active columns (<= W)
    int off;       // W when the previous panel is applied first (rows above the diagonal), else 0
    const double *Yp;  // previous panel's diagonal element (its Y, unit lower trapezoidal), if off
    const double *Tp;  // previous panel's T (W x W, ld W), plane stride tps
    double *beta;  // beta of the panel's first column, plane stride bps
    long bps;
    double *T;  // panel T, W x W column-major (ld W), plane stride tps
    long tps;
    double *gpart;  // [2][G][W*W + 2W][P] exchange slots between workgroups
    unsigned *gbar; // barrier counter of this launch, zero on entry
    int *err;       // set to 1 if a barrier times out
    int G;          // workgroups in the launch
    unsigned spin;  // polls before a barrier gives up
};

// Entry (r, c) of a block of Householder vectors stored below the diagonal of A: zero above
// the diagonal, the implicit one on it, the stored value below; zero outside h x wact.
template <int P>
__device__ __forceinline__ V<P> y_entry(const double *Y, long ldy, long psy, long r, int c, int h, int wact)
{
    if (r >= h || c >= wact || r < c) return zero<P>();
    if (r == c) return from_double<P>(1.0);
    return ldm<P>(Y, psy, (long)c * ldy + r);
}

// All workgroups of the launch meet here (called by one whole wave per workgroup).  The
// spin is bounded (spin polls, each after a short sleep): a timed-out barrier raises *err and
// lets the wave continue, so the grid always drains; the host turns *err into a status.
__device__ inline void grid_sync(unsigned *ctr, unsigned target, int *err, unsigned spin)
{
    const int lane = threadIdx.x & 63;
    // the fence before the relaxed arrival releases this workgroup's stores; the relaxed
    // polls need no cache invalidation each, the fence after them acquires the others' stores
    // (a release and an acquire fence: neither side needs the other half of a full fence)
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    if (lane == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > spin) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
}

// Sum over a workgroup of per-thread partials of WW pairs: thread t holds a partial of pair
// t % WW.  Partials of one pair inside a wave are combined with a butterfly, those of
// different waves through LDS; out[q] (LDS, WW x P doubles) receives the renormalised total,
// negated if NEG.  Called by every thread; ends with a workgroup barrier.
template <int P, int WW, int NT, bool NEG>
__device__ __forceinline__ void pair_sum(Acc<P> t, double *s_comb, double *out)
{
    constexpr int WV = (WW < 64) ? 64 : WW;  // threads that hold each pair once
    constexpr int NP = NT / WV;              // partials per pair left after the butterfly
    static_assert(NT % WV == 0, "pair_sum layout");
    const int tid = threadIdx.x;
#pragma unroll
    for (int m = WW; m < 64; m <<= 1) acc_add_acc(t, shfl_xor_acc(t, m));
    if (tid % WV < WW) {
#pragma unroll
        for (int k = 0; k < P; ++k) s_comb[((tid / WV) * WW + tid % WV) * P + k] = t.s[k];
    }
    __syncthreads();
    for (int q = tid; q < WW; q += NT) {
        Acc<P> s = acc_zero<P>();
        for (int k = 0; k < NP; ++k) {
            Acc<P> o;
#pragma unroll
            for (int e = 0; e < P; ++e) o.s[e] = s_comb[(k * WW + q) * P + e];
            acc_add_acc(s, o);
        }
        const V<P> v = acc_get(s);
        lds_st(&out[q * P], NEG ? neg(v) : v);
    }
    __syncthreads();
}

// Sum of NA lazy accumulators per lane over the row-slot bits of a wave (lane masks 32, 16,
// ..., MMIN): while a lane holds two or more accumulators each level halves the set (the
// partner keeps the other half), then plain butterfly levels follow.  Lane l keeps
// slot_scatter_kept<W>() accumulators, starting at index slot_scatter_index<W>(l); equal
// totals sit on the lanes that differ only in slot_plain_mask bits.
template <int P, int NA, int NH, int MMIN, int M>
__device__ __forceinline__ void slot_scatter(Acc<P> (&s)[NA], int lane)
{
    if constexpr (M >= MMIN) {
        if constexpr (NH >= 2) {
            constexpr int HALF = NH / 2;
            const bool hi = (lane & M) != 0;
#pragma unroll
            for (int q = 0; q < HALF; ++q) {
                Acc<P> mine, give;
#pragma unroll
                for (int k = 0; k < P; ++k) {
                    mine.s[k] = hi ? s[q + HALF].s[k] : s[q].s[k];
                    give.s[k] = hi ? s[q].s[k] : s[q + HALF].s[k];
                }
                acc_add_acc(mine, shfl_xor_acc(give, M));
                s[q] = mine;
            }
            slot_scatter<P, NA, HALF, MMIN, M / 2>(s, lane);
        } else {
            acc_add_acc(s[0], shfl_xor_acc(s[0], M));
            slot_scatter<P, NA, NH, MMIN, M / 2>(s, lane);
        }
    }
}

template <int W>
constexpr int slot_levels()
{
    int n = 0;
    for (int m = 32; m >= W; m >>= 1) ++n;
    return n;
}

template <int W>
constexpr int slot_scatter_kept()
{
    int na = W;
    for (int t = 0; t < slot_levels<W>() && na >= 2; ++t) na /= 2;
    return na;
}

template <int W, int MMIN, int M>
constexpr int slot_plain_mask()
{
    int na = W, mask = 0;
    for (int m = M; m >= MMIN; m >>= 1) {
        if (na >= 2)
            na /= 2;
        else
            mask |= m;
    }
    return mask;
}

// first accumulator index kept by lane l after slot_scatter over masks 32 .. W
template <int W>
__device__ __forceinline__ int slot_scatter_index(int lane)
{
    int idx = 0, na = W;
    for (int m = 32; m >= W && na >= 2; m >>= 1) {
        na /= 2;
        if (lane & m) idx += na;
    }
    return idx;
}

// Thread (slot, c) of workgroup b holds column c of rows b*S + slot + k*G*S, k < R, where
// S = NT/W row slots per workgroup: the W threads of a row are consecutive lanes.  Rows are
// counted from `off` rows above the panel's diagonal.
//
// When off = W the kernel first applies the previous panel's block reflector to its own
// columns, C := C - Y' T'^T (Y'^T C) over the rows from the previous diagonal down (this is
// the look-ahead: the rest of the trailing matrix is updated by the k_apply_s/t/u kernels
// concurrently).
//
// Column j of the panel, x = A(j:h, j) with x1 = a_jj, sigma = sum_{i>j} x_i^2, q = x1^2 + sigma,
// mu = sqrt(q): the Householder vector of Golub-Van Loan 5.1.1 is v = x rho below the
// diagonal with v_j = 1, where rho = 1/v1 and v1 = x1 - mu (x1 <= 0) or -sigma/(x1 + mu)
// (x1 > 0), so rho = -1/(mu - x1) = -(mu + x1)/sigma in both cases; beta = 2/(v^T v) and
// beta rho = -1/mu, so beta = 1 - x1/mu.  For c > j, with d_c = sum_{i>j} x_i a_ic from the
// same reduction as sigma, w_c = v^T a_c = a_jc + rho d_c and the update is
// a_ic += (w_c/mu) x_i (i > j), a_jc -= beta w_c.  The per-column chain is the square root;
// the reciprocals 1/q and 1/sigma are formed beside it in other waves, and then
// 1/mu = mu (1/q), rho = -(mu + x1) (1/sigma) cost one product each.  Where these forms
// cancel (sigma < x1^2: mu + x1 for x1 < 0, 1 - x1/mu for x1 > 0) rho = -1/(mu - x1) and
// beta = -(1/mu)/rho are used instead.  Column j of T follows from
// T(0:j, j) = -beta_j T(0:j, 0:j) (Y(:, 0:j)^T v_j) (Schreiber and Van Loan's compact WY).
template <int P, int W, int R, int NT>
__device__ __forceinline__ void panel_run(const PanelArgs &g, int bid)
{
    constexpr int S = NT / W;
    constexpr int NW = NT / 64;
    constexpr int SLOT = (W * W + 2 * W) * P;  // doubles per workgroup exchange slot
    static_assert(64 % W == 0 && S >= 2 * W && NW >= 4, "panel layout");
    __shared__ double s_part[NW * W * W * P];
    __shared__ double s_comb[NT * P];     // pair_sum partials
    __shared__ double s_head[W * P];
    __shared__ double s_tot[W * P];       // column j's reduction: sigma (l = j), d_l, Gram sums
    __shared__ double s_hd[W * P];        // row j: a_jl
    __shared__ double s_mu[P];
    __shared__ double s_iq[P];            // 1/q
    __shared__ double s_is[P];            // 1/sigma
    __shared__ double s_fc[W * W * P];    // [j][c]: w_c = v_j^T a_c (deferred row-j update)
    __shared__ double s_info[W * 2 * P];  // per column: 1/mu, x1
    __shared__ double s_gram[W * W * P];  // [j][l]: sum_{i>j} x_j(i) x_l(i), l < j
    __shared__ double s_hrow[W * W * P];  // [j][l]: a_jl when column j is processed, l < j
    __shared__ double s_rho[W * P];
    __shared__ double s_beta[W * P];
    __shared__ double s_T[W * W * P];     // T, column-major
    __shared__ int s_flag[W];             // per column: 1 sigma == 0, 2 beta from rho (x1 > 0, sigma < x1^2)

    // The panel is the critical path of the factorisation: its waves take issue priority over
    // the trailing-update waves that may share their compute unit.
    __builtin_amdgcn_s_setprio(3);
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int c = tid % W, slot = tid / W;
    const long rstride = (long)g.G * S;
    const long rbase = (long)bid * S + slot;
    const int src0 = lane & ~(W - 1);
    const int off = g.off;
    const long hh = (long)g.h + off;
    unsigned nbar = 0;

    // Off-chain pieces of the compact-WY factor (block 0; beta and T are written by it only).
    // beta_jj = 1 - x1/mu, or -(1/mu)/rho where that form cancels (wave 2)
    auto t_beta = [&](int jj) __attribute__((always_inline)) {
        V<P> beta = zero<P>();
        if (!(s_flag[jj] & 1)) {
            const V<P> r = lds_ld<P>(&s_info[(jj * 2 + 0) * P]);
            if (s_flag[jj] & 2)
                beta = neg(mul(r, recip(lds_ld<P>(&s_rho[jj * P]))));
            else
                beta = fma(from_double<P>(1.0), neg(lds_ld<P>(&s_info[(jj * 2 + 1) * P])), r);
        }
        if (lane == 0) {
            lds_st(&s_beta[jj * P], beta);
            stm(g.beta, g.bps, jj, beta);
        }
    };
    // lane l < jj: g(l, jj) = y_l^T v_jj = rho_l (a_jj,l + rho_jj gsum_jj,l) (wave 3)
    auto t_g = [&](int jj) __attribute__((always_inline)) {
        V<P> gv = zero<P>();
        if (lane < jj) {
            const V<P> rl = lds_ld<P>(&s_rho[lane * P]), rj = lds_ld<P>(&s_rho[jj * P]);
            gv = mul(rl, fma(lds_ld<P>(&s_hrow[(jj * W + lane) * P]), rj, lds_ld<P>(&s_gram[(jj * W + lane) * P])));
        }
        return gv;
    };
    // lane l < jj: w_l = sum_{l <= k < jj} T(l, k) g(k, jj) (wave 3); even and odd k in two
    // accumulators, so the two halves of the sum overlap
    auto t_w = [&](int jj, const V<P> &gv) __attribute__((always_inline)) {
        Acc<P> w0 = acc_zero<P>(), w1 = acc_zero<P>();
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (k < jj) {
                const V<P> gk = shfl_md(gv, k);
                if (lane <= k) {
                    if (k & 1)
                        acc_fma(w1, lds_ld<P>(&s_T[(k * W + lane) * P]), gk);
                    else
                        acc_fma(w0, lds_ld<P>(&s_T[(k * W + lane) * P]), gk);
                }
            }
        }
        acc_add_acc(w0, w1);
        return acc_get(w0);
    };
    // T(0:jj, jj) = -beta_jj w, T(jj, jj) = beta_jj, zero below (wave 3)
    auto t_store = [&](int jj, const V<P> &w) __attribute__((always_inline)) {
        const V<P> bj = lds_ld<P>(&s_beta[jj * P]);
        if (lane < W) {
            V<P> t = zero<P>();
            if (lane < jj && !(s_flag[jj] & 1)) t = neg(mul(bj, w));
            if (lane == jj) t = bj;
            lds_st(&s_T[(jj * W + lane) * P], t);
            stm(g.T, g.tps, (long)jj * W + lane, t);
        }
    };

    V<P> a[R];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const long r = rbase + k * rstride;
        a[k] = (r < hh && c < g.wact) ? ldm<P>(g.A, g.ps, c * g.lda + r) : zero<P>();
    }

    // ---- 0. apply the previous panel's reflectors to this panel (look-ahead update):
    //         S = Y'^T C (W x W), -U = -T'^T S, C += Y' (-U)
    if (off) {
        Acc<P> sacc[W];
#pragma unroll
        for (int i = 0; i < W; ++i) sacc[i] = acc_zero<P>();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const long r = rbase + k * rstride;
            if (r < hh) {
#pragma unroll
                for (int i = 0; i < W; ++i)
                    acc_fma_step(sacc[i], y_entry<P>(g.Yp, g.lda, g.ps, r, i, (int)hh, W), a[k], k);
            }
        }
        // sum over the wave's row slots; lane (.., c) ends with NF accumulators of column c
        constexpr int NF = slot_scatter_kept<W>();
        slot_scatter<P, W, W, W, 32>(sacc, lane);
        if ((lane & slot_plain_mask<W, W, 32>()) == 0) {
            const int i0 = slot_scatter_index<W>(lane);
#pragma unroll
            for (int f = 0; f < NF; ++f)
#pragma unroll
                for (int k = 0; k < P; ++k) s_part[((wid * W + i0 + f) * W + c) * P + k] = sacc[f].s[k];
        }
        __syncthreads();
        // pairs q = (i, cc) = (q / W, q % W); thread t takes pair t % W^2 and every K-th part
        // of its sums (K = NT / W^2 threads per pair), pair_sum combines them
        constexpr int WW = W * W;
        constexpr int K = NT / WW;
        const int pq = tid % WW, psub = tid / WW;
        {
            Acc<P> t = acc_zero<P>();
            for (int w = psub; w < NW; w += K) {
                Acc<P> o;
#pragma unroll
                for (int k = 0; k < P; ++k) o.s[k] = s_part[(w * WW + pq) * P + k];
                acc_add_acc(t, o);
            }
            pair_sum<P, WW, NT, false>(t, s_comb, s_gram);  // this workgroup's S
        }
        if (g.G > 1) {
            if (wid == 0) {
                double *mine = g.gpart + (size_t)((nbar & 1) * g.G + bid) * SLOT;
                for (int q = lane; q < WW; q += 64) {
#pragma unroll
                    for (int k = 0; k < P; ++k) st_coherent(mine + q * P + k, s_gram[q * P + k]);
                }
                grid_sync(g.gbar, (nbar + 1) * (unsigned)g.G, g.err, g.spin);
            }
            __syncthreads();
            const double *base = g.gpart + (size_t)((nbar & 1) * g.G) * SLOT;
            // the workgroups' slots are loaded in batches of NB before they are added (same
            // order), so a batch costs one round trip
            constexpr int NB = (P >= 8) ? 1 : 8;
            Acc<P> t = acc_zero<P>();
            for (int b0 = psub; b0 < g.G; b0 += NB * K) {
                Acc<P> o[NB];
#pragma unroll
                for (int u = 0; u < NB; ++u) {
                    const int b = b0 + u * K;
#pragma unroll
                    for (int k = 0; k < P; ++k)
                        o[u].s[k] = (b < g.G) ? ld_coherent(base + (size_t)b * SLOT + pq * P + k) : 0.0;
                }
#pragma unroll
                for (int u = 0; u < NB; ++u)
                    if (b0 + u * K < g.G) acc_add_acc(t, o[u]);
            }
            pair_sum<P, WW, NT, false>(t, s_comb, s_gram);
        }
        ++nbar;
        // -U(i, cc) = -sum_{l<=i} T'(l, i) S(l, cc) into s_hrow (scratch); the K threads of a
        // pair split the sum over l
        {
            const int i = pq / W, cc = pq % W;
            Acc<P> u = acc_zero<P>();
            for (int l = psub; l <= i; l += K)
                acc_fma(u, ldm<P>(g.Tp, g.tps, (long)i * W + l), lds_ld<P>(&s_gram[(l * W + cc) * P]));
            pair_sum<P, WW, NT, true>(u, s_comb, s_hrow);
        }
        // even and odd i in two accumulators, so the two halves of the sum overlap
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const long r = rbase + k * rstride;
            if (r < hh && c < g.wact) {
                Acc<P> t0 = acc_from(a[k]), t1 = acc_zero<P>();
#pragma unroll
                for (int i = 0; i < W; i += 2) {
                    acc_fma(t0, y_entry<P>(g.Yp, g.lda, g.ps, r, i, (int)hh, W), lds_ld<P>(&s_hrow[(i * W + c) * P]));
                    acc_fma(t1, y_entry<P>(g.Yp, g.lda, g.ps, r, i + 1, (int)hh, W),
                            lds_ld<P>(&s_hrow[((i + 1) * W + c) * P]));
                }
                acc_add_acc(t0, t1);
                a[k] = acc_get(t0);
            }
        }
        __syncthreads();
    }

    // Per column j the serial chain (reduction, mu, 1/mu, w_c) runs through waves 0 and 1; the
    // other waves do the off-chain work between the same workgroup barriers:
    //   [B1, B2]  wave 0: reduction of the partial sums (and the grid exchange);
    //             wave 2: beta of column j-1; wave 3: g(l, j-1) (block 0 only), and for
    //             P <= 4 also w = T(:, :j-1) g(:, j-1), which is longer than mu there
    //   [B2, M]   wave 0: mu = sqrt(q); wave 1: 1/q; wave 2: 1/sigma; wave 3 (P = 8): w
    //   [M, Tb]   wave 0: 1/mu = mu (1/q); wave 1: rho_j and w_c = a_jc + rho_j d_c;
    //             wave 3: T(:, j-1) = -beta w
    //   after Tb  every thread: coef_c = w_c / mu and the update of its rows below row j.
    // Row j of the columns c > j (a_jc -= beta w_c) is not needed again inside the panel, so
    // that update waits for the end of the panel.
    // wave 3 carries g, then w, across barriers
    V<P> cx = zero<P>();
    // where w is formed: beside the reduction while the md scalars are cheap (P <= 4); beside mu
    // for od, whose reduction window is the shorter one in late panels
    constexpr bool kEarlyW = P <= 4;
    for (int j = 0; j < g.wact; ++j) {
        const long dj = off + j;  // row of the diagonal element of column j
        // ---- 1. one reduction per column: thread (slot, c) sums x_j(i) a_c(i) over its rows i > j:
        //         sigma (c = j), d_c (c > j), the Gram sums for T (c < j)
        Acc<P> acc = acc_zero<P>();
#pragma unroll
        for (int k = 0; k < R; ++k) {
            const long r = rbase + k * rstride;
            const V<P> xk = shfl_md(a[k], src0 + j);
            if (r > dj && r < hh) acc_fma_step(acc, xk, a[k], k);
        }
        // the partial sums stay lazy (level sums) through every reduction level below and are
        // renormalised once, in wave 0
#pragma unroll
        for (int m = W; m < 64; m <<= 1) acc_add_acc(acc, shfl_xor_acc(acc, m));
        if (lane < W) {
#pragma unroll
            for (int k = 0; k < P; ++k) s_part[(wid * W + lane) * P + k] = acc.s[k];
        }
        if (bid == 0 && slot == dj) lds_st(&s_head[c * P], a[0]);
        __syncthreads();  // B1
        if (wid == 0) {
            Acc<P> ta = acc_zero<P>();
            for (int i = lane; i < NW * W; i += 64) {
                Acc<P> o;
#pragma unroll
                for (int k = 0; k < P; ++k) o.s[k] = s_part[i * P + k];
                acc_add_acc(ta, o);
            }
#pragma unroll
            for (int m = W; m < (NW * W < 64 ? NW * W : 64); m <<= 1) acc_add_acc(ta, shfl_xor_acc(ta, m));
            V<P> hd = (bid == 0) ? lds_ld<P>(&s_head[(lane % W) * P]) : zero<P>();
            if (g.G > 1) {
                double *mine = g.gpart + (size_t)((nbar & 1) * g.G + bid) * SLOT;
                if (lane < W) {
#pragma unroll
                    for (int k = 0; k < P; ++k) st_coherent(mine + lane * P + k, ta.s[k]);
                    if (bid == 0) {
#pragma unroll
                        for (int k = 0; k < P; ++k) st_coherent(mine + (W + lane) * P + k, hd.x[k]);
                    }
                }
                grid_sync(g.gbar, (nbar + 1) * (unsigned)g.G, g.err, g.spin);
                const double *base = g.gpart + (size_t)((nbar & 1) * g.G) * SLOT;
                // all loads of a batch are issued before the first sum needs them (one round
                // trip per batch instead of one per term; od, with one term per lane, keeps
                // its registers); the summation order is unchanged
                constexpr int NB = (P >= 8) ? 1 : 4;
#pragma unroll
                for (int k = 0; k < P; ++k) hd.x[k] = ld_coherent(base + (W + lane % W) * P + k);
                ta = acc_zero<P>();
                const int tot = g.G * W;
                for (int i0 = lane; i0 < tot; i0 += NB * 64) {
                    Acc<P> o[NB];
#pragma unroll
                    for (int u = 0; u < NB; ++u) {
                        const int i = i0 + u * 64;
                        const double *q = base + (size_t)(i / W) * SLOT + (i % W) * P;
#pragma unroll
                        for (int k = 0; k < P; ++k) o[u].s[k] = (i < tot) ? ld_coherent(q + k) : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < NB; ++u)
                        if (i0 + u * 64 < tot) acc_add_acc(ta, o[u]);
                }
                const int lim = (g.G * W < 64) ? g.G * W : 64;
                for (int m = W; m < lim; m <<= 1) acc_add_acc(ta, shfl_xor_acc(ta, m));
            }
            const V<P> tot = acc_get(ta);
            // lanes l < W now hold tot = total of column l and hd = a_jl
            if (lane < W) {
                lds_st(&s_tot[lane * P], tot);
                lds_st(&s_hd[lane * P], hd);
            }
            if (lane < j) {
                lds_st(&s_gram[(j * W + lane) * P], tot);
                lds_st(&s_hrow[(j * W + lane) * P], hd);
            }
        } else if (bid == 0 && j > 0) {
            if (wid == 2) t_beta(j - 1);
            if (wid == 3) {
                cx = t_g(j - 1);
                if constexpr (kEarlyW) cx = t_w(j - 1, cx);  // in the shadow of the reduction
            }
        }
        ++nbar;
        __syncthreads();  // B2
        // ---- 2. Householder scalars, identical in every lane and every workgroup
        const V<P> sig = lds_ld<P>(&s_tot[j * P]);
        const V<P> x1 = lds_ld<P>(&s_hd[j * P]);
        const bool zs = is_zero(sig);
        const bool pos = x1.x[0] > 0.0;
        const bool small = sig.x[0] < x1.x[0] * x1.x[0];  // sigma < x1^2: the cancelling forms are avoided
        if (wid == 0) {
            if (!zs) {
                const V<P> mu = sqrt_md(fma(sig, x1, x1));
                if (lane == 0) lds_st(s_mu, mu);
            }
            if (lane == 0) s_flag[j] = zs ? 1 : ((pos && small) ? 2 : 0);
        } else if (wid == 1) {
            if (!zs) {
                const V<P> iq = recip(fma(sig, x1, x1));
                if (lane == 0) lds_st(s_iq, iq);
            }
        } else if (wid == 2) {
            if (!zs && (pos || !small)) {
                const V<P> is = recip(sig);
                if (lane == 0) lds_st(s_is, is);
            }
        } else if (wid == 3 && bid == 0 && j > 0) {
            if constexpr (!kEarlyW) cx = t_w(j - 1, cx);
        }
        __syncthreads();  // M
        if (wid == 0) {
            if (!zs && lane == 0) {
                lds_st(&s_info[(j * 2 + 0) * P], mul(lds_ld<P>(s_mu), lds_ld<P>(s_iq)));  // 1/mu
                lds_st(&s_info[(j * 2 + 1) * P], x1);
            }
        } else if (wid == 1) {
            // rho = 1/v1, then w_c = a_jc + rho d_c for the columns right of j
            V<P> rho = from_double<P>(1.0);
            if (!zs) {
                const V<P> mu = lds_ld<P>(s_mu);
                rho = (!pos && small) ? neg(recip(sub(mu, x1))) : neg(mul(add(mu, x1), lds_ld<P>(s_is)));
                if (lane > j && lane < W)
                    lds_st(&s_fc[(j * W + lane) * P], fma(lds_ld<P>(&s_hd[lane * P]), lds_ld<P>(&s_tot[lane * P]), rho));
            }
            if (lane == 0) lds_st(&s_rho[j * P], rho);
        } else if (wid == 3 && bid == 0 && j > 0) {
            t_store(j - 1, cx);
        }
        __syncthreads();  // Tb
        // ---- 3. reflector j applied to the columns c > j below row j; mu on the diagonal
        if (!zs) {
            const V<P> mu = lds_ld<P>(s_mu);
            V<P> coef = zero<P>();  // w_c / mu
            if (c > j) coef = mul(lds_ld<P>(&s_fc[(j * W + c) * P]), lds_ld<P>(&s_info[(j * 2 + 0) * P]));
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const long r = rbase + k * rstride;
                const V<P> xk = shfl_md(a[k], src0 + j);  // column j is unchanged below row j
                if (r == dj) {
                    if (c == j) a[k] = mu;
                } else if (r > dj && r < hh && c > j) {
                    a[k] = fma(a[k], coef, xk);
                }
            }
        }
    }
    __syncthreads();
    // ---- 4. the last column's beta and T column; the deferred row updates; v = x rho below
    //         the diagonal; store the panel (rows from the previous diagonal)
    if (bid == 0 && g.wact > 0) {
        if (wid == 2) t_beta(g.wact - 1);
        if (wid == 3) cx = t_w(g.wact - 1, t_g(g.wact - 1));
    }
    const V<P> rc = lds_ld<P>(&s_rho[c * P]);
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const long r = rbase + k * rstride;
        if (r < hh && c < g.wact) {
            const long jr = r - off;  // panel row
            if (jr >= 0 && jr < c) {
                if (!(s_flag[jr] & 1))
                    a[k] = fma(a[k], neg(lds_ld<P>(&s_beta[jr * P])), lds_ld<P>(&s_fc[(jr * W + c) * P]));
            } else if (jr > c && !(s_flag[c] & 1)) {
                a[k] = mul(a[k], rc);
            }
            stm(g.A, g.ps, c * g.lda + r, a[k]);
        }
    }
    __syncthreads();
    if (bid == 0 && wid == 3) {
        if (g.wact > 0) t_store(g.wact - 1, cx);
        for (int jj = g.wact; jj < W; ++jj)
            if (lane < W) stm(g.T, g.tps, (long)jj * W + lane, zero<P>());
    }
}

// One panel launch: workgroup b runs panel_run(g, b).
template <int P, int W, int R, int NT>
__global__ __launch_bounds__(NT) void k_panel(PanelArgs g)
{
    panel_run<P, W, R, NT>(g, blockIdx.x);
}

// ============================================================================ trailing update
// C := C - Y T^T (Y^T C) for the columns right of the panel (those of C, then those of B, as
// one index space).  The work is cut into units of four columns (one per wave) by rb rows, so
// that every launch has many equal units whatever its shape:
//   k_apply_s -- each unit's partial sums Y^T c over its rows (lazy level sums, not rounded);
//   k_apply_t -- per column, the partial sums combined in a fixed order into S = Y^T c, and
//                -U = -T^T S;
//   k_apply_u -- each unit's rows: c -= Y U.
// All three walk their units grid-stride, so a capped grid leaves CUs free for a concurrent
// panel.  Y is staged through LDS per unit; lanes walk rows (unit-stride limb planes).
// most rows per unit: 256, or 128 where W P 256 doubles of staged Y would exceed 64 KiB of LDS
template <int P, int W>
constexpr int rb_max()
{
    return W * P * 256 * 8 <= 65536 ? 256 : 128;
}

struct ApplyArgs {
    const double *Y;  // panel top-left (diagonal) element; Y is unit lower trapezoidal
    long ldy, psy;
    int h, wact;
    const double *T;  // W x W (ld W)
    long tps;
    double *C;  // first trailing column, panel's first row
    long ldc, psc;
    int nc;
    double *B;  // extra columns (right-hand sides), panel's first row
    long ldb, psb;
    int nb;
    int c0, ncol;  // this launch covers columns c0 .. c0 + ncol - 1 of the (C, B) index space
    int rb, nrb;   // rows per unit (a multiple of 64, at most rb_max) and row blocks
    double *part;  // [ncol][nrb][W][P] partial sums
    double *nu;    // [ncol][W][P] -U
};

// Column gc of this launch (null past the end); its plane stride in *cps.
__device__ __forceinline__ double *apply_col(const ApplyArgs &g, int gc, long *cps)
{
    if (gc >= g.ncol) return nullptr;
    const int q = g.c0 + gc;
    if (q < g.nc) {
        *cps = g.psc;
        return g.C + (long)q * g.ldc;
    }
    *cps = g.psb;
    return g.B + (long)(q - g.nc) * g.ldb;
}

template <int P, int W>
__device__ __forceinline__ void stage_y(const ApplyArgs &g, double *sY, long r0, int tid)
{
    for (int e = tid; e < W * g.rb; e += kThreads) {
        const int r = e % g.rb, i = e / g.rb;
        const V<P> y = y_entry<P>(g.Y, g.ldy, g.psy, r0 + r, i, g.h, g.wact);
#pragma unroll
        for (int k = 0; k < P; ++k) sY[(i * P + k) * rb_max<P, W>() + r] = y.x[k];
    }
}

// Sum W lazy accumulators over the 64 lanes of a wave; afterwards s[0] of lane l holds the
// total of accumulator l / (64 / W).  Each level first halves the set a lane keeps (the
// partner keeps the other half), so W accumulators cost W - 1 + 6 - log2(W) additions
// instead of 6 W.
template <int P, int W, int HALF, int M>
__device__ __forceinline__ void reduce_scatter_level(Acc<P> (&s)[W], int lane)
{
    if constexpr (HALF >= 1) {
        const bool hi = (lane & M) != 0;
#pragma unroll
        for (int q = 0; q < HALF; ++q) {
            Acc<P> mine, give;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                mine.s[k] = hi ? s[q + HALF].s[k] : s[q].s[k];
                give.s[k] = hi ? s[q].s[k] : s[q + HALF].s[k];
            }
            acc_add_acc(mine, shfl_xor_acc(give, M));
            s[q] = mine;
        }
        reduce_scatter_level<P, W, HALF / 2, M / 2>(s, lane);
    } else {
#pragma unroll
        for (int m = M; m >= 1; m >>= 1) acc_add_acc(s[0], shfl_xor_acc(s[0], m));
    }
}

template <int P, int W>
__device__ __forceinline__ void reduce_scatter(Acc<P> (&s)[W], int lane)
{
    static_assert(W >= 1 && W <= 32 && (W & (W - 1)) == 0, "reduce_scatter: W a power of two");
    reduce_scatter_level<P, W, W / 2, 32>(s, lane);
}

// Accumulators a lane keeps at once in k_apply_s: all W, or for octo double at most 4 (the
// partial sums of the other columns of Y take further passes over the unit's rows), so that
// the kernel keeps two waves per SIMD.
template <int P, int W>
constexpr int apply_pass_width()
{
    return (P >= 8 && W > 4) ? 4 : W;
}

template <int P, int W>
__global__ __launch_bounds__(kThreads, 2) void k_apply_s(ApplyArgs g)
{
    constexpr int WH = apply_pass_width<P, W>();
    __shared__ double sY[W * P * rb_max<P, W>()];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int ncg = (g.ncol + 3) / 4;
    const int units = ncg * g.nrb;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int cg = u % ncg, rbk = u / ncg;
        const long r0 = (long)rbk * g.rb;
        __syncthreads();
        stage_y<P, W>(g, sY, r0, tid);
        __syncthreads();
        const int gc = cg * 4 + wid;
        long cps = 0;
        const double *col = apply_col(g, gc, &cps);
        if (!col) continue;  // whole wave
#pragma unroll 1
        for (int i0 = 0; i0 < W; i0 += WH) {
            Acc<P> s[WH];
#pragma unroll
            for (int i = 0; i < WH; ++i) s[i] = acc_zero<P>();
            int nterm = 0;
            for (int r = lane; r < g.rb; r += 64) {
                const long gr = r0 + r;
                if (gr < g.h) {
                    const V<P> cv = ldm<P>(col, cps, gr);
#pragma unroll
                    for (int i = 0; i < WH; ++i) {
                        V<P> y;
#pragma unroll
                        for (int k = 0; k < P; ++k) y.x[k] = sY[((i0 + i) * P + k) * rb_max<P, W>() + r];
                        acc_fma_step(s[i], y, cv, nterm);
                    }
                    ++nterm;
                }
            }
            reduce_scatter<P, WH>(s, lane);
            constexpr int LPI = 64 / WH;
            if (lane % LPI == 0) {
                double *dst = g.part + (((long)gc * g.nrb + rbk) * W + i0 + lane / LPI) * P;
#pragma unroll
                for (int k = 0; k < P; ++k) dst[k] = s[0].s[k];
            }
        }
    }
}

template <int P, int W>
__global__ __launch_bounds__(kThreads) void k_apply_t(ApplyArgs g)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int gc = blockIdx.x * 4 + wid; gc < g.ncol; gc += gridDim.x * 4) {
        // lane q adds the partial sums (b, i) = (q / W + 64 k / W, q % W), then the lanes of
        // one i are combined
        Acc<P> t = acc_zero<P>();
        const double *src = g.part + (long)gc * g.nrb * W * P;
        for (int q = lane; q < g.nrb * W; q += 64) {
            Acc<P> o;
#pragma unroll
            for (int k = 0; k < P; ++k) o.s[k] = src[(long)q * P + k];
            acc_add_acc(t, o);
        }
#pragma unroll
        for (int m = W; m < 64; m <<= 1) acc_add_acc(t, shfl_xor_acc(t, m));
        const V<P> S = acc_get(t);  // lane l: S_(l mod W)
        // U_i = sum_{l <= i} T(l, i) S_l: lane p = i W + l (+ 64 k) forms one product, then
        // the W lanes of an i are summed
        constexpr int NQ = (W * W + 63) / 64;
        Acc<P> u[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) u[k] = acc_zero<P>();
        const int l = lane % W;
        const V<P> sl = shfl_md(S, l);
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const int i = (lane + 64 * k) / W;
            if (l <= i && i < g.wact) acc_fma(u[k], ldm<P>(g.T, g.tps, (long)i * W + l), sl);
#pragma unroll
            for (int m = 1; m < W; m <<= 1) acc_add_acc(u[k], shfl_xor_acc(u[k], m));
            if (l == 0 && i < W) {
                const V<P> nv = neg(acc_get(u[k]));
#pragma unroll
                for (int q = 0; q < P; ++q) g.nu[((long)gc * W + i) * P + q] = nv.x[q];
            }
        }
    }
}

template <int P, int W>
__global__ __launch_bounds__(kThreads) void k_apply_u(ApplyArgs g)
{
    __shared__ double sY[W * P * rb_max<P, W>()];
    __shared__ double sU[4][W * P];  // -U of each wave's column
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int ncg = (g.ncol + 3) / 4;
    const int units = ncg * g.nrb;
    for (int u = blockIdx.x; u < units; u += gridDim.x) {
        const int cg = u % ncg, rbk = u / ncg;
        const long r0 = (long)rbk * g.rb;
        __syncthreads();
        stage_y<P, W>(g, sY, r0, tid);
        const int gc = cg * 4 + wid;
        if (gc < g.ncol && lane < W * P) sU[wid][lane] = g.nu[(long)gc * W * P + lane];
        __syncthreads();
        long cps = 0;
        double *col = apply_col(g, gc, &cps);
        if (!col) continue;  // whole wave
        for (int r = lane; r < g.rb; r += 64) {
            const long gr = r0 + r;
            if (gr < g.h) {
                Acc<P> t = acc_from(ldm<P>(col, cps, gr));
#pragma unroll
                for (int i = 0; i < W; ++i) {
                    V<P> y;
#pragma unroll
                    for (int k = 0; k < P; ++k) y.x[k] = sY[(i * P + k) * rb_max<P, W>() + r];
                    acc_fma(t, y, lds_ld<P>(&sU[wid][i * P]));
                }
                stm(col, cps, gr, acc_get(t));
            }
        }
    }
}

// ============================================================================ batched solves
// Many independent least-squares problems (m <= kBatchRows) in one persistent launch.  Each
// workgroup takes the next slot from a counter; a slot names a problem and a member index.
// The plan lists the problems largest m n^2 first and gives the largest a team of T
// workgroups (T consecutive slots at the head of the list, so every team is resident from
// the start), the others one.  A team solves its problem with narrow Householder panels
// (panel_run with T workgroups and the team's own barrier counters and exchange slots), the
// update of the columns right of the panel and of b split over the team's waves (one column
// per wave), a team barrier after each step, and member 0 does the back substitution of
// R x = (Q^T b) with the reciprocals of R's diagonal formed in parallel.  Start and end
// times (wall clock ticks) are recorded per problem.
constexpr int kBatchRows = 512;
constexpr int kTeamMax = 16;      // most workgroups on one problem
constexpr int kTeamSlots = 128;   // most workgroups in teams (T > 1) per batch
constexpr int kTeamCtrs = 2 + kBatchRows / 4;  // team barrier + one counter per panel (W >= 4)

struct BatchDesc {
    int m, n;
    long long a_off, b_off, x_off;  // doubles from the A, b, x base pointers
    int idx;                        // position of the problem in the caller's list
    int team;                       // workgroups on this problem
};

struct BatchArgs {
    const BatchDesc *desc;  // in processing order
    const int *slots;       // per slot: index into desc * kTeamMax + member
    const int *nslots;      // number of slots (device)
    double *A, *b, *x;
    double *scratch;    // per workgroup: beta (kBatchRows*P)
    unsigned *counter;  // zero on entry
    unsigned *tctr;     // per problem: kTeamCtrs barrier counters, zero on entry
    double *xch;        // per problem: T (W^2 P) and panel_run's exchange slots (2 kTeamMax (W^2 + 2W) P)
    int *err;           // set if a team barrier times out
    unsigned spin;      // polls before a team barrier gives up
    int *info;          // per problem
    long long *times;   // per problem: start, end; or null
};

// C := C - Y T^T (Y^T C) for the ncols columns at C0 (plane stride ps, ld lda) and the column
// b0 (plane stride bps, index ncols), h rows from the panel's diagonal; one column per wave,
// columns first, first + step, ... for this wave.
template <int P, int W, int NT, bool STAGED>
__device__ __forceinline__ void batch_update(const double *Y, long lda, long ps, int h, int wact, const double *T,
                                             double *C0, int ncols, double *b0, long bps, int first, int step,
                                             const double *sY)
{
    constexpr int LPI = 64 / W, NQ = (W * W + 63) / 64;
    const int lane = threadIdx.x & 63;
    // Y(r, i): from the LDS copy (limb k of column i at sY[(i P + k) kBatchRows + r]) or global
    auto yv = [&](int r, int i) __attribute__((always_inline)) {
        if constexpr (STAGED) {
            V<P> y;
#pragma unroll
            for (int k = 0; k < P; ++k) y.x[k] = sY[(i * P + k) * kBatchRows + r];
            return y;
        } else {
            return y_entry<P>(Y, lda, ps, r, i, h, wact);
        }
    };
    for (int col = first; col <= ncols; col += step) {
        double *cp = (col < ncols) ? C0 + (long)col * lda : b0;
        const long cps = (col < ncols) ? ps : bps;
        Acc<P> s[W];
#pragma unroll
        for (int i = 0; i < W; ++i) s[i] = acc_zero<P>();
        int nt = 0;
        for (int r = lane; r < h; r += 64) {
            const V<P> cv = ldm<P>(cp, cps, r);
#pragma unroll
            for (int i = 0; i < W; ++i) acc_fma_step(s[i], yv(r, i), cv, nt);
            ++nt;
        }
        reduce_scatter<P, W>(s, lane);
        const V<P> S = acc_get(s[0]);  // lane q: S_(q / LPI)
        // -U_i = -sum_{l <= i} T(l, i) S_l: lane q = i W + l (+ 64 k) forms one product
        const int l = lane % W;
        const V<P> sl = shfl_md(S, l * LPI);
        V<P> un[NQ];
#pragma unroll
        for (int k = 0; k < NQ; ++k) {
            const int i = (lane + 64 * k) / W;
            Acc<P> u = acc_zero<P>();
            if (l <= i && i < wact) acc_fma(u, ldm<P>(T, (long)W * W, (long)i * W + l), sl);
#pragma unroll
            for (int m = 1; m < W; m <<= 1) acc_add_acc(u, shfl_xor_acc(u, m));
            un[k] = neg(acc_get(u));
        }
        V<P> nU[W];
#pragma unroll
        for (int i = 0; i < W; ++i) nU[i] = shfl_md(un[(i * W) / 64], (i * W) % 64);
        for (int r = lane; r < h; r += 64) {
            Acc<P> t = acc_from(ldm<P>(cp, cps, r));
#pragma unroll
            for (int i = 0; i < W; ++i) acc_fma(t, yv(r, i), nU[i]);
            stm(cp, cps, r, acc_get(t));
        }
    }
}

// x = R^-1 y for the n x n upper triangle of A and y = b(0:n) (Algorithm 1 with one tile,
// column-oriented): x_i = y_i / R_ii, then y_t -= R_ti x_i for t < i.  Returns the 1-based
// index of the first exactly-zero diagonal element, or 0.
template <int P, int NT>
__device__ __forceinline__ int batch_backsub(const double *A, long lda, long ps, int n, const double *b, long bps,
                                             double *x, long xps, double *s_y, double *s_r, int *s_zero)
{
    const int tid = threadIdx.x;
    if (tid == 0) *s_zero = INT_MAX;
    __syncthreads();
    for (int i = tid; i < n; i += NT) {
        const V<P> d = ldm<P>(A, ps, (long)i * lda + i);
        const bool z = is_zero(d);
        if (z) atomicMin(s_zero, i);
        lds_st(&s_r[i * P], z ? zero<P>() : recip(d));
        lds_st(&s_y[i * P], ldm<P>(b, bps, i));
    }
    __syncthreads();
    const int zi = *s_zero;
    for (int i = n - 1; i >= 0; --i) {
        const V<P> xi = mul(lds_ld<P>(&s_y[i * P]), lds_ld<P>(&s_r[i * P]));
        if (tid == 0) stm(x, xps, i, xi);
        for (int t = tid; t < i; t += NT)
            lds_st(&s_y[t * P], fma(lds_ld<P>(&s_y[t * P]), neg(ldm<P>(A, ps, (long)i * lda + t)), xi));
        __syncthreads();
    }
    return zi == INT_MAX ? 0 : zi + 1;
}

template <int P, int W, int R, int NT>
__global__ __launch_bounds__(NT) void k_batch(BatchArgs g)
{
    static_assert((NT / W) * R >= kBatchRows, "k_batch: a panel must hold kBatchRows rows");
    constexpr int NW = NT / 64;
    constexpr long WWP = (long)W * W * P;
    constexpr long XCHP = WWP + 2L * kTeamMax * (W * W + 2 * W) * P;
    constexpr bool STAGED = W * P <= 16;  // the panel's Y staged in LDS (at most 64 KiB)
    __shared__ double sY[STAGED ? W * P * kBatchRows : 1];
    __shared__ double s_y[kBatchRows * P];
    __shared__ double s_r[kBatchRows * P];
    __shared__ int s_next, s_zero;
    const int wid = threadIdx.x >> 6;
    double *beta = g.scratch + (long)blockIdx.x * kBatchRows * P;
    const int nslots = *g.nslots;
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_next = (int)atomicAdd(g.counter, 1u);
        __syncthreads();
        const int slot = s_next;
        if (slot >= nslots) break;  // every workgroup leaves once the list is exhausted
        const long long t0 = wall_clock64();
        const int q = g.slots[slot] / kTeamMax, mem = g.slots[slot] % kTeamMax;
        const BatchDesc d = g.desc[q];
        const int team = d.team;
        unsigned *ctr = g.tctr + (long)d.idx * kTeamCtrs;
        unsigned nsync = 0;
        // all members meet (team > 1); the barrier's fences make every member's stores visible
        auto team_sync = [&]() __attribute__((always_inline)) {
            if (team > 1) {
                __syncthreads();
                ++nsync;
                if (wid == 0) grid_sync(ctr, nsync * (unsigned)team, g.err, g.spin);
                __syncthreads();
            }
        };
        double *A = g.A + d.a_off;
        double *bp = g.b + d.b_off;
        double *pxch = g.xch + (long)d.idx * XCHP;
        const long lda = d.m, ps = (long)d.m * d.n;
        for (int c0 = 0; c0 < d.n; c0 += W) {
            PanelArgs pa;
            pa.A = A + (long)c0 * lda + c0;
            pa.lda = lda;
            pa.ps = ps;
            pa.h = d.m - c0;
            pa.wact = (d.n - c0 < W) ? (d.n - c0) : W;
            pa.off = 0;
            pa.Yp = nullptr;
            pa.Tp = nullptr;
            pa.beta = beta + c0;
            pa.bps = kBatchRows;
            pa.T = pxch;  // written by member 0, read by every member after the team barrier
            pa.tps = (long)W * W;
            pa.gpart = pxch + WWP;
            pa.gbar = ctr + 1 + c0 / W;
            pa.err = g.err;
            pa.G = team;
            pa.spin = g.spin;
            panel_run<P, W, R, NT>(pa, mem);
            team_sync();
            if constexpr (STAGED) {
                for (int e = threadIdx.x; e < W * pa.h; e += NT) {
                    const int r = e % pa.h, i = e / pa.h;
                    const V<P> y = y_entry<P>(pa.A, lda, ps, r, i, pa.h, pa.wact);
#pragma unroll
                    for (int k = 0; k < P; ++k) sY[(i * P + k) * kBatchRows + r] = y.x[k];
                }
                __syncthreads();
            }
            batch_update<P, W, NT, STAGED>(pa.A, lda, ps, pa.h, pa.wact, pa.T, A + (long)(c0 + pa.wact) * lda + c0,
                                           d.n - c0 - pa.wact, bp + c0, d.m, mem * NW + wid, team * NW, sY);
            __syncthreads();
            team_sync();
        }
        if (mem == 0) {
            const int inf = batch_backsub<P, NT>(A, lda, ps, d.n, bp, d.m, g.x + d.x_off, d.n, s_y, s_r, &s_zero);
            if (threadIdx.x == 0) {
                const bool late = team > 1 && __hip_atomic_load(g.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
                g.info[d.idx] = late ? -1 : inf;
                if (g.times) {
                    g.times[2L * d.idx] = t0;
                    g.times[2L * d.idx + 1] = wall_clock64();
                }
            }
        }
    }
}

// ============================================================================ iterative refinement
// Mixed-precision kernels of the refined solve: the residual r = b - A x of a PA-limb matrix
// and a PX-limb vector, formed in PX limbs, and x += d with running maxima of |d| and |x|.
constexpr int kResidCols = 128;  // columns per residual chunk

// part[ch][k][i] = level sums of sum_{j in chunk ch} A_ij x_j (not renormalised), one row per
// thread, chunk ch = blockIdx.y of kResidCols columns
template <int PA, int PX>
__global__ __launch_bounds__(kThreads) void k_resid_part(const double *A, long lda, long psa, int m, int n,
                                                         const double *x, long xps, double *part, const int *skip)
{
    __shared__ double sx[kResidCols * PX];
    if (*skip) return;
    const int c0 = blockIdx.y * kResidCols;
    const int c1 = (n - c0 < kResidCols) ? n : c0 + kResidCols;
    for (int j = threadIdx.x; j < c1 - c0; j += kThreads) lds_st(&sx[j * PX], ldm<PX>(x, xps, c0 + j));
    __syncthreads();
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= m) return;
    Acc<PX> acc = acc_zero<PX>();
    for (int j = c0; j < c1; ++j) {
        const V<PA> a = ldm<PA>(A, psa, (long)j * lda + i);
        const V<PX> xv = lds_ld<PX>(&sx[(j - c0) * PX]);
        casc_fma<PX, PA, PX, 0, 0, true>(acc.s, a.x, xv.x, nullptr);
        if (((j - c0 + 1) % kLazy<PX>) == 0) acc = acc_from(acc_get(acc));
    }
#pragma unroll
    for (int k = 0; k < PX; ++k) part[((long)blockIdx.y * PX + k) * m + i] = acc.s[k];
}

// r_i = b_i - c_i - sum_ch part[ch][.][i] (chunks in order; c, PX limbs, may be null)
template <int PX>
__global__ __launch_bounds__(kThreads) void k_resid_fin(const double *b, long bps, const double *c, long cps,
                                                        const double *part, int m, int nch, double *r, long rps,
                                                        const int *skip)
{
    if (*skip) return;
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= m) return;
    Acc<PX> t = acc_from(ldm<PX>(b, bps, i));
    if (c) acc_add(t, neg(ldm<PX>(c, cps, i)));
    for (int ch = 0; ch < nch; ++ch) {
        V<PX> o;
#pragma unroll
        for (int k = 0; k < PX; ++k) o.x[k] = -part[((long)ch * PX + k) * m + i];
        acc_add(t, o);
    }
    stm(r, rps, i, acc_get(t));
}

// g_i = -sum_k A_ki r_k (A of PA limbs, r of PX limbs, formed in PX limbs), rounded to PG <= PX
// limbs: one wave per column of A, the lanes walk its rows
template <int PA, int PX, int PG>
__global__ __launch_bounds__(kThreads) void k_resid_t(const double *A, long lda, long psa, int m, int n,
                                                      const double *r, long rps, double *g, long gps, const int *skip)
{
    if (*skip) return;
    const int lane = threadIdx.x & 63;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= n) return;
    Acc<PX> acc = acc_zero<PX>();
    int nt = 0;
    for (int i = lane; i < m; i += 64) {
        const V<PA> a = ldm<PA>(A, psa, (long)col * lda + i);
        const V<PX> rv = ldm<PX>(r, rps, i);
        casc_fma<PX, PA, PX, 0, 0, true>(acc.s, a.x, rv.x, nullptr);
        if (((++nt) % kLazy<PX>) == 0) acc = acc_from(acc_get(acc));
    }
    const V<PX> t = wave_sum(acc_get(acc));
    if (lane == 0) stm(g, gps, col, resize<PG>(neg(t)));
}

// i < n: y_i = d_i - h_i, then d_i = h_i (d of length >= n; all P limbs)
template <int P>
__global__ __launch_bounds__(kThreads) void k_aug_split(double *d, long dps, const double *h, long hps, double *y,
                                                        long yps, int n, const int *skip)
{
    if (*skip) return;
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const V<P> hv = ldm<P>(h, hps, i);
    stm(y, yps, i, sub(ldm<P>(d, dps, i), hv));
    stm(d, dps, i, hv);
}

// x_i += d_i (d of PD <= PX limbs), i < n
template <int PX, int PD>
__global__ __launch_bounds__(kThreads) void k_md_add(double *x, long xps, const double *d, long dps, int n,
                                                     const int *skip)
{
    if (*skip) return;
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    stm(x, xps, i, add(ldm<PX>(x, xps, i), resize<PX>(ldm<PD>(d, dps, i))));
}

// x_i += d_i (d of PD <= PX limbs); norms[0] = max |d_i|, norms[1] = max |x_i| (leading limbs;
// non-negative doubles ordered as their bit patterns; both zero on entry)
template <int PX, int PD>
__global__ __launch_bounds__(kThreads) void k_refine_add(double *x, long xps, const double *d, long dps, int n,
                                                         unsigned long long *norms, const int *skip)
{
    if (*skip) return;
    const long i = (long)blockIdx.x * kThreads + threadIdx.x;
    if (i >= n) return;
    const V<PD> dv = ldm<PD>(d, dps, i);
    const V<PX> xn = add(ldm<PX>(x, xps, i), resize<PX>(dv));
    stm(x, xps, i, xn);
    atomicMax(&norms[0], (unsigned long long)__double_as_longlong(fabs(dv.x[0])));
    atomicMax(&norms[1], (unsigned long long)__double_as_longlong(fabs(xn.x[0])));
}

// After refinement step it: stop (*done = 1) once x has converged to PX limbs, judged from the
// correction norms d_k = max |d| of the steps so far: converged when d_it <= u max|x|, or when
// the next correction, estimated from the observed contraction as d_it^2 / d_(it-1), would be
// below u max|x| (u = 2^-(53 PX - (PX - 1))).  Otherwise the next step's norms are cleared
// (they hold -1 until a step runs, so the steps taken can be counted).  One thread.
template <int PX>
__global__ void k_refine_check(int it, int iters, double *norms, int *done)
{
    if (threadIdx.x != 0 || *done) return;
    const double u = ldexp(1.0, -(53 * PX - (PX - 1)));
    const double d = norms[2 * it], xm = norms[2 * it + 1];
    bool conv = d <= u * xm;
    if (!conv && it > 0) {
        const double dp = norms[2 * it - 2];
        conv = dp > 0.0 && d * (d / dp) <= u * xm;
    }
    if (conv) {
        *done = 1;
    } else if (it + 1 < iters) {
        norms[2 * it + 2] = 0.0;
        norms[2 * it + 3] = 0.0;
    }
}

namespace {
// norms := -1 (steps not taken), except step 0's pair := 0; *done := 0
__global__ void k_refine_init(double *norms, int iters, int *done)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < 2 * iters) norms[i] = (i < 2) ? 0.0 : -1.0;
    if (i == 0) *done = 0;
}
}  // namespace

namespace {
__global__ void k_zero_f64(double *p, long n)
{
    const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0;
}
}  // namespace

// ============================================================================ small kernels
namespace {
__global__ void k_zero_u32(unsigned *p, int n)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

__global__ void k_copy(const double *src, long sps, double *dst, long dps, int n, int P)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        for (int k = 0; k < P; ++k) dst[k * dps + i] = src[k * sps + i];
}

// k_copy unless *skip
__global__ void k_copy_if(const double *src, long sps, double *dst, long dps, int n, int P, const int *skip)
{
    if (*skip) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        for (int k = 0; k < P; ++k) dst[k * dps + i] = src[k * sps + i];
}

// *d_info = smallest 1-based i with R(i,i) exactly zero, else 0
__global__ __launch_bounds__(kThreads) void k_diag_check(const double *R, long ldr, long ps, int n, int P, int *d_info)
{
    __shared__ int smin;
    if (threadIdx.x == 0) smin = INT_MAX;
    __syncthreads();
    for (int i = threadIdx.x; i < n; i += kThreads) {
        bool z = true;
        for (int k = 0; k < P; ++k) z = z && (R[k * ps + (long)i * ldr + i] == 0.0);
        if (z) atomicMin(&smin, i);
    }
    __syncthreads();
    if (threadIdx.x == 0) *d_info = (smin == INT_MAX) ? 0 : smin + 1;
}

// A grid barrier of the factorisation timed out (*err != 0): *d_info := -1 (x unspecified)
__global__ void k_fold_err(const int *err, int *d_info)
{
    if (threadIdx.x == 0 && *err != 0) *d_info = -1;
}

// *d_info := -1 if a grid barrier timed out, else 0
__global__ void k_set_info(const int *err, int *d_info)
{
    if (threadIdx.x == 0) *d_info = (*err != 0) ? -1 : 0;
}
}  // namespace

// ============================================================================ tile inversion
// X = U^{-1} for upper-triangular tiles, NC columns per workgroup.  Column j solves
// U x = e_j (paper Algorithm 1, stage 1); here all NC columns advance together one row
// at a time from the bottom: x_i = r_i * d_i, then r_k -= U(k,i) x_i for k < i.
// d_i = 1/U(i,i), or supplied (then U's diagonal is not read): forming T from
// K = striu(Y^T Y) + diag(1/beta) passes d_i = beta_i, which also covers beta_i = 0.
struct InvArgs {
    const double *U;  // tile t: U + t * ustride
    long ldu, psu, ustride;
    const double *dsup;  // supplied diagonal (tile t: dsup + t * tile), or null
    long dps;
    double *X;  // tile t: X + t * xstride, ld ldx
    long ldx, psx, xstride;
    int tile;
};

template <int P, int NC, int RPT>
__global__ __launch_bounds__(kThreads) void k_invert(InvArgs g)
{
    constexpr int RG = kThreads / NC;  // row groups
    __shared__ double sD[256 * P];
    __shared__ double sX[2][NC * P];
    __shared__ double sU[2][256 * P];  // column i of the tile; column i-1 is loaded during step i
    const int t = blockIdx.y;
    const int c0 = blockIdx.x * NC;
    const int tid = threadIdx.x;
    const int jl = tid % NC, rg = tid / NC;
    const int j = c0 + jl;
    const double *U = g.U + (long)t * g.ustride;
    double *X = g.X + (long)t * g.xstride;
    const int c1 = min(c0 + NC, g.tile);

    for (int i = tid; i < c1; i += kThreads) {
        V<P> d;
        if (g.dsup)
            d = ldm<P>(g.dsup + (long)t * g.tile, g.dps, i);
        else
            d = recip(ldm<P>(U, g.psu, (long)i * g.ldu + i));
        lds_st(&sD[i * P], d);
    }
    // the rows' right-hand sides stay lazy accumulators (level sums), renormalised every
    // kLazy<P> steps and when their row is published
    Acc<P> r[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int k = rg + q * RG;
        r[q] = acc_from((k == j) ? from_double<P>(1.0) : zero<P>());
        if (j < g.tile && k < g.tile && k > j) stm(X, g.psx, (long)j * g.ldx + k, zero<P>());
    }
    if (c1 > 0 && tid < c1 - 1) lds_st(&sU[(c1 - 1) & 1][tid * P], ldm<P>(U, g.psu, (long)(c1 - 1) * g.ldu + tid));
    __syncthreads();
    for (int i = c1 - 1; i >= 0; --i) {
        const int buf = i & 1;
        // column i-1 (rows above i-1) for the next step, in flight during this one
        V<P> unext = zero<P>();
        const bool pre = i > 0 && tid < i - 1;
        if (pre) unext = ldm<P>(U, g.psu, (long)(i - 1) * g.ldu + tid);
        // owner of row i in column j publishes x_ij
        if (j < c1 && j >= i && (i % RG) == rg) {
            const int qi = i / RG;
            V<P> xv = zero<P>();
#pragma unroll
            for (int q = 0; q < RPT; ++q)
                if (q == qi) xv = mul(acc_get(r[q]), lds_ld<P>(&sD[i * P]));
            lds_st(&sX[buf][jl * P], xv);
            stm(X, g.psx, (long)j * g.ldx + i, xv);
        }
        __syncthreads();
        if (j < c1 && j >= i) {
            const V<P> xv = neg(lds_ld<P>(&sX[buf][jl * P]));
            const bool renorm = ((c1 - i) % kLazy<P>) == 0;
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int k = rg + q * RG;
                if (k < i) {
                    acc_fma(r[q], lds_ld<P>(&sU[buf][k * P]), xv);
                    if (renorm) r[q] = acc_from(acc_get(r[q]));
                }
            }
        }
        // sU[buf ^ 1] was last read in step i + 1, before this step's barrier
        if (pre) lds_st(&sU[buf ^ 1][tid * P], unext);
    }
}

// Blocked tile inversion (Algorithm 1, stage 1, for tiles of 64 rows or more): with the
// 32 x 32 diagonal blocks U_II of every tile inverted first (k_invert, 32 dependent row steps
// instead of one per row of the tile), the blocks of X = U^-1 above the diagonal follow by
// block rows from the bottom, X_IK = -X_II sum_{I < J <= K} U_IJ X_JK.  Workgroup (slice, K - 1,
// tile) forms block column K for NCB of its columns: thread (r, c) holds row r of the block
// row being formed, column c.  The block column is kept in LDS; the diagonal blocks' inverses
// come from Xd (nb x nb each, ld nb, tile t's block I at Xd + (t NB + I) nb^2, plane stride
// dps).
constexpr int kInvNB = 32;  // rows of a diagonal block

template <int P>
constexpr int inv_blk_cols()
{
    return P >= 8 ? 4 : 8;  // columns per workgroup: (tile rows x NCB x P) doubles of LDS <= 64 KiB
}

struct InvBlkArgs {
    const double *U;  // tile t at U + t (tile ldu + tile)
    long ldu, psu;
    const double *Xd;  // diagonal-block inverses
    long dps;
    double *X;  // tile t at X + t tile^2, ld tile, plane stride psx
    long psx;
    int tile;
    const int *skip;
};

template <int P>
__global__ __launch_bounds__(kThreads) void k_inv_blocks(InvBlkArgs g)
{
    constexpr int NB = kInvNB, NCB = inv_blk_cols<P>();
    constexpr int NTH = NB * NCB;  // threads that hold an entry
    __shared__ double sX[256 * NCB * P];  // rows 0 .. (K+1) NB - 1 of this workgroup's columns
    __shared__ double sR[NB * NCB * P];
    if (g.skip && *g.skip) return;
    const int tid = threadIdx.x;
    const int r = tid % NB, c = tid / NB;
    const int K = blockIdx.y + 1, t = blockIdx.z;
    const int col = K * NB + blockIdx.x * NCB + c;  // column of the tile
    const bool act = tid < NTH;
    const long tt = (long)t * g.tile;
    const double *U = g.U + tt * g.ldu + tt;
    double *X = g.X + tt * g.tile;
    const int nbt = g.tile / NB;
    auto xd = [&](int I, int row, int k) __attribute__((always_inline)) {
        return ldm<P>(g.Xd, g.dps, ((long)t * nbt + I) * NB * NB + (long)k * NB + row);
    };
    // the diagonal block X_KK: copied into place and into LDS (block column 1 also places X_00)
    if (act) {
        const V<P> v = xd(K, r, blockIdx.x * NCB + c);
        lds_st(&sX[((K * NB + r) * NCB + c) * P], v);
        stm(X, g.psx, (long)col * g.tile + K * NB + r, v);
        if (K == 1) {
            const int c0 = blockIdx.x * NCB + c;
            stm(X, g.psx, (long)c0 * g.tile + r, xd(0, r, c0));
        }
    }
    __syncthreads();
    for (int I = K - 1; I >= 0; --I) {
        // R(r, c) = sum over the rows k of block rows I+1 .. K of U(I NB + r, k) X(k, c)
        if (act) {
            Acc<P> a0 = acc_zero<P>(), a1 = acc_zero<P>();
            const int k0 = (I + 1) * NB, k1 = (K + 1) * NB;
            int nt = 0;
            for (int k = k0; k < k1; k += 2) {
                acc_fma(a0, ldm<P>(U, g.psu, (long)k * g.ldu + I * NB + r), lds_ld<P>(&sX[(k * NCB + c) * P]));
                acc_fma(a1, ldm<P>(U, g.psu, (long)(k + 1) * g.ldu + I * NB + r), lds_ld<P>(&sX[((k + 1) * NCB + c) * P]));
                if ((++nt) % kLazy<P> == 0) {
                    a0 = acc_from(acc_get(a0));
                    a1 = acc_from(acc_get(a1));
                }
            }
            acc_add_acc(a0, a1);
            lds_st(&sR[(r * NCB + c) * P], acc_get(a0));
        }
        __syncthreads();
        // X_IK(r, c) = -sum_{k >= r} X_II(r, k) R(k, c)
        if (act) {
            Acc<P> a = acc_zero<P>();
            int nt = 0;
            for (int k = r; k < NB; ++k) acc_fma_step(a, xd(I, r, k), lds_ld<P>(&sR[(k * NCB + c) * P]), nt++);
            const V<P> v = neg(acc_get(a));
            lds_st(&sX[((I * NB + r) * NCB + c) * P], v);
            stm(X, g.psx, (long)col * g.tile + I * NB + r, v);
        }
        __syncthreads();
    }
}

// x_i := Xinv_i y_i, one wave per output row
template <int P>
__global__ __launch_bounds__(kThreads) void k_bs_xi(const double *Xi, long ldx, long psx, const double *y, long yps,
                                                   double *x, long xps, int tile, const int *skip)
{
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int row = blockIdx.x * 4 + wid;
    if (row >= tile) return;
    Acc<P> acc = acc_zero<P>();
    int nt = 0;
    for (int c = row + lane; c < tile; c += 64) acc_fma_step(acc, ldm<P>(Xi, psx, (long)c * ldx + row), ldm<P>(y, yps, c), nt++);
    const V<P> s = wave_sum(acc_get(acc));
    if (lane == 0) stm(x, xps, row, s);
}

// The update of the sweep split over column slices, for more workgroups in flight: workgroup
// (row block, slice cs) forms part[cs][row] = R(row, cols of slice cs) x_i(slice) for 64 rows,
// the slice's columns split over the four waves (four accumulators per lane each); k_bs_comb then
// subtracts the slices' partial sums from y in a fixed order.
constexpr int kBsSlices = 4;

template <int P>
__global__ __launch_bounds__(kThreads) void k_bs_upd_part(const double *Rc, long ldr, long psr, const double *xi,
                                                         long xps, double *part, long pps, int rows, int tile,
                                                         const int *skip)
{
    __shared__ double sx[256 * P];
    __shared__ double sp[4][64 * P];
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int per = tile / kBsSlices;
    const int s0 = blockIdx.y * per;
    for (int c = threadIdx.x; c < per; c += kThreads) lds_st(&sx[c * P], ldm<P>(xi, xps, s0 + c));
    __syncthreads();
    const long row = (long)blockIdx.x * 64 + lane;
    const int q = (per + 3) / 4;
    const int cb = wid * q, ce = min(per, cb + q);
    constexpr int NA = 4;
    Acc<P> acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = acc_zero<P>();
    if (row < rows) {
        int nt = 0;
        for (int c = cb; c < ce; c += NA) {
            V<P> u[NA];
#pragma unroll
            for (int k = 0; k < NA; ++k) u[k] = (c + k < ce) ? ldm<P>(Rc, psr, (long)(s0 + c + k) * ldr + row) : zero<P>();
#pragma unroll
            for (int k = 0; k < NA; ++k)
                if (c + k < ce) acc_fma(acc[k], u[k], lds_ld<P>(&sx[(c + k) * P]));
            if ((++nt) % kLazy<P> == 0) {
#pragma unroll
                for (int a = 0; a < NA; ++a) acc[a] = acc_from(acc_get(acc[a]));
            }
        }
#pragma unroll
        for (int a = 1; a < NA; ++a) acc_add_acc(acc[0], acc[a]);
    }
    lds_st(&sp[wid][lane * P], acc_get(acc[0]));
    __syncthreads();
    if (wid == 0 && row < rows) {
        V<P> v = lds_ld<P>(&sp[0][lane * P]);
        for (int w = 1; w < 4; ++w) v = add(v, lds_ld<P>(&sp[w][lane * P]));
        stm(part + (long)blockIdx.y * rows, pps, row, v);
    }
}

// y(row) -= sum over the slices cs of part[cs][row] (in slice order)
template <int P>
__global__ __launch_bounds__(kThreads) void k_bs_comb(const double *part, long pps, double *y, long yps, int rows,
                                                     const int *skip)
{
    if (skip && *skip) return;
    const long row = (long)blockIdx.x * kThreads + threadIdx.x;
    if (row >= rows) return;
    V<P> v = ldm<P>(part, pps, row);
    for (int cs = 1; cs < kBsSlices; ++cs) v = add(v, ldm<P>(part + (long)cs * rows, pps, row));
    stm(y, yps, row, sub(ldm<P>(y, yps, row), v));
}

// The transposed sweep (forward substitution with R^T, whose diagonal tiles have the inverses
// Xinv_i^T): h_i := Xinv_i^T g_i, one wave per output row; skipped while *skip is set
template <int P>
__global__ __launch_bounds__(kThreads) void k_bs_xi_t(const double *Xi, long ldx, long psx, const double *g, long gps,
                                                     double *h, long hps, int tile, const int *skip)
{
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int row = blockIdx.x * 4 + wid;
    if (row >= tile) return;
    Acc<P> acc = acc_zero<P>();
    int nt = 0;
    for (int c = lane; c <= row; c += 64) acc_fma_step(acc, ldm<P>(Xi, psx, (long)row * ldx + c), ldm<P>(g, gps, c), nt++);
    const V<P> s = wave_sum(acc_get(acc));
    if (lane == 0) stm(h, hps, row, s);
}

// g(col) -= sum_k R(k, col) h_k over the tile's rows k, for the ncols columns right of the tile
// (R points at the tile's first row and the first of those columns); one wave per column
template <int P>
__global__ __launch_bounds__(kThreads) void k_bs_upd_t(const double *R, long ldr, long psr, const double *h, long hps,
                                                      double *g, long gps, int ncols, int tile, const int *skip)
{
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63;
    const int col = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (col >= ncols) return;
    Acc<P> acc = acc_zero<P>();
    int nt = 0;
    for (int k = lane; k < tile; k += 64) acc_fma_step(acc, ldm<P>(R, psr, (long)col * ldr + k), ldm<P>(h, hps, k), nt++);
    const V<P> s = wave_sum(acc_get(acc));
    if (lane == 0) stm(g, gps, col, sub(ldm<P>(g, gps, col), s));
}

// y(0:rows) -= R(0:rows, cols of tile i) x_i ; 64 rows per workgroup, the tile's columns
// split over the 4 waves and combined in a fixed order
template <int P>
__global__ __launch_bounds__(kThreads) void k_bs_upd(const double *Rc, long ldr, long psr, const double *xi, long xps,
                                                    double *y, long yps, int rows, int tile, const int *skip)
{
    __shared__ double sx[256 * P];
    __shared__ double sp[4][64 * P];
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c = threadIdx.x; c < tile; c += kThreads) lds_st(&sx[c * P], ldm<P>(xi, xps, c));
    __syncthreads();
    const long row = (long)blockIdx.x * 64 + lane;
    const int q = (tile + 3) / 4;
    const int cb = wid * q, ce = min(tile, cb + q);
    // NA independent accumulators (column k goes to k mod NA), so that NA multiply-adds are
    // in flight at once, added in a fixed order at the end
    constexpr int NA = 4;
    Acc<P> acc[NA];
#pragma unroll
    for (int a = 0; a < NA; ++a) acc[a] = acc_zero<P>();
    if (row < rows) {
        // B columns of R per batch; the next batch's loads are issued before the current
        // batch's multiply-adds, so the HBM latency overlaps the accumulation
        constexpr int B = 32 / P < NA ? NA : 32 / P;
        static_assert(B % NA == 0, "k_bs_upd batch");
        V<P> cur[B], nxt[B];
        auto load = [&](V<P> (&u)[B], int c) __attribute__((always_inline)) {
#pragma unroll
            for (int k = 0; k < B; ++k) u[k] = (c + k < ce) ? ldm<P>(Rc, psr, (long)(c + k) * ldr + row) : zero<P>();
        };
        load(cur, cb);
        int nt = 0;
        for (int c = cb; c < ce; c += B) {
            if (c + B < ce) load(nxt, c + B);
#pragma unroll
            for (int k = 0; k < B; ++k)
                if (c + k < ce) acc_fma(acc[k % NA], cur[k], lds_ld<P>(&sx[(c + k) * P]));
            nt += B / NA;
            if (nt % kLazy<P> == 0) {
#pragma unroll
                for (int a = 0; a < NA; ++a) acc[a] = acc_from(acc_get(acc[a]));
            }
#pragma unroll
            for (int k = 0; k < B; ++k) cur[k] = nxt[k];
        }
#pragma unroll
        for (int a = 1; a < NA; ++a) acc_add_acc(acc[0], acc[a]);
    }
    lds_st(&sp[wid][lane * P], acc_get(acc[0]));
    __syncthreads();
    if (wid == 0 && row < rows) {
        V<P> s = lds_ld<P>(&sp[0][lane * P]);
        for (int w = 1; w < 4; ++w) s = add(s, lds_ld<P>(&sp[w][lane * P]));
        stm(y, yps, row, sub(ldm<P>(y, yps, row), s));
    }
}

// ============================================================================ T, W, Q^T B helpers
// G(l, j) = y_l^T y_j (l < j) for tile block k: block (j, k), one wave per l.
template <int P>
__global__ __launch_bounds__(kThreads) void k_gram(const double *A, long lda, long ps, int m, int tile, double *G,
                                                  long gps)
{
    const int j = blockIdx.x, k = blockIdx.y;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const long kt = (long)k * tile;
    const double *Y = A + kt * lda + kt;
    const int h = m - (int)kt;
    double *Gk = G + kt * tile;
    for (int l = wid; l < tile; l += 4) {
        if (l >= j) {
            if (lane == 0) stm(Gk, gps, (long)j * tile + l, zero<P>());
            continue;
        }
        Acc<P> acc = acc_zero<P>();
        int nt = 0;
        for (int r = j + lane; r < h; r += 64)  // y_j is zero above row j
            acc_fma_step(acc, y_entry<P>(Y, lda, ps, r, l, h, tile), y_entry<P>(Y, lda, ps, r, j, h, tile), nt++);
        const V<P> s = wave_sum(acc_get(acc));
        if (lane == 0) stm(Gk, gps, (long)j * tile + l, s);
    }
}

// W(r, k*tile + j) = -sum_{l<=j} Y_k(r, l) T_k(l, j) for r >= k*tile; zero above.
template <int P>
__global__ __launch_bounds__(kThreads) void k_form_w(const double *A, long lda, long ps, const double *T, long ldt,
                                                    long tps, double *W, long ldw, long wps, int m, int tile)
{
    const long r = (long)blockIdx.x * kThreads + threadIdx.x;
    const int gj = blockIdx.y;
    if (r >= m) return;
    const int k = gj / tile, j = gj % tile;
    const long kt = (long)k * tile;
    if (r < kt) {
        stm(W, wps, (long)gj * ldw + r, zero<P>());
        return;
    }
    const double *Y = A + kt * lda + kt;
    const int h = m - (int)kt;
    Acc<P> acc = acc_zero<P>();
    for (int l = 0; l <= j; ++l)
        acc_fma_step(acc, y_entry<P>(Y, lda, ps, r - kt, l, h, tile), ldm<P>(T, tps, (long)gj * ldt + l), l);
    stm(W, wps, (long)gj * ldw + r, neg(acc_get(acc)));
}

// S(l, c) = Y_k(:, l)^T B(kt:, c): one wave per (l, c)
template <int P>
__global__ __launch_bounds__(kThreads) void k_tn(const double *Y, long lda, long ps, int h, int tile, const double *B,
                                                long ldb, long bps, int nrhs, double *S, long sps, const int *skip)
{
    if (skip && *skip) return;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int l = blockIdx.x * 4 + wid, c = blockIdx.y;
    if (l >= tile || c >= nrhs) return;
    Acc<P> acc = acc_zero<P>();
    int nt = 0;
    for (int r = l + lane; r < h; r += 64)
        acc_fma_step(acc, y_entry<P>(Y, lda, ps, r, l, h, tile), ldm<P>(B, bps, (long)c * ldb + r), nt++);
    const V<P> s = wave_sum(acc_get(acc));
    if (lane == 0) stm(S, sps, (long)c * tile + l, s);
}

// U(i, c) = sum_{l<=i} T(l, i) S(l, c), written over S (U in a separate buffer)
template <int P>
__global__ __launch_bounds__(kThreads) void k_trmm_t(const double *T, long ldt, long tps, const double *S, long sps,
                                                    double *U, int tile, int nrhs, const int *skip)
{
    if (skip && *skip) return;
    const int i = blockIdx.x * kThreads + threadIdx.x, c = blockIdx.y;
    if (i >= tile || c >= nrhs) return;
    Acc<P> acc = acc_zero<P>();
    for (int l = 0; l <= i; ++l) acc_fma_step(acc, ldm<P>(T, tps, (long)i * ldt + l), ldm<P>(S, sps, (long)c * tile + l), l);
    stm(U, sps, (long)c * tile + i, acc_get(acc));
}

// U(i, c) = sum_{l>=i} T(i, l) S(l, c) (T upper triangular, applied without transposition)
template <int P>
__global__ __launch_bounds__(kThreads) void k_trmm_n(const double *T, long ldt, long tps, const double *S, long sps,
                                                    double *U, int tile, int nrhs, const int *skip)
{
    if (skip && *skip) return;
    const int i = blockIdx.x * kThreads + threadIdx.x, c = blockIdx.y;
    if (i >= tile || c >= nrhs) return;
    Acc<P> acc = acc_zero<P>();
    for (int l = i; l < tile; ++l)
        acc_fma_step(acc, ldm<P>(T, tps, (long)l * ldt + i), ldm<P>(S, sps, (long)c * tile + l), l - i);
    stm(U, sps, (long)c * tile + i, acc_get(acc));
}

namespace {
// B(i, c) = 1 if i == c else 0, for i < rows and c < cols (P planes, ld ldb)
__global__ void k_identity(double *B, long ldb, long bps, int rows, int cols, int P)
{
    const long r = (long)blockIdx.x * blockDim.x + threadIdx.x;
    const int c = blockIdx.y;
    if (r >= rows || c >= cols) return;
    for (int k = 0; k < P; ++k) B[k * bps + (long)c * ldb + r] = (k == 0 && r == c) ? 1.0 : 0.0;
}
}  // namespace

// B(kt + r, c) -= sum_l Y_k(r, l) U(l, c)
template <int P>
__global__ __launch_bounds__(kThreads) void k_nn_sub(const double *Y, long lda, long ps, int h, int tile, const double *U,
                                                    long ups, double *B, long ldb, long bps, const int *skip)
{
    if (skip && *skip) return;
    const long r = (long)blockIdx.x * kThreads + threadIdx.x;
    const int c = blockIdx.y;
    if (r >= h) return;
    Acc<P> acc = acc_from(ldm<P>(B, bps, (long)c * ldb + r));
    const long lmax = ((long)tile - 1 < r) ? (long)tile - 1 : r;
    for (int l = 0; l <= (int)lmax; ++l)
        acc_fma_step(acc, neg(y_entry<P>(Y, lda, ps, r, l, h, tile)), ldm<P>(U, ups, (long)c * tile + l), l);
    stm(B, bps, (long)c * ldb + r, acc_get(acc));
}

// ============================================================================ launch timing
// When timing is on (mdls_timing_enable), every launch is bracketed by two events on its
// stream and recorded with the kernel's name, precision and algorithmic md multiply-add
// count.  Defined in mdls_capi.hip.
bool timing_on();
void timing_begin(hipStream_t s, void **ev);
void timing_end(hipStream_t s, void *ev, const char *name, int P, double work);

// Side stream and events of the calling host thread on the current device, created by
// mdls_init (default priority); null when mdls_init has not run on this thread for this device,
// and then the trailing updates run on the caller's stream.
struct SideStream {
    hipStream_t q;
    hipEvent_t ev_panel, ev_wide[2];
};
SideStream *side_stream();

// Process-wide tuning (mdls_set_tuning); the defaults are compile-time constants and nothing is
// read from the environment.  Only panel_variant changes results (the panel's reduction order).
struct Tuning {
    int lookahead;         // 1: trailing updates concurrently on the side stream (when it exists)
    int panel_variant;     // 0: default panel shape, 1: the alternative shape (more rows per thread)
    int apply_grid_cap;    // > 0: workgroups of a concurrent trailing update; 0: the built-in rule
    int apply_wide_rows;   // od: trailing updates of at least this many rows take two workgroups per CU
    unsigned spin_limit;   // polls before a grid barrier gives up
    int split_update;      // 1: the refined solve's factorisation forms Y^T C on the matrix cores
    int cpanel;            // complex QR panels: 0 a launch per column, 1 persistent, 2 persistent for qd and od
};
Tuning tuning();
int apply_grid_cap(int P, int h);
// Workgroups of the panel kernel of precision P (current variant) that can be resident at once on
// the current device (occupancy x compute units); 0 if the device cannot be queried.
int panel_capacity(int P, int m);

#define MDLS_LAUNCH(NAME, PREC, WORK, KERNEL, GRID, BLOCK, STREAM, ...)                       \
    do {                                                                                     \
        void *ev_ = nullptr;                                                                 \
        const bool tm_ = timing_on();                                                        \
        if (tm_) timing_begin((STREAM), &ev_);                                               \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, __VA_ARGS__);                     \
        if (tm_) timing_end((STREAM), ev_, (NAME), (PREC), (double)(WORK));                  \
    } while (0)

// the same with SHM bytes of dynamic LDS
#define MDLS_LAUNCH_SHM(NAME, PREC, WORK, KERNEL, GRID, BLOCK, SHM, STREAM, ...)              \
    do {                                                                                     \
        void *ev_ = nullptr;                                                                 \
        const bool tm_ = timing_on();                                                        \
        if (tm_) timing_begin((STREAM), &ev_);                                               \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, (SHM), STREAM, __VA_ARGS__);                 \
        if (tm_) timing_end((STREAM), ev_, (NAME), (PREC), (double)(WORK));                  \
    } while (0)

// ============================================================================ host side
constexpr int kGMax = 256;  // most workgroups one panel launch may use
constexpr int kCUs = 256;   // compute units of an MI355X

template <int P>
struct Cfg;
template <>
struct Cfg<1> {
    static constexpr int W = 16, NCI = 16;
};
template <>
struct Cfg<2> {
    static constexpr int W = 16, NCI = 16;
};
template <>
struct Cfg<4> {
    static constexpr int W = 8, NCI = 8;
};
template <>
struct Cfg<8> {
    static constexpr int W = 8, NCI = 4;
};

inline int leaf_width(int P)
{
    switch (P) {
    case 1: return Cfg<1>::W;
    case 2: return Cfg<2>::W;
    case 4: return Cfg<4>::W;
    case 8: return Cfg<8>::W;
    }
    return 0;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t beta, leafT, gpart, ctr, err, yw, apart, anu, big, total;
    int W, nleaves, acols;
};

inline Layout layout(int P, int m, int n, int tile)
{
    Layout L{};
    L.W = leaf_width(P);
    L.nleaves = (n + L.W - 1) / L.W;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += align256(bytes);
        return at;
    };
    L.beta = take(sizeof(double) * (size_t)P * n);
    L.leafT = take(sizeof(double) * (size_t)P * L.W * L.W * L.nleaves);
    L.gpart = take(sizeof(double) * 2 * kGMax * (L.W * L.W + 2 * L.W) * P);
    L.ctr = take(sizeof(unsigned) * (size_t)(L.nleaves + 1));
    L.err = take(sizeof(int) * 4);
    L.yw = take(sizeof(double) * (size_t)P * (m > n ? m : n));
    // trailing update: partial sums and -U of at most acols columns per launch
    L.acols = n + 1;
    L.apart = take(sizeof(double) * (size_t)P * L.W * L.acols * ((m + 63) / 64));
    L.anu = take(sizeof(double) * (size_t)P * L.W * L.acols);
    // back substitution inverses / Gram blocks (P x tile x n) or Q^T B scratch (2 x P x tile x 64)
    // tile inverses (P x tile x n), and for blocked inversion the 32 x 32 diagonal blocks' (P x 32 x n)
    const size_t big1 = sizeof(double) * (size_t)P * (tile + (tile >= 64 ? kInvNB : 0)) * n;
    const size_t big2 = sizeof(double) * 2 * (size_t)P * tile * 64;
    L.big = take(big1 > big2 ? big1 : big2);
    L.total = off;
    (void)m;
    return L;
}

inline bool valid_p(int p) { return p == 1 || p == 2 || p == 4 || p == 8; }
inline bool valid_tile(int t) { return t >= 1 && t <= 256; }

template <int P>
struct Ctx {
    char *ws;
    Layout L;
    hipStream_t s;
    // scratch of the split-limb trailing-update product (double double only), or null: then the
    // products Y^T C run on the vector units
    double *split = nullptr;
    double *beta() const { return (double *)(ws + L.beta); }
    double *leafT() const { return (double *)(ws + L.leafT); }
    double *gpart() const { return (double *)(ws + L.gpart); }
    unsigned *ctr() const { return (unsigned *)(ws + L.ctr); }
    int *err() const { return (int *)(ws + L.err); }
    double *yw() const { return (double *)(ws + L.yw); }
    double *apart() const { return (double *)(ws + L.apart); }
    double *anu() const { return (double *)(ws + L.anu); }
    double *big() const { return (double *)(ws + L.big); }
};

struct PanelCfg {
    int nt, r;
};

// Threads per workgroup and rows per thread of the panel kernel: variant 0 (default) or 1 (the
// alternative shape, for tests of the multi-workgroup path and for tuning).
inline PanelCfg panel_cfg(int P, int variant)
{
    switch (P) {
    case 1:
    case 2: return variant ? PanelCfg{512, 8} : PanelCfg{512, 2};
    case 4: return variant ? PanelCfg{256, 4} : PanelCfg{256, 1};
    default: return variant ? PanelCfg{256, 2} : PanelCfg{256, 1};
    }
}

// The shape an m-row factorisation uses: the tuning variant, except that octo-double panels of
// more than 1024 rows always hold two rows per thread (half the workgroups, which leaves more
// compute units to the concurrent trailing update; measured on the 2048 x 1024 solve).
inline int panel_variant_for(int P, int m) { return (tuning().panel_variant || (P >= 8 && m > 1024)) ? 1 : 0; }
inline PanelCfg panel_cfg_for(int P, int m) { return panel_cfg(P, panel_variant_for(P, m)); }

inline int panel_groups(int P, int m)
{
    const PanelCfg cf = panel_cfg_for(P, m);
    const int rows_per_wg = cf.nt / leaf_width(P) * cf.r;
    const int g = (m + rows_per_wg - 1) / rows_per_wg;
    return g < 1 ? 1 : g;
}

template <int P, int W>
void launch_panel(const PanelArgs &a, PanelCfg cf, hipStream_t s)
{
    double work = a.off ? 2.0 * (a.h + a.off) * a.off * a.wact : 0.0;  // the look-ahead update
    for (int j = 0; j < a.wact; ++j) work += (a.h - j - 1) + 2.0 * (a.wact - j - 1) * (a.h - j);
#define MDLS_PANEL_CASE(NT_, R_)                                                                       \
    if (cf.nt == NT_ && cf.r == R_) {                                                                 \
        MDLS_LAUNCH("k_panel", P, work, (k_panel<P, W, R_, NT_>), dim3(a.G), dim3(NT_), s, a);        \
        return;                                                                                       \
    }
    if constexpr (P <= 2) {
        MDLS_PANEL_CASE(512, 8)
        MDLS_PANEL_CASE(512, 2)
    } else if constexpr (P == 4) {
        MDLS_PANEL_CASE(256, 4)
        MDLS_PANEL_CASE(256, 1)
    } else {
        MDLS_PANEL_CASE(256, 1)
        MDLS_PANEL_CASE(256, 2)
    }
#undef MDLS_PANEL_CASE
}

// Resident workgroups per CU of the panel kernel of shape cf (0 if the query fails).
template <int P>
int panel_occupancy_t(PanelCfg cf)
{
    constexpr int W = Cfg<P>::W;
    int per_cu = 0;
    hipError_t e = hipErrorInvalidValue;
#define MDLS_OCC_CASE(NT_, R_) \
    if (cf.nt == NT_ && cf.r == R_) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_panel<P, W, R_, NT_>, NT_, 0);
    if constexpr (P <= 2) {
        MDLS_OCC_CASE(512, 8)
        MDLS_OCC_CASE(512, 2)
    } else if constexpr (P == 4) {
        MDLS_OCC_CASE(256, 4)
        MDLS_OCC_CASE(256, 1)
    } else {
        MDLS_OCC_CASE(256, 1)
        MDLS_OCC_CASE(256, 2)
    }
#undef MDLS_OCC_CASE
    return e == hipSuccess ? per_cu : 0;
}

// Householder QR of A (m x n) in narrow panels; B (nb columns, may be null) receives Q^T B.
// The trailing update (k_apply_s, k_apply_t, k_apply_u) in launches of at most L.acols
// columns.  Rows per unit: the largest of 256, 128, 64 that still gives two units per CU.
// Bytes of Ctx::split for factorisations of n columns: the panel's Householder block staged
// densely (2 planes of kSplitMaxRows x 16), the exact level sums and the column exponents.
inline size_t split_scratch_bytes(int n)
{
    return align256(sizeof(double) * 2 * (size_t)kSplitMaxRows * 16) + split_workspace_bytes(16, n + 1) + 256;
}

// The trailing update of a double-double panel with S = Y^T C formed exactly on the FP64 matrix
// cores (k_split_tn; the precision form's split-limb product), then -U = -T^T S and C -= Y U on
// the vector units as in launch_apply.
template <int P>
void launch_apply_split(const Ctx<P> &cx, ApplyArgs aa, int grid_cap, hipStream_t st)
{
    constexpr int W = Cfg<P>::W;
    static_assert(P == 2 && W <= 16, "split-limb products: double double, at most 16 columns of Y");
    double *Yd = cx.split;
    double *spart = Yd + 2L * kSplitMaxRows * 16;
    const size_t spart_bytes = align256(sizeof(double) * (size_t)((cx.L.acols + 15) / 16) * kSplitK * kSlices * 256);
    int *exps = (int *)((char *)spart + spart_bytes);
    MDLS_LAUNCH("k_stage_y", P, 0, k_stage_y, dim3((unsigned)(((long)aa.h * W + kThreads - 1) / kThreads)), dim3(kThreads),
                st, aa.Y, aa.ldy, aa.psy, aa.h, aa.wact, W, Yd);
    aa.part = cx.apart();
    aa.nu = cx.anu();
    for (int c0 = 0; c0 < aa.nc; c0 += cx.L.acols) {
        aa.c0 = c0;
        aa.ncol = (aa.nc - c0 < cx.L.acols) ? (aa.nc - c0) : cx.L.acols;
        SplitArgs sa{Yd, (long)aa.h, (long)aa.h * W, aa.C + (long)c0 * aa.ldc, aa.ldc, aa.psc, spart, exps, aa.h, W,
                     aa.ncol};
        const int tiles = (aa.ncol + 15) / 16;
        MDLS_LAUNCH("k_split_exp", P, 0, k_split_exp, dim3((W + aa.ncol + 3) / 4), dim3(kThreads), st, sa);
        MDLS_LAUNCH("k_split_tn", P, (double)aa.h * aa.wact * aa.ncol, k_split_tn, dim3(tiles, kSplitK),
                    dim3(64 * kSplitWaves), st, sa);
        MDLS_LAUNCH("k_split_fin", P, 0, k_split_fin_part, dim3(tiles), dim3(256), st, sa, aa.part);
        const int ncg = (aa.ncol + 3) / 4;
        ApplyArgs at = aa;
        at.rb = aa.h;
        at.nrb = 1;  // S is complete: one partial sum per column
        int tgrid = ncg;
        if (grid_cap > 0 && tgrid > grid_cap) tgrid = grid_cap;
        MDLS_LAUNCH("k_apply_t", P, 0.5 * aa.wact * (aa.wact + 1) * aa.ncol, (k_apply_t<P, W>), dim3(tgrid),
                    dim3(kThreads), st, at);
        int rb = rb_max<P, W>();
        while (rb > 64 && (long)ncg * ((aa.h + rb - 1) / rb) < 2L * kCUs) rb >>= 1;
        aa.rb = rb;
        aa.nrb = (aa.h + rb - 1) / rb;
        int grid = ncg * aa.nrb;
        if (grid_cap > 0 && grid > grid_cap) grid = grid_cap;
        MDLS_LAUNCH("k_apply_u", P, (double)aa.h * aa.wact * aa.ncol, (k_apply_u<P, W>), dim3(grid), dim3(kThreads), st,
                    aa);
    }
}

template <int P>
void launch_apply(const Ctx<P> &cx, ApplyArgs aa, int grid_cap, hipStream_t st)
{
    constexpr int W = Cfg<P>::W;
    if constexpr (P == 2) {
        if (cx.split && aa.nb == 0 && aa.h <= kSplitMaxRows) {
            launch_apply_split<P>(cx, aa, grid_cap, st);
            return;
        }
    }
    const int ntot = aa.nc + aa.nb;
    aa.part = cx.apart();
    aa.nu = cx.anu();
    for (int c0 = 0; c0 < ntot; c0 += cx.L.acols) {
        aa.c0 = c0;
        aa.ncol = (ntot - c0 < cx.L.acols) ? (ntot - c0) : cx.L.acols;
        const int ncg = (aa.ncol + 3) / 4;
        int rb = rb_max<P, W>();
        while (rb > 64 && (long)ncg * ((aa.h + rb - 1) / rb) < 2L * kCUs) rb >>= 1;
        aa.rb = rb;
        aa.nrb = (aa.h + rb - 1) / rb;
        int grid = ncg * aa.nrb, tgrid = ncg;
        if (grid_cap > 0 && grid > grid_cap) grid = grid_cap;
        if (grid_cap > 0 && tgrid > grid_cap) tgrid = grid_cap;
        const double half = (double)aa.h * aa.wact * aa.ncol;
        MDLS_LAUNCH("k_apply_s", P, half, (k_apply_s<P, W>), dim3(grid), dim3(kThreads), st, aa);
        MDLS_LAUNCH("k_apply_t", P, 0.5 * aa.wact * (aa.wact + 1) * aa.ncol, (k_apply_t<P, W>), dim3(tgrid),
                    dim3(kThreads), st, aa);
        MDLS_LAUNCH("k_apply_u", P, half, (k_apply_u<P, W>), dim3(grid), dim3(kThreads), st, aa);
    }
}

// Householder QR of A (m x n) in narrow panels of W columns; B (nb columns, may be null)
// receives Q^T B.  Panel l (l > 0) first applies panel l-1 to its own columns (k_panel with
// off = W); apply(l) (k_apply_s, k_apply_t, k_apply_u) updates the columns from panel l+2 on,
// and B.  With look-ahead (default; MDLS_LOOKAHEAD=0 turns it off) apply(l) runs on a side
// stream concurrently with panel l+1:
//   caller: panel(l) -> [wait apply(l-1)] -> panel(l+1) -> [wait apply(l)] -> panel(l+2) ...
//   side:   [wait panel(l)] -> apply(l) -> [wait panel(l+1)] -> apply(l+1) ...
// and its grid is capped so that CUs stay free for the panel's workgroups.
template <int P>
int qr_panels(const Ctx<P> &cx, int m, int n, double *A, long lda, long psa, double *B, long ldb, long psb, int nb)
{
    constexpr int W = Cfg<P>::W;
    const PanelCfg cf = panel_cfg_for(P, m);
    const int rows_per_wg = cf.nt / W * cf.r;
    const int nleaves = cx.L.nleaves;
    const Tuning tu = tuning();
    MDLS_LAUNCH("k_zero", P, 0, k_zero_u32, dim3((nleaves + 1 + 255) / 256), dim3(256), cx.s, cx.ctr(), nleaves + 1);
    MDLS_LAUNCH("k_zero", P, 0, k_zero_u32, dim3(1), dim3(256), cx.s, (unsigned *)cx.err(), 4);
    const long tps = (long)W * W * nleaves;
    SideStream *ss = (nleaves > 1 && tu.lookahead) ? side_stream() : nullptr;
    for (int l = 0; l < nleaves; ++l) {
        const int c0 = l * W;
        const int wact = (n - c0 < W) ? (n - c0) : W;
        const int h = m - c0;
        const int off = (l > 0) ? W : 0;
        PanelArgs pa;
        pa.A = A + (long)c0 * lda + (c0 - off);
        pa.lda = lda;
        pa.ps = psa;
        pa.h = h;
        pa.wact = wact;
        pa.off = off;
        pa.Yp = off ? A + (long)(c0 - W) * lda + (c0 - W) : nullptr;
        pa.Tp = off ? cx.leafT() + (long)(l - 1) * W * W : nullptr;
        pa.beta = cx.beta() + c0;
        pa.bps = n;
        pa.T = cx.leafT() + (long)l * W * W;
        pa.tps = tps;
        pa.gpart = cx.gpart();
        pa.gbar = cx.ctr() + l;
        pa.err = cx.err();
        pa.spin = tu.spin_limit;
        int G = (h + off + rows_per_wg - 1) / rows_per_wg;
        if (G < 1) G = 1;
        pa.G = G;
        if (ss && l >= 2 && hipStreamWaitEvent(cx.s, ss->ev_wide[l & 1], 0) != hipSuccess)  // apply(l-2)
            return MDLS_EHIP;
        launch_panel<P, W>(pa, cf, cx.s);

        // the update of everything right of the next panel, and of B
        const int nc = n - c0 - wact;
        const int nn = (nc < W) ? nc : W;  // the next panel's columns: updated by panel l+1 itself
        ApplyArgs aa;
        aa.Y = A + (long)c0 * lda + c0;
        aa.ldy = lda;
        aa.psy = psa;
        aa.h = h;
        aa.wact = wact;
        aa.T = pa.T;
        aa.tps = tps;
        aa.C = A + (long)(c0 + wact + nn) * lda + c0;
        aa.ldc = lda;
        aa.psc = psa;
        aa.nc = nc - nn;
        aa.B = B ? B + c0 : nullptr;
        aa.ldb = ldb;
        aa.psb = psb;
        aa.nb = B ? nb : 0;
        if (ss) {
            if (hipEventRecord(ss->ev_panel, cx.s) != hipSuccess ||
                hipStreamWaitEvent(ss->q, ss->ev_panel, 0) != hipSuccess)
                return MDLS_EHIP;
            launch_apply<P>(cx, aa, apply_grid_cap(P, h), ss->q);
            if (hipEventRecord(ss->ev_wide[l & 1], ss->q) != hipSuccess) return MDLS_EHIP;
        } else {
            launch_apply<P>(cx, aa, 0, cx.s);
        }
    }
    if (ss && (hipStreamWaitEvent(cx.s, ss->ev_wide[(nleaves - 1) & 1], 0) != hipSuccess ||
               (nleaves >= 2 && hipStreamWaitEvent(cx.s, ss->ev_wide[nleaves & 1], 0) != hipSuccess)))
        return MDLS_EHIP;
    return 0;
}

template <int P>
void invert_tiles(const Ctx<P> &cx, const InvArgs &ia, int ntiles)
{
    constexpr int NC = Cfg<P>::NCI;
    constexpr int RPT = 256 / (kThreads / NC);
    dim3 grid((ia.tile + NC - 1) / NC, ntiles);
    MDLS_LAUNCH("k_invert", P, (double)ntiles * ia.tile * ia.tile * ia.tile / 6.0, (k_invert<P, NC, RPT>), grid,
                dim3(kThreads), cx.s, ia);
}

// Stage 1 of the tiled back substitution (Algorithm 1): *d_info from R's diagonal, and the
// inverses of the n / tile diagonal tiles into Xinv (tile t at Xinv + t tile^2, ld tile, plane
// stride tile n).
template <int P>
void backsub_prep(const Ctx<P> &cx, int n, int tile, const double *R, long ldr, long psr, double *Xinv, int *d_info)
{
    const int N = n / tile;
    MDLS_LAUNCH("k_diag_check", P, 0, k_diag_check, dim3(1), dim3(kThreads), cx.s, R, ldr, psr, n, P, d_info);
    const long xips = (long)tile * n;
    InvArgs ia;
    ia.U = R;
    ia.ldu = ldr;
    ia.psu = psr;
    ia.ustride = (long)tile * (ldr + 1);
    ia.dsup = nullptr;
    ia.dps = 0;
    if (tile < 64 || tile % kInvNB != 0) {
        ia.X = Xinv;
        ia.ldx = tile;
        ia.psx = xips;
        ia.xstride = (long)tile * tile;
        ia.tile = tile;
        invert_tiles<P>(cx, ia, N);
        return;
    }
    // blocked: the 32 x 32 diagonal blocks first (into Xd, after the P planes of Xinv), then the
    // blocks above them by block rows
    double *Xd = Xinv + (long)P * xips;
    const long dps = (long)kInvNB * n;
    ia.ustride = (long)kInvNB * (ldr + 1);
    ia.X = Xd;
    ia.ldx = kInvNB;
    ia.psx = dps;
    ia.xstride = (long)kInvNB * kInvNB;
    ia.tile = kInvNB;
    invert_tiles<P>(cx, ia, n / kInvNB);
    InvBlkArgs ib;
    ib.U = R;
    ib.ldu = ldr;
    ib.psu = psr;
    ib.Xd = Xd;
    ib.dps = dps;
    ib.X = Xinv;
    ib.psx = xips;
    ib.tile = tile;
    ib.skip = nullptr;
    constexpr int NCB = inv_blk_cols<P>();
    const int nbt = tile / kInvNB;
    double work = 0.0;  // md multiply-adds: per block column K, sum over I < K of (K - I) + 1 blocks
    for (int K = 1; K < nbt; ++K) work += (double)(K * (K + 1) / 2 + K) * kInvNB * kInvNB * kInvNB;
    MDLS_LAUNCH("k_inv_blocks", P, work * N, (k_inv_blocks<P>), dim3(kInvNB / NCB, nbt - 1, N), dim3(kThreads), cx.s,
                ib);
}

// Stage 2 (Algorithm 1): for i = N-1 .. 0, x_i := U_i^-1 y_i, then y_j -= R_{j,i} x_i for every
// j < i; y (P planes of n) is overwritten.  Every kernel returns at once while *skip is set.
template <int P>
void backsub_sweep(const Ctx<P> &cx, int n, int tile, const double *R, long ldr, long psr, const double *Xinv,
                   double *y, double *x, long xps, const int *skip)
{
    const int N = n / tile;
    const long xips = (long)tile * n;
    const long yps = n;
    for (int i = N - 1; i >= 0; --i) {
        const long it = (long)i * tile;
        MDLS_LAUNCH("k_bs_xi", P, 0.5 * tile * tile, (k_bs_xi<P>), dim3((tile + 3) / 4), dim3(kThreads), cx.s,
                    Xinv + (long)i * tile * tile, (long)tile, xips, y + it, yps, x + it, xps, tile, skip);
        if (i > 0) {
            const int rows = i * tile;
            if (tile % (4 * kBsSlices) == 0) {
                // the update split over column slices; partial sums in the trailing-update scratch
                double *part = cx.apart();
                MDLS_LAUNCH("k_bs_upd", P, (double)rows * tile, (k_bs_upd_part<P>), dim3((rows + 63) / 64, kBsSlices),
                            dim3(kThreads), cx.s, R + it * ldr, ldr, psr, x + it, xps, part, (long)kBsSlices * rows,
                            rows, tile, skip);
                MDLS_LAUNCH("k_bs_comb", P, 0, (k_bs_comb<P>), dim3((rows + kThreads - 1) / kThreads), dim3(kThreads), cx.s,
                            part, (long)kBsSlices * rows, y, yps, rows, skip);
            } else {
                MDLS_LAUNCH("k_bs_upd", P, (double)rows * tile, (k_bs_upd<P>), dim3((rows + 63) / 64), dim3(kThreads),
                            cx.s, R + it * ldr, ldr, psr, x + it, xps, y, yps, rows, tile, skip);
            }
        }
    }
}

// tiled back substitution of y (P planes of n, in ws.yw); x receives the solution
template <int P>
void backsub_tiles(const Ctx<P> &cx, int n, int tile, const double *R, long ldr, long psr, double *x, long xps,
                   int *d_info)
{
    backsub_prep<P>(cx, n, tile, R, ldr, psr, cx.big(), d_info);
    backsub_sweep<P>(cx, n, tile, R, ldr, psr, cx.big(), cx.yw(), x, xps, nullptr);
}

template <int P>
int solve_t(int m, int n, int tile, double *A, int lda, double *b, double *x, void *ws, int *d_info, hipStream_t s)
{
    Ctx<P> cx{(char *)ws, layout(P, m, n, tile), s};
    const long psa = (long)lda * n;
    if (qr_panels<P>(cx, m, n, A, lda, psa, b, m, m, 1) != 0) return MDLS_EHIP;
    MDLS_LAUNCH("k_copy", P, 0, k_copy, dim3((n + 255) / 256), dim3(256), s, b, (long)m, cx.yw(), (long)n, n, P);
    backsub_tiles<P>(cx, n, tile, A, lda, psa, x, n, d_info);
    MDLS_LAUNCH("k_fold_err", P, 0, k_fold_err, dim3(1), dim3(64), s, cx.err(), d_info);
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

template <int P>
int qr_impl(int m, int n, int tile, double *A, int lda, double *beta, double *T, int ldt, void *ws, int *d_info,
            hipStream_t s, double *split)
{
    Ctx<P> cx{(char *)ws, layout(P, m, n, tile), s};
    cx.split = split;
    const long psa = (long)lda * n;
    if (qr_panels<P>(cx, m, n, A, lda, psa, nullptr, 0, 0, 0) != 0) return MDLS_EHIP;
    if (beta)
        MDLS_LAUNCH("k_copy", P, 0, k_copy, dim3((n + 255) / 256), dim3(256), s, cx.beta(), (long)n, beta, (long)n, n,
                    P);
    if (d_info) MDLS_LAUNCH("k_set_info", P, 0, k_set_info, dim3(1), dim3(64), s, cx.err(), d_info);
    if (T) {
        const int N = n / tile;
        double *G = cx.big();
        const long gps = (long)tile * n;
        MDLS_LAUNCH("k_gram", P, 0, (k_gram<P>), dim3(tile, N), dim3(kThreads), s, A, (long)lda, psa, m, tile, G, gps);
        InvArgs ia;
        ia.U = G;
        ia.ldu = tile;
        ia.psu = gps;
        ia.ustride = (long)tile * tile;
        ia.dsup = cx.beta();
        ia.dps = n;
        ia.X = T;
        ia.ldx = ldt;
        ia.psx = (long)ldt * n;
        ia.xstride = (long)tile * ldt;
        ia.tile = tile;
        invert_tiles<P>(cx, ia, N);
    }
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

template <int P>
int qr_t(int m, int n, int tile, double *A, int lda, double *beta, double *T, int ldt, void *ws, int *d_info,
         hipStream_t s)
{
    return qr_impl<P>(m, n, tile, A, lda, beta, T, ldt, ws, d_info, s, nullptr);
}

// The double-double QR with its trailing-update products Y^T C on the matrix cores (split ->
// split_scratch_bytes(n) bytes); the refined solve's factorisation.
template <int P>
int qr_split_t(int m, int n, int tile, double *A, int lda, double *T, int ldt, void *ws, double *split, hipStream_t s)
{
    return qr_impl<P>(m, n, tile, A, lda, nullptr, T, ldt, ws, nullptr, s, split);
}

// B := Q^T B by the tile blocks in order, B := B - Y_k T_k^T (Y_k^T B), 64 columns of B at a
// time; S and U are scratch of P tile 64 doubles each.  Every kernel returns at once while
// *skip is set (skip may be null).
template <int P>
void apply_qt_blocks(int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *B, int ldb,
                     int nrhs, double *S, double *U, const int *skip, hipStream_t s)
{
    const long psa = (long)lda * n, tps = (long)ldt * n, bps = (long)ldb * nrhs;
    const long sps = (long)tile * 64;
    const int N = n / tile;
    for (int c0 = 0; c0 < nrhs; c0 += 64) {
        const int nc = (nrhs - c0 < 64) ? nrhs - c0 : 64;
        double *Bc = B + (long)c0 * ldb;
        for (int k = 0; k < N; ++k) {
            const long kt = (long)k * tile;
            const double *Y = A + kt * lda + kt;
            const int h = m - (int)kt;
            MDLS_LAUNCH("k_tn", P, (double)h * tile * nc, (k_tn<P>), dim3((tile + 3) / 4, nc), dim3(kThreads), s, Y,
                        (long)lda, psa, h, tile, Bc + kt, (long)ldb, bps, nc, S, sps, skip);
            MDLS_LAUNCH("k_trmm_t", P, 0.5 * tile * tile * nc, (k_trmm_t<P>), dim3((tile + kThreads - 1) / kThreads, nc),
                        dim3(kThreads), s, T + kt * ldt, (long)ldt, tps, S, sps, U, tile, nc, skip);
            MDLS_LAUNCH("k_nn_sub", P, (double)h * tile * nc, (k_nn_sub<P>), dim3((h + kThreads - 1) / kThreads, nc),
                        dim3(kThreads), s, Y, (long)lda, psa, h, tile, U, sps, Bc + kt, (long)ldb, bps, skip);
        }
    }
}

template <int P>
int apply_qt_t(int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *B, int ldb, int nrhs,
               void *ws, hipStream_t s)
{
    Ctx<P> cx{(char *)ws, layout(P, m, n, tile), s};
    double *S = cx.big();
    apply_qt_blocks<P>(m, n, tile, A, lda, T, ldt, B, ldb, nrhs, S, S + (size_t)P * tile * 64, nullptr, s);
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

// B := Q B = Q_0 Q_1 ... Q_{N-1} B with Q_k = I - Y_k T_k Y_k^T: the tiles in reverse order,
// B -= Y_k T_k (Y_k^T B) (the paper forms Q itself, Algorithm 2; with B = I this is that Q).
// S and U are scratch of P tile 64 doubles each; every kernel returns at once while *skip is set.
template <int P>
void apply_q_blocks(int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *B, int ldb,
                    int nrhs, double *S, double *U, const int *skip, hipStream_t s)
{
    const long psa = (long)lda * n, tps = (long)ldt * n, bps = (long)ldb * nrhs;
    const long sps = (long)tile * 64;
    const int N = n / tile;
    for (int c0 = 0; c0 < nrhs; c0 += 64) {
        const int nc = (nrhs - c0 < 64) ? nrhs - c0 : 64;
        double *Bc = B + (long)c0 * ldb;
        for (int k = N - 1; k >= 0; --k) {
            const long kt = (long)k * tile;
            const double *Y = A + kt * lda + kt;
            const int h = m - (int)kt;
            MDLS_LAUNCH("k_tn", P, (double)h * tile * nc, (k_tn<P>), dim3((tile + 3) / 4, nc), dim3(kThreads), s, Y,
                        (long)lda, psa, h, tile, Bc + kt, (long)ldb, bps, nc, S, sps, skip);
            MDLS_LAUNCH("k_trmm_n", P, 0.5 * tile * tile * nc, (k_trmm_n<P>), dim3((tile + kThreads - 1) / kThreads, nc),
                        dim3(kThreads), s, T + kt * ldt, (long)ldt, tps, S, sps, U, tile, nc, skip);
            MDLS_LAUNCH("k_nn_sub", P, (double)h * tile * nc, (k_nn_sub<P>), dim3((h + kThreads - 1) / kThreads, nc),
                        dim3(kThreads), s, Y, (long)lda, psa, h, tile, U, sps, Bc + kt, (long)ldb, bps, skip);
        }
    }
}

template <int P>
int apply_q_t(int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *B, int ldb, int nrhs,
              void *ws, hipStream_t s)
{
    Ctx<P> cx{(char *)ws, layout(P, m, n, tile), s};
    double *S = cx.big();
    apply_q_blocks<P>(m, n, tile, A, lda, T, ldt, B, ldb, nrhs, S, S + (size_t)P * tile * 64, nullptr, s);
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

// Q(:, 0:ncols) := the first ncols columns of Q (m x m orthogonal factor), ld ldq
template <int P>
int form_q_t(int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *Q, int ldq, int ncols,
             void *ws, hipStream_t s)
{
    const long qps = (long)ldq * ncols;
    MDLS_LAUNCH("k_identity", P, 0, k_identity, dim3((m + 255) / 256, ncols), dim3(256), s, Q, (long)ldq, qps, m, ncols,
                P);
    return apply_q_t<P>(m, n, tile, A, lda, T, ldt, Q, ldq, ncols, ws, s);
}

template <int P>
int form_w_t(int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *W, int ldw,
             hipStream_t s)
{
    MDLS_LAUNCH("k_form_w", P, 0, (k_form_w<P>), dim3((m + kThreads - 1) / kThreads, n), dim3(kThreads), s, A, (long)lda,
                       (long)lda * n, T, (long)ldt, (long)ldt * n, W, (long)ldw, (long)ldw * n, m, tile);
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

template <int P>
int backsub_t(int n, int tile, const double *R, int ldr, double *x, void *ws, int *d_info, hipStream_t s)
{
    Ctx<P> cx{(char *)ws, layout(P, n, n, tile), s};
    MDLS_LAUNCH("k_copy", P, 0, k_copy, dim3((n + 255) / 256), dim3(256), s, x, (long)n, cx.yw(), (long)n, n, P);
    backsub_tiles<P>(cx, n, tile, R, ldr, (long)ldr * n, x, n, d_info);
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

// ---------------------------------------------------------------- batched solves (host)
// Kernel variants (threads, panel width, rows per thread) tried by the autotuner; each holds
// kBatchRows rows per panel.
constexpr int kBatchVariants = 3;
constexpr int kBatchWMax = 16;

inline int batch_variants(int P) { return (P == 2 || P == 4) ? kBatchVariants : 0; }

struct BatchLayout {
    size_t plan, slots, nslots, ctr, tctr, xch, scratch, total;
    int maxgrid;
};

inline BatchLayout batch_layout(int P, int count)
{
    BatchLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        size_t at = off;
        off += align256(bytes);
        return at;
    };
    const size_t cnt = (size_t)(count > 0 ? count : 1);
    const size_t xchp = ((size_t)kBatchWMax * kBatchWMax + 2 * (size_t)kTeamMax * (kBatchWMax * kBatchWMax + 2 * kBatchWMax)) * P;
    L.maxgrid = 8 * kCUs;
    L.plan = take(sizeof(BatchDesc) * cnt);
    L.slots = take(sizeof(int) * cnt * kTeamMax);
    L.nslots = take(sizeof(int));
    L.ctr = take(sizeof(unsigned) * 64);  // [0] slot counter, [1] barrier time-out flag
    L.tctr = take(sizeof(unsigned) * cnt * kTeamCtrs);
    L.xch = take(sizeof(double) * cnt * xchp);
    L.scratch = take(sizeof(double) * (size_t)L.maxgrid * kBatchRows * P);
    L.total = off;
    return L;
}

// Order and teams of a batch: problems largest m n^2 first (longest processing time
// first); a problem whose work (m n^2 - n^3/3 multiply-adds) is at least twice the average
// work per resident workgroup (total / 2 kCUs) gets that many workgroups, at most kTeamMax,
// while at most kTeamSlots workgroups are in teams.  Returns the slot list (problem index
// in the sorted plan * kTeamMax + member).
inline std::vector<int> batch_schedule(std::vector<BatchDesc> &plan)
{
    auto work = [](const BatchDesc &d) { return (double)d.m * d.n * d.n - (double)d.n * d.n * d.n / 3.0 + d.n; };
    std::stable_sort(plan.begin(), plan.end(), [&](const BatchDesc &x, const BatchDesc &y) { return work(x) > work(y); });
    double total = 0.0;
    for (const BatchDesc &d : plan) total += work(d);
    const double per = total / (2.0 * kCUs);
    int used = 0;
    std::vector<int> slots;
    for (size_t q = 0; q < plan.size(); ++q) {
        int t = (int)(work(plan[q]) / per);
        if (t > kTeamMax) t = kTeamMax;
        if (t < 2 || used + t > kTeamSlots)
            t = 1;
        else
            used += t;
        plan[q].team = t;
        for (int k = 0; k < t; ++k) slots.push_back((int)q * kTeamMax + k);
    }
    return slots;
}

template <int P, int W, int R, int NT>
int launch_batch(BatchArgs a, int count, int maxgrid, hipStream_t s)
{
    int per_cu = 0, cus = 0, dev = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_batch<P, W, R, NT>, NT, 0) != hipSuccess || per_cu < 1)
        per_cu = 1;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) !=
                                                hipSuccess || cus < 1)
        cus = kCUs;
    // every workgroup of the grid is resident at once, so the members of every team meet
    int grid = per_cu * cus;
    if (grid > maxgrid) grid = maxgrid;
    if (grid > count * kTeamMax) grid = count * kTeamMax;
    const int nz = count * kTeamCtrs;
    MDLS_LAUNCH("k_zero", P, 0, k_zero_u32, dim3(1), dim3(64), s, a.counter, 64);
    MDLS_LAUNCH("k_zero", P, 0, k_zero_u32, dim3((nz + 255) / 256), dim3(256), s, a.tctr, nz);
    MDLS_LAUNCH("k_batch", P, 0, (k_batch<P, W, R, NT>), dim3(grid), dim3(NT), s, a);
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

template <int P>
int batch_solve_t(int count, double *A, double *b, double *x, int variant, void *ws, int *d_info, long long *d_times,
                  hipStream_t s)
{
    const BatchLayout L = batch_layout(P, count);
    char *w = (char *)ws;
    BatchArgs a;
    a.desc = (const BatchDesc *)(w + L.plan);
    a.slots = (const int *)(w + L.slots);
    a.nslots = (const int *)(w + L.nslots);
    a.A = A;
    a.b = b;
    a.x = x;
    a.scratch = (double *)(w + L.scratch);
    a.counter = (unsigned *)(w + L.ctr);
    a.err = (int *)(w + L.ctr) + 1;
    a.spin = tuning().spin_limit;
    a.tctr = (unsigned *)(w + L.tctr);
    a.xch = (double *)(w + L.xch);
    a.info = d_info;
    a.times = d_times;
    if constexpr (P == 2) {
        switch (variant) {
        case 0: return launch_batch<2, 8, 16, 256>(a, count, L.maxgrid, s);
        case 1: return launch_batch<2, 8, 8, 512>(a, count, L.maxgrid, s);
        case 2: return launch_batch<2, 4, 8, 256>(a, count, L.maxgrid, s);
        }
    } else if constexpr (P == 4) {
        switch (variant) {
        case 0: return launch_batch<4, 4, 8, 256>(a, count, L.maxgrid, s);
        case 1: return launch_batch<4, 4, 4, 512>(a, count, L.maxgrid, s);
        case 2: return launch_batch<4, 8, 16, 256>(a, count, L.maxgrid, s);
        }
    }
    return MDLS_EUNSUPPORTED;
}

#define MDLS_BATCH_FOR_PRECISION(X, P) \
    X template int batch_solve_t<P>(int, double *, double *, double *, int, void *, int *, long long *, hipStream_t);

// ---------------------------------------------------------------- refined solve (host)
// Least squares to PX limbs from a double-double factorisation: F := A, QR of F in dd (with
// the tile T factors), the inverses of R's diagonal tiles (once), then at most `iters` steps,
// stopping on the device once the correction norms show convergence (k_refine_check; the
// remaining steps' kernels return at once, so the call stays asynchronous).
//  * m == n (a square system is consistent): x := 0, r := b; each step d := R^-1 (Q^T r) in dd
//    (r rounded to dd), x += d, r := b - A x in PX limbs.
//  * m > n: refinement of the augmented system [I A; A^T 0][r; x] = [b; 0] (Bjorck 1967), which
//    refines the residual with x, so that a nonzero residual does not limit the accuracy:
//    x := 0, r := 0; each step f := b - r - A x and g := -A^T r in PX limbs, rounded to dd;
//    h := R^-T g (forward substitution with the transposed tile inverses), d := Q^T f,
//    dx := R^-1 (d(0:n) - h), dr := Q [h; d(n:m)], x += dx, r += dr.
// Converges when kappa(A) 2^-105 << 1; norms[2 it], norms[2 it + 1] receive max |dx| and max |x|
// of step it, -1 for steps not taken.
inline size_t refine_extra_bytes(int px, int m, int n, int tile)
{
    const size_t nch = (size_t)(n + kResidCols - 1) / kResidCols;
    return sizeof(double) * (2 * (size_t)n * tile + 2 * (size_t)px * m + 2 * (size_t)m + 6 * (size_t)n +
                             nch * px * m + 4 * (size_t)tile * 64) +
           10 * 256 + split_scratch_bytes(n);
}

template <int PX>
int refine_t(int m, int n, int tile, const double *A, int lda, const double *b, double *x, int iters, double *F,
             void *ws, int *d_info, double *norms, hipStream_t s)
{
    const Layout L = layout(2, m, n, tile);
    Ctx<2> cx{(char *)ws, L, s};
    char *e = (char *)ws + align256(L.total);
    auto take = [&](size_t bytes) {
        char *p = e;
        e += align256(bytes);
        return p;
    };
    const int nch = (n + kResidCols - 1) / kResidCols;
    const bool aug = m > n;
    double *T = (double *)take(sizeof(double) * 2 * (size_t)n * tile);
    double *r = (double *)take(sizeof(double) * (size_t)PX * m);    // residual b - A x, or f
    double *rr = (double *)take(sizeof(double) * (size_t)PX * m);   // augmented form: the residual iterate
    double *rdd = (double *)take(sizeof(double) * 2 * (size_t)m);
    double *dd = (double *)take(sizeof(double) * 2 * (size_t)n);
    double *gdd = (double *)take(sizeof(double) * 2 * (size_t)n);
    double *hdd = (double *)take(sizeof(double) * 2 * (size_t)n);
    double *part = (double *)take(sizeof(double) * (size_t)nch * PX * m);
    double *S = (double *)take(sizeof(double) * 4 * (size_t)tile * 64);
    int *done = (int *)take(sizeof(int) * 4);
    double *split = (double *)take(split_scratch_bytes(n));
    double *U = S + 2 * (size_t)tile * 64;
    const long psa = (long)lda * n;
    const int N = n / tile;
    MDLS_LAUNCH("k_copy", PX, 0, k_copy, dim3((unsigned)((psa + 255) / 256)), dim3(256), s, A, psa, F, psa, (int)psa, 2);
    MDLS_LAUNCH("k_copy", PX, 0, k_copy, dim3((m + 255) / 256), dim3(256), s, b, (long)m, r, (long)m, m, PX);
    MDLS_LAUNCH("k_zero", PX, 0, k_zero_f64, dim3((PX * n + 255) / 256), dim3(256), s, x, (long)PX * n);
    if (aug) {
        MDLS_LAUNCH("k_zero", PX, 0, k_zero_f64, dim3((PX * m + 255) / 256), dim3(256), s, rr, (long)PX * m);
        MDLS_LAUNCH("k_zero", PX, 0, k_zero_f64, dim3((2 * n + 255) / 256), dim3(256), s, gdd, 2L * n);
    }
    MDLS_LAUNCH("k_refine_init", PX, 0, k_refine_init, dim3((2 * iters + 255) / 256), dim3(256), s, norms, iters, done);
    // with MDLS_TUNE_SPLIT_UPDATE the factorisation's trailing-update products Y^T C run on the
    // FP64 matrix cores (split limbs); by default on the vector units
    int rc = qr_split_t<2>(m, n, tile, F, lda, T, tile, ws, tuning().split_update ? split : nullptr, s);
    if (rc != 0) return rc;
    double *Xinv = cx.big();
    const long xips = (long)tile * n;
    backsub_prep<2>(cx, n, tile, F, lda, psa, Xinv, d_info);
    for (int it = 0; it < iters; ++it) {
        if (it > 0) {
            // r := b - A x (square), f := b - r - A x and g := -A^T r (augmented), in PX limbs
            MDLS_LAUNCH("k_resid_part", PX, (double)m * n, (k_resid_part<2, PX>), dim3((m + kThreads - 1) / kThreads, nch),
                        dim3(kThreads), s, A, (long)lda, psa, m, n, x, (long)n, part, done);
            MDLS_LAUNCH("k_resid_fin", PX, 0, (k_resid_fin<PX>), dim3((m + kThreads - 1) / kThreads), dim3(kThreads), s, b,
                        (long)m, aug ? rr : nullptr, (long)m, part, m, nch, r, (long)m, done);
            if (aug)
                MDLS_LAUNCH("k_resid_t", PX, (double)m * n, (k_resid_t<2, PX, 2>), dim3((n + 3) / 4), dim3(kThreads), s, A,
                            (long)lda, psa, m, n, rr, (long)m, gdd, (long)n, done);
        }
        MDLS_LAUNCH("k_copy", PX, 0, k_copy_if, dim3((m + 255) / 256), dim3(256), s, r, (long)m, rdd, (long)m, m, 2, done);
        if (aug) {
            // h := R^-T g: for each tile from the top, h_i = Xinv_i^T g_i, then g_j -= R_ij^T h_i
            for (int i = 0; i < N; ++i) {
                const long it0 = (long)i * tile;
                MDLS_LAUNCH("k_bs_xi_t", PX, 0.5 * tile * tile, (k_bs_xi_t<2>), dim3((tile + 3) / 4), dim3(kThreads), s,
                            Xinv + (long)i * tile * tile, (long)tile, xips, gdd + it0, (long)n, hdd + it0, (long)n, tile,
                            done);
                const int rest = n - (int)it0 - tile;
                if (rest > 0)
                    MDLS_LAUNCH("k_bs_upd_t", PX, (double)rest * tile, (k_bs_upd_t<2>), dim3((rest + 3) / 4),
                                dim3(kThreads), s, F + (it0 + tile) * lda + it0, (long)lda, psa, hdd + it0, (long)n,
                                gdd + it0 + tile, (long)n, rest, tile, done);
            }
        }
        apply_qt_blocks<2>(m, n, tile, F, lda, T, tile, rdd, m, 1, S, U, done, s);
        if (aug)
            MDLS_LAUNCH("k_aug_split", PX, 0, (k_aug_split<2>), dim3((n + kThreads - 1) / kThreads), dim3(kThreads), s,
                        rdd, (long)m, hdd, (long)n, cx.yw(), (long)n, n, done);
        else
            MDLS_LAUNCH("k_copy", PX, 0, k_copy_if, dim3((n + 255) / 256), dim3(256), s, rdd, (long)m, cx.yw(), (long)n,
                        n, 2, done);
        backsub_sweep<2>(cx, n, tile, F, lda, psa, Xinv, cx.yw(), dd, n, done);
        MDLS_LAUNCH("k_refine_add", PX, 0, (k_refine_add<PX, 2>), dim3((n + kThreads - 1) / kThreads), dim3(kThreads), s,
                    x, (long)n, dd, (long)n, n, (unsigned long long *)(norms + 2 * it), done);
        if (aug) {
            apply_q_blocks<2>(m, n, tile, F, lda, T, tile, rdd, m, 1, S, U, done, s);
            MDLS_LAUNCH("k_md_add", PX, 0, (k_md_add<PX, 2>), dim3((m + kThreads - 1) / kThreads), dim3(kThreads), s, rr,
                        (long)m, rdd, (long)m, m, done);
        }
        MDLS_LAUNCH("k_refine_check", PX, 0, (k_refine_check<PX>), dim3(1), dim3(64), s, it, iters, norms, done);
    }
    MDLS_LAUNCH("k_fold_err", PX, 0, k_fold_err, dim3(1), dim3(64), s, cx.err(), d_info);
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

#define MDLS_REFINE_FOR_PRECISION(X, P) \
    X template int refine_t<P>(int, int, int, const double *, int, const double *, double *, int, double *, void *, \
                               int *, double *, hipStream_t);

#define MDLS_FOR_PRECISION(X, P)                                                                        \
    X template int solve_t<P>(int, int, int, double *, int, double *, double *, void *, int *, hipStream_t);     \
    X template int qr_t<P>(int, int, int, double *, int, double *, double *, int, void *, int *, hipStream_t); \
    X template int qr_split_t<P>(int, int, int, double *, int, double *, int, void *, double *, hipStream_t); \
    X template int apply_qt_t<P>(int, int, int, const double *, int, const double *, int, double *, int, int,   \
                                 void *, hipStream_t);                                                         \
    X template int form_w_t<P>(int, int, int, const double *, int, const double *, int, double *, int,         \
                               hipStream_t);                                                                   \
    X template int backsub_t<P>(int, int, const double *, int, double *, void *, int *, hipStream_t);          \
    X template int apply_q_t<P>(int, int, int, const double *, int, const double *, int, double *, int, int,    \
                                void *, hipStream_t);                                                          \
    X template int form_q_t<P>(int, int, int, const double *, int, const double *, int, double *, int, int,     \
                               void *, hipStream_t);                                                          \
    X template int panel_occupancy_t<P>(PanelCfg);

}  // namespace mdls_impl
