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
//     k_apply  -- the trailing update C := C + Y (W^T C) = C - Y T^T (Y^T C) (paper's
//                 "YWT*C" and "R + YWTC" fused), applied to every column right of the panel and
//                 to the right-hand side, so Q^T b comes out of the factorisation.
//   Back substitution (Section 2, Algorithm 1):
//     k_invert -- invert the diagonal tiles (all columns of a tile in parallel, one row step at
//                 a time);
//     k_bs_xi  -- x_i := U_i^{-1} b_i;
//     k_bs_upd -- b_j -= A_{j,i} x_i for every j < i at once.
//
// Multiple-double numbers are P limb planes (limb 0 most significant); see md.hpp for the
// arithmetic.
#include <climits>
#include <cstdint>
#include <cstdlib>

#pragma once
#include "mdls.h"
#include "mdls_kernels.hpp"

namespace mdls_impl {
using namespace mdk;

// ============================================================================ panel kernel
struct PanelArgs {
    double *A;  // top-left (diagonal) element of the panel
    long lda, ps;
    int h, wact;   // panel rows (from the diagonal down), active columns (<= W)
    double *beta;  // beta of the panel's first column, plane stride bps
    long bps;
    double *T;  // panel T, W x W column-major (ld W), plane stride tps
    long tps;
    double *gpart;  // [2][G][2W][P] exchange slots between workgroups
    unsigned *gbar; // barrier counter of this launch, zero on entry
    int *err;       // set to 1 if a barrier times out
    int G;          // workgroups in the launch
};

// All workgroups of the launch meet here (called by one whole wave per workgroup).  The
// spin is bounded: a timed-out barrier raises *err and lets the wave continue, so the grid
// always drains.
__device__ inline void grid_sync(unsigned *ctr, unsigned target, int *err)
{
    const int lane = threadIdx.x & 63;
    __threadfence();
    if (lane == 0) {
        __hip_atomic_fetch_add(ctr, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        unsigned spins = 0;
        while (__hip_atomic_load(ctr, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
            __builtin_amdgcn_s_sleep(1);
            if (++spins > (1u << 20)) {
                __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                break;
            }
        }
    }
    __threadfence();
}

template <int P, int W, int R>
__global__ __launch_bounds__(kThreads) void k_panel(PanelArgs g)
{
    __shared__ double s_wred[4][W][P];
    __shared__ double s_head[W][P];
    __shared__ double s_bw[W][P];
    __shared__ double s_sc[2][P];  // rv = 1/v1, mu
    __shared__ int s_flag;

    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const long stride = (long)g.G * kThreads;
    const long gt = (long)blockIdx.x * kThreads + tid;

    V<P> a[R][W];
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const long r = gt + k * stride;
#pragma unroll
        for (int c = 0; c < W; ++c)
            a[k][c] = (r < g.h && c < g.wact) ? ldm<P>(g.A, g.ps, c * g.lda + r) : zero<P>();
    }
    V<P> trow[W];  // row `lane` of T, kept by wave 0 of workgroup 0
#pragma unroll
    for (int c = 0; c < W; ++c) trow[c] = zero<P>();

#pragma unroll
    for (int j = 0; j < W; ++j) {
        if (j >= g.wact) break;
        // ---- 1. one reduction per column: sigma = sum_{i>j} a_ij^2, d_c = sum_{i>j} a_ij a_ic
        //         (c > j) and the Gram entries sum_{i>j} a_ij y_il (l < j) for T.
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const int col = (q == 0) ? j : (q <= j ? q - 1 : q);
            Acc<P> acc = acc_zero<P>();
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const long r = gt + k * stride;
                if (r > j && r < g.h) acc_fma(acc, a[k][j], a[k][col]);
            }
            const V<P> s = wave_sum(acc_get(acc));
            if (lane == 0) lds_st(s_wred[wid][q], s);
        }
        if (blockIdx.x == 0 && tid == j) {
#pragma unroll
            for (int c = 0; c < W; ++c) lds_st(s_head[c], a[0][c]);
        }
        __syncthreads();
        if (wid == 0) {
            // lane q < W holds total q and head-row entry q
            V<P> tot = zero<P>(), hd = zero<P>();
            if (lane < W) {
                tot = lds_ld<P>(s_wred[0][lane]);
#pragma unroll
                for (int w = 1; w < 4; ++w) tot = add(tot, lds_ld<P>(s_wred[w][lane]));
                if (blockIdx.x == 0) hd = lds_ld<P>(s_head[lane]);
            }
            if (g.G > 1) {
                double *slot = g.gpart + (size_t)((j & 1) * g.G + blockIdx.x) * (2 * W * P);
                if (lane < W) {
#pragma unroll
                    for (int k = 0; k < P; ++k) st_coherent(slot + lane * P + k, tot.x[k]);
                    if (blockIdx.x == 0) {
#pragma unroll
                        for (int k = 0; k < P; ++k) st_coherent(slot + (W + lane) * P + k, hd.x[k]);
                    }
                }
                grid_sync(g.gbar, (unsigned)(j + 1) * (unsigned)g.G, g.err);
                if (lane < W) {
                    const double *base = g.gpart + (size_t)((j & 1) * g.G) * (2 * W * P);
                    V<P> t2, h2;
#pragma unroll
                    for (int k = 0; k < P; ++k) {
                        t2.x[k] = ld_coherent(base + lane * P + k);
                        h2.x[k] = ld_coherent(base + (W + lane) * P + k);
                    }
                    for (int b = 1; b < g.G; ++b) {
                        V<P> o;
#pragma unroll
                        for (int k = 0; k < P; ++k) o.x[k] = ld_coherent(base + (size_t)b * (2 * W * P) + lane * P + k);
                        t2 = add(t2, o);
                    }
                    tot = t2;
                    hd = h2;
                }
            }
            // ---- 2. Householder scalars (identical in every lane and every workgroup)
            const V<P> sig = shfl_md(tot, 0);
            const V<P> x1 = shfl_md(hd, j);
            const bool zsig = is_zero(sig);
            V<P> mu = x1, beta = zero<P>(), rv = zero<P>();
            if (!zsig) {
                mu = sqrt_md(fma(sig, x1, x1));  // ||x||_2
                V<P> v1;
                if (x1.x[0] <= 0.0)
                    v1 = sub(x1, mu);
                else
                    v1 = neg(mul(sig, recip(add(x1, mu))));  // -sigma/(x1 + mu), no cancellation
                const V<P> z = recip(mul(mu, v1));
                beta = neg(mul(mul(v1, v1), z));  // 2 v1^2/(sigma + v1^2) = -v1/mu
                rv = mul(mu, z);                  // 1/v1
            }
            // ---- 3. per-column values: lane c > j gets beta * (a_jc + d_c / v1)
            if (lane > j && lane < W) lds_st(s_bw[lane], mul(beta, fma(hd, tot, rv)));
            // T column j: g_l = y_l^T v_j = y_jl + (sum_{i>j} y_il a_ij) / v1 in lane l < j,
            // T(l, j) = -beta_j sum_{k=l}^{j-1} T(l, k) g_k, T(j, j) = beta_j
            const V<P> gs = shfl_md(tot, (lane + 1) & 63);
            V<P> gl = zero<P>();
            if (lane < j) gl = fma(hd, gs, rv);
            Acc<P> tacc = acc_zero<P>();
#pragma unroll
            for (int k = 0; k < j; ++k) {
                const V<P> gk = shfl_md(gl, k);
                if (lane <= k) acc_fma(tacc, trow[k], gk);
            }
            if (lane < j) trow[j] = neg(mul(beta, acc_get(tacc)));
            if (lane == j) trow[j] = beta;
            if (lane == 0) {
                lds_st(s_sc[0], rv);
                lds_st(s_sc[1], mu);
                s_flag = zsig ? 1 : 0;
                if (blockIdx.x == 0) stm(g.beta, g.bps, j, beta);
            }
        }
        __syncthreads();
        // ---- 4. scale v = x / v1, put mu on the diagonal, apply the reflector to columns > j
        if (!s_flag) {
            const V<P> rv = lds_ld<P>(s_sc[0]);
            const V<P> mu = lds_ld<P>(s_sc[1]);
            V<P> nbw[W];
#pragma unroll
            for (int c = 0; c < W; ++c) nbw[c] = (c > j) ? neg(lds_ld<P>(s_bw[c])) : zero<P>();
#pragma unroll
            for (int k = 0; k < R; ++k) {
                const long r = gt + k * stride;
                if (r == j) {
                    a[k][j] = mu;
#pragma unroll
                    for (int c = j + 1; c < W; ++c) a[k][c] = add(a[k][c], nbw[c]);
                } else if (r > j && r < g.h) {
                    const V<P> v = mul(a[k][j], rv);
                    a[k][j] = v;
#pragma unroll
                    for (int c = j + 1; c < W; ++c) a[k][c] = fma(a[k][c], nbw[c], v);
                }
            }
        }
    }
#pragma unroll
    for (int k = 0; k < R; ++k) {
        const long r = gt + k * stride;
        if (r < g.h) {
#pragma unroll
            for (int c = 0; c < W; ++c)
                if (c < g.wact) stm(g.A, g.ps, c * g.lda + r, a[k][c]);
        }
    }
    if (blockIdx.x == 0 && wid == 0 && lane < W) {
#pragma unroll
        for (int c = 0; c < W; ++c) stm(g.T, g.tps, (long)c * W + lane, trow[c]);
    }
}

// ============================================================================ trailing update
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
};

template <int P>
__device__ __forceinline__ V<P> y_entry(const double *Y, long ldy, long psy, long r, int c, int h, int wact)
{
    if (r >= h || c >= wact || r < c) return zero<P>();
    if (r == c) return from_double<P>(1.0);
    return ldm<P>(Y, psy, (long)c * ldy + r);
}

// C := C - Y T^T (Y^T C) over CW columns per workgroup (C's columns, then B's).
template <int P, int W, int CW>
__global__ __launch_bounds__(kThreads) void k_apply(ApplyArgs g)
{
    constexpr int CH = 64;       // rows per staged chunk
    constexpr int CHP = CH + 1;  // padded row stride in LDS
    constexpr int NO = W * CW;   // entries of S = Y^T C
    constexpr int NPART = kThreads / NO;
    static_assert(kThreads % NO == 0, "W*CW must divide the workgroup");
    __shared__ double sY[W * P * CHP];
    __shared__ double sC[CW * P * CHP];
    __shared__ double sR[NPART * NO * P];
    __shared__ double sU[NO * P];

    const int tid = threadIdx.x;
    const int col0 = blockIdx.x * CW;
    double *cbase[CW];
    long cps[CW];
#pragma unroll
    for (int cc = 0; cc < CW; ++cc) {
        const int gc = col0 + cc;
        if (gc < g.nc) {
            cbase[cc] = g.C + (long)gc * g.ldc;
            cps[cc] = g.psc;
        } else if (gc - g.nc < g.nb) {
            cbase[cc] = g.B + (long)(gc - g.nc) * g.ldb;
            cps[cc] = g.psb;
        } else {
            cbase[cc] = nullptr;
            cps[cc] = 0;
        }
    }

    // ---- phase 1: S = Y^T C (lazy accumulation per thread, then a fixed-order tree)
    const int o = tid % NO, part = tid / NO;
    const int oi = o / CW, occ = o % CW;
    Acc<P> acc = acc_zero<P>();
    int nterm = 0;
    for (int r0 = 0; r0 < g.h; r0 += CH) {
        for (int e = tid; e < W * CH; e += kThreads) {
            const int r = e % CH, c = e / CH;
            const V<P> y = y_entry<P>(g.Y, g.ldy, g.psy, (long)r0 + r, c, g.h, g.wact);
#pragma unroll
            for (int k = 0; k < P; ++k) sY[(c * P + k) * CHP + r] = y.x[k];
        }
        for (int e = tid; e < CW * CH; e += kThreads) {
            const int r = e % CH, cc = e / CH;
            const long gr = (long)r0 + r;
            V<P> v = zero<P>();
#pragma unroll
            for (int c2 = 0; c2 < CW; ++c2)
                if (c2 == cc && cbase[c2] && gr < g.h) v = ldm<P>(cbase[c2], cps[c2], gr);
#pragma unroll
            for (int k = 0; k < P; ++k) sC[(cc * P + k) * CHP + r] = v.x[k];
        }
        __syncthreads();
        for (int r = part; r < CH; r += NPART) {
            V<P> y, c;
#pragma unroll
            for (int k = 0; k < P; ++k) {
                y.x[k] = sY[(oi * P + k) * CHP + r];
                c.x[k] = sC[(occ * P + k) * CHP + r];
            }
            acc_fma_step(acc, y, c, nterm++);
        }
        __syncthreads();
    }
    lds_st(&sR[(part * NO + o) * P], acc_get(acc));
    __syncthreads();
    if (tid < NO) {
        V<P> s = lds_ld<P>(&sR[tid * P]);
        for (int p2 = 1; p2 < NPART; ++p2) s = add(s, lds_ld<P>(&sR[(p2 * NO + tid) * P]));
        lds_st(&sR[tid * P], s);
    }
    __syncthreads();
    // ---- phase 2: U = T^T S
    if (tid < NO) {
        const int i = tid / CW, cc = tid % CW;
        Acc<P> u = acc_zero<P>();
        for (int l = 0; l <= i; ++l) acc_fma(u, ldm<P>(g.T, g.tps, (long)i * W + l), lds_ld<P>(&sR[(l * CW + cc) * P]));
        lds_st(&sU[tid * P], acc_get(u));
    }
    __syncthreads();
    // ---- phase 3: C -= Y U
    for (int r0 = 0; r0 < g.h; r0 += CH) {
        for (int e = tid; e < W * CH; e += kThreads) {
            const int r = e % CH, c = e / CH;
            const V<P> y = y_entry<P>(g.Y, g.ldy, g.psy, (long)r0 + r, c, g.h, g.wact);
#pragma unroll
            for (int k = 0; k < P; ++k) sY[(c * P + k) * CHP + r] = y.x[k];
        }
        __syncthreads();
        for (int e = tid; e < CW * CH; e += kThreads) {
            const int r = e % CH, cc = e / CH;
            const long gr = (long)r0 + r;
#pragma unroll
            for (int c2 = 0; c2 < CW; ++c2) {
                if (c2 == cc && cbase[c2] && gr < g.h) {
                    Acc<P> t = acc_from(ldm<P>(cbase[c2], cps[c2], gr));
#pragma unroll
                    for (int i = 0; i < W; ++i) {
                        V<P> y;
#pragma unroll
                        for (int k = 0; k < P; ++k) y.x[k] = -sY[(i * P + k) * CHP + r];
                        acc_fma(t, y, lds_ld<P>(&sU[(i * CW + cc) * P]));
                    }
                    stm(cbase[c2], cps[c2], gr, acc_get(t));
                }
            }
        }
        __syncthreads();
    }
}

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
    V<P> r[RPT];
#pragma unroll
    for (int q = 0; q < RPT; ++q) {
        const int k = rg + q * RG;
        r[q] = (k == j) ? from_double<P>(1.0) : zero<P>();
        if (j < g.tile && k < g.tile && k > j) stm(X, g.psx, (long)j * g.ldx + k, zero<P>());
    }
    __syncthreads();
    for (int i = c1 - 1; i >= 0; --i) {
        const int buf = i & 1;
        // owner of row i in column j publishes x_ij
        if (j < c1 && j >= i && (i % RG) == rg) {
            const int qi = i / RG;
            V<P> xv = zero<P>();
#pragma unroll
            for (int q = 0; q < RPT; ++q)
                if (q == qi) xv = mul(r[q], lds_ld<P>(&sD[i * P]));
            lds_st(&sX[buf][jl * P], xv);
            stm(X, g.psx, (long)j * g.ldx + i, xv);
        }
        __syncthreads();
        if (j < c1 && j >= i) {
            const V<P> xv = lds_ld<P>(&sX[buf][jl * P]);
#pragma unroll
            for (int q = 0; q < RPT; ++q) {
                const int k = rg + q * RG;
                if (k < i) r[q] = fma(r[q], neg(ldm<P>(U, g.psu, (long)i * g.ldu + k)), xv);
            }
        }
    }
}

// x_i := Xinv_i y_i, one wave per output row
template <int P>
__global__ __launch_bounds__(kThreads) void k_bs_xi(const double *Xi, long ldx, long psx, const double *y, long yps,
                                                   double *x, long xps, int tile)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int row = blockIdx.x * 4 + wid;
    if (row >= tile) return;
    Acc<P> acc = acc_zero<P>();
    int nt = 0;
    for (int c = row + lane; c < tile; c += 64) acc_fma_step(acc, ldm<P>(Xi, psx, (long)c * ldx + row), ldm<P>(y, yps, c), nt++);
    const V<P> s = wave_sum(acc_get(acc));
    if (lane == 0) stm(x, xps, row, s);
}

// y(0:rows) -= R(0:rows, cols of tile i) x_i ; 64 rows per workgroup, the tile's columns
// split over the 4 waves and combined in a fixed order
template <int P>
__global__ __launch_bounds__(kThreads) void k_bs_upd(const double *Rc, long ldr, long psr, const double *xi, long xps,
                                                    double *y, long yps, int rows, int tile)
{
    __shared__ double sx[256 * P];
    __shared__ double sp[4][64 * P];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    for (int c = threadIdx.x; c < tile; c += kThreads) lds_st(&sx[c * P], ldm<P>(xi, xps, c));
    __syncthreads();
    const long row = (long)blockIdx.x * 64 + lane;
    const int q = (tile + 3) / 4;
    const int cb = wid * q, ce = min(tile, cb + q);
    Acc<P> acc = acc_zero<P>();
    if (row < rows)
        for (int c = cb; c < ce; ++c) acc_fma_step(acc, ldm<P>(Rc, psr, (long)c * ldr + row), lds_ld<P>(&sx[c * P]), c - cb);
    lds_st(&sp[wid][lane * P], acc_get(acc));
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
                                                long ldb, long bps, int nrhs, double *S, long sps)
{
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
                                                    double *U, int tile, int nrhs)
{
    const int i = blockIdx.x * kThreads + threadIdx.x, c = blockIdx.y;
    if (i >= tile || c >= nrhs) return;
    Acc<P> acc = acc_zero<P>();
    for (int l = 0; l <= i; ++l) acc_fma_step(acc, ldm<P>(T, tps, (long)i * ldt + l), ldm<P>(S, sps, (long)c * tile + l), l);
    stm(U, sps, (long)c * tile + i, acc_get(acc));
}

// B(kt + r, c) -= sum_l Y_k(r, l) U(l, c)
template <int P>
__global__ __launch_bounds__(kThreads) void k_nn_sub(const double *Y, long lda, long ps, int h, int tile, const double *U,
                                                    long ups, double *B, long ldb, long bps)
{
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

#define MDLS_LAUNCH(NAME, PREC, WORK, KERNEL, GRID, BLOCK, STREAM, ...)                       \
    do {                                                                                     \
        void *ev_ = nullptr;                                                                 \
        const bool tm_ = timing_on();                                                        \
        if (tm_) timing_begin((STREAM), &ev_);                                               \
        hipLaunchKernelGGL(KERNEL, GRID, BLOCK, 0, STREAM, __VA_ARGS__);                     \
        if (tm_) timing_end((STREAM), ev_, (NAME), (PREC), (double)(WORK));                  \
    } while (0)

// ============================================================================ host side
constexpr int kGMax = 256;  // most workgroups one panel launch may use

template <int P>
struct Cfg;
template <>
struct Cfg<1> {
    static constexpr int W = 8, CW = 4, NCI = 16;
};
template <>
struct Cfg<2> {
    static constexpr int W = 8, CW = 4, NCI = 16;
};
template <>
struct Cfg<4> {
    static constexpr int W = 4, CW = 4, NCI = 16;
};
template <>
struct Cfg<8> {
    static constexpr int W = 4, CW = 4, NCI = 8;
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

// rows per thread of the panel kernel (1, 2 or 4); MDLS_PANEL_R overrides the default
inline int panel_rows_per_thread(int P)
{
    const char *e = getenv("MDLS_PANEL_R");
    if (e) {
        const int r = atoi(e);
        if (r == 1 || r == 2 || (r == 4 && P <= 4)) return r;
    }
    return (P <= 2) ? 4 : 1;
}

inline size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

struct Layout {
    size_t beta, leafT, gpart, ctr, err, yw, big, total;
    int W, nleaves;
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
    L.gpart = take(sizeof(double) * 2 * kGMax * 2 * L.W * P);
    L.ctr = take(sizeof(unsigned) * (size_t)(L.nleaves + 1));
    L.err = take(sizeof(int) * 4);
    L.yw = take(sizeof(double) * (size_t)P * (m > n ? m : n));
    // back substitution inverses / Gram blocks (P x tile x n) or Q^T B scratch (2 x P x tile x 64)
    const size_t big1 = sizeof(double) * (size_t)P * tile * n;
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
    double *beta() const { return (double *)(ws + L.beta); }
    double *leafT() const { return (double *)(ws + L.leafT); }
    double *gpart() const { return (double *)(ws + L.gpart); }
    unsigned *ctr() const { return (unsigned *)(ws + L.ctr); }
    int *err() const { return (int *)(ws + L.err); }
    double *yw() const { return (double *)(ws + L.yw); }
    double *big() const { return (double *)(ws + L.big); }
};

template <int P, int W, int R>
void launch_panel(const PanelArgs &a, hipStream_t s)
{
    double work = 0;
    for (int j = 0; j < a.wact; ++j) work += (a.h - j - 1) + 2.0 * (a.wact - j - 1) * (a.h - j);
    MDLS_LAUNCH("k_panel", P, work, (k_panel<P, W, R>), dim3(a.G), dim3(kThreads), s, a);
}

// Householder QR of A (m x n) in narrow panels; B (nb columns, may be null) receives Q^T B.
template <int P>
void qr_panels(const Ctx<P> &cx, int m, int n, double *A, long lda, long psa, double *B, long ldb, long psb, int nb)
{
    constexpr int W = Cfg<P>::W, CW = Cfg<P>::CW;
    const int R = panel_rows_per_thread(P);
    const int nleaves = cx.L.nleaves;
    MDLS_LAUNCH("k_zero", P, 0, k_zero_u32, dim3((nleaves + 1 + 255) / 256), dim3(256), cx.s, cx.ctr(), nleaves + 1);
    MDLS_LAUNCH("k_zero", P, 0, k_zero_u32, dim3(1), dim3(256), cx.s, (unsigned *)cx.err(), 4);
    const long tps = (long)W * W * nleaves;
    for (int l = 0; l < nleaves; ++l) {
        const int c0 = l * W;
        const int wact = (n - c0 < W) ? (n - c0) : W;
        const int h = m - c0;
        PanelArgs pa;
        pa.A = A + (long)c0 * lda + c0;
        pa.lda = lda;
        pa.ps = psa;
        pa.h = h;
        pa.wact = wact;
        pa.beta = cx.beta() + c0;
        pa.bps = n;
        pa.T = cx.leafT() + (long)l * W * W;
        pa.tps = tps;
        pa.gpart = cx.gpart();
        pa.gbar = cx.ctr() + l;
        pa.err = cx.err();
        int G = (h + kThreads * R - 1) / (kThreads * R);
        if (G < 1) G = 1;
        pa.G = G;
        if (R == 1)
            launch_panel<P, W, 1>(pa, cx.s);
        else if (R == 2)
            launch_panel<P, W, 2>(pa, cx.s);
        else {
            if constexpr (P <= 4) launch_panel<P, W, 4>(pa, cx.s);
        }
        const int nc = n - c0 - wact;
        const int ntot = nc + (B ? nb : 0);
        if (ntot > 0) {
            ApplyArgs aa;
            aa.Y = pa.A;
            aa.ldy = lda;
            aa.psy = psa;
            aa.h = h;
            aa.wact = wact;
            aa.T = pa.T;
            aa.tps = tps;
            aa.C = A + (long)(c0 + wact) * lda + c0;
            aa.ldc = lda;
            aa.psc = psa;
            aa.nc = nc;
            aa.B = B ? B + c0 : nullptr;
            aa.ldb = ldb;
            aa.psb = psb;
            aa.nb = B ? nb : 0;
            MDLS_LAUNCH("k_apply", P, 2.0 * h * wact * ntot, (k_apply<P, W, CW>), dim3((ntot + CW - 1) / CW), dim3(kThreads),
                        cx.s, aa);
        }
    }
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

// tiled back substitution on y (P planes of n, in ws.yw); x receives the solution
template <int P>
void backsub_tiles(const Ctx<P> &cx, int n, int tile, const double *R, long ldr, long psr, double *x, long xps,
                   int *d_info)
{
    const int N = n / tile;
    MDLS_LAUNCH("k_diag_check", P, 0, k_diag_check, dim3(1), dim3(kThreads), cx.s, R, ldr, psr, n, P, d_info);
    double *Xinv = cx.big();
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
    invert_tiles<P>(cx, ia, N);
    double *y = cx.yw();
    const long yps = n;
    for (int i = N - 1; i >= 0; --i) {
        const long it = (long)i * tile;
        MDLS_LAUNCH("k_bs_xi", P, 0.5 * tile * tile, (k_bs_xi<P>), dim3((tile + 3) / 4), dim3(kThreads), cx.s,
                    Xinv + (long)i * tile * tile,
                           (long)tile, xips, y + it, yps, x + it, xps, tile);
        if (i > 0) {
            const int rows = i * tile;
            MDLS_LAUNCH("k_bs_upd", P, (double)rows * tile, (k_bs_upd<P>), dim3((rows + 63) / 64), dim3(kThreads), cx.s,
                        R + it * ldr, ldr, psr,
                               x + it, xps, y, yps, rows, tile);
        }
    }
}

template <int P>
int solve_t(int m, int n, int tile, double *A, int lda, double *b, double *x, void *ws, int *d_info, hipStream_t s)
{
    Ctx<P> cx{(char *)ws, layout(P, m, n, tile), s};
    const long psa = (long)lda * n;
    qr_panels<P>(cx, m, n, A, lda, psa, b, m, m, 1);
    MDLS_LAUNCH("k_copy", P, 0, k_copy, dim3((n + 255) / 256), dim3(256), s, b, (long)m, cx.yw(), (long)n, n, P);
    backsub_tiles<P>(cx, n, tile, A, lda, psa, x, n, d_info);
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

template <int P>
int qr_t(int m, int n, int tile, double *A, int lda, double *T, int ldt, void *ws, hipStream_t s)
{
    Ctx<P> cx{(char *)ws, layout(P, m, n, tile), s};
    const long psa = (long)lda * n;
    qr_panels<P>(cx, m, n, A, lda, psa, nullptr, 0, 0, 0);
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
int apply_qt_t(int m, int n, int tile, const double *A, int lda, const double *T, int ldt, double *B, int ldb, int nrhs,
               void *ws, hipStream_t s)
{
    Ctx<P> cx{(char *)ws, layout(P, m, n, tile), s};
    const long psa = (long)lda * n, tps = (long)ldt * n, bps = (long)ldb * nrhs;
    double *S = cx.big();
    double *U = S + (size_t)P * tile * 64;
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
                        (long)lda, psa, h, tile,
                               Bc + kt, (long)ldb, bps, nc, S, sps);
            MDLS_LAUNCH("k_trmm_t", P, 0.5 * tile * tile * nc, (k_trmm_t<P>), dim3((tile + kThreads - 1) / kThreads, nc),
                        dim3(kThreads), s,
                               T + kt * ldt, (long)ldt, tps, S, sps, U, tile, nc);
            MDLS_LAUNCH("k_nn_sub", P, (double)h * tile * nc, (k_nn_sub<P>), dim3((h + kThreads - 1) / kThreads, nc),
                        dim3(kThreads), s, Y,
                               (long)lda, psa, h, tile, U, sps, Bc + kt, (long)ldb, bps);
        }
    }
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
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

#define MDLS_FOR_PRECISION(X, P)                                                                        \
    X template int solve_t<P>(int, int, int, double *, int, double *, double *, void *, int *, hipStream_t);     \
    X template int qr_t<P>(int, int, int, double *, int, double *, int, void *, hipStream_t);                 \
    X template int apply_qt_t<P>(int, int, int, const double *, int, const double *, int, double *, int, int,   \
                                 void *, hipStream_t);                                                         \
    X template int form_w_t<P>(int, int, int, const double *, int, const double *, int, double *, int,         \
                               hipStream_t);                                                                   \
    X template int backsub_t<P>(int, int, const double *, int, double *, void *, int *, hipStream_t);

}  // namespace mdls_impl
