// mdls_split.hpp -- the double-double trailing-update product S = Y^T C on the FP64 matrix
// cores (gfx950 v_mfma_f64_16x16x4f64) by exact slicing, beside the same product on the FP64
// vector units.  This is the split-limb form of the update products named for the precision
// form of the method (the paper's note that its GEMM-shaped stages suit GPU acceleration,
// Section 3); the slicing follows Ozaki, Ogita, Oishi and Rump, "Error-free transformations
// of matrix multiplication by using fast routines of matrix multiplication and its
// applications", Numer. Algorithms 59 (2012).
//
// Each column of Y and of C is scaled by a power of two so that its entries lie below 1 in
// magnitude, and every double-double entry x is cut into kSlices doubles d_0 + d_1 + ... with
// d_p a multiple of 2^-(kSliceBits (p+1)) and |d_p| <= 2^-(kSliceBits p): at most
// kSliceBits + 1 significant bits each (the remainder after each cut is exact in double
// double).  A slice product d_p(Y) d_q(C) then has at most 2 kSliceBits + 1 bits on the grid
// 2^-(kSliceBits (p+q+2)), and the sum of all products of one level L = p + q over at most
// kSlices pairs and 1024 rows stays below 2^53 units of that grid, so every MFMA accumulation
// is exact.  Levels L < kSlices are kept (the dropped ones are below 2^-113 of the largest
// product), the split-K partial level sums are added exactly, and the kSlices level sums,
// largest first, are renormalised to a double double and scaled back.
#pragma once
#include "mdls_impl.hpp"

namespace mdls_impl {

constexpr int kSliceBits = 18;
constexpr int kSlices = 7;
constexpr int kSplitMaxRows = 1024;  // the exactness bound above
constexpr int kSplitK = 4;           // workgroups per output tile (split over rows)
constexpr int kSplitWaves = 4;       // waves per workgroup (split over rows again)

typedef double d4_t __attribute__((ext_vector_type(4)));

// x = hi + lo with |x| < 1 -> d[0..kSlices-1], each a multiple of 2^-(kSliceBits (p+1))
__device__ __forceinline__ void dd_slices(double hi, double lo, double (&d)[kSlices])
{
#pragma unroll
    for (int p = 0; p < kSlices; ++p) {
        // 1.5 * 2^(52 - kSliceBits (p+1)): adding and subtracting it rounds to its ulp
        const double sig = 1.5 * __builtin_ldexp(1.0, 52 - kSliceBits * (p + 1));
        const double t = (hi + sig) - sig;
        d[p] = t;
        const double r = hi - t;  // exact: t is hi on a coarser grid
        two_sum(r, lo, hi, lo);   // the remainder, renormalised exactly
    }
}

// exponent E with |x| < 2^E for the largest leading limb of a column (0 for a zero column)
__device__ __forceinline__ int col_exp(double v)
{
    int e = 0;
    if (v != 0.0) (void)__builtin_frexp(v, &e);
    return e;
}

struct SplitArgs {
    const double *Y;  // h x w, 2 planes of ldy * w
    long ldy, ysp;
    const double *C;  // h x c, 2 planes of ldc * c
    long ldc, csp;
    double *part;     // [tile][kSplitK][kSlices][256] exact partial level sums
    int *exps;        // column exponents: w of Y, then c of C
    int h, w, c;
};

// exps[col] = E with |x| < 2^E for every entry of the column (Y's w columns, then C's c);
// one wave per column
__global__ __launch_bounds__(kThreads) void k_split_exp(SplitArgs g)
{
    const int lane = threadIdx.x & 63, col = blockIdx.x * (kThreads / 64) + (threadIdx.x >> 6);
    if (col >= g.w + g.c) return;
    const double *x = col < g.w ? g.Y + (long)col * g.ldy : g.C + (long)(col - g.w) * g.ldc;
    double m = 0.0;
    for (int k = lane; k < g.h; k += 64) m = fmax(m, fabs(x[k]));
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) m = fmax(m, __shfl_xor(m, o, 64));
    if (lane == 0) g.exps[col] = col_exp(m);
}

// Workgroup (tile t, split s): columns t*16.. of C, rows of its share; wave v of the workgroup
// takes every kSplitWaves-th 4-row step of that share.  A lane holds Y(k, l = lane % 16) and
// C(k, c0 + lane % 16) with k = k0 + lane / 16 (the operand layout of the 16x16x4 f64 MFMA).
__global__ __launch_bounds__(64 * kSplitWaves) void k_split_tn(SplitArgs g)
{
    __shared__ double sacc[kSplitWaves / 2][kSlices][256];
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int tile = blockIdx.x, split = blockIdx.y;
    const int c0 = tile * 16;
    const int r16 = lane & 15, kq = lane >> 4;
    const bool yok = r16 < g.w, cok = c0 + r16 < g.c;
    const double sy = __builtin_ldexp(1.0, yok ? -g.exps[r16] : 0);
    const double sc = __builtin_ldexp(1.0, cok ? -g.exps[g.w + c0 + r16] : 0);
    d4_t acc[kSlices];
#pragma unroll
    for (int l = 0; l < kSlices; ++l) acc[l] = d4_t{0.0, 0.0, 0.0, 0.0};
    const int steps = (g.h + 3) / 4;                   // 4-row steps in all
    const int per = (steps + kSplitK - 1) / kSplitK;   // steps of this workgroup
    const int s_lo = split * per, s_hi = min(steps, s_lo + per);
    for (int st = s_lo + wid; st < s_hi; st += kSplitWaves) {
        const int k = st * 4 + kq;
        double yh = 0.0, yl = 0.0, ch = 0.0, cl = 0.0;
        if (k < g.h) {
            if (yok) {
                yh = g.Y[(long)r16 * g.ldy + k] * sy;
                yl = g.Y[g.ysp + (long)r16 * g.ldy + k] * sy;
            }
            if (cok) {
                ch = g.C[(long)(c0 + r16) * g.ldc + k] * sc;
                cl = g.C[g.csp + (long)(c0 + r16) * g.ldc + k] * sc;
            }
        }
        double a[kSlices], b[kSlices];
        dd_slices(yh, yl, a);
        dd_slices(ch, cl, b);
#pragma unroll
        for (int p = 0; p < kSlices; ++p)
#pragma unroll
            for (int q = 0; p + q < kSlices; ++q)
                acc[p + q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc[p + q], 0, 0, 0);
    }
    // combine the waves' partial level sums (exact) in LDS, halving each round
    for (int half = kSplitWaves / 2; half >= 1; half >>= 1) {
        if (wid >= half && wid < 2 * half) {
#pragma unroll
            for (int l = 0; l < kSlices; ++l)
#pragma unroll
                for (int v = 0; v < 4; ++v) sacc[wid - half][l][v * 64 + lane] = acc[l][v];
        }
        __syncthreads();
        if (wid < half) {
#pragma unroll
            for (int l = 0; l < kSlices; ++l)
#pragma unroll
                for (int v = 0; v < 4; ++v) acc[l][v] += sacc[wid][l][v * 64 + lane];
        }
        __syncthreads();
    }
    if (wid == 0) {
        double *out = g.part + ((long)tile * kSplitK + split) * kSlices * 256;
#pragma unroll
        for (int l = 0; l < kSlices; ++l)
#pragma unroll
            for (int v = 0; v < 4; ++v) out[l * 256 + v * 64 + lane] = acc[l][v];
    }
}

// S(i, c0 + j) = 2^(ey_i + ec_j) * renorm(sum over splits of the level sums); one thread per
// output of a tile.  The result layout of the 16x16x4 f64 MFMA: register r of lane L holds
// D(4 r + L / 16, L % 16), i.e. D(i, j) is lane j + 16 (i % 4), item i / 4.
__global__ __launch_bounds__(256) void k_split_fin(SplitArgs g, double *S, long lds, long ssp)
{
    const int tile = blockIdx.x, t = threadIdx.x;
    const int i = t >> 4, j = t & 15;  // output row (Y column) and column within the tile
    const int c0 = tile * 16;
    const int lane = j + 16 * (i & 3), item = i >> 2;
    double lev[kSlices];
#pragma unroll
    for (int l = 0; l < kSlices; ++l) {
        double s = 0.0;
        for (int sp = 0; sp < kSplitK; ++sp)
            s += g.part[((long)tile * kSplitK + sp) * kSlices * 256 + l * 256 + item * 64 + lane];
        lev[l] = s;  // exact: every partial and sum fits the level's 53-bit budget
    }
    if (i >= g.w || c0 + j >= g.c) return;
    const V<2> r = renorm<kSlices, 2>(lev);
    const double sc = __builtin_ldexp(1.0, g.exps[i] + g.exps[g.w + c0 + j]);
    S[(long)(c0 + j) * lds + i] = r.x[0] * sc;
    S[ssp + (long)(c0 + j) * lds + i] = r.x[1] * sc;
}

// The same product on the vector units: one wave per output, lanes over the rows, lazy md
// accumulation, a fixed butterfly
__global__ __launch_bounds__(kThreads) void k_dense_tn2(const double *Y, long ldy, long ysp, const double *C, long ldc,
                                                       long csp, double *S, long lds, long ssp, int h, int w, int c)
{
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int l = blockIdx.x * (kThreads / 64) + wid, cc = blockIdx.y;
    if (l >= w || cc >= c) return;
    Acc<2> acc = acc_zero<2>();
    int nt = 0;
    for (int k = lane; k < h; k += 64)
        acc_fma_step(acc, ldm<2>(Y, ysp, (long)l * ldy + k), ldm<2>(C, csp, (long)cc * ldc + k), nt++);
    const V<2> s = wave_sum(acc_get(acc));
    if (lane == 0) stm(S, ssp, (long)cc * lds + l, s);
}

inline size_t split_workspace_bytes(int w, int c)
{
    return align256(sizeof(double) * (size_t)((c + 15) / 16) * kSplitK * kSlices * 256) + sizeof(int) * (size_t)(w + c);
}

// S (2 planes of lds x c) = Y^T C; method 0: vector units, 1: matrix cores by exact slicing
inline int dd_gemm_tn(int method, int h, int w, int c, const double *Y, int ldy, const double *C, int ldc, double *S,
                      int lds, void *ws, hipStream_t s)
{
    const long ysp = (long)ldy * w, csp = (long)ldc * c, ssp = (long)lds * c;
    if (method == 0) {
        MDLS_LAUNCH("k_dense_tn2", 2, (double)h * w * c, k_dense_tn2, dim3((w + 3) / 4, c), dim3(kThreads), s, Y,
                    (long)ldy, ysp, C, (long)ldc, csp, S, (long)lds, ssp, h, w, c);
    } else {
        const int tiles = (c + 15) / 16;
        double *part = (double *)ws;
        int *exps = (int *)((char *)ws + align256(sizeof(double) * (size_t)tiles * kSplitK * kSlices * 256));
        SplitArgs a{Y, (long)ldy, ysp, C, (long)ldc, csp, part, exps, h, w, c};
        MDLS_LAUNCH("k_split_exp", 2, 0, k_split_exp, dim3((w + c + 3) / 4), dim3(kThreads), s, a);
        MDLS_LAUNCH("k_split_tn", 2, (double)h * w * c, k_split_tn, dim3(tiles, kSplitK), dim3(64 * kSplitWaves), s, a);
        MDLS_LAUNCH("k_split_fin", 2, 0, k_split_fin, dim3(tiles), dim3(256), s, a, S, (long)lds, ssp);
    }
    return hipGetLastError() == hipSuccess ? 0 : MDLS_EHIP;
}

}  // namespace mdls_impl
