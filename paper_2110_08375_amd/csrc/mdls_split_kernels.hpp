// mdls_split_kernels.hpp -- the exact split-limb double-double product S = Y^T C on the FP64
// matrix cores (gfx950 v_mfma_f64_16x16x4f64), shared by the C ABI's standalone product and the
// double-double factorisation of the refined solve (its trailing-update products).
// Each column of Y and of C is scaled by a power of two so that its entries lie below 1 in
// magnitude, and every double-double entry x is cut into kSlices doubles d_0 + d_1 + ... with
// d_p a multiple of 2^-(kSliceBits (p+1)) and |d_p| <= 2^-(kSliceBits p): at most
// kSliceBits + 1 significant bits each (the remainder after each cut is exact in double
// double).  A slice product d_p(Y) d_q(C) then has at most 2 kSliceBits + 2 bits on the grid
// 2^-(kSliceBits (p+q+2)), and the sum of all products of one level L = p + q over at most
// kSlices pairs and 2048 rows stays below 7 * 2048 * 2^38 < 2^53 units of that grid, so every
// MFMA accumulation is exact.  Levels L < kSlices are kept (the dropped ones are below 2^-113 of the largest
// product), the split-K partial level sums are added exactly, and the kSlices level sums,
// largest first, are renormalised to a double double and scaled back.
#pragma once
#include "mdls_kernels.hpp"

namespace mdls_impl {
using namespace mdk;

constexpr int kSliceBits = 18;
constexpr int kSlices = 7;
constexpr int kSplitMaxRows = 2048;  // the exactness bound above
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
namespace {
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

// Workgroup (tile t, split s): columns t*16.. of C and the w <= 16 columns of Y, over the rows of
// its share in chunks of 64.  Each chunk of Y and C (hi and lo limbs, scaled by the column powers
// of two) is staged in LDS row-major (16 columns per row), loaded with consecutive lanes on
// consecutive rows of a column (unit stride in HBM); the next chunk's loads are issued before the
// current chunk's products.  Wave v takes every kSplitWaves-th 4-row step of the chunk; lane
// (r16, kq) = (lane % 16, lane / 16) reads Y(k, r16) and C(k, c0 + r16) with k = 4 step + kq (the
// operand layout of the 16x16x4 f64 MFMA; consecutive lanes read consecutive doubles of LDS).
constexpr int kSplitChunk = 64;

__global__ __launch_bounds__(64 * kSplitWaves) void k_split_tn(SplitArgs g)
{
    constexpr int CH = kSplitChunk, NT = 64 * kSplitWaves;
    constexpr int PER = 16 * CH / NT;  // elements of one operand limb a thread stages per chunk
    __shared__ double sacc[kSplitWaves / 2][kSlices][256];
    __shared__ double sO[4][CH * 16];  // Y hi, Y lo, C hi, C lo: [row][column]
    const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
    const int tile = blockIdx.x, split = blockIdx.y;
    const int c0 = tile * 16;
    const int r16 = lane & 15, kq = lane >> 4;
    d4_t acc[kSlices];
#pragma unroll
    for (int l = 0; l < kSlices; ++l) acc[l] = d4_t{0.0, 0.0, 0.0, 0.0};
    const int chunks = (g.h + CH - 1) / CH;
    const int per = (chunks + kSplitK - 1) / kSplitK;
    const int ch_lo = split * per, ch_hi = min(chunks, ch_lo + per);
    // staged element e = tid + u NT of a chunk: column e / CH, row e % CH
    double ld[4][PER];
    auto fetch = [&](int ch) __attribute__((always_inline)) {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT, col = e / CH, k = ch * CH + e % CH;
            const bool yok = col < g.w && k < g.h, cok = c0 + col < g.c && k < g.h;
            ld[0][u] = yok ? g.Y[(long)col * g.ldy + k] : 0.0;
            ld[1][u] = yok ? g.Y[g.ysp + (long)col * g.ldy + k] : 0.0;
            ld[2][u] = cok ? g.C[(long)(c0 + col) * g.ldc + k] : 0.0;
            ld[3][u] = cok ? g.C[g.csp + (long)(c0 + col) * g.ldc + k] : 0.0;
        }
    };
    if (ch_lo < ch_hi) fetch(ch_lo);
    for (int ch = ch_lo; ch < ch_hi; ++ch) {
        __syncthreads();  // the previous chunk's operands are no longer read
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int e = tid + u * NT, col = e / CH, row = e % CH;
            const double sy = __builtin_ldexp(1.0, col < g.w ? -g.exps[col] : 0);
            const double sc = __builtin_ldexp(1.0, c0 + col < g.c ? -g.exps[g.w + c0 + col] : 0);
            sO[0][row * 16 + col] = ld[0][u] * sy;
            sO[1][row * 16 + col] = ld[1][u] * sy;
            sO[2][row * 16 + col] = ld[2][u] * sc;
            sO[3][row * 16 + col] = ld[3][u] * sc;
        }
        __syncthreads();
        if (ch + 1 < ch_hi) fetch(ch + 1);  // in flight during this chunk's products
        for (int st = wid; st < CH / 4; st += kSplitWaves) {
            const int o = (st * 4 + kq) * 16 + r16;
            double a[kSlices], b[kSlices];
            dd_slices(sO[0][o], sO[1][o], a);
            dd_slices(sO[2][o], sO[3][o], b);
#pragma unroll
            for (int p = 0; p < kSlices; ++p)
#pragma unroll
                for (int q = 0; p + q < kSlices; ++q)
                    acc[p + q] = __builtin_amdgcn_mfma_f64_16x16x4f64(a[p], b[q], acc[p + q], 0, 0, 0);
        }
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

// Y (h x w, dense, 2 planes of h x w) := the panel's Householder block, unit lower trapezoidal
// (the implicit unit diagonal written out, zeros above it and in the columns past wact)
__global__ __launch_bounds__(kThreads) void k_stage_y(const double *A, long lda, long psa, int h, int wact, int w,
                                                     double *Y)
{
    const long e = (long)blockIdx.x * kThreads + threadIdx.x;
    if (e >= (long)h * w) return;
    const int r = (int)(e % h), c = (int)(e / h);
    double v0 = 0.0, v1 = 0.0;
    if (c < wact && r >= c) {
        if (r == c) {
            v0 = 1.0;
        } else {
            v0 = A[(long)c * lda + r];
            v1 = A[psa + (long)c * lda + r];
        }
    }
    Y[e] = v0;
    Y[(long)h * w + e] = v1;
}

// The double-double level sums of k_split_tn renormalised and scaled back, written as the one
// partial sum per column that the trailing update's combine step reads: part[(col * w + i) * 2 + k]
// for the launch's columns col (k_apply_t with one row block).
__global__ __launch_bounds__(256) void k_split_fin_part(SplitArgs g, double *part)
{
    const int tile = blockIdx.x, t = threadIdx.x;
    const int i = t >> 4, j = t & 15;
    const int c0 = tile * 16;
    const int lane = j + 16 * (i & 3), item = i >> 2;
    double lev[kSlices];
#pragma unroll
    for (int l = 0; l < kSlices; ++l) {
        double s = 0.0;
        for (int sp = 0; sp < kSplitK; ++sp)
            s += g.part[((long)tile * kSplitK + sp) * kSlices * 256 + l * 256 + item * 64 + lane];
        lev[l] = s;
    }
    if (i >= g.w || c0 + j >= g.c) return;
    const V<2> r = renorm<kSlices, 2>(lev);
    const double sc = __builtin_ldexp(1.0, g.exps[i] + g.exps[g.w + c0 + j]);
    double *dst = part + ((long)(c0 + j) * g.w + i) * 2;
    dst[0] = r.x[0] * sc;
    dst[1] = r.x[1] * sc;
}
}  // namespace

// bytes of the exact-product scratch for products of w <= 16 columns of Y and c columns of C
inline size_t split_workspace_bytes(int w, int c)
{
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    return al(sizeof(double) * (size_t)((c + 15) / 16) * kSplitK * kSlices * 256) + sizeof(int) * (size_t)(w + c);
}

}  // namespace mdls_impl
