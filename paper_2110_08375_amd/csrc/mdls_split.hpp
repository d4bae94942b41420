// mdls_split.hpp -- the double-double trailing-update product S = Y^T C on the FP64 matrix
// cores (gfx950 v_mfma_f64_16x16x4f64) by exact slicing, beside the same product on the FP64
// vector units.  This is the split-limb form of the update products named for the precision
// form of the method (the paper's note that its GEMM-shaped stages suit GPU acceleration,
// Section 3); the slicing follows Ozaki, Ogita, Oishi and Rump, "Error-free transformations
// of matrix multiplication by using fast routines of matrix multiplication and its
// applications", Numer. Algorithms 59 (2012).
//
// The exact split-limb product itself (slicing, the MFMA kernel, the renormalisation) is in
// mdls_split_kernels.hpp; this file adds the same product on the vector units and the C ABI's
// standalone entry.
#pragma once
#include "mdls_impl.hpp"

namespace mdls_impl {

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
