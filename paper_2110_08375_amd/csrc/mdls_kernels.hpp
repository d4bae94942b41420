// mdls_kernels.hpp -- gfx950 kernels of the multiple-double least-squares hot path.
//
// Storage: a matrix is P limb planes (limb 0 most significant), each column-major with a
// leading dimension ld; plane k starts ps doubles after plane k-1 (paper, end of
// Section 2).  Consecutive lanes always walk consecutive rows of one column, so every
// limb plane is read and written with unit stride.
#pragma once

#include "md.hpp"

namespace mdk {

constexpr int kThreads = 256;  // threads per workgroup for every kernel below

template <int P>
__device__ __forceinline__ V<P> ldm(const double *X, long ps, long off)
{
    V<P> v;
#pragma unroll
    for (int k = 0; k < P; ++k) v.x[k] = X[k * ps + off];
    return v;
}

template <int P>
__device__ __forceinline__ void stm(double *X, long ps, long off, const V<P> &v)
{
#pragma unroll
    for (int k = 0; k < P; ++k) X[k * ps + off] = v.x[k];
}

// shared-memory md value stored as [P] doubles
template <int P>
__device__ __forceinline__ V<P> lds_ld(const double *s)
{
    V<P> v;
#pragma unroll
    for (int k = 0; k < P; ++k) v.x[k] = s[k];
    return v;
}

template <int P>
__device__ __forceinline__ void lds_st(double *s, const V<P> &v)
{
#pragma unroll
    for (int k = 0; k < P; ++k) s[k] = v.x[k];
}

template <int P>
__device__ __forceinline__ V<P> shfl_xor_md(const V<P> &v, int mask)
{
    V<P> o;
#pragma unroll
    for (int k = 0; k < P; ++k) o.x[k] = __shfl_xor(v.x[k], mask, 64);
    return o;
}

template <int P>
__device__ __forceinline__ V<P> shfl_md(const V<P> &v, int src)
{
    V<P> o;
#pragma unroll
    for (int k = 0; k < P; ++k) o.x[k] = __shfl(v.x[k], src, 64);
    return o;
}

template <int P>
__device__ __forceinline__ Acc<P> shfl_xor_acc(const Acc<P> &v, int mask)
{
    Acc<P> o;
#pragma unroll
    for (int k = 0; k < P; ++k) o.s[k] = __shfl_xor(v.s[k], mask, 64);
    return o;
}

// a += b for two lazy accumulators (b's level sums enter as limbs); symmetric in a and b
template <int P>
__device__ __forceinline__ void acc_add_acc(Acc<P> &a, const Acc<P> &b)
{
    V<P> bv;
#pragma unroll
    for (int k = 0; k < P; ++k) bv.x[k] = b.s[k];
    acc_add(a, bv);
}

// Butterfly sum over the 64 lanes of a wave.  md add is symmetric in its operands, so
// every lane ends with the same bits.
template <int P>
__device__ __forceinline__ V<P> wave_sum(V<P> v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v = add(v, shfl_xor_md(v, m));
    return v;
}

// Coherent (agent-scope) scalar accesses for data exchanged between workgroups inside one
// launch: they bypass the non-coherent caches of the other XCDs.
__device__ __forceinline__ void st_coherent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double ld_coherent(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

}  // namespace mdk
