// md_host_shim.cpp -- host build of the GPU library's multiple-double header, so that the
// exact same arithmetic the kernels run can be checked on the CPU.  Test aid only: the GPU
// library does not link it.
#include <cstring>

#include "md.hpp"

namespace {
template <int P>
mdk::V<P> ld(const double *p)
{
    mdk::V<P> v;
    for (int k = 0; k < P; ++k) v.x[k] = p[k];
    return v;
}
template <int P>
void st(double *p, const mdk::V<P> &v)
{
    for (int k = 0; k < P; ++k) p[k] = v.x[k];
}

template <int P>
int run(int op, const double *a, const double *b, const double *c, double *r)
{
    using namespace mdk;
    V<P> A = ld<P>(a), B = ld<P>(b), C = ld<P>(c);
    switch (op) {
    case 0: st(r, add(A, B)); break;
    case 1: st(r, sub(A, B)); break;
    case 2: st(r, mul(A, B)); break;
    case 3: st(r, div(A, B)); break;
    case 4: st(r, sqrt_md(A)); break;
    case 5: st(r, fma(C, A, B)); break;
    case 6: st(r, recip(B)); break;
    case 7: st(r, mul_d(A, b[0])); break;
    default: return -1;
    }
    return 0;
}

// dot product c + sum_i a_i b_i accumulated the way the kernels do it
template <int P>
void dot(int n, const double *a, const double *b, const double *c, double *r)
{
    using namespace mdk;
    Acc<P> acc = acc_from(ld<P>(c));
    for (int i = 0; i < n; ++i) acc_fma_step(acc, ld<P>(a + (long)i * P), ld<P>(b + (long)i * P), i);
    st(r, acc_get(acc));
}
}  // namespace

extern "C" int mdh_op(int P, int op, const double *a, const double *b, const double *c, double *r)
{
    switch (P) {
    case 1: return run<1>(op, a, b, c, r);
    case 2: return run<2>(op, a, b, c, r);
    case 4: return run<4>(op, a, b, c, r);
    case 8: return run<8>(op, a, b, c, r);
    }
    return -1;
}

// a, b: n md values, limbs contiguous per value
extern "C" int mdh_dot(int P, int n, const double *a, const double *b, const double *c, double *r)
{
    switch (P) {
    case 1: dot<1>(n, a, b, c, r); return 0;
    case 2: dot<2>(n, a, b, c, r); return 0;
    case 4: dot<4>(n, a, b, c, r); return 0;
    case 8: dot<8>(n, a, b, c, r); return 0;
    }
    return -1;
}
