// mdls_p1.hip -- kernels and drivers instantiated for 1-limb numbers.
#include "mdls_cplx.hpp"

namespace mdls_impl {
MDLS_FOR_PRECISION(, 1)
MDLS_CPLX_FOR_PRECISION(, 1)
}  // namespace mdls_impl
