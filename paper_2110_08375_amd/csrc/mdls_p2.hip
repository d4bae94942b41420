// mdls_p2.hip -- kernels and drivers instantiated for 2-limb numbers.
#include "mdls_cplx.hpp"

namespace mdls_impl {
MDLS_FOR_PRECISION(, 2)
MDLS_BATCH_FOR_PRECISION(, 2)
MDLS_CPLX_FOR_PRECISION(, 2)
}  // namespace mdls_impl
