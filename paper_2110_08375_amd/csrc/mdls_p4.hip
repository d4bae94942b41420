// mdls_p4.hip -- kernels and drivers instantiated for 4-limb numbers.
#include "mdls_cplx.hpp"

namespace mdls_impl {
MDLS_FOR_PRECISION(extern, 2)  // the refined solve factors in double double (mdls_p2.hip)
MDLS_FOR_PRECISION(, 4)
MDLS_REFINE_FOR_PRECISION(, 4)
MDLS_BATCH_FOR_PRECISION(, 4)
MDLS_CPLX_FOR_PRECISION(, 4)
}  // namespace mdls_impl
