// mdls_p8.hip -- kernels and drivers instantiated for 8-limb numbers.
#include "mdls_impl.hpp"

namespace mdls_impl {
MDLS_FOR_PRECISION(, 8)
}  // namespace mdls_impl
