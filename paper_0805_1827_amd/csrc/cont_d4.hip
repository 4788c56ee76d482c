// Continuation kernel instantiation for dimension bound 4.
#include "cont_kernel.hpp"

namespace bmc {
template hipError_t launch_cont_d<4, true>(int, const ContArgs&, int, int, size_t, hipStream_t);
template hipError_t launch_cont_multi_d<4, true>(int, const ContArgs*, const uint32_t*, int, uint32_t,
                                                      uint32_t, int, size_t, hipStream_t, bool);
}  // namespace bmc
