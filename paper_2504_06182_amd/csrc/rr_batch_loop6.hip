// rr_batch_loop6.hip -- the batching loop kernels with 6 register slots (one per local constraint,
// one-instance and many-instance forms).
#include "rr_batch_loop_kernels.hpp"

namespace rr {
RR_LOOP_KERNELS(, 6)
}  // namespace rr
