// rr_batch_loop8.hip -- the batching loop kernels with 8 register slots (one per local constraint,
// one-instance and many-instance forms).
#include "rr_batch_loop_kernels.hpp"

namespace rr {
RR_LOOP_KERNELS(, 8)
}  // namespace rr
