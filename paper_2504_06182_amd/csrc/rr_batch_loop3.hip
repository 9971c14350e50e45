// rr_batch_loop3.hip -- the batching loop kernels with 3 register slots (one per local constraint,
// one-instance and many-instance forms).
#include "rr_batch_loop_kernels.hpp"

namespace rr {
RR_LOOP_KERNELS(, 3)
}  // namespace rr
