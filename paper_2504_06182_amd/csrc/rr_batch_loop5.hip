// rr_batch_loop5.hip -- the batching loop kernels with 5 register slots (one per local constraint,
// one-instance and many-instance forms).
#include "rr_batch_loop_kernels.hpp"

namespace rr {
RR_LOOP_KERNELS(, 5)
}  // namespace rr
