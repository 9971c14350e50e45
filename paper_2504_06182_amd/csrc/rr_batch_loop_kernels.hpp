// rr_batch_loop_kernels.hpp -- definitions of the loop kernels of the batching routine (§IV,
// Alg. 3): included by rr_batch_loop2/5/6.hip, each instantiating one register-slot count.
#pragma once
#include "rr_batch_common.hpp"
#include "rr_batch_loop.hpp"

namespace rr {

extern __shared__ __attribute__((aligned(16))) uint8_t dyn_lds[];

// ---- loop kernels

template <int S, uint32_t F>
__device__ __forceinline__ void loop_entry(const fast::Inst &I, uint32_t lds_bytes)
{
    const fast::Layout L = fast::layout(I.W, I.H, I.move_cap, I.step_cap);
    uint32_t *hdr = (uint32_t *)(I.ws + L.hdr);
    if (hdr[fast::H_STATE] != fast::ST_FAST) return;
    // a ready set that outgrows the registers hands the instance to the general path
    if (fast::loop_fast<S, F>(I, dyn_lds, lds_bytes) && lane_id() == 0) hdr[fast::H_STATE] = fast::ST_GENERIC;
}

template <int S, uint32_t F>
__global__ __launch_bounds__(kWave) void k_loop_one(fast::Inst I, uint32_t lds_bytes)
{
    loop_entry<S, F>(I, lds_bytes);
}

template <int S, uint32_t F>
__global__ __launch_bounds__(kWave, loop_waves(S)) void k_loop_many(const rr_desc *__restrict__ desc, int maxw, int maxh,
                                                     const rr_move *mv, const uint32_t *ga,
                                                     const rr_solve_info *sinfos, uint32_t *bat, uint32_t *stp,
                                                     rr_batch_info *binfos, uint8_t *ws, uint64_t ws_bytes,
                                                     uint32_t lds_bytes)
{
    const uint32_t i = blockIdx.x;
    const rr_desc d = desc[i];
    if (!desc_usable(d, maxw, maxh, ws_bytes)) return;
    loop_entry<S, F>(inst_of(d, i, mv, ga, sinfos, bat, stp, binfos, ws), lds_bytes);
}

}  // namespace rr
