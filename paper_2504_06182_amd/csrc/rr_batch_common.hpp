// rr_batch_common.hpp -- what the batching translation units share: descriptor checks, the
// per-instance view of a many-instance launch, and the loop kernels' declarations (their
// definitions are instantiated in rr_batch_loop2/5/6.hip, one file per register-slot count, so
// that the three compile in parallel).
#pragma once
#include "rr_device.hpp"
#include "rr.h"
#include "rr_batch_graph.hpp"

namespace rr {

constexpr uint32_t kFlagGeneric = 1u << 16;

// shape check of a many-instance descriptor for the kernels of grids up to RR_LDS_SIDE
__device__ __forceinline__ bool shape_usable(const rr_shape s, int maxw, int maxh)
{
    return s.w >= 1 && s.h >= 1 && s.w <= maxw && s.h <= maxh && s.w <= RR_LDS_SIDE && s.h <= RR_LDS_SIDE &&
           s.x0 < s.x1 && s.x1 <= s.w && s.y0 < s.y1 && s.y1 <= s.h;
}

// an instance of the wide kernels (rr_batch_wide.hip) in a launch whose bounds admit it: the
// kernels of the smaller grids leave it alone
__device__ __forceinline__ bool wide_instance(const rr_shape s, int maxw, int maxh)
{
    return (s.w > RR_LDS_SIDE || s.h > RR_LDS_SIDE) && s.w <= maxw && s.h <= maxh;
}

// the instance's workspace region [ws_off, ws_off + layout total) is 256-byte aligned and lies
// inside the workspace
__device__ __forceinline__ bool ws_fits(const rr_desc &d, uint64_t ws_bytes)
{
    const uint64_t need = fast::layout(d.shape.w, d.shape.h, d.move_cap, d.step_cap).total;
    return (d.ws_off & 255u) == 0 && d.ws_off <= ws_bytes && need <= ws_bytes - d.ws_off;
}

// a descriptor the kernels may run: valid shape, room found by the planner, workspace in bounds
__device__ __forceinline__ bool desc_usable(const rr_desc &d, int maxw, int maxh, uint64_t ws_bytes)
{
    return shape_usable(d.shape, maxw, maxh) && d.step_cap != 0xFFFFFFFFu && ws_fits(d, ws_bytes);
}

__device__ __forceinline__ fast::Inst inst_of(const rr_desc &d, uint32_t i, const rr_move *mv, const uint32_t *ga,
                                              const rr_solve_info *sinfos, uint32_t *bat, uint32_t *stp,
                                              rr_batch_info *binfos, uint8_t *ws)
{
    fast::Inst I;
    I.W = d.shape.w; I.H = d.shape.h;
    I.moves = mv + d.move_off;
    I.goff = ga + d.group_off;
    I.sinfo = sinfos + i;
    I.move_cap = d.move_cap;
    I.step_cap = d.step_cap;
    I.batch_cap = d.batch_cap;
    I.boff = bat + d.batch_off;
    I.steps = stp + d.step_off;
    I.binfo = binfos + i;
    I.ws = ws + d.ws_off;
    return I;
}

extern __shared__ __attribute__((aligned(16))) uint8_t dyn_lds[];

// ---- loop kernels (S register slots, F the local constraint: one kernel per constraint)

// Waves per SIMD the many-instance loop kernel is compiled for: 8 with 2 register slots (its
// own choice, 106 SGPRs, leaves room for 7, so an 8192-instance launch would run a second round
// on 1024 SIMDs; the bound of 8 spills uniform values to VGPR lanes and still runs faster); the
// larger ready sets keep the compiler's choice (8 would spill them to scratch).
constexpr int loop_waves(int S) { return S == 2 ? 8 : 1; }

template <int S, uint32_t F>
__global__ __launch_bounds__(kWave) void k_loop_one(fast::Inst I, uint32_t lds_bytes);

template <int S, uint32_t F>
__global__ __launch_bounds__(kWave, loop_waves(S)) void k_loop_many(const rr_desc *__restrict__ desc, int maxw, int maxh,
                                                     const rr_move *mv, const uint32_t *ga,
                                                     const rr_solve_info *sinfos, uint32_t *bat, uint32_t *stp,
                                                     rr_batch_info *binfos, uint8_t *ws, uint64_t ws_bytes,
                                                     uint32_t lds_bytes);

#define RR_LOOP_KERNELS(PREFIX, SS)                                                                                \
    PREFIX template __global__ void k_loop_one<SS, 0u>(fast::Inst, uint32_t);                                      \
    PREFIX template __global__ void k_loop_one<SS, 1u>(fast::Inst, uint32_t);                                      \
    PREFIX template __global__ void k_loop_one<SS, 2u>(fast::Inst, uint32_t);                                      \
    PREFIX template __global__ void k_loop_many<SS, 0u>(const rr_desc *__restrict__, int, int, const rr_move *,     \
                                                        const uint32_t *, const rr_solve_info *, uint32_t *,          \
                                                        uint32_t *, rr_batch_info *, uint8_t *, uint64_t, uint32_t);  \
    PREFIX template __global__ void k_loop_many<SS, 1u>(const rr_desc *__restrict__, int, int, const rr_move *,     \
                                                        const uint32_t *, const rr_solve_info *, uint32_t *,          \
                                                        uint32_t *, rr_batch_info *, uint8_t *, uint64_t, uint32_t);  \
    PREFIX template __global__ void k_loop_many<SS, 2u>(const rr_desc *__restrict__, int, int, const rr_move *,     \
                                                        const uint32_t *, const rr_solve_info *, uint32_t *,          \
                                                        uint32_t *, rr_batch_info *, uint8_t *, uint64_t, uint32_t);

}  // namespace rr
