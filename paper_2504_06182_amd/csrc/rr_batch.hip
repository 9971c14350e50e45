// rr_batch.hip -- batching routine (arXiv 2504.06182, §IV, Alg. 3) on gfx950: kernels, launch
// plans and the C entry points.
//
// A batching call runs three kernels on its stream:
//   k_graph_*   one 512-thread workgroup per instance: validation, total steps, the reduced
//               dependency graph and the loop data (rr_batch_graph.hpp);
//   k_loop_*    one wave64 per instance: Alg. 3 with the ready set in registers
//               (rr_batch_loop.hpp), for every instance the graph kernel passed on;
//   k_generic_* one wave64 per instance: the general path (rr_batch_generic.hpp) for the
//               instances outside the fast path's limits (more than 65535 moves, unusual
//               graphs, a ready set that outgrew the registers during the loop, which then
//               hands the instance over) -- every other wave exits.
// Each instance's status moves through a header word in its workspace, so the three launches
// need no host round trip.  Results do not depend on which path ran.  Grids beyond RR_LDS_SIDE
// run the wide path instead (rr_batch_wide.hip: its own graph and loop kernels); a
// many-instance launch whose bounds admit such grids runs both, each skipping the other's
// instances.
#include "rr_device.hpp"
#include "rr.h"
#include "rr_batch_generic.hpp"
#include "rr_batch_graph.hpp"
#include "rr_batch_common.hpp"
#include "rr_batch_wide.hpp"

#include <atomic>
#include <mutex>

static_assert(sizeof(rr_desc) == 80, "rr_desc layout");
static_assert(sizeof(rr_move) == 8, "rr_move layout");

namespace rr {

// ---- graph kernels

// NT threads per instance (graph wavefronts per instance: flags bits 20..23)
template <int NT>
__global__ __launch_bounds__(NT) void k_graph_one(fast::Inst I, uint32_t lds_bytes, uint32_t flags)
{
    __shared__ fast::GraphShared<NT / kWave> S;
    fast::graph_build<NT>(I, S, dyn_lds, lds_bytes, (flags & kFlagGeneric) != 0);
}

template <int NT>
__global__ __launch_bounds__(NT) void k_graph_many(const rr_desc *__restrict__ desc, int maxw, int maxh,
                                                          const rr_move *mv, const uint32_t *ga,
                                                          const rr_solve_info *sinfos, uint32_t *bat, uint32_t *stp,
                                                          rr_batch_info *binfos, uint8_t *ws, uint64_t ws_bytes,
                                                          uint32_t lds_bytes, uint32_t flags)
{
    __shared__ fast::GraphShared<NT / kWave> S;
    const uint32_t i = blockIdx.x;
    const rr_desc d = desc[i];
    if (wide_instance(d.shape, maxw, maxh)) return;
    if (!desc_usable(d, maxw, maxh, ws_bytes)) {
        if (threadIdx.x == 0) {
            const rr_solve_info si = sinfos[i];
            // a workspace region out of bounds is a malformed descriptor (the planner never
            // gives one to an instance it found room for)
            if (!shape_usable(d.shape, maxw, maxh) || (d.step_cap != 0xFFFFFFFFu && !ws_fits(d, ws_bytes)))
                fast::put_info(binfos + i, RR_E_INVAL, 0, 0, 0, 0);
            else if (si.status == RR_INFEASIBLE || (si.status == RR_OK && si.n_moves == 0))
                fast::put_info(binfos + i, RR_OK, 0, 0, 0, 0);   // nothing to batch (no room needed)
            else if (si.status == RR_OK)
                fast::put_info(binfos + i, RR_E_CAPACITY, 0, 0, si.n_steps, si.n_steps);
            else
                fast::put_info(binfos + i, RR_E_INVAL, 0, 0, 0, 0);
        }
        return;
    }
    fast::graph_build<NT>(inst_of(d, i, mv, ga, sinfos, bat, stp, binfos, ws), S, dyn_lds, lds_bytes,
                      (flags & kFlagGeneric) != 0);
}

// ---- loop kernels: instantiated in rr_batch_loop2/5/6.hip

RR_LOOP_KERNELS(extern, 2)
RR_LOOP_KERNELS(extern, 5)
RR_LOOP_KERNELS(extern, 6)

// ---- general path

__device__ __forceinline__ void generic_entry(const fast::Inst &I, gen::BatchLds &S, uint32_t lds_bytes,
                                              uint32_t flags)
{
    const fast::Layout L = fast::layout(I.W, I.H, I.move_cap, I.step_cap);
    const uint32_t *hdr = (const uint32_t *)(I.ws + L.hdr);
    if (hdr[fast::H_STATE] != fast::ST_GENERIC) return;
    gen::BatchArgs A;
    A.W = I.W; A.H = I.H;
    A.moves = I.moves; A.goff = I.goff; A.sinfo = I.sinfo; A.move_cap = I.move_cap;
    A.flags = flags & 0xFFu;
    A.boff = I.boff; A.batch_cap = I.batch_cap; A.steps = I.steps; A.step_cap = I.step_cap; A.binfo = I.binfo;
    A.ws = I.ws + L.gen;
    A.lds16_cap = lds_bytes / 2;
    gen::batch_one(S, A);
}

__global__ __launch_bounds__(kWave) void k_generic_one(fast::Inst I, uint32_t lds_bytes, uint32_t flags)
{
    __shared__ gen::BatchLds S;
    generic_entry(I, S, lds_bytes, flags);
}

__global__ __launch_bounds__(kWave) void k_generic_many(const rr_desc *__restrict__ desc, int maxw, int maxh,
                                                        const rr_move *mv, const uint32_t *ga,
                                                        const rr_solve_info *sinfos, uint32_t *bat, uint32_t *stp,
                                                        rr_batch_info *binfos, uint8_t *ws, uint64_t ws_bytes,
                                                        uint32_t lds_bytes, uint32_t flags)
{
    __shared__ gen::BatchLds S;
    const uint32_t i = blockIdx.x;
    const rr_desc d = desc[i];
    if (!desc_usable(d, maxw, maxh, ws_bytes)) return;
    generic_entry(inst_of(d, i, mv, ga, sinfos, bat, stp, binfos, ws), S, lds_bytes, flags);
}

// ---- arena planner: one 1024-thread workgroup scans the instances in chunks of 1024

constexpr int kPlanThreads = 1024;

__global__ __launch_bounds__(kPlanThreads) void k_plan_many(uint32_t n, rr_desc *desc, const rr_solve_info *infos,
                                                            uint64_t step_pool, uint64_t batch_pool,
                                                            uint64_t ws_pool, uint64_t *totals)
{
    __shared__ uint64_t part[3][kPlanThreads / kWave];
    __shared__ uint64_t carry[3];
    const int tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
    if (tid < 3) carry[tid] = 0;
    __syncthreads();
    for (uint32_t base = 0; base < n; base += kPlanThreads) {
        const uint32_t i = base + tid;
        uint64_t v[3] = {0, 0, 0};
        rr_desc d;
        if (i < n) {
            d = desc[i];
            const rr_solve_info si = infos[i];
            uint32_t sc = (si.status == RR_OK && si.n_steps > 0) ? si.n_steps : 1u;
            v[0] = sc;
            v[1] = (uint64_t)sc + 1;
            v[2] = wide::wide_shape(d.shape.w, d.shape.h) ? wide::al256(wide::layout(d.shape.w, d.shape.h, d.move_cap).total)
                                                           : fast::al256(fast::layout(d.shape.w, d.shape.h, d.move_cap, sc).total);
        }
        uint64_t incl[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            uint64_t x = v[q];
#pragma unroll
            for (int o = 1; o < kWave; o <<= 1) {
                const uint64_t t = shfl_u64(x, lane >= o ? lane - o : lane);
                if (lane >= o) x += t;
            }
            incl[q] = x;
            if (lane == kWave - 1) part[q][wid] = x;
        }
        __syncthreads();
        uint64_t off[3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            uint64_t pre = carry[q];
            for (int w = 0; w < wid; ++w) pre += part[q][w];
            off[q] = pre + incl[q] - v[q];
        }
        if (i < n) {
            const bool fits = off[0] + v[0] <= step_pool && off[1] + v[1] <= batch_pool && off[2] + v[2] <= ws_pool;
            d.step_cap = fits ? (uint32_t)v[0] : 0xFFFFFFFFu;
            d.batch_cap = fits ? (uint32_t)v[0] : 0u;
            d.step_off = fits ? off[0] : 0;
            d.batch_off = fits ? off[1] : 0;
            d.ws_off = fits ? off[2] : 0;
            desc[i] = d;
        }
        __syncthreads();
        if (tid < 3) {
            uint64_t tot = 0;
            for (int w = 0; w < kPlanThreads / kWave; ++w) tot += part[tid][w];
            carry[tid] += tot;
        }
        __syncthreads();
    }
    if (totals && tid < 3) totals[tid] = carry[tid];
}

// ---- launch plan

// Register slots of the loop kernel by the largest grid side.  The ready sets of red-rec
// outputs stay near two moves per target row (88 or 89 at most on 64 x 64 grids with a 44 x 44
// target); 128 positions hold them for 64-trap sides, with registers to spare for 8 waves per
// SIMD.  An instance whose set outgrows the slots is redone by the general path.
static int loop_slots(uint32_t max_side) { return max_side <= 64 ? 2 : (max_side <= 128 ? 5 : 6); }

// LDS one workgroup may take on the current device (read once per device, so that later calls,
// also under stream capture, make no device query)
static uint32_t device_lds_limit()
{
    constexpr int kMaxDevices = 64;
    static std::atomic<uint32_t> cache[kMaxDevices];
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0) return 65536u;
    if (dev < kMaxDevices) {
        const uint32_t c = cache[dev].load(std::memory_order_relaxed);
        if (c) return c;
    }
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        v = 65536;
    if (dev < kMaxDevices) cache[dev].store((uint32_t)v, std::memory_order_relaxed);
    return (uint32_t)v;
}

struct Plan {
    int S;
    uint32_t graph_lds, loop_lds, gen_lds;
    uint32_t graph_threads;      // threads per instance of the graph kernel
};

// batching flags: bits 17..19 zero, bits 20..23 the graph kernel's wavefronts per instance
// divided by four (0: the default, 8 wavefronts; 1, 2 or 4: 4, 8 or 16 wavefronts)
static bool batch_flags_valid(uint32_t flags)
{
    const uint32_t gw = (flags >> 20) & 0xFu;
    return (flags & 0xFFu) <= RR_LAMBDA_NONE && ((flags >> 17) & 0x7u) == 0u &&
           (gw == 0u || gw == 1u || gw == 2u || gw == 4u);
}

static uint32_t graph_threads_of(uint32_t flags)
{
    const uint32_t gw = (flags >> 20) & 0xFu;
    return gw == 0u ? (uint32_t)fast::kGT : 256u * gw;
}

// LDS budgets.  Graph kernel: 64 KiB for grids up to 64 x 64, two workgroups per CU (a 64 x 64
// shot of ~21k trap visits needs about 62 KiB; larger ones build in the workspace; measured:
// 3.6 ms with 64 KiB against 5.6 ms with 96 KiB and 8.3 ms all in the workspace); flags bits
// 24..31 override it in KiB (0 = default).  Loop
// kernel: for many-instance launches the loop data stays in the workspace by default -- the
// kernel is latency-bound, and leaving LDS free lets every SIMD hold as many waves as its
// registers allow (measured on the 8192-shot 64 x 64 workload: 10.2 ms with 1 KiB per wave
// against 21.5 ms with 24 KiB); a single instance keeps its data in LDS.  Flags bits 8..15
// override the loop budget in KiB.  General path: its 16-bit loop state.
static Plan make_plan(uint32_t flags, uint32_t max_w, uint32_t max_h, bool single)
{
    const uint32_t side = max_w > max_h ? max_w : max_h;
    const uint32_t lim = device_lds_limit();
    const uint32_t gen_static = (uint32_t)sizeof(gen::BatchLds);
    Plan P;
    P.S = loop_slots(side);
    const uint32_t gkib = (flags >> 24) & 0xFFu;
    if (gkib) P.graph_lds = gkib * 1024u;
    else P.graph_lds = single ? 120u * 1024u : 64u * 1024u;
    if (P.graph_lds + sizeof(fast::GraphShared<16>) > lim) P.graph_lds = lim - (uint32_t)sizeof(fast::GraphShared<16>);
    P.graph_threads = graph_threads_of(flags);
    uint32_t kib = (flags >> 8) & 0xFFu;
    if (kib == 0) kib = single ? 64u : 1u;
    P.loop_lds = kib * 1024u;
    // the loop always keeps its group counts and merge scratch in LDS
    const uint32_t small = 8u * fast::fast_group_cap((int)max_w, (int)max_h, 0xFFFFFFFFu) + 16u * kWave * P.S + 16u;
    if (P.loop_lds < small) P.loop_lds = small;
    if (P.loop_lds > lim) P.loop_lds = lim;
    const uint32_t gkb = kib < 24u ? 24u : kib;
    P.gen_lds = gkb > 56u ? 56u * 1024u : gkb * 1024u;
    if (P.gen_lds + gen_static > lim) P.gen_lds = lim - gen_static;
    return P;
}

}  // namespace rr

using namespace rr;

extern "C" rr_status rr_plan_many(uint32_t n, rr_desc *desc, const rr_solve_info *infos, uint64_t step_pool,
                                  uint64_t batch_pool, uint64_t ws_pool_bytes, uint64_t *totals, void *stream)
{
    if (n == 0) return RR_OK;
    if (!desc || !infos) return RR_E_INVAL;
    hipLaunchKernelGGL(k_plan_many, dim3(1), dim3(kPlanThreads), 0, (hipStream_t)stream, n, desc, infos, step_pool,
                       batch_pool, ws_pool_bytes, totals);
    return hipGetLastError() == hipSuccess ? RR_OK : RR_E_DEVICE;
}

extern "C" size_t rr_batch_workspace_bytes(rr_shape shape, uint32_t move_cap, uint32_t step_cap)
{
    if (wide::wide_shape(shape.w, shape.h)) return wide::layout(shape.w, shape.h, move_cap).total;
    return fast::layout(shape.w, shape.h, move_cap, step_cap).total;
}

extern "C" rr_status rr_batch_moves(rr_shape shape, const rr_move *moves, const uint32_t *group_off,
                                    const rr_solve_info *sinfo, uint32_t move_cap, uint32_t flags,
                                    uint32_t *batch_off, uint32_t batch_cap, uint32_t *steps, uint32_t step_cap,
                                    rr_batch_info *binfo, void *workspace, size_t workspace_bytes, void *stream)
{
    if (!(shape.w >= 1 && shape.h >= 1 && shape.x0 < shape.x1 && shape.x1 <= shape.w && shape.y0 < shape.y1 &&
          shape.y1 <= shape.h))
        return RR_E_INVAL;
    if (shape.w > RR_MAX_SIDE || shape.h > RR_MAX_SIDE) return RR_E_UNSUPPORTED;
    if (!batch_flags_valid(flags)) return RR_E_INVAL;
    if (!group_off || !sinfo || !batch_off || !binfo || (move_cap > 0 && !moves) || (step_cap > 0 && !steps))
        return RR_E_INVAL;
    if (((uintptr_t)moves & 7u) != 0) return RR_E_INVAL;
    if (!workspace || workspace_bytes < rr_batch_workspace_bytes(shape, move_cap, step_cap)) return RR_E_NOMEM;
    fast::Inst I;
    I.W = shape.w; I.H = shape.h;
    I.moves = moves; I.goff = group_off; I.sinfo = sinfo;
    I.move_cap = move_cap; I.step_cap = step_cap; I.batch_cap = batch_cap;
    I.boff = batch_off; I.steps = steps; I.binfo = binfo;
    I.ws = (uint8_t *)workspace;
    hipStream_t st = (hipStream_t)stream;
    if (wide::wide_shape(shape.w, shape.h)) {
        if (((uintptr_t)workspace & 255u) != 0) return RR_E_INVAL;
        return wide::launch_one(I, flags, st) == hipSuccess ? RR_OK : RR_E_DEVICE;
    }
    const Plan P = make_plan(flags, shape.w, shape.h, true);
    if (P.graph_threads == 256u)
        hipLaunchKernelGGL(k_graph_one<256>, dim3(1), dim3(256), P.graph_lds, st, I, P.graph_lds, flags);
    else if (P.graph_threads == 1024u)
        hipLaunchKernelGGL(k_graph_one<1024>, dim3(1), dim3(1024), P.graph_lds, st, I, P.graph_lds, flags);
    else
        hipLaunchKernelGGL(k_graph_one<512>, dim3(1), dim3(512), P.graph_lds, st, I, P.graph_lds, flags);
#define RR_LOOP_ONE(SS, FF) hipLaunchKernelGGL((k_loop_one<SS, FF>), dim3(1), dim3(kWave), P.loop_lds, st, I, P.loop_lds)
#define RR_LOOP_ONE_F(SS)                                                                                          \
    switch (flags & 0xFFu) {                                                                                       \
    case RR_LAMBDA_LINE_OR_COL: RR_LOOP_ONE(SS, RR_LAMBDA_LINE_OR_COL); break;                                     \
    case RR_LAMBDA_ALONG: RR_LOOP_ONE(SS, RR_LAMBDA_ALONG); break;                                                 \
    default: RR_LOOP_ONE(SS, RR_LAMBDA_NONE); break;                                                               \
    }
    switch (P.S) {
    case 2: RR_LOOP_ONE_F(2); break;
    case 5: RR_LOOP_ONE_F(5); break;
    default: RR_LOOP_ONE_F(6); break;
    }
#undef RR_LOOP_ONE_F
#undef RR_LOOP_ONE
    hipLaunchKernelGGL(k_generic_one, dim3(1), dim3(kWave), P.gen_lds, st, I, P.gen_lds, flags);
    return hipGetLastError() == hipSuccess ? RR_OK : RR_E_DEVICE;
}

extern "C" rr_status rr_batch_moves_many_staged(uint32_t n, const rr_desc *desc, uint32_t max_w, uint32_t max_h,
                                                const rr_move *move_arena, const uint32_t *group_arena,
                                                const rr_solve_info *sinfos, uint32_t flags, uint32_t *batch_arena,
                                                uint32_t *step_arena, rr_batch_info *binfos, void *workspace,
                                                size_t workspace_bytes, void *stream, void *graph_done_event,
                                                void *loop_done_event)
{
    if (n == 0) return RR_OK;
    if (!desc || !move_arena || !group_arena || !sinfos || !batch_arena || !step_arena || !binfos || !workspace)
        return RR_E_INVAL;
    if (!batch_flags_valid(flags) || max_w < 1 || max_h < 1) return RR_E_INVAL;
    if (max_w > RR_MAX_SIDE || max_h > RR_MAX_SIDE) return RR_E_UNSUPPORTED;
    if (((uintptr_t)move_arena & 7u) != 0) return RR_E_INVAL;
    hipStream_t st = (hipStream_t)stream;
    uint8_t *ws = (uint8_t *)workspace;
    const bool wide_too = max_w > RR_LDS_SIDE || max_h > RR_LDS_SIDE;
    if (wide_too && wide::launch_graph_many(n, desc, (int)max_w, (int)max_h, move_arena, group_arena, sinfos,
                                            batch_arena, step_arena, binfos, ws, (uint64_t)workspace_bytes,
                                            st) != hipSuccess)
        return RR_E_DEVICE;
    const Plan P = make_plan(flags, max_w < RR_LDS_SIDE ? max_w : RR_LDS_SIDE, max_h < RR_LDS_SIDE ? max_h : RR_LDS_SIDE,
                             false);
#define RR_GRAPH_MANY(NT)                                                                                          \
    hipLaunchKernelGGL(k_graph_many<NT>, dim3(n), dim3(NT), P.graph_lds, st, desc, (int)max_w, (int)max_h,          \
                       move_arena, group_arena, sinfos, batch_arena, step_arena, binfos, ws, (uint64_t)workspace_bytes, \
                       P.graph_lds, flags)
    if (P.graph_threads == 256u) RR_GRAPH_MANY(256);
    else if (P.graph_threads == 1024u) RR_GRAPH_MANY(1024);
    else RR_GRAPH_MANY(512);
#undef RR_GRAPH_MANY
    if (graph_done_event && hipEventRecord((hipEvent_t)graph_done_event, st) != hipSuccess) return RR_E_DEVICE;
    if (wide_too && wide::launch_loop_many(n, desc, (int)max_w, (int)max_h, move_arena, group_arena, sinfos,
                                           batch_arena, step_arena, binfos, ws, (uint64_t)workspace_bytes, flags,
                                           st) != hipSuccess)
        return RR_E_DEVICE;
#define RR_LOOP_MANY(SS, FF)                                                                                       \
    hipLaunchKernelGGL((k_loop_many<SS, FF>), dim3(n), dim3(kWave), P.loop_lds, st, desc, (int)max_w, (int)max_h,  \
                       move_arena, group_arena, sinfos, batch_arena, step_arena, binfos, ws,                       \
                       (uint64_t)workspace_bytes, P.loop_lds)
#define RR_LOOP_MANY_F(SS)                                                                                         \
    switch (flags & 0xFFu) {                                                                                       \
    case RR_LAMBDA_LINE_OR_COL: RR_LOOP_MANY(SS, RR_LAMBDA_LINE_OR_COL); break;                                    \
    case RR_LAMBDA_ALONG: RR_LOOP_MANY(SS, RR_LAMBDA_ALONG); break;                                                \
    default: RR_LOOP_MANY(SS, RR_LAMBDA_NONE); break;                                                              \
    }
    switch (P.S) {
    case 2: RR_LOOP_MANY_F(2); break;
    case 5: RR_LOOP_MANY_F(5); break;
    default: RR_LOOP_MANY_F(6); break;
    }
#undef RR_LOOP_MANY_F
#undef RR_LOOP_MANY
    if (loop_done_event && hipEventRecord((hipEvent_t)loop_done_event, st) != hipSuccess) return RR_E_DEVICE;
    hipLaunchKernelGGL(k_generic_many, dim3(n), dim3(kWave), P.gen_lds, st, desc, (int)max_w, (int)max_h, move_arena,
                       group_arena, sinfos, batch_arena, step_arena, binfos, ws, (uint64_t)workspace_bytes, P.gen_lds,
                       flags);
    return hipGetLastError() == hipSuccess ? RR_OK : RR_E_DEVICE;
}

extern "C" rr_status rr_batch_moves_many(uint32_t n, const rr_desc *desc, uint32_t max_w, uint32_t max_h,
                                         const rr_move *move_arena, const uint32_t *group_arena,
                                         const rr_solve_info *sinfos, uint32_t flags, uint32_t *batch_arena,
                                         uint32_t *step_arena, rr_batch_info *binfos, void *workspace,
                                         size_t workspace_bytes, void *stream)
{
    return rr_batch_moves_many_staged(n, desc, max_w, max_h, move_arena, group_arena, sinfos, flags, batch_arena,
                                      step_arena, binfos, workspace, workspace_bytes, stream, nullptr, nullptr);
}

// ---- batching with no allocation: the workspace is a file-scope device array

// One per device (the code object is loaded on every device the library runs on).  In host code
// `scratch` names a host-side stand-in, never the device memory: its device address comes from
// hipGetSymbolAddress, taken once per device with that device current.
static __device__ __align__(256) uint8_t scratch[RR_NOALLOC_WORKSPACE_BYTES];

namespace {
constexpr int kMaxScratchDevices = 64;
std::once_flag scratch_once[kMaxScratchDevices];
void *scratch_addr[kMaxScratchDevices];
hipError_t scratch_err[kMaxScratchDevices];

// device address of the current device's scratch array (nullptr on failure)
void *scratch_for_current_device()
{
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxScratchDevices) return nullptr;
    std::call_once(scratch_once[dev], [dev] {
        void *p = nullptr;
        scratch_err[dev] = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        scratch_addr[dev] = scratch_err[dev] == hipSuccess ? p : nullptr;
    });
    return scratch_addr[dev];
}
}  // namespace

extern "C" rr_status rr_batch_moves_noalloc(rr_shape shape, const rr_move *moves, const uint32_t *group_off,
                                            const rr_solve_info *sinfo, uint32_t move_cap, uint32_t flags,
                                            uint32_t *batch_off, uint32_t batch_cap, uint32_t *steps,
                                            uint32_t step_cap, rr_batch_info *binfo, void *stream)
{
    if (!(shape.w >= 1 && shape.h >= 1 && shape.x0 < shape.x1 && shape.x1 <= shape.w && shape.y0 < shape.y1 &&
          shape.y1 <= shape.h))
        return RR_E_INVAL;
    if (shape.w > RR_LDS_SIDE || shape.h > RR_LDS_SIDE) return RR_E_UNSUPPORTED;
    if (rr_batch_workspace_bytes(shape, move_cap, step_cap) > (size_t)RR_NOALLOC_WORKSPACE_BYTES) return RR_E_NOMEM;
    void *ws = scratch_for_current_device();
    if (!ws) return RR_E_DEVICE;
    return rr_batch_moves(shape, moves, group_off, sinfo, move_cap, flags, batch_off, batch_cap, steps, step_cap,
                          binfo, ws, (size_t)RR_NOALLOC_WORKSPACE_BYTES, stream);
}
