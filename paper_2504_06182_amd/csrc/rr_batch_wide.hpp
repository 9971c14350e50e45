// rr_batch_wide.hpp -- the batching path for grids beyond RR_LDS_SIDE per side (up to
// RR_MAX_SIDE): its workspace layout, shared with the arena planner, and its host launchers
// (kernels in rr_batch_wide.hip).
#pragma once
#include "rr_device.hpp"
#include "rr.h"
#include "rr_batch_graph.hpp"

namespace rr {
namespace wide {

constexpr uint32_t kMaxMoves = (1u << 21) - 1;   // move index in 21 bits of a ready key
constexpr uint32_t kMaxGroups = 2048;             // group in 11 bits
constexpr int kMaxPreds = 8;                      // in-group predecessor set of one move
constexpr uint32_t kGroupCap = 2048;              // moves of one group staged in LDS

__host__ __device__ inline bool wide_shape(int w, int h) { return w > (int)RR_LDS_SIDE || h > (int)RR_LDS_SIDE; }

// groups an instance may have: W + H (rr_solve gives at most sw + sh), at most kMaxGroups
__host__ __device__ inline uint32_t group_bound(int W, int H)
{
    const uint32_t g = (uint32_t)W + (uint32_t)H;
    return g < kMaxGroups ? g : kMaxGroups;
}

__host__ __device__ inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// Workspace of one instance (offsets 256-byte aligned):
//   hdr    header words (state, total steps, moves, groups)
//   lastg  last group to touch each trap (the graph kernel's sweep)
//   gbits  predecessor groups of each group, one bit row of gw words per group
//   preds  in-group predecessor set of each move (kMaxPreds words), pend their count
//   scnt   successor list offsets (K + 1), sfill fill counters, slist successor lists
//   gpend  predecessor groups per group, gcnt / gfill / glist the groups waiting on each group
//   hoff   head-move list offsets per group (G + 1), heads the head moves
//   rec    release record of each move (16 B): how it releases its successors -- none, one
//          successor that waits on nothing else (its index and packed move), or a list
struct Layout {
    size_t hdr, lastg, gbits, preds, pend, scnt, sfill, slist, gpend, gcnt, gfill, glist, hoff, heads, rec, total;
    uint32_t gw;
};

__host__ __device__ inline Layout layout(int W, int H, uint32_t move_cap)
{
    Layout L;
    const size_t K = (size_t)move_cap + 1, G = group_bound(W, H);
    L.gw = (uint32_t)((G + 31) / 32);
    size_t p = 0;
    auto take = [&](size_t bytes) { const size_t at = p; p = al256(p + bytes); return at; };
    L.hdr = take(64);
    L.lastg = take(4 * (size_t)W * H);
    L.gbits = take(4 * G * L.gw);
    L.preds = take(4 * K * kMaxPreds);
    L.pend = take(4 * K);
    L.scnt = take(4 * (K + 1));
    L.sfill = take(4 * K);
    L.slist = take(4 * K * kMaxPreds);
    L.gpend = take(4 * G);
    L.gcnt = take(4 * (G + 1));
    L.gfill = take(4 * G);
    L.glist = take(4 * G * G);
    L.hoff = take(4 * (G + 1));
    L.heads = take(4 * K);
    L.rec = take(16 * K);
    L.total = p;
    return L;
}

// One instance: graph kernel then loop kernel (Λ = flags bits 0..7).
hipError_t launch_one(const fast::Inst &I, uint32_t flags, hipStream_t st);

// The instances beyond RR_LDS_SIDE of a many-instance launch (every other one is skipped).
hipError_t launch_graph_many(uint32_t n, const rr_desc *desc, int maxw, int maxh, const rr_move *mv,
                             const uint32_t *ga, const rr_solve_info *sinfos, uint32_t *bat, uint32_t *stp,
                             rr_batch_info *binfos, uint8_t *ws, uint64_t ws_bytes, hipStream_t st);
hipError_t launch_loop_many(uint32_t n, const rr_desc *desc, int maxw, int maxh, const rr_move *mv,
                            const uint32_t *ga, const rr_solve_info *sinfos, uint32_t *bat, uint32_t *stp,
                            rr_batch_info *binfos, uint8_t *ws, uint64_t ws_bytes, uint32_t flags, hipStream_t st);

}  // namespace wide
}  // namespace rr
