/*
 * rr.h -- red-rec solver and batching routine for atom reconfiguration on MI355X (gfx950).
 *
 * Method: "Efficient algorithms to solve atom reconfiguration problems III: the bird and
 * batching algorithms and other parallel implementations on GPUs" (arXiv 2504.06182):
 * the redistribution-reconfiguration solver (§III.C, Alg. 1, run in the order of its parallel
 * form, §III.D) on a rectangular trap grid, and the batching routine that merges its
 * elementary displacements into simultaneous ones (§IV, Alg. 3, with its local constraint).
 *
 * Conventions shared by every entry point
 *  - Grid: W columns x H rows, 1 <= W, H <= 256 for the device kernels.  Column x runs left to
 *    right, row y bottom to top (§III.C).  Target T = [x0,x1) x [y0,y1), non-empty, inside the
 *    grid.
 *  - Occupancy layout ("bit rows"): uint64_t[H][ws], ws = ceil(W/64); trap (x, y) is bit x%64 of
 *    word y*ws + x/64.  Bits at x >= W are ignored on input and written as 0 on output.
 *  - Unless stated otherwise every pointer argument is a DEVICE pointer owned by the caller; the
 *    library never allocates, frees or synchronises inside these calls.  Work is enqueued on
 *    `stream` (a hipStream_t; NULL = the default stream) and completes asynchronously.
 *  - The return value reports only what the host can detect before launching: invalid
 *    arguments (RR_E_INVAL), a grid beyond the supported size (RR_E_UNSUPPORTED), a workspace
 *    smaller than the matching *_workspace_bytes() (RR_E_NOMEM) or a launch failure
 *    (RR_E_DEVICE).  Outcomes that depend on the data are written to the device-side info
 *    struct: RR_OK, RR_INFEASIBLE (no move, final = input), RR_E_CAPACITY (an output array is too
 *    small; need_* hold the exact sizes, contents of the outputs are unspecified), RR_E_INVAL
 *    (malformed device-side input, e.g. a move off the grid) or, from the batching path of grids
 *    beyond RR_LDS_SIDE, RR_E_UNSUPPORTED (an instance beyond that path's fixed capacities).
 *  - Every result is deterministic: the same input gives the same bytes, whatever the launch
 *    configuration, and equals the CPU reference bit for bit.
 *  - Calls on different streams that share no output or workspace memory may run concurrently.
 */
#ifndef RR_H
#define RR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    RR_OK = 0,
    RR_INFEASIBLE = 1,
    RR_E_INVAL = -1,
    RR_E_CAPACITY = -2,
    RR_E_DEVICE = -3,
    RR_E_NOMEM = -4,
    RR_E_INTERNAL = -5,
    RR_E_UNSUPPORTED = -6
} rr_status;

/* Grid W x H and target rectangle [x0,x1) x [y0,y1). */
typedef struct { uint16_t w, h, x0, y0, x1, y1; } rr_shape;

/* One displacement (a path of the path system, §II.C): the token at (sx, sy) runs along row sy
 * to column dx, then along column dx to (dx, dy).  Every emitted move has at least one step. */
typedef struct { uint16_t sx, sy, dx, dy; } rr_move;

/* Device-side result of a solve.  n_steps = summed path length (Manhattan) of all moves.
 * need_moves / need_groups: exact sizes, filled in whenever the instance was solved or the
 * capacity was short. */
typedef struct {
    int32_t status;
    uint32_t n_moves, n_groups, n_steps, need_moves, need_groups;
} rr_solve_info;

/* Device-side result of a batching call. */
typedef struct {
    int32_t status;
    uint32_t n_batches, n_steps, need_batches, need_steps;
} rr_batch_info;

/* Local constraints of the batching routine (§IV, "constrained batching"). */
#define RR_LAMBDA_LINE_OR_COL 0u  /* same direction, and the moving tokens share a row or a column */
#define RR_LAMBDA_ALONG       1u  /* same direction, on one line that runs along that direction */
#define RR_LAMBDA_NONE        2u  /* only the vertex-disjointness of Alg. 3 */
/* Run every instance on the general batching path (no ready-set register limit; slower).  The
 * default picks the fast path per instance and falls back to the general one by itself: for
 * instances beyond its limits, and for one whose ready set outgrows the loop kernel's
 * registers while it runs (that instance is then redone from its inputs). */
#define RR_BATCH_GENERIC      (1u << 16)

/* Order of Alg. 1 in rr_solve (flags bits 0..7): the parallel form of §III.D, where every
 * column of zero or positive surplus is solved from the outset and a donor hands over its
 * excess (the default), or the serial form of §III.C, where only zero-surplus columns are
 * solved first, a donor hands over its reservoir tokens nearest the target first and is solved
 * when it settles (after its receiver when both settle, before its tokens are marked when it
 * is exhausted), and donors still unsolved after the loop are solved last, in ascending x.
 * Both orders pair the same columns in the same order; they differ in which donor tokens move
 * and in the order of the groups. */
#define RR_REDREC_PARALLEL 0u
#define RR_REDREC_SERIAL   1u
/* bird (§III.E, Alg. 2) instead of red-rec, same flags field: after the row pre-pass and the
 * columns of non-negative surplus (solved as in RR_REDREC_PARALLEL), each column of negative
 * surplus, leftmost first, is filled by the generalized exact 1D from its own tokens and the
 * reservoir tokens of every other column, a token at (x, y) standing at the virtual row
 * y + |x - j| above the target or y - |x - j| below it; among tokens of one virtual row the
 * nearest column comes first, then the left one.  One group per such column. */
#define RR_BIRD            2u
/* Wavefronts per instance of the solve kernels (flags bits 8..11): 1, 2 or 4 (0 = the default,
 * 4).  A launch needs at least one thread per grid side: 64 * waves >= the largest side of the
 * call's grids up to RR_LDS_SIDE, else the call returns RR_E_INVAL.  Grids beyond RR_LDS_SIDE
 * always run 16 wavefronts (rr_solve then wants 0 in this field).  A schedule knob: results do
 * not depend on it. */
#define RR_SOLVE_WAVES(n)  ((uint32_t)(n) << 8)

/* Largest grid side the device kernels take. */
#define RR_MAX_SIDE 1024u
/* Largest grid side whose per-instance state stays in LDS.  Larger grids run the wide kernels:
 * the solve keeps its state in the caller's workspace (rr_solve_workspace_bytes), and batching
 * runs a path of its own (rr_batch_moves). */
#define RR_LDS_SIDE 256u

/* ------------------------------------------------------------------------------------------ */
/* Single instance                                                                             */

/* Bytes of device workspace rr_solve needs for this shape: 0 up to RR_LDS_SIDE per side, about
 * 0.75 MiB beyond.  The workspace must be 256-byte aligned. */
size_t rr_solve_workspace_bytes(rr_shape shape);

/* Solve one instance with red-rec (§III.C-D, Alg. 1).
 *   occ        [in]  bit rows of the initial loading (H*ws words).
 *   moves      [out] rr_move[move_cap]; move_cap >= 2*(x1-x0)*(y1-y0) always suffices.
 *   group_off  [out] uint32_t[group_cap + 1]: moves of group g are [group_off[g], group_off[g+1]);
 *                    group_cap >= (x1-x0) + (y1-y0) always suffices.  Groups are, in order: one
 *                    per target row with moves (row pre-pass), one per column of non-negative
 *                    surplus with moves, one per receiver column in the order it was saturated.
 *   final_occ  [out] bit rows of the grid after all moves (H*ws words).
 *   info       [out] one rr_solve_info.
 *   flags      [in]  bits 0..7: RR_REDREC_PARALLEL, RR_REDREC_SERIAL or RR_BIRD; bits 8..11:
 *                    RR_SOLVE_WAVES(1, 2 or 4) or 0; other bits 0 (else RR_E_INVAL).
 * An instance is solved iff F = N - D - (x1-x0)*(y1-y0) >= 0, decided before any move: N is
 * the number of tokens and D the number of target-row tokens beyond the target width,
 * counted only when the target leaves side columns (the row pre-pass parks those tokens in
 * the side columns and they never move again).  For a target spanning every column this is
 * |S| >= |T| (§II.B); with side columns it is stricter, so an instance whose target is
 * reachable can still be refused (a failure of the heuristic, e.g. a 4 x 4 grid whose row 1
 * is full against the target [1,3) x [1,3)).  A refused instance gives status
 * RR_INFEASIBLE, zero moves and final_occ = occ. */
rr_status rr_solve(rr_shape shape, const uint64_t *occ,
                   rr_move *moves, uint32_t move_cap,
                   uint32_t *group_off, uint32_t group_cap,
                   uint64_t *final_occ, rr_solve_info *info, uint32_t flags,
                   void *workspace, size_t workspace_bytes, void *stream);

/* Bytes of device workspace rr_batch_moves needs for this shape and these capacities. */
size_t rr_batch_workspace_bytes(rr_shape shape, uint32_t move_cap, uint32_t step_cap);

/* Batch the moves of one solve (§IV, Alg. 3).
 *   moves, group_off, sinfo [in]  the outputs of rr_solve (sinfo->n_moves / n_groups are read
 *                                 on the device; a solve that did not end in RR_OK or
 *                                 RR_INFEASIBLE makes the batch status RR_E_INVAL, and so does a
 *                                 move off the grid, a move of length 0 or a malformed group_off).
 *   move_cap   [in]  capacity of `moves` (>= sinfo->n_moves), used to size the workspace.
 *   flags      [in]  bits 0..7: RR_LAMBDA_*; bits 8..15: LDS budget in KiB (1..255) for the loop
 *                    data of one instance, 0 = the library's default; bit 16: RR_BATCH_GENERIC;
 *                    bits 24..31: LDS budget in KiB for the dependency-graph build of one
 *                    instance, 0 = the library's default.  Bits 8..16 and 24..31 are tuning and
 *                    testing knobs: results do not depend on them.  The loop budget is raised
 *                    to what the loop always keeps in LDS (8 B per group and 16 B per register
 *                    position of the ready set: about 4 KiB for 64 x 64 grids); a graph budget
 *                    too small for one row of traps builds the graph in the workspace.
 *                    Bits 20..23: wavefronts per instance of the graph kernel divided by 4
 *                    (1, 2 or 4: 4, 8 or 16 wavefronts; 0 = the default, 8), another tuning
 *                    knob.  Bits 17..19 must be 0.
 *                    At most 2^20 - 1 moves in at most 1024 groups (always true for rr_solve
 *                    outputs on grids up to 256 x 256); more gives RR_E_INVAL.  Grids beyond
 *                    RR_LDS_SIDE run the wide path: at most 2^21 - 1 moves, at most W + H (and
 *                    2048) groups of at most 2048 moves each (RR_E_INVAL beyond), every flag
 *                    bit but the constraint ignored; an instance whose in-group predecessor
 *                    sets or ready set outgrow the path's fixed capacities (8 members after
 *                    pruning; 4096 ready moves, 2048 made ready at once -- rr_solve outputs
 *                    stay far below) gives RR_E_UNSUPPORTED.
 *   batch_off  [out] uint32_t[batch_cap + 1]: steps of batch k are [batch_off[k], batch_off[k+1]).
 *   steps      [out] uint32_t[step_cap]: dir << 30 | x << 15 | y, the source trap of each unit
 *                    step, dir 0 = +x, 1 = -x, 2 = +y, 3 = -y.  step_cap >= sinfo->n_steps and
 *                    batch_cap >= sinfo->n_steps always suffice.
 *   binfo      [out] one rr_batch_info.  When the summed path length exceeds step_cap the status
 *                    is RR_E_CAPACITY with need_steps exact and need_batches = need_steps (an
 *                    upper bound); when only batch_cap is short, both need_* are exact.
 *   workspace  [in]  device scratch of rr_batch_workspace_bytes(shape, move_cap, step_cap) bytes,
 *                    owned by the caller, not shared with a concurrent call. */
rr_status rr_batch_moves(rr_shape shape, const rr_move *moves, const uint32_t *group_off,
                         const rr_solve_info *sinfo, uint32_t move_cap, uint32_t flags,
                         uint32_t *batch_off, uint32_t batch_cap,
                         uint32_t *steps, uint32_t step_cap, rr_batch_info *binfo,
                         void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------------------------ */
/* Many independent instances in one launch                                                   */

/* Per-instance descriptor of a many-instance launch (device memory, one per instance, 80
 * bytes, no implicit padding).  Offsets are element counts into the arenas passed to the call:
 *   occ_off    uint64 words: the instance's input bit rows and its final bit rows (same offset
 *              in the input arena and in the final arena)
 *   move_off   rr_move elements (move_cap of them)
 *   group_off  uint32 elements (group_cap + 1 of them)
 *   step_off   uint32 elements (step_cap of them)           -- rr_batch_moves_many only
 *   batch_off  uint32 elements (batch_cap + 1 of them)      -- rr_batch_moves_many only
 *   ws_off     bytes into the batching workspace, a multiple of 256, the instance's region of
 *              rr_batch_workspace_bytes(shape, move_cap, step_cap) bytes inside the workspace
 *              and shared with no other instance -- rr_batch_moves_many only */
typedef struct {
    rr_shape shape;
    uint16_t pad0, pad1;
    uint32_t move_cap, group_cap, step_cap, batch_cap;
    uint64_t occ_off, move_off, group_off, step_off, batch_off, ws_off;
} rr_desc;

/* Solve n instances in one launch; instance i reads occ_arena + desc[i].occ_off and writes
 * moves/group offsets/final bit rows at its offsets and infos[i].  Results are bit-identical to
 * n calls of rr_solve with the same flags (the algorithm, as in rr_solve).  max_w / max_h
 * bound every instance's grid (they pick the kernel variant; an instance beyond them gets
 * RR_E_INVAL).  workspace / workspace_bytes: n * rr_solve_workspace_bytes of a grid beyond
 * RR_LDS_SIDE when max_w or max_h is beyond it (instance i uses the i-th such slice), else
 * nothing (NULL is then accepted); too little gives RR_E_NOMEM.  With max_w or max_h beyond
 * RR_LDS_SIDE the call launches two kernels, one for the instances beyond RR_LDS_SIDE, one for
 * the others; the wavefront field of flags applies to the latter and must give at least 256
 * threads. */
rr_status rr_solve_many(uint32_t n, const rr_desc *desc, uint32_t max_w, uint32_t max_h,
                        const uint64_t *occ_arena, rr_move *move_arena, uint32_t *group_arena,
                        uint64_t *final_arena, rr_solve_info *infos, uint32_t flags,
                        void *workspace, size_t workspace_bytes, void *stream);

/* Batch the moves of n solved instances in one launch (same semantics and flags as
 * rr_batch_moves; the LDS budget in flags bits 8..15 applies to every instance).
 * workspace_bytes is the size of `workspace`: an instance whose region (ws_off and
 * rr_batch_workspace_bytes of its shape and capacities) is misaligned or runs past it gets
 * status RR_E_INVAL in binfos[i], and nothing of that instance is written, workspace
 * included. */
rr_status rr_batch_moves_many(uint32_t n, const rr_desc *desc, uint32_t max_w, uint32_t max_h,
                              const rr_move *move_arena, const uint32_t *group_arena,
                              const rr_solve_info *sinfos, uint32_t flags,
                              uint32_t *batch_arena, uint32_t *step_arena, rr_batch_info *binfos,
                              void *workspace, size_t workspace_bytes, void *stream);

/* rr_batch_moves_many with its stages marked for profiling: when non-NULL, graph_done_event and
 * loop_done_event (hipEvent_t, created by the caller) are recorded on `stream` after the graph
 * kernel (validation and dependency graph of every instance) and after the loop kernel (Alg. 3
 * on the fast path), so that elapsed times between them give each stage's device time.  The
 * general-path kernel runs after loop_done_event.  Results are those of rr_batch_moves_many;
 * a failed event record returns RR_E_DEVICE. */
rr_status rr_batch_moves_many_staged(uint32_t n, const rr_desc *desc, uint32_t max_w, uint32_t max_h,
                                     const rr_move *move_arena, const uint32_t *group_arena,
                                     const rr_solve_info *sinfos, uint32_t flags,
                                     uint32_t *batch_arena, uint32_t *step_arena, rr_batch_info *binfos,
                                     void *workspace, size_t workspace_bytes, void *stream,
                                     void *graph_done_event, void *loop_done_event);

/* Lay out the batching arenas of n solved instances on the device, with no host round trip: an
 * exclusive scan over the instances, in order, gives instance i step_cap = batch_cap =
 * max(1, infos[i].n_steps) (exact for an RR_OK solve) and its step_off, batch_off and ws_off in
 * pools of step_pool uint32 steps, batch_pool uint32 batch offsets and ws_pool_bytes bytes.  An
 * instance that does not fit gets step_cap = 0xFFFFFFFF: rr_batch_moves_many then reports
 * RR_E_CAPACITY for it (need_steps = its step count) and writes nothing else for it.
 * totals (device, 3 x uint64_t, may be NULL) receives the pool sizes all n instances need.
 * desc is updated in place (shape, move_cap, group_cap and the solve offsets are kept). */
rr_status rr_plan_many(uint32_t n, rr_desc *desc, const rr_solve_info *infos, uint64_t step_pool,
                       uint64_t batch_pool, uint64_t ws_pool_bytes, uint64_t *totals, void *stream);

/* ------------------------------------------------------------------------------------------ */
/* Exact 1D on chains                                                                           */

/* Longest chain rr_solve_chains takes (move coordinates are 16-bit). */
#define RR_MAX_CHAIN 65535u

/* Bytes of device workspace rr_solve_chains needs for n chains of at most max_len traps: 0 up
 * to 8192 traps (token positions stay in LDS), else n * 8 * (max_len + 2). */
size_t rr_solve_chains_workspace_bytes(uint32_t n, uint32_t max_len);

/* Exact 1D on n independent chains of traps in one launch (§III.A: distance-minimising
 * assignment of tokens to a contiguous target and moves along the chain; its parallel form,
 * §III.B).  A chain is a 1 x N grid: desc[i].shape = {N, 1, b, 0, b + t, 1} with 1 <= N <=
 * max_len <= RR_MAX_CHAIN and target [b, b+t); its bit row, moves, group offsets (one group, or
 * none when nothing moves) and final bit row go to the arenas at desc[i]'s offsets as in
 * rr_solve_many.  A chain with fewer tokens than targets gives RR_INFEASIBLE (no move, final =
 * input); a malformed shape gives RR_E_INVAL in infos[i].  The matching is the cheapest run of
 * t consecutive tokens onto [b, b+t) (ties: the leftmost run); moves towards larger positions
 * come first, largest target first, then the others, smallest target first.  For N up to
 * RR_MAX_SIDE the results are byte for byte those of rr_solve on the same 1 x N grid.
 * move_cap >= t always suffices.  workspace: rr_solve_chains_workspace_bytes(n, max_len) bytes
 * (NULL when that is 0). */
rr_status rr_solve_chains(uint32_t n, const rr_desc *desc, uint32_t max_len, const uint64_t *occ_arena,
                          rr_move *move_arena, uint32_t *group_arena, uint64_t *final_arena,
                          rr_solve_info *infos, void *workspace, size_t workspace_bytes, void *stream);

/* ------------------------------------------------------------------------------------------ */
/* Batching with no allocation                                                                 */

/* Size of the library's own batching workspace: one file-scope device array per GPU, held from
 * the library's load until the process ends. */
#define RR_NOALLOC_WORKSPACE_BYTES (64u << 20)

/* rr_batch_moves for callers that cannot allocate device memory (code under stream or graph
 * capture, serving loops that must not call the allocator, harnesses that forbid it): same
 * arguments, semantics and results, but the workspace is the library's array on the current
 * device instead of a caller buffer.  The call itself allocates and frees nothing.
 *   - Returns RR_E_NOMEM, before touching the device, when
 *     rr_batch_workspace_bytes(shape, move_cap, step_cap) exceeds RR_NOALLOC_WORKSPACE_BYTES
 *     (every grid up to 256 x 256 with move_cap = 2*(x1-x0)*(y1-y0) fits for step_cap up to
 *     3 million); RR_E_DEVICE when the array's device address cannot be obtained.
 *   - The first call on a device looks up the array's address on that device (once per
 *     device, with that device current); later calls make no device query.
 *   - Every call on one device shares that device's array, which keeps the last call's
 *     contents (the kernels initialise whatever they read).  Calls that overlap on one device
 *     race: serialise them (one stream, or events between streams). */
rr_status rr_batch_moves_noalloc(rr_shape shape, const rr_move *moves, const uint32_t *group_off,
                                 const rr_solve_info *sinfo, uint32_t move_cap, uint32_t flags,
                                 uint32_t *batch_off, uint32_t batch_cap,
                                 uint32_t *steps, uint32_t step_cap, rr_batch_info *binfo, void *stream);

/* Library version string (host). */
const char *rr_version(void);

#ifdef __cplusplus
}
#endif
#endif /* RR_H */
