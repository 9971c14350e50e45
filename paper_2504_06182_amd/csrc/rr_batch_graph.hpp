// rr_batch_graph.hpp -- dependency graph of the batching routine (arXiv 2504.06182, §IV) for the
// fast path: one 512-thread workgroup per instance.
//
// Gamma (§IV): within a group, move a precedes move b (a < b) when their paths share a trap;
// across groups, every move of an earlier group precedes every move of a later group when the
// two groups share a trap.  Any two moves that touch a common trap are therefore ordered, so
// the moves touching one trap finish in index order and readiness only depends on the previous
// toucher of each trap (the reduction the loop kernel runs on):
//   * in-group predecessors of b: the previous toucher of each trap of b, when it is in b's
//     group (kept once per distinct move);
//   * group predecessors of group h: the group of the previous toucher of each trap of each
//     move of h, when it is another group (kept once per distinct group).
//
// Construction, all by counting: per-trap toucher counts (atomics) -> exclusive scan ->
// scatter of move indices -> each trap's list sorted by index -> each move walks its path and
// looks itself up in every list it is on to find its previous toucher.  The per-trap arrays
// live in LDS when they fit the launch's budget; larger grids are built in LDS tiles of whole
// rows (graph_tiled, which scans the unsorted lists instead: there they are long and uneven);
// a row too large for the budget falls back to the workspace.
//
// Output (workspace, read by the loop kernel): for every move its packed coordinates and a
// 16-bit release code (no successor / exactly one successor that waits on nothing else / a
// list), successor lists and wait counts for the general case, and per group its number of
// group predecessors, the groups waiting on it and its head moves (no in-group predecessor).
// The header also carries a bound on the size of the ready set: the head moves of all groups
// plus one per extra successor of a move.  It is loose (groups become ready one after another),
// so the loop does not use it: it keeps ready sets of up to 64*S moves in registers and hands
// an instance to the general path only when its ready set actually grows past that.
#pragma once
#include "rr_device.hpp"
#include "rr.h"
#include "rr_batch_generic.hpp"

namespace rr {
namespace fast {

constexpr uint32_t kMaxK = 65535;       // move indices fit 16 bits on the fast path
constexpr int kMaxPreds = 8;            // distinct in-group predecessors of one move
constexpr int kGT = 512;                // default threads of the graph workgroup (8 waves)

// release code of a move (16 bits): kind << 14 | next - b
constexpr uint32_t kRelNone = 0, kRelNext = 1, kRelList = 2;
constexpr uint32_t kMaxDelta = (1u << 14) - 1;

// header words
enum { H_STATE = 0, H_K, H_G, H_T, H_E, H_GE, H_HN, H_BOUND, H_NWORDS = 16 };
// H_STATE: what the next kernel does with the instance
enum { ST_FAST = 0, ST_DONE = 1, ST_GENERIC = 2 };

struct Layout {
    size_t hdr, mv, nx, gpend, gloff, hdoff, hd, gl, soff, sfill, slist, pend, preds, gbits, gcnt, hcnt, grp, cell,
        touch, gen, total;
    uint32_t Gc, GW;
    size_t GEc;
};

__host__ __device__ inline size_t al256(size_t v) { return (v + 255) & ~(size_t)255; }

// groups the fast path takes: at most W + H (every rr_solve output), 1024 and the move count
__host__ __device__ inline uint32_t fast_group_cap(int W, int H, uint32_t move_cap)
{
    uint32_t g = (uint32_t)(W + H);
    if (g > 1024u) g = 1024u;
    if (g > move_cap) g = move_cap;
    return g < 1u ? 1u : g;
}

__host__ __device__ inline Layout layout(int W, int H, uint32_t move_cap, uint32_t step_cap)
{
    Layout L;
    const size_t K = (size_t)move_cap + 1, WH = (size_t)W * H, OCC = (size_t)move_cap + step_cap + 1;
    L.Gc = fast_group_cap(W, H, move_cap);
    L.GW = (L.Gc + 31) / 32;
    L.GEc = (size_t)L.Gc * L.Gc < OCC ? (size_t)L.Gc * L.Gc : OCC;
    size_t p = 0;
    auto take = [&](size_t bytes) { const size_t at = p; p = al256(p + bytes); return at; };
    L.hdr = take(4 * H_NWORDS);
    L.mv = take(4 * K);
    L.nx = take(2 * K);
    L.gpend = take(2 * (size_t)L.Gc);
    L.gloff = take(2 * ((size_t)L.Gc + 1));
    L.hdoff = take(2 * ((size_t)L.Gc + 1));
    L.hd = take(2 * K);
    L.gl = take(2 * L.GEc);
    L.soff = take(4 * (K + 1));
    L.sfill = take(4 * K);
    L.slist = take(4 * kMaxPreds * K);
    L.pend = take(4 * K);
    L.preds = take(2 * kMaxPreds * K);
    L.gbits = take(4 * (size_t)L.Gc * L.GW);
    L.gcnt = take(4 * ((size_t)L.Gc + 1));
    L.hcnt = take(4 * ((size_t)L.Gc + 1));
    L.grp = take(2 * K);
    L.cell = take(4 * (WH + 1));
    L.touch = take(2 * OCC);
    // the general path's region overlaps the fast path's arrays: it redoes an instance from its
    // inputs, after the fast path has given it up, and needs nothing the fast path built; only
    // the header (which holds the instance's state) stays apart
    L.gen = L.mv;
    const size_t gen_end = L.gen + al256(gen::ws_layout(W, H, move_cap, step_cap).total);
    L.total = p > gen_end ? p : gen_end;
    return L;
}

// One instance of a batching call.
struct Inst {
    int W, H;
    const rr_move *moves;
    const uint32_t *goff;
    const rr_solve_info *sinfo;
    uint32_t move_cap, step_cap, batch_cap;
    uint32_t *boff, *steps;
    rr_batch_info *binfo;
    uint8_t *ws;
};

__device__ __forceinline__ void put_info(rr_batch_info *bi, int status, uint32_t nb, uint32_t ns, uint32_t needb,
                                         uint32_t needs)
{
    rr_batch_info v;
    v.status = status; v.n_batches = nb; v.n_steps = ns; v.need_batches = needb; v.need_steps = needs;
    *bi = v;
}

__device__ __forceinline__ void load_move(const rr_move *mv, uint32_t b, int &sx, int &sy, int &dx, int &dy)
{
    const uint64_t v = reinterpret_cast<const uint64_t *>(mv)[b];
    sx = (int)(v & 0xFFFF); sy = (int)((v >> 16) & 0xFFFF); dx = (int)((v >> 32) & 0xFFFF); dy = (int)(v >> 48);
}

__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }

// trap s (0..len) of the path: along row sy to column dx, then along column dx
__device__ __forceinline__ int path_trap(int W, int sx, int sy, int dx, int dy, int s)
{
    const int hx = iabs(dx - sx);
    if (s <= hx) return sy * W + (dx >= sx ? sx + s : sx - s);
    const int v = s - hx;
    return (dy >= sy ? sy + v : sy - v) * W + dx;
}

template <int NW>
struct GraphShared {
    uint32_t part[NW];
    uint32_t red[NW];
    uint32_t flags;
    uint32_t nr;            // row ranges of the tiled build
    uint32_t nlong;         // long horizontal legs of the current range, searched wave by wave
    uint32_t nedge;         // one-piece build: in-group edges appended so far
    uint16_t longq[512];
};

constexpr uint32_t kSortLo = 32;        // tiled build: lists longer than this (up to 128) are sorted
constexpr int kLongLeg = 32;            // horizontal legs longer than this: one wave each
constexpr uint32_t kLongCap = 512;

__device__ __forceinline__ uint32_t add_wg32(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// workgroup sum of one value per thread (all threads get the total)
template <int NT>
__device__ __forceinline__ uint32_t block_sum(uint32_t v, GraphShared<NT / kWave> &S)
{
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    v = (uint32_t)wave_sum((int)v);
    if (lane == 0) S.red[wid] = v;
    __syncthreads();
    uint32_t t = 0;
#pragma unroll
    for (int w = 0; w < (NT / kWave); ++w) t += S.red[w];
    __syncthreads();
    return t;
}

// exclusive scan of a[0..n) in place, a[n] = total (a: LDS or global, visible to the workgroup);
// kIncl gives a[i] = a[0] + ... + a[i] instead (the end of entry i's range)
template <int NT, bool kIncl = false>
__device__ __forceinline__ void block_scan(uint32_t *a, uint32_t n, GraphShared<NT / kWave> &S)
{
    const int tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
    uint32_t carry = 0;
    for (uint32_t base = 0; base <= n; base += NT) {
        const uint32_t i = base + tid;
        const uint32_t v = i < n ? a[i] : 0u;
        const uint32_t inc = (uint32_t)wave_incl_scan((int)v);
        if (lane == kWave - 1) S.part[wid] = inc;
        __syncthreads();
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (int w = 0; w < (NT / kWave); ++w) {
            const uint32_t pw = S.part[w];
            pre += w < wid ? pw : 0u;
            tot += pw;
        }
        if (i <= n) a[i] = carry + pre + inc - (kIncl ? 0u : v);
        carry += tot;
        __syncthreads();
    }
}

// sort a[0..n) ascending (n <= N), one thread: a bitonic network over N registers
template <int N>
__device__ __forceinline__ void sort_regs(uint16_t *a, int n)
{
    uint32_t r[N];
#pragma unroll
    for (int i = 0; i < N; ++i) r[i] = i < n ? (uint32_t)a[i] : 0xFFFFFFFFu;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1)
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
            for (int i = 0; i < N; ++i) {
                const int l = i ^ j;
                if (l > i) {
                    const bool up = (i & k) == 0;
                    const uint32_t lo = r[i] < r[l] ? r[i] : r[l], hi = r[i] < r[l] ? r[l] : r[i];
                    r[i] = up ? lo : hi;
                    r[l] = up ? hi : lo;
                }
            }
#pragma unroll
    for (int i = 0; i < N; ++i)
        if (i < n) a[i] = (uint16_t)r[i];
}

// sort a[0..n) ascending (distinct 16-bit values), one thread: in registers up to 16 entries,
// by insertion beyond (a 32-entry network doubles the graph kernels' registers)
__device__ __forceinline__ void sort_list(uint16_t *a, int n)
{
    if (n <= 1) return;
    if (n <= 16) { sort_regs<16>(a, n); return; }
    for (int k = 1; k < n; ++k) {
        const uint16_t v = a[k];
        int m = k;
        while (m > 0 && a[m - 1] > v) { a[m] = a[m - 1]; --m; }
        a[m] = v;
    }
}

// packed coordinates sx | sy << 8 | dx << 16 | dy << 24 of move b
__device__ __forceinline__ uint32_t packed_move(const rr_move *mv, uint32_t b)
{
    int sx, sy, dx, dy;
    load_move(mv, b, sx, sy, dx, dy);
    return (uint32_t)sx | ((uint32_t)sy << 8) | ((uint32_t)dx << 16) | ((uint32_t)dy << 24);
}

__device__ __forceinline__ bool spans(int v, int a, int b) { return a <= b ? (a <= v && v <= b) : (b <= v && v <= a); }

__device__ __forceinline__ bool overlap(int a1, int b1, int a2, int b2)
{
    const int lo1 = a1 < b1 ? a1 : b1, hi1 = a1 < b1 ? b1 : a1, lo2 = a2 < b2 ? a2 : b2, hi2 = a2 < b2 ? b2 : a2;
    return (lo1 > lo2 ? lo1 : lo2) <= (hi1 < hi2 ? hi1 : hi2);
}

// Do the paths of two moves (packed coordinates) share a trap?  A path runs along row sy from sx
// to dx, then along column dx from sy to dy, endpoints included.
__device__ __forceinline__ bool paths_meet(uint32_t p, uint32_t q)
{
    const int psx = p & 0xFF, psy = (p >> 8) & 0xFF, pdx = (p >> 16) & 0xFF, pdy = p >> 24;
    const int qsx = q & 0xFF, qsy = (q >> 8) & 0xFF, qdx = (q >> 16) & 0xFF, qdy = q >> 24;
    const bool hh = psy == qsy && overlap(psx, pdx, qsx, qdx);
    const bool hv = spans(qdx, psx, pdx) && spans(psy, qsy, qdy);     // p's row leg, q's column leg
    const bool vh = spans(pdx, qsx, qdx) && spans(qsy, psy, pdy);     // p's column leg, q's row leg
    const bool vv = pdx == qdx && overlap(psy, pdy, qsy, qdy);
    return hh || hv || vh || vv;
}

// Add in-group predecessor v to the set s[0..n) of one move, keeping the set free of redundant
// members: two moves of one group whose paths meet are joined by an edge of the dependency
// graph (the earlier precedes the later), so of two members whose paths meet the earlier is an
// ancestor of the later and adds nothing to the move's readiness.  Such earlier members are
// dropped (v too, when a later member meets it); readiness, hence every batch, is unchanged.
// Sets ovf when a needed member does not fit.  pc[] holds the members' packed coordinates, 0
// while not read yet (a move is never all zero): they are read only once a set has a member,
// so the usual sets of zero or one (red-rec's) cost no extra reads.  Returns whether the set
// changed.
__device__ __forceinline__ bool pred_add(uint32_t (&s)[kMaxPreds], uint32_t (&pc)[kMaxPreds], int &n, uint32_t v,
                                         const rr_move *mv, bool &ovf)
{
    bool have = false;
#pragma unroll
    for (int i = 0; i < kMaxPreds; ++i) have |= (i < n) && s[i] == v;
    if (have) return false;
    if (n == 0) {
        s[0] = v;
        pc[0] = 0u;
        n = 1;
        return true;
    }
    const uint32_t vc = packed_move(mv, v);
    bool redundant = false;
    uint32_t ks[kMaxPreds], kc[kMaxPreds];
    int m = 0;
#pragma unroll
    for (int i = 0; i < kMaxPreds; ++i) {
        ks[i] = 0; kc[i] = 0;
        if (i >= n) continue;
        if (pc[i] == 0u) pc[i] = packed_move(mv, s[i]);
        const bool meet = paths_meet(pc[i], vc);
        redundant |= meet && s[i] > v;
        const bool keep = !(meet && s[i] < v);
#pragma unroll
        for (int j = 0; j < kMaxPreds; ++j)
            if (keep && j == m) { ks[j] = s[i]; kc[j] = pc[i]; }
        m += keep ? 1 : 0;
    }
    if (!redundant) {
        if (m == kMaxPreds) { ovf = true; return false; }
#pragma unroll
        for (int j = 0; j < kMaxPreds; ++j)
            if (j == m) { ks[j] = v; kc[j] = vc; }
        ++m;
    }
#pragma unroll
    for (int i = 0; i < kMaxPreds; ++i) { s[i] = ks[i]; pc[i] = kc[i]; }
    n = m;
    return true;
}

template <int NT, bool kEdges>
__device__ __forceinline__ void graph_tail(const Inst &I, GraphShared<NT / kWave> &S, const Layout &L, uint32_t K, uint32_t G,
                                          uint32_t T, uint32_t *cnt, uint32_t *gt);

// The graph of one instance from its validated moves; cell (W*H + 1 words), grp (K) and touch
// (K + T) are the per-trap scratch arrays; cnt (K + 1 words, LDS or the workspace's successor
// offsets) takes the successor counts once the per-trap arrays are no longer needed, and may
// overlap them; so may gt (G * GW words of LDS, or null), the transposed group bit matrix.
template <int NT>
__device__ __forceinline__ void graph_core(const Inst &I, GraphShared<NT / kWave> &S, const Layout &L, uint32_t K, uint32_t G,
                                           uint32_t T, uint32_t *cell, uint16_t *grp, uint16_t *touch, uint32_t *cnt,
                                           uint32_t *gt)
{
    const int tid = threadIdx.x;
    const int W = I.W, H = I.H;
    const uint32_t WH = (uint32_t)(W * H);
    uint32_t *hdr = (uint32_t *)(I.ws + L.hdr);
    uint32_t *mv32 = (uint32_t *)(I.ws + L.mv);
    uint16_t *nx = (uint16_t *)(I.ws + L.nx);
    uint32_t *pend = (uint32_t *)(I.ws + L.pend);
    uint16_t *preds = (uint16_t *)(I.ws + L.preds);
    uint32_t *gbits = (uint32_t *)(I.ws + L.gbits);
    const uint32_t GW = L.GW;

    for (uint32_t g = tid; g < G; g += NT)
        for (uint32_t b = I.goff[g]; b < I.goff[g + 1]; ++b) grp[b] = (uint16_t)g;
    for (uint32_t b = tid; b < K; b += NT) {
        int sx, sy, dx, dy;
        load_move(I.moves, b, sx, sy, dx, dy);
        mv32[b] = (uint32_t)sx | ((uint32_t)sy << 8) | ((uint32_t)dx << 16) | ((uint32_t)dy << 24);
    }
    for (uint32_t c = tid; c <= WH; c += NT) cell[c] = 0;
    for (uint32_t i = tid; i < G * GW; i += NT) gbits[i] = 0;
    if (tid == 0) { S.flags = 0; S.nedge = 0; }
    __syncthreads();

    // ---- touch lists: count, scan, scatter (post-increment: afterwards trap c's list is
    //      [c ? cell[c-1] : 0, cell[c]))
    for (uint32_t b = tid; b < K; b += NT) {
        int sx, sy, dx, dy;
        load_move(I.moves, b, sx, sy, dx, dy);
        const int len = iabs(dx - sx) + iabs(dy - sy);
        for (int s = 0; s <= len; ++s) add_wg32(&cell[path_trap(W, sx, sy, dx, dy, s)], 1u);
    }
    __syncthreads();
    block_scan<NT>(cell, WH, S);
    for (uint32_t b = tid; b < K; b += NT) {
        int sx, sy, dx, dy;
        load_move(I.moves, b, sx, sy, dx, dy);
        const int len = iabs(dx - sx) + iabs(dy - sy);
        for (int s = 0; s <= len; ++s) {
            const uint32_t at = add_wg32(&cell[path_trap(W, sx, sy, dx, dy, s)], 1u);
            touch[at] = (uint16_t)b;
        }
    }
    __syncthreads();
    // traps in column-major order: the long lists gather in a few columns (the receivers'), and
    //   a stride of NT in row-major order would give each thread traps of one column only
    for (uint32_t i = tid; i < WH; i += NT) {
        const uint32_t x = i / (uint32_t)H, c = (i - x * (uint32_t)H) * (uint32_t)W + x;
        const uint32_t lo = c ? cell[c - 1] : 0u;
        sort_list(touch + lo, (int)(cell[c] - lo));
    }
    __syncthreads();

    // ---- previous toucher of every trap of every move.  The in-group edges (a -> b) go to a
    //      packed list (a | b << 16, in the region of the per-move predecessor slots, which
    //      holds 4 * kMaxPreds 16-bit words per move, i.e. 4 edges per move on average): each wave
    //      reserves its edges' places with one LDS atomic and places them by ballot prefix counts.
    uint32_t *edge = (uint32_t *)preds;
    const uint32_t ecap = 4u * K;
    const int lane = lane_id();
    for (uint32_t b = tid; b < K; b += NT) {
        int sx, sy, dx, dy;
        load_move(I.moves, b, sx, sy, dx, dy);
        const int len = iabs(dx - sx) + iabs(dy - sy);
        const uint32_t g = grp[b];
        uint32_t ps[kMaxPreds], pc[kMaxPreds];
        int np = 0;
        bool ovf = false;
        uint32_t last = 0xFFFFFFFFu, lastg = 0xFFFFFFFFu;
        for (int s = 0; s <= len; ++s) {
            const uint32_t c = (uint32_t)path_trap(W, sx, sy, dx, dy, s);
            uint32_t lo = c ? cell[c - 1] : 0u, hi = cell[c];
            if (touch[lo] == b) continue;             // first toucher of this trap
            while (hi - lo > 1) {                     // largest position with touch[pos] < b
                const uint32_t mid = (lo + hi) >> 1;
                if (touch[mid] < b) lo = mid; else hi = mid;
            }
            const uint32_t a = touch[lo];
            if (a == last) continue;
            last = a;
            const uint32_t ga = grp[a];
            if (ga == g) {
                pred_add(ps, pc, np, a, I.moves, ovf);
            } else if (ga != lastg) {        // a group predecessor: the bit matrix keeps it once
                lastg = ga;
                __hip_atomic_fetch_or(&gbits[g * GW + ga / 32], 1u << (ga & 31), __ATOMIC_RELAXED,
                                      __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
        pend[b] = (uint32_t)np;
        // place of this move's first edge: prefix of np over the wave's active lanes (np <= 8
        // takes four bits), the wave's block from one LDS atomic of its first active lane
        const uint64_t below = low_mask(lane);
        uint32_t pre = 0, tot = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const uint64_t m = ballot(((uint32_t)np >> k) & 1u);
            pre += (uint32_t)popc(m & below) << k;
            tot += (uint32_t)popc(m) << k;
        }
        const int leader = __builtin_ctzll(ballot(true));
        uint32_t base = 0;
        if (lane == leader) base = add_wg32(&S.nedge, tot);
        base = (uint32_t)__builtin_amdgcn_readlane((int)base, leader) + pre;
#pragma unroll
        for (int i = 0; i < kMaxPreds; ++i)
            if (i < np && base + (uint32_t)i < ecap) edge[base + (uint32_t)i] = ps[i] | (b << 16);
        if (ovf) S.flags = 1;
    }
    __syncthreads();
    if (S.flags || S.nedge > ecap) {
        if (tid == 0) hdr[H_STATE] = ST_GENERIC;
        return;
    }
    graph_tail<NT, true>(I, S, L, K, G, T, cnt, gt);
}

// Second half of the graph build, from the in-group predecessor sets (pend, and either preds as
// per-move slots with their successor counts in soff, or, with kEdges, the packed edge list of
// S.nedge entries in the same region, counted here into cnt) and the group bit matrix (gbits),
// all in the workspace: successor lists, release codes, heads, group lists and the header.
// gt (G * GW words of LDS, or null) takes the group bit matrix transposed: row g then holds the
// groups waiting on g, read as a row instead of a column of the workspace matrix.
template <int NT, bool kEdges>
__device__ __forceinline__ void graph_tail(const Inst &I, GraphShared<NT / kWave> &S, const Layout &L, uint32_t K, uint32_t G,
                                          uint32_t T, uint32_t *cnt, uint32_t *gt)
{
    const int tid = threadIdx.x;
    uint32_t *hdr = (uint32_t *)(I.ws + L.hdr);
    uint16_t *nx = (uint16_t *)(I.ws + L.nx);
    uint32_t *soff = (uint32_t *)(I.ws + L.soff), *sfill = (uint32_t *)(I.ws + L.sfill);
    uint32_t *slist = (uint32_t *)(I.ws + L.slist), *pend = (uint32_t *)(I.ws + L.pend);
    uint16_t *preds = (uint16_t *)(I.ws + L.preds);
    uint32_t *gbits = (uint32_t *)(I.ws + L.gbits), *gcnt = (uint32_t *)(I.ws + L.gcnt), *hcnt = (uint32_t *)(I.ws + L.hcnt);
    const uint32_t GW = L.GW;

    // ---- successor lists (CSR) and release codes
    if (kEdges) {
        // successor counts from the edges, an inclusive scan, then cnt[a] counts down from the
        // end of a's range to its start as the list fills (the order within a list is free: the
        // loop inserts released moves by index); a copy in LDS goes to soff at the end
        const uint32_t *edge = (const uint32_t *)preds, E = S.nedge;
        for (uint32_t b = tid; b <= K; b += NT) cnt[b] = 0;
        __syncthreads();
        for (uint32_t e = tid; e < E; e += NT) add_wg32(&cnt[edge[e] & 0xFFFFu], 1u);
        __syncthreads();
        block_scan<NT, true>(cnt, K, S);
        for (uint32_t e = tid; e < E; e += NT) {
            const uint32_t v = edge[e];
            slist[add_wg32(&cnt[v & 0xFFFFu], 0xFFFFFFFFu) - 1u] = v >> 16;
        }
        __syncthreads();
        if (cnt != soff)
            for (uint32_t b = tid; b <= K; b += NT) soff[b] = cnt[b];
    } else {
        cnt = soff;
        block_scan<NT>(soff, K, S);
        for (uint32_t b = tid; b < K; b += NT) {
            const uint32_t np = pend[b];
            for (uint32_t i = 0; i < np; ++i) {
                const uint32_t a = preds[(size_t)b * kMaxPreds + i];
                slist[soff[a] + add_wg32(&sfill[a], 1u)] = b;
            }
        }
    }
    __syncthreads();
    uint32_t extra = 0;
    for (uint32_t a = tid; a < K; a += NT) {
        const uint32_t lo = cnt[a], ns = cnt[a + 1] - lo;
        uint32_t code = kRelNone << 14;
        if (ns == 1) {
            const uint32_t n = slist[lo];
            code = (pend[n] == 1u && n - a <= kMaxDelta) ? ((kRelNext << 14) | (n - a)) : (kRelList << 14);
        } else if (ns > 1) {
            code = kRelList << 14;
            extra += ns - 1;
        }
        nx[a] = (uint16_t)code;
    }
    extra = block_sum<NT>(extra, S);

    // ---- heads of every group, and the groups waiting on every group
    if (gt) {          // row h of gbits has bit a set when group a precedes group h
        for (uint32_t i = tid; i < G * GW; i += NT) gt[i] = 0;
        __syncthreads();
        for (uint32_t i = tid; i < G * GW; i += NT) {
            const uint32_t h = i / GW, a0 = (i - h * GW) * 32u;
            for (uint32_t m = gbits[i]; m; m &= m - 1u)
                __hip_atomic_fetch_or(&gt[(a0 + (uint32_t)__builtin_ctz(m)) * GW + h / 32], 1u << (h & 31),
                                      __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        }
        __syncthreads();
    }
    uint16_t *gpend = (uint16_t *)(I.ws + L.gpend), *gloff = (uint16_t *)(I.ws + L.gloff);
    uint16_t *hdoff = (uint16_t *)(I.ws + L.hdoff), *hd = (uint16_t *)(I.ws + L.hd), *gl = (uint16_t *)(I.ws + L.gl);
    for (uint32_t g = tid; g < G; g += NT) {
        uint32_t c = 0;
        for (uint32_t b = I.goff[g]; b < I.goff[g + 1]; ++b) c += pend[b] == 0u;
        hcnt[g] = c;
        uint32_t np = 0, nw = 0;
        for (uint32_t w = 0; w < GW; ++w) np += (uint32_t)__popc(gbits[g * GW + w]);
        if (gt)
            for (uint32_t w = 0; w < GW; ++w) nw += (uint32_t)__popc(gt[g * GW + w]);
        else
            for (uint32_t h = 0; h < G; ++h) nw += (gbits[h * GW + g / 32] >> (g & 31)) & 1u;
        gpend[g] = (uint16_t)np;
        gcnt[g] = nw;
    }
    __syncthreads();
    block_scan<NT>(hcnt, G, S);
    block_scan<NT>(gcnt, G, S);
    for (uint32_t g = tid; g <= G; g += NT) {
        hdoff[g] = (uint16_t)hcnt[g];
        gloff[g] = (uint16_t)gcnt[g];
        if (g == G) continue;
        uint32_t o = hcnt[g];
        for (uint32_t b = I.goff[g]; b < I.goff[g + 1]; ++b)
            if (pend[b] == 0u) hd[o++] = (uint16_t)b;
        o = gcnt[g];
        if (gt) {
            for (uint32_t w = 0; w < GW; ++w)
                for (uint32_t m = gt[g * GW + w]; m; m &= m - 1u) gl[o++] = (uint16_t)(w * 32u + (uint32_t)__builtin_ctz(m));
        } else {
            for (uint32_t h = 0; h < G; ++h)
                if ((gbits[h * GW + g / 32] >> (g & 31)) & 1u) gl[o++] = (uint16_t)h;
        }
    }
    if (tid == 0) {
        const uint32_t HN = hcnt[G], GE = gcnt[G];
        hdr[H_K] = K; hdr[H_G] = G; hdr[H_T] = T; hdr[H_E] = cnt[K]; hdr[H_GE] = GE; hdr[H_HN] = HN;
        hdr[H_BOUND] = HN + extra;
        hdr[H_STATE] = (HN > 65535u || GE > 65535u) ? ST_GENERIC : ST_FAST;
    }
}

// Visit the traps of the path (sx, sy) -> (dx, sy) -> (dx, dy) that lie in rows [y0, y1):
// f(c) for each trap index c = y * W + x, the horizontal leg first.
template <class F>
__device__ __forceinline__ void walk_rows(int W, int sx, int sy, int dx, int dy, int y0, int y1, F &&f)
{
    if (sy >= y0 && sy < y1) {
        const int hx = iabs(dx - sx), st = dx >= sx ? 1 : -1;
        int c = sy * W + sx;
        for (int s = 0; s <= hx; ++s, c += st) f(c);
    }
    const int vy = iabs(dy - sy);
    if (vy) {
        int lo, hi;                             // steps v (1..vy) of the vertical leg inside the rows
        if (dy > sy) { lo = max(1, y0 - sy); hi = min(vy, y1 - 1 - sy); }
        else { lo = max(1, sy - y1 + 1); hi = min(vy, sy - y0); }
        const int st = dy > sy ? W : -W;
        int c = (dy > sy ? sy + lo : sy - lo) * W + dx;
        for (int v = lo; v <= hi; ++v, c += st) f(c);
    }
}

// Tiled build, for instances whose per-trap arrays exceed the LDS budget: the grid is cut into
// ranges of whole rows whose trap counts, offsets and touch lists fit in LDS together; each
// range runs count -> scan -> scatter -> previous touchers for the moves whose path
// crosses it (per-range move lists, built first), and every move's in-group predecessor set
// accumulates in the workspace over the ranges it crosses.  Same results as the one-piece
// build.  Returns false, having changed nothing the workspace build does not redo, when a
// single row does not fit.
template <int NT>
__device__ __forceinline__ bool graph_tiled(const Inst &I, GraphShared<NT / kWave> &S, const Layout &L, uint32_t K, uint32_t G,
                                            uint32_t T, uint8_t *lds, uint32_t lds_bytes)
{
    const int tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
    const int W = I.W, H = I.H;
    uint32_t *hdr = (uint32_t *)(I.ws + L.hdr);
    uint32_t *mv32 = (uint32_t *)(I.ws + L.mv);
    uint32_t *soff = (uint32_t *)(I.ws + L.soff), *sfill = (uint32_t *)(I.ws + L.sfill);
    uint32_t *pend = (uint32_t *)(I.ws + L.pend);
    uint16_t *preds = (uint16_t *)(I.ws + L.preds);
    uint32_t *gbits = (uint32_t *)(I.ws + L.gbits);
    uint16_t *grp = (uint16_t *)(I.ws + L.grp);
    uint16_t *rlist = (uint16_t *)(I.ws + L.touch);        // per-range move lists (at most K + T entries)
    const uint32_t GW = L.GW;

    // LDS: rowc (H + 1 words: row visit counts, then their inclusive prefix), rs (H + 1: first
    // row of each range), roff (H + 1: move-list offsets), rrow (H halves: range of each row),
    // then the tile: a range's cell offsets (4 B per trap + 4) and touch lists (2 B per visit)
    const size_t fixed = al256(12 * ((size_t)H + 1) + 2 * (size_t)H);
    if (fixed + 1024 > lds_bytes) return false;
    uint32_t *rowc = (uint32_t *)lds, *rs = rowc + (H + 1), *roff = rs + (H + 1);
    uint16_t *rrow = (uint16_t *)(roff + (H + 1));
    uint8_t *tile = lds + fixed;
    const uint32_t tile_bytes = lds_bytes - (uint32_t)fixed;

    // ---- set-up; visits per row through a difference array
    for (uint32_t g = tid; g < G; g += NT)
        for (uint32_t b = I.goff[g]; b < I.goff[g + 1]; ++b) grp[b] = (uint16_t)g;
    for (uint32_t b = tid; b < K; b += NT) {
        int sx, sy, dx, dy;
        load_move(I.moves, b, sx, sy, dx, dy);
        mv32[b] = (uint32_t)sx | ((uint32_t)sy << 8) | ((uint32_t)dx << 16) | ((uint32_t)dy << 24);
        sfill[b] = 0;
        pend[b] = 0;
    }
    for (uint32_t b = tid; b <= K; b += NT) soff[b] = 0;
    for (uint32_t i = tid; i < G * GW; i += NT) gbits[i] = 0;
    for (int y = tid; y <= H; y += NT) rowc[y] = 0;
    if (tid == 0) S.flags = 0;
    __syncthreads();
    for (uint32_t b = tid; b < K; b += NT) {
        int sx, sy, dx, dy;
        load_move(I.moves, b, sx, sy, dx, dy);
        const uint32_t nh = (uint32_t)iabs(dx - sx) + 1u;
        add_wg32(&rowc[sy], nh);
        add_wg32(&rowc[sy + 1], 0u - nh);
        if (dy != sy) {
            const int vlo = dy > sy ? sy + 1 : dy, vhi = dy > sy ? dy : sy - 1;
            add_wg32(&rowc[vlo], 1u);
            add_wg32(&rowc[vhi + 1], 0xFFFFFFFFu);
        }
    }
    __syncthreads();

    // ---- row ranges (one wave): prefix of the row counts, then greedy ranges of up to 64 rows
    if (wid == 0) {
        uint32_t acc = 0, carry = 0;            // acc: difference prefix; carry: visits before the chunk
        for (int y0 = 0; y0 < H; y0 += kWave) {
            const int y = y0 + lane;
            const uint32_t dv = y < H ? rowc[y] : 0u;
            const uint32_t cnt = acc + (uint32_t)wave_incl_scan((int)dv);      // visits of row y
            acc = (uint32_t)__shfl((int)cnt, kWave - 1, kWave);
            const uint32_t cum = carry + (uint32_t)wave_incl_scan((int)cnt);   // visits of rows <= y
            carry = (uint32_t)__shfl((int)cum, kWave - 1, kWave);
            if (y < H) rowc[y] = cum;
        }
        wave_sync();
        uint32_t nr = 0, before = 0;
        bool bad = false;
        for (int y0 = 0; y0 < H && !bad;) {
            const int y1 = y0 + 1 + lane;       // candidate end (exclusive)
            bool fits = false;
            if (y1 <= H) {
                const uint64_t need = 4ull * ((uint64_t)(y1 - y0) * W + 1) + 2ull * (rowc[y1 - 1] - before);
                fits = need <= tile_bytes;
            }
            const int n = popc(ballot(fits));   // the cost grows with y1: the fitting ends are a prefix
            if (n == 0) { bad = true; break; }
            if (lane == 0) rs[nr] = (uint32_t)y0;
            for (int y = y0 + lane; y < y0 + n; y += kWave) rrow[y] = (uint16_t)nr;
            before = rowc[y0 + n - 1];
            ++nr;
            y0 += n;
        }
        if (lane == 0) {
            rs[nr] = (uint32_t)H;
            S.nr = nr;
            if (bad) S.flags = 2;
        }
    }
    __syncthreads();
    if (S.flags) return false;
    const uint32_t R = S.nr;

    // ---- per-range move lists: a path's rows are contiguous, so a move lies in ranges ra..rb
    for (uint32_t r = tid; r <= R; r += NT) roff[r] = 0;
    __syncthreads();
    for (uint32_t b = tid; b < K; b += NT) {
        int sx, sy, dx, dy;
        load_move(I.moves, b, sx, sy, dx, dy);
        const uint32_t ra = rrow[min(sy, dy)], rb = rrow[max(sy, dy)];
        for (uint32_t r = ra; r <= rb; ++r) add_wg32(&roff[r], 1u);
    }
    __syncthreads();
    block_scan<NT>(roff, R, S);
    for (uint32_t b = tid; b < K; b += NT) {
        int sx, sy, dx, dy;
        load_move(I.moves, b, sx, sy, dx, dy);
        const uint32_t ra = rrow[min(sy, dy)], rb = rrow[max(sy, dy)];
        for (uint32_t r = ra; r <= rb; ++r) rlist[add_wg32(&roff[r], 1u)] = (uint16_t)b;
    }
    __syncthreads();                            // roff[r] is now the end of range r's list

    // ---- the ranges
    for (uint32_t r = 0; r < R; ++r) {
        const int y0 = (int)rs[r], y1 = (int)rs[r + 1];
        const uint32_t c0 = (uint32_t)(y0 * W), nc = (uint32_t)((y1 - y0) * W);
        uint32_t *cell = (uint32_t *)tile;
        uint16_t *touch = (uint16_t *)(tile + 4 * ((size_t)nc + 1));
        const uint32_t mlo = r ? roff[r - 1] : 0u, mhi = roff[r];
        for (uint32_t c = tid; c <= nc; c += NT) cell[c] = 0;
        if (tid == 0) S.nlong = 0;
        __syncthreads();
        for (uint32_t t = mlo + tid; t < mhi; t += NT) {
            int sx, sy, dx, dy;
            load_move(I.moves, rlist[t], sx, sy, dx, dy);
            walk_rows(W, sx, sy, dx, dy, y0, y1, [&](int c) { add_wg32(&cell[(uint32_t)c - c0], 1u); });
        }
        __syncthreads();
        block_scan<NT>(cell, nc, S);
        for (uint32_t t = mlo + tid; t < mhi; t += NT) {
            const uint32_t b = rlist[t];
            int sx, sy, dx, dy;
            load_move(I.moves, b, sx, sy, dx, dy);
            walk_rows(W, sx, sy, dx, dy, y0, y1,
                      [&](int c) { touch[add_wg32(&cell[(uint32_t)c - c0], 1u)] = (uint16_t)b; });
        }
        __syncthreads();
        // previous toucher of every visit in the range: the largest index below b on the
        // trap's list, read unsorted two entries at a time (the lists are short; a scan of
        // independent reads beats sorting them and searching).  A thread per move -- except
        // that a long horizontal leg (more than kLongLeg traps, in this range) is queued and
        // searched afterwards by a whole wave, its lanes taking the leg's traps: one such leg
        // in a wave of short walks would otherwise hold the other 63 lanes.
        // Lists of kSortLo+1..128 entries (the receiver columns') are sorted first, a wave each
        // (two entries per lane, bitonic network), and searched by bisection.
        for (uint32_t cb = (uint32_t)wid * kWave; cb < nc; cb += (uint32_t)NT) {
            const uint32_t c = cb + lane;
            uint32_t n = 0;
            if (c < nc) n = cell[c] - (c ? cell[c - 1] : 0u);
            uint64_t lm = ballot(n > kSortLo && n <= 2u * kWave);
            while (lm) {
                const int l = (int)__builtin_ctzll(lm);
                lm &= lm - 1;
                const uint32_t cl = cb + (uint32_t)l;
                const uint32_t lo = cl ? cell[cl - 1] : 0u, n2 = cell[cl] - lo;
                uint32_t ea = (uint32_t)lane < n2 ? touch[lo + lane] : 0xFFFFu;
                uint32_t eb = (uint32_t)lane + kWave < n2 ? touch[lo + kWave + lane] : 0xFFFFu;
                for (int k = 2; k <= 2 * kWave; k <<= 1) {
                    for (int j = k >> 1; j > 0; j >>= 1) {
                        if (j == kWave) {               // the two entries of a lane (k = 128)
                            const uint32_t mn = ea < eb ? ea : eb, mx = ea < eb ? eb : ea;
                            ea = mn; eb = mx;
                        } else {
                            const uint32_t xa = (uint32_t)__shfl_xor((int)ea, j, kWave);
                            const uint32_t xb = (uint32_t)__shfl_xor((int)eb, j, kWave);
                            const bool lower = (lane & j) == 0;
                            const bool upa = (lane & k) == 0, upb = ((lane + kWave) & k) == 0;
                            ea = (lower == upa) ? (ea < xa ? ea : xa) : (ea < xa ? xa : ea);
                            eb = (lower == upb) ? (eb < xb ? eb : xb) : (eb < xb ? xb : eb);
                        }
                    }
                }
                if ((uint32_t)lane < n2) touch[lo + lane] = (uint16_t)ea;
                if ((uint32_t)lane + kWave < n2) touch[lo + kWave + lane] = (uint16_t)eb;
            }
        }
        __syncthreads();
        const uint32_t *t32 = (const uint32_t *)touch;
        auto prev_of = [&](uint32_t c, uint32_t b) -> uint32_t {   // previous toucher + 1, 0 if none
            const uint32_t lo = c ? cell[c - 1] : 0u, hi = cell[c];
            if (hi - lo > kSortLo && hi - lo <= 2u * kWave) {     // sorted: the entry before b
                if (touch[lo] >= b) return 0u;
                uint32_t l = lo, h = hi;
                while (h - l > 1) {
                    const uint32_t mid = (l + h) >> 1;
                    if (touch[mid] < b) l = mid; else h = mid;
                }
                return (uint32_t)touch[l] + 1u;
            }
            uint32_t best = 0;
            for (uint32_t w = lo >> 1; w < (hi + 1) >> 1; ++w) {
                const uint32_t v = t32[w], x0 = v & 0xFFFFu, x1 = v >> 16;
                best = (2 * w >= lo && x0 < b && x0 >= best) ? x0 + 1 : best;
                best = (2 * w + 1 < hi && x1 < b && x1 >= best) ? x1 + 1 : best;
            }
            return best;
        };
        for (uint32_t t = mlo + tid; t < mhi; t += NT) {
            const uint32_t b = rlist[t];
            int sx, sy, dx, dy;
            load_move(I.moves, b, sx, sy, dx, dy);
            const uint32_t g = grp[b], glo = I.goff[g];     // b's group holds the moves glo..
            bool defer = false;
            if (sy >= y0 && sy < y1 && iabs(dx - sx) >= kLongLeg) {
                const uint32_t at = add_wg32(&S.nlong, 1u);
                if (at < kLongCap) { S.longq[at] = (uint16_t)b; defer = true; }
            }
            uint32_t ps[kMaxPreds], pc[kMaxPreds];
            int np = 0;
            bool loaded = false, changed = false, ovf = false;
            uint32_t last = 0xFFFFFFFFu, lastg = 0xFFFFFFFFu;
            const int rowlo = sy * W;
            walk_rows(W, sx, sy, dx, dy, y0, y1, [&](int cg) {
                if (defer && (uint32_t)(cg - rowlo) < (uint32_t)W) return;  // the queued leg (corner included)
                const uint32_t best = prev_of((uint32_t)cg - c0, b);
                if (best == 0) return;
                const uint32_t a = best - 1;
                if (a == last) return;
                last = a;
                if (a >= glo) {                 // same group (a < b)
                    if (!loaded) {
                        np = (int)pend[b];
#pragma unroll
                        for (int i = 0; i < kMaxPreds; ++i)
                            if (i < np) { ps[i] = preds[(size_t)b * kMaxPreds + i]; pc[i] = 0u; }
                        loaded = true;
                    }
                    changed |= pred_add(ps, pc, np, a, I.moves, ovf);
                } else {
                    const uint32_t ga = grp[a];
                    if (ga != lastg) {
                        lastg = ga;
                        __hip_atomic_fetch_or(&gbits[g * GW + ga / 32], 1u << (ga & 31), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
                    }
                }
            });
            if (changed) {
                pend[b] = (uint32_t)np;
#pragma unroll
                for (int i = 0; i < kMaxPreds; ++i)
                    if (i < np) preds[(size_t)b * kMaxPreds + i] = (uint16_t)ps[i];
            }
            if (ovf) S.flags = 1;
        }
        __syncthreads();
        // the queued long legs, one wave each
        const uint32_t nq = S.nlong < kLongCap ? S.nlong : kLongCap;
        for (uint32_t qi = (uint32_t)wid; qi < nq; qi += (uint32_t)(NT / kWave)) {
            const uint32_t b = S.longq[qi];
            int sx, sy, dx, dy;
            load_move(I.moves, b, sx, sy, dx, dy);
            const uint32_t g = grp[b], glo = I.goff[g];
            const int nh = iabs(dx - sx) + 1, sth = dx >= sx ? 1 : -1;
            uint32_t ps[kMaxPreds], pc[kMaxPreds];
            int np = 0;
            bool loaded = false, changed = false, ovf = false;
            uint32_t lastg = 0xFFFFFFFFu;
            for (int s0 = 0; s0 < nh; s0 += kWave) {
                const int sv = s0 + lane;
                uint32_t a = 0xFFFFFFFFu, ga = 0xFFFFFFFFu;
                if (sv < nh) {
                    const uint32_t best = prev_of((uint32_t)(sy * W + sx + sth * sv) - c0, b);
                    if (best) {
                        a = best - 1;
                        if (a < glo) ga = grp[a];
                    }
                }
                uint64_t act = ballot(a != 0xFFFFFFFFu);
                while (act) {                   // the distinct previous touchers, one by one
                    const int l = (int)__builtin_ctzll(act);
                    const uint32_t u = (uint32_t)__builtin_amdgcn_readlane((int)a, l);
                    act &= ~ballot(a == u);
                    if (u >= glo) {
                        if (!loaded) {
                            np = (int)pend[b];
#pragma unroll
                            for (int i = 0; i < kMaxPreds; ++i)
                                if (i < np) { ps[i] = preds[(size_t)b * kMaxPreds + i]; pc[i] = 0u; }
                            loaded = true;
                        }
                        changed |= pred_add(ps, pc, np, u, I.moves, ovf);
                    } else {
                        const uint32_t gu = (uint32_t)__builtin_amdgcn_readlane((int)ga, l);
                        if (gu != lastg) {
                            lastg = gu;
                            if (lane == 0)
                                __hip_atomic_fetch_or(&gbits[g * GW + gu / 32], 1u << (gu & 31), __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_WORKGROUP);
                        }
                    }
                }
            }
            if (changed && lane == 0) {
                pend[b] = (uint32_t)np;
#pragma unroll
                for (int i = 0; i < kMaxPreds; ++i)
                    if (i < np) preds[(size_t)b * kMaxPreds + i] = (uint16_t)ps[i];
            }
            if (ovf && lane == 0) S.flags = 1;
        }
        __syncthreads();
    }
    if (S.flags) {
        if (tid == 0) hdr[H_STATE] = ST_GENERIC;
        return true;
    }
    // ---- successor counts, then the common second half
    for (uint32_t b = tid; b < K; b += NT) {
        const uint32_t np = pend[b];
        for (uint32_t i = 0; i < np; ++i) add_wg32(&soff[preds[(size_t)b * kMaxPreds + i]], 1u);
    }
    __syncthreads();
    graph_tail<NT, false>(I, S, L, K, G, T, nullptr, nullptr);
    return true;
}

// Build the graph of one instance (whole workgroup).  lds: dynamic LDS of lds_bytes bytes.
template <int NT>
__device__ void graph_build(const Inst &I, GraphShared<NT / kWave> &S, uint8_t *lds, uint32_t lds_bytes, bool force_generic)
{
    const int tid = threadIdx.x;
    const int W = I.W, H = I.H;
    const Layout L = layout(W, H, I.move_cap, I.step_cap);
    uint32_t *hdr = (uint32_t *)(I.ws + L.hdr);
    const rr_solve_info si = *I.sinfo;

    // ---- trivial and invalid instances: finished here
    if (si.status == RR_INFEASIBLE || (si.status == RR_OK && si.n_moves == 0)) {
        if (tid == 0) { I.boff[0] = 0; put_info(I.binfo, RR_OK, 0, 0, 0, 0); hdr[H_STATE] = ST_DONE; }
        return;
    }
    const uint32_t K = si.n_moves, G = si.n_groups;
    if (si.status != RR_OK || K > I.move_cap || G > K || K > gen::kMaxMoves || G > gen::kMaxGroups) {
        if (tid == 0) { put_info(I.binfo, RR_E_INVAL, 0, 0, 0, 0); hdr[H_STATE] = ST_DONE; }
        return;
    }
    // ---- validate moves and groups; total steps
    bool bad = false;
    uint32_t T = 0;
    for (uint32_t b = tid; b < K; b += NT) {
        int sx, sy, dx, dy;
        load_move(I.moves, b, sx, sy, dx, dy);
        const int len = iabs(dx - sx) + iabs(dy - sy);
        bad |= sx >= W || dx >= W || sy >= H || dy >= H || len == 0;
        T += (uint32_t)len;
    }
    for (uint32_t g = tid; g < G; g += NT) bad |= I.goff[g] > I.goff[g + 1];
    if (tid == 0) bad |= I.goff[0] != 0 || I.goff[G] != K;
    const uint32_t nbad = block_sum<NT>(bad ? 1u : 0u, S);
    T = block_sum<NT>(T, S);
    if (nbad) {
        if (tid == 0) { put_info(I.binfo, RR_E_INVAL, 0, 0, 0, 0); hdr[H_STATE] = ST_DONE; }
        return;
    }
    if (T > I.step_cap) {
        if (tid == 0) { put_info(I.binfo, RR_E_CAPACITY, 0, 0, T, T); hdr[H_STATE] = ST_DONE; }
        return;
    }
    if (force_generic || K > kMaxK || G > L.Gc) {
        if (tid == 0) hdr[H_STATE] = ST_GENERIC;
        return;
    }

    // ---- per-trap arrays: LDS when they fit, else the workspace (two copies of the code, so the
    //      LDS one compiles to ds_* operations)
    const uint32_t WH = (uint32_t)(W * H);
    const size_t OCC = (size_t)K + T;
    const size_t need = 4 * ((size_t)WH + 1) + 2 * (size_t)K + 2 * OCC + 16;
    if (need <= lds_bytes) {
        uint16_t *grp = (uint16_t *)(lds + 4 * ((size_t)WH + 1));
        uint16_t *touch = (uint16_t *)(lds + 4 * ((size_t)WH + 1) + 2 * (((size_t)K + 1) & ~(size_t)1));
        // after the per-trap arrays: the successor counts at the start of the LDS, then the
        // transposed group bit matrix when it fits beside them
        const size_t gt_at = (4 * ((size_t)K + 1) + 15) & ~(size_t)15;
        uint32_t *gt = gt_at + 4 * (size_t)G * L.GW <= lds_bytes ? (uint32_t *)(lds + gt_at) : nullptr;
        graph_core<NT>(I, S, L, K, G, T, (uint32_t *)lds, grp, touch, (uint32_t *)lds, gt);
    } else if (!graph_tiled<NT>(I, S, L, K, G, T, lds, lds_bytes)) {
        graph_core<NT>(I, S, L, K, G, T, (uint32_t *)(I.ws + L.cell), (uint16_t *)(I.ws + L.grp),
                   (uint16_t *)(I.ws + L.touch), (uint32_t *)(I.ws + L.soff), nullptr);
    }
}


}  // namespace fast
}  // namespace rr
