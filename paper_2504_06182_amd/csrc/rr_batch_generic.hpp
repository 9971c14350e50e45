// rr_batch_generic.hpp -- general batching path (arXiv 2504.06182, §IV, Alg. 3): one wave64 per
// instance, any number of moves (< 2^20) and any size of the ready set.  The fast path
// (rr_batch_graph.hpp + rr_batch_loop.hpp) falls back to it for instances outside its limits.
//
// The dependency graph Gamma is never materialised.  Any two moves that touch a common trap are
// ordered in Gamma (same group: their paths meet; different groups: their groups meet), so the
// moves touching one trap finish in index order, and Gamma has the same readiness as its
// reduction to consecutive touchers of each trap:
//   * move b waits for the previous toucher of each of its traps when that one is in b's group
//     (a successor edge a -> b, kept once however many traps a and b share);
//   * group h waits for the group that touched each of its traps last before it (a group edge,
//     kept once per pair of groups).
// A move is ready when it has no pending successor edge and its group none pending group edge.
// When a move finishes it releases its successors; when the last move of a group finishes, the
// groups waiting on it are released, and a released group contributes its head moves (those
// with no predecessor in the group).
//
// Each iteration of Alg. 3 takes the ready moves in index order: the first one is always
// accepted, and with the deployed constraint the batch is the first move plus the ready moves
// stepping the same way on the one line (row or column through its current trap) that the next
// compatible ready move picks.  Ready moves never share a trap (two that did would be ordered in
// Gamma), so the vertex-disjointness test of Alg. 3 never rejects a step and is not evaluated.
//
// Storage.  Up to 128 ready moves live in registers, two per lane, sorted by move index; larger
// ready sets live in LDS with a spill to the workspace.  Steps and batch ends are staged in LDS
// and written out in coalesced stretches.  The loop state (wait counts, successor lists, group
// data) is copied into dynamic LDS as 16-bit arrays when it fits the launch's budget, else it is
// used from the workspace.  The graph is built in the workspace: per-trap touch lists by
// counting sort, each list sorted by index (sorting network for short lists).
#pragma once
#include "rr_device.hpp"
#include "rr.h"

namespace rr {
namespace gen {

constexpr int kSlots = 2;                 // register slots per lane
constexpr int kRegCap = kSlots * kWave;   // ready sets up to this size stay in registers
constexpr int kRcap = 128;                // LDS part of the list-form ready buffers
constexpr int kStage = 256;               // output staging
constexpr uint32_t kMaxMoves = (1u << 20) - 1;
constexpr uint32_t kMaxGroups = 1024;

struct BatchArgs {
    int W, H;
    const rr_move *moves;
    const uint32_t *goff;
    const rr_solve_info *sinfo;
    uint32_t move_cap;
    uint32_t flags;
    uint32_t *boff;
    uint32_t batch_cap;
    uint32_t *steps;
    uint32_t step_cap;
    rr_batch_info *binfo;
    uint8_t *ws;
    uint32_t lds16_cap;       // 16-bit words of dynamic LDS for the loop state
};

struct BatchLds {
    uint64_t buf[3][kRcap];     // ready lists of the list form (rotating), LDS part
    uint32_t stage[kStage];     // steps of the current stretch of batches
    uint32_t bstage[kStage];    // batch ends of the current stretch
    uint32_t fin_list[kRegCap]; // moves completed in the current batch: idx | grp << 20
    int nnew;
    int err;
};

extern __shared__ __attribute__((aligned(16))) uint16_t dyn16[];

// workspace carve-up (all offsets 256-byte aligned).  OCC = moves + steps bounds the number of
// (move, trap) incidences and therefore every list below.
struct WsLayout {
    size_t coff, cfill, touch, scnt, sfill, sm, gcnt, gfill, gm;
    size_t pend, soff, slist, gpend, grem, goff, glist, hoff, heads, ov[3], total;
};

__host__ __device__ inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

__host__ __device__ inline WsLayout ws_layout(int W, int H, uint32_t move_cap, uint32_t step_cap)
{
    WsLayout L;
    const size_t WH = (size_t)W * H;
    const size_t K = (size_t)move_cap + 1;
    const size_t OCC = (size_t)move_cap + step_cap + 1;
    size_t p = 0;
    auto take = [&](size_t bytes) { const size_t at = p; p = align256(p + bytes); return at; };
    L.coff = take(4 * (WH + 1));
    L.cfill = take(4 * WH);
    L.touch = take(4 * OCC);
    L.scnt = take(4 * (K + 1));
    L.sfill = take(4 * K);
    L.sm = take(4 * OCC);
    L.gcnt = take(4 * (K + 1));
    L.gfill = take(4 * K);
    L.gm = take(4 * OCC);
    L.pend = take(4 * K);
    L.soff = take(4 * (K + 1));
    L.slist = take(4 * OCC);
    L.gpend = take(4 * K);
    L.grem = take(4 * K);
    L.goff = take(4 * (K + 1));
    L.glist = take(4 * OCC);
    L.hoff = take(4 * (K + 1));
    L.heads = take(4 * K);
    for (int i = 0; i < 3; ++i) L.ov[i] = take(8 * K);
    L.total = p;
    return L;
}

// two-level array: the first kRcap entries in LDS, the rest in the workspace
struct TwoLevel {
    uint64_t *lds;
    uint64_t *glb;
    int cap;
    __device__ __forceinline__ uint64_t get(int e) const
    {
        return e < kRcap ? lds[e] : (e < cap ? glb[e - kRcap] : ~0ull);
    }
    __device__ __forceinline__ void put(int e, uint64_t v) const
    {
        if (e < kRcap) lds[e] = v;
        else if (e < cap) glb[e - kRcap] = v;
    }
};

// The workspace of an instance is touched by its own wave only, so workgroup scope is enough for
// every atomic and fence on it (an agent-scope fence would write back and invalidate L2).
__device__ __forceinline__ uint32_t ld_rlx(const uint32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ __forceinline__ uint32_t add_wg(uint32_t *p, uint32_t v) { return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ __forceinline__ uint32_t sub_wg(uint32_t *p, uint32_t v) { return __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP); }
__device__ __forceinline__ void fence_wg() { __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup"); }

__device__ __forceinline__ void unpack_move(const rr_move *mv, uint32_t b, int &sx, int &sy, int &dx, int &dy)
{
    const uint64_t v = reinterpret_cast<const uint64_t *>(mv)[b];
    sx = (int)(v & 0xFFFF); sy = (int)((v >> 16) & 0xFFFF); dx = (int)((v >> 32) & 0xFFFF); dy = (int)(v >> 48);
}

// trap s (0..len) of the path: along row sy to column dx, then along column dx
__device__ __forceinline__ void path_cell(int sx, int sy, int dx, int dy, int s, int &x, int &y)
{
    const int hx = dx > sx ? dx - sx : sx - dx;
    if (s <= hx) { x = dx >= sx ? sx + s : sx - s; y = sy; }
    else { x = dx; y = dy >= sy ? sy + (s - hx) : sy - (s - hx); }
}

// Ready entry, sorted by move index (top bits):
//   idx << 44 | grp << 34 | dir << 32 | x << 24 | y << 16 | dx << 8 | dy     (coordinates < 256)
__device__ __forceinline__ uint64_t make_entry(uint32_t b, uint32_t g, int x, int y, int dx, int dy)
{
    uint32_t dir;
    if (x != dx) dir = dx > x ? 0u : 1u;
    else dir = dy > y ? 2u : 3u;
    return ((uint64_t)b << 44) | ((uint64_t)g << 34) | ((uint64_t)dir << 32) | ((uint64_t)x << 24) |
           ((uint64_t)y << 16) | ((uint64_t)dx << 8) | (uint64_t)dy;
}
__device__ __forceinline__ uint32_t e_dir(uint64_t v) { return (uint32_t)(v >> 32) & 3u; }
__device__ __forceinline__ uint32_t e_x(uint64_t v) { return (uint32_t)(v >> 24) & 0xFFu; }
__device__ __forceinline__ uint32_t e_y(uint64_t v) { return (uint32_t)(v >> 16) & 0xFFu; }
__device__ __forceinline__ uint32_t e_idx(uint64_t v) { return (uint32_t)(v >> 44); }
__device__ __forceinline__ uint32_t e_grp(uint64_t v) { return (uint32_t)(v >> 34) & 0x3FFu; }
// output step code: dir << 30 | x << 15 | y
__device__ __forceinline__ uint32_t e_code(uint64_t v) { return (e_dir(v) << 30) | (e_x(v) << 15) | e_y(v); }
// advance an accepted entry by its step; sets done when the move has arrived
__device__ __forceinline__ uint64_t e_advance(uint64_t v, bool &done)
{
    const uint32_t d = e_dir(v);
    const int x = (int)e_x(v) + (d == 0 ? 1 : (d == 1 ? -1 : 0));
    const int y = (int)e_y(v) + (d == 2 ? 1 : (d == 3 ? -1 : 0));
    const int dx = (int)((v >> 8) & 0xFFu), dy = (int)(v & 0xFFu);
    done = (x == dx && y == dy);
    return done ? ~0ull : make_entry(e_idx(v), e_grp(v), x, y, dx, dy);
}

__device__ __forceinline__ void put_binfo(rr_batch_info *bi, int status, uint32_t nb, uint32_t ns, uint32_t needb, uint32_t needs)
{
    rr_batch_info v;
    v.status = status; v.n_batches = nb; v.n_steps = ns; v.need_batches = needb; v.need_steps = needs;
    *bi = v;
}

// exclusive scan of a[0..n) in place into a[0..n] (a[n] = total), one wave
__device__ __forceinline__ void wave_scan_u32(uint32_t *a, int n)
{
    const int lane = lane_id();
    uint32_t carry = 0;
    for (int base = 0; base <= n; base += kWave) {
        const int c = base + lane;
        const uint32_t v = c < n ? ld_rlx(&a[c]) : 0u;
        const int inc = wave_incl_scan((int)v);
        if (c <= n) a[c] = carry + (uint32_t)inc - v;
        carry += (uint32_t)__shfl(inc, kWave - 1, kWave);
    }
}

// Sort a[0..n) ascending (one lane).  Up to 16 values go through a bitonic network in
// registers; longer lists are insertion-sorted in place.  With `unique`, equal values are
// collapsed and the number kept is returned.
__device__ __forceinline__ int sort_small(uint32_t *a, int n, bool unique)
{
    if (n <= 1) return n;
    if (n <= 16) {
        uint32_t r[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) r[i] = i < n ? a[i] : 0xFFFFFFFFu;
#pragma unroll
        for (int k = 2; k <= 16; k <<= 1)
#pragma unroll
            for (int j = k >> 1; j > 0; j >>= 1)
#pragma unroll
                for (int i = 0; i < 16; ++i) {
                    const int l = i ^ j;
                    if (l > i) {
                        const bool up = (i & k) == 0;
                        const uint32_t lo = r[i] < r[l] ? r[i] : r[l], hi = r[i] < r[l] ? r[l] : r[i];
                        r[i] = up ? lo : hi;
                        r[l] = up ? hi : lo;
                    }
                }
        int m = 0;
#pragma unroll
        for (int i = 0; i < 16; ++i)
            if (i < n && (!unique || m == 0 || r[i] != a[m - 1])) { a[m] = r[i]; ++m; }
        return m;
    }
    for (int k = 1; k < n; ++k) {
        const uint32_t v = a[k];
        int m = k;
        while (m > 0 && a[m - 1] > v) { a[m] = a[m - 1]; --m; }
        a[m] = v;
    }
    if (!unique) return n;
    int m = 1;
    for (int k = 1; k < n; ++k)
        if (a[k] != a[m - 1]) a[m++] = a[k];
    return m;
}

// Loop state: 16-bit arrays in dynamic LDS when they fit, else 32-bit arrays in the workspace.
struct LoopState {
    bool lds;
    uint16_t *pend16, *soff16, *slist16, *gpend16, *grem16, *goff16, *glist16, *hoff16, *heads16;
    uint32_t *pend, *soff, *slist, *gpend, *grem, *goff, *glist, *hoff, *heads;
    __device__ __forceinline__ uint32_t rd(const uint16_t *a16, const uint32_t *a32, uint32_t i) const
    {
        return lds ? (uint32_t)a16[i] : a32[i];
    }
    // atomic decrement, returns the old count
    __device__ __forceinline__ uint32_t dec(uint16_t *a16, uint32_t *a32, uint32_t i) const
    {
        if (lds) {
            uint32_t *w = reinterpret_cast<uint32_t *>(a16 + (i & ~1u));
            const uint32_t sh = (i & 1u) * 16u;
            return (atomicSub(w, 1u << sh) >> sh) & 0xFFFFu;   // counts never go below zero: no borrow
        }
        return sub_wg(&a32[i], 1u);
    }
};

__device__ void batch_one(BatchLds &S, const BatchArgs &A)
{
    const int lane = lane_id();
    const int W = A.W, H = A.H;
    const rr_solve_info si = *A.sinfo;
    if (si.status == RR_INFEASIBLE || (si.status == RR_OK && si.n_moves == 0)) {
        if (lane == 0) { A.boff[0] = 0; put_binfo(A.binfo, RR_OK, 0, 0, 0, 0); }
        return;
    }
    const uint32_t K = si.n_moves, G = si.n_groups;
    if (si.status != RR_OK || K > A.move_cap || G > K || K > kMaxMoves || G > kMaxGroups) {
        if (lane == 0) put_binfo(A.binfo, RR_E_INVAL, 0, 0, 0, 0);
        return;
    }
    // ---- validate moves and groups; total steps
    bool bad = false;
    uint32_t T = 0;
    for (uint32_t b = lane; b < K; b += kWave) {
        int sx, sy, dx, dy;
        unpack_move(A.moves, b, sx, sy, dx, dy);
        const int len = (dx > sx ? dx - sx : sx - dx) + (dy > sy ? dy - sy : sy - dy);
        bad |= sx >= W || dx >= W || sy >= H || dy >= H || len == 0;
        T += (uint32_t)len;
    }
    for (uint32_t g = lane; g < G; g += kWave) bad |= A.goff[g] > A.goff[g + 1];
    if (lane == 0) bad |= A.goff[0] != 0 || A.goff[G] != K;
    bad = ballot(bad) != 0ull;
    T = (uint32_t)wave_sum((int)T);
    if (bad) {
        if (lane == 0) put_binfo(A.binfo, RR_E_INVAL, 0, 0, 0, 0);
        return;
    }
    if (T > A.step_cap) {
        if (lane == 0) put_binfo(A.binfo, RR_E_CAPACITY, 0, 0, T, T);
        return;
    }

    const WsLayout Lw = ws_layout(W, H, A.move_cap, A.step_cap);
    auto W32 = [&](size_t off) { return (uint32_t *)(A.ws + off); };
    uint32_t *coff = W32(Lw.coff), *cfill = W32(Lw.cfill), *touch = W32(Lw.touch);
    uint32_t *scnt = W32(Lw.scnt), *sfill = W32(Lw.sfill), *sm = W32(Lw.sm);
    uint32_t *gcnt = W32(Lw.gcnt), *gfill = W32(Lw.gfill), *gm = W32(Lw.gm);
    uint32_t *pend = W32(Lw.pend), *soff = W32(Lw.soff), *slist = W32(Lw.slist);
    uint32_t *gpend = W32(Lw.gpend), *grem = W32(Lw.grem), *gof = W32(Lw.goff), *glist = W32(Lw.glist);
    uint32_t *hoff = W32(Lw.hoff), *heads = W32(Lw.heads);
    const int WH = W * H;

    // ---- group of every move (kept in scnt's slot until the counts need it: use sfill)
    for (int c = lane; c <= WH; c += kWave) coff[c] = 0;
    for (int c = lane; c < WH; c += kWave) cfill[c] = 0;
    for (uint32_t b = lane; b <= K; b += kWave) {
        scnt[b] = 0; gcnt[b] = 0;
        if (b < K) { pend[b] = 0; gpend[b] = 0; gfill[b] = 0; }
    }
    uint32_t *grp = sfill;   // group of each move, until the successor lists are built
    for (uint32_t g = lane; g < G; g += kWave) {
        const uint32_t lo = A.goff[g], hi = A.goff[g + 1];
        grem[g] = hi - lo;
        for (uint32_t b = lo; b < hi; ++b) grp[b] = g;
    }
    fence_wg();
    wave_sync();

    // ---- touch lists: the moves touching each trap, by move index
    for (uint32_t b = lane; b < K; b += kWave) {
        int sx, sy, dx, dy;
        unpack_move(A.moves, b, sx, sy, dx, dy);
        const int len = (dx > sx ? dx - sx : sx - dx) + (dy > sy ? dy - sy : sy - dy);
        for (int s = 0; s <= len; ++s) {
            int x, y;
            path_cell(sx, sy, dx, dy, s, x, y);
            add_wg(&coff[y * W + x], 1u);
        }
    }
    fence_wg();
    wave_sync();
    wave_scan_u32(coff, WH);
    fence_wg();
    wave_sync();
    for (uint32_t b = lane; b < K; b += kWave) {
        int sx, sy, dx, dy;
        unpack_move(A.moves, b, sx, sy, dx, dy);
        const int len = (dx > sx ? dx - sx : sx - dx) + (dy > sy ? dy - sy : sy - dy);
        for (int s = 0; s <= len; ++s) {
            int x, y;
            path_cell(sx, sy, dx, dy, s, x, y);
            const int c = y * W + x;
            touch[coff[c] + add_wg(&cfill[c], 1u)] = b;
        }
    }
    fence_wg();
    wave_sync();
    // consecutive touchers of a trap: same group -> successor edge, else group edge (counted with
    // multiplicity here, deduplicated below)
    for (int c = lane; c < WH; c += kWave) {
        const uint32_t lo = coff[c], n = coff[c + 1] - lo;
        sort_small(touch + lo, (int)n, false);
        for (uint32_t k = 1; k < n; ++k) {
            const uint32_t a = touch[lo + k - 1], b = touch[lo + k];
            const uint32_t ga = grp[a], gb = grp[b];
            if (ga == gb) add_wg(&scnt[a], 1u);
            else add_wg(&gcnt[ga], 1u);
        }
    }
    fence_wg();
    wave_sync();
    wave_scan_u32(scnt, (int)K);
    wave_scan_u32(gcnt, (int)G);
    for (int c = lane; c < WH; c += kWave) cfill[c] = 0;   // reused below as nothing
    fence_wg();
    wave_sync();
    // grp is still needed: move it to pend's... keep it in sfill and use heads[] as fill counters
    uint32_t *sfl = heads;   // temporary fill counters for the successor lists
    for (uint32_t b = lane; b < K; b += kWave) sfl[b] = 0;
    fence_wg();
    wave_sync();
    for (int c = lane; c < WH; c += kWave) {
        const uint32_t lo = coff[c], n = coff[c + 1] - lo;
        for (uint32_t k = 1; k < n; ++k) {
            const uint32_t a = touch[lo + k - 1], b = touch[lo + k];
            const uint32_t ga = grp[a], gb = grp[b];
            if (ga == gb) sm[scnt[a] + add_wg(&sfl[a], 1u)] = b;
            else gm[gcnt[ga] + add_wg(&gfill[ga], 1u)] = gb;
        }
    }
    fence_wg();
    wave_sync();
    // deduplicate: each successor / waiting group once
    for (uint32_t b = lane; b < K; b += kWave) {
        const uint32_t lo = scnt[b];
        const int m = sort_small(sm + lo, (int)(scnt[b + 1] - lo), true);
        sfl[b] = (uint32_t)m;
        for (int k = 0; k < m; ++k) add_wg(&pend[sm[lo + k]], 1u);
    }
    for (uint32_t g = lane; g < G; g += kWave) {
        const uint32_t lo = gcnt[g];
        const int m = sort_small(gm + lo, (int)(gcnt[g + 1] - lo), true);
        gfill[g] = (uint32_t)m;
        for (int k = 0; k < m; ++k) add_wg(&gpend[gm[lo + k]], 1u);
    }
    fence_wg();
    wave_sync();
    for (uint32_t b = lane; b <= K; b += kWave) soff[b] = b < K ? sfl[b] : 0u;
    for (uint32_t g = lane; g <= G; g += kWave) gof[g] = g < G ? gfill[g] : 0u;
    fence_wg();
    wave_sync();
    wave_scan_u32(soff, (int)K);
    wave_scan_u32(gof, (int)G);
    fence_wg();
    wave_sync();
    for (uint32_t b = lane; b < K; b += kWave) {
        const uint32_t lo = scnt[b], o = soff[b], m = soff[b + 1] - o;
        for (uint32_t k = 0; k < m; ++k) slist[o + k] = sm[lo + k];
    }
    for (uint32_t g = lane; g < G; g += kWave) {
        const uint32_t lo = gcnt[g], o = gof[g], m = gof[g + 1] - o;
        for (uint32_t k = 0; k < m; ++k) glist[o + k] = gm[lo + k];
    }
    // heads of every group: its moves with no predecessor in the group
    for (uint32_t g = lane; g <= G; g += kWave) {
        uint32_t c = 0;
        if (g < G)
            for (uint32_t b = A.goff[g]; b < A.goff[g + 1]; ++b) c += ld_rlx(&pend[b]) == 0u;
        hoff[g] = c;
    }
    fence_wg();
    wave_sync();
    wave_scan_u32(hoff, (int)G);
    fence_wg();
    wave_sync();
    for (uint32_t g = lane; g < G; g += kWave) {
        uint32_t o = hoff[g];
        for (uint32_t b = A.goff[g]; b < A.goff[g + 1]; ++b)
            if (ld_rlx(&pend[b]) == 0u) heads[o++] = b;
    }
    fence_wg();
    wave_sync();

    // ---- loop state: 16-bit copy in dynamic LDS when it fits
    const uint32_t E = soff[K], GE = gof[G], HN = hoff[G];
    const uint32_t need16 = 2u * ((K + 2) / 2) + 2u * ((K + 3) / 2) + 2u * ((E + 2) / 2) + 2u * ((G + 2) / 2) * 2u +
                            2u * ((G + 3) / 2) * 2u + 2u * ((GE + 2) / 2) + 2u * ((HN + 2) / 2);
    LoopState st;
    st.lds = need16 <= A.lds16_cap && K < 65535u && E < 65535u && GE < 65535u;
    st.pend = pend; st.soff = soff; st.slist = slist; st.gpend = gpend; st.grem = grem;
    st.goff = gof; st.glist = glist; st.hoff = hoff; st.heads = heads;
    {
        uint16_t *p = dyn16;
        auto carve = [&](uint32_t n) { uint16_t *at = p; p += 2u * ((n + 1) / 2); return at; };   // even sizes keep 4-byte alignment
        st.pend16 = carve(K + 1); st.soff16 = carve(K + 2); st.slist16 = carve(E + 1);
        st.gpend16 = carve(G + 1); st.grem16 = carve(G + 1); st.goff16 = carve(G + 2);
        st.glist16 = carve(GE + 1); st.hoff16 = carve(G + 2); st.heads16 = carve(HN + 1);
    }
    if (st.lds) {
        for (uint32_t i = lane; i < K; i += kWave) st.pend16[i] = (uint16_t)ld_rlx(&pend[i]);
        for (uint32_t i = lane; i <= K; i += kWave) st.soff16[i] = (uint16_t)soff[i];
        for (uint32_t i = lane; i < E; i += kWave) st.slist16[i] = (uint16_t)slist[i];
        for (uint32_t i = lane; i < G; i += kWave) { st.gpend16[i] = (uint16_t)ld_rlx(&gpend[i]); st.grem16[i] = (uint16_t)grem[i]; }
        for (uint32_t i = lane; i <= G; i += kWave) { st.goff16[i] = (uint16_t)gof[i]; st.hoff16[i] = (uint16_t)hoff[i]; }
        for (uint32_t i = lane; i < GE; i += kWave) st.glist16[i] = (uint16_t)glist[i];
        for (uint32_t i = lane; i < HN; i += kWave) st.heads16[i] = (uint16_t)heads[i];
    }
    wave_sync();

    // ---- ready buffers and the initial ready set: heads of the groups nothing waits for
    uint64_t *const ov0 = (uint64_t *)(A.ws + Lw.ov[0]);
    const size_t ovs = (Lw.ov[1] - Lw.ov[0]) / sizeof(uint64_t);
    const int rcap = kRcap + (int)K;
    auto B = [&](int i) { return TwoLevel{S.buf[i], ov0 + (size_t)i * ovs, rcap}; };
    if (lane == 0) { A.boff[0] = 0; S.nnew = 0; S.err = 0; }
    wave_sync();
    int cur = 0;
    {
        const TwoLevel NW = B(1);
        for (uint32_t g = lane; g < G; g += kWave)
            if (st.rd(st.gpend16, gpend, g) == 0u)
                for (uint32_t t = st.rd(st.hoff16, hoff, g); t < st.rd(st.hoff16, hoff, g + 1); ++t)
                    NW.put(atomicAdd(&S.nnew, 1), (uint64_t)st.rd(st.heads16, heads, t) | ((uint64_t)g << 20));
    }
    wave_sync();

    const uint32_t flags = A.flags & 0xFFu;
    uint32_t out = 0, nb = 0, alive = K;
    uint32_t sbase = 0, bbase = 1;            // first step / batch end held in the stage
    auto flush_steps = [&]() {
        for (uint32_t q = lane; q < out - sbase; q += kWave)
            if (sbase + q < A.step_cap) A.steps[sbase + q] = S.stage[q];
        sbase = out;
    };
    auto flush_batches = [&]() {
        for (uint32_t q = lane; q < nb + 1 - bbase; q += kWave)
            if (bbase + q <= A.batch_cap) A.boff[bbase + q] = S.bstage[q];
        bbase = nb + 1;
    };
    auto end_batch = [&](uint32_t na) {
        out += na;
        if (nb + 1 - bbase >= (uint32_t)kStage) { wave_sync(); flush_batches(); }   // writes bbase..nb
        ++nb;
        if (lane == 0) S.bstage[nb - bbase] = out;
    };
    // completed moves (S.fin_list[0..nfc), idx | grp << 20) release their successors and, when a
    // group completes, the groups waiting on it; newly ready moves are appended to NW
    auto release = [&](int nfc, const TwoLevel &NW) {
        for (int q = lane; q < nfc; q += kWave) {
            const uint32_t fl = S.fin_list[q];
            const uint32_t b = fl & 0xFFFFFu, g = fl >> 20;
            const uint32_t lo = st.rd(st.soff16, soff, b), hi = st.rd(st.soff16, soff, b + 1);
            for (uint32_t t = lo; t < hi; ++t) {
                const uint32_t nx = st.rd(st.slist16, slist, t);
                if (st.dec(st.pend16, pend, nx) == 1u) NW.put(atomicAdd(&S.nnew, 1), (uint64_t)nx | ((uint64_t)g << 20));
            }
            if (st.dec(st.grem16, grem, g) == 1u) {
                const uint32_t glo = st.rd(st.goff16, gof, g), ghi = st.rd(st.goff16, gof, g + 1);
                for (uint32_t t = glo; t < ghi; ++t) {
                    const uint32_t h = st.rd(st.glist16, glist, t);
                    if (st.dec(st.gpend16, gpend, h) == 1u)
                        for (uint32_t u = st.rd(st.hoff16, hoff, h); u < st.rd(st.hoff16, hoff, h + 1); ++u)
                            NW.put(atomicAdd(&S.nnew, 1), (uint64_t)st.rd(st.heads16, heads, u) | ((uint64_t)h << 20));
                }
            }
        }
    };
    // sort the nn new moves of NW (idx | grp << 20) by index into F as entries, then merge them
    // with the ns sorted survivors of Sv into Out by co-ranking
    auto merge = [&](const TwoLevel &Sv, int ns, const TwoLevel &F, const TwoLevel &NW, int nn, const TwoLevel &Out) {
        for (int k = lane; k < nn; k += kWave) {
            const uint32_t v = (uint32_t)NW.get(k), b = v & 0xFFFFFu;
            int r = 0;
            for (int q = 0; q < nn; ++q) r += ((uint32_t)NW.get(q) & 0xFFFFFu) < b;
            int sx, sy, dx, dy;
            unpack_move(A.moves, b, sx, sy, dx, dy);
            F.put(r, make_entry(b, v >> 20, sx, sy, dx, dy));
        }
        wave_sync();
        for (int i = lane; i < ns; i += kWave) {
            const uint64_t v = Sv.get(i);
            int lo = 0, hi = nn;
            while (lo < hi) { const int mid = (lo + hi) >> 1; if (F.get(mid) < v) lo = mid + 1; else hi = mid; }
            Out.put(i + lo, v);
        }
        for (int k = lane; k < nn; k += kWave) {
            const uint64_t v = F.get(k);
            int lo = 0, hi = ns;
            while (lo < hi) { const int mid = (lo + hi) >> 1; if (Sv.get(mid) < v) lo = mid + 1; else hi = mid; }
            Out.put(k + lo, v);
        }
        wave_sync();
    };

    // initial ready list: merge the heads into an empty list
    int n = S.nnew;
    merge(B(2), 0, B(2), B(1), n, B(0));
    if (lane == 0) S.nnew = 0;
    wave_sync();

    // ---- Alg. 3: one iteration per batch
    bool regm = false;        // register form: lane e holds entries e and 64 + e
    uint64_t r0 = ~0ull, r1 = ~0ull;
    while (alive > 0) {
        if (nb >= T) { if (lane == 0) S.err = 1; break; }   // every batch has a step: at most T
        if (n == 0) { if (lane == 0) S.err = 1; break; }    // unreachable: the lowest unfinished move is ready
        const int nwb = cur == 2 ? 0 : cur + 1;             // new ready moves collect here
        const int third = 3 - cur - nwb;
        const TwoLevel NW = B(nwb);

        if (n <= kRegCap) {
            // ---------------- register form ----------------
            if (!regm) {
                const TwoLevel R = B(cur);
                r0 = lane < n ? R.get(lane) : ~0ull;
                r1 = kWave + lane < n ? R.get(kWave + lane) : ~0ull;
                regm = true;
            }
            const bool val0 = lane < n, val1 = kWave + lane < n;
            const uint64_t v1 = ((uint64_t)(uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(r0 >> 32)) << 32) |
                                (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)r0);
            const uint32_t d1 = e_dir(v1), x1 = e_x(v1), y1 = e_y(v1);
            const uint32_t da = e_dir(r0), xa = e_x(r0), ya = e_y(r0);
            const uint32_t db = e_dir(r1), xb = e_x(r1), yb = e_y(r1);
            bool acc0, acc1;
            if (flags == RR_LAMBDA_NONE) { acc0 = val0; acc1 = val1; }
            else if (flags == RR_LAMBDA_ALONG) {
                acc0 = val0 && da == d1 && (d1 >= 2 ? xa == x1 : ya == y1);
                acc1 = val1 && db == d1 && (d1 >= 2 ? xb == x1 : yb == y1);
            } else {
                // the first compatible ready move after the first one fixes the line
                const uint64_t mc0 = ballot(val0 && lane > 0 && da == d1 && (xa == x1 || ya == y1));
                const uint64_t mc1 = ballot(val1 && db == d1 && (xb == x1 || yb == y1));
                acc0 = lane == 0;
                acc1 = false;
                if (mc0 | mc1) {
                    uint32_t yf;
                    if (mc0) yf = ((uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)r0, __ffsll((unsigned long long)mc0) - 1) >> 16) & 0xFFu;
                    else yf = ((uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)r1, __ffsll((unsigned long long)mc1) - 1) >> 16) & 0xFFu;
                    const bool row = yf == y1;
                    acc0 = acc0 || (val0 && da == d1 && (row ? ya == y1 : xa == x1));
                    acc1 = val1 && db == d1 && (row ? yb == y1 : xb == x1);
                }
            }
            const uint64_t ma0 = ballot(acc0), ma1 = ballot(acc1);
            const uint32_t n0 = (uint32_t)popc(ma0);
            const uint32_t na = n0 + (uint32_t)popc(ma1);
            if (out - sbase + na > (uint32_t)kStage) { wave_sync(); flush_steps(); }
            bool done0 = false, done1 = false;
            const uint32_t fl0 = e_idx(r0) | (e_grp(r0) << 20), fl1 = e_idx(r1) | (e_grp(r1) << 20);
            if (acc0) { S.stage[out - sbase + popc(ma0 & low_mask(lane))] = e_code(r0); r0 = e_advance(r0, done0); }
            if (acc1) { S.stage[out - sbase + n0 + popc(ma1 & low_mask(lane))] = e_code(r1); r1 = e_advance(r1, done1); }
            const uint64_t fm0 = ballot(done0), fm1 = ballot(done1);
            end_batch(na);
            const int f0 = popc(fm0), nfc = f0 + popc(fm1);
            if (nfc) {
                if (done0) S.fin_list[popc(fm0 & low_mask(lane))] = fl0;
                if (done1) S.fin_list[f0 + popc(fm1 & low_mask(lane))] = fl1;
                wave_sync();
                release(nfc, NW);
                alive -= (uint32_t)nfc;
                wave_sync();
            }
            const int nn = S.nnew;
            if (nfc == 0 && nn == 0) continue;
            // survivors keep their order; merge the new ready moves through LDS
            const uint64_t sm0 = ballot(r0 != ~0ull), sm1 = ballot(r1 != ~0ull);
            const int s0 = popc(sm0), ns = s0 + popc(sm1);
            const TwoLevel Sv = B(third);
            if (r0 != ~0ull) Sv.put(popc(sm0 & low_mask(lane)), r0);
            if (r1 != ~0ull) Sv.put(s0 + popc(sm1 & low_mask(lane)), r1);
            wave_sync();
            if (nn > 0) {
                merge(Sv, ns, B(cur), NW, nn, NW);
                cur = nwb;
            } else {
                cur = third;
            }
            n = ns + nn;
            const TwoLevel R = B(cur);
            r0 = lane < n ? R.get(lane) : ~0ull;
            r1 = kWave + lane < n ? R.get(kWave + lane) : ~0ull;
            regm = n <= kRegCap;
            if (lane == 0) S.nnew = 0;
            wave_sync();
            continue;
        }

        // ---------------- list form (more than kRegCap ready moves) ----------------
        regm = false;
        const TwoLevel R = B(cur);
        const uint64_t v1 = R.get(0);
        const uint32_t d1 = e_dir(v1), x1 = e_x(v1), y1 = e_y(v1);
        int first = n;
        bool row = false;
        if (flags == RR_LAMBDA_LINE_OR_COL) {
            for (int base = 0; base < n; base += kWave) {
                const int e = base + lane;
                bool cand = false;
                if (e > 0 && e < n) {
                    const uint64_t v = R.get(e);
                    cand = e_dir(v) == d1 && (e_x(v) == x1 || e_y(v) == y1);
                }
                const uint64_t m = ballot(cand);
                if (m) { first = base + __ffsll((unsigned long long)m) - 1; break; }
            }
            if (first < n) row = e_y(R.get(first)) == y1;
        }
        if (out - sbase + (uint32_t)n > (uint32_t)kStage) { wave_sync(); flush_steps(); }
        const bool direct = (uint32_t)n > (uint32_t)kStage;   // a huge ready list writes straight out
        uint32_t acc_before = 0;
        int nf = 0;
        for (int base = 0; base < n; base += kWave) {
            const int e = base + lane;
            bool acc = false;
            uint64_t v = 0;
            if (e < n) {
                v = R.get(e);
                const uint32_t d = e_dir(v), x = e_x(v), y = e_y(v);
                if (flags == RR_LAMBDA_NONE) acc = true;
                else if (flags == RR_LAMBDA_ALONG) acc = d == d1 && (d1 >= 2 ? x == x1 : y == y1);
                else acc = (e == 0) || (first < n && d == d1 && (row ? y == y1 : x == x1));
            }
            const uint64_t m = ballot(acc);
            bool done = false;
            const uint32_t fl = e_idx(v) | (e_grp(v) << 20);
            if (acc) {
                const uint32_t rank = acc_before + (uint32_t)popc(m & low_mask(lane));
                if (direct) { if (out + rank < A.step_cap) A.steps[out + rank] = e_code(v); }
                else S.stage[out - sbase + rank] = e_code(v);
                R.put(e, e_advance(v, done));
            }
            const uint64_t fm = ballot(done);
            if (done) S.fin_list[popc(fm & low_mask(lane))] = fl;
            acc_before += (uint32_t)popc(m);
            wave_sync();
            const int nfc = popc(fm);
            release(nfc, NW);
            nf += nfc;
            wave_sync();
        }
        if (direct) sbase = out + acc_before;
        end_batch(acc_before);
        alive -= (uint32_t)nf;
        const int nn = S.nnew;
        wave_sync();
        if (nf == 0 && nn == 0) continue;
        int sbuf = cur, freeb = third;
        int ns = n;
        if (nf > 0) {
            ns = 0;
            for (int base = 0; base < n; base += kWave) {
                const int e = base + lane;
                const uint64_t v = e < n ? R.get(e) : ~0ull;
                const bool keep = v != ~0ull;
                const uint64_t m = ballot(keep);
                if (keep) B(third).put(ns + popc(m & low_mask(lane)), v);
                ns += popc(m);
            }
            sbuf = third; freeb = cur;
            wave_sync();
        }
        if (nn > 0) {
            merge(B(sbuf), ns, B(freeb), NW, nn, NW);
            cur = nwb;
            n = ns + nn;
        } else {
            cur = sbuf;
            n = ns;
        }
        if (lane == 0) S.nnew = 0;
        wave_sync();
    }

    wave_sync();
    flush_steps();
    flush_batches();
    const bool err = S.err != 0;
    if (lane == 0) {
        const bool cap = nb > A.batch_cap;
        const int st_ = err ? RR_E_INTERNAL : (cap ? RR_E_CAPACITY : RR_OK);
        const bool ok = st_ == RR_OK;
        put_binfo(A.binfo, st_, ok ? nb : 0u, ok ? out : 0u, nb, T);
    }
}

}  // namespace gen
}  // namespace rr
