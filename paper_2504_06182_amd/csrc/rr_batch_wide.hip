// rr_batch_wide.hip -- batching (arXiv 2504.06182, §IV, Alg. 3) for grids beyond RR_LDS_SIDE per
// side, up to RR_MAX_SIDE, on gfx950.  Two kernels per instance:
//
//   k_wide_graph_*  one 1024-thread workgroup: validation, total steps, and the dependency graph
//                   Γ in a reduced form that has the same readiness.  The groups are walked in
//                   order.  For each group its moves are staged in LDS and
//                     * every move gets its in-group predecessors: the earlier moves of the
//                       group whose paths meet its own (two moves of one group whose paths meet
//                       are ordered in Γ), scanned from the nearest down, a candidate skipped
//                       when its path meets a member already kept (it is then an ancestor of
//                       that member), at most 8 kept;
//                     * every trap of every move reads the last group that touched it before
//                       (a per-trap word in the workspace), giving the group's predecessor
//                       groups as a bit row; then the group stamps its traps.
//                   From these: successor lists, the groups waiting on each group, each
//                   group's head moves (no in-group predecessor), and a release record per
//                   move (its one successor that waits on nothing else, with that successor's
//                   packed move, when it has such a single successor).
//   k_wide_loop_*   one wave64: Alg. 3 with the ready set in LDS, sorted by move index, as
//                   entries (current step code, end of the current leg, next leg, key).  Each
//                   trip forms one batch -- the first ready move, and under the line-or-column
//                   constraint the ready moves stepping its way on the row or column that the
//                   first compatible one shares with it -- and then repeats it while nothing
//                   can change it: no member ends a leg and no waiting move reaches the line
//                   that sweeps with the first one (the convoy).  Moves that end their path
//                   release their successors and, when a group completes, the heads of the
//                   groups waiting on it; new ready moves are sorted and merged in.
//
// The same trip logic as the register-resident loop of the smaller grids, with 15-bit
// coordinates in the step codes and 21-bit move indices; the ready set holds up to 4096 moves
// (a seeded 1024 x 1024 shot peaks at 1560).
#include "rr_device.hpp"
#include "rr.h"
#include "rr_batch_common.hpp"
#include "rr_batch_wide.hpp"

namespace rr {
namespace wide {

constexpr int kGT = 1024;                  // graph kernel threads per instance
constexpr int kGWaves = kGT / kWave;
constexpr uint32_t INV = 0xFFFFFFFFu;
constexpr uint32_t kRcap = 4096;           // ready entries in LDS
constexpr uint32_t kNcap = 2048;           // moves made ready in one trip
enum { REC_NONE = 0u, REC_DIRECT = 1u, REC_LIST = 2u };   // release record kinds (bits 30..31)
constexpr uint32_t ST_READY = 0x52454459u; // header state: graph built, the loop runs
enum { H_STATE = 0, H_T = 1, H_K = 2, H_G = 3 };
enum { ERR_INTERNAL = 1, ERR_CAPACITY = 2 };

// step codes: dir << 30 | x << 15 | y
constexpr uint32_t MY = 0xC0007FFFu;       // direction and row
constexpr uint32_t MX = 0xFFFF8000u;       // direction and column

__device__ __forceinline__ uint32_t atomic_add_wg(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ uint32_t atomic_sub_wg(uint32_t *p, uint32_t v)
{
    return __hip_atomic_fetch_sub(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void unpack(uint64_t v, int &sx, int &sy, int &dx, int &dy)
{
    sx = (int)(v & 0xFFFFu); sy = (int)((v >> 16) & 0xFFFFu); dx = (int)((v >> 32) & 0xFFFFu); dy = (int)(v >> 48);
}

__device__ __forceinline__ int iabs(int v) { return v < 0 ? -v : v; }

__device__ __forceinline__ uint32_t path_len(uint64_t v)
{
    int sx, sy, dx, dy;
    unpack(v, sx, sy, dx, dy);
    return (uint32_t)(iabs(dx - sx) + iabs(dy - sy));
}

// trap s (0..len) of a path: along row sy to column dx, then along column dx
__device__ __forceinline__ uint32_t path_trap(int W, int sx, int sy, int dx, int dy, int s)
{
    const int hx = iabs(dx - sx);
    if (s <= hx) return (uint32_t)(sy * W + (dx >= sx ? sx + s : sx - s));
    const int v = s - hx;
    return (uint32_t)((dy >= sy ? sy + v : sy - v) * W + dx);
}

__device__ __forceinline__ bool spans(int v, int a, int b) { return a <= b ? (a <= v && v <= b) : (b <= v && v <= a); }

__device__ __forceinline__ bool overlap(int a1, int b1, int a2, int b2)
{
    const int lo1 = a1 < b1 ? a1 : b1, hi1 = a1 < b1 ? b1 : a1, lo2 = a2 < b2 ? a2 : b2, hi2 = a2 < b2 ? b2 : a2;
    return (lo1 > lo2 ? lo1 : lo2) <= (hi1 < hi2 ? hi1 : hi2);
}

// do the row-then-column paths of two moves share a trap (endpoints included)?
__device__ __forceinline__ bool paths_meet(uint64_t p, uint64_t q)
{
    int psx, psy, pdx, pdy, qsx, qsy, qdx, qdy;
    unpack(p, psx, psy, pdx, pdy);
    unpack(q, qsx, qsy, qdx, qdy);
    const bool hh = psy == qsy && overlap(psx, pdx, qsx, qdx);
    const bool hv = spans(qdx, psx, pdx) && spans(psy, qsy, qdy);
    const bool vh = spans(pdx, qsx, qdx) && spans(qsy, psy, pdy);
    const bool vv = pdx == qdx && overlap(psy, pdy, qsy, qdy);
    return hh || hv || vh || vv;
}

// ------------------------------------------------------------------------------------------
// graph kernel

struct GraphShared {
    uint64_t mv[kGroupCap];          // the current group's moves
    uint32_t inc[kGroupCap + 1];     // exclusive prefix of their trap counts
    uint32_t gb[kMaxGroups / 32];    // the current group's predecessor groups
    uint32_t part[kGWaves];
    uint64_t part64[kGWaves];
    uint32_t flags;
};

__device__ __forceinline__ uint32_t block_excl(uint32_t v, GraphShared &S, uint32_t *total)
{
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    const uint32_t inc = (uint32_t)wave_incl_scan((int)v);
    if (lane == kWave - 1) S.part[wid] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kGWaves; ++w) {
        const uint32_t t = S.part[w];
        off += w < wid ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__device__ __forceinline__ uint64_t block_sum64(uint64_t v, GraphShared &S)
{
    const int lane = lane_id(), wid = threadIdx.x >> 6;
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += shfl_xor_u64(v, m);
    if (lane == 0) S.part64[wid] = v;
    __syncthreads();
    uint64_t tot = 0;
#pragma unroll
    for (int w = 0; w < kGWaves; ++w) tot += S.part64[w];
    __syncthreads();
    return tot;
}

// exclusive scan of a[0..n) in place, a[n] = total; every thread a contiguous chunk
__device__ void scan_ws(uint32_t *a, uint32_t n, GraphShared &S)
{
    __syncthreads();
    const uint32_t tid = threadIdx.x;
    const uint32_t ch = (n + kGT - 1) / kGT;
    const uint32_t lo = tid * ch < n ? tid * ch : n, hi = lo + ch < n ? lo + ch : n;
    uint32_t s = 0;
    for (uint32_t i = lo; i < hi; ++i) s += a[i];
    uint32_t tot;
    uint32_t run = block_excl(s, S, &tot);
    for (uint32_t i = lo; i < hi; ++i) {
        const uint32_t v = a[i];
        a[i] = run;
        run += v;
    }
    if (tid == 0) a[n] = tot;
    __syncthreads();
}

struct Ptrs {
    uint32_t *hdr, *lastg, *gbits, *preds, *pend, *scnt, *sfill, *slist, *gpend, *gcnt, *gfill, *glist, *hoff, *heads;
    uint4 *rec;
    uint32_t gw;
};

__device__ __forceinline__ Ptrs ptrs_of(const fast::Inst &I)
{
    const Layout L = layout(I.W, I.H, I.move_cap);
    auto W32 = [&](size_t off) { return (uint32_t *)(I.ws + off); };
    Ptrs P;
    P.hdr = W32(L.hdr); P.lastg = W32(L.lastg); P.gbits = W32(L.gbits); P.preds = W32(L.preds);
    P.pend = W32(L.pend); P.scnt = W32(L.scnt); P.sfill = W32(L.sfill); P.slist = W32(L.slist);
    P.gpend = W32(L.gpend); P.gcnt = W32(L.gcnt); P.gfill = W32(L.gfill); P.glist = W32(L.glist);
    P.hoff = W32(L.hoff); P.heads = W32(L.heads);
    P.rec = (uint4 *)(I.ws + L.rec);
    P.gw = L.gw;
    return P;
}

__device__ void graph(const fast::Inst &I, GraphShared &S)
{
    const uint32_t tid = threadIdx.x;
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    const int W = I.W, H = I.H;
    const Ptrs P = ptrs_of(I);
    const uint64_t *mv64 = reinterpret_cast<const uint64_t *>(I.moves);
    if (tid == 0) P.hdr[H_STATE] = 0u;
    const rr_solve_info si = *I.sinfo;
    if (si.status == RR_INFEASIBLE || (si.status == RR_OK && si.n_moves == 0)) {
        if (tid == 0) { I.boff[0] = 0; fast::put_info(I.binfo, RR_OK, 0, 0, 0, 0); }
        return;
    }
    const uint32_t K = si.n_moves, G = si.n_groups;
    if (si.status != RR_OK || K > I.move_cap || K > kMaxMoves || G == 0 || G > K || G > group_bound(W, H)) {
        if (tid == 0) fast::put_info(I.binfo, RR_E_INVAL, 0, 0, 0, 0);
        return;
    }

    // ---- validate the moves and groups; total steps
    bool bad = false;
    uint64_t T = 0;
    for (uint32_t b = tid; b < K; b += kGT) {
        int sx, sy, dx, dy;
        unpack(mv64[b], sx, sy, dx, dy);
        const int len = iabs(dx - sx) + iabs(dy - sy);
        bad |= sx >= W || dx >= W || sy >= H || dy >= H || len == 0;
        T += (uint64_t)len;
    }
    for (uint32_t g = tid; g < G; g += kGT) {
        const uint32_t lo = I.goff[g], hi = I.goff[g + 1];
        bad |= lo > hi || hi - lo > kGroupCap;
    }
    if (tid == 0) bad |= I.goff[0] != 0u || I.goff[G] != K;
    uint32_t nbad;
    block_excl(bad ? 1u : 0u, S, &nbad);
    T = block_sum64(T, S);
    if (nbad) {
        if (tid == 0) fast::put_info(I.binfo, RR_E_INVAL, 0, 0, 0, 0);
        return;
    }
    if (T > I.step_cap) {
        const uint32_t t32 = T > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)T;
        if (tid == 0) fast::put_info(I.binfo, RR_E_CAPACITY, 0, 0, t32, t32);
        return;
    }

    const uint32_t GW = P.gw;
    for (uint32_t c = tid; c < (uint32_t)(W * H); c += kGT) P.lastg[c] = INV;
    for (uint32_t b = tid; b <= K; b += kGT) {
        P.scnt[b] = 0u;
        if (b < K) P.sfill[b] = 0u;
    }
    for (uint32_t g = tid; g <= G; g += kGT) {
        P.gcnt[g] = 0u;
        if (g < G) P.gfill[g] = 0u;
    }
    if (tid == 0) S.flags = 0u;
    __syncthreads();

    // ---- groups in order
    for (uint32_t h = 0; h < G; ++h) {
        const uint32_t lo = I.goff[h], n = I.goff[h + 1] - lo;
        for (uint32_t i = tid; i < n; i += kGT) S.mv[i] = mv64[lo + i];
        if (tid < GW) S.gb[tid] = 0u;
        __syncthreads();
        {
            const uint32_t i0 = 2 * tid, i1 = i0 + 1;
            const uint32_t c0 = i0 < n ? path_len(S.mv[i0]) + 1u : 0u, c1 = i1 < n ? path_len(S.mv[i1]) + 1u : 0u;
            uint32_t tot;
            const uint32_t ex = block_excl(c0 + c1, S, &tot);
            if (i0 < n) S.inc[i0] = ex;
            if (i1 < n) S.inc[i1] = ex + c0;
            if (tid == 0) S.inc[n] = tot;
        }
        __syncthreads();

        // in-group predecessor sets, nearest candidates first.  A wave per move (moves dealt
        // round-robin to the waves), its lanes testing 64 earlier moves at once: the nearest one
        // whose path meets the move's is kept; of the rest only those whose paths meet the move's
        // but not the kept one's can be kept too -- a lane-parallel filter -- and those few go in
        // order, each kept unless its path meets one already kept.  The same sets as a scan from
        // the nearest down, candidate by candidate.
        for (uint32_t i = (uint32_t)wid; i < n; i += kGWaves) {
            const uint64_t mb = S.mv[i];
            int m1 = -1;
            for (int top = (int)i - 1; top >= 0 && m1 < 0; top -= kWave) {
                const int a = top - lane;
                const bool meet = a >= 0 && paths_meet(S.mv[a], mb);
                const uint64_t mk = ballot(meet);
                if (mk) m1 = top - (__ffsll((unsigned long long)mk) - 1);   // lowest lane: nearest
            }
            uint32_t ps[kMaxPreds];
            uint64_t pc[kMaxPreds];
#pragma unroll
            for (int k = 0; k < kMaxPreds; ++k) { ps[k] = 0u; pc[k] = 0ull; }
            int np = 0;
            bool ovf = false;
            if (m1 >= 0) {
                ps[0] = (uint32_t)m1;
                pc[0] = S.mv[m1];
                np = 1;
                for (int top = m1 - 1; top >= 0 && !ovf; top -= kWave) {
                    const int a = top - lane;
                    bool cand = false;
                    if (a >= 0) {
                        const uint64_t ma = S.mv[a];
                        cand = paths_meet(ma, mb) && !paths_meet(ma, pc[0]);
                    }
                    uint64_t mk = ballot(cand);
                    while (mk) {                                   // nearest first
                        const int l = __ffsll((unsigned long long)mk) - 1;
                        mk &= mk - 1;
                        const int ac = top - l;
                        const uint64_t mac = S.mv[ac];
                        bool red = false;
#pragma unroll
                        for (int k = 1; k < kMaxPreds; ++k)
                            if (k < np && !red) red = paths_meet(pc[k], mac);
                        if (red) continue;
                        if (np == kMaxPreds) { ovf = true; break; }
#pragma unroll
                        for (int k = 1; k < kMaxPreds; ++k)
                            if (k == np) { ps[k] = (uint32_t)ac; pc[k] = mac; }
                        ++np;
                    }
                }
            }
            if (lane == 0) {
                const uint32_t b = lo + i;
                P.pend[b] = (uint32_t)np;
#pragma unroll
                for (int k = 0; k < kMaxPreds; ++k)
                    if (k < np) {
                        P.preds[(size_t)b * kMaxPreds + k] = lo + ps[k];
                        atomic_add_wg(&P.scnt[lo + ps[k]], 1u);
                    }
                if (ovf) S.flags = 1u;
            }
        }
        // the group's traps: read the previous group of each (contiguous chunks of the traps)
        const uint32_t tot = S.inc[n];
        const uint32_t ch = (tot + kGT - 1) / kGT;
        const uint32_t q0 = tid * ch < tot ? tid * ch : tot, q1 = q0 + ch < tot ? q0 + ch : tot;
        int i0 = 0;
        if (q0 < q1) {
            int l = 0, r = (int)n - 1;               // last move with inc <= q0
            while (l < r) {
                const int mid = (l + r + 1) >> 1;
                if (S.inc[mid] <= q0) l = mid; else r = mid - 1;
            }
            i0 = l;
            int i = i0;
            int sx, sy, dx, dy;
            unpack(S.mv[i], sx, sy, dx, dy);
            int len = iabs(dx - sx) + iabs(dy - sy);
            int s = (int)(q0 - S.inc[i]);
            uint32_t lastpg = INV;
            constexpr int kB = 8;                  // traps per round: their loads in flight together
            for (uint32_t q = q0; q < q1; q += kB) {
                uint32_t cell[kB], pg[kB];
#pragma unroll
                for (int u = 0; u < kB; ++u) {
                    cell[u] = INV;
                    if (q + u < q1) {
                        if (s > len) {
                            ++i;
                            s = 0;
                            unpack(S.mv[i], sx, sy, dx, dy);
                            len = iabs(dx - sx) + iabs(dy - sy);
                        }
                        cell[u] = path_trap(W, sx, sy, dx, dy, s);
                        ++s;
                    }
                }
#pragma unroll
                for (int u = 0; u < kB; ++u) pg[u] = cell[u] != INV ? P.lastg[cell[u]] : INV;
#pragma unroll
                for (int u = 0; u < kB; ++u)
                    if (pg[u] != INV && pg[u] != lastpg) {
                        lastpg = pg[u];
                        atomicOr(&S.gb[pg[u] >> 5], 1u << (pg[u] & 31u));
                    }
            }
        }
        __syncthreads();
        // the group's bit row and its count; the groups it waits on count one more waiter
        if (tid < kWave) {
            const uint32_t bits = tid < GW ? S.gb[tid] : 0u;
            if (tid < GW) P.gbits[(size_t)h * GW + tid] = bits;
            const int c = wave_sum(popc((uint64_t)bits));
            if (tid == 0) P.gpend[h] = (uint32_t)c;
            uint32_t m = bits;
            while (m) {
                const uint32_t pg = 32u * tid + (uint32_t)(__ffs((int)m) - 1);
                m &= m - 1u;
                atomic_add_wg(&P.gcnt[pg], 1u);
            }
        }
        // then stamp the traps with this group
        if (q0 < q1) {
            int i = i0;
            int sx, sy, dx, dy;
            unpack(S.mv[i], sx, sy, dx, dy);
            int len = iabs(dx - sx) + iabs(dy - sy);
            int s = (int)(q0 - S.inc[i]);
            for (uint32_t q = q0; q < q1; ++q) {
                if (s > len) {
                    ++i;
                    s = 0;
                    unpack(S.mv[i], sx, sy, dx, dy);
                    len = iabs(dx - sx) + iabs(dy - sy);
                }
                P.lastg[path_trap(W, sx, sy, dx, dy, s)] = h;
                ++s;
            }
        }
        __syncthreads();
    }
    if (S.flags) {
        if (tid == 0) fast::put_info(I.binfo, RR_E_UNSUPPORTED, 0, 0, 0, 0);
        return;
    }

    // ---- successor lists
    scan_ws(P.scnt, K, S);
    for (uint32_t b = tid; b < K; b += kGT) {
        const uint32_t np = P.pend[b];
        for (uint32_t k = 0; k < np; ++k) {
            const uint32_t a = P.preds[(size_t)b * kMaxPreds + k];
            P.slist[P.scnt[a] + atomic_add_wg(&P.sfill[a], 1u)] = b;
        }
    }
    // ---- the groups waiting on each group
    scan_ws(P.gcnt, G, S);
    for (uint32_t h = tid; h < G; h += kGT)
        for (uint32_t w = 0; w < GW; ++w) {
            uint32_t m = P.gbits[(size_t)h * GW + w];
            while (m) {
                const uint32_t pg = 32u * w + (uint32_t)(__ffs((int)m) - 1);
                m &= m - 1u;
                P.glist[P.gcnt[pg] + atomic_add_wg(&P.gfill[pg], 1u)] = h;
            }
        }
    // ---- head moves of every group
    for (uint32_t g = tid; g < G; g += kGT) {
        uint32_t c = 0;
        for (uint32_t b = I.goff[g]; b < I.goff[g + 1]; ++b) c += P.pend[b] == 0u;
        P.hoff[g] = c;
    }
    scan_ws(P.hoff, G, S);
    for (uint32_t g = tid; g < G; g += kGT) {
        uint32_t o = P.hoff[g];
        for (uint32_t b = I.goff[g]; b < I.goff[g + 1]; ++b)
            if (P.pend[b] == 0u) P.heads[o++] = b;
    }
    // ---- release records (the successor lists are complete: scan_ws ended on a barrier)
    for (uint32_t a = tid; a < K; a += kGT) {
        const uint32_t lo = P.scnt[a], ns = P.scnt[a + 1] - lo;
        uint4 r = make_uint4(REC_NONE << 30, 0u, 0u, 0u);
        if (ns == 1u && P.pend[P.slist[lo]] == 1u) {
            const uint32_t s2 = P.slist[lo];
            const uint64_t m = mv64[s2];
            r = make_uint4((REC_DIRECT << 30) | s2, 0u, (uint32_t)m, (uint32_t)(m >> 32));
        } else if (ns > 0u) {
            r.x = REC_LIST << 30;
        }
        P.rec[a] = r;
    }
    if (tid == 0) { P.hdr[H_T] = (uint32_t)T; P.hdr[H_K] = K; P.hdr[H_G] = G; }
    __syncthreads();
    if (tid == 0) P.hdr[H_STATE] = ST_READY;
}

// ------------------------------------------------------------------------------------------
// loop kernel

struct LoopLds {
    uint32_t rc[kRcap], re[kRcap], rn[kRcap], rk[kRcap];   // ready entries, ascending key
    uint32_t nk[kNcap];                                     // keys made ready this trip
    uint32_t npos[kNcap];                                   // their places in the merged set
    uint64_t nmv[kNcap];                                    // their packed moves (0: not known yet)
    uint16_t mlr[kRcap], mlc[kRcap];                        // ready moves on the first one's row /
                                                            // column stepping its way (index order)
    uint32_t gpend[kMaxGroups], grem[kMaxGroups];          // group count-downs
    uint32_t nnew, err;
};

extern __shared__ __attribute__((aligned(16))) uint8_t wide_lds[];

__device__ __forceinline__ uint32_t delta_of(uint32_t d)
{
    return d == 0u ? (1u << 15) : (d == 1u ? (uint32_t)(-(1 << 15)) : (d == 2u ? 1u : 0xFFFFFFFFu));
}

__device__ __forceinline__ uint32_t axis_of(uint32_t c, bool horiz) { return horiz ? (c >> 15) & 0x7FFFu : c & 0x7FFFu; }

// ready entry of move m at its start: current code, end of the first leg, second leg or INV
__device__ __forceinline__ void entry_of(uint64_t m, uint32_t &c, uint32_t &e, uint32_t &nx)
{
    int sx, sy, dx, dy;
    unpack(m, sx, sy, dx, dy);
    if (sx != dx) {
        const uint32_t d = dx > sx ? 0u : 1u;
        c = (d << 30) | ((uint32_t)sx << 15) | (uint32_t)sy;
        e = (d << 30) | ((uint32_t)dx << 15) | (uint32_t)sy;
        nx = dy != sy ? (((dy > sy ? 2u : 3u) << 30) | ((uint32_t)dx << 15) | (uint32_t)dy) : INV;
    } else {
        const uint32_t d = dy > sy ? 2u : 3u;
        c = (d << 30) | ((uint32_t)sx << 15) | (uint32_t)sy;
        e = (d << 30) | ((uint32_t)dx << 15) | (uint32_t)dy;
        nx = INV;
    }
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) {
        const uint32_t o = (uint32_t)__shfl_xor((int)v, m, kWave);
        v = o < v ? o : v;
    }
    return v;
}

__device__ __forceinline__ void push_ready(LoopLds &S, uint32_t key, uint64_t mv)
{
    const uint32_t p = atomicAdd(&S.nnew, 1u);
    if (p < kNcap) { S.nk[p] = key; S.nmv[p] = mv; }
    else S.err = ERR_CAPACITY;
}

// a move ended its path: its successors (one record read for the usual single successor that
// waits on nothing else), and when its group completes the groups waiting on it
__device__ __forceinline__ void release(LoopLds &S, const Ptrs &P, uint32_t key)
{
    const uint32_t b = key >> 11, g = key & 0x7FFu;
    const uint4 r = P.rec[b];
    const uint32_t kind = r.x >> 30;
    if (kind == REC_DIRECT) {
        push_ready(S, ((r.x & 0x3FFFFFFFu) << 11) | g, (uint64_t)r.z | ((uint64_t)r.w << 32));
    } else if (kind == REC_LIST) {
        for (uint32_t t = P.scnt[b], te = P.scnt[b + 1]; t < te; ++t) {
            const uint32_t s2 = P.slist[t];
            if (atomic_sub_wg(&P.pend[s2], 1u) == 1u) push_ready(S, (s2 << 11) | g, 0ull);
        }
    }
    if (atomicSub(&S.grem[g], 1u) == 1u)
        for (uint32_t w = P.gcnt[g], we = P.gcnt[g + 1]; w < we; ++w) {
            const uint32_t h = P.glist[w];
            if (atomicSub(&S.gpend[h], 1u) == 1u)
                for (uint32_t u = P.hoff[h], ue = P.hoff[h + 1]; u < ue; ++u) push_ready(S, (P.heads[u] << 11) | h, 0ull);
        }
}

// sort S.nk[0..nn) ascending, their moves along (bitonic network over the next power of two)
__device__ void sort_keys(LoopLds &S, uint32_t nn)
{
    const uint32_t lane = (uint32_t)lane_id();
    uint32_t P2 = 1;
    while (P2 < nn) P2 <<= 1;
    for (uint32_t i = nn + lane; i < P2; i += kWave) { S.nk[i] = INV; S.nmv[i] = 0ull; }
    wave_sync();
    for (uint32_t k = 2; k <= P2; k <<= 1)
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = lane; i < P2; i += kWave) {
                const uint32_t l = i ^ j;
                if (l > i) {
                    const uint32_t a = S.nk[i], b = S.nk[l];
                    const bool up = (i & k) == 0u;
                    if ((a > b) == up) {
                        const uint64_t ma = S.nmv[i], mb = S.nmv[l];
                        S.nk[i] = b; S.nk[l] = a;
                        S.nmv[i] = mb; S.nmv[l] = ma;
                    }
                }
            }
            wave_sync();
        }
}

// merge the nn keys of S.nk into the n sorted entries (n += nn)
__device__ void merge_new(LoopLds &S, const uint64_t *mv64, uint32_t &n, uint32_t nn)
{
    const uint32_t lane = (uint32_t)lane_id();
    sort_keys(S, nn);
    for (uint32_t k = lane; k < nn; k += kWave) {
        const uint32_t key = S.nk[k];
        uint32_t lo = 0, hi = n;
        while (lo < hi) {
            const uint32_t mid = (lo + hi) >> 1;
            if (S.rk[mid] < key) lo = mid + 1; else hi = mid;
        }
        S.npos[k] = k + lo;
    }
    wave_sync();
    // survivors move up, highest first (a survivor's place never lies below its index); the
    // ones below the smallest new key stay, so the walk stops at the first chunk of those
    for (int base = ((int)n - 1) & ~(kWave - 1); base >= 0; base -= kWave) {
        const uint32_t i = (uint32_t)base + lane;
        const bool v = i < n;
        uint32_t c = 0, e = 0, x = 0, k = 0, pos = 0;
        if (v) {
            c = S.rc[i]; e = S.re[i]; x = S.rn[i]; k = S.rk[i];
            uint32_t lo = 0, hi = nn;
            while (lo < hi) {
                const uint32_t mid = (lo + hi) >> 1;
                if (S.nk[mid] < k) lo = mid + 1; else hi = mid;
            }
            pos = i + lo;
        }
        const bool moves = v && pos != i;
        wave_sync();
        if (moves) { S.rc[pos] = c; S.re[pos] = e; S.rn[pos] = x; S.rk[pos] = k; }
        wave_sync();
        if (ballot(v && pos == i) != 0ull) break;      // this chunk holds the first survivor that stays
    }
    for (uint32_t k = lane; k < nn; k += kWave) {
        const uint32_t key = S.nk[k], p = S.npos[k];
        uint64_t m = S.nmv[k];
        if (m == 0ull) m = mv64[key >> 11];              // a valid move is never all zero
        uint32_t c, e, x;
        entry_of(m, c, e, x);
        S.rc[p] = c; S.re[p] = e; S.rn[p] = x; S.rk[p] = key;
    }
    wave_sync();
    n += nn;
}

// drop the entries whose key is INV, keeping the order; returns the count left.  Entries below
// `from` are all kept and stay where they are.
__device__ uint32_t compact(LoopLds &S, uint32_t n, uint32_t from)
{
    const uint32_t lane = (uint32_t)lane_id();
    uint32_t ns = from & ~(uint32_t)(kWave - 1);
    for (uint32_t base = ns; base < n; base += kWave) {
        const uint32_t i = base + lane;
        const bool keep = i < n && S.rk[i] != INV;
        uint32_t c = 0, e = 0, x = 0, k = 0;
        if (keep) { c = S.rc[i]; e = S.re[i]; x = S.rn[i]; k = S.rk[i]; }
        const uint64_t m = ballot(keep);
        const uint32_t pos = ns + (uint32_t)popc(m & low_mask((int)lane));
        wave_sync();
        if (keep) { S.rc[pos] = c; S.re[pos] = e; S.rn[pos] = x; S.rk[pos] = k; }
        ns += (uint32_t)popc(m);
        wave_sync();
    }
    return ns;
}

template <uint32_t F>
__device__ void loop(const fast::Inst &I, LoopLds &S)
{
    const uint32_t lane = (uint32_t)lane_id();
    const Ptrs P = ptrs_of(I);
    if (P.hdr[H_STATE] != ST_READY) return;
    const uint32_t T = P.hdr[H_T], K = P.hdr[H_K], G = P.hdr[H_G];
    const uint64_t *mv64 = reinterpret_cast<const uint64_t *>(I.moves);
    for (uint32_t g = lane; g < G; g += kWave) {
        S.gpend[g] = P.gpend[g];
        S.grem[g] = I.goff[g + 1] - I.goff[g];
    }
    if (lane == 0) { S.nnew = 0u; S.err = 0u; }
    wave_sync();
    for (uint32_t g = lane; g < G; g += kWave)
        if (S.gpend[g] == 0u)
            for (uint32_t u = P.hoff[g], ue = P.hoff[g + 1]; u < ue; ++u) push_ready(S, (P.heads[u] << 11) | g, 0ull);
    wave_sync();
    uint32_t n = 0;
    {
        const uint32_t nn = S.nnew;
        if (nn > kRcap && lane == 0) S.err = ERR_CAPACITY;
        wave_sync();
        if (S.err == 0u) merge_new(S, mv64, n, nn);
        if (lane == 0) S.nnew = 0u;
        wave_sync();
    }
    uint32_t out = 0, nb = 0, alive = K;
    if (lane == 0) I.boff[0] = 0u;
    while (alive > 0u) {
        if (S.err != 0u) break;
        if (n == 0u || nb >= T) {
            if (lane == 0) S.err = ERR_INTERNAL;
            break;
        }
        // ---- the first ready move
        const uint32_t lc = S.rc[0];
        const uint32_t d1 = lc >> 30;
        const bool horiz = d1 < 2u;
        const uint32_t delta = delta_of(d1);
        const uint32_t ky = lc & MY, kx = lc & MX;
        const uint32_t p1 = axis_of(lc + delta, horiz);

        // ---- one pass over the ready set: the moves stepping its way on its row and on its
        //      column (both lists start with it), the first of them after it (which fixes the
        //      line), and for the convoy the nearest waiting move the sweeping line would reach,
        //      for each choice of line
        uint32_t m = 0;                       // members of the batch
        const uint16_t *ml = S.mlr;           // their places, in index order (unused for NONE)
        uint32_t tv = INV;                    // convoy bound from waiting moves
        if (F == RR_LAMBDA_NONE) {
            m = n;
        } else if (F == RR_LAMBDA_ALONG) {
            const uint32_t M = horiz ? MY : MX, kk = horiz ? ky : kx;
            for (uint32_t base = 0; base < n; base += kWave) {
                const uint32_t e = base + lane;
                const bool acc = e < n && (S.rc[e] & M) == kk;
                const uint64_t b = ballot(acc);
                if (acc) S.mlr[m + (uint32_t)popc(b & low_mask((int)lane))] = (uint16_t)e;
                m += (uint32_t)popc(b);
            }
        } else {
            uint32_t mr = 0, mc = 0, fl = kWave;
            bool found = false, row = horiz;
            uint32_t tA = INV, tR = INV, tC = INV;
            for (uint32_t base = 0; base < n; base += kWave) {
                const uint32_t e = base + lane;
                const bool valid = e < n;
                const uint32_t c = valid ? S.rc[e] : 0u;
                const bool rm = valid && (c & MY) == ky, cm = valid && (c & MX) == kx;
                const uint64_t br = ballot(rm), bc = ballot(cm);
                if (rm) S.mlr[mr + (uint32_t)popc(br & low_mask((int)lane))] = (uint16_t)e;
                if (cm) S.mlc[mc + (uint32_t)popc(bc & low_mask((int)lane))] = (uint16_t)e;
                mr += (uint32_t)popc(br);
                mc += (uint32_t)popc(bc);
                const bool before = !found;   // this chunk's lanes ahead of the first compatible
                fl = kWave;
                const uint64_t comp = (br | bc) & (base == 0u ? ~1ull : ~0ull);
                if (!found && comp) {
                    fl = (uint32_t)__ffsll((unsigned long long)comp) - 1u;
                    found = true;
                    row = ((br >> fl) & 1ull) != 0ull;
                }
                if (valid && e > 0u && (c >> 30) == d1) {
                    const uint32_t p = axis_of(c, horiz);
                    const uint32_t t = (d1 & 1u) ? p1 - p : p - p1;
                    if (before && lane < fl) tA = t < tA ? t : tA;
                    if (!rm) tR = t < tR ? t : tR;
                    if (!cm) tC = t < tC ? t : tC;
                }
            }
            // a waiting move that the sweeping line reaches in t steps would change the batch:
            // along the motion, only those ahead of the first compatible one in index order
            if (!found) {
                m = 1;                        // the first move alone (mlr[0] is it)
                tv = wave_min_u32(tR);
            } else {
                const bool along = row == horiz;
                ml = row ? S.mlr : S.mlc;
                m = row ? mr : mc;
                tv = wave_min_u32(along ? tA : (row ? tR : tC));
            }
        }
        wave_sync();

        // ---- the batch: members step in index order; for up to 64 members, member r's state
        //      stays in lane r for the convoy
        bool arrived = false;
        uint32_t tm = INV, my_c = 0, my_dl = 0, my_e = 0;
        for (uint32_t r0 = 0; r0 < m; r0 += kWave) {
            const uint32_t r = r0 + lane;
            if (r < m) {
                const uint32_t e = F == RR_LAMBDA_NONE ? r : (uint32_t)ml[r];
                const uint32_t c = S.rc[e];
                if (out + r < I.step_cap) I.steps[out + r] = c;
                const uint32_t dl = F == RR_LAMBDA_NONE ? delta_of(c >> 30) : delta;
                const uint32_t c2 = c + dl, ee = S.re[e];
                S.rc[e] = c2;
                const bool h = (c2 >> 30) < 2u;
                const uint32_t a1 = axis_of(ee, h), a2 = axis_of(c2, h);
                const uint32_t rem = a1 > a2 ? a1 - a2 : a2 - a1;
                tm = rem < tm ? rem : tm;
                arrived |= c2 == ee;
                if (r0 == 0u) { my_c = c2; my_dl = dl; my_e = e; }
            }
        }
        bool any = ballot(arrived) != 0ull;
        const uint32_t na = m;
        out += na;
        ++nb;
        if (lane == 0 && nb <= I.batch_cap) I.boff[nb] = out;

        // ---- the convoy: the same batch ts more times
        if (!any) {
            const uint32_t tmin = wave_min_u32(tm);
            const uint32_t ts = tmin < tv ? tmin : tv;
            if (ts > 0u) {
                if ((uint64_t)nb + ts > T || (uint64_t)out + (uint64_t)ts * na > T) {
                    if (lane == 0) S.err = ERR_INTERNAL;
                    break;
                }
                const uint32_t total = ts * na, dj = (uint32_t)kWave / na, dr = (uint32_t)kWave % na;
                uint32_t j = lane / na, r = lane % na;
                if (na <= (uint32_t)kWave) {
                    for (uint32_t q0 = 0; q0 < total; q0 += kWave) {
                        const uint32_t c = (uint32_t)__shfl((int)my_c, (int)r, kWave);
                        const uint32_t dl = (uint32_t)__shfl((int)my_dl, (int)r, kWave);
                        const uint32_t q = q0 + lane;
                        if (q < total && out + q < I.step_cap) I.steps[out + q] = c + j * dl;
                        j += dj;
                        r += dr;
                        if (r >= na) { r -= na; ++j; }
                    }
                } else {
                    for (uint32_t q = lane; q < total; q += kWave) {
                        const uint32_t c = S.rc[F == RR_LAMBDA_NONE ? r : (uint32_t)ml[r]];
                        const uint32_t dl = F == RR_LAMBDA_NONE ? delta_of(c >> 30) : delta;
                        if (out + q < I.step_cap) I.steps[out + q] = c + j * dl;
                        j += dj;
                        r += dr;
                        if (r >= na) { r -= na; ++j; }
                    }
                }
                for (uint32_t jj = lane; jj < ts; jj += kWave)
                    if (nb + jj + 1u <= I.batch_cap) I.boff[nb + jj + 1u] = out + (jj + 1u) * na;
                wave_sync();
                bool arr = false;
                for (uint32_t rr = lane; rr < na; rr += kWave) {
                    const uint32_t e = F == RR_LAMBDA_NONE ? rr : (uint32_t)ml[rr];
                    const uint32_t c = S.rc[e];
                    const uint32_t dl = F == RR_LAMBDA_NONE ? delta_of(c >> 30) : delta;
                    const uint32_t c2 = c + ts * dl;
                    S.rc[e] = c2;
                    arr |= c2 == S.re[e];
                }
                any = ballot(arr) != 0ull;
                out += total;
                nb += ts;
                wave_sync();
            }
        }
        (void)my_e;
        if (!any) continue;

        // ---- legs ended: turn, or finish and release
        uint32_t ndone = 0, first_done = INV;
        for (uint32_t r0 = 0; r0 < na; r0 += kWave) {
            const uint32_t rr = r0 + lane;
            bool done = false;
            uint32_t key = 0;
            if (rr < na) {
                const uint32_t e = F == RR_LAMBDA_NONE ? rr : (uint32_t)ml[rr];
                const uint32_t c = S.rc[e];
                if (c == S.re[e]) {
                    const uint32_t nx = S.rn[e];
                    if (nx != INV) {
                        S.rc[e] = (c & 0x3FFFFFFFu) | (nx & 0xC0000000u);
                        S.re[e] = nx;
                        S.rn[e] = INV;
                    } else {
                        done = true;
                        key = S.rk[e];
                        S.rk[e] = INV;
                        first_done = e < first_done ? e : first_done;
                    }
                }
            }
            if (done) release(S, P, key);
            ndone += (uint32_t)popc(ballot(done));
        }
        first_done = wave_min_u32(first_done);
        wave_sync();
        if (ndone == 0u) continue;
        alive -= ndone;
        n = compact(S, n, first_done);
        const uint32_t nn = S.nnew;
        if (S.err != 0u) break;
        if (n + nn > kRcap) {
            if (lane == 0) S.err = ERR_CAPACITY;
            break;
        }
        if (nn) {
            merge_new(S, mv64, n, nn);
            if (lane == 0) S.nnew = 0u;
            wave_sync();
        }
    }
    wave_sync();
    if (lane == 0) {
        const uint32_t er = S.err;
        const int st = er == ERR_CAPACITY ? RR_E_UNSUPPORTED
                                          : (er != 0u ? RR_E_INTERNAL : (nb > I.batch_cap ? RR_E_CAPACITY : RR_OK));
        const bool ok = st == RR_OK;
        fast::put_info(I.binfo, st, ok ? nb : 0u, ok ? out : 0u, nb, T);
    }
}

// ------------------------------------------------------------------------------------------
// kernels

__device__ __forceinline__ bool shape_ok(const rr_shape s, int maxw, int maxh)
{
    return s.w <= maxw && s.h <= maxh && s.w <= RR_MAX_SIDE && s.h <= RR_MAX_SIDE && s.x0 < s.x1 && s.x1 <= s.w &&
           s.y0 < s.y1 && s.y1 <= s.h;
}

__device__ __forceinline__ bool region_ok(const rr_desc &d, uint64_t ws_bytes)
{
    const uint64_t need = layout(d.shape.w, d.shape.h, d.move_cap).total;
    return (d.ws_off & 255u) == 0 && d.ws_off <= ws_bytes && need <= ws_bytes - d.ws_off;
}

__global__ __launch_bounds__(kGT) void k_wide_graph_one(fast::Inst I)
{
    __shared__ GraphShared S;
    graph(I, S);
}

__global__ __launch_bounds__(kGT) void k_wide_graph_many(const rr_desc *__restrict__ desc, int maxw, int maxh,
                                                         const rr_move *mv, const uint32_t *ga,
                                                         const rr_solve_info *sinfos, uint32_t *bat, uint32_t *stp,
                                                         rr_batch_info *binfos, uint8_t *ws, uint64_t ws_bytes)
{
    __shared__ GraphShared S;
    const uint32_t i = blockIdx.x;
    const rr_desc d = desc[i];
    if (!wide_shape(d.shape.w, d.shape.h)) return;              // the smaller grids' kernels take it
    const bool sok = shape_ok(d.shape, maxw, maxh), room = d.step_cap != 0xFFFFFFFFu;
    if (!sok || !room || !region_ok(d, ws_bytes)) {
        if (threadIdx.x == 0) {
            const rr_solve_info si = sinfos[i];
            if (!sok || (room && !region_ok(d, ws_bytes)))
                fast::put_info(binfos + i, RR_E_INVAL, 0, 0, 0, 0);
            else if (si.status == RR_INFEASIBLE || (si.status == RR_OK && si.n_moves == 0))
                fast::put_info(binfos + i, RR_OK, 0, 0, 0, 0);
            else if (si.status == RR_OK)
                fast::put_info(binfos + i, RR_E_CAPACITY, 0, 0, si.n_steps, si.n_steps);
            else
                fast::put_info(binfos + i, RR_E_INVAL, 0, 0, 0, 0);
        }
        return;
    }
    graph(inst_of(d, i, mv, ga, sinfos, bat, stp, binfos, ws), S);
}

template <uint32_t F>
__global__ __launch_bounds__(kWave) void k_wide_loop_one(fast::Inst I)
{
    loop<F>(I, *reinterpret_cast<LoopLds *>(wide_lds));
}

template <uint32_t F>
__global__ __launch_bounds__(kWave) void k_wide_loop_many(const rr_desc *__restrict__ desc, int maxw, int maxh,
                                                          const rr_move *mv, const uint32_t *ga,
                                                          const rr_solve_info *sinfos, uint32_t *bat, uint32_t *stp,
                                                          rr_batch_info *binfos, uint8_t *ws, uint64_t ws_bytes)
{
    const uint32_t i = blockIdx.x;
    const rr_desc d = desc[i];
    if (!wide_shape(d.shape.w, d.shape.h) || !shape_ok(d.shape, maxw, maxh) || d.step_cap == 0xFFFFFFFFu ||
        !region_ok(d, ws_bytes))
        return;
    loop<F>(inst_of(d, i, mv, ga, sinfos, bat, stp, binfos, ws), *reinterpret_cast<LoopLds *>(wide_lds));
}

// ------------------------------------------------------------------------------------------
// host launchers

hipError_t launch_one(const fast::Inst &I, uint32_t flags, hipStream_t st)
{
    hipLaunchKernelGGL(k_wide_graph_one, dim3(1), dim3(kGT), 0, st, I);
    const size_t lds = sizeof(LoopLds);
    switch (flags & 0xFFu) {
    case RR_LAMBDA_LINE_OR_COL: hipLaunchKernelGGL(k_wide_loop_one<RR_LAMBDA_LINE_OR_COL>, dim3(1), dim3(kWave), lds, st, I); break;
    case RR_LAMBDA_ALONG: hipLaunchKernelGGL(k_wide_loop_one<RR_LAMBDA_ALONG>, dim3(1), dim3(kWave), lds, st, I); break;
    default: hipLaunchKernelGGL(k_wide_loop_one<RR_LAMBDA_NONE>, dim3(1), dim3(kWave), lds, st, I); break;
    }
    return hipGetLastError();
}

hipError_t launch_graph_many(uint32_t n, const rr_desc *desc, int maxw, int maxh, const rr_move *mv,
                             const uint32_t *ga, const rr_solve_info *sinfos, uint32_t *bat, uint32_t *stp,
                             rr_batch_info *binfos, uint8_t *ws, uint64_t ws_bytes, hipStream_t st)
{
    hipLaunchKernelGGL(k_wide_graph_many, dim3(n), dim3(kGT), 0, st, desc, maxw, maxh, mv, ga, sinfos, bat, stp,
                       binfos, ws, ws_bytes);
    return hipGetLastError();
}

hipError_t launch_loop_many(uint32_t n, const rr_desc *desc, int maxw, int maxh, const rr_move *mv,
                            const uint32_t *ga, const rr_solve_info *sinfos, uint32_t *bat, uint32_t *stp,
                            rr_batch_info *binfos, uint8_t *ws, uint64_t ws_bytes, uint32_t flags, hipStream_t st)
{
    const size_t lds = sizeof(LoopLds);
#define RR_WIDE_LOOP(FF)                                                                                           \
    hipLaunchKernelGGL(k_wide_loop_many<FF>, dim3(n), dim3(kWave), lds, st, desc, maxw, maxh, mv, ga, sinfos, bat,  \
                       stp, binfos, ws, ws_bytes)
    switch (flags & 0xFFu) {
    case RR_LAMBDA_LINE_OR_COL: RR_WIDE_LOOP(RR_LAMBDA_LINE_OR_COL); break;
    case RR_LAMBDA_ALONG: RR_WIDE_LOOP(RR_LAMBDA_ALONG); break;
    default: RR_WIDE_LOOP(RR_LAMBDA_NONE); break;
    }
#undef RR_WIDE_LOOP
    return hipGetLastError();
}

}  // namespace wide
}  // namespace rr
