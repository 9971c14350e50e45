// rr_batch_loop.hpp -- the iterations of the batching routine (arXiv 2504.06182, §IV, Alg. 3)
// on the fast path: one wave64 per instance, the ready set in registers.
//
// Alg. 3 takes, in each iteration, the moves whose Gamma-predecessors are all done (the ready
// set), in ascending move index, and adds each one's next unit step to the batch when it is
// vertex-disjoint from the steps already taken and satisfies the local constraint with each of
// them.  Ready moves never share a trap (two that did would be ordered in Gamma), so the
// disjointness test never rejects.  With the deployed constraint (same direction, current traps
// on one row or one column) the batch is: the first ready move (the leader), plus every ready
// move stepping the same way on the row or the column of the leader's trap -- whichever line
// holds the next compatible ready move in index order.
//
// Ready set.  Entries sit in S register slots per lane, at positions p = 64*slot + lane, in
// ascending move index with holes; a 64-bit mask per slot marks the valid ones.  An entry is
// four words: current trap and direction packed as the output step code (dir << 30 | x << 15 |
// y), the code the current leg ends on, the end code of the vertical leg still to come (or
// none), and the key idx << 10 | group.  Batches are found with ballots: two masked compares per
// slot give the moves on the leader's row and column, the first set bit in slot order picks
// the line, and output positions are prefix popcounts, so the steps of a batch are written in
// index order with one store.
//
// Convoys.  After a batch, nothing changes until some member ends its leg or a waiting move
// comes onto the line that sweeps with the leader (its column on a horizontal leg, its row on a
// vertical one), so the same members keep stepping together: the batch repeats.  The repeat
// count is the smaller of the members' remaining leg lengths and the distance to the first
// waiting move on the sweeping line that would change the batch (any one when the batch is the
// leader alone or runs across the motion, one ordered before the first other member when it
// runs along it), one DPP wave minimum; the repeats are written in one go.  On the 64x64
// workload this turns ~10k batches into ~1.9k trips of the loop.  While the ready set fits one
// slot (the common case) the trip runs on slot 0 alone.
//
// Completions.  A finished move leaves a hole.  Its release code (LDS) gives its successor:
// the common case -- one successor waiting on nothing else -- takes the finished move's place
// when no ready index lies between them, else any hole between its neighbours in index order,
// else the ready set is compacted through LDS.  General successor lists and wait counts live in
// the workspace.  When the last move of a group finishes, the groups waiting on it are counted
// down in parallel and the head moves of those that reach zero join the ready set.
#pragma once
#include "rr_batch_graph.hpp"

namespace rr {
namespace fast {

constexpr uint32_t kInv = 0xFFFFFFFFu;
constexpr uint32_t kMaskY = 0xC00001FFu;                  // direction + 9-bit row field
constexpr uint32_t kMaskX = 0xC0000000u | (0x1FFu << 15); // direction + 9-bit column field

__device__ __forceinline__ uint32_t step_delta(uint32_t d)
{
    return d == 0u ? (1u << 15) : (d == 1u ? (uint32_t)(-(1 << 15)) : (d == 2u ? 1u : 0xFFFFFFFFu));
}

// entry words of a move from its packed coordinates sx | sy << 8 | dx << 16 | dy << 24
__device__ __forceinline__ void entry_of(uint32_t m, uint32_t &c, uint32_t &e, uint32_t &n)
{
    const uint32_t sx = m & 0xFFu, sy = (m >> 8) & 0xFFu, dx = (m >> 16) & 0xFFu, dy = m >> 24;
    if (sx != dx) {
        const uint32_t d = dx > sx ? 0u : 1u;
        c = (d << 30) | (sx << 15) | sy;
        e = (d << 30) | (dx << 15) | sy;
        n = dy != sy ? (((dy > sy ? 2u : 3u) << 30) | (dx << 15) | dy) : kInv;
    } else {
        const uint32_t d = dy > sy ? 2u : 3u;
        c = (d << 30) | (sx << 15) | sy;
        e = (d << 30) | (dx << 15) | dy;
        n = kInv;
    }
}

__device__ __forceinline__ uint32_t rdl(uint32_t v, int l) { return (uint32_t)__builtin_amdgcn_readlane((int)v, l); }
__device__ __forceinline__ uint32_t wrl(uint32_t v, int l, uint32_t old) { return lane_id() == l ? v : old; }
__device__ __forceinline__ uint32_t rfl(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }
__device__ __forceinline__ uint32_t mbcnt(uint64_t m)
{
    return __builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}
__device__ __forceinline__ int ffs64(uint64_t m) { return __ffsll((unsigned long long)m) - 1; }
__device__ __forceinline__ int fls64(uint64_t m) { return 63 - __clzll((unsigned long long)m); }

// loop data of one instance (LDS when it fits the launch's budget, else the workspace)
struct LoopMem {
    const uint32_t *mv;
    const uint16_t *nx;
    uint32_t *grem, *gpend;
    const uint16_t *gloff, *gl, *hdoff, *hd;
    const uint32_t *soff, *slist;
    uint32_t *pend;
    uint4 *scratch;
};

template <int S>
struct Ready {
    uint32_t c[S], e[S], n[S], k[S];
    uint64_t vm[S];
};

template <int S>
__device__ __forceinline__ void put_entry(Ready<S> &R, int s, int l, uint32_t c, uint32_t e, uint32_t n, uint32_t k)
{
#pragma unroll
    for (int i = 0; i < S; ++i)
        if (i == s) {
            R.c[i] = wrl(c, l, R.c[i]);
            R.e[i] = wrl(e, l, R.e[i]);
            R.n[i] = wrl(n, l, R.n[i]);
            R.k[i] = wrl(k, l, R.k[i]);
            R.vm[i] |= 1ull << l;
        }
}

// Compact the ready set through LDS scratch, adding one entry at its place in index order.
// Returns false when the set would exceed 64*S entries.
template <int S>
__device__ __forceinline__ bool merge_insert(Ready<S> &R, uint4 *scr, uint32_t c0, uint32_t e0, uint32_t n0, uint32_t k0)
{
    const int lane = lane_id();
    uint32_t total = 1;
#pragma unroll
    for (int s = 0; s < S; ++s) total += (uint32_t)popc(R.vm[s]);
    if (total > (uint32_t)(kWave * S)) return false;
    uint32_t base = 0, nlt = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const uint64_t v = R.vm[s];
        nlt += (uint32_t)popc(ballot(R.k[s] < k0) & v);
        if ((v >> lane) & 1ull) {
            const uint32_t r = base + mbcnt(v) + (R.k[s] > k0 ? 1u : 0u);
            scr[r] = make_uint4(R.c[s], R.e[s], R.n[s], R.k[s]);
        }
        base += (uint32_t)popc(v);
    }
    if (lane == 0) scr[nlt] = make_uint4(c0, e0, n0, k0);
    wave_sync();
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const uint32_t p = (uint32_t)(s * kWave + lane);
        const bool v = p < total;
        const uint4 q = v ? scr[p] : make_uint4(kInv, kInv, kInv, kInv);
        R.c[s] = q.x; R.e[s] = q.y; R.n[s] = q.z; R.k[s] = q.w;
        R.vm[s] = ballot(v);
    }
    wave_sync();
    return true;
}

// Add ready move b (group g).  (ps, pl) is the slot/lane of the move that released it (a hole
// now) or ps < 0.  Returns false on overflow (cannot happen when the ready-set bound holds).
// NS: slots that may hold entries (slots NS.. are empty when NS < S; checked here, so that an
// earlier insertion of the same release that went beyond slot NS-1 is seen).
template <int NS, int S>
__device__ __forceinline__ bool insert_ready(Ready<S> &R, const LoopMem &M, uint32_t b, uint32_t g, int ps, int pl,
                                             bool &moved)
{
    if (NS < S) {
        uint64_t high = 0;
#pragma unroll
        for (int s = NS; s < S; ++s) high |= R.vm[s];
        if (high) return insert_ready<S, S>(R, M, b, g, ps, pl, moved);
    }
    uint32_t c0, e0, n0;
    entry_of(rfl(M.mv[b]), c0, e0, n0);
    const uint32_t k0 = (b << 10) | g;
    int lo = -1, hi = kWave * NS;               // with NS < S, position 64*NS starts the empty slots
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const uint64_t v = R.vm[s];
        if (v) {
            const uint64_t lt = ballot(R.k[s] < k0) & v, gt = v & ~lt;
            if (lt) lo = s * kWave + fls64(lt);
            if (gt && hi == kWave * NS) hi = s * kWave + ffs64(gt);
        }
    }
    int pos = -1;
    if (ps >= 0 && ps < NS) {
        const int pp = ps * kWave + pl;
        uint64_t hv = 0;
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (s == ps) hv = R.vm[s];
        if (lo < pp && pp < hi && !((hv >> pl) & 1ull)) pos = pp;
    }
    if (pos < 0 && hi - lo > 1) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (pos >= 0) continue;
            const int a = lo + 1 - s * kWave, z = hi - 1 - s * kWave;
            const uint64_t holes = ~R.vm[s] & range_mask(a, z);
            if (holes) pos = s * kWave + ffs64(holes);
        }
    }
    if (NS < S && pos < 0 && hi == kWave * NS) pos = kWave * NS;   // after every entry: first empty slot
    if (pos >= 0) {
        put_entry(R, pos / kWave, pos % kWave, c0, e0, n0, k0);
        return true;
    }
    moved = true;
    return merge_insert(R, M.scratch, c0, e0, n0, k0);
}

// Successors of finished move b (group g) -- unless the caller placed it already -- and, when b
// was its group's last move (group_done: the caller counted the group down), the groups waiting
// on that group.
template <int NS, int S>
__device__ __forceinline__ bool release_move(Ready<S> &R, const LoopMem &M, uint32_t b, uint32_t g, int ps, int pl, bool &moved,
                                             bool successors, bool group_done)
{
    const int lane = lane_id();
    bool ok = true;
    const uint32_t code = successors ? rfl(M.nx[b]) : 0u;
    const uint32_t kind = code >> 14;
    if (kind == kRelNext) {
        ok &= insert_ready<NS, S>(R, M, b + (code & kMaxDelta), g, ps, pl, moved);
    } else if (kind == kRelList) {
        const uint32_t lo = rfl(M.soff[b]), hi = rfl(M.soff[b + 1]);
        for (uint32_t t = lo; t < hi; ++t) {
            const uint32_t nx = rfl(M.slist[t]);
            uint32_t old = 0;
            if (lane == 0) old = M.pend[nx]--;
            old = rfl(old);
            if (old == 1u) ok &= insert_ready<NS, S>(R, M, nx, g, ps, pl, moved);
        }
    }
    if (group_done) {
        const uint32_t lo = rfl(M.gloff[g]), hi = rfl(M.gloff[g + 1]);
        for (uint32_t t0 = lo; t0 < hi; t0 += kWave) {
            const uint32_t t = t0 + lane;
            uint32_t h = 0;
            bool zero = false;
            if (t < hi) {                       // distinct groups: one lane each
                h = M.gl[t];
                zero = M.gpend[h]-- == 1u;
            }
            uint64_t zm = ballot(zero);
            while (zm) {
                const int l = ffs64(zm);
                zm &= zm - 1;
                const uint32_t hh = rdl(h, l);
                const uint32_t ulo = rfl(M.hdoff[hh]), uhi = rfl(M.hdoff[hh + 1]);
                for (uint32_t u = ulo; u < uhi; ++u)
                    ok &= insert_ready<NS, S>(R, M, rfl(M.hd[u]), hh, -1, -1, moved);
            }
        }
    }
    return ok;
}


template <int S>
__device__ __forceinline__ void find_leader(const Ready<S> &R, int &ls, int &ll, uint32_t &lc, uint32_t &le,
                                            uint32_t &ln, uint32_t &lk)
{
    ls = -1; ll = 0;
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (ls < 0 && R.vm[s]) { ls = s; ll = ffs64(R.vm[s]); }
    lc = le = ln = lk = kInv;
#pragma unroll
    for (int s = 0; s < S; ++s)
        if (s == ls) { lc = rdl(R.c[s], ll); le = rdl(R.e[s], ll); ln = rdl(R.n[s], ll); lk = rdl(R.k[s], ll); }
}

// Minimum of one value per lane, uniform: DPP prefix minimum inside each 16-lane row, row
// broadcasts to lane 63, then a read of lane 63 (no LDS traffic).
__device__ __forceinline__ uint32_t wave_min_dpp(uint32_t v)
{
    auto m = [](uint32_t a, uint32_t b) { return a < b ? a : b; };
    v = m(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x111, 0xF, 0xF, false));   // row_shr:1
    v = m(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x112, 0xF, 0xF, false));   // row_shr:2
    v = m(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x114, 0xF, 0xF, false));   // row_shr:4
    v = m(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x118, 0xF, 0xF, false));   // row_shr:8
    v = m(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x142, 0xA, 0xF, false));   // row_bcast:15
    v = m(v, (uint32_t)__builtin_amdgcn_update_dpp((int)v, (int)v, 0x143, 0xC, 0xF, false));   // row_bcast:31
    return rdl(v, kWave - 1);
}

// position of a step code along the axis of a leg (column for a horizontal leg, row else)
__device__ __forceinline__ uint32_t axis_pos(uint32_t c, bool horiz) { return horiz ? (c >> 15) & 0x1FFu : c & 0x1FFu; }

// Scalar state of the loop (kept in SGPRs).
struct LoopCtx {
    uint32_t alive, out, nb, T;
    int ls, ll;                 // leader position
    uint32_t lc, le, ln, lk;    // leader entry
    uint32_t err;               // kNoErr, kOverflow (the general path takes over) or kBroken
};

enum : uint32_t { kNoErr = 0, kOverflow = 1, kBroken = 2 };

// Compact the ready set into the lowest positions through LDS scratch (index order kept).
template <int S>
__device__ __forceinline__ void compact(Ready<S> &R, uint4 *scr)
{
    const int lane = lane_id();
    uint32_t base = 0;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const uint64_t v = R.vm[s];
        if ((v >> lane) & 1ull) scr[base + mbcnt(v)] = make_uint4(R.c[s], R.e[s], R.n[s], R.k[s]);
        base += (uint32_t)popc(v);
    }
    wave_sync();
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const uint32_t p = (uint32_t)(s * kWave + lane);
        const bool v = p < base;
        const uint4 q = v ? scr[p] : make_uint4(kInv, kInv, kInv, kInv);
        R.c[s] = q.x; R.e[s] = q.y; R.n[s] = q.z; R.k[s] = q.w;
        R.vm[s] = ballot(v);
    }
    wave_sync();
}

// One trip of the loop over the first NS slots (the others are empty when NS < S): a batch --
// the leader alone, or the leader and the ready moves stepping its way on its row or column --
// then the same batch repeated while it stays the batch Alg. 3 would pick (the convoy), then
// the legs that ended turn or finish and the finished moves release their successors.
template <int NS, int S, uint32_t flags>
__device__ __forceinline__ void trip(Ready<S> &R, LoopCtx &X, const Inst &I, const LoopMem &M)
{
    const int lane = lane_id();
    const uint32_t d1 = X.lc >> 30;
    const uint32_t delta = step_delta(d1);
    const bool horiz = d1 < 2u;
    const uint64_t lbit = 1ull << X.ll;
    uint64_t acc[NS];
    bool along = false;
    uint32_t amin = kInv;                       // key of the first member after the leader
    if (flags == RR_LAMBDA_NONE) {
#pragma unroll
        for (int s = 0; s < NS; ++s) acc[s] = R.vm[s];
    } else {
        const uint32_t ky = X.lc & kMaskY, kx = X.lc & kMaskX;
        const bool use_row = flags != RR_LAMBDA_ALONG || horiz;
        const bool use_col = flags != RR_LAMBDA_ALONG || !horiz;
        bool found = false, row = false;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            if (found || !R.vm[s]) continue;
            uint64_t mr = use_row ? ballot((R.c[s] & kMaskY) == ky) : 0ull;
            uint64_t mc = use_col ? ballot((R.c[s] & kMaskX) == kx) : 0ull;
            if (s == X.ls) { mr &= ~lbit; mc &= ~lbit; }
            if (mr | mc) {
                found = true;
                row = (mr >> ffs64(mr | mc)) & 1ull;
            }
        }
        if (found) {
            along = row == horiz;
            const uint32_t km = row ? kMaskY : kMaskX, kv = row ? ky : kx;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                acc[s] = R.vm[s] ? ballot((R.c[s] & km) == kv) : 0ull;
                if (along && amin == kInv) {
                    const uint64_t m = s == X.ls ? acc[s] & ~lbit : acc[s];
                    if (m) amin = rdl(R.k[s], ffs64(m));
                }
            }
        } else {
#pragma unroll
            for (int s = 0; s < NS; ++s) acc[s] = 0;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s)
            if (s == X.ls) acc[s] |= lbit;
    }

    // ---- the batch: members store their step codes in index order and step
    uint32_t base = 0;
    uint64_t arr[NS];
    bool any_arr = false;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        arr[s] = 0;
        const uint64_t a = acc[s];
        if (!a) continue;
        const bool me = (a >> lane) & 1ull;
        const uint32_t at = X.out + base + mbcnt(a);
        if (me) {
            if (at < I.step_cap) I.steps[at] = R.c[s];
            R.c[s] += flags == RR_LAMBDA_NONE ? step_delta(R.c[s] >> 30) : delta;
        }
        arr[s] = ballot(me && R.c[s] == R.e[s]);
        any_arr |= arr[s] != 0ull;
        base += (uint32_t)popc(a);
    }
    X.out += base;
    ++X.nb;
    if (lane == 0 && X.nb <= I.batch_cap) I.boff[X.nb] = X.out;
    X.lc += delta;

    // ---- the convoy: the same members step again until one ends its leg, or until a waiting
    //      move on the line that sweeps with the leader would change the batch
    if (!any_arr) {
        uint32_t tv = 1u << 20;
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const uint64_t a = acc[s];
            if (!a) continue;
            if ((a >> lane) & 1ull) {
                const bool h = (R.c[s] >> 30) < 2u;
                const uint32_t pc = axis_pos(R.c[s], h), pe = axis_pos(R.e[s], h);
                const uint32_t rem = pc > pe ? pc - pe : pe - pc;
                tv = rem < tv ? rem : tv;
            }
        }
        if (flags == RR_LAMBDA_LINE_OR_COL) {
            const uint32_t p1 = axis_pos(X.lc, horiz);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const uint64_t waiting = R.vm[s] & ~acc[s];
                if (!waiting) continue;
                const uint32_t c = R.c[s];
                const uint32_t p = axis_pos(c, horiz);
                const uint32_t t = (d1 & 1u) ? p1 - p : p - p1;          // wraps when behind
                const bool blk = ((waiting >> lane) & 1ull) && (c >> 30) == d1 && (!along || R.k[s] < amin);
                tv = blk && t < tv ? t : tv;
            }
        }
        const uint32_t ts = wave_min_dpp(tv);
        if (ts > 0) {
            // the members' codes go to LDS in rank order; then the ts x base new steps are
            // written lane-parallel in output order: entry i is repeat i / base of member i % base
            uint32_t *sc = (uint32_t *)M.scratch;
            uint32_t rb = 0;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const uint64_t a = acc[s];
                if (!a) continue;
                if ((a >> lane) & 1ull) sc[rb + mbcnt(a)] = R.c[s];
                rb += (uint32_t)popc(a);
            }
            wave_sync();
            const uint32_t total = ts * base;
            const float inv = 1.0f / (float)base;
            for (uint32_t i0 = 0; i0 < total; i0 += kWave) {
                const uint32_t i = i0 + (uint32_t)lane;
                if (i < total) {
                    uint32_t j = (uint32_t)((float)i * inv);          // i / base, give or take one
                    while (j * base > i) --j;
                    while ((j + 1) * base <= i) ++j;
                    const uint32_t v = sc[i - j * base];
                    const uint32_t dl = flags == RR_LAMBDA_NONE ? step_delta(v >> 30) : delta;
                    const uint32_t at = X.out + i;
                    if (at < I.step_cap) I.steps[at] = v + j * dl;
                }
            }
            wave_sync();
            for (uint32_t j = lane; j < ts; j += kWave)
                if (X.nb + 1 + j <= I.batch_cap) I.boff[X.nb + 1 + j] = X.out + (j + 1) * base;
            X.out += ts * base;
            X.nb += ts;
            X.lc += ts * delta;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const uint64_t a = acc[s];
                if (!a) continue;
                const bool me = (a >> lane) & 1ull;
                if (me) R.c[s] += ts * (flags == RR_LAMBDA_NONE ? step_delta(R.c[s] >> 30) : delta);
                arr[s] = ballot(me && R.c[s] == R.e[s]);
                any_arr |= arr[s] != 0ull;
            }
        }
    }
    if (!any_arr) return;

    // ---- legs ended: turn onto the vertical leg, or finish
    uint64_t done[NS];
    uint32_t ndone = 0;
    bool ldone = false;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        done[s] = 0;
        if (!arr[s]) continue;
        const bool me = (arr[s] >> lane) & 1ull;
        const bool turn = me && R.n[s] != kInv;
        done[s] = ballot(me && !turn);
        if (turn) {
            R.c[s] = (R.c[s] & 0x3FFFFFFFu) | (R.n[s] & 0xC0000000u);
            R.e[s] = R.n[s];
            R.n[s] = kInv;
        }
        if (s == X.ls && ((arr[s] >> X.ll) & 1ull)) {
            if ((done[s] >> X.ll) & 1ull) ldone = true;
            else { X.lc = (X.lc & 0x3FFFFFFFu) | (X.ln & 0xC0000000u); X.le = X.ln; X.ln = kInv; }
        }
        ndone += (uint32_t)popc(done[s]);
    }
    if (ndone == 0) return;

    // ---- finished moves release what waited on them.  The common release -- the next move
    //      index, waiting on nothing else -- takes the finished move's position (no index lies
    //      between them); the others leave a hole and go through the general insertion.
    uint32_t dk[NS];
    uint64_t slow[NS];
    bool any_slow = false;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        slow[s] = 0;
        if (!done[s]) continue;
        dk[s] = R.k[s];
        // every finished lane of the slot reads its release code and the next move at once
        const bool me = (done[s] >> lane) & 1ull;
        uint32_t code = 0, nm = 0;
        if (me) {
            const uint32_t b = R.k[s] >> 10;
            code = M.nx[b];
            nm = M.mv[b + 1];                   // the array holds move_cap + 1 words
        }
        const bool fast = me && code == ((kRelNext << 14) | 1u);
        if (fast) {
            uint32_t c0, e0, n0;
            entry_of(nm, c0, e0, n0);
            R.c[s] = c0; R.e[s] = e0; R.n[s] = n0; R.k[s] += 1u << 10;
        }
        slow[s] = ballot(me && !fast);
        if (s == X.ls && ((done[s] & ~slow[s]) >> X.ll) & 1ull) {
            X.lc = rdl(R.c[s], X.ll); X.le = rdl(R.e[s], X.ll); X.ln = rdl(R.n[s], X.ll); X.lk = rdl(R.k[s], X.ll);
            ldone = false;
        }
        if (slow[s]) {
            if ((slow[s] >> lane) & 1ull) { R.c[s] = kInv; R.k[s] = kInv; }
            R.vm[s] &= ~slow[s];
            any_slow = true;
        }
    }
    X.alive -= ndone;
    // every finished lane counts its group down at once; the last one of a group frees the
    // groups waiting on it
    uint64_t gdone[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        gdone[s] = 0;
        if (!done[s]) continue;
        const bool me = (done[s] >> lane) & 1ull;
        uint32_t old = 0;
        if (me) old = __hip_atomic_fetch_sub(&M.grem[dk[s] & 0x3FFu], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        gdone[s] = ballot(me && old == 1u);
    }
    bool moved = false, ok = true;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        uint64_t m = slow[s] | gdone[s];
        while (m) {
            const int l = ffs64(m);
            m &= m - 1;
            const uint32_t kk = rdl(dk[s], l);
            ok &= release_move<NS, S>(R, M, kk >> 10, kk & 0x3FFu, s, l, moved, ((slow[s] >> l) & 1ull) != 0,
                                      ((gdone[s] >> l) & 1ull) != 0);
        }
    }
    (void)any_slow;
    if (!ok) { X.err = kOverflow; return; }
    // keep the set in as few slots as it fits (1; with 5 or more slots also 2; with 6 or more, 4) so
    // that trips scan only those
    if (S > 1) {
        uint32_t total = 0;
        uint64_t h1 = 0, h2 = 0, h4 = 0;
#pragma unroll
        for (int s = 0; s < S; ++s) {
            total += (uint32_t)popc(R.vm[s]);
            if (s >= 1) h1 |= R.vm[s];
            if (s >= 2) h2 |= R.vm[s];
            if (s >= 4) h4 |= R.vm[s];
        }
        const bool c1 = h1 && total <= (uint32_t)kWave;
        const bool c2 = S >= 5 && h2 && total <= 2u * kWave;
        const bool c4 = S >= 6 && h4 && total <= 4u * kWave;
        if (c1 || c2 || c4) { compact(R, M.scratch); moved = true; }
    }
    if (ldone || moved) find_leader(R, X.ls, X.ll, X.lc, X.le, X.ln, X.lk);
}

// Alg. 3 iterations of one instance over its loop data M.  Returns true when the ready set
// outgrew the 64*S register positions: nothing is reported then, the general path redoes the
// instance from its inputs.
template <int S, uint32_t flags>
__device__ __forceinline__ bool loop_run(const Inst &I, const LoopMem &M, uint32_t K, uint32_t G, uint32_t T)
{
    const int lane = lane_id();
    // ---- initial ready set: head moves of the groups that wait on nothing, in index order
    Ready<S> R;
    uint32_t n0 = 0;
    for (uint32_t g0 = 0; g0 < G; g0 += kWave) {
        const uint32_t g = g0 + lane;
        uint32_t cnt = 0;
        if (g < G && M.gpend[g] == 0u) cnt = (uint32_t)(M.hdoff[g + 1] - M.hdoff[g]);
        const uint32_t inc = (uint32_t)wave_incl_scan((int)cnt);
        uint32_t at = n0 + inc - cnt;
        for (uint32_t u = 0; u < cnt && at < (uint32_t)(kWave * S); ++u, ++at) {
            const uint32_t b = M.hd[M.hdoff[g] + u];
            uint32_t c, e, n;
            entry_of(M.mv[b], c, e, n);
            M.scratch[at] = make_uint4(c, e, n, (b << 10) | g);
        }
        n0 += rfl((uint32_t)__shfl((int)inc, kWave - 1, kWave));
    }
    wave_sync();
    LoopCtx X;
    X.err = n0 > (uint32_t)(kWave * S) ? kOverflow : kNoErr;
#pragma unroll
    for (int s = 0; s < S; ++s) {
        const uint32_t p = (uint32_t)(s * kWave + lane);
        const bool v = !X.err && p < n0;
        const uint4 q = v ? M.scratch[p] : make_uint4(kInv, kInv, kInv, kInv);
        R.c[s] = q.x; R.e[s] = q.y; R.n[s] = q.z; R.k[s] = q.w;
        R.vm[s] = ballot(v);
    }
    wave_sync();

    X.alive = X.err ? 0u : K;
    X.out = 0;
    X.nb = 0;
    X.T = T;
    if (lane == 0) I.boff[0] = 0;
    find_leader(R, X.ls, X.ll, X.lc, X.le, X.ln, X.lk);

    while (X.alive > 0) {
        if (X.nb >= T || X.ls < 0) { X.err = kBroken; break; }   // every batch holds a step: at most T
        // trips scan only the slots that can hold entries: 1, 2 or 4 of them when the higher
        // ones are empty (2 and 4 only for the larger register sets, whose ready sets often
        // span a few slots), else all S
        uint64_t h1 = 0, h2 = 0, h4 = 0;
#pragma unroll
        for (int s = 1; s < S; ++s) {
            h1 |= R.vm[s];
            if (s >= 2) h2 |= R.vm[s];
            if (s >= 4) h4 |= R.vm[s];
        }
        if (!h1) trip<1, S, flags>(R, X, I, M);
        else if (S >= 5 && !h2) trip<(S >= 5 ? 2 : S), S, flags>(R, X, I, M);
        else if (S >= 6 && !h4) trip<(S >= 6 ? 4 : S), S, flags>(R, X, I, M);
        else trip<S, S, flags>(R, X, I, M);
        if (X.err) break;
    }

    if (X.err == kOverflow) return true;
    if (lane == 0) {
        if (X.err) put_info(I.binfo, RR_E_INTERNAL, 0, 0, 0, 0);
        else if (X.nb > I.batch_cap) put_info(I.binfo, RR_E_CAPACITY, 0, 0, X.nb, T);
        else put_info(I.binfo, RR_OK, X.nb, X.out, X.nb, T);
    }
    return false;
}

// Run Alg. 3 on one instance whose graph is built (header state ST_FAST).  Returns true when
// the instance goes to the general path.
template <int S, uint32_t flags>
__device__ __forceinline__ bool loop_fast(const Inst &I, uint8_t *lds, uint32_t lds_bytes)
{
    const int lane = lane_id();
    const Layout L = layout(I.W, I.H, I.move_cap, I.step_cap);
    const uint32_t *hdr = (const uint32_t *)(I.ws + L.hdr);
    const uint32_t K = hdr[H_K], G = hdr[H_G], T = hdr[H_T], GE = hdr[H_GE], HN = hdr[H_HN];

    // ---- loop data: LDS when it fits
    const size_t need = 16 * (size_t)kWave * S + 4 * (size_t)K + 2 * (((size_t)K + 1) & ~(size_t)1) + 8 * (size_t)G +
                        2 * (2 * ((size_t)G + 1) + GE + HN) + 16;
    LoopMem M;
    M.soff = (const uint32_t *)(I.ws + L.soff);
    M.slist = (const uint32_t *)(I.ws + L.slist);
    M.pend = (uint32_t *)(I.ws + L.pend);
    const uint32_t *gmv = (const uint32_t *)(I.ws + L.mv);
    const uint16_t *gnx = (const uint16_t *)(I.ws + L.nx);
    const uint16_t *ggp = (const uint16_t *)(I.ws + L.gpend), *ggo = (const uint16_t *)(I.ws + L.gloff);
    const uint16_t *ghdo = (const uint16_t *)(I.ws + L.hdoff), *ghd = (const uint16_t *)(I.ws + L.hd);
    const uint16_t *ggl = (const uint16_t *)(I.ws + L.gl);
    if (need <= lds_bytes) {
        uint8_t *p = lds;
        M.scratch = (uint4 *)p; p += 16 * (size_t)kWave * S;
        uint32_t *mv = (uint32_t *)p; p += 4 * (size_t)K;
        uint32_t *grem = (uint32_t *)p; p += 4 * (size_t)G;
        uint32_t *gpend = (uint32_t *)p; p += 4 * (size_t)G;
        uint16_t *nx = (uint16_t *)p; p += 2 * (((size_t)K + 1) & ~(size_t)1);
        uint16_t *go = (uint16_t *)p; p += 2 * ((size_t)G + 1);
        uint16_t *hdo = (uint16_t *)p; p += 2 * ((size_t)G + 1);
        uint16_t *gl = (uint16_t *)p; p += 2 * (size_t)GE;
        uint16_t *hd = (uint16_t *)p;
        for (uint32_t i = lane; i < K; i += kWave) { mv[i] = gmv[i]; nx[i] = gnx[i]; }
        for (uint32_t i = lane; i < G; i += kWave) {
            grem[i] = I.goff[i + 1] - I.goff[i];
            gpend[i] = ggp[i];
        }
        for (uint32_t i = lane; i <= G; i += kWave) { go[i] = ggo[i]; hdo[i] = ghdo[i]; }
        for (uint32_t i = lane; i < GE; i += kWave) gl[i] = ggl[i];
        for (uint32_t i = lane; i < HN; i += kWave) hd[i] = ghd[i];
        M.mv = mv; M.nx = nx; M.grem = grem; M.gpend = gpend; M.gloff = go; M.hdoff = hdo; M.gl = gl; M.hd = hd;
        wave_sync();
        return loop_run<S, flags>(I, M, K, G, T);   // every LDS access of this copy compiles to ds_* operations
    } else {
        // the workspace copy: the move data stays in the workspace, but the per-group counts
        // (read and written at every finished move) and the merge scratch live in LDS -- the
        // launch plan gives every launch room for them (loop_small_lds)
        const size_t sat = (8 * (size_t)G + 15) & ~(size_t)15;
        if (sat + 16 * (size_t)kWave * S > lds_bytes) return true;    // not reached: the general path
        uint32_t *grem = (uint32_t *)lds, *gpend = grem + G;
        for (uint32_t i = lane; i < G; i += kWave) {
            grem[i] = I.goff[i + 1] - I.goff[i];
            gpend[i] = ggp[i];
        }
        M.scratch = (uint4 *)(lds + sat);
        M.mv = gmv; M.nx = gnx; M.grem = grem; M.gpend = gpend; M.gloff = ggo; M.hdoff = ghdo; M.gl = ggl; M.hd = ghd;
        wave_sync();
        return loop_run<S, flags>(I, M, K, G, T);
    }
}


}  // namespace fast
}  // namespace rr
