// rr_batch.hip -- batching routine (arXiv 2504.06182, §IV, Alg. 3) on gfx950: one wave64 per
// instance.
//
// The dependency graph Gamma is never materialised.  Any two moves that touch a common trap are
// ordered in Gamma (same group: their paths meet; different groups: their groups meet), so the
// moves touching one trap finish in index order.  It is then enough, for each trap, to keep its
// touching moves sorted by index and a count of finished ones:
//   * move b waits on trap c for the previous toucher of c when that one is in b's group;
//   * group h waits on trap c for the whole group that touched c last before h.
// A move is ready when both its counts are zero.  Each iteration of Alg. 3 then takes the ready
// moves in index order: the first one is always accepted, and with the deployed constraint the
// batch is the first move plus the ready moves stepping the same way on the one line (row or
// column through its current trap) that the next compatible move picks.  Ready moves never share
// a trap (two ready moves that did would be ordered in Gamma), so the vertex-disjointness test
// of Alg. 3 never rejects a step and is not evaluated.
//
// Storage: the ready list is kept sorted by move index in LDS (spilling to the workspace past
// kRcap entries), so the first ready move, the first compatible move and every output position
// come from ballots and prefix popcounts.  Per-trap counts, touch lists and per-move counters
// live in the instance's workspace.
#include "rr_device.hpp"
#include "rr.h"

static_assert(sizeof(rr_desc) == 80, "rr_desc layout");
static_assert(sizeof(rr_move) == 8, "rr_move layout");

namespace rr {

constexpr int kRcap = 256;   // ready-list entries held in LDS per instance

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
};

struct BatchLds {
    uint64_t buf[3][kRcap];     // ready lists (rotating), LDS part
    uint32_t fin_list[kWave];
    int nnew;
    int err;
};

// workspace carve-up (all offsets 256-byte aligned)
struct WsLayout {
    size_t off, fin, touch, pend, grp, gpend, grem, ov[3], total;
};

__host__ __device__ inline size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

__host__ __device__ inline WsLayout ws_layout(int W, int H, uint32_t move_cap, uint32_t step_cap)
{
    WsLayout L;
    const size_t WH = (size_t)W * H;
    const size_t K = move_cap ? move_cap : 1;
    size_t p = 0;
    L.off = p;   p = align256(p + 4 * (WH + 1));
    L.fin = p;   p = align256(p + 4 * WH);
    L.touch = p; p = align256(p + 4 * ((size_t)move_cap + step_cap + 1));
    L.pend = p;  p = align256(p + 4 * K);
    L.grp = p;   p = align256(p + 4 * K);
    L.gpend = p; p = align256(p + 4 * K);
    L.grem = p;  p = align256(p + 4 * K);
    for (int i = 0; i < 3; ++i) { L.ov[i] = p; p = align256(p + 8 * K); }
    L.total = p;
    return L;
}

// two-level array: the first kRcap entries in LDS, the rest in the workspace
struct TwoLevel {
    uint64_t *lds;
    uint64_t *glb;
    int cap;   // total entries (kRcap in LDS + the workspace part)
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

__device__ __forceinline__ uint32_t ld_rlx(const uint32_t *p) { return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }
__device__ __forceinline__ void st_rlx(uint32_t *p, uint32_t v) { __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT); }

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

// step code of the unit step leaving (x, y) on the path towards (dx, dy)
__device__ __forceinline__ uint32_t step_code(int x, int y, int dx, int dy)
{
    uint32_t dir;
    if (x != dx) dir = dx > x ? 0u : 1u;
    else dir = dy > y ? 2u : 3u;
    return (dir << 30) | ((uint32_t)x << 15) | (uint32_t)y;
}

__device__ __forceinline__ void put_binfo(rr_batch_info *bi, int status, uint32_t nb, uint32_t ns, uint32_t needb, uint32_t needs)
{
    rr_batch_info v;
    v.status = status; v.n_batches = nb; v.n_steps = ns; v.need_batches = needb; v.need_steps = needs;
    *bi = v;
}

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
    if (si.status != RR_OK || K > A.move_cap || G > K) {
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
    uint32_t *off = (uint32_t *)(A.ws + Lw.off);
    uint32_t *fin = (uint32_t *)(A.ws + Lw.fin);
    uint32_t *touch = (uint32_t *)(A.ws + Lw.touch);
    uint32_t *pend = (uint32_t *)(A.ws + Lw.pend);
    uint32_t *grp = (uint32_t *)(A.ws + Lw.grp);
    uint32_t *gpend = (uint32_t *)(A.ws + Lw.gpend);
    uint32_t *grem = (uint32_t *)(A.ws + Lw.grem);
    const int WH = W * H;

    // ---- per-trap touch counts
    for (int c = lane; c <= WH; c += kWave) off[c] = 0;
    for (int c = lane; c < WH; c += kWave) fin[c] = 0;
    for (uint32_t b = lane; b < K; b += kWave) { pend[b] = 0; gpend[b] = 0; }
    for (uint32_t g = lane; g < G; g += kWave) {
        const uint32_t lo = A.goff[g], hi = A.goff[g + 1];
        grem[g] = hi - lo;
        for (uint32_t b = lo; b < hi; ++b) grp[b] = g;
    }
    __threadfence();
    wave_sync();
    for (uint32_t b = lane; b < K; b += kWave) {
        int sx, sy, dx, dy;
        unpack_move(A.moves, b, sx, sy, dx, dy);
        const int len = (dx > sx ? dx - sx : sx - dx) + (dy > sy ? dy - sy : sy - dy);
        for (int s = 0; s <= len; ++s) {
            int x, y;
            path_cell(sx, sy, dx, dy, s, x, y);
            atomicAdd(&off[y * W + x], 1u);
        }
    }
    __threadfence();
    wave_sync();
    // exclusive scan of the counts -> offsets
    {
        uint32_t carry = 0;
        for (int base = 0; base <= WH; base += kWave) {
            const int c = base + lane;
            const uint32_t v = c <= WH ? ld_rlx(&off[c]) : 0u;
            const int inc = wave_incl_scan((int)v);
            if (c <= WH) off[c] = carry + (uint32_t)inc - v;
            carry += (uint32_t)__shfl(inc, kWave - 1, kWave);
        }
    }
    __threadfence();
    wave_sync();
    // fill the touch lists (arrival order), then sort each trap's list by move index
    for (uint32_t b = lane; b < K; b += kWave) {
        int sx, sy, dx, dy;
        unpack_move(A.moves, b, sx, sy, dx, dy);
        const int len = (dx > sx ? dx - sx : sx - dx) + (dy > sy ? dy - sy : sy - dy);
        for (int s = 0; s <= len; ++s) {
            int x, y;
            path_cell(sx, sy, dx, dy, s, x, y);
            const int c = y * W + x;
            const uint32_t slot = atomicAdd(&fin[c], 1u);
            touch[off[c] + slot] = b;
        }
    }
    __threadfence();
    wave_sync();
    for (int c = lane; c < WH; c += kWave) {
        const uint32_t lo = off[c], hi = off[c + 1];
        for (uint32_t k = lo + 1; k < hi; ++k) {
            const uint32_t v = touch[k];
            uint32_t m = k;
            while (m > lo && touch[m - 1] > v) { touch[m] = touch[m - 1]; --m; }
            touch[m] = v;
        }
        for (uint32_t k = lo + 1; k < hi; ++k) {
            const uint32_t a = touch[k - 1], b = touch[k];
            const uint32_t ga = grp[a], gb = grp[b];
            if (ga == gb) atomicAdd(&pend[b], 1u);
            else atomicAdd(&gpend[gb], 1u);
        }
        fin[c] = 0;
    }
    __threadfence();
    wave_sync();

    // ---- initial ready list (sorted: lanes append in index order)
    uint64_t *const ov0 = (uint64_t *)(A.ws + Lw.ov[0]);
    const size_t ovs = (Lw.ov[1] - Lw.ov[0]) / sizeof(uint64_t);
    const int rcap = kRcap + (int)K;
    auto B = [&](int i) { return TwoLevel{S.buf[i], ov0 + (size_t)i * ovs, rcap}; };
    int cur = 0;
    int n = 0;
    for (uint32_t base = 0; base < K; base += kWave) {
        const uint32_t b = base + lane;
        bool rd = false;
        uint32_t code = 0;
        if (b < K) {
            rd = ld_rlx(&pend[b]) == 0u && ld_rlx(&gpend[grp[b]]) == 0u;
            if (rd) {
                int sx, sy, dx, dy;
                unpack_move(A.moves, b, sx, sy, dx, dy);
                code = step_code(sx, sy, dx, dy);
            }
        }
        const uint64_t m = ballot(rd);
        if (rd) B(cur).put(n + popc(m & low_mask(lane)), ((uint64_t)b << 32) | code);
        n += popc(m);
    }
    if (lane == 0) { A.boff[0] = 0; S.nnew = 0; S.err = 0; }
    wave_sync();

    // ---- Alg. 3: one iteration per batch
    const uint32_t flags = A.flags;
    uint32_t out = 0, nb = 0, alive = K;
    while (alive > 0) {
        if (nb >= T) { if (lane == 0) S.err = 1; break; }   // every batch has a step: at most T
        const TwoLevel R = B(cur);
        const int nwb = cur == 2 ? 0 : cur + 1;        // new ready moves collect here
        const int third = 3 - cur - nwb;
        const TwoLevel NW = B(nwb);
        if (n == 0) { if (lane == 0) S.err = 1; break; }   // unreachable: the lowest unfinished move is ready
        const uint32_t c1 = (uint32_t)R.get(0);
        const uint32_t d1 = c1 >> 30, x1 = (c1 >> 15) & 0x7FFFu, y1 = c1 & 0x7FFFu;
        // deployed constraint: the next compatible ready move fixes the line (row or column)
        int first = n;
        bool row = false;
        if (flags == RR_LAMBDA_LINE_OR_COL) {
            for (int base = 0; base < n; base += kWave) {
                const int e = base + lane;
                bool cand = false;
                if (e > 0 && e < n) {
                    const uint32_t c = (uint32_t)R.get(e);
                    cand = (c >> 30) == d1 && (((c >> 15) & 0x7FFFu) == x1 || (c & 0x7FFFu) == y1);
                }
                const uint64_t m = ballot(cand);
                if (m) { first = base + __ffsll((unsigned long long)m) - 1; break; }
            }
            if (first < n) row = ((uint32_t)R.get(first) & 0x7FFFu) == y1;
        }
        // accept, emit in index order, advance; completed moves release their traps
        uint32_t acc_before = 0;
        int nf = 0;
        for (int base = 0; base < n; base += kWave) {
            const int e = base + lane;
            bool acc = false;
            uint64_t v = 0;
            if (e < n) {
                v = R.get(e);
                const uint32_t c = (uint32_t)v;
                const uint32_t d = c >> 30, x = (c >> 15) & 0x7FFFu, y = c & 0x7FFFu;
                if (flags == RR_LAMBDA_NONE) acc = true;
                else if (flags == RR_LAMBDA_ALONG) acc = d == d1 && (d1 >= 2 ? x == x1 : y == y1);
                else acc = (e == 0) || (first < n && d == d1 && (row ? y == y1 : x == x1));
            }
            const uint64_t m = ballot(acc);
            bool done = false;
            if (acc) {
                const uint32_t rank = acc_before + (uint32_t)popc(m & low_mask(lane));
                const uint32_t c = (uint32_t)v;
                if (out + rank < A.step_cap) A.steps[out + rank] = c;
                const uint32_t b = (uint32_t)(v >> 32);
                int sx, sy, dx, dy;
                unpack_move(A.moves, b, sx, sy, dx, dy);
                int x = (int)((c >> 15) & 0x7FFFu), y = (int)(c & 0x7FFFu);
                const uint32_t d = c >> 30;
                x += d == 0 ? 1 : (d == 1 ? -1 : 0);
                y += d == 2 ? 1 : (d == 3 ? -1 : 0);
                done = (x == dx && y == dy);
                R.put(e, done ? ~0ull : (((uint64_t)b << 32) | step_code(x, y, dx, dy)));
            }
            const uint64_t fm = ballot(done);
            if (done) S.fin_list[popc(fm & low_mask(lane))] = (uint32_t)(v >> 32);
            acc_before += (uint32_t)popc(m);
            wave_sync();
            const int nfc = popc(fm);
            for (int q = 0; q < nfc; ++q) {
                if (S.fin_list[q] >= K) { if (lane == 0) S.err = 1; continue; }
                const uint32_t b = S.fin_list[q];
                int sx, sy, dx, dy;
                unpack_move(A.moves, b, sx, sy, dx, dy);
                const int len = (dx > sx ? dx - sx : sx - dx) + (dy > sy ? dy - sy : sy - dy);
                const uint32_t gb = grp[b];
                // per trap: one more finished toucher; the next toucher in the same group
                // loses one wait (its group is running, so it is ready when none is left)
                for (int s = lane; s <= len; s += kWave) {
                    int x, y;
                    path_cell(sx, sy, dx, dy, s, x, y);
                    const int cc = y * W + x;
                    const uint32_t f = ld_rlx(&fin[cc]) + 1u;
                    st_rlx(&fin[cc], f);
                    const uint32_t o = off[cc], nc = off[cc + 1] - o;
                    if (f < nc) {
                        const uint32_t nx = touch[o + f];
                        if (grp[nx] == gb) {
                            const uint32_t old = atomicSub(&pend[nx], 1u);
                            if (old == 1u) NW.put(atomicAdd(&S.nnew, 1), (uint64_t)nx);
                        }
                    }
                }
                __threadfence();
                wave_sync();
                uint32_t rem = 0;
                if (lane == 0) rem = atomicSub(&grem[gb], 1u) - 1u;
                rem = (uint32_t)__shfl((int)rem, 0, kWave);
                if (rem == 0) {
                    // the whole group has finished: each trap it touched hands over to the
                    // next group touching it; a group with no wait left is unlocked
                    const uint32_t lo = A.goff[gb], hi = A.goff[gb + 1];
                    for (uint32_t bb = lo + lane; bb < hi; bb += kWave) {
                        int ax, ay, bx, by;
                        unpack_move(A.moves, bb, ax, ay, bx, by);
                        const int l2 = (bx > ax ? bx - ax : ax - bx) + (by > ay ? by - ay : ay - by);
                        for (int s = 0; s <= l2; ++s) {
                            int x, y;
                            path_cell(ax, ay, bx, by, s, x, y);
                            const int cc = y * W + x;
                            const uint32_t f = ld_rlx(&fin[cc]);
                            const uint32_t o = off[cc], nc = off[cc + 1] - o;
                            if (f < nc && touch[o + f - 1] == bb) {
                                const uint32_t h = grp[touch[o + f]];
                                if (atomicSub(&gpend[h], 1u) == 1u) {
                                    for (uint32_t b3 = A.goff[h]; b3 < A.goff[h + 1]; ++b3)
                                        if (ld_rlx(&pend[b3]) == 0u) NW.put(atomicAdd(&S.nnew, 1), (uint64_t)b3);
                                }
                            }
                        }
                    }
                    __threadfence();
                    wave_sync();
                }
            }
            nf += nfc;
            wave_sync();
        }
        out += acc_before;
        ++nb;
        if (lane == 0 && nb <= A.batch_cap) A.boff[nb] = out;
        alive -= (uint32_t)nf;
        const int nn = S.nnew;
        wave_sync();
        if (nf == 0 && nn == 0) continue;

        // ---- keep the ready list sorted: drop completed moves, merge the newly ready ones
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
            // sort the new moves by index into the free buffer (rank by counting)
            const TwoLevel F = B(freeb);
            for (int k = lane; k < nn; k += kWave) {
                const uint32_t b = (uint32_t)NW.get(k);
                int r = 0;
                for (int q = 0; q < nn; ++q) {
                    const uint32_t o = (uint32_t)NW.get(q);
                    r += (o < b) || (o == b && q < k);
                }
                int sx, sy, dx, dy;
                unpack_move(A.moves, b, sx, sy, dx, dy);
                F.put(r, ((uint64_t)b << 32) | step_code(sx, sy, dx, dy));
            }
            wave_sync();
            // merge survivors (sbuf) and new moves (freeb) into nwb by co-ranking
            const TwoLevel Sv = B(sbuf);
            for (int i = lane; i < ns; i += kWave) {
                const uint64_t v = Sv.get(i);
                int lo = 0, hi = nn;
                while (lo < hi) { const int mid = (lo + hi) >> 1; if (F.get(mid) < v) lo = mid + 1; else hi = mid; }
                NW.put(i + lo, v);
            }
            for (int k = lane; k < nn; k += kWave) {
                const uint64_t v = F.get(k);
                int lo = 0, hi = ns;
                while (lo < hi) { const int mid = (lo + hi) >> 1; if (Sv.get(mid) < v) lo = mid + 1; else hi = mid; }
                NW.put(k + lo, v);
            }
            cur = nwb;
            n = ns + nn;
        } else {
            cur = sbuf;
            n = ns;
        }
        if (lane == 0) S.nnew = 0;
        wave_sync();
    }

    const bool err = S.err != 0;
    if (lane == 0) {
        const bool cap = nb > A.batch_cap;
        const int st = err ? RR_E_INTERNAL : (cap ? RR_E_CAPACITY : RR_OK);
        const bool ok = st == RR_OK;
        put_binfo(A.binfo, st, ok ? nb : 0u, ok ? out : 0u, nb, T);
    }
}

__global__ __launch_bounds__(kWave) void k_batch_one(BatchArgs A)
{
    __shared__ BatchLds S;
    batch_one(S, A);
}

__global__ __launch_bounds__(kWave) void k_batch_many(const rr_desc *__restrict__ desc, int maxw, int maxh,
                                                      const rr_move *mv, const uint32_t *ga,
                                                      const rr_solve_info *sinfos, uint32_t flags,
                                                      uint32_t *bat, uint32_t *stp, rr_batch_info *binfos,
                                                      uint8_t *ws)
{
    __shared__ BatchLds S;
    const rr_desc d = desc[blockIdx.x];
    const rr_shape s = d.shape;
    const bool ok = s.w >= 1 && s.h >= 1 && s.w <= maxw && s.h <= maxh && s.w <= RR_MAX_SIDE &&
                    s.h <= RR_MAX_SIDE && s.x0 < s.x1 && s.x1 <= s.w && s.y0 < s.y1 && s.y1 <= s.h;
    if (!ok) {
        if (threadIdx.x == 0) put_binfo(binfos + blockIdx.x, RR_E_INVAL, 0, 0, 0, 0);
        return;
    }
    if (d.step_cap == 0xFFFFFFFFu) {
        // the planner found no room for this instance: report the size it needs
        if (threadIdx.x == 0) {
            const rr_solve_info si = sinfos[blockIdx.x];
            if (si.status == RR_INFEASIBLE || (si.status == RR_OK && si.n_moves == 0))
                put_binfo(binfos + blockIdx.x, RR_OK, 0, 0, 0, 0);
            else if (si.status == RR_OK)
                put_binfo(binfos + blockIdx.x, RR_E_CAPACITY, 0, 0, si.n_steps, si.n_steps);
            else
                put_binfo(binfos + blockIdx.x, RR_E_INVAL, 0, 0, 0, 0);
        }
        return;
    }
    BatchArgs A;
    A.W = s.w; A.H = s.h;
    A.moves = mv + d.move_off;
    A.goff = ga + d.group_off;
    A.sinfo = sinfos + blockIdx.x;
    A.move_cap = d.move_cap;
    A.flags = flags;
    A.boff = bat + d.batch_off;
    A.batch_cap = d.batch_cap;
    A.steps = stp + d.step_off;
    A.step_cap = d.step_cap;
    A.binfo = binfos + blockIdx.x;
    A.ws = ws + d.ws_off;
    batch_one(S, A);
}

// Arena planner: one 1024-thread workgroup scans the instances in chunks of 1024.
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
            v[2] = align256(ws_layout(d.shape.w, d.shape.h, d.move_cap, sc).total);
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
    return ws_layout(shape.w, shape.h, move_cap, step_cap).total;
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
    if (flags > RR_LAMBDA_NONE) return RR_E_INVAL;
    if (!group_off || !sinfo || !batch_off || !binfo || (move_cap > 0 && !moves) || (step_cap > 0 && !steps))
        return RR_E_INVAL;
    if (((uintptr_t)moves & 7u) != 0) return RR_E_INVAL;
    if (!workspace || workspace_bytes < rr_batch_workspace_bytes(shape, move_cap, step_cap)) return RR_E_NOMEM;
    BatchArgs A;
    A.W = shape.w; A.H = shape.h;
    A.moves = moves; A.goff = group_off; A.sinfo = sinfo; A.move_cap = move_cap; A.flags = flags;
    A.boff = batch_off; A.batch_cap = batch_cap; A.steps = steps; A.step_cap = step_cap; A.binfo = binfo;
    A.ws = (uint8_t *)workspace;
    hipLaunchKernelGGL(k_batch_one, dim3(1), dim3(kWave), 0, (hipStream_t)stream, A);
    return hipGetLastError() == hipSuccess ? RR_OK : RR_E_DEVICE;
}

extern "C" rr_status rr_batch_moves_many(uint32_t n, const rr_desc *desc, uint32_t max_w, uint32_t max_h,
                                         const rr_move *move_arena, const uint32_t *group_arena,
                                         const rr_solve_info *sinfos, uint32_t flags, uint32_t *batch_arena,
                                         uint32_t *step_arena, rr_batch_info *binfos, void *workspace,
                                         size_t workspace_bytes, void *stream)
{
    (void)workspace_bytes;
    if (n == 0) return RR_OK;
    if (!desc || !move_arena || !group_arena || !sinfos || !batch_arena || !step_arena || !binfos || !workspace)
        return RR_E_INVAL;
    if (flags > RR_LAMBDA_NONE || max_w < 1 || max_h < 1) return RR_E_INVAL;
    if (max_w > RR_MAX_SIDE || max_h > RR_MAX_SIDE) return RR_E_UNSUPPORTED;
    if (((uintptr_t)move_arena & 7u) != 0) return RR_E_INVAL;
    hipLaunchKernelGGL(k_batch_many, dim3(n), dim3(kWave), 0, (hipStream_t)stream, desc, (int)max_w, (int)max_h,
                       move_arena, group_arena, sinfos, flags, batch_arena, step_arena, binfos,
                       (uint8_t *)workspace);
    return hipGetLastError() == hipSuccess ? RR_OK : RR_E_DEVICE;
}
