// rr_solve.hip -- red-rec solve on gfx950: one workgroup per instance, 1 to 4 wave64 for grids
// up to 256 per side (state in LDS), 16 wave64 for larger grids up to 1024 per side (the same
// state in a per-instance region of the caller's workspace, served by L2).
//
// Method (arXiv 2504.06182): exact 1D on lines (§III.A), red-rec with every column of
// non-negative surplus solved from the outset and donor/receiver pairs identified one after the
// other (§III.C, Alg. 1; ordering of §III.D).  Targets narrower than the grid get a row
// pre-pass first (each target row solved on its own line), and the column stage then treats
// side columns as donors with no target.
//
// Data flow inside one workgroup, all in LDS:
//   bit rows (coalesced load)  -> row pre-pass, one wave per target row
//   -> column bits by ballot transposition (one ballot per column and 64-row slab)
//   -> column counts and surplus by popcount
//   -> non-negative columns: exact 1D by prefix sums of d_k = q_k - k, one wave per column
//   -> donor/receiver loop on wave 0 (ballot masks of unsettled columns, 64-bit pair keys,
//      receiver split cost in closed form from prefix sums)
//   -> receiver solves, whole workgroup, ranks by counting
//   -> every output position from a workgroup exclusive scan (no atomics decide an order)
//   -> final grid by ballot transposition back to bit rows.
#include "rr_device.hpp"
#include "rr.h"

namespace rr {

constexpr int kThreads = 256;              // default threads per instance (4 waves)

enum { M_STEPS = 0, M_NEV = 1, M_ERR = 2, M_CNT = 3 };

constexpr uint32_t kOrderSerial = 1u;   // RR_REDREC_SERIAL
constexpr uint32_t kBird = 2u;          // RR_BIRD

// NW waves per instance; the per-wave scratch P, Q has at least three rows (the pair loop, the
// serial donor solves and bird use rows 0..2 from one wave)
template <int S, int NW>
struct SolveLds {
    static constexpr int WS = S / 64;
    uint64_t rows[S * WS];   // bit rows, stride ws
    uint64_t cols[S * WS];   // column bits after the row pre-pass, stride hs
    uint64_t elig[S * WS];   // column bits that count towards the column surplus, stride hs
    int rowW[S], rowT0[S], rowN[S], rowR[S], rowCnt[S], rowOff[S];
    int colA[S], colW[S], colU[S], colCnt[S], colOff[S], sp[S], sig[S], bcnt[S], ubeg[S];
    int mNb[S], mSb[S], mNt[S], mSt[S];
    int cNb[S], cNbd[S];     // eligible tokens below the band / inside it, per column
    int8_t dsol[S];          // column solved (the serial order leaves central donors unsolved)
    int16_t evI[S + 1], evJ[S + 1], evK[S + 1], evC[S + 1], evBlo[S + 1], evBhi[S + 1], evUlo[S + 1], evUhi[S + 1];
    // donor solved with the event (serial order): window start over its remaining tokens, and
    // its remaining pool bounds at that moment ([0,bc) below, [ub,a) above); evDW < 0: none
    int16_t evDW[S + 1], evDbc[S + 1], evDub[S + 1];
    // bird: histograms of reservoir tokens by virtual distance from the band (above: u = v - y1,
    // below: u = y0 - 1 - v) and their exclusive prefix counts and sums of virtual rows
    int hT[2 * S + 2], hB[2 * S + 2], cT[2 * S + 3], cB[2 * S + 3], sT[2 * S + 3], sB[2 * S + 3];
    int P[NW < 3 ? 3 : NW][S + 1];
    int Q[NW < 3 ? 3 : NW][S + 2];
    uint64_t rkey[S];
    int16_t ry[S], rorg[S], byRank[S];
    int scanA[NW];
    int scanB[NW];
    int misc[8];
};

struct SolveArgs {
    int W, H, x0, y0, x1, y1;
    uint32_t flags;
    const uint64_t *occ;
    rr_move *moves;
    uint32_t move_cap;
    uint32_t *goff;
    uint32_t group_cap;
    uint64_t *fin;
    rr_solve_info *info;
};

// ------------------------------------------------------------------------------------------
// workgroup helpers

template <int NW>
__device__ __forceinline__ int block_excl_scan(int v, int *tmp, int *total)
{
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    int inc = wave_incl_scan(v);
    if (lane == kWave - 1) tmp[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) {
        int t = tmp[w];
        off += (w < wid) ? t : 0;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

template <int NW>
__device__ __forceinline__ int block_sum(int v, int *tmp)
{
    int tot;
    block_excl_scan<NW>(v, tmp, &tot);
    return tot;
}

// positions of the set bits of bits[0..nw) (word j = positions 64j..64j+63) -> P, in order
__device__ __forceinline__ int compact_bits_wave(const uint64_t *bits, int nw, int *P)
{
    const int lane = lane_id();
    int base = 0;
    for (int j = 0; j < nw; ++j) {
        uint64_t w = bits[j];
        if ((w >> lane) & 1ull) P[base + popc(w & low_mask(lane))] = 64 * j + lane;
        base += popc(w);
    }
    wave_sync();
    return base;
}

// Qs[m] = sum_{k<m} V[k], m = 0..n
__device__ __forceinline__ void prefix_sums_wave(const int *V, int n, int *Qs)
{
    const int lane = lane_id();
    int carry = 0;
    for (int base = 0; base < n; base += kWave) {
        int k = base + lane;
        int v = k < n ? V[k] : 0;
        int inc = wave_incl_scan(v);
        if (k < n) Qs[k + 1] = carry + inc;
        carry += __shfl(inc, kWave - 1, kWave);
    }
    if (lane == 0) Qs[0] = 0;
    wave_sync();
}

// Exact-1D assignment on a line (§III.A): sorted sources P[0..a), targets b..b+t-1, a >= t.
// The optimum is an order-preserving match of a run of t consecutive sources starting at w;
// cost(w) = sum_{k in [w,w+t)} |d_k - (b - w)| with d_k = P[k] - k non-decreasing, evaluated in
// O(log a) from prefix sums of d and a binary search for the sign change.  Lanes take
// windows; the minimum cost wins, on equal cost the smallest w.
__device__ int e1d_window_wave(const int *P, int *Qs, int a, int b, int t)
{
    const int lane = lane_id();
    if (t >= a) return 0;
    int carry = 0;
    for (int base = 0; base < a; base += kWave) {
        int k = base + lane;
        int d = k < a ? P[k] - k : 0;
        int inc = wave_incl_scan(d);
        if (k < a) Qs[k + 1] = carry + inc;
        carry += __shfl(inc, kWave - 1, kWave);
    }
    if (lane == 0) Qs[0] = 0;
    wave_sync();
    uint64_t best = ~0ull;
    for (int w = lane; w + t <= a; w += kWave) {
        const int c = b - w;
        int lo = w, hi = w + t;
        while (lo < hi) {
            int mid = (lo + hi) >> 1;
            if (P[mid] - mid < c) lo = mid + 1; else hi = mid;
        }
        const int s = lo;
        long cost = (long)c * (s - w) - (long)(Qs[s] - Qs[w]) + (long)(Qs[w + t] - Qs[s]) - (long)c * (w + t - s);
        uint64_t key = ((uint64_t)cost << 20) | (uint64_t)w;
        best = key < best ? key : best;
    }
    best = wave_min_u64(best);
    wave_sync();
    return (int)(best & 0xFFFFFull);
}

// k-th set bit (0-based) of a multi-word bitset
__device__ __forceinline__ int select_in_bits(const uint64_t *bits, int nw, int k)
{
    for (int j = 0; j < nw; ++j) {
        int c = popc(bits[j]);
        if (k < c) return 64 * j + select_bit(bits[j], k);
        k -= c;
    }
    return -1;
}

__device__ __forceinline__ void put_move(const SolveArgs &A, uint32_t pos, int sx, int sy, int dx, int dy)
{
    if (pos < A.move_cap) {
        uint64_t v = (uint64_t)(uint16_t)sx | ((uint64_t)(uint16_t)sy << 16) |
                     ((uint64_t)(uint16_t)dx << 32) | ((uint64_t)(uint16_t)dy << 48);
        reinterpret_cast<uint64_t *>(A.moves)[pos] = v;
    }
}

// Emit the moves of one exact-1D line: matched pairs P[w0+k] -> t0+k, k < n.  Paths towards
// larger coordinates first, largest target first; then paths towards smaller coordinates,
// smallest target first (§III.A, generating moves).  Positions by ballot prefix counts.
__device__ __forceinline__ void emit_line_wave(const SolveArgs &A, const int *P, int w0, int t0, int n, int R,
                                               uint32_t off, bool horizontal, int fixed)
{
    const int lane = lane_id();
    int rb = 0, lb = 0;
    for (int base = 0; base < n; base += kWave) {
        const int k = base + lane;
        int s = 0, t = 0;
        bool isR = false, isL = false;
        if (k < n) { s = P[w0 + k]; t = t0 + k; isR = s < t; isL = s > t; }
        const uint64_t mR = ballot(isR), mL = ballot(isL);
        int pos = -1;
        if (isR) pos = R - (rb + popc(mR & low_mask(lane + 1)));
        else if (isL) pos = R + lb + popc(mL & low_mask(lane));
        if (pos >= 0) {
            if (horizontal) put_move(A, off + pos, s, fixed, t, fixed);
            else put_move(A, off + pos, fixed, s, fixed, t);
        }
        rb += popc(mR);
        lb += popc(mL);
    }
}

// Rows a donor still holds in the serial order: its eligible list F[0..a) (sorted) minus what
// it handed over -- F[0,bc) below the band, its band tokens F[nb0, nb0+nbd), F[ub,a) above --
// written to R in order; returns their count.
__device__ __forceinline__ int remaining_rows_wave(const int *F, int a, int bc, int nb0, int nbd, int ub, int *R)
{
    const int lane = lane_id();
    const int n1 = bc, n2 = nbd, n3 = a - ub;
    for (int m = lane; m < n1 + n2 + n3; m += kWave)
        R[m] = m < n1 ? F[m] : (m < n1 + n2 ? F[nb0 + (m - n1)] : F[ub + (m - n1 - n2)]);
    wave_sync();
    return n1 + n2 + n3;
}

// ------------------------------------------------------------------------------------------
// donor/receiver loop (Alg. 1 main loop, pairing rule of §III.C), run by wave 0

template <int S, int NW>
__device__ void pair_loop(SolveLds<S, NW> &L, int W, int hs, int y0, int y1, int sh)
{
    const int lane = lane_id();
    constexpr int CW = S / 64;
    int nev = 0, err = 0;
    for (int iter = 0; iter <= W; ++iter) {
        uint64_t nz[CW];
        bool anyneg = false;
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int x = 64 * c + lane;
            const int v = x < W ? L.sp[x] : 0;
            nz[c] = ballot(v != 0);
            anyneg |= ballot(v < 0) != 0ull;
        }
        if (!anyneg) break;
        if (iter == W) { err = 1; break; }
        // candidate pairs: adjacent unsettled columns of opposite sign
        uint64_t best = 0;
#pragma unroll
        for (int c = 0; c < CW; ++c) {
            const int x = 64 * c + lane;
            if (!((nz[c] >> lane) & 1ull)) continue;
            int nx = -1;
            const uint64_t rest = nz[c] & ~low_mask(lane + 1);
            if (rest) nx = 64 * c + __ffsll((unsigned long long)rest) - 1;
            else {
#pragma unroll
                for (int c2 = c + 1; c2 < CW; ++c2)
                    if (nx < 0 && nz[c2]) nx = 64 * c2 + __ffsll((unsigned long long)nz[c2]) - 1;
            }
            if (nx < 0) continue;
            const int vx = L.sp[x], vn = L.sp[nx];
            if ((vx > 0) == (vn > 0)) continue;
            const int i = vx > 0 ? x : nx, j = vx > 0 ? nx : x;
            const int si = vx > 0 ? vx : vn, need = vx > 0 ? -vn : -vx;
            const int m = si < need ? si : need;
            const int dist = i > j ? i - j : j - i;
            // larger exchange, then fewer columns between, then receiver closer to saturation,
            // then smaller receiver index, then smaller donor index
            const uint64_t key = ((uint64_t)m << 50) | ((uint64_t)(4095 - dist) << 38) |
                                 ((uint64_t)(8191 - need) << 25) | ((uint64_t)(4095 - j) << 13) |
                                 (uint64_t)(8191 - i);
            best = key > best ? key : best;
        }
        best = wave_max_u64(best);
        if (best == 0) { err = 1; break; }
        const int j = 4095 - (int)((best >> 13) & 4095ull);
        const int i = 8191 - (int)(best & 8191ull);
        const int si = L.sp[i], d = -L.sp[j];
        const int ai = L.colA[i], bc = L.bcnt[i], ub = L.ubeg[i];
        int *P0 = L.P[0];
        int *Q0 = L.Q[0];
        compact_bits_wave(&L.elig[i * hs], hs, P0);
        prefix_sums_wave(P0, ai, Q0);
        int dw = -1, dbc = 0, dub = 0;
        if (si < d && !L.dsol[i]) {
            // serial order, case 3: the donor is solved first over the tokens it still holds;
            // its unmatched ones (outside the band, exact-1D lemma) form the pool then marked
            int *R = L.P[1], *RQ = L.Q[1];
            const int nb0 = L.cNb[i], nbd = L.cNbd[i];
            const int ar = remaining_rows_wave(P0, ai, bc, nb0, nbd, ub, R);
            const int w = e1d_window_wave(R, RQ, ar, y0, sh);
            if (w > bc || w + sh < bc + nbd) err = 1;
            dw = w; dbc = bc; dub = ub;
        }
        if (si < d) {
            // case 3: the donor's whole pool is marked for the receiver
            const int bc = dw >= 0 ? dw : L.bcnt[i];
            const int ub = dw >= 0 ? dub + (dw + sh - dbc - L.cNbd[i]) : L.ubeg[i];
            if (lane == 0) {
                L.mNb[j] += bc;
                L.mSb[j] += Q0[bc];
                L.mNt[j] += ai - ub;
                L.mSt[j] += Q0[ai] - Q0[ub];
                L.evI[nev] = (int16_t)i; L.evJ[nev] = (int16_t)j; L.evC[nev] = 3; L.evK[nev] = -1;
                L.evBlo[nev] = 0; L.evBhi[nev] = (int16_t)bc; L.evUlo[nev] = (int16_t)ub; L.evUhi[nev] = (int16_t)ai;
                L.bcnt[i] = 0; L.ubeg[i] = ai;
                L.sp[j] = si - d; L.sp[i] = 0;
                L.evDW[nev] = (int16_t)dw; L.evDbc[nev] = (int16_t)dbc; L.evDub[nev] = (int16_t)dub;
                L.dsol[i] = 1;
            }
        } else {
            // cases 1-2: d tokens, the k nearest below the band and the d-k nearest above it,
            // k minimising the receiver's 1-D cost (ties: largest k)
            int *P1 = L.P[1], *Q1 = L.Q[1], *E = L.P[2], *EQ = L.Q[2];
            const int aj = L.colA[j];
            compact_bits_wave(&L.elig[j * hs], hs, P1);
            prefix_sums_wave(P1, aj, Q1);
            int nbO = 0, ntO = 0;
            for (int sl = 0; sl < hs; ++sl) {
                const uint64_t e = L.elig[j * hs + sl];
                nbO += popc(e & low_mask(y0 - 64 * sl));
                ntO += popc(e & ~low_mask(y1 - 64 * sl));
            }
            const int nband = aj - nbO - ntO;
            const int sbO = Q1[nbO], stO = Q1[aj] - Q1[aj - ntO];
            for (int m = lane; m < nband; m += kWave) E[m] = P1[nbO + m] - y0 - m;
            wave_sync();
            prefix_sums_wave(E, nband, EQ);
            const int nbF = nbO + L.mNb[j], sbF = sbO + L.mSb[j], ntF = ntO + L.mNt[j], stF = stO + L.mSt[j];
            const int uav = ai - ub;
            const int klo = d - uav > 0 ? d - uav : 0, khi = d < bc ? d : bc;
            uint64_t bk = ~0ull;
            for (int k = klo + lane; k <= khi; k += kWave) {
                const long nb = nbF + k, nt = ntF + d - k;
                const long Sb = sbF + (Q0[bc] - Q0[bc - k]);
                const long St = stF + (Q0[ub + d - k] - Q0[ub]);
                const long cb = nb * y0 + nb * (nb - 1) / 2 - Sb;
                const long ct = St - nt * y0 - nt * (2L * sh - nt - 1) / 2;
                int lo = 0, hi = nband;
                while (lo < hi) {
                    int mid = (lo + hi) >> 1;
                    if (E[mid] < nb) lo = mid + 1; else hi = mid;
                }
                const long cband = nb * lo - EQ[lo] + (EQ[nband] - EQ[lo]) - nb * (nband - lo);
                const long cost = cb + cband + ct;
                const uint64_t key = ((uint64_t)cost << 16) | (uint64_t)(0xFFFF - k);
                bk = key < bk ? key : bk;
            }
            bk = wave_min_u64(bk);
            const int k = 0xFFFF - (int)(bk & 0xFFFFull);
            // serial order, case 2: the donor, left with exactly sh tokens, is solved after the
            // receiver (window 0 over what it holds; nothing of it stays in the reservoir)
            const bool dsolve = si == d && !L.dsol[i];
            if (lane == 0) {
                L.evI[nev] = (int16_t)i; L.evJ[nev] = (int16_t)j; L.evC[nev] = (int16_t)(si == d ? 2 : 1);
                L.evK[nev] = (int16_t)k;
                L.evBlo[nev] = (int16_t)(bc - k); L.evBhi[nev] = (int16_t)bc;
                L.evUlo[nev] = (int16_t)ub; L.evUhi[nev] = (int16_t)(ub + d - k);
                L.bcnt[i] = dsolve ? 0 : bc - k; L.ubeg[i] = dsolve ? ai : ub + d - k;
                L.sp[i] = si - d; L.sp[j] = 0;
                L.evDW[nev] = (int16_t)(dsolve ? 0 : -1);
                L.evDbc[nev] = (int16_t)(bc - k); L.evDub[nev] = (int16_t)(ub + d - k);
                if (dsolve) L.dsol[i] = 1;
            }
        }
        ++nev;
        wave_sync();
    }
    if (lane == 0) { L.misc[M_NEV] = nev; L.misc[M_ERR] |= err; }
}

// ------------------------------------------------------------------------------------------
// bird (§III.E, Alg. 2): the columns of negative surplus, leftmost first, each filled by the
// generalized exact 1D.  For column j every reservoir token of another column x stands at the
// virtual row y + |x - j| (above the band) or y - |x - j| (below): the row with the same
// Manhattan distance to the target of column j; its own tokens stand at their rows.  The
// cheapest run of sh sorted virtual tokens holds every own band token (exact-1D lemma), so it
// is fixed by k, the tokens taken from below: the k nearest below, the band tokens and the
// sh - band - k nearest above.  Among tokens of one virtual row the nearest column comes
// first, then the left one.  L.cols holds the current grid, column by column.

// Column x once settled: its band full (central) or its parked band tokens (side), plus, for a
// donor, the pool left in its reservoir -- indices [0, bcnt) and [ubeg, a) of its sorted
// eligible rows.
template <int S, int NW>
__device__ __forceinline__ void settle_column(SolveLds<S, NW> &L, int x, int hs, int y0, int y1, bool central, bool donor)
{
    int keepLow = L.bcnt[x], dropLow = L.ubeg[x];
    for (int sl = 0; sl < hs; ++sl) {
        const uint64_t band = range_mask(y0 - 64 * sl, y1 - 1 - 64 * sl);
        uint64_t f = central ? band : (L.cols[x * hs + sl] & band);
        if (donor) {
            const uint64_t e = L.elig[x * hs + sl];
            const int c = popc(e);
            uint64_t lowPart;
            if (keepLow >= c) lowPart = e;
            else lowPart = keepLow > 0 ? (e & low_mask(select_bit(e, keepLow))) : 0ull;
            uint64_t dropPart;
            if (dropLow >= c) dropPart = e;
            else dropPart = dropLow > 0 ? (e & low_mask(select_bit(e, dropLow))) : 0ull;
            f |= lowPart | (e & ~dropPart);
            keepLow = keepLow > c ? keepLow - c : 0;
            dropLow = dropLow > c ? dropLow - c : 0;
        }
        L.cols[x * hs + sl] = f;
    }
}

// tokens of column x in rows below y
__device__ __forceinline__ int popc_below(const uint64_t *cols, int hs, int x, int y)
{
    int c = 0;
    for (int sl = 0; sl < hs; ++sl) c += popc(cols[x * hs + sl] & low_mask(y - 64 * sl));
    return c;
}

__device__ __forceinline__ bool col_bit(const uint64_t *cols, int hs, int x, int y)
{
    return (cols[x * hs + (y >> 6)] >> (y & 63)) & 1ull;
}

// rank among the tokens of one virtual row (nearest column first, then left): occupied traps of
// that row's diagonal closer to column j, and the left trap at the same distance for a right one
__device__ __forceinline__ int diag_rank(const uint64_t *cols, int hs, int W, int H, int j, int x, int y, bool above)
{
    const int d = x > j ? x - j : j - x;
    const int v = above ? y + d : y - d;
    int q = 0;
    for (int e = 0; e < d; ++e) {
        const int r = above ? v - e : v + e;
        if (r < 0 || r >= H) continue;
        if (e == 0) { q += col_bit(cols, hs, j, r); continue; }
        if (j - e >= 0) q += col_bit(cols, hs, j - e, r);
        if (j + e < W) q += col_bit(cols, hs, j + e, r);
    }
    if (x > j && j - d >= 0) q += col_bit(cols, hs, j - d, y);
    return q;
}

template <int S, int T>
__device__ void bird_columns(SolveLds<S, T / kWave> &L, const SolveArgs &A, int &off, int &g)
{
    constexpr int kThreads = T, kWaves = T / kWave;
    const int tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
    const int W = A.W, H = A.H, x0 = A.x0, y0 = A.y0, x1 = A.x1, y1 = A.y1, sh = y1 - y0;
    const int hs = (H + 63) >> 6;
    const int nT = H - y1 + W, nBl = y0 + W;        // histogram lengths above / below
    for (int j = x0; j < x1; ++j) {
        if (L.sig[j] >= 0) continue;
        for (int u = tid; u < 2 * S + 2; u += kThreads) { L.hT[u] = 0; L.hB[u] = 0; }
        __syncthreads();
        // pass 1: every reservoir token (own ones too) by virtual distance from the band
        for (int p = tid; p < W * hs; p += kThreads) {
            const int x = p / hs, sl = p - x * hs;
            const int d = x > j ? x - j : j - x;
            uint64_t c = L.cols[p] & ~range_mask(y0 - 64 * sl, y1 - 1 - 64 * sl);
            while (c) {
                const int b = __ffsll((unsigned long long)c) - 1;
                c &= c - 1;
                const int y = 64 * sl + b;
                if (y >= y1) atomicAdd(&L.hT[y + d - y1], 1);
                else atomicAdd(&L.hB[y0 - 1 - (y - d)], 1);
            }
        }
        __syncthreads();
        if (wid == 0) {
            // exclusive prefix counts and sums of virtual rows, above and below
            int carryC = 0, carryS = 0;
            for (int base = 0; base < nT; base += kWave) {
                const int u = base + lane;
                const int c = u < nT ? L.hT[u] : 0, sv = c * (y1 + u);
                const int ic = wave_incl_scan(c), is = wave_incl_scan(sv);
                if (u < nT) { L.cT[u + 1] = carryC + ic; L.sT[u + 1] = carryS + is; }
                carryC += __shfl(ic, kWave - 1, kWave); carryS += __shfl(is, kWave - 1, kWave);
            }
            carryC = 0; carryS = 0;
            for (int base = 0; base < nBl; base += kWave) {
                const int u = base + lane;
                const int c = u < nBl ? L.hB[u] : 0, sv = c * (y0 - 1 - u);
                const int ic = wave_incl_scan(c), is = wave_incl_scan(sv);
                if (u < nBl) { L.cB[u + 1] = carryC + ic; L.sB[u + 1] = carryS + is; }
                carryC += __shfl(ic, kWave - 1, kWave); carryS += __shfl(is, kWave - 1, kWave);
            }
            if (lane == 0) { L.cT[0] = 0; L.sT[0] = 0; L.cB[0] = 0; L.sB[0] = 0; }
            wave_sync();
            // own band tokens: E[m] = r_m - y0 - m over their sorted rows, and prefix sums
            int *P0 = L.P[0], *E = L.P[1], *EQ = L.Q[1];
            const int aj = compact_bits_wave(&L.cols[j * hs], hs, P0);
            int nb0 = 0;
            for (int sl = 0; sl < hs; ++sl) nb0 += popc(L.cols[j * hs + sl] & low_mask(y0 - 64 * sl));
            int nbd = 0;
            for (int sl = 0; sl < hs; ++sl) nbd += popc(L.cols[j * hs + sl] & range_mask(y0 - 64 * sl, y1 - 1 - 64 * sl));
            (void)aj;
            for (int m = lane; m < nbd; m += kWave) E[m] = P0[nb0 + m] - y0 - m;
            wave_sync();
            prefix_sums_wave(E, nbd, EQ);
            const int NT = L.cT[nT], NB = L.cB[nBl], need = sh - nbd;
            const int klo = need - NT > 0 ? need - NT : 0, khi = need < NB ? need : NB;
            uint64_t best = ~0ull;
            for (int k = klo + lane; k <= khi; k += kWave) {
                // k nearest below onto y0.., band tokens onto y0+k.., need-k nearest above
                int lo = 0, hi = nBl;                   // last u with cB[u] <= k
                while (lo < hi) { const int mid = (lo + hi + 1) >> 1; if (L.cB[mid] <= k) lo = mid; else hi = mid - 1; }
                const long sumB = L.sB[lo] + (long)(k - L.cB[lo]) * (y0 - 1 - lo);
                const int nt = need - k;
                lo = 0; hi = nT;
                while (lo < hi) { const int mid = (lo + hi + 1) >> 1; if (L.cT[mid] <= nt) lo = mid; else hi = mid - 1; }
                const long sumT = L.sT[lo] + (long)(nt - L.cT[lo]) * (y1 + lo);
                const long cb = (long)k * y0 + (long)k * (k - 1) / 2 - sumB;
                const long ct = sumT - ((long)nt * y1 - (long)nt * (nt + 1) / 2);
                int a = 0, b = nbd;
                while (a < b) { const int mid = (a + b) >> 1; if (E[mid] < k) a = mid + 1; else b = mid; }
                const long cband = (long)k * a - EQ[a] + (EQ[nbd] - EQ[a]) - (long)k * (nbd - a);
                const uint64_t key = ((uint64_t)(cb + cband + ct) << 16) | (uint64_t)(0xFFFF - k);
                best = key < best ? key : best;
            }
            best = wave_min_u64(best);
            if (best == ~0ull && lane == 0) L.misc[M_ERR] = 1;
            const int k = 0xFFFF - (int)(best & 0xFFFFull);
            if (lane == 0) { L.misc[4] = k; L.misc[5] = nb0; L.misc[6] = nbd; }
        }
        __syncthreads();
        const int k = L.misc[4], nb0 = L.misc[5], nbd = L.misc[6];
        const int nt = sh - nbd - k;
        // boundaries: the virtual distance where the k-th (nt-th) nearest token lies, and how
        // many tokens of that virtual row are taken
        int uB = 0, uT = 0;
        {
            int lo = 0, hi = nBl;
            while (lo < hi) { const int mid = (lo + hi + 1) >> 1; if (L.cB[mid] <= k) lo = mid; else hi = mid - 1; }
            uB = lo;
            lo = 0; hi = nT;
            while (lo < hi) { const int mid = (lo + hi + 1) >> 1; if (L.cT[mid] <= nt) lo = mid; else hi = mid - 1; }
            uT = lo;
        }
        const int qB = k - L.cB[uB], qT = nt - L.cT[uT];
        // pass 2: chosen tokens and their targets (sorted virtual order onto y0, y0+1, ...)
        for (int p = tid; p < W * hs; p += kThreads) {
            const int x = p / hs, sl = p - x * hs;
            uint64_t c = L.cols[p];
            if (x != j) c &= ~range_mask(y0 - 64 * sl, y1 - 1 - 64 * sl);
            while (c) {
                const int b = __ffsll((unsigned long long)c) - 1;
                c &= c - 1;
                const int y = 64 * sl + b;
                const int d = x > j ? x - j : j - x;
                int t = -1;
                if (y >= y1) {
                    const int u = y + d - y1;
                    if (u < uT || (u == uT && qT > 0)) {
                        const int q = diag_rank(L.cols, hs, W, H, j, x, y, true);
                        if (u < uT || q < qT) t = y0 + k + nbd + L.cT[u] + q;
                    }
                } else if (y < y0) {
                    const int u = y0 - 1 - (y - d);
                    if (u < uB || (u == uB && qB > 0)) {
                        const int q = diag_rank(L.cols, hs, W, H, j, x, y, false);
                        if (u < uB || q < qB) t = y0 + k - 1 - L.cB[u] - q;
                    }
                } else {
                    t = y0 + k + popc_below(L.cols, hs, j, y) - nb0;
                }
                if (t >= y0 && t < y1) { L.ry[t - y0] = (int16_t)y; L.rorg[t - y0] = (int16_t)x; }
                else if (t != -1) L.misc[M_ERR] = 1;
            }
        }
        __syncthreads();
        // emission: movers towards larger rows by target descending, then towards smaller rows
        // by target ascending
        int up = 0, dn = 0, x = j, y = 0, t = y0 + tid;
        if (tid < sh) {
            y = L.ry[tid]; x = L.rorg[tid];
            const bool moving = (x != j) || (y != t);
            const bool isUp = (x == j) ? (y < t) : (y < y0);
            up = moving && isUp;
            dn = moving && !isUp;
        }
        int nUp, nDn;
        const int upEx = block_excl_scan<kWaves>(up, L.scanA, &nUp);
        const int dnEx = block_excl_scan<kWaves>(dn, L.scanB, &nDn);
        if (up) put_move(A, (uint32_t)(off + nUp - (upEx + 1)), x, y, j, t);
        if (dn) put_move(A, (uint32_t)(off + nUp + dnEx), x, y, j, t);
        int st = (up || dn) ? ((x > j ? x - j : j - x) + (t > y ? t - y : y - t)) : 0;
        st = wave_sum(st);
        if (lane == 0 && st) atomicAdd(&L.misc[M_STEPS], st);
        if (up || dn) atomicAnd((unsigned long long *)&L.cols[x * hs + (y >> 6)], ~(1ull << (y & 63)));
        if (nUp + nDn > 0) {
            if (tid == 0 && g <= (int)A.group_cap) A.goff[g] = (uint32_t)off;
            ++g;
            off += nUp + nDn;
        }
        __syncthreads();
        if (tid < hs) L.cols[j * hs + tid] |= range_mask(y0 - 64 * tid, y1 - 1 - 64 * tid);
        __syncthreads();
    }
}

// ------------------------------------------------------------------------------------------

template <int S, int T>
__device__ void solve_one(SolveLds<S, T / kWave> &L, const SolveArgs &A)
{
    constexpr int kThreads = T, kWaves = T / kWave;
    static_assert(T >= S && T % kWave == 0, "one thread per grid side at least");
    const int tid = threadIdx.x, lane = lane_id(), wid = tid >> 6;
    const int W = A.W, H = A.H, x0 = A.x0, y0 = A.y0, x1 = A.x1, y1 = A.y1;
    const int sw = x1 - x0, sh = y1 - y0;
    const int ws = (W + 63) >> 6, hs = (H + 63) >> 6;
    const bool side = (x0 > 0 || x1 < W);
    const bool serial = (A.flags & 0xFFu) == kOrderSerial;
    const bool birdAlg = (A.flags & 0xFFu) == kBird;
    int *P = L.P[wid];
    int *Q = L.Q[wid];

    // bit rows in, padding dropped
    for (int i = tid; i < H * ws; i += kThreads) {
        const int j = i % ws;
        L.rows[i] = A.occ[i] & low_mask(W - 64 * j);
    }
    if (tid < 8) L.misc[tid] = 0;
    __syncthreads();

    // feasibility: F = N - D - sw*sh, D = band-row tokens beyond sw (parked in side columns)
    int myN = 0, myD = 0;
    if (tid < H) {
        int a = 0;
        for (int j = 0; j < ws; ++j) a += popc(L.rows[tid * ws + j]);
        myN = a;
        if (side && tid >= y0 && tid < y1) myD = a > sw ? a - sw : 0;
    }
    const int N = block_sum<kWaves>(myN, L.scanA);
    const int D = block_sum<kWaves>(myD, L.scanB);
    if ((long)N - D - (long)sw * sh < 0) {
        for (int i = tid; i < H * ws; i += kThreads) A.fin[i] = L.rows[i];
        if (tid == 0) {
            A.goff[0] = 0;
            rr_solve_info inf = {RR_INFEASIBLE, 0u, 0u, 0u, 0u, 0u};
            *A.info = inf;
        }
        return;
    }

    // ---- row pre-pass: each target row solved on its own line -----------------------------
    int nH = 0, gH = 0;
    if (side) {
        for (int y = y0 + wid; y < y1; y += kWaves) {
            const int a = compact_bits_wave(&L.rows[y * ws], ws, P);
            int w0, t0, n;
            if (a >= sw) { w0 = e1d_window_wave(P, Q, a, x0, sw); t0 = x0; n = sw; }
            else { w0 = 0; t0 = x0 + (sw - a) / 2; n = a; }
            int r = 0, c = 0, st = 0;
            for (int k = lane; k < n; k += kWave) {
                const int s = P[w0 + k], t = t0 + k;
                r += s < t; c += s != t; st += s < t ? t - s : s - t;
            }
            r = wave_sum(r); c = wave_sum(c); st = wave_sum(st);
            if (lane == 0) {
                L.rowW[y] = w0; L.rowT0[y] = t0; L.rowN[y] = n; L.rowR[y] = r; L.rowCnt[y] = c;
                atomicAdd(&L.misc[M_STEPS], st);
            }
            wave_sync();
        }
        __syncthreads();
        const int cnt = tid < sh ? L.rowCnt[y0 + tid] : 0;
        const int off = block_excl_scan<kWaves>(cnt, L.scanA, &nH);
        const int gi = block_excl_scan<kWaves>(cnt > 0 ? 1 : 0, L.scanB, &gH);
        if (tid < sh) {
            L.rowOff[y0 + tid] = off;
            if (cnt > 0 && gi <= (int)A.group_cap) A.goff[gi] = (uint32_t)off;
        }
        __syncthreads();
        for (int y = y0 + wid; y < y1; y += kWaves) {
            const int a = compact_bits_wave(&L.rows[y * ws], ws, P);
            const int w0 = L.rowW[y], t0 = L.rowT0[y], n = L.rowN[y];
            if (L.rowCnt[y] > 0) emit_line_wave(A, P, w0, t0, n, L.rowR[y], (uint32_t)L.rowOff[y], true, y);
            if (lane < ws) {
                const uint64_t old = L.rows[y * ws + lane];
                const int sh64 = 64 * lane;
                uint64_t nw;
                if (a >= sw) {
                    const int lo = P[w0], hi = P[w0 + sw - 1];
                    nw = (old & ~range_mask(lo - sh64, hi - sh64)) | range_mask(x0 - sh64, x1 - 1 - sh64);
                } else {
                    nw = range_mask(t0 - sh64, t0 + a - 1 - sh64);
                }
                L.rows[y * ws + lane] = nw;
            }
            wave_sync();
        }
        __syncthreads();
    }

    // ---- column bits by ballot transposition ----------------------------------------------
    for (int p = wid; p < W * hs; p += kWaves) {
        const int x = p / hs, sl = p - x * hs;
        const int y = 64 * sl + lane;
        const bool bit = (y < H) && ((L.rows[y * ws + (x >> 6)] >> (x & 63)) & 1ull);
        const uint64_t m = ballot(bit);
        if (lane == 0) L.cols[x * hs + sl] = m;
    }
    __syncthreads();

    // ---- surplus per column (Alg. 1): central columns count every token, side columns only
    //      their reservoir rows
    if (tid < W) {
        const int x = tid;
        const bool central = (x >= x0 && x < x1);
        int a = 0, nbelow = 0, nband = 0;
        for (int sl = 0; sl < hs; ++sl) {
            const uint64_t c = L.cols[x * hs + sl];
            const uint64_t band = range_mask(y0 - 64 * sl, y1 - 1 - 64 * sl);
            const uint64_t e = central ? c : (c & ~band);
            L.elig[x * hs + sl] = e;
            a += popc(e);
            nbelow += popc(e & low_mask(y0 - 64 * sl));
            nband += popc(e & band);
        }
        const int sigma = a - (central ? sh : 0);
        L.colA[x] = a; L.sig[x] = sigma; L.sp[x] = sigma; L.colCnt[x] = 0;
        // pool of a donor not yet solved: its reservoir tokens, below [0, nbelow) and above
        // [nbelow + nband, a) (side columns: no band tokens)
        L.bcnt[x] = nbelow; L.ubeg[x] = nbelow + nband;
        L.cNb[x] = nbelow; L.cNbd[x] = nband;
        L.dsol[x] = (int8_t)!(serial && central && sigma > 0);
        L.mNb[x] = 0; L.mSb[x] = 0; L.mNt[x] = 0; L.mSt[x] = 0;
    }
    __syncthreads();

    // ---- columns of non-negative surplus, solved from the outset (§III.D); the serial order
    //      of Alg. 1 solves only the columns of zero surplus here ------------------------------
    for (int x = x0 + wid; x < x1; x += kWaves) {
        if (L.sig[x] < 0 || !L.dsol[x]) continue;
        const int a = compact_bits_wave(&L.elig[x * hs], hs, P);
        const int w0 = e1d_window_wave(P, Q, a, y0, sh);
        int u = 0, c = 0, st = 0;
        for (int k = lane; k < sh; k += kWave) {
            const int s = P[w0 + k], t = y0 + k;
            u += s < t; c += s != t; st += s < t ? t - s : s - t;
        }
        u = wave_sum(u); c = wave_sum(c); st = wave_sum(st);
        if (lane == 0) {
            L.colW[x] = w0; L.colU[x] = u; L.colCnt[x] = c;
            L.bcnt[x] = w0; L.ubeg[x] = w0 + sh;
            atomicAdd(&L.misc[M_STEPS], st);
        }
        wave_sync();
    }
    __syncthreads();
    int nA, gA;
    {
        const int cnt = tid < W ? L.colCnt[tid] : 0;
        const int off = block_excl_scan<kWaves>(cnt, L.scanA, &nA);
        const int gi = block_excl_scan<kWaves>(cnt > 0 ? 1 : 0, L.scanB, &gA);
        if (tid < W) {
            L.colOff[tid] = nH + off;
            if (cnt > 0 && gH + gi <= (int)A.group_cap) A.goff[gH + gi] = (uint32_t)(nH + off);
        }
    }
    __syncthreads();
    for (int x = x0 + wid; x < x1; x += kWaves) {
        if (L.sig[x] < 0 || L.colCnt[x] == 0) continue;
        compact_bits_wave(&L.elig[x * hs], hs, P);
        emit_line_wave(A, P, L.colW[x], y0, sh, L.colU[x], (uint32_t)L.colOff[x], false, x);
        wave_sync();
    }
    __syncthreads();

    int off = nH + nA, g = gH + gA;
    if (birdAlg) {
        // ---- bird: the grid after the non-negative columns (band full, their excess where it
        //      stood), then the negative columns leftmost first ----------------------------------
        if (tid < W && tid >= x0 && tid < x1 && L.sig[tid] >= 0) settle_column<S, kWaves>(L, tid, hs, y0, y1, true, true);
        __syncthreads();
        bird_columns<S, T>(L, A, off, g);
    } else {
    // ---- donor/receiver pairs ---------------------------------------------------------------
    if (wid == 0) pair_loop<S, kWaves>(L, W, hs, y0, y1, sh);
    __syncthreads();
    const int nev = L.misc[M_NEV];

    // ---- receiver solves, in the order receivers were saturated; in the serial order a
    //      donor solved with the event follows (case 2) or stands alone (case 3) --------------
    for (int e = 0; e < nev; ++e) {
        if (L.evC[e] != 3) {
        const int j = L.evJ[e];
        const int aj = L.colA[j];
        if (tid < aj && tid < S) { L.ry[tid] = (int16_t)select_in_bits(&L.elig[j * hs], hs, tid); L.rorg[tid] = (int16_t)j; }
        int base = aj;
        for (int e2 = 0; e2 <= e; ++e2) {
            if (L.evJ[e2] != j) continue;
            const int i = L.evI[e2];
            const int blo = L.evBlo[e2], nb = L.evBhi[e2] - blo;
            const int ulo = L.evUlo[e2], nu = L.evUhi[e2] - ulo;
            if (tid < nb + nu && base + tid < S) {
                const int idx = tid < nb ? blo + tid : ulo + (tid - nb);
                L.ry[base + tid] = (int16_t)select_in_bits(&L.elig[i * hs], hs, idx);
                L.rorg[base + tid] = (int16_t)i;
            }
            base += nb + nu;
        }
        if (base != sh) { if (tid == 0) L.misc[M_ERR] = 1; break; }
        __syncthreads();
        // order of sources: by row; tokens standing in one row reach column j in order of
        // distance (own first, then nearer donor, then left donor) and the first to arrive
        // takes the target farther from that row
        if (tid < sh) {
            const int y = L.ry[tid], o = L.rorg[tid];
            const long h = (long)(o > j ? o - j : j - o) * W + o;
            const long tau = (y >= y1) ? h : (y < y0 ? -h : 0);
            L.rkey[tid] = ((uint64_t)y << 32) + (uint64_t)(tau + (1L << 30));
        }
        __syncthreads();
        int up = 0, dn = 0;
        if (tid < sh) {
            const uint64_t k = L.rkey[tid];
            int r = 0;
            for (int s = 0; s < sh; ++s) r += L.rkey[s] < k;
            L.byRank[r] = (int16_t)tid;
        }
        __syncthreads();
        int y = 0, o = 0, t = 0;
        if (tid < sh) {
            const int src = L.byRank[tid];
            y = L.ry[src]; o = L.rorg[src]; t = y0 + tid;
            const bool moving = (o != j) || (y != t);
            up = moving && t >= y;
            dn = moving && t < y;
        }
        int nUp, nDn;
        const int upEx = block_excl_scan<kWaves>(up, L.scanA, &nUp);
        const int dnEx = block_excl_scan<kWaves>(dn, L.scanB, &nDn);
        if (up) put_move(A, (uint32_t)(off + nUp - (upEx + 1)), o, y, j, t);
        if (dn) put_move(A, (uint32_t)(off + nUp + dnEx), o, y, j, t);
        int st = (up || dn) ? ((o > j ? o - j : j - o) + (t > y ? t - y : y - t)) : 0;
        st = wave_sum(st);
        if (lane == 0 && st) atomicAdd(&L.misc[M_STEPS], st);
        if (nUp + nDn > 0) {
            if (tid == 0 && g <= (int)A.group_cap) A.goff[g] = (uint32_t)off;
            ++g;
            off += nUp + nDn;
        }
        __syncthreads();
        }
        if (L.evDW[e] >= 0) {
            // the donor's own solve: exact 1D over the rows it held at that moment
            if (wid == 0) {
                const int i = L.evI[e];
                const int ai = compact_bits_wave(&L.elig[i * hs], hs, L.P[0]);
                const int *R = L.P[1];
                remaining_rows_wave(L.P[0], ai, L.evDbc[e], L.cNb[i], L.cNbd[i], L.evDub[e], L.P[1]);
                const int w = L.evDW[e];
                int u = 0, c = 0, st = 0;
                for (int k = lane; k < sh; k += kWave) {
                    const int s = R[w + k], t = y0 + k;
                    u += s < t; c += s != t; st += s < t ? t - s : s - t;
                }
                u = wave_sum(u); c = wave_sum(c); st = wave_sum(st);
                if (c > 0) emit_line_wave(A, R, w, y0, sh, u, (uint32_t)off, false, i);
                if (lane == 0) {
                    if (c > 0 && g <= (int)A.group_cap) A.goff[g] = (uint32_t)off;
                    L.misc[M_CNT] = c;
                    atomicAdd(&L.misc[M_STEPS], st);
                }
            }
            __syncthreads();
            const int c = L.misc[M_CNT];
            if (c > 0) { ++g; off += c; }
            __syncthreads();
        }
    }

    // ---- serial order: donors still unsolved after the loop, in ascending x, over the tokens
    //      they still hold; their excess stays in the reservoir ----------------------------------
    if (serial) {
        for (int x = x0 + wid; x < x1; x += kWaves) {
            if (L.dsol[x]) continue;
            const int ai = compact_bits_wave(&L.elig[x * hs], hs, Q);
            const int bc = L.bcnt[x], ub = L.ubeg[x], nbd = L.cNbd[x];
            const int ar = remaining_rows_wave(Q, ai, bc, L.cNb[x], nbd, ub, P);
            const int w0 = e1d_window_wave(P, Q, ar, y0, sh);
            int u = 0, c = 0, st = 0;
            for (int k = lane; k < sh; k += kWave) {
                const int s2 = P[w0 + k], t = y0 + k;
                u += s2 < t; c += s2 != t; st += s2 < t ? t - s2 : s2 - t;
            }
            u = wave_sum(u); c = wave_sum(c); st = wave_sum(st);
            if (lane == 0) {
                if (w0 > bc || w0 + sh < bc + nbd) L.misc[M_ERR] = 1;
                L.colW[x] = w0; L.colU[x] = u; L.colCnt[x] = c;
                atomicAdd(&L.misc[M_STEPS], st);
            }
            wave_sync();
        }
        __syncthreads();
        int nZ, gZ;
        const int x = x0 + tid;
        const bool last = x < x1 && !L.dsol[x];
        const int cnt = last ? L.colCnt[x] : 0;
        const int zoff = block_excl_scan<kWaves>(cnt, L.scanA, &nZ);
        const int gi = block_excl_scan<kWaves>(cnt > 0 ? 1 : 0, L.scanB, &gZ);
        if (cnt > 0) {
            L.colOff[x] = off + zoff;
            if (g + gi <= (int)A.group_cap) A.goff[g + gi] = (uint32_t)(off + zoff);
        }
        __syncthreads();
        for (int x2 = x0 + wid; x2 < x1; x2 += kWaves) {
            if (L.dsol[x2]) continue;
            const int ai = compact_bits_wave(&L.elig[x2 * hs], hs, Q);
            const int bc = L.bcnt[x2], ub = L.ubeg[x2];
            remaining_rows_wave(Q, ai, bc, L.cNb[x2], L.cNbd[x2], ub, P);
            const int w0 = L.colW[x2];
            if (L.colCnt[x2] > 0)
                emit_line_wave(A, P, w0, y0, sh, L.colU[x2], (uint32_t)L.colOff[x2], false, x2);
            wave_sync();
            if (lane == 0) {
                // tokens left in the reservoir: those below and above the window
                L.bcnt[x2] = w0;
                L.ubeg[x2] = ub + (w0 + sh - bc - L.cNbd[x2]);
            }
        }
        __syncthreads();
        off += nZ;
        g += gZ;
    }

    // ---- final grid: band full in central columns, parked tokens, remaining pools -----------
    if (tid < W) {
        const bool central = (tid >= x0 && tid < x1);
        settle_column<S, kWaves>(L, tid, hs, y0, y1, central, !central || L.sig[tid] >= 0);
    }
    __syncthreads();
    }
    for (int p = wid; p < H * ws; p += kWaves) {
        const int y = p / ws, j = p - y * ws;
        const int x = 64 * j + lane;
        const bool bit = (x < W) && ((L.cols[x * hs + (y >> 6)] >> (y & 63)) & 1ull);
        const uint64_t m = ballot(bit);
        if (lane == 0) A.fin[p] = m;
    }

    if (tid == 0) {
        const uint32_t nm = (uint32_t)off, ng = (uint32_t)g;
        if (ng <= A.group_cap) A.goff[ng] = nm;
        rr_solve_info inf;
        const bool err = L.misc[M_ERR] != 0;
        const bool cap = nm > A.move_cap || ng > A.group_cap;
        inf.status = err ? RR_E_INTERNAL : (cap ? RR_E_CAPACITY : RR_OK);
        const bool ok = inf.status == RR_OK;
        inf.n_moves = ok ? nm : 0u;
        inf.n_groups = ok ? ng : 0u;
        inf.n_steps = ok ? (uint32_t)L.misc[M_STEPS] : 0u;
        inf.need_moves = nm;
        inf.need_groups = ng;
        *A.info = inf;
    }
}

template <int S, int T>
__global__ __launch_bounds__(T) void k_solve_one(SolveArgs A)
{
    __shared__ SolveLds<S, T / kWave> L;
    solve_one<S, T>(L, A);
}

// Grids beyond RR_LDS_SIDE: the instance's state lives in the workspace (same layout).
constexpr int kWideSide = (int)RR_MAX_SIDE, kWideThreads = 1024;
using WideLds = SolveLds<kWideSide, kWideThreads / kWave>;
constexpr size_t kWideBytes = (sizeof(WideLds) + 255) & ~(size_t)255;

__device__ __forceinline__ bool wide_shape(const rr_shape s) { return s.w > RR_LDS_SIDE || s.h > RR_LDS_SIDE; }

__global__ __launch_bounds__(kWideThreads) void k_solve_wide_one(SolveArgs A, uint8_t *ws)
{
    solve_one<kWideSide, kWideThreads>(*reinterpret_cast<WideLds *>(ws), A);
}

template <int S, int T>
__global__ __launch_bounds__(T) void k_solve_many(const rr_desc *__restrict__ desc, int maxw, int maxh,
                                                  const uint64_t *occ, rr_move *mv, uint32_t *ga,
                                                  uint64_t *fa, rr_solve_info *infos, uint32_t flags)
{
    __shared__ SolveLds<S, T / kWave> L;
    const rr_desc d = desc[blockIdx.x];
    const rr_shape s = d.shape;
    const bool ok = s.w >= 1 && s.h >= 1 && s.w <= maxw && s.h <= maxh && s.w <= S && s.h <= S &&
                    s.x0 < s.x1 && s.x1 <= s.w && s.y0 < s.y1 && s.y1 <= s.h;
    if (!ok && wide_shape(s) && s.w <= maxw && s.h <= maxh) return;   // k_solve_wide_many's instance
    if (!ok) {
        if (threadIdx.x == 0) {
            rr_solve_info inf = {RR_E_INVAL, 0u, 0u, 0u, 0u, 0u};
            infos[blockIdx.x] = inf;
        }
        return;
    }
    SolveArgs A;
    A.W = s.w; A.H = s.h; A.x0 = s.x0; A.y0 = s.y0; A.x1 = s.x1; A.y1 = s.y1;
    A.flags = flags;
    A.occ = occ + d.occ_off;
    A.moves = mv + d.move_off;
    A.move_cap = d.move_cap;
    A.goff = ga + d.group_off;
    A.group_cap = d.group_cap;
    A.fin = fa + d.occ_off;
    A.info = infos + blockIdx.x;
    solve_one<S, T>(L, A);
}

// instances beyond RR_LDS_SIDE of a many-instance launch; instance i's state at ws + i * kWideBytes
__global__ __launch_bounds__(kWideThreads) void k_solve_wide_many(const rr_desc *__restrict__ desc, int maxw, int maxh,
                                                                  const uint64_t *occ, rr_move *mv, uint32_t *ga,
                                                                  uint64_t *fa, rr_solve_info *infos, uint32_t flags,
                                                                  uint8_t *ws)
{
    const rr_desc d = desc[blockIdx.x];
    const rr_shape s = d.shape;
    if (!wide_shape(s)) return;                                       // the LDS launch's instance
    const bool ok = s.w <= maxw && s.h <= maxh && s.w <= kWideSide && s.h <= kWideSide && s.x0 < s.x1 &&
                    s.x1 <= s.w && s.y0 < s.y1 && s.y1 <= s.h;
    if (!ok) {
        if (threadIdx.x == 0) {
            rr_solve_info inf = {RR_E_INVAL, 0u, 0u, 0u, 0u, 0u};
            infos[blockIdx.x] = inf;
        }
        return;
    }
    SolveArgs A;
    A.W = s.w; A.H = s.h; A.x0 = s.x0; A.y0 = s.y0; A.x1 = s.x1; A.y1 = s.y1;
    A.flags = flags;
    A.occ = occ + d.occ_off;
    A.moves = mv + d.move_off;
    A.move_cap = d.move_cap;
    A.goff = ga + d.group_off;
    A.group_cap = d.group_cap;
    A.fin = fa + d.occ_off;
    A.info = infos + blockIdx.x;
    solve_one<kWideSide, kWideThreads>(*reinterpret_cast<WideLds *>(ws + (size_t)blockIdx.x * kWideBytes), A);
}

}  // namespace rr

using namespace rr;

static bool shape_valid(const rr_shape &s)
{
    return s.w >= 1 && s.h >= 1 && s.x0 < s.x1 && s.x1 <= s.w && s.y0 < s.y1 && s.y1 <= s.h;
}

extern "C" size_t rr_solve_workspace_bytes(rr_shape shape)
{
    return (shape.w > RR_LDS_SIDE || shape.h > RR_LDS_SIDE) ? kWideBytes : 0;
}

// flags: bits 0..7 the algorithm, bits 8..11 wavefronts per instance (0: the default, 4)
static bool flags_valid(uint32_t flags)
{
    const uint32_t algo = flags & 0xFFu, waves = (flags >> 8) & 0xFu;
    return algo <= RR_BIRD && (flags >> 12) == 0u && (waves == 0u || waves == 1u || waves == 2u || waves == 4u);
}

static uint32_t threads_of(uint32_t flags)
{
    const uint32_t waves = (flags >> 8) & 0xFu;
    return 64u * (waves ? waves : (uint32_t)(kThreads / kWave));
}

// one launch of the solve kernel for size class S (largest grid side) at T threads per instance
#define RR_SOLVE_DISPATCH(LAUNCH, SIDE, T, OK)                                                              \
    do {                                                                                                    \
        OK = true;                                                                                          \
        if (SIDE <= 64 && T == 64) LAUNCH(64, 64);                                                          \
        else if (SIDE <= 64 && T == 128) LAUNCH(64, 128);                                                   \
        else if (SIDE <= 64 && T == 256) LAUNCH(64, 256);                                                   \
        else if (SIDE > 64 && SIDE <= 128 && T == 128) LAUNCH(128, 128);                                    \
        else if (SIDE > 64 && SIDE <= 128 && T == 256) LAUNCH(128, 256);                                    \
        else if (SIDE > 128 && T == 256) LAUNCH(256, 256);                                                  \
        else OK = false;                                                                                    \
    } while (0)

extern "C" rr_status rr_solve(rr_shape shape, const uint64_t *occ, rr_move *moves, uint32_t move_cap,
                              uint32_t *group_off, uint32_t group_cap, uint64_t *final_occ,
                              rr_solve_info *info, uint32_t flags, void *workspace, size_t workspace_bytes,
                              void *stream)
{
    if (!shape_valid(shape) || !flags_valid(flags)) return RR_E_INVAL;
    if (shape.w > RR_MAX_SIDE || shape.h > RR_MAX_SIDE) return RR_E_UNSUPPORTED;
    if (!occ || !group_off || !final_occ || !info || (move_cap > 0 && !moves)) return RR_E_INVAL;
    if (((uintptr_t)moves & 7u) != 0) return RR_E_INVAL;
    SolveArgs A;
    A.W = shape.w; A.H = shape.h; A.x0 = shape.x0; A.y0 = shape.y0; A.x1 = shape.x1; A.y1 = shape.y1;
    A.flags = flags;
    A.occ = occ; A.moves = moves; A.move_cap = move_cap; A.goff = group_off; A.group_cap = group_cap;
    A.fin = final_occ; A.info = info;
    hipStream_t st = (hipStream_t)stream;
    const uint32_t side = shape.w > shape.h ? shape.w : shape.h;
    if (side > RR_LDS_SIDE) {
        if (((flags >> 8) & 0xFu) != 0u) return RR_E_INVAL;    // the wide kernel runs 16 wavefronts
        if (!workspace || workspace_bytes < kWideBytes || ((uintptr_t)workspace & 255u) != 0) return RR_E_NOMEM;
        hipLaunchKernelGGL(k_solve_wide_one, dim3(1), dim3(kWideThreads), 0, st, A, (uint8_t *)workspace);
        return hipGetLastError() == hipSuccess ? RR_OK : RR_E_DEVICE;
    }
    const uint32_t T = threads_of(flags);
    bool ok;
#define RR_LAUNCH_ONE(SS, TT) hipLaunchKernelGGL((k_solve_one<SS, TT>), dim3(1), dim3(TT), 0, st, A)
    RR_SOLVE_DISPATCH(RR_LAUNCH_ONE, side, T, ok);
#undef RR_LAUNCH_ONE
    if (!ok) return RR_E_INVAL;                  // fewer threads per instance than the grid side
    return hipGetLastError() == hipSuccess ? RR_OK : RR_E_DEVICE;
}

extern "C" rr_status rr_solve_many(uint32_t n, const rr_desc *desc, uint32_t max_w, uint32_t max_h,
                                   const uint64_t *occ_arena, rr_move *move_arena, uint32_t *group_arena,
                                   uint64_t *final_arena, rr_solve_info *infos, uint32_t flags, void *workspace,
                                   size_t workspace_bytes, void *stream)
{
    if (n == 0) return RR_OK;
    if (!flags_valid(flags)) return RR_E_INVAL;
    if (!desc || !occ_arena || !group_arena || !final_arena || !infos || !move_arena) return RR_E_INVAL;
    if (max_w < 1 || max_h < 1) return RR_E_INVAL;
    if (max_w > RR_MAX_SIDE || max_h > RR_MAX_SIDE) return RR_E_UNSUPPORTED;
    if (((uintptr_t)move_arena & 7u) != 0) return RR_E_INVAL;
    hipStream_t st = (hipStream_t)stream;
    const uint32_t max_side = max_w > max_h ? max_w : max_h;
    if (max_side > RR_LDS_SIDE) {
        // instances beyond RR_LDS_SIDE run in the wide kernel, the others in the LDS kernel of
        // the 256 class; each kernel skips the other's instances
        if (!workspace || workspace_bytes / kWideBytes < n || ((uintptr_t)workspace & 255u) != 0) return RR_E_NOMEM;
        hipLaunchKernelGGL(k_solve_wide_many, dim3(n), dim3(kWideThreads), 0, st, desc, (int)max_w, (int)max_h,
                           occ_arena, move_arena, group_arena, final_arena, infos, flags, (uint8_t *)workspace);
        if (hipGetLastError() != hipSuccess) return RR_E_DEVICE;
    }
    const uint32_t side = max_side > RR_LDS_SIDE ? RR_LDS_SIDE : max_side;
    const uint32_t T = threads_of(flags);
    bool ok;
#define RR_LAUNCH_MANY(SS, TT)                                                                              \
    hipLaunchKernelGGL((k_solve_many<SS, TT>), dim3(n), dim3(TT), 0, st, desc, (int)max_w, (int)max_h,       \
                       occ_arena, move_arena, group_arena, final_arena, infos, flags)
    RR_SOLVE_DISPATCH(RR_LAUNCH_MANY, side, T, ok);
#undef RR_LAUNCH_MANY
    if (!ok) return RR_E_INVAL;                  // fewer threads per instance than the grid side
    return hipGetLastError() == hipSuccess ? RR_OK : RR_E_DEVICE;
}

extern "C" const char *rr_version(void) { return "librr 0.1 (gfx950)"; }
