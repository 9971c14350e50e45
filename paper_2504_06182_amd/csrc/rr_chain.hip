// rr_chain.hip -- exact 1D on chains of traps (arXiv 2504.06182, §III.A: assignment and move
// generation; its parallel form, §III.B) on gfx950: one workgroup per chain, many chains per
// launch, chains of up to 65535 traps.
//
// A chain of N traps holds a tokens (bit row, as a 1 x N grid) and a contiguous target
// [b, b+t).  With a >= t the distance-minimising matching is order-preserving on a run of t
// consecutive sorted tokens (exact-1D lemma), so the matching is fixed by the run's start w;
// cost(w) = sum_{k in [w, w+t)} |d_k - (b - w)| with d_k = p_k - k non-decreasing.  The
// workgroup compacts the token positions (scan over the words), scans d into prefix sums,
// prices every run in O(log a) (one bisection for the sign change), takes the cheapest (ties:
// the leftmost run) by a workgroup minimum of 64-bit keys, and emits the moves by scans: paths
// towards larger positions first, largest target first, then the others, smallest target
// first.  Where the paper decomposes the chain into balanced sub-problems by levels and
// profits, a contiguous target needs only the run start; every step here is a scan, a
// reduction or independent per-lane work.
#include "rr_device.hpp"
#include "rr.h"

namespace rr {
namespace chain {

constexpr uint32_t kLdsLen = 8192;   // chains up to this length keep token positions in LDS

struct Args {
    int N, b, t;
    const uint64_t *occ;
    rr_move *moves;
    uint32_t move_cap;
    uint32_t *goff;
    uint32_t group_cap;
    uint64_t *fin;
    rr_solve_info *info;
    int *P, *Qs;                     // token positions and prefix sums of d (LDS or workspace)
};

template <int T>
struct Shared {
    int part[T / kWave];
    uint64_t key[T / kWave];
    int misc[4];
};

// exclusive scan of one int per thread over the workgroup; *total gets the sum
template <int T>
__device__ __forceinline__ int block_excl(int v, Shared<T> &S, int *total)
{
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    const int inc = wave_incl_scan(v);
    if (lane == kWave - 1) S.part[wid] = inc;
    __syncthreads();
    int off = 0, tot = 0;
#pragma unroll
    for (int q = 0; q < T / kWave; ++q) {
        const int p = S.part[q];
        off += q < wid ? p : 0;
        tot += p;
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

template <int T>
__device__ __forceinline__ uint64_t block_min_u64(uint64_t v, Shared<T> &S)
{
    const int lane = lane_id(), wid = threadIdx.x >> 6;
    v = wave_min_u64(v);
    if (lane == 0) S.key[wid] = v;
    __syncthreads();
    uint64_t m = ~0ull;
#pragma unroll
    for (int q = 0; q < T / kWave; ++q) m = S.key[q] < m ? S.key[q] : m;
    __syncthreads();
    return m;
}

template <int T>
__device__ void solve_chain(const Args &A, Shared<T> &S)
{
    const int tid = threadIdx.x;
    const int N = A.N, b = A.b, t = A.t;
    const int nw = (N + 63) >> 6;
    int *P = A.P, *Qs = A.Qs;

    // token positions: one word per thread, scanned into place
    uint64_t word = 0;
    if (tid < nw) word = A.occ[tid] & low_mask(N - 64 * tid);
    int a;
    const int base = block_excl<T>(popc(word), S, &a);
    if (a < t) {                                   // too few tokens: nothing moves
        if (tid < nw) A.fin[tid] = word;
        if (tid == 0) {
            A.goff[0] = 0;
            rr_solve_info inf = {RR_INFEASIBLE, 0u, 0u, 0u, 0u, 0u};
            *A.info = inf;
        }
        return;
    }
    {
        uint64_t w = word;
        int k = base;
        while (w) {
            P[k++] = 64 * tid + __ffsll((unsigned long long)w) - 1;
            w &= w - 1;
        }
    }
    __syncthreads();

    // prefix sums of d_k = p_k - k over contiguous chunks of the tokens
    const int ch = (a + T - 1) / T;
    const int lo = tid * ch < a ? tid * ch : a, hi = lo + ch < a ? lo + ch : a;
    int s = 0;
    for (int k = lo; k < hi; ++k) s += P[k] - k;
    int tot;
    int run = block_excl<T>(s, S, &tot);
    for (int k = lo; k < hi; ++k) { run += P[k] - k; Qs[k + 1] = run; }
    if (tid == 0) Qs[0] = 0;
    __syncthreads();

    // price every run start; cheapest wins, on equal cost the leftmost
    uint64_t best = ~0ull;
    for (int w = tid; w + t <= a; w += T) {
        const int c = b - w;
        int l = w, h = w + t;
        while (l < h) {
            const int m = (l + h) >> 1;
            if (P[m] - m < c) l = m + 1; else h = m;
        }
        const long cost = (long)c * (l - w) - (long)(Qs[l] - Qs[w]) + (long)(Qs[w + t] - Qs[l]) -
                          (long)c * (w + t - l);
        const uint64_t key = ((uint64_t)cost << 24) | (uint64_t)w;
        best = key < best ? key : best;
    }
    best = block_min_u64<T>(best, S);
    const int w0 = (int)(best & 0xFFFFFFull);

    // emission by scans over contiguous chunks of the matched pairs
    const int cht = (t + T - 1) / T;
    const int klo = tid * cht < t ? tid * cht : t, khi = klo + cht < t ? klo + cht : t;
    int r = 0, l = 0, st = 0;
    for (int k = klo; k < khi; ++k) {
        const int p = P[w0 + k], q = b + k;
        r += p < q; l += p > q; st += p < q ? q - p : p - q;
    }
    int R, Lt, steps;
    int rEx = block_excl<T>(r, S, &R);
    int lEx = block_excl<T>(l, S, &Lt);
    block_excl<T>(st, S, &steps);
    const uint32_t nm = (uint32_t)(R + Lt);
    for (int k = klo; k < khi; ++k) {
        const int p = P[w0 + k], q = b + k;
        uint32_t pos;
        if (p < q) pos = (uint32_t)(R - 1 - rEx++);
        else if (p > q) pos = (uint32_t)(R + lEx++);
        else continue;
        if (pos < A.move_cap) {
            const uint64_t v = (uint64_t)(uint16_t)p | ((uint64_t)(uint16_t)q << 32);
            reinterpret_cast<uint64_t *>(A.moves)[pos] = v;
        }
    }

    // final chain: the run's tokens leave [P[w0], P[w0+t-1]], the target fills
    if (tid < nw) {
        const int sh64 = 64 * tid;
        A.fin[tid] = (word & ~range_mask(P[w0] - sh64, P[w0 + t - 1] - sh64)) |
                     range_mask(b - sh64, b + t - 1 - sh64);
    }
    if (tid == 0) {
        const uint32_t ng = nm > 0 ? 1u : 0u;
        if (A.group_cap >= ng) {
            A.goff[0] = 0;
            if (ng) A.goff[1] = nm;
        }
        rr_solve_info inf;
        const bool cap = nm > A.move_cap || ng > A.group_cap;
        inf.status = cap ? RR_E_CAPACITY : RR_OK;
        inf.n_moves = cap ? 0u : nm;
        inf.n_groups = cap ? 0u : ng;
        inf.n_steps = cap ? 0u : (uint32_t)steps;
        inf.need_moves = nm;
        inf.need_groups = ng;
        *A.info = inf;
    }
}

__device__ __forceinline__ bool chain_shape_ok(const rr_shape s, uint32_t max_len)
{
    return s.h == 1 && s.w >= 1 && s.w <= max_len && s.y0 == 0 && s.y1 == 1 && s.x0 < s.x1 && s.x1 <= s.w;
}

extern __shared__ __attribute__((aligned(16))) int chain_lds[];

template <int T>
__global__ __launch_bounds__(T) void k_chains(const rr_desc *__restrict__ desc, uint32_t max_len, const uint64_t *occ,
                                              rr_move *mv, uint32_t *ga, uint64_t *fa, rr_solve_info *infos,
                                              int *ws, uint32_t ws_ints)
{
    __shared__ Shared<T> S;
    const rr_desc d = desc[blockIdx.x];
    if (!chain_shape_ok(d.shape, max_len)) {
        if (threadIdx.x == 0) {
            rr_solve_info inf = {RR_E_INVAL, 0u, 0u, 0u, 0u, 0u};
            infos[blockIdx.x] = inf;
        }
        return;
    }
    Args A;
    A.N = d.shape.w; A.b = d.shape.x0; A.t = d.shape.x1 - d.shape.x0;
    A.occ = occ + d.occ_off;
    A.moves = mv + d.move_off;
    A.move_cap = d.move_cap;
    A.goff = ga + d.group_off;
    A.group_cap = d.group_cap;
    A.fin = fa + d.occ_off;
    A.info = infos + blockIdx.x;
    int *base = ws ? ws + (size_t)blockIdx.x * ws_ints : chain_lds;
    A.P = base;
    A.Qs = base + (max_len + 1);
    solve_chain<T>(A, S);
}

// ints of token positions and prefix sums one chain of max_len traps needs
__host__ __device__ inline size_t chain_ints(uint32_t max_len) { return 2 * ((size_t)max_len + 2); }

}  // namespace chain
}  // namespace rr

using namespace rr;

extern "C" size_t rr_solve_chains_workspace_bytes(uint32_t n, uint32_t max_len)
{
    if (max_len <= chain::kLdsLen) return 0;
    return (size_t)n * chain::chain_ints(max_len) * sizeof(int);
}

extern "C" rr_status rr_solve_chains(uint32_t n, const rr_desc *desc, uint32_t max_len, const uint64_t *occ_arena,
                                     rr_move *move_arena, uint32_t *group_arena, uint64_t *final_arena,
                                     rr_solve_info *infos, void *workspace, size_t workspace_bytes, void *stream)
{
    if (n == 0) return RR_OK;
    if (!desc || !occ_arena || !move_arena || !group_arena || !final_arena || !infos || max_len < 1) return RR_E_INVAL;
    if (max_len > RR_MAX_CHAIN) return RR_E_UNSUPPORTED;
    if (((uintptr_t)move_arena & 7u) != 0) return RR_E_INVAL;
    const size_t need = rr_solve_chains_workspace_bytes(n, max_len);
    if (need && (!workspace || workspace_bytes < need)) return RR_E_NOMEM;
    hipStream_t st = (hipStream_t)stream;
    const uint32_t ints = (uint32_t)chain::chain_ints(max_len);
    int *ws = need ? (int *)workspace : nullptr;
    const size_t lds = need ? 0 : (size_t)ints * sizeof(int);
    if (max_len <= 64u * 256u)
        hipLaunchKernelGGL(chain::k_chains<256>, dim3(n), dim3(256), lds, st, desc, max_len, occ_arena, move_arena,
                           group_arena, final_arena, infos, ws, ints);
    else
        hipLaunchKernelGGL(chain::k_chains<1024>, dim3(n), dim3(1024), lds, st, desc, max_len, occ_arena, move_arena,
                           group_arena, final_arena, infos, ws, ints);
    return hipGetLastError() == hipSuccess ? RR_OK : RR_E_DEVICE;
}
