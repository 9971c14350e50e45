// rr_device.hpp -- wave64 primitives and bit helpers for the CDNA4 kernels of librr.
//
// Everything here is written for gfx950: 64-lane wavefronts, LDS shared by the waves of a
// workgroup, 64-bit ballots.  No warp-32 assumptions anywhere.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rr {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __builtin_amdgcn_mbcnt_hi(~0u, __builtin_amdgcn_mbcnt_lo(~0u, 0u)); }

// Make this wave's LDS/global writes visible to the other lanes of the same wave and keep the
// compiler from moving memory operations across the point.
__device__ __forceinline__ void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

__device__ __forceinline__ int popc(uint64_t v) { return __popcll(v); }

// mask of the n lowest bits, n in [0, 64]
__device__ __forceinline__ uint64_t low_mask(int n) { return n >= 64 ? ~0ull : ((n <= 0) ? 0ull : ((1ull << n) - 1ull)); }

// bits lo..hi (inclusive) of a 64-bit word, clamped to the word
__device__ __forceinline__ uint64_t range_mask(int lo, int hi)
{
    if (hi < lo || hi < 0 || lo > 63) return 0ull;
    lo = lo < 0 ? 0 : lo;
    hi = hi > 63 ? 63 : hi;
    return low_mask(hi + 1) & ~low_mask(lo);
}

// position of the k-th (0-based) set bit of w; w must hold more than k set bits
__device__ __forceinline__ int select_bit(uint64_t w, int k)
{
    int pos = 0;
    int c = __popc((uint32_t)w);
    if (k >= c) { k -= c; w >>= 32; pos += 32; }
    c = __popc((uint32_t)(w & 0xFFFFull));
    if (k >= c) { k -= c; w >>= 16; pos += 16; }
    c = __popc((uint32_t)(w & 0xFFull));
    if (k >= c) { k -= c; w >>= 8; pos += 8; }
    c = __popc((uint32_t)(w & 0xFull));
    if (k >= c) { k -= c; w >>= 4; pos += 4; }
    c = __popc((uint32_t)(w & 0x3ull));
    if (k >= c) { k -= c; w >>= 2; pos += 2; }
    c = (int)(w & 1ull);
    if (k >= c) { pos += 1; }
    return pos;
}

// sum of the positions of the set bits of w (six masked popcounts)
__device__ __forceinline__ int bit_pos_sum(uint64_t w)
{
    return popc(w & 0xAAAAAAAAAAAAAAAAull) + 2 * popc(w & 0xCCCCCCCCCCCCCCCCull) +
           4 * popc(w & 0xF0F0F0F0F0F0F0F0ull) + 8 * popc(w & 0xFF00FF00FF00FF00ull) +
           16 * popc(w & 0xFFFF0000FFFF0000ull) + 32 * popc(w & 0xFFFFFFFF00000000ull);
}

__device__ __forceinline__ int shfl_xor_i(int v, int m) { return __shfl_xor(v, m, kWave); }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = (uint32_t)__shfl_xor((int)lo, m, kWave);
    hi = (uint32_t)__shfl_xor((int)hi, m, kWave);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = (uint32_t)__shfl((int)lo, src, kWave);
    hi = (uint32_t)__shfl((int)hi, src, kWave);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ int wave_sum(int v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) v += shfl_xor_i(v, m);
    return v;
}

__device__ __forceinline__ int wave_min_i(int v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) { int o = shfl_xor_i(v, m); v = o < v ? o : v; }
    return v;
}

__device__ __forceinline__ int wave_max_i(int v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) { int o = shfl_xor_i(v, m); v = o > v ? o : v; }
    return v;
}

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) { uint64_t o = shfl_xor_u64(v, m); v = o < v ? o : v; }
    return v;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t v)
{
#pragma unroll
    for (int m = 32; m > 0; m >>= 1) { uint64_t o = shfl_xor_u64(v, m); v = o > v ? o : v; }
    return v;
}

// inclusive prefix sum over the 64 lanes
__device__ __forceinline__ int wave_incl_scan(int v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        int t = __shfl_up(v, o, kWave);
        if (lane >= o) v += t;
    }
    return v;
}

}  // namespace rr
