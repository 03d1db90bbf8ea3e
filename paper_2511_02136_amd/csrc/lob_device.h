/*
 * Device-side building blocks of the LOB environment step (gfx950, wave64).
 *
 * One wavefront owns one environment.  Its book lives in LDS as records of four int32
 * fields (price, qty, oid, tid) plus a time reference each, per side in priority order
 * from the worst order (record 0) to the best (record n-1).  Record j of a side is
 * handled by lane j % 64 in "row" j / 64, so a row access is one 128-bit LDS
 * instruction for the records and one 32-bit one for the time references.
 * Searches are ballots over rows from the top of the book down, and insertion /
 * removal move the records of the rows they touch by whole-wave LDS copies.
 *
 * All control flow that decides what happens to the book is wave-uniform.  LDS accesses
 * of one wavefront are performed in order by the hardware; WAVE_SYNC() stops the compiler
 * from moving LDS loads and stores across the phases of a shift.
 */
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define WAVE_SYNC() __asm__ volatile("" ::: "memory")

namespace lobk {

constexpr int WAVE = 64;
constexpr int NF = 6; /* fields per slot */
enum { FP = 0, FQ = 1, FO = 2, FT = 3, FS = 4, FN = 5 };
enum { T_LIMIT = 1, T_PCANCEL = 2, T_DELETE = 3, T_MARKET = 4, T_EXECUTE = 5, T_IGNORED = 6 };
enum { C_MSGS, C_TRADES, C_MISS, C_EVICT, C_EVICTED_QTY, C_DROP, C_DROPPED_QTY, C_MARKET_UNFILLED,
       C_BAD, C_TRADE_OVERFLOW, C_IGNORED, NCTR };

/* ---------------------------------------------------------------- wave primitives */
__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & (WAVE - 1)); }

/* the comparison's lane mask itself (no round trip through an int predicate) */
__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

/* lane masks of a comparison (bit l = lane l); every lane of the wave is active where
 * these are used */
__device__ __forceinline__ uint64_t lanes_eq(int a, int b) { return __builtin_amdgcn_sicmp(a, b, 32); }
__device__ __forceinline__ uint64_t lanes_gt(int a, int b) { return __builtin_amdgcn_sicmp(a, b, 38); }
__device__ __forceinline__ uint64_t lanes_ge(int a, int b) { return __builtin_amdgcn_sicmp(a, b, 39); }
__device__ __forceinline__ uint64_t lanes_lt(int a, int b) { return __builtin_amdgcn_sicmp(a, b, 40); }
__device__ __forceinline__ uint64_t lanes_le(int a, int b) { return __builtin_amdgcn_sicmp(a, b, 41); }

/* lane l takes lane l + 1's value (lane 63 takes 0): the whole-wave DPP shift */
__device__ __forceinline__ int shl1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x130, 0xF, 0xF, false); }
__device__ __forceinline__ int2 shl1(int2 v) { return make_int2(shl1(v.x), shl1(v.y)); }

/* lane l takes lane l - 1's value (lane 0 takes 0) */
__device__ __forceinline__ int shr1(int v) { return __builtin_amdgcn_update_dpp(0, v, 0x138, 0xF, 0xF, false); }

/* inclusive prefix sum over the 64 lanes, saturating at 2^31 - 1: shifts within each row
 * of 16 lanes, then the broadcasts of lane 15 into rows 1 and 3 and of lane 31 into rows
 * 2 and 3 */
__device__ __forceinline__ unsigned sat_add(unsigned a, unsigned b) {
    const unsigned s = a + b;
    return s > 0x7fffffffu ? 0x7fffffffu : s;
}
__device__ __forceinline__ unsigned scan_sat(unsigned x) {
    x = sat_add(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xF, 0xF, true)); /* row_shr:1 */
    x = sat_add(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xF, 0xF, true)); /* row_shr:2 */
    x = sat_add(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xF, 0xF, true)); /* row_shr:4 */
    x = sat_add(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xF, 0xF, true)); /* row_shr:8 */
    x = sat_add(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xA, 0xF, false)); /* row_bcast:15 */
    x = sat_add(x, (unsigned)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xC, 0xF, false)); /* row_bcast:31 */
    return x;
}

__device__ __forceinline__ int rdlane(int v, int l) { return __builtin_amdgcn_readlane(v, l); }

__device__ __forceinline__ int64_t rdlane64(int64_t v, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)v >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int uni(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int64_t uni64(int64_t v) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)v);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)((uint64_t)v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

/* inclusive prefix sum over the 64 lanes (int64) */
__device__ __forceinline__ int64_t wave_incl_scan64(int64_t x, int lane) {
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        int64_t y = __shfl_up(x, d, WAVE);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ int64_t wave_sum64(int64_t x) {
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) x += __shfl_xor(x, d, WAVE);
    return x;
}

/* ---------------------------------------------------------------- counter hash
 * SplitMix64's output function (Steele, Lea, Flood 2014) applied in a chain over the key
 * words.  Used for the shuffle keys and the random policy. */
__device__ __forceinline__ uint64_t sm64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t hash4(uint64_t seed, uint64_t dom, uint64_t a, uint64_t b, uint64_t c) {
    return sm64(sm64(sm64(sm64(seed ^ dom) ^ a) ^ b) ^ c);
}
constexpr uint64_t DOM_SHUFFLE = 0x5348554646ULL;
constexpr uint64_t DOM_ACTION = 0x414354ULL;

} // namespace lobk
