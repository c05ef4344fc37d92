// Wave-level top-64 selection for gfx950 (wave64).
//
// Keys pack (count, cell) so that one unsigned compare orders cells by vote
// count descending, then cell index ascending:
//     key = count << 32 | (0xFFFFFFFF - idx),   empty cells: key = 0.
// Every key of a nonempty cell is unique.  A wave keeps its best 64 keys
// sorted descending across its lanes (lane 0 holds the best).  New keys that
// beat the current 64th are merged in: one at a time (ballot finds the slot,
// a one-lane shift opens it) when few lanes qualify, else by a bitonic sort of
// the batch and a bitonic merge with the list.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace rv {

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int m)
{
    const int lo = __shfl_xor((int)(uint32_t)v, m);
    const int hi = __shfl_xor((int)(uint32_t)(v >> 32), m);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ uint64_t shfl_u64(uint64_t v, int src)
{
    const int lo = __shfl((int)(uint32_t)v, src);
    const int hi = __shfl((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

__device__ __forceinline__ uint64_t shfl_up1_u64(uint64_t v)
{
    const int lo = __shfl_up((int)(uint32_t)v, 1);
    const int hi = __shfl_up((int)(uint32_t)(v >> 32), 1);
    return ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
}

// Value of v in lane src, as a wave-uniform (scalar) value.
__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int src)
{
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint64_t cell_key(uint32_t count, uint32_t idx)
{
    return count ? (((uint64_t)count << 32) | (uint64_t)(0xFFFFFFFFu - idx)) : 0ull;
}

__device__ __forceinline__ uint64_t wave_sort_desc(uint64_t key, int lane)
{
#pragma unroll
    for (int k = 2; k <= 64; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint64_t o = shfl_xor_u64(key, j);
            const bool keep_max = ((lane & j) == 0) == ((lane & k) == 0);
            key = keep_max ? umax64(key, o) : umin64(key, o);
        }
    }
    return key;
}

// list and batch both sorted descending; returns the best 64 of the two.
__device__ __forceinline__ uint64_t wave_merge_sorted(uint64_t list, uint64_t batch, int lane)
{
    uint64_t t = umax64(list, shfl_u64(batch, 63 - lane));
#pragma unroll
    for (int j = 32; j > 0; j >>= 1) {
        const uint64_t o = shfl_xor_u64(t, j);
        t = ((lane & j) == 0) ? umax64(t, o) : umin64(t, o);
    }
    return t;
}

// Inserts, one by one, the keys of the lanes set in the uniform mask m.
__device__ __forceinline__ uint64_t wave_insert_each(uint64_t list, uint64_t key, uint64_t m, int lane)
{
    while (m) {
        const int src = __builtin_ctzll(m);
        m &= m - 1;
        const uint64_t k = lane_u64(key, src);
        if (k <= lane_u64(list, 63))
            continue;
        const int p = __popcll(__ballot(list > k));
        const uint64_t up = shfl_up1_u64(list);
        list = (lane > p) ? up : ((lane == p) ? k : list);
    }
    return list;
}

__device__ __forceinline__ uint64_t wave_insert(uint64_t list, uint64_t key, int lane)
{
    const uint64_t m = __ballot(key > lane_u64(list, 63));
    if (m == 0)
        return list;
    if (__popcll(m) > 12)
        return wave_merge_sorted(list, wave_sort_desc(key, lane), lane);
    return wave_insert_each(list, key, m, lane);
}

// Same, for a list whose first K lanes are all that matter: keys that do not
// beat lane K-1 are skipped (lanes K..63 then hold sorted leftovers, real
// keys that no longer matter; lanes 0..K-1 stay the K best keys seen).
__device__ __forceinline__ uint64_t wave_insert_top(uint64_t list, uint64_t key, int lane, int K)
{
    const uint64_t m = __ballot(key > lane_u64(list, K - 1));
    if (m == 0)
        return list;
    if (__popcll(m) > 12)
        return wave_merge_sorted(list, wave_sort_desc(key, lane), lane);
    return wave_insert_each(list, key, m, lane);
}

// Same for a batch that is already sorted descending across the lanes.
__device__ __forceinline__ uint64_t wave_insert_sorted(uint64_t list, uint64_t sorted, int lane)
{
    const uint64_t m = __ballot(sorted > lane_u64(list, 63));
    if (m == 0)
        return list;
    if (__popcll(m) > 12)
        return wave_merge_sorted(list, sorted, lane);
    return wave_insert_each(list, sorted, m, lane);
}

// Merges the lists of the block's waves (through LDS) into wave 0's list, as
// a tree: in each round the lower half of the remaining waves merges in the
// upper half's lists (log2(kWaves) rounds instead of kWaves - 1 merges in one
// wave while the others wait).
template <int kWaves>
__device__ __forceinline__ uint64_t block_merge(uint64_t list, uint64_t (*lists)[64], int wave, int lane)
{
    static_assert((kWaves & (kWaves - 1)) == 0, "power-of-two wave count");
    lists[wave][lane] = list;
    __syncthreads();
#pragma unroll
    for (int half = kWaves / 2; half >= 1; half >>= 1) {
        // round readers use waves [half, 2 half), writers [0, half)
        if (wave < half) {
            list = wave_insert_sorted(list, lists[wave + half][lane], lane);
            lists[wave][lane] = list;
        }
        __syncthreads();
    }
    return list;
}

}  // namespace rv
