// HIP kernels of the rotation-voting solve for gfx950 (CDNA4, wave64).
//
// Stages (one solve, all on one stream):
//   clear grid -> vote (sample circles, bin, accumulate) -> top-K partial ->
//   top-K final (+ decode candidates) -> rescore (exact inlier counts) ->
//   mask (winner, inlier mask, result record).
// The vote is scatter/count work, not a dense contraction, so no MFMA is used.
#include "rv_device.h"
#include "rv_internal.h"

namespace rv {

// ---------------------------------------------------------------- utilities

__global__ __launch_bounds__(256) void k_fill(int32_t* __restrict__ p, int64_t count, int32_t value)
{
    const int64_t nvec = count >> 2;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    int4* p4 = reinterpret_cast<int4*>(p);
    const int4 v4 = make_int4(value, value, value, value);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nvec; i += stride)
        p4[i] = v4;
    const int64_t tail = (int64_t)blockIdx.x * blockDim.x + threadIdx.x + (nvec << 2);
    if (tail < count)
        p[tail] = value;
}

hipError_t launch_fill(int32_t* p, int64_t count, int32_t value, hipStream_t s)
{
    if (count <= 0)
        return hipSuccess;
    const int64_t nvec = (count >> 2) + 1;
    const int blocks = (int)std::min<int64_t>((nvec + 255) / 256, 4096);
    hipLaunchKernelGGL(k_fill, dim3(blocks), dim3(256), 0, s, p, count, value);
    return hipGetLastError();
}

__device__ __forceinline__ void atomic_add_relaxed(int32_t* p, int32_t v)
{
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// --------------------------------------------------------------------- vote

// Alg. 1's loop, one wave per (group of 64 correspondences, chunk of samples):
// every lane owns one correspondence, all lanes walk the same sample indices
// so the (cos, sin) table entry is wave-uniform (scalar loads).  Consecutive
// samples of one circle usually fall in the same cell, so each lane merges
// them into a run and adds the run length with one atomic when the cell
// changes.  The sum over runs equals one vote per sample exactly.
template <bool kFastRecip>
__global__ __launch_bounds__(256) void k_vote_global(const float* __restrict__ x,
                                                     const float* __restrict__ y, int64_t n,
                                                     int G, float H, int J, int chunk,
                                                     int ngroups, int nwaves,
                                                     const float2* __restrict__ table,
                                                     int32_t* __restrict__ hist)
{
    const int wave = __builtin_amdgcn_readfirstlane((int)(blockIdx.x * 4 + (threadIdx.x >> 6)));
    if (wave >= nwaves)
        return;
    const int lane = threadIdx.x & 63;
    const int c = wave / ngroups;
    const int g = wave - c * ngroups;
    const int j0 = c * chunk;
    const int j1 = min(J, j0 + chunk);
    const int64_t i = (int64_t)g * kWave + lane;

    float a[3], b[3];
    bool ok = false;
    if (i < n) {
        const bool oka = load_unit(x, n, i, a);
        const bool okb = load_unit(y, n, i, b);
        ok = oka && okb;
    }
    if (!ok) {
        a[0] = 1.0f; a[1] = 0.0f; a[2] = 0.0f;
        b[0] = 1.0f; b[1] = 0.0f; b[2] = 0.0f;
    }
    const int inc = ok ? 1 : 0;
    Quat u, v;
    circle_basis(a, b, u, v);

    int cur = 0;
    int cnt = 0;
#pragma unroll 4
    for (int j = j0; j < j1; ++j) {
        const float2 cs = table[j];
        const int idx = sample_cell<kFastRecip>(u, v, cs.x, cs.y, H, G);
        if (idx != cur) {
            if (cnt > 0)
                atomic_add_relaxed(hist + cur, cnt);
            cur = idx;
            cnt = 0;
        }
        cnt += inc;
    }
    if (cnt > 0)
        atomic_add_relaxed(hist + cur, cnt);
}

hipError_t launch_vote_global(const float* x, const float* y, int64_t n, int G, int J,
                              const float2* table, int32_t* hist, int chunk, hipStream_t s)
{
    if (n <= 0 || J <= 0)
        return hipSuccess;
    if (chunk <= 0 || chunk > J)
        chunk = J;
    const int64_t ngroups = (n + kWave - 1) / kWave;
    const int64_t nchunks = (J + chunk - 1) / chunk;
    const int64_t nwaves = ngroups * nchunks;
    if (nwaves > (int64_t)INT32_MAX - 4)
        return hipErrorInvalidValue;
    const int blocks = (int)((nwaves + 3) / 4);
    const float H = (float)G * 0.5f;
    hipLaunchKernelGGL(k_vote_global<false>, dim3(blocks), dim3(256), 0, s, x, y, n, G, H, J,
                       chunk, (int)ngroups, (int)nwaves, table, hist);
    return hipGetLastError();
}

// -------------------------------------------------------------------- top-K
//
// Keys pack (count, index) so that one unsigned compare orders cells by count
// descending, then index ascending: key = count << 32 | (0xFFFFFFFF - idx).
// Empty cells have key 0 and are never candidates.  Each wave keeps its best
// 64 keys sorted descending across its 64 lanes; a batch of 64 new keys is
// skipped unless one beats the current 64th key, else it is bitonic-sorted
// and merged in (max against the reversed batch, then a bitonic clean).

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

__device__ __forceinline__ uint64_t lane_u64(uint64_t v, int src)
{
    const uint32_t lo = __builtin_amdgcn_readlane((int)(uint32_t)v, src);
    const uint32_t hi = __builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t umax64(uint64_t a, uint64_t b) { return a > b ? a : b; }
__device__ __forceinline__ uint64_t umin64(uint64_t a, uint64_t b) { return a < b ? a : b; }

__device__ __forceinline__ uint64_t wave_sort_desc(uint64_t key, int lane)
{
#pragma unroll
    for (int k = 2; k <= kWave; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            const uint64_t o = shfl_xor_u64(key, j);
            const bool keep_max = ((lane & j) == 0) == ((lane & k) == 0);
            key = keep_max ? umax64(key, o) : umin64(key, o);
        }
    }
    return key;
}

// list and batch both sorted descending; returns the best 64 of both, sorted.
__device__ __forceinline__ uint64_t wave_merge_sorted(uint64_t list, uint64_t batch, int lane)
{
    uint64_t t = umax64(list, shfl_u64(batch, kWave - 1 - lane));
#pragma unroll
    for (int j = kWave / 2; j > 0; j >>= 1) {
        const uint64_t o = shfl_xor_u64(t, j);
        t = ((lane & j) == 0) ? umax64(t, o) : umin64(t, o);
    }
    return t;
}

__device__ __forceinline__ uint64_t wave_insert(uint64_t list, uint64_t key, int lane)
{
    const uint64_t thr = lane_u64(list, kWave - 1);
    if (__ballot(key > thr) == 0)
        return list;
    return wave_merge_sorted(list, wave_sort_desc(key, lane), lane);
}

__device__ __forceinline__ uint64_t wave_insert_sorted(uint64_t list, uint64_t sorted, int lane)
{
    const uint64_t thr = lane_u64(list, kWave - 1);
    if (__ballot(sorted > thr) == 0)
        return list;
    return wave_merge_sorted(list, sorted, lane);
}

__device__ __forceinline__ uint64_t cell_key(int32_t count, int64_t idx)
{
    return count > 0 ? (((uint64_t)(uint32_t)count << 32) | (uint32_t)(0xFFFFFFFFu - (uint32_t)idx))
                     : 0ull;
}

constexpr int kTopkThreads = 1024;
constexpr int kTopkWaves = kTopkThreads / kWave;

// Merges the block's per-wave lists (in lists[]) into wave 0's register list.
__device__ __forceinline__ uint64_t block_merge(uint64_t list, uint64_t (*lists)[kWave], int wave,
                                                int lane)
{
    lists[wave][lane] = list;
    __syncthreads();
    if (wave == 0) {
        for (int w = 1; w < kTopkWaves; ++w)
            list = wave_insert_sorted(list, lists[w][lane], lane);
    }
    return list;
}

__global__ __launch_bounds__(kTopkThreads) void k_topk_partial(const int32_t* __restrict__ hist,
                                                               int64_t ncell,
                                                               uint64_t* __restrict__ partial)
{
    __shared__ uint64_t lists[kTopkWaves][kWave];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int64_t ntiles = (ncell + 255) / 256;
    const int64_t gw = (int64_t)blockIdx.x * kTopkWaves + wave;
    const int64_t stride = (int64_t)gridDim.x * kTopkWaves;
    uint64_t list = 0;
    for (int64_t t = gw; t < ntiles; t += stride) {
        const int64_t base = t * 256 + lane * 4;
        int32_t h[4];
        if (t * 256 + 256 <= ncell) {
            const int4 v = *reinterpret_cast<const int4*>(hist + base);
            h[0] = v.x; h[1] = v.y; h[2] = v.z; h[3] = v.w;
        } else {
#pragma unroll
            for (int s = 0; s < 4; ++s)
                h[s] = (base + s < ncell) ? hist[base + s] : 0;
        }
        uint64_t k[4];
#pragma unroll
        for (int s = 0; s < 4; ++s)
            k[s] = cell_key(h[s], base + s);
        const uint64_t thr = lane_u64(list, kWave - 1);
        const bool any = (k[0] > thr) | (k[1] > thr) | (k[2] > thr) | (k[3] > thr);
        if (__ballot(any) != 0) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
                list = wave_insert(list, k[s], lane);
        }
    }
    list = block_merge(list, lists, wave, lane);
    if (wave == 0)
        partial[(int64_t)blockIdx.x * kWave + lane] = list;
}

int topk_blocks(int64_t ncell)
{
    const int64_t tiles = (ncell + 255) / 256;
    const int64_t per_block = kTopkWaves * 4;  // about four tiles per wave
    return (int)std::max<int64_t>(1, std::min<int64_t>(kTopkMaxBlocks, (tiles + per_block - 1) / per_block));
}

hipError_t launch_topk_partial(const int32_t* hist, int64_t ncell, int nblocks, uint64_t* partial,
                               hipStream_t s)
{
    hipLaunchKernelGGL(k_topk_partial, dim3(nblocks), dim3(kTopkThreads), 0, s, hist, ncell,
                       partial);
    return hipGetLastError();
}

__global__ __launch_bounds__(kTopkThreads) void k_topk_final(const uint64_t* __restrict__ partial,
                                                             int nblocks, int K, int G,
                                                             Candidates c)
{
    __shared__ uint64_t lists[kTopkWaves][kWave];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    uint64_t list = 0;
    for (int b = wave; b < nblocks; b += kTopkWaves)
        list = wave_insert_sorted(list, partial[(int64_t)b * kWave + lane], lane);
    list = block_merge(list, lists, wave, lane);
    if (wave != 0)
        return;
    const bool valid = lane < K && list != 0;
    const int ncand = __popcll(__ballot(valid));
    const int32_t votes = (int32_t)(list >> 32);
    const int32_t idx = (int32_t)(0xFFFFFFFFu - (uint32_t)list);
    if (valid) {
        const Quat q = decode_cell(idx, G);
        c.q[lane] = make_float4(q.w, q.x, q.y, q.z);
        c.votes[lane] = votes;
        c.idx[lane] = idx;
    }
    c.inliers[lane] = 0u;
    if (lane == 0)
        c.result->n_cand = ncand;
}

hipError_t launch_topk_final(const uint64_t* partial, int nblocks, int K, int G,
                             const Candidates& c, hipStream_t s)
{
    hipLaunchKernelGGL(k_topk_final, dim3(1), dim3(kTopkThreads), 0, s, partial, nblocks, K, G, c);
    return hipGetLastError();
}

// ------------------------------------------------------------------ rescore
//
// Exact inlier counts of every candidate over all correspondences: the
// residual of App. D's constraint against the bound 4 sin^2(eps/2), a wave
// ballot + popcount per candidate, lane k of each wave accumulating candidate
// k's count, a block reduction in LDS, one atomic per candidate per block.

constexpr int kRescoreThreads = 256;

__global__ __launch_bounds__(kRescoreThreads) void k_rescore(const float* __restrict__ x,
                                                             const float* __restrict__ y,
                                                             int64_t n, float T2, Candidates c)
{
    __shared__ uint32_t partial[kRescoreThreads / kWave][kWave];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int ncand = __builtin_amdgcn_readfirstlane(c.result->n_cand);
    uint32_t acc = 0;
    const int64_t stride = (int64_t)gridDim.x * kRescoreThreads;
    for (int64_t base = (int64_t)blockIdx.x * kRescoreThreads + wave * kWave; base < n;
         base += stride) {
        const int64_t i = base + lane;
        float a[3] = {1.0f, 0.0f, 0.0f};
        float b[3] = {1.0f, 0.0f, 0.0f};
        bool ok = false;
        if (i < n) {
            const bool oka = load_unit(x, n, i, a);
            const bool okb = load_unit(y, n, i, b);
            ok = oka && okb;
        }
        float D[3], P[3];
#pragma unroll
        for (int m = 0; m < 3; ++m) {
            D[m] = a[m] - b[m];
            P[m] = a[m] + b[m];
        }
        for (int k = 0; k < ncand; ++k) {
            const float4 q4 = c.q[k];
            const Quat q{q4.x, q4.y, q4.z, q4.w};
            const bool in = ok && (residual2(D, P, q) <= T2);
            const uint32_t cnt = (uint32_t)__popcll(__ballot(in));
            acc += (lane == k) ? cnt : 0u;
        }
    }
    partial[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && lane < ncand) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < kRescoreThreads / kWave; ++w)
            s += partial[w][lane];
        if (s)
            __hip_atomic_fetch_add(c.inliers + lane, s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

hipError_t launch_rescore(const float* x, const float* y, int64_t n, float T2, const Candidates& c,
                          hipStream_t s)
{
    if (n <= 0)
        return hipSuccess;
    const int blocks = (int)std::min<int64_t>((n + kRescoreThreads - 1) / kRescoreThreads, 2048);
    hipLaunchKernelGGL(k_rescore, dim3(blocks), dim3(kRescoreThreads), 0, s, x, y, n, T2, c);
    return hipGetLastError();
}

// --------------------------------------------------------------------- mask
//
// Winner = most inliers, ties to the earlier candidate (more votes, then lower
// cell index).  Every block finds it from the <= 64 counts; block 0 writes the
// result record.

__global__ __launch_bounds__(256) void k_mask(const float* __restrict__ x,
                                              const float* __restrict__ y, int64_t n, float T2,
                                              Candidates c, uint8_t* __restrict__ mask)
{
    __shared__ int s_win;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < kWave) {
        const int ncand = c.result->n_cand;
        uint64_t key = 0;
        if (lane < ncand)
            key = (((uint64_t)c.inliers[lane] + 1ull) << 6) | (uint64_t)(kWave - 1 - lane);
#pragma unroll
        for (int m = kWave / 2; m > 0; m >>= 1)
            key = umax64(key, shfl_xor_u64(key, m));
        if (lane == 0)
            s_win = key ? (kWave - 1 - (int)(key & 63)) : -1;
    }
    __syncthreads();
    const int win = s_win;
    Quat q{1.0f, 0.0f, 0.0f, 0.0f};
    if (win >= 0) {
        const float4 q4 = c.q[win];
        q = Quat{q4.x, q4.y, q4.z, q4.w};
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        Result* r = c.result;
        r->q[0] = q.w;
        r->q[1] = q.x;
        r->q[2] = q.y;
        r->q[3] = q.z;
        r->count = win >= 0 ? (int64_t)c.inliers[win] : 0;
        r->winner = win;
    }
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        float a[3], b[3];
        const bool oka = load_unit(x, n, i, a);
        const bool okb = load_unit(y, n, i, b);
        bool in = false;
        if (oka && okb && win >= 0) {
            float D[3], P[3];
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                D[m] = a[m] - b[m];
                P[m] = a[m] + b[m];
            }
            in = residual2(D, P, q) <= T2;
        }
        mask[i] = in ? 1 : 0;
    }
}

hipError_t launch_mask(const float* x, const float* y, int64_t n, float T2, const Candidates& c,
                       uint8_t* mask, hipStream_t s)
{
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048));
    hipLaunchKernelGGL(k_mask, dim3(blocks), dim3(256), 0, s, x, y, n, T2, c, mask);
    return hipGetLastError();
}

}  // namespace rv
