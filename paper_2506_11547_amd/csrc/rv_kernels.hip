// HIP kernels of the rotation-voting solve for gfx950 (CDNA4, wave64).
//
// Stages (one solve, all on one stream):
//   clear grid -> vote (sample circles, bin, accumulate) -> top-K partial ->
//   top-K final (+ decode candidates) -> rescore (exact inlier counts) ->
//   mask (winner, inlier mask, result record).
// The vote is scatter/count work, not a dense contraction, so no MFMA is used.
#include <algorithm>

#include "rv_device.h"
#include "rv_internal.h"
#include "rv_topk.h"

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
__global__ __launch_bounds__(256) void k_vote_global(const float* __restrict__ x,
                                                     const float* __restrict__ y, int64_t n,
                                                     int G, float H, float gm, int J, int chunk,
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
    Quat u, v;
    const bool ok = load_circle(x, y, n, (int64_t)g * kWave + lane, u, v);
    const int inc = ok ? 1 : 0;
    unsigned cur = 0xFFFFFFFFu;
    int cnt = 0;
    for_samples<true>(u, v, table, j0, j1, H, gm, [&](const Cell& cell, int) {
        const unsigned idx = linear_index(cell, (unsigned)G);
        if (idx != cur) {
            if (cnt > 0)
                atomic_add_relaxed(hist + cur, cnt);
            cur = idx;
            cnt = 0;
        }
        cnt += inc;
    });
    if (cnt > 0)
        atomic_add_relaxed(hist + cur, cnt);
}

hipError_t launch_vote_global(const float* x, const float* y, int64_t n, int G, int J,
                              const float2* table, int32_t* hist, int chunk, hipStream_t s)
{
    if (n <= 0 || J <= 0)
        return hipSuccess;
    const int64_t ngroups = (n + kWave - 1) / kWave;
    if (chunk <= 0) {
        // Split J into chunks of whole table rows (8 samples) until there
        // are about 8192 waves (8 per SIMD): a few thousand correspondences
        // would otherwise keep a few CUs busy for the whole circle.  A cut
        // only ends a run early; the counts are the same.
        constexpr int64_t kTargetWaves = 8192;
        const int64_t rows = (J + 7) / 8;
        const int64_t want = (kTargetWaves + ngroups - 1) / ngroups;
        const int64_t nch = std::min<int64_t>(std::max<int64_t>(want, 1), rows);
        chunk = (int)(((rows + nch - 1) / nch) * 8);
    }
    if (chunk >= J)
        chunk = J;
    else
        chunk = (chunk + 7) & ~7;  // sample chunks start on table rows of 8
    const int64_t nchunks = (J + chunk - 1) / chunk;
    const int64_t nwaves = ngroups * nchunks;
    if (nwaves > (int64_t)INT32_MAX - 4)
        return hipErrorInvalidValue;
    const int blocks = (int)((nwaves + 3) / 4);
    const float H = (float)G * 0.5f;
    const float gm = (float)G - 0.5f;
    hipLaunchKernelGGL(k_vote_global, dim3(blocks), dim3(256), 0, s, x, y, n, G, H, gm, J, chunk,
                       (int)ngroups, (int)nwaves, table, hist);
    return hipGetLastError();
}

// -------------------------------------------------------------------- top-K
//
// Per-block sorted top-64 lists over disjoint parts of the grid (or the brick
// accumulation's per-brick lists), then one block merges the lists that can
// hold a key of the top K (their maximum reaches the K-th largest maximum),
// decodes the K best cells and clears their counters.

constexpr int kTopkThreads = 1024;
constexpr int kTopkWaves = kTopkThreads / kWave;
constexpr int kTopkFloorLists = 256;  // more lists than this: the final merge prunes them

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
            k[s] = h[s] > 0 ? cell_key((uint32_t)h[s], (uint32_t)(base + s)) : 0ull;
        const uint64_t thr = lane_u64(list, kWave - 1);
        const bool any = (k[0] > thr) | (k[1] > thr) | (k[2] > thr) | (k[3] > thr);
        if (__ballot(any) != 0) {
#pragma unroll
            for (int s = 0; s < 4; ++s)
                list = wave_insert(list, k[s], lane);
        }
    }
    list = block_merge<kTopkWaves>(list, lists, wave, lane);
    if (wave == 0)
        partial[(int64_t)blockIdx.x * kWave + lane] = list;
}

int topk_blocks(int64_t ncell)
{
    const int64_t tiles = (ncell + 255) / 256;
    const int64_t per_block = kTopkWaves;  // about one tile per wave (small grids: more blocks)
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
    __shared__ uint64_t s_floor;
    __shared__ uint16_t s_keep[kTopkMaxBlocks];
    __shared__ uint32_t s_nkeep;
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    // Many lists: first a floor, the K-th largest of the lists' maxima (each
    // list's lane 0).  K distinct cells reach it, so every key of the top K
    // does, and a list whose maximum is below it holds none of them: only the
    // lists that reach it are merged, without their entries below it.  (Few
    // lists are merged whole: the floor would cost more than it saves.)
    const bool pruned = nblocks > kTopkFloorLists;
    uint64_t floor_k = 0;
    int nkeep = nblocks;
    if (pruned) {
        if (threadIdx.x == 0)
            s_nkeep = 0u;
        uint64_t m = 0;
        for (int base = wave * kWave; base < nblocks; base += kTopkThreads) {
            const int b = base + lane;
            const uint64_t v = b < nblocks ? partial[(int64_t)b * kWave] : 0ull;
            m = wave_insert_sorted(m, wave_sort_desc(v, lane), lane);
        }
        m = block_merge<kTopkWaves>(m, lists, wave, lane);
        if (wave == 0 && lane == 0)
            s_floor = lane_u64(m, K - 1);
        __syncthreads();
        floor_k = s_floor;
        for (int base = wave * kWave; base < nblocks; base += kTopkThreads) {
            const int b = base + lane;
            const uint64_t v = b < nblocks ? partial[(int64_t)b * kWave] : 0ull;
            const bool reach = v != 0ull && v >= floor_k;
            const uint64_t mk = __ballot(reach);
            uint32_t first = 0u;
            if (lane == 0 && mk)
                first = atomicAdd(&s_nkeep, (uint32_t)__popcll(mk));
            first = __shfl(first, 0);
            const uint32_t r = __builtin_amdgcn_mbcnt_hi((uint32_t)(mk >> 32),
                                                         __builtin_amdgcn_mbcnt_lo((uint32_t)mk, 0u));
            if (reach)
                s_keep[first + r] = (uint16_t)b;
        }
        __syncthreads();
        nkeep = (int)s_nkeep;
    }
    // eight lists in flight per wave, so the merge does not wait on each load
    uint64_t list = 0;
    for (int i0 = wave; i0 < nkeep; i0 += kTopkWaves * 8) {
        uint64_t pre[8];
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            const int i = i0 + r * kTopkWaves;
            const int b = i < nkeep ? (pruned ? (int)s_keep[i] : i) : 0;
            const uint64_t e = i < nkeep ? partial[(int64_t)b * kWave + lane] : 0ull;
            pre[r] = e >= floor_k ? e : 0ull;
        }
#pragma unroll
        for (int r = 0; r < 8; ++r)
            list = wave_insert_sorted(list, pre[r], lane);
    }
    list = block_merge<kTopkWaves>(list, lists, wave, lane);
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
    if (nblocks < 0 || nblocks > kTopkMaxBlocks)
        return hipErrorInvalidValue;  // the kernel indexes at most kTopkMaxBlocks lists
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
// groups of 64 correspondences a wave holds at once: 4, or 1 below this many
// correspondences (fewer waves would then share the work)
constexpr int64_t kRescoreTileMinN = 65536;

template <int kRescoreTile>
__global__ __launch_bounds__(kRescoreThreads) void k_rescore(const float* __restrict__ x,
                                                             const float* __restrict__ y,
                                                             int64_t n, float T2, Candidates c)
{
    __shared__ uint32_t partial[kRescoreThreads / kWave][kWave];
    __shared__ float4 s_q[kWave];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int ncand = __builtin_amdgcn_readfirstlane(c.result->n_cand);
    // the candidates' rotations, read once per block (a scalar load per
    // candidate waited on its latency in every iteration)
    if (threadIdx.x < ncand)
        s_q[threadIdx.x] = c.q[threadIdx.x];
    __syncthreads();
    uint32_t acc = 0;
    // each wave holds kRescoreTile groups of 64 correspondences in registers
    // and tests every candidate against all of them: the count of candidate
    // k goes to lane k of acc once per tile, not once per group
    const int64_t stride = (int64_t)gridDim.x * kRescoreThreads * kRescoreTile;
    for (int64_t base = ((int64_t)blockIdx.x * (kRescoreThreads / kWave) + wave) * kWave * kRescoreTile;
         base < n; base += stride) {
        float D[kRescoreTile][3], P[kRescoreTile][3];
        uint64_t okm[kRescoreTile];
#pragma unroll
        for (int r = 0; r < kRescoreTile; ++r) {
            const int64_t i = base + r * kWave + lane;
            float a[3] = {1.0f, 0.0f, 0.0f};
            float b[3] = {1.0f, 0.0f, 0.0f};
            bool ok = false;
            if (i < n) {
                const bool oka = load_unit(x, n, i, a);
                const bool okb = load_unit(y, n, i, b);
                ok = oka && okb;
            }
            okm[r] = __builtin_amdgcn_ballot_w64(ok);
#pragma unroll
            for (int m = 0; m < 3; ++m) {
                D[r][m] = a[m] - b[m];
                P[r][m] = a[m] + b[m];
            }
        }
        for (int k = 0; k < ncand; ++k) {
            const float4 q4 = s_q[k];
            const Quat q{q4.x, q4.y, q4.z, q4.w};
            // unusable lanes hold finite placeholders: tested too, then
            // dropped by their group's mask (no branch per candidate)
            uint32_t cnt = 0;
#pragma unroll
            for (int r = 0; r < kRescoreTile; ++r)
                cnt += (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(residual2(D[r], P[r], q) <= T2) &
                                          okm[r]);
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
    const int tile = n >= kRescoreTileMinN ? 4 : 1;
    const int64_t per_block = (int64_t)kRescoreThreads * tile;
    const int blocks = (int)std::min<int64_t>((n + per_block - 1) / per_block, 2048);
    if (tile == 4)
        hipLaunchKernelGGL(k_rescore<4>, dim3(blocks), dim3(kRescoreThreads), 0, s, x, y, n, T2, c);
    else
        hipLaunchKernelGGL(k_rescore<1>, dim3(blocks), dim3(kRescoreThreads), 0, s, x, y, n, T2, c);
    return hipGetLastError();
}

// --------------------------------------------------------------------- mask
//
// Winner = most inliers, ties to the earlier candidate (more votes, then lower
// cell index).  Every block finds it from the <= 64 counts; block 0 writes the
// result record.

__global__ __launch_bounds__(256) void k_mask(const float* __restrict__ x,
                                              const float* __restrict__ y, int64_t n, float T2,
                                              Candidates c, uint8_t* __restrict__ mask,
                                              Result* __restrict__ host_result)
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
        if (host_result) {
            // the same record straight into the caller's pinned host memory
            // (visible to the host once the kernel has completed)
            Result h;
            h.q[0] = q.w;
            h.q[1] = q.x;
            h.q[2] = q.y;
            h.q[3] = q.z;
            h.count = r->count;
            h.winner = win;
            h.n_cand = r->n_cand;
            *host_result = h;
        }
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
                       uint8_t* mask, hipStream_t s, Result* host_result)
{
    const int blocks = (int)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 2048));
    hipLaunchKernelGGL(k_mask, dim3(blocks), dim3(256), 0, s, x, y, n, T2, c, mask, host_result);
    return hipGetLastError();
}

}  // namespace rv
