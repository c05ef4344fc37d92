// Batched solves: many independent instances (same G, J, K, eps), each a
// contiguous column range of one SoA input.  The binned vote and the brick
// accumulation are the one-solve kernels run over (instance, unit) and
// (instance, brick); these kernels finish each instance: merge its bricks'
// sorted lists, rescore its candidates on its own correspondences, pick its
// winner and write its mask and result record.
#include "rv_device.h"
#include "rv_internal.h"
#include "rv_topk.h"

namespace rv {

// One wave per instance: merge the nb brick lists, decode the K best cells,
// clear the inlier counters and write a default result record (identity,
// count 0), which the mask kernel overwrites for instances with
// correspondences.
__global__ __launch_bounds__(64) void k_topk_final_batch(const uint64_t* __restrict__ partial, int nb,
                                                         int K, int G, Candidates c)
{
    const int inst = blockIdx.x;
    const int lane = threadIdx.x;
    uint64_t list = 0;
    for (int b = 0; b < nb; ++b)
        list = wave_insert_sorted(list, partial[((int64_t)inst * nb + b) * 64 + lane], lane);
    const bool valid = lane < K && list != 0;
    const int ncand = __popcll(__ballot(valid));
    const int64_t o = (int64_t)inst * kMaxTopK + lane;
    if (valid) {
        const int32_t idx = (int32_t)(0xFFFFFFFFu - (uint32_t)list);
        const Quat q = decode_cell(idx, G);
        c.q[o] = make_float4(q.w, q.x, q.y, q.z);
        c.votes[o] = (int32_t)(list >> 32);
        c.idx[o] = idx;
    }
    c.inliers[o] = 0u;
    if (lane == 0) {
        Result* r = c.result + inst;
        r->q[0] = 1.0f;
        r->q[1] = r->q[2] = r->q[3] = 0.0f;
        r->count = 0;
        r->winner = -1;
        r->n_cand = ncand;
    }
}

constexpr int kUnitThreads = 512;  // the binned vote's unit size
constexpr int kUnitWaves = kUnitThreads / 64;

// One block per unit: the instance's candidates against the unit's
// correspondences (ballot + popcount per candidate, lane k of each wave
// accumulates candidate k), one atomic per candidate per block.
__global__ __launch_bounds__(kUnitThreads) void k_rescore_batch(const float* __restrict__ x,
                                                                const float* __restrict__ y,
                                                                int64_t n, float T2,
                                                                const Unit* __restrict__ units,
                                                                Candidates c)
{
    __shared__ uint32_t part[kUnitWaves][64];
    const Unit un = units[blockIdx.x];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int ncand = __builtin_amdgcn_readfirstlane(c.result[un.inst].n_cand);
    const float4* cq = c.q + (int64_t)un.inst * kMaxTopK;
    const int64_t i = un.first + threadIdx.x;
    float a[3] = {1.0f, 0.0f, 0.0f};
    float b[3] = {1.0f, 0.0f, 0.0f};
    bool ok = false;
    if ((int)threadIdx.x < un.count) {
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
    uint32_t acc = 0;
    for (int k = 0; k < ncand; ++k) {
        const float4 q4 = cq[k];
        const Quat q{q4.x, q4.y, q4.z, q4.w};
        const bool in = ok && (residual2(D, P, q) <= T2);
        // the ballot runs on every lane (inside the select it would see lane k only)
        const uint32_t cnt = (uint32_t)__popcll(__ballot(in));
        acc += (lane == k) ? cnt : 0u;
    }
    part[wave][lane] = acc;
    __syncthreads();
    if (wave == 0 && lane < ncand) {
        uint32_t s = 0;
#pragma unroll
        for (int w = 0; w < kUnitWaves; ++w)
            s += part[w][lane];
        if (s)
            __hip_atomic_fetch_add(c.inliers + (int64_t)un.inst * kMaxTopK + lane, s, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_AGENT);
    }
}

// One block per unit: the instance's winner (most inliers, earlier candidate
// on ties), the unit's mask entries; the instance's first unit writes the
// result record.
__global__ __launch_bounds__(kUnitThreads) void k_mask_batch(const float* __restrict__ x,
                                                             const float* __restrict__ y, int64_t n,
                                                             float T2, const Unit* __restrict__ units,
                                                             const int64_t* __restrict__ offsets,
                                                             Candidates c, uint8_t* __restrict__ mask)
{
    __shared__ int s_win;
    const Unit un = units[blockIdx.x];
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 64) {
        const int ncand = c.result[un.inst].n_cand;
        uint64_t key = 0;
        if (lane < ncand)
            key = (((uint64_t)c.inliers[(int64_t)un.inst * kMaxTopK + lane] + 1ull) << 6) |
                  (uint64_t)(63 - lane);
#pragma unroll
        for (int m = 32; m > 0; m >>= 1)
            key = umax64(key, shfl_xor_u64(key, m));
        if (lane == 0)
            s_win = key ? (63 - (int)(key & 63)) : -1;
    }
    __syncthreads();
    const int win = s_win;
    Quat q{1.0f, 0.0f, 0.0f, 0.0f};
    if (win >= 0) {
        const float4 q4 = c.q[(int64_t)un.inst * kMaxTopK + win];
        q = Quat{q4.x, q4.y, q4.z, q4.w};
    }
    if (threadIdx.x == 0 && un.first == offsets[un.inst]) {
        Result* r = c.result + un.inst;
        r->q[0] = q.w;
        r->q[1] = q.x;
        r->q[2] = q.y;
        r->q[3] = q.z;
        r->count = win >= 0 ? (int64_t)c.inliers[(int64_t)un.inst * kMaxTopK + win] : 0;
        r->winner = win;
    }
    if ((int)threadIdx.x < un.count) {
        const int64_t i = un.first + threadIdx.x;
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

// Gathers separate requests' SoA columns into one batch array (and scatters
// the batch mask back): one 512-thread block per unit of one item.
__global__ __launch_bounds__(kUnitThreads) void k_gather(const GatherItem* __restrict__ items,
                                                         const Unit* __restrict__ units,
                                                         float* __restrict__ dx,
                                                         float* __restrict__ dy, int64_t total)
{
    const Unit un = units[blockIdx.x];
    const GatherItem it = items[un.inst];
    if ((int)threadIdx.x >= un.count)
        return;
    const int64_t j = un.first + threadIdx.x;
    const int64_t o = it.offset + j;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        dx[c * total + o] = it.x[c * it.n + j];
        dy[c * total + o] = it.y[c * it.n + j];
    }
}

__global__ __launch_bounds__(kUnitThreads) void k_scatter_mask(const GatherItem* __restrict__ items,
                                                               const Unit* __restrict__ units,
                                                               const uint8_t* __restrict__ dmask)
{
    const Unit un = units[blockIdx.x];
    const GatherItem it = items[un.inst];
    if ((int)threadIdx.x >= un.count)
        return;
    const int64_t j = un.first + threadIdx.x;
    it.mask[j] = dmask[it.offset + j];
}

hipError_t launch_gather(const GatherItem* items, const Unit* units, int nunits, float* dx,
                         float* dy, int64_t total, hipStream_t s)
{
    if (nunits <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3(nunits), dim3(kUnitThreads), 0, s, items, units, dx, dy, total);
    return hipGetLastError();
}

hipError_t launch_scatter_masks(const GatherItem* items, const Unit* units, int nunits,
                                const uint8_t* dmask, hipStream_t s)
{
    if (nunits <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_scatter_mask, dim3(nunits), dim3(kUnitThreads), 0, s, items, units, dmask);
    return hipGetLastError();
}

hipError_t launch_batch_finish(const float* x, const float* y, int64_t n, float T2, int B, int nb,
                               int K, int G, const uint64_t* partial, const Unit* units, int nunits,
                               const int64_t* offsets, const Candidates& c, uint8_t* mask,
                               hipStream_t s, hipEvent_t after_topk, hipEvent_t after_rescore)
{
    hipLaunchKernelGGL(k_topk_final_batch, dim3(B), dim3(64), 0, s, partial, nb, K, G, c);
    if (hipError_t e = hipGetLastError(); e != hipSuccess)
        return e;
    if (after_topk)
        (void)hipEventRecord(after_topk, s);
    if (nunits > 0) {
        hipLaunchKernelGGL(k_rescore_batch, dim3(nunits), dim3(kUnitThreads), 0, s, x, y, n, T2,
                           units, c);
        if (hipError_t e = hipGetLastError(); e != hipSuccess)
            return e;
    }
    if (after_rescore)
        (void)hipEventRecord(after_rescore, s);
    if (nunits > 0) {
        hipLaunchKernelGGL(k_mask_batch, dim3(nunits), dim3(kUnitThreads), 0, s, x, y, n, T2, units,
                           offsets, c, mask);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace rv
