// Batched solves: many independent instances (same G, J, K, eps), each a
// contiguous column range of one SoA input.  A plan kernel sizes everything
// on the device from the instances' offsets (so a batch needs no host round
// trip and can be captured in a HIP graph): each instance's brick-size class
// (from its size bucket), its work units, its queues' capacities and pool
// offsets.  The binned vote and the brick accumulation are the one-solve
// kernels run over (instance, unit) and (instance, brick) of each class;
// these kernels finish each instance: merge its bricks' sorted lists, rescore
// its candidates on its own correspondences, pick its winner and write its
// mask and result record.
#include <cmath>

#include "rv_device.h"
#include "rv_internal.h"
#include "rv_topk.h"

namespace rv {

// ------------------------------------------------------------------ plan

constexpr int kPlanThreads = 1024;
constexpr int kPlanWaves = kPlanThreads / 64;
// scanned per instance: class-0 instances, class-0 units, class-1 units,
// units (32-bit), and run-pool slots (64-bit)
constexpr int kScan32 = 4;

// Inclusive scans across the workgroup (per wave with shuffles, then over the
// wave totals): v and r become this thread's exclusive prefixes plus the
// carries, and the block's totals are added to the carries.
__device__ __forceinline__ void block_scan(uint32_t (&v)[kScan32], uint64_t& r,
                                           uint32_t (&carry)[kScan32], uint64_t& rcarry,
                                           uint32_t (*s_w)[kScan32], uint64_t* s_r, int wave,
                                           int lane)
{
    uint32_t incl[kScan32];
#pragma unroll
    for (int k = 0; k < kScan32; ++k) {
        incl[k] = v[k];
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const uint32_t w = __shfl_up(incl[k], off);
            incl[k] += lane >= off ? w : 0u;
        }
    }
    uint64_t rincl = r;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t lo = __shfl_up((uint32_t)rincl, off);
        const uint32_t hi = __shfl_up((uint32_t)(rincl >> 32), off);
        rincl += lane >= off ? (((uint64_t)hi << 32) | lo) : 0ull;
    }
    if (lane == 63) {
#pragma unroll
        for (int k = 0; k < kScan32; ++k)
            s_w[wave][k] = incl[k];
        s_r[wave] = rincl;
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScan32; ++k) {
        uint32_t pre = 0, tot = 0;
        for (int w = 0; w < kPlanWaves; ++w) {
            const uint32_t x = s_w[w][k];
            pre += w < wave ? x : 0u;
            tot += x;
        }
        v[k] = carry[k] + pre + incl[k] - v[k];  // exclusive
        carry[k] += tot;
    }
    uint64_t rpre = 0, rtot = 0;
    for (int w = 0; w < kPlanWaves; ++w) {
        const uint64_t x = s_r[w];
        rpre += w < wave ? x : 0ull;
        rtot += x;
    }
    r = rcarry + rpre + rincl - r;
    rcarry += rtot;
    __syncthreads();
}

// The brick-size class (0: 16^3, 1: 32^3) of an instance of n
// correspondences, from its size bucket.  Plain selects: indexing the
// by-value kernel argument would copy it to scratch memory.
__device__ __forceinline__ int class_of(const BatchPlanArgs& p, int64_t n)
{
    const int8_t e = n < kBucketBound[0]   ? p.bucket_edge[0]
                     : n < kBucketBound[1] ? p.bucket_edge[1]
                     : n < kBucketBound[2] ? p.bucket_edge[2]
                                           : p.bucket_edge[3];
    return e == 4 ? 0 : 1;
}

// Queue capacity of every brick of an instance of n correspondences: its
// planned share of the runs plus slack, in multiples of 64 (queues start on
// 256-byte boundaries), optionally scaled down to fit the pool.
__device__ __forceinline__ uint64_t inst_cap(const BatchPlanArgs& p, int cls, int64_t n, double f)
{
    if (n <= 0)
        return 0;
    const double share = cls ? p.share[1] : p.share[0];
    const uint32_t slack = cls ? p.slack[1] : p.slack[0];
    uint64_t c = ((uint64_t)ceil(share * (double)n) + slack + 63u) & ~63ull;
    if (f < 1.0)
        c = (uint64_t)((double)c * f) & ~63ull;
    return c;
}

// One workgroup: checks the offsets, then two passes over the instances in
// chunks of 1024 (pass 1: total runs, for the pool; pass 2: the scans and the
// per-instance plan).
__global__ __launch_bounds__(kPlanThreads) void k_batch_plan(BatchPlanArgs p)
{
    __shared__ uint32_t s_w[kPlanWaves][kScan32];
    __shared__ uint64_t s_r[kPlanWaves];
    __shared__ int s_bad;
    __shared__ uint64_t s_runs;
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int B = p.B;
    if (t == 0) {
        s_bad = (p.offsets[0] != 0 || p.offsets[B] > p.n_cols) ? 1 : 0;
        s_runs = 0;
    }
    __syncthreads();
    uint64_t runs = 0;
    for (int b = t; b < B; b += kPlanThreads) {
        const int64_t n = p.offsets[b + 1] - p.offsets[b];
        if (n < 0 || n * (int64_t)p.J > (int64_t)INT32_MAX)
            atomicOr(&s_bad, 1);
        const int cls = class_of(p, n);
        runs += inst_cap(p, cls, n, 1.0) * (uint64_t)(cls ? p.nb[1] : p.nb[0]);
    }
    atomicAdd((unsigned long long*)&s_runs, (unsigned long long)runs);
    __syncthreads();
    if (s_bad) {
        for (int b = t; b < B; b += kPlanThreads) {
            Result* r = p.results + b;
            r->q[0] = 1.0f;
            r->q[1] = r->q[2] = r->q[3] = 0.0f;
            r->count = 0;
            r->winner = -2;
            r->n_cand = 0;
        }
        if (t < 6)
            p.counts[t] = 0;
        return;
    }
    const double f = s_runs > p.pool_runs ? (double)p.pool_runs / (double)s_runs : 1.0;
    uint32_t carry[kScan32] = {0, 0, 0, 0};
    uint64_t rcarry = 0;
    for (int base = 0; base < B; base += kPlanThreads) {
        const int b = base + t;
        int64_t n = 0;
        int cls = 0;
        uint64_t cap = 0;
        if (b < B) {
            n = p.offsets[b + 1] - p.offsets[b];
            cls = class_of(p, n);
            cap = inst_cap(p, cls, n, f);
        }
        const uint32_t units = (uint32_t)((n + kUnitSize - 1) / kUnitSize);
        uint32_t v[kScan32] = {(b < B && cls == 0) ? 1u : 0u, cls == 0 ? units : 0u,
                               cls == 1 ? units : 0u, units};
        uint64_t r = b < B ? cap * (uint64_t)(cls ? p.nb[1] : p.nb[0]) : 0ull;
        block_scan(v, r, carry, rcarry, s_w, s_r, wave, lane);
        if (b < B) {
            InstPlan ip;
            ip.cls = cls;
            ip.ci = cls == 0 ? (int32_t)v[0] : (int32_t)((uint32_t)b - v[0]);
            ip.unit0 = (int32_t)(cls == 0 ? v[1] : v[2]);
            ip.gunit0 = (int32_t)v[3];
            ip.nunits = (int32_t)units;
            ip.cap = (uint32_t)cap;
            ip.rbase = (uint32_t)r;
            ip.reserved = 0;
            p.inst[b] = ip;
        }
    }
    if (t == 0) {
        p.counts[0] = (int32_t)carry[1];
        p.counts[1] = (int32_t)carry[0];
        p.counts[2] = (int32_t)carry[2];
        p.counts[3] = B - (int32_t)carry[0];
        p.counts[4] = (int32_t)carry[3];
        p.counts[5] = 1;
    }
}

// One wave per instance: its class-local index, its queues (capacity, pool
// offset, cleared fill count and overflow flag) and its work units.
__global__ __launch_bounds__(256) void k_batch_expand(BatchPlanArgs p)
{
    const int b = blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (b >= p.B || p.counts[5] == 0)
        return;
    const InstPlan ip = p.inst[b];
    // plain selects (see class_of)
    const bool c1 = ip.cls != 0;
    const int nb = c1 ? p.nb[1] : p.nb[0];
    uint32_t* cap = c1 ? p.cap[1] : p.cap[0];
    uint32_t* qbase = c1 ? p.qbase[1] : p.qbase[0];
    uint32_t* fill = c1 ? p.fill[1] : p.fill[0];
    uint32_t* flags = c1 ? p.flags[1] : p.flags[0];
    Unit* units = c1 ? p.units[1] : p.units[0];
    if (lane == 0)
        (c1 ? p.inst_of[1] : p.inst_of[0])[ip.ci] = b;
    for (int k = lane; k < nb; k += 64) {
        const int64_t q = (int64_t)ip.ci * nb + k;
        cap[q] = ip.cap;
        qbase[q] = ip.rbase + (uint32_t)k * ip.cap;
        fill[q] = 0u;
        flags[q] = 0u;
    }
    const int64_t first = p.offsets[b];
    const int64_t n = p.offsets[b + 1] - first;
    for (int j = lane; j < ip.nunits; j += 64) {
        const int64_t f = first + (int64_t)j * kUnitSize;
        const int32_t cnt = (int32_t)min<int64_t>(kUnitSize, n - (int64_t)j * kUnitSize);
        units[ip.unit0 + j] = Unit{ip.ci, cnt, f};
        p.units_all[ip.gunit0 + j] = Unit{b, cnt, f};
    }
}

hipError_t launch_batch_plan(const BatchPlanArgs& p, hipStream_t s)
{
    if (p.B <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_batch_plan, dim3(1), dim3(kPlanThreads), 0, s, p);
    if (hipError_t e = hipGetLastError(); e != hipSuccess)
        return e;
    hipLaunchKernelGGL(k_batch_expand, dim3((unsigned)((p.B + 3) / 4)), dim3(256), 0, s, p);
    return hipGetLastError();
}

// --------------------------------------------------------------- finish

// One wave per instance of a class: merge the nb brick lists, decode the K
// best cells, clear the inlier counters and write a default result record
// (identity, count 0), which the mask kernel overwrites for instances with
// correspondences.
__global__ __launch_bounds__(64) void k_topk_final_batch(const uint64_t* __restrict__ partial, int nb,
                                                         int K, int G, const int32_t* counts,
                                                         const int32_t* inst_of, Candidates c)
{
    const int ci = blockIdx.x;
    if (counts && ci >= counts[1])
        return;
    const int inst = inst_of ? inst_of[ci] : ci;
    const int lane = threadIdx.x;
    uint64_t list = 0;
    for (int b = 0; b < nb; ++b)
        list = wave_insert_sorted(list, partial[((int64_t)ci * nb + b) * 64 + lane], lane);
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
                                                                const int32_t* nunits,
                                                                Candidates c)
{
    __shared__ uint32_t part[kUnitWaves][64];
    __shared__ float4 s_q[kMaxTopK];
    if (nunits && (int)blockIdx.x >= *nunits)
        return;
    const Unit un = units[blockIdx.x];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int ncand = __builtin_amdgcn_readfirstlane(c.result[un.inst].n_cand);
    // the instance's candidates, read once per block (not a scalar load
    // waited on in every iteration)
    if ((int)threadIdx.x < ncand)
        s_q[threadIdx.x] = c.q[(int64_t)un.inst * kMaxTopK + threadIdx.x];
    __syncthreads();
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
    const uint64_t okm = __builtin_amdgcn_ballot_w64(ok);
    for (int k = 0; k < ncand; ++k) {
        const float4 q4 = s_q[k];
        const Quat q{q4.x, q4.y, q4.z, q4.w};
        // unusable lanes hold finite placeholders: tested too, then dropped by
        // the mask (no branch per candidate); the ballot runs on every lane
        const uint32_t cnt =
            (uint32_t)__popcll(__builtin_amdgcn_ballot_w64(residual2(D, P, q) <= T2) & okm);
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
                                                             const int32_t* nunits,
                                                             const int64_t* __restrict__ offsets,
                                                             Candidates c, uint8_t* __restrict__ mask)
{
    __shared__ int s_win;
    if (nunits && (int)blockIdx.x >= *nunits)
        return;
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

hipError_t launch_batch_topk(const uint64_t* partial, int B, int nb, int K, int G,
                             const int32_t* counts, const int32_t* inst_of, const Candidates& c,
                             hipStream_t s)
{
    if (B <= 0)
        return hipSuccess;
    hipLaunchKernelGGL(k_topk_final_batch, dim3(B), dim3(64), 0, s, partial, nb, K, G, counts,
                       inst_of, c);
    return hipGetLastError();
}

hipError_t launch_batch_rescore_mask(const float* x, const float* y, int64_t n, float T2,
                                     const Unit* units, int max_units, const int32_t* nunits,
                                     const int64_t* offsets, const Candidates& c, uint8_t* mask,
                                     hipStream_t s, hipEvent_t after_rescore)
{
    if (max_units > 0) {
        hipLaunchKernelGGL(k_rescore_batch, dim3(max_units), dim3(kUnitThreads), 0, s, x, y, n, T2,
                           units, nunits, c);
        if (hipError_t e = hipGetLastError(); e != hipSuccess)
            return e;
    }
    if (after_rescore)
        (void)hipEventRecord(after_rescore, s);
    if (max_units > 0) {
        hipLaunchKernelGGL(k_mask_batch, dim3(max_units), dim3(kUnitThreads), 0, s, x, y, n, T2,
                           units, nunits, offsets, c, mask);
        return hipGetLastError();
    }
    return hipSuccess;
}

}  // namespace rv
