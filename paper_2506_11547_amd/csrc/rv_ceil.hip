// Micro-benchmarks of the ceilings that can bound the solve's kernels on the
// GPU they run on: 32-bit VALU issue (independent FMA chains), LDS atomic adds
// (random and bank-distinct addresses), relaxed device-scope atomic adds on a
// grid of a given size (random cells), a streaming device copy and a
// streaming read.  The
// benchmark divides the vote's achieved rate by these as well as by the
// published peaks.  Measurement hooks only: not used by a solve.
//
// Every entry point allocates its own buffers, runs one untimed and one timed
// launch on the null stream (HIP events around the timed one), checks what it
// can of the result, frees everything and returns 0, or a HIP error code, or
// -1 for an invalid argument or a failed result check.
#include <hip/hip_runtime.h>

#include <cstdint>
#include <vector>

#pragma GCC visibility push(default)
#include "rotvote_probe.h"
#pragma GCC visibility pop

#define RVP_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr int kChains = 8;       // independent FMA chains per lane
constexpr int kLdsCells = 32768; // 128 KiB of LDS, the accumulation's brick
constexpr int kLdsThreads = 1024;

__global__ __launch_bounds__(256) void k_ceil_valu(float* out, int iters, float a, float b)
{
    float x[kChains];
#pragma unroll
    for (int u = 0; u < kChains; ++u)
        x[u] = (float)(threadIdx.x + u);
#pragma unroll 4
    for (int i = 0; i < iters; ++i) {
#pragma unroll
        for (int u = 0; u < kChains; ++u)
            x[u] = __builtin_fmaf(x[u], a, b);
    }
    float s = 0.0f;
#pragma unroll
    for (int u = 0; u < kChains; ++u)
        s += x[u];
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = s;
}

// kRandom: each lane draws its cells from its own linear congruential
// sequence (15 high bits); otherwise the block's 1024 lanes hit 1024
// consecutive cells, moving by 1024 every iteration (no bank conflicts).
template <bool kRandom>
__global__ __launch_bounds__(kLdsThreads) void k_ceil_lds(uint32_t* out, int iters, uint32_t seed)
{
    __shared__ uint32_t s[kLdsCells];
    for (int k = threadIdx.x; k < kLdsCells; k += kLdsThreads)
        s[k] = 0u;
    __syncthreads();
    uint32_t h = seed ^ ((uint32_t)(blockIdx.x * kLdsThreads + threadIdx.x) * 0x9E3779B9u);
    for (int i = 0; i < iters; ++i) {
        uint32_t c;
        if (kRandom) {
            h = h * 1664525u + 1013904223u;
            c = h >> 17;
        } else {
            c = (threadIdx.x + (uint32_t)i * kLdsThreads) & (kLdsCells - 1);
        }
        atomicAdd(&s[c], 1u);
    }
    __syncthreads();
    uint32_t t = 0;
    for (int k = threadIdx.x; k < kLdsCells; k += kLdsThreads)
        t += s[k];
    out[(int64_t)blockIdx.x * kLdsThreads + threadIdx.x] = t;
}

// kContiguous: the 64 lanes of a wave add to 64 consecutive cells at a random
// 64-cell-aligned base (one draw per wave and iteration); otherwise every lane
// draws its own random cell.
template <bool kContiguous>
__global__ __launch_bounds__(256) void k_ceil_gatomic(int32_t* grid, uint32_t mask, int iters,
                                                      uint32_t seed)
{
    const uint32_t id = kContiguous ? (blockIdx.x * 256 + threadIdx.x) >> 6
                                    : blockIdx.x * 256 + threadIdx.x;
    uint32_t h = seed ^ (id * 0x9E3779B9u);
    for (int i = 0; i < iters; ++i) {
        h = h * 1664525u + 1013904223u;
        const uint32_t c = kContiguous ? (((h >> 4) & mask & ~63u) | (threadIdx.x & 63u))
                                       : ((h >> 4) & mask);
        __hip_atomic_fetch_add(grid + c, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

__global__ __launch_bounds__(256) void k_ceil_copy(const uint4* __restrict__ src,
                                                   uint4* __restrict__ dst, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

// Streaming read: every thread sums four independent 16-byte loads per
// step (so several are in flight), writing one word per thread at the end.
__global__ __launch_bounds__(256) void k_ceil_read(const uint4* __restrict__ src,
                                                   uint32_t* __restrict__ out, int64_t n)
{
    const int64_t stride = (int64_t)gridDim.x * 256;
    uint32_t acc[4] = {0u, 0u, 0u, 0u};
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    for (; i + 3 * stride < n; i += 4 * stride) {
        uint4 v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            v[u] = src[i + u * stride];
#pragma unroll
        for (int u = 0; u < 4; ++u)
            acc[u] += v[u].x ^ v[u].y ^ v[u].z ^ v[u].w;
    }
    for (; i < n; i += stride) {
        const uint4 v = src[i];
        acc[0] += v.x ^ v.y ^ v.z ^ v.w;
    }
    out[(int64_t)blockIdx.x * 256 + threadIdx.x] = acc[0] + acc[1] + acc[2] + acc[3];
}

// Runs launch() twice and returns the second run's milliseconds in *ms.
template <class F>
int timed(F&& launch, float* ms)
{
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess)
        return -1;
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return -1;
    }
    launch();
    hipError_t e = hipGetLastError();
    if (e == hipSuccess)
        e = hipEventRecord(e0, 0);
    if (e == hipSuccess) {
        launch();
        e = hipGetLastError();
    }
    if (e == hipSuccess)
        e = hipEventRecord(e1, 0);
    if (e == hipSuccess)
        e = hipEventSynchronize(e1);
    if (e == hipSuccess)
        e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return e == hipSuccess ? 0 : (int)e;
}

}  // namespace

// 32-bit FMA lane-operations per second over `blocks` workgroups of 256
// threads, each lane running `iters` x 8 independent FMAs.
RVP_API int rvp_ceil_valu(int blocks, int iters, double* ops_per_s)
{
    if (blocks <= 0 || iters <= 0 || !ops_per_s)
        return -1;
    float* out = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 256 * sizeof(float)) != hipSuccess)
        return -1;
    float ms = 0.0f;
    const int rc = timed([&] {
        hipLaunchKernelGGL(k_ceil_valu, dim3(blocks), dim3(256), 0, 0, out, iters, 0.999999f,
                           1e-7f);
    }, &ms);
    (void)hipFree(out);
    if (rc)
        return rc;
    *ops_per_s = (double)blocks * 256 * iters * kChains / (ms * 1e-3);
    return 0;
}

// LDS atomic adds per second: `blocks` workgroups of 1024 threads, each lane
// adding 1 `iters` times into a 128 KiB LDS array; random != 0 draws random
// cells.  The adds of every workgroup are summed back and checked.
RVP_API int rvp_ceil_lds_atomic(int blocks, int iters, int random, double* atomics_per_s)
{
    if (blocks <= 0 || iters <= 0 || !atomics_per_s)
        return -1;
    const size_t n = (size_t)blocks * kLdsThreads;
    uint32_t* out = nullptr;
    if (hipMalloc(&out, n * sizeof(uint32_t)) != hipSuccess)
        return -1;
    float ms = 0.0f;
    int rc = timed([&] {
        if (random)
            hipLaunchKernelGGL(k_ceil_lds<true>, dim3(blocks), dim3(kLdsThreads), 0, 0, out, iters,
                               12345u);
        else
            hipLaunchKernelGGL(k_ceil_lds<false>, dim3(blocks), dim3(kLdsThreads), 0, 0, out,
                               iters, 12345u);
    }, &ms);
    std::vector<uint32_t> h(n);
    if (!rc && hipMemcpy(h.data(), out, n * sizeof(uint32_t), hipMemcpyDeviceToHost) != hipSuccess)
        rc = -1;
    (void)hipFree(out);
    if (rc)
        return rc;
    for (int b = 0; b < blocks; ++b) {
        uint64_t s = 0;
        for (int t = 0; t < kLdsThreads; ++t)
            s += h[(size_t)b * kLdsThreads + t];
        if (s != (uint64_t)kLdsThreads * (uint64_t)iters)
            return -1;
    }
    *atomics_per_s = (double)n * iters / (ms * 1e-3);
    return 0;
}

// Relaxed device-scope atomic adds per second into an int32 grid of `cells`
// entries (a power of two, from 64 to 2^26): `blocks` workgroups of 256
// threads, `iters` adds per lane, at random cells or (contiguous != 0) a wave
// at a time into 64 consecutive cells.  The grid's total is checked.
RVP_API int rvp_ceil_global_atomic(int64_t cells, int blocks, int iters, int contiguous,
                                   double* atomics_per_s)
{
    if (cells < 64 || cells > (int64_t(1) << 26) || (cells & (cells - 1)) || blocks <= 0 ||
        iters <= 0 || !atomics_per_s)
        return -1;
    int32_t* grid = nullptr;
    if (hipMalloc(&grid, (size_t)cells * sizeof(int32_t)) != hipSuccess)
        return -1;
    int rc = hipMemset(grid, 0, (size_t)cells * sizeof(int32_t)) == hipSuccess ? 0 : -1;
    float ms = 0.0f;
    if (!rc)
        rc = timed([&] {
            if (contiguous)
                hipLaunchKernelGGL(k_ceil_gatomic<true>, dim3(blocks), dim3(256), 0, 0, grid,
                                   (uint32_t)(cells - 1), iters, 777u);
            else
                hipLaunchKernelGGL(k_ceil_gatomic<false>, dim3(blocks), dim3(256), 0, 0, grid,
                                   (uint32_t)(cells - 1), iters, 777u);
        }, &ms);
    std::vector<int32_t> h(rc ? 0 : (size_t)cells);
    if (!rc && hipMemcpy(h.data(), grid, (size_t)cells * sizeof(int32_t),
                         hipMemcpyDeviceToHost) != hipSuccess)
        rc = -1;
    (void)hipFree(grid);
    if (rc)
        return rc;
    int64_t total = 0;
    for (int32_t v : h)
        total += v;
    const int64_t adds = (int64_t)blocks * 256 * iters;
    if (total != 2 * adds)  // two launches
        return -1;
    *atomics_per_s = (double)adds / (ms * 1e-3);
    return 0;
}

// Streaming read of `bytes` (a multiple of 16): bytes read per second.
RVP_API int rvp_ceil_read(int64_t bytes, double* bytes_per_s)
{
    if (bytes <= 0 || bytes % 16 || !bytes_per_s)
        return -1;
    constexpr int kBlocks = 256 * 32;
    uint4* src = nullptr;
    uint32_t* out = nullptr;
    if (hipMalloc(&src, (size_t)bytes) != hipSuccess)
        return -1;
    if (hipMalloc(&out, (size_t)kBlocks * 256 * sizeof(uint32_t)) != hipSuccess) {
        (void)hipFree(src);
        return -1;
    }
    // every word 0x01010101: each 16-byte load xors to 0, so every sum is 0
    int rc = hipMemset(src, 1, (size_t)bytes) == hipSuccess ? 0 : -1;
    const int64_t n = bytes / 16;
    float ms = 0.0f;
    if (!rc)
        rc = timed([&] {
            hipLaunchKernelGGL(k_ceil_read, dim3(kBlocks), dim3(256), 0, 0, src, out, n);
        }, &ms);
    uint32_t first = 1u;
    if (!rc && hipMemcpy(&first, out, sizeof(first), hipMemcpyDeviceToHost) != hipSuccess)
        rc = -1;
    (void)hipFree(src);
    (void)hipFree(out);
    if (rc)
        return rc;
    if (first != 0u)
        return -1;
    *bytes_per_s = (double)bytes / (ms * 1e-3);
    return 0;
}

// Device copy of `bytes` (a multiple of 16) from one buffer to another:
// bytes read + bytes written per second.
RVP_API int rvp_ceil_copy(int64_t bytes, double* bytes_per_s)
{
    if (bytes <= 0 || bytes % 16 || !bytes_per_s)
        return -1;
    uint4 *src = nullptr, *dst = nullptr;
    if (hipMalloc(&src, (size_t)bytes) != hipSuccess)
        return -1;
    if (hipMalloc(&dst, (size_t)bytes) != hipSuccess) {
        (void)hipFree(src);
        return -1;
    }
    int rc = hipMemset(src, 1, (size_t)bytes) == hipSuccess ? 0 : -1;
    const int64_t n = bytes / 16;
    float ms = 0.0f;
    if (!rc)
        rc = timed([&] {
            hipLaunchKernelGGL(k_ceil_copy, dim3(256 * 32), dim3(256), 0, 0, src, dst, n);
        }, &ms);
    uint4 last{};
    if (!rc && hipMemcpy(&last, dst + (n - 1), 16, hipMemcpyDeviceToHost) != hipSuccess)
        rc = -1;
    (void)hipFree(src);
    (void)hipFree(dst);
    if (rc)
        return rc;
    if (last.x != 0x01010101u || last.w != 0x01010101u)
        return -1;
    *bytes_per_s = 2.0 * (double)bytes / (ms * 1e-3);
    return 0;
}
