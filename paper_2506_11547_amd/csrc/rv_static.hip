// rot_vote_solve_noalloc: one solve without a handle and without any
// allocation, for callers that cannot allocate device memory (HIP graph
// capture, serving loops, harnesses that forbid hipMalloc).
//
// Its scratch (the vote grid, the sample table, the top-K lists and the
// candidates) lives in one fixed device array of this file, which every GPU
// the library runs on holds from the code object's load until the process
// ends.  The kernels are the handle path's global-atomic vote, top-K,
// rescoring and mask; only the grid clear and the sample table (computed on
// the device, since there is no host staging buffer) are done here.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <mutex>

#include "rotvote.h"
#include "rv_device.h"
#include "rv_internal.h"
#include "rv_table.h"

#define RV_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr int kMaxGrid = RV_NOALLOC_MAX_GRID;
constexpr int kMaxJ = RV_NOALLOC_MAX_SAMPLES;
constexpr int kMaxDevices = 64;
constexpr size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
// top-K lists of the largest grid (rv::topk_blocks(64^3) = 64 lists of 64 keys)
constexpr int kMaxLists = 64;
// Byte offsets of the parts of the array, each 256-byte aligned.
constexpr size_t kGridBytes = (size_t)kMaxGrid * kMaxGrid * kMaxGrid * sizeof(int32_t);
constexpr size_t kOffTable = align256(kGridBytes);
constexpr size_t kOffLists = kOffTable + align256((size_t)kMaxJ * sizeof(float2));
constexpr size_t kOffCandQ = kOffLists + align256((size_t)kMaxLists * 64 * sizeof(uint64_t));
constexpr size_t kOffVotes = kOffCandQ + align256(64 * sizeof(float4));
constexpr size_t kOffIdx = kOffVotes + align256(64 * sizeof(int32_t));
constexpr size_t kOffInliers = kOffIdx + align256(64 * sizeof(int32_t));
constexpr size_t kScratchBytes = kOffInliers + align256(64 * sizeof(uint32_t));
static_assert(kScratchBytes <= (size_t)1152 * 1024, "the fixed scratch stays near 1.1 MiB");

}  // namespace

// The fixed scratch.  In host code this name is only a stand-in for the
// symbol: its device address (one per GPU) comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

// Device address of `scratch` on each device, looked up on the first call
// made with that device current.
std::atomic<unsigned char*> g_scratch[kMaxDevices];
std::mutex g_scratch_mu;

hipError_t scratch_on(int dev, unsigned char** out)
{
    unsigned char* p = g_scratch[dev].load(std::memory_order_acquire);
    if (!p) {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        p = g_scratch[dev].load(std::memory_order_relaxed);
        if (!p) {
            void* sym = nullptr;
            const hipError_t e = hipGetSymbolAddress(&sym, HIP_SYMBOL(scratch));
            if (e != hipSuccess)
                return e;
            p = static_cast<unsigned char*>(sym);
            g_scratch[dev].store(p, std::memory_order_release);
        }
    }
    *out = p;
    return hipSuccess;
}

// Clears the grid, writes the sample table of J entries and, for an empty
// solve, the result record of a solve without votes.
__global__ __launch_bounds__(256) void k_noalloc_prepare(int32_t* __restrict__ grid, int64_t ncell,
                                                         float2* __restrict__ table, int J,
                                                         rv::Result* __restrict__ result, int empty)
{
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t nvec = ncell >> 2;
    int4* g4 = reinterpret_cast<int4*>(grid);
    for (int64_t i = t0; i < nvec; i += stride)
        g4[i] = make_int4(0, 0, 0, 0);
    for (int64_t i = (nvec << 2) + t0; i < ncell; i += stride)
        grid[i] = 0;
    for (int64_t j = t0; j < J; j += stride)
        table[j] = rv::table_entry((int)j, J);
    if (empty && t0 == 0) {
        result->q[0] = 1.0f;
        result->q[1] = 0.0f;
        result->q[2] = 0.0f;
        result->q[3] = 0.0f;
        result->count = 0;
        result->winner = -1;
        result->n_cand = 0;
    }
}

rv_status fail(rv_status st, const char* msg)
{
    rv::set_null_error(msg);
    return st;
}

}  // namespace

RV_API rv_status rot_vote_solve_noalloc(const float* x, const float* y, int64_t n, int32_t grid,
                                        int32_t samples_per_circle, int32_t topk, float eps_rad,
                                        void* stream, rv_result* result_device,
                                        uint8_t* inlier_mask)
{
    if (n < 0)
        return fail(RV_EINVAL, "rot_vote_solve_noalloc: n < 0");
    if (grid < 1)
        return fail(RV_EINVAL, "rot_vote_solve_noalloc: grid < 1");
    if (grid > kMaxGrid)
        return fail(RV_EUNSUPPORTED,
                    "rot_vote_solve_noalloc: grid above RV_NOALLOC_MAX_GRID (64), the fixed "
                    "scratch's grid");
    if (samples_per_circle < 0)
        return fail(RV_EINVAL, "rot_vote_solve_noalloc: samples_per_circle < 0");
    const int J = samples_per_circle > 0 ? samples_per_circle : 8 * grid;
    if (J > kMaxJ)
        return fail(RV_EUNSUPPORTED,
                    "rot_vote_solve_noalloc: samples_per_circle above RV_NOALLOC_MAX_SAMPLES "
                    "(4096), the fixed scratch's table");
    if (topk < 1 || topk > RV_MAX_TOPK)
        return fail(RV_EINVAL, "rot_vote_solve_noalloc: topk outside 1..64");
    if (!(eps_rad > 0.0f) || !(eps_rad <= (float)M_PI))
        return fail(RV_EINVAL, "rot_vote_solve_noalloc: eps_rad outside (0, pi]");
    if ((int64_t)J * n > (int64_t)INT32_MAX)
        return fail(RV_EUNSUPPORTED, "rot_vote_solve_noalloc: n*J exceeds int32 vote counts");
    if (!result_device || !rv::is_device_memory(result_device) ||
        reinterpret_cast<uintptr_t>(result_device) % alignof(rv_result) != 0)
        return fail(RV_EINVAL, "rot_vote_solve_noalloc: result_device must be aligned device memory");
    if (n > 0 && (!x || !y || !inlier_mask || !rv::is_device_memory(x) ||
                  !rv::is_device_memory(y) || !rv::is_device_memory(inlier_mask)))
        return fail(RV_EINVAL, "rot_vote_solve_noalloc: x, y and inlier_mask must be device memory");

    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(RV_EDEVICE, "rot_vote_solve_noalloc: no current HIP device");
    unsigned char* base = nullptr;
    if (scratch_on(dev, &base) != hipSuccess)
        return fail(RV_EDEVICE, "rot_vote_solve_noalloc: hipGetSymbolAddress of the fixed scratch failed");

    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t* d_grid = reinterpret_cast<int32_t*>(base);
    float2* d_table = reinterpret_cast<float2*>(base + kOffTable);
    uint64_t* d_lists = reinterpret_cast<uint64_t*>(base + kOffLists);
    rv::Result* d_result = reinterpret_cast<rv::Result*>(result_device);
    const rv::Candidates c{reinterpret_cast<float4*>(base + kOffCandQ),
                           reinterpret_cast<int32_t*>(base + kOffVotes),
                           reinterpret_cast<int32_t*>(base + kOffIdx),
                           reinterpret_cast<uint32_t*>(base + kOffInliers), d_result};
    const int64_t ncell = (int64_t)grid * grid * grid;
    const int nlists = rv::topk_blocks(ncell);
    if (nlists > kMaxLists)
        return fail(RV_EUNSUPPORTED, "rot_vote_solve_noalloc: top-K lists beyond the fixed scratch");

    const int pblocks = (int)std::min<int64_t>(256, std::max<int64_t>(1, ((ncell >> 2) + 255) / 256));
    hipLaunchKernelGGL(k_noalloc_prepare, dim3(pblocks), dim3(256), 0, s, d_grid,
                       n > 0 ? ncell : 0, d_table, n > 0 ? J : 0, d_result, n > 0 ? 0 : 1);
    if (hipGetLastError() != hipSuccess)
        return fail(RV_EDEVICE, "rot_vote_solve_noalloc: launch of the grid clear failed");
    if (n == 0)
        return RV_OK;
    const float T2 = rv::residual_bound(eps_rad);
    if (rv::launch_vote_global(x, y, n, grid, J, d_table, d_grid, 0, s) != hipSuccess ||
        rv::launch_topk_partial(d_grid, ncell, nlists, d_lists, s) != hipSuccess ||
        rv::launch_topk_final(d_lists, nlists, topk, grid, c, s) != hipSuccess ||
        rv::launch_rescore(x, y, n, T2, c, s) != hipSuccess ||
        rv::launch_mask(x, y, n, T2, c, inlier_mask, s) != hipSuccess)
        return fail(RV_EDEVICE, "rot_vote_solve_noalloc: a kernel launch failed");
    return RV_OK;
}
