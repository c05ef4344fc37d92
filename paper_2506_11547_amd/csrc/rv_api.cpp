// C-ABI of the rotation-voting library: argument checks, scratch ownership,
// stage sequencing on one HIP stream, and the two small readbacks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstddef>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rotvote.h"
#include "rv_internal.h"

#define RV_API extern "C" __attribute__((visibility("default")))

namespace rv {

bool is_device_memory(const void* p)
{
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();  // clear the sticky "invalid value" for host pointers
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

// |L q|^2 = 4 sin^2(psi / 2) for the angle psi between R(q) a and b.
float residual_bound(float eps)
{
    const double s = std::sin(0.5 * (double)eps);
    return (float)(4.0 * s * s);
}

}  // namespace rv

using rv::is_device_memory;
using rv::residual_bound;

namespace {

constexpr int kStages = RV_NUM_STAGES;
// Below this grid (<= 1.4 MiB of int32 cells at 72^3) the global-atomic vote
// (one kernel, no queues) measured faster than binning: the solves there are
// small enough that binning's extra stages cost more than its atomics save.
constexpr int kBrickMinGrid = 72;
// Batch queue capacities: a brick's share of the instance's expected runs,
// times this factor (the heaviest brick of an instance with half inliers
// holds about 1.75 shares at G = 64), plus a fixed slack.
constexpr double kBatchCapFactor = 1.75;
constexpr uint32_t kBatchCapSlack = 256;

// Expected runs of one circle: about 1.7 G cell changes (at most J), plus
// the cuts every 240 samples.
int64_t runs_per_circle(int G, int J)
{
    return std::min<int64_t>(J, (int64_t)(1.7 * G) + J / 240 + 2);
}

std::string g_create_error;  // reason of the last failed create (NULL handle)
// The last failed handle-free call's reason when it was not a create: a
// string literal, or null when the create's message is the latest.
std::atomic<const char*> g_null_reason{nullptr};

// rot_vote_solve_async copies the internal result record to the caller's
// rv_result: the two layouts are one.
static_assert(sizeof(rv_result) == sizeof(rv::Result), "result layout");
static_assert(offsetof(rv_result, count) == offsetof(rv::Result, count), "result layout");
static_assert(offsetof(rv_result, winner) == offsetof(rv::Result, winner), "result layout");
static_assert(offsetof(rv_result, n_cand) == offsetof(rv::Result, n_cand), "result layout");

}  // namespace

void rv::set_null_error(const char* msg) { g_null_reason.store(msg); }

struct rv_handle {
    rv_config cfg{};
    hipStream_t stream = nullptr;
    int device = 0;
    int64_t max_n = 0;
    int32_t max_grid = 0;
    int32_t max_J = 0;
    int32_t K = 16;

    int32_t* d_hist = nullptr;          // max_grid^3
    float2* d_table = nullptr;          // max_J (cos, sin)
    uint64_t* d_partial = nullptr;      // kTopkMaxBlocks * 64
    float4* d_cand_q = nullptr;         // 64
    int32_t* d_cand_votes = nullptr;    // 64
    int32_t* d_cand_idx = nullptr;      // 64
    uint32_t* d_cand_inl = nullptr;     // 64
    rv::Result* d_result = nullptr;
    rv::Result* h_result = nullptr;     // pinned
    rv::Result* d_empty = nullptr;      // the result of a solve without votes (q = 1, count 0)
    float2* h_table = nullptr;          // pinned staging for the table
    int32_t table_J = -1;               // J the device table holds

    // brick strategy scratch (allocated when the config allows that strategy)
    bool brick_ok = false;
    rv::BinArgs bin{};
    int32_t* d_ovf = nullptr;           // max_grid^3, zero between solves

    // batch scratch (max_batch > 0)
    int32_t max_batch = 0;
    int32_t batch_grid = 0;             // largest grid of a batch
    int64_t max_units = 0;
    bool batch_grids = false;           // RV_FLAG_BATCH_GRIDS
    rv::Unit* d_units = nullptr;        // max_units
    rv::Unit* h_units = nullptr;        // pinned staging
    uint32_t* d_bplan = nullptr;        // [cap | qbase], 2 * max_batch * 8
    uint32_t* h_bplan = nullptr;        // pinned staging
    int64_t* d_offsets = nullptr;       // max_batch + 1
    int64_t* h_offsets = nullptr;       // pinned staging
    uint32_t* d_bfill = nullptr;        // max_batch * 8
    uint32_t* d_bflags = nullptr;       // max_batch * 8
    uint64_t* d_bpartial = nullptr;     // max_batch * 8 * 64
    float4* d_bcand_q = nullptr;        // max_batch * 64
    int32_t* d_bcand_votes = nullptr;
    int32_t* d_bcand_idx = nullptr;
    uint32_t* d_bcand_inl = nullptr;
    rv::Result* d_bresult = nullptr;    // max_batch
    rv::Result* h_bresult = nullptr;    // pinned
    int32_t* d_bovf = nullptr;          // max_batch * batch_grid^3, zero between batches
    int32_t* d_bgrids = nullptr;        // max_batch * batch_grid^3 (RV_FLAG_BATCH_GRIDS)

    // several rotations
    uint64_t* d_mbits = nullptr;          // max_n candidate sets
    rv::MultiState* d_mstate = nullptr;
    rv::MultiState* h_mstate = nullptr;   // pinned

    // rigid pose: pair buffers of rot_vote_solve_rigid (max_pairs) and the stage state
    int64_t max_pairs = 0;
    float* d_pm = nullptr;                // [3][max_pairs]
    float* d_pn = nullptr;                // [3][max_pairs]
    uint8_t* d_pmask = nullptr;           // max_pairs
    rv::RigidState* d_rigid = nullptr;
    rv::RigidState* h_rigid = nullptr;    // pinned

    // refinement
    rv::RefineState* d_rstate = nullptr;
    rv::RefineState* h_rstate = nullptr;  // pinned
    double* d_rpartial = nullptr;         // kRefineMaxBlocks * kRefineSums

    hipEvent_t ev[kStages + 1] = {};
    bool timing = false;
    bool events_recorded = false;

    // last solve
    bool solved = false;
    int32_t last_grid = 0;
    int32_t last_J = 0;
    int32_t last_strategy = 0;
    int32_t last_ncand = 0;
    int32_t last_winner = -1;
    int64_t last_count = 0;
    bool last_async = false;             // the fields above are read back on demand
    // last batch
    bool batched = false;
    int32_t last_B = 0;
    int32_t last_batch_edge = 0;
    int32_t last_bgrid = 0;

    int64_t device_bytes = 0;           // sum of the handle's device allocations
    int8_t tuned[RV_MAX_GRID + 1] = {};  // per grid: strategy chosen by rot_vote_tune (0: none)
    int8_t batch_edge_log2[RV_MAX_BATCH_GRID + 1] = {};  // per grid: by rot_vote_tune_batch (0: none)
    int32_t forced_strategy = 0;         // while tuning

    std::string err;
};

namespace {

template <typename T>
hipError_t dev_alloc(rv_handle* h, T** p, size_t bytes)
{
    const hipError_t e = hipMalloc(p, bytes);
    if (e == hipSuccess)
        h->device_bytes += (int64_t)bytes;
    return e;
}

rv_status fail(rv_handle* h, rv_status st, const std::string& msg)
{
    if (h)
        h->err = msg;
    else {
        g_create_error = msg;
        g_null_reason.store(nullptr);
    }
    return st;
}

rv_status hip_fail(rv_handle* h, hipError_t e, const char* what)
{
    std::string m = std::string(what) + ": " + hipGetErrorString(e);
    return fail(h, e == hipErrorOutOfMemory ? RV_ENOMEM : RV_EDEVICE, m);
}

#define RV_HIP(h, expr, what)                  \
    do {                                       \
        hipError_t e_ = (expr);                \
        if (e_ != hipSuccess)                  \
            return hip_fail((h), e_, (what));  \
    } while (0)

void release(rv_handle* h)
{
    if (!h)
        return;
    (void)hipSetDevice(h->device);
    (void)hipStreamSynchronize(h->stream);  // scratch may still be in use by queued work
    (void)hipFree(h->d_hist);
    (void)hipFree(h->d_table);
    (void)hipFree(h->d_partial);
    (void)hipFree(h->d_cand_q);
    (void)hipFree(h->d_cand_votes);
    (void)hipFree(h->d_cand_idx);
    (void)hipFree(h->d_cand_inl);
    (void)hipFree(h->d_result);
    (void)hipFree(h->d_empty);
    (void)hipFree(h->bin.pool);
    (void)hipFree(h->bin.fill);
    (void)hipFree(h->bin.qbase);
    (void)hipFree(h->bin.cap);
    (void)hipFree(h->bin.est);
    (void)hipFree(h->bin.flags);
    (void)hipFree(h->bin.order);
    (void)hipFree(h->d_ovf);
    (void)hipFree(h->d_units);
    (void)hipFree(h->d_bplan);
    (void)hipFree(h->d_offsets);
    (void)hipFree(h->d_bfill);
    (void)hipFree(h->d_bflags);
    (void)hipFree(h->d_bpartial);
    (void)hipFree(h->d_bcand_q);
    (void)hipFree(h->d_bcand_votes);
    (void)hipFree(h->d_bcand_idx);
    (void)hipFree(h->d_bcand_inl);
    (void)hipFree(h->d_bresult);
    (void)hipFree(h->d_bovf);
    (void)hipFree(h->d_bgrids);
    (void)hipFree(h->d_pm);
    (void)hipFree(h->d_pn);
    (void)hipFree(h->d_pmask);
    (void)hipFree(h->d_rigid);
    (void)hipHostFree(h->h_rigid);
    (void)hipFree(h->d_mbits);
    (void)hipFree(h->d_mstate);
    (void)hipHostFree(h->h_mstate);
    (void)hipFree(h->d_rstate);
    (void)hipFree(h->d_rpartial);
    (void)hipHostFree(h->h_rstate);
    (void)hipHostFree(h->h_units);
    (void)hipHostFree(h->h_bplan);
    (void)hipHostFree(h->h_offsets);
    (void)hipHostFree(h->h_bresult);
    (void)hipHostFree(h->h_result);
    (void)hipHostFree(h->h_table);
    for (auto& e : h->ev)
        if (e)
            (void)hipEventDestroy(e);
}

// Step 0 of the rule: theta_j = ((2j + 1 - J) / J) * (pi / 2) in binary64,
// cos and sin rounded once to binary32.
void fill_table(float2* t, int J)
{
    for (int j = 0; j < J; ++j) {
        const double th = ((double)(2 * j + 1 - J) / (double)J) * M_PI_2;
        t[j].x = (float)std::cos(th);
        t[j].y = (float)std::sin(th);
    }
}

rv::Candidates candidates(rv_handle* h)
{
    return rv::Candidates{h->d_cand_q, h->d_cand_votes, h->d_cand_idx, h->d_cand_inl, h->d_result};
}

}  // namespace

RV_API void rot_vote_default_config(rv_config* cfg)
{
    if (!cfg)
        return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->device = 0;
    cfg->stream = nullptr;
    cfg->max_n = 1 << 20;
    cfg->max_grid = 256;
    cfg->samples_per_circle = 0;
    cfg->topk = 16;
    cfg->vote_strategy = RV_VOTE_AUTO;
    cfg->flags = 0;
    cfg->max_batch = 0;
    cfg->batch_brick_edge = 0;
}

RV_API rv_status rot_vote_create(rv_handle** out, const rv_config* cfg)
{
    if (!out || !cfg)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: NULL argument");
    if (cfg->max_n < 0)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: max_n < 0");
    if (cfg->max_grid < 1 || cfg->max_grid > RV_MAX_GRID)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: max_grid outside 1..1024");
    if (cfg->samples_per_circle < 0)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: samples_per_circle < 0");
    if (cfg->topk < 1 || cfg->topk > RV_MAX_TOPK)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: topk outside 1..64");
    if (cfg->vote_strategy < RV_VOTE_AUTO || cfg->vote_strategy > RV_VOTE_BRICK)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: unknown vote_strategy");
    if (cfg->flags & ~(uint32_t)(RV_FLAG_TIMING | RV_FLAG_BATCH_GRIDS))
        return fail(nullptr, RV_EINVAL, "rot_vote_create: unknown flags");
    if (cfg->max_batch < 0)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: max_batch < 0");
    if (cfg->batch_brick_edge != 0 && cfg->batch_brick_edge != 16 && cfg->batch_brick_edge != 32)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: batch_brick_edge must be 0, 16 or 32");
    if (cfg->max_batch > 0 && cfg->vote_strategy == RV_VOTE_GLOBAL)
        return fail(nullptr, RV_EUNSUPPORTED,
                    "rot_vote_create: batches use the brick strategy (vote_strategy global)");
    if (cfg->reserved != 0)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: reserved fields must be 0");
    if (cfg->max_pairs < 0 || cfg->max_pairs > cfg->max_n)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: max_pairs outside 0..max_n");
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || cfg->device < 0 || cfg->device >= ndev)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: no such HIP device");

    rv_handle* h = new (std::nothrow) rv_handle();
    if (!h)
        return fail(nullptr, RV_ENOMEM, "rot_vote_create: out of host memory");
    h->cfg = *cfg;
    h->device = cfg->device;
    h->stream = static_cast<hipStream_t>(cfg->stream);
    h->max_n = cfg->max_n;
    h->max_grid = cfg->max_grid;
    h->K = cfg->topk;
    h->max_J = cfg->samples_per_circle > 0 ? cfg->samples_per_circle : 8 * cfg->max_grid;
    h->timing = (cfg->flags & RV_FLAG_TIMING) != 0;

    auto bail = [&](hipError_t e, const char* what) {
        std::string m = std::string("rot_vote_create: ") + what + ": " + hipGetErrorString(e);
        release(h);
        delete h;
        return fail(nullptr, e == hipErrorOutOfMemory ? RV_ENOMEM : RV_EDEVICE, m);
    };
    hipError_t e;
    if ((e = hipSetDevice(h->device)) != hipSuccess)
        return bail(e, "hipSetDevice");
    const size_t ncell = (size_t)h->max_grid * h->max_grid * h->max_grid;
    if ((e = dev_alloc(h, &h->d_hist, ncell * sizeof(int32_t))) != hipSuccess)
        return bail(e, "vote grid");
    if ((e = dev_alloc(h, &h->d_table, (size_t)h->max_J * sizeof(float2))) != hipSuccess)
        return bail(e, "sample table");
    if ((e = dev_alloc(h, &h->d_partial, (size_t)rv::kTopkMaxBlocks * 64 * sizeof(uint64_t))) !=
        hipSuccess)
        return bail(e, "top-K scratch");
    if ((e = dev_alloc(h, &h->d_cand_q, 64 * sizeof(float4))) != hipSuccess ||
        (e = dev_alloc(h, &h->d_cand_votes, 64 * sizeof(int32_t))) != hipSuccess ||
        (e = dev_alloc(h, &h->d_cand_idx, 64 * sizeof(int32_t))) != hipSuccess ||
        (e = dev_alloc(h, &h->d_cand_inl, 64 * sizeof(uint32_t))) != hipSuccess ||
        (e = dev_alloc(h, &h->d_result, sizeof(rv::Result))) != hipSuccess ||
        (e = dev_alloc(h, &h->d_empty, sizeof(rv::Result))) != hipSuccess)
        return bail(e, "candidate buffers");
    {
        rv::Result empty{};
        empty.q[0] = 1.0f;
        empty.winner = -1;
        if ((e = hipMemcpy(h->d_empty, &empty, sizeof(empty), hipMemcpyHostToDevice)) != hipSuccess)
            return bail(e, "empty result");
    }
    if ((e = hipHostMalloc(&h->h_result, sizeof(rv::Result), hipHostMallocDefault)) != hipSuccess)
        return bail(e, "pinned result");
    if ((e = hipHostMalloc(&h->h_table, (size_t)h->max_J * sizeof(float2), hipHostMallocDefault)) !=
        hipSuccess)
        return bail(e, "pinned table");
    for (auto& ev : h->ev)
        if ((e = hipEventCreate(&ev)) != hipSuccess)
            return bail(e, "events");
    if ((e = dev_alloc(h, &h->d_rstate, sizeof(rv::RefineState))) != hipSuccess ||
        (e = dev_alloc(h, &h->d_rpartial,
                       (size_t)rv::kRefineMaxBlocks * rv::kRefineSums * sizeof(double))) != hipSuccess)
        return bail(e, "refinement scratch");
    if ((e = hipHostMalloc(&h->h_rstate, sizeof(rv::RefineState), hipHostMallocDefault)) != hipSuccess)
        return bail(e, "pinned refinement state");
    if ((e = dev_alloc(h, &h->d_mbits, (size_t)std::max<int64_t>(1, h->max_n) * sizeof(uint64_t))) !=
            hipSuccess ||
        (e = dev_alloc(h, &h->d_mstate, sizeof(rv::MultiState))) != hipSuccess)
        return bail(e, "model scratch");
    if ((e = hipHostMalloc(&h->h_mstate, sizeof(rv::MultiState), hipHostMallocDefault)) != hipSuccess)
        return bail(e, "pinned model state");
    if ((e = dev_alloc(h, &h->d_rigid, sizeof(rv::RigidState))) != hipSuccess)
        return bail(e, "rigid state");
    if ((e = hipHostMalloc(&h->h_rigid, sizeof(rv::RigidState), hipHostMallocDefault)) != hipSuccess)
        return bail(e, "pinned rigid state");
    h->max_pairs = cfg->max_pairs;
    if (h->max_pairs > 0) {
        const size_t P = (size_t)h->max_pairs;
        if ((e = dev_alloc(h, &h->d_pm, 3 * P * sizeof(float))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_pn, 3 * P * sizeof(float))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_pmask, P)) != hipSuccess)
            return bail(e, "pair buffers");
    }
    h->max_batch = cfg->max_batch;
    h->batch_grid = std::min(h->max_grid, rv::kMaxBatchGrid);
    h->batch_grids = (cfg->flags & RV_FLAG_BATCH_GRIDS) != 0;
    // the brick strategy serves grids up to kMaxBrickGrid (its scratch is sized for
    // min(max_grid, kMaxBrickGrid)); larger grids use global atomics
    const bool want_brick = cfg->vote_strategy != RV_VOTE_GLOBAL && h->max_grid >= 1;
    const int64_t brick_grid = std::min<int64_t>(h->max_grid, rv::kMaxBrickGrid);
    const size_t brick_cells = (size_t)(brick_grid * brick_grid * brick_grid);
    uint64_t runs = 0;
    if (want_brick) {
        // One solve: about 1.7 G runs per circle are expected at J = 8 G (at
        // most J); room for 3 G per circle plus the per-queue slack.
        const uint64_t per_circle = (uint64_t)std::min<int64_t>(h->max_J, 3 * (int64_t)h->max_grid);
        runs = (uint64_t)h->max_n * per_circle + (uint64_t)rv::kQueueSets * rv::kMaxBricksAll * 320u;
    }
    if (h->max_batch > 0) {
        // A batch reserves kBatchCapFactor expected runs per circle plus the
        // slack and rounding of every queue.
        const uint64_t per_circle =
            (uint64_t)std::ceil(kBatchCapFactor * (double)runs_per_circle(h->batch_grid, h->max_J));
        const uint64_t b = (uint64_t)h->max_n * per_circle +
                           (uint64_t)h->max_batch * rv::kMaxBatchBricks * (kBatchCapSlack + 128u);
        runs = std::max(runs, b);
    }
    runs = std::min<uint64_t>(runs, 0xFFFFFFFFull - 64);
    h->bin.pool_runs = runs;
    if (runs > 0 && (e = dev_alloc(h, &h->bin.pool, runs * sizeof(uint32_t))) != hipSuccess)
        return bail(e, "brick run pool");
    h->bin.nsets = rv::kQueueSets;
    h->bin.qstride = rv::kMaxBricksAll;
    h->bin.units = nullptr;
    h->bin.batch = 0;
    if (want_brick) {
        const size_t nq = (size_t)rv::kQueueSets * rv::kMaxBricksAll;
        if ((e = dev_alloc(h, &h->bin.fill, nq * sizeof(uint32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->bin.qbase, nq * sizeof(uint32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->bin.cap, rv::kMaxBricksAll * sizeof(uint32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->bin.est, rv::kMaxBricksAll * sizeof(uint32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->bin.flags, rv::kMaxBricksAll * sizeof(uint32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->bin.order, rv::kMaxBricksAll * sizeof(uint32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_ovf, brick_cells * sizeof(int32_t))) != hipSuccess)
            return bail(e, "brick scratch");
        if ((e = hipMemset(h->bin.est, 0, rv::kMaxBricksAll * sizeof(uint32_t))) != hipSuccess ||
            (e = hipMemset(h->d_ovf, 0, brick_cells * sizeof(int32_t))) != hipSuccess ||
            (e = hipDeviceSynchronize()) != hipSuccess)
            return bail(e, "brick scratch init");
        h->bin.ovf = h->d_ovf;
        h->brick_ok = true;
    }
    if (h->max_batch > 0) {
        const int64_t B = h->max_batch;
        const int64_t nq = B * rv::kMaxBatchBricks;
        const int64_t bg = h->batch_grid;
        const size_t gcells = (size_t)B * (size_t)(bg * bg * bg);
        h->max_units = (h->max_n + rv::kUnitSize - 1) / rv::kUnitSize + B;
        if ((e = dev_alloc(h, &h->d_units, (size_t)h->max_units * sizeof(rv::Unit))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bplan, (size_t)(2 * nq) * sizeof(uint32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_offsets, (size_t)(B + 1) * sizeof(int64_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bfill, (size_t)nq * sizeof(uint32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bflags, (size_t)nq * sizeof(uint32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bpartial, (size_t)nq * 64 * sizeof(uint64_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bcand_q, (size_t)B * 64 * sizeof(float4))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bcand_votes, (size_t)B * 64 * sizeof(int32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bcand_idx, (size_t)B * 64 * sizeof(int32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bcand_inl, (size_t)B * 64 * sizeof(uint32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bresult, (size_t)B * sizeof(rv::Result))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bovf, gcells * sizeof(int32_t))) != hipSuccess)
            return bail(e, "batch scratch");
        if (h->batch_grids && (e = dev_alloc(h, &h->d_bgrids, gcells * sizeof(int32_t))) != hipSuccess)
            return bail(e, "batch grids");
        if ((e = hipHostMalloc(&h->h_units, (size_t)h->max_units * sizeof(rv::Unit),
                               hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc(&h->h_bplan, (size_t)(2 * nq) * sizeof(uint32_t),
                               hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc(&h->h_offsets, (size_t)(B + 1) * sizeof(int64_t),
                               hipHostMallocDefault)) != hipSuccess ||
            (e = hipHostMalloc(&h->h_bresult, (size_t)B * sizeof(rv::Result),
                               hipHostMallocDefault)) != hipSuccess)
            return bail(e, "pinned batch staging");
        if ((e = hipMemset(h->d_bovf, 0, gcells * sizeof(int32_t))) != hipSuccess ||
            (e = hipDeviceSynchronize()) != hipSuccess)
            return bail(e, "batch scratch init");
    }
    *out = h;
    return RV_OK;
}

RV_API rv_status rot_vote_destroy(rv_handle* h)
{
    if (!h)
        return RV_OK;
    release(h);
    delete h;
    return RV_OK;
}

RV_API const char* rot_vote_last_error(const rv_handle* h)
{
    if (h)
        return h->err.c_str();
    const char* r = g_null_reason.load();
    return r ? r : g_create_error.c_str();
}

RV_API rv_status rot_vote_set_stream(rv_handle* h, void* stream)
{
    if (!h)
        return RV_EINVAL;
    h->stream = static_cast<hipStream_t>(stream);
    h->err.clear();
    return RV_OK;
}

namespace {

// Argument checks shared by the solve entry points; sets *J.
rv_status check_solve(rv_handle* h, const char* fn, const float* x, const float* y, int64_t n,
                      int32_t grid, float eps_rad, const void* out_mask, int32_t* J)
{
    const std::string f(fn);
    if (n < 0)
        return fail(h, RV_EINVAL, f + ": n < 0");
    if (n > h->max_n)
        return fail(h, RV_EINVAL, f + ": n exceeds the handle's max_n");
    if (grid < 1 || grid > h->max_grid)
        return fail(h, RV_EINVAL, f + ": grid outside 1..max_grid");
    if (!(eps_rad > 0.0f) || !(eps_rad <= (float)M_PI))
        return fail(h, RV_EINVAL, f + ": eps_rad outside (0, pi]");
    *J = h->cfg.samples_per_circle > 0 ? h->cfg.samples_per_circle : 8 * grid;
    if (*J > h->max_J)
        return fail(h, RV_EINVAL, f + ": J = 8*grid exceeds the table sized at create");
    if ((int64_t)*J * n > (int64_t)INT32_MAX)
        return fail(h, RV_EUNSUPPORTED, f + ": n*J exceeds int32 vote counts");
    if (n > 0) {
        if (!x || !y || !out_mask)
            return fail(h, RV_EINVAL, f + ": x, y and the mask or labels must not be NULL");
        if (!is_device_memory(x) || !is_device_memory(y) || !is_device_memory(out_mask))
            return fail(h, RV_EINVAL, f + ": x, y and the mask or labels must be device memory");
    }
    return RV_OK;
}

// Stages 0-3 of a solve on the handle's stream: vote (either strategy),
// reduce, and for n > 0 the decoded top-K candidates with cleared inlier
// counters.  Records events 0..4 when timing.
rv_status vote_candidates(rv_handle* h, const float* x, const float* y, int64_t n, int32_t grid,
                          int32_t J, const char* fn)
{
    const std::string f(fn);
    hipStream_t s = h->stream;
    const int64_t ncell = (int64_t)grid * grid * grid;
    int strategy = h->forced_strategy ? h->forced_strategy : h->cfg.vote_strategy;
    if (strategy == RV_VOTE_AUTO && h->tuned[grid] != 0)
        strategy = h->tuned[grid];  // measured by rot_vote_tune
    if (strategy == RV_VOTE_AUTO)
        strategy = (h->brick_ok && grid >= kBrickMinGrid && grid <= rv::kMaxBrickGrid)
                       ? RV_VOTE_BRICK : RV_VOTE_GLOBAL;
    if (strategy == RV_VOTE_BRICK && !(h->brick_ok && grid <= rv::kMaxBrickGrid))
        return fail(h, RV_EUNSUPPORTED,
                    f + ": the brick strategy needs grid <= 384 and a handle created for it");

    if (h->table_J != J) {
        RV_HIP(h, hipStreamSynchronize(s), "sync before table upload");
        fill_table(h->h_table, J);
        RV_HIP(h, hipMemcpyAsync(h->d_table, h->h_table, (size_t)J * sizeof(float2),
                                 hipMemcpyHostToDevice, s),
               "table upload");
        h->table_J = J;
    }

    const bool tm = h->timing;
    const bool brick = strategy == RV_VOTE_BRICK;
    h->solved = true;
    h->last_async = false;
    h->last_grid = grid;
    h->last_J = J;
    h->last_strategy = strategy;
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[0], s), "event");
    const int edge = rv::solve_edge_log2(grid);
    if (brick)
        RV_HIP(h, rv::launch_bin_prepare(x, y, n, grid, J, edge, h->d_table, h->bin, s),
               "brick plan");
    else
        RV_HIP(h, rv::launch_fill(h->d_hist, ncell, 0, s), "clear grid");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[1], s), "event");
    if (brick)
        RV_HIP(h, rv::launch_bin_vote(x, y, n, grid, J, edge, h->d_table, h->bin, s),
               "binned vote");
    else
        RV_HIP(h, rv::launch_vote_global(x, y, n, grid, J, h->d_table, h->d_hist, 0, s), "vote");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[2], s), "event");
    int nlists;
    if (brick) {
        RV_HIP(h, rv::launch_brick_accum(grid, h->K, edge, h->d_hist, h->d_partial, h->bin, s),
               "brick accumulate");
        const int nba = rv::brick_axis(grid, edge);
        nlists = nba * nba * nba;
    } else {
        nlists = rv::topk_blocks(ncell);
        RV_HIP(h, rv::launch_topk_partial(h->d_hist, ncell, nlists, h->d_partial, s), "top-K partial");
    }
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[3], s), "event");
    if (n == 0)
        return RV_OK;
    RV_HIP(h, rv::launch_topk_final(h->d_partial, nlists, h->K, grid, candidates(h), s),
           "top-K final");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[4], s), "event");
    return RV_OK;
}

void record_empty(rv_handle* h)
{
    h->last_ncand = 0;
    h->last_winner = -1;
    h->last_count = 0;
    h->events_recorded = false;
}

}  // namespace

RV_API rv_status rot_vote_solve(rv_handle* h, const float* x, const float* y, int64_t n,
                                int32_t grid, float eps_rad, float q_out[4],
                                int64_t* inlier_count, uint8_t* inlier_mask)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (!q_out || !inlier_count)
        return fail(h, RV_EINVAL, "rot_vote_solve: q_out and inlier_count must not be NULL");
    int32_t J = 0;
    if (rv_status st = check_solve(h, "rot_vote_solve", x, y, n, grid, eps_rad, inlier_mask, &J))
        return st;
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    hipStream_t s = h->stream;
    if (rv_status st = vote_candidates(h, x, y, n, grid, J, "rot_vote_solve"))
        return st;
    if (n == 0) {
        RV_HIP(h, hipStreamSynchronize(s), "sync");
        q_out[0] = 1.0f;
        q_out[1] = q_out[2] = q_out[3] = 0.0f;
        *inlier_count = 0;
        record_empty(h);
        return RV_OK;
    }
    const bool tm = h->timing;
    const float T2 = residual_bound(eps_rad);
    const rv::Candidates c = candidates(h);
    RV_HIP(h, rv::launch_rescore(x, y, n, T2, c, s), "rescore");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[5], s), "event");
    RV_HIP(h, rv::launch_mask(x, y, n, T2, c, inlier_mask, s), "mask");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[6], s), "event");
    RV_HIP(h, hipMemcpyAsync(h->h_result, h->d_result, sizeof(rv::Result), hipMemcpyDeviceToHost, s),
           "result readback");
    RV_HIP(h, hipStreamSynchronize(s), "sync");
    h->events_recorded = tm;
    const rv::Result& r = *h->h_result;
    std::memcpy(q_out, r.q, sizeof(r.q));
    *inlier_count = r.count;
    h->last_ncand = r.n_cand;
    h->last_winner = r.winner;
    h->last_count = r.count;
    return RV_OK;
}

RV_API rv_status rot_vote_solve_async(rv_handle* h, const float* x, const float* y, int64_t n,
                                      int32_t grid, float eps_rad, rv_result* result_device,
                                      uint8_t* inlier_mask)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (!result_device || !is_device_memory(result_device) ||
        reinterpret_cast<uintptr_t>(result_device) % alignof(rv_result) != 0)
        return fail(h, RV_EINVAL,
                    "rot_vote_solve_async: result_device must be aligned device memory");
    int32_t J = 0;
    if (rv_status st = check_solve(h, "rot_vote_solve_async", x, y, n, grid, eps_rad, inlier_mask,
                                   &J))
        return st;
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    hipStream_t s = h->stream;
    if (rv_status st = vote_candidates(h, x, y, n, grid, J, "rot_vote_solve_async"))
        return st;
    const rv::Result* src = h->d_empty;
    h->events_recorded = false;
    if (n > 0) {
        const bool tm = h->timing;
        const float T2 = residual_bound(eps_rad);
        const rv::Candidates c = candidates(h);
        RV_HIP(h, rv::launch_rescore(x, y, n, T2, c, s), "rescore");
        if (tm)
            RV_HIP(h, hipEventRecord(h->ev[5], s), "event");
        RV_HIP(h, rv::launch_mask(x, y, n, T2, c, inlier_mask, s), "mask");
        if (tm)
            RV_HIP(h, hipEventRecord(h->ev[6], s), "event");
        h->events_recorded = tm;
        src = h->d_result;
    }
    RV_HIP(h, hipMemcpyAsync(result_device, src, sizeof(rv::Result), hipMemcpyDeviceToDevice, s),
           "result copy");
    if (n > 0) {
        h->last_async = true;
    } else {
        record_empty(h);
    }
    return RV_OK;
}

RV_API rv_status rot_vote_tune(rv_handle* h, const float* x, const float* y, int64_t n,
                               int32_t grid, float eps_rad, int32_t reps, uint8_t* mask_scratch,
                               int32_t* strategy_out, float ms_out[2])
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (reps < 1 || reps > 1000)
        return fail(h, RV_EINVAL, "rot_vote_tune: reps outside 1..1000");
    if (n < 1)
        return fail(h, RV_EINVAL, "rot_vote_tune: needs n >= 1");
    int32_t J = 0;
    if (rv_status st = check_solve(h, "rot_vote_tune", x, y, n, grid, eps_rad, mask_scratch, &J))
        return st;
    const bool brick_ok = h->brick_ok && grid <= rv::kMaxBrickGrid;
    const int cand[2] = {RV_VOTE_GLOBAL, RV_VOTE_BRICK};
    float ms[2] = {-1.0f, -1.0f};
    float q[4];
    int64_t cnt = 0;
    for (int c = 0; c < 2; ++c) {
        if (cand[c] == RV_VOTE_BRICK && !brick_ok)
            continue;
        h->forced_strategy = cand[c];
        rv_status st = rot_vote_solve(h, x, y, n, grid, eps_rad, q, &cnt, mask_scratch);  // warm-up
        const auto t0 = std::chrono::steady_clock::now();
        for (int r = 0; st == RV_OK && r < reps; ++r)
            st = rot_vote_solve(h, x, y, n, grid, eps_rad, q, &cnt, mask_scratch);
        const auto t1 = std::chrono::steady_clock::now();
        h->forced_strategy = 0;
        if (st != RV_OK)
            return st;
        ms[c] = (float)(std::chrono::duration<double, std::milli>(t1 - t0).count() / reps);
    }
    const int best = (ms[1] >= 0.0f && ms[1] < ms[0]) ? RV_VOTE_BRICK : RV_VOTE_GLOBAL;
    h->tuned[grid] = (int8_t)best;
    if (strategy_out)
        *strategy_out = best;
    if (ms_out) {
        ms_out[0] = ms[0];
        ms_out[1] = ms[1];
    }
    return RV_OK;
}

RV_API rv_status rot_vote_solve_multi(rv_handle* h, const float* x, const float* y, int64_t n,
                                      int32_t grid, float eps_rad, int32_t max_models,
                                      float sep_rad, int64_t min_inliers, float* q_out,
                                      int64_t* counts, int32_t* n_models, uint8_t* labels)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (!q_out || !counts || !n_models)
        return fail(h, RV_EINVAL, "rot_vote_solve_multi: q_out, counts and n_models must not be NULL");
    if (max_models < 1 || max_models > h->K)
        return fail(h, RV_EINVAL, "rot_vote_solve_multi: max_models outside 1..topk");
    if (!(sep_rad >= 0.0f) || !(sep_rad <= (float)M_PI))
        return fail(h, RV_EINVAL, "rot_vote_solve_multi: sep_rad outside [0, pi]");
    if (min_inliers < 1)
        return fail(h, RV_EINVAL, "rot_vote_solve_multi: min_inliers < 1");
    int32_t J = 0;
    if (rv_status st = check_solve(h, "rot_vote_solve_multi", x, y, n, grid, eps_rad, labels, &J))
        return st;
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    hipStream_t s = h->stream;
    if (rv_status st = vote_candidates(h, x, y, n, grid, J, "rot_vote_solve_multi"))
        return st;
    if (n == 0) {
        RV_HIP(h, hipStreamSynchronize(s), "sync");
        *n_models = 0;
        record_empty(h);
        return RV_OK;
    }
    const bool tm = h->timing;
    const float cos_half_sep = (float)std::cos(0.5 * (double)sep_rad);
    RV_HIP(h, rv::launch_multi(x, y, n, residual_bound(eps_rad), max_models, cos_half_sep,
                               min_inliers, candidates(h), h->d_mbits, labels, h->d_mstate, s),
           "models");
    if (tm) {
        RV_HIP(h, hipEventRecord(h->ev[5], s), "event");
        RV_HIP(h, hipEventRecord(h->ev[6], s), "event");
    }
    RV_HIP(h, hipMemcpyAsync(h->h_mstate, h->d_mstate, sizeof(rv::MultiState), hipMemcpyDeviceToHost,
                             s),
           "models readback");
    RV_HIP(h, hipMemcpyAsync(h->h_result, h->d_result, sizeof(rv::Result), hipMemcpyDeviceToHost, s),
           "result readback");
    RV_HIP(h, hipStreamSynchronize(s), "sync");
    h->events_recorded = tm;
    const rv::MultiState& ms = *h->h_mstate;
    *n_models = ms.n_models;
    for (int m = 0; m < ms.n_models; ++m) {
        std::memcpy(q_out + 4 * m, ms.m_q[m], sizeof(ms.m_q[m]));
        counts[m] = ms.m_count[m];
    }
    const rv::Result& r = *h->h_result;
    h->last_ncand = r.n_cand;
    h->last_winner = r.winner;
    h->last_count = r.count;
    return RV_OK;
}

RV_API rv_status rot_vote_refine(rv_handle* h, const float* x, const float* y, int64_t n,
                                 float eps_rad, int32_t max_rounds, float q_io[4],
                                 int64_t* inlier_count, uint8_t* inlier_mask, int32_t* rounds_run)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (!q_io || !inlier_count)
        return fail(h, RV_EINVAL, "rot_vote_refine: q_io and inlier_count must not be NULL");
    if (n < 0 || n > h->max_n)
        return fail(h, RV_EINVAL, "rot_vote_refine: n outside 0..max_n");
    if (!(eps_rad > 0.0f) || !(eps_rad <= (float)M_PI))
        return fail(h, RV_EINVAL, "rot_vote_refine: eps_rad outside (0, pi]");
    if (max_rounds < 1 || max_rounds > RV_MAX_REFINE_ROUNDS)
        return fail(h, RV_EINVAL, "rot_vote_refine: max_rounds outside 1..64");
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(q_io[k]))
            return fail(h, RV_EINVAL, "rot_vote_refine: q_io must be finite");
    if (n == 0) {
        *inlier_count = 0;
        if (rounds_run)
            *rounds_run = 0;
        return RV_OK;
    }
    if (!x || !y || !inlier_mask)
        return fail(h, RV_EINVAL, "rot_vote_refine: x, y and inlier_mask must not be NULL");
    if (!is_device_memory(x) || !is_device_memory(y) || !is_device_memory(inlier_mask))
        return fail(h, RV_EINVAL, "rot_vote_refine: x, y and inlier_mask must be device memory");
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    hipStream_t s = h->stream;
    RV_HIP(h, rv::launch_refine(x, y, n, residual_bound(eps_rad), max_rounds, q_io, inlier_mask,
                                h->d_rstate, h->d_rpartial, s),
           "refine");
    RV_HIP(h, hipMemcpyAsync(h->h_rstate, h->d_rstate, sizeof(rv::RefineState),
                             hipMemcpyDeviceToHost, s),
           "refine readback");
    RV_HIP(h, hipStreamSynchronize(s), "sync");
    const rv::RefineState& st = *h->h_rstate;
    std::memcpy(q_io, st.q, sizeof(st.q));
    *inlier_count = (int64_t)st.count;
    if (rounds_run)
        *rounds_run = st.rounds;
    return RV_OK;
}

RV_API rv_status rot_vote_pairs(rv_handle* h, const float* x, const float* y, int64_t n, float mu,
                                int64_t capacity, float* m_out, float* n_out, int32_t* idx_out,
                                int64_t* pairs)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (!pairs)
        return fail(h, RV_EINVAL, "rot_vote_pairs: pairs must not be NULL");
    if (n < 0 || n > h->max_n)
        return fail(h, RV_EINVAL, "rot_vote_pairs: n outside 0..max_n");
    if (n > (int64_t)RV_MAX_RIGID_N)
        return fail(h, RV_EUNSUPPORTED, "rot_vote_pairs: n above RV_MAX_RIGID_N (quadratic work)");
    if (!(mu >= 0.0f))
        return fail(h, RV_EINVAL, "rot_vote_pairs: mu must be >= 0");
    if (capacity < 0)
        return fail(h, RV_EINVAL, "rot_vote_pairs: capacity < 0");
    if (n < 2) {
        *pairs = 0;
        return RV_OK;
    }
    if (!x || !y || !is_device_memory(x) || !is_device_memory(y))
        return fail(h, RV_EINVAL, "rot_vote_pairs: x and y must be device memory");
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    hipStream_t s = h->stream;
    RV_HIP(h, rv::launch_pairs_count(x, y, n, mu, h->d_mbits, h->d_rigid, s), "pair count");
    RV_HIP(h, hipMemcpyAsync(h->h_rigid, h->d_rigid, sizeof(rv::RigidState), hipMemcpyDeviceToHost, s),
           "pair count readback");
    RV_HIP(h, hipStreamSynchronize(s), "sync");
    const int64_t P = (int64_t)h->h_rigid->pairs;
    *pairs = P;
    if (P > capacity)
        return fail(h, RV_ENOMEM, "rot_vote_pairs: " + std::to_string(P) +
                                      " pairs pass the length check, more than the capacity " +
                                      std::to_string(capacity));
    if (P == 0)
        return RV_OK;
    if (!m_out || !n_out || !is_device_memory(m_out) || !is_device_memory(n_out) ||
        (idx_out && !is_device_memory(idx_out)))
        return fail(h, RV_EINVAL, "rot_vote_pairs: m_out, n_out (and idx_out) must be device memory");
    RV_HIP(h, rv::launch_pairs_emit(x, y, n, mu, h->d_mbits, P, m_out, n_out, idx_out, s),
           "pair emit");
    RV_HIP(h, hipStreamSynchronize(s), "sync");
    return RV_OK;
}

RV_API rv_status rot_vote_translation(rv_handle* h, const float* x, const float* y, int64_t n,
                                      const float q[4], float t_min, float t_step, int32_t t_cells,
                                      float t_inlier, float t_out[3], int64_t* t_votes,
                                      int64_t* inliers, uint8_t* inlier_mask)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (!q || !t_out || !t_votes || !inliers)
        return fail(h, RV_EINVAL, "rot_vote_translation: q, t_out, t_votes and inliers must not be NULL");
    if (n < 0 || n > h->max_n)
        return fail(h, RV_EINVAL, "rot_vote_translation: n outside 0..max_n");
    if (n > (int64_t)RV_MAX_RIGID_N)
        return fail(h, RV_EUNSUPPORTED,
                    "rot_vote_translation: n above RV_MAX_RIGID_N (quadratic work)");
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(q[k]))
            return fail(h, RV_EINVAL, "rot_vote_translation: q must be finite");
    if (!std::isfinite(t_min) || !(t_step > 0.0f) || !std::isfinite(t_step))
        return fail(h, RV_EINVAL, "rot_vote_translation: t_min must be finite and t_step > 0");
    if (t_cells < 1 || t_cells > RV_MAX_T_CELLS)
        return fail(h, RV_EINVAL, "rot_vote_translation: t_cells outside 1..1024");
    if (!(t_inlier >= 0.0f) || !std::isfinite(t_inlier))
        return fail(h, RV_EINVAL, "rot_vote_translation: t_inlier must be finite and >= 0");
    if (n > 0 && (!x || !y || !inlier_mask || !is_device_memory(x) || !is_device_memory(y) ||
                  !is_device_memory(inlier_mask)))
        return fail(h, RV_EINVAL, "rot_vote_translation: x, y and inlier_mask must be device memory");
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    hipStream_t s = h->stream;
    const float T2 = (float)((double)t_inlier * (double)t_inlier);
    RV_HIP(h, rv::launch_translation(x, y, n, q, t_min, t_step, t_cells, T2,
                                     reinterpret_cast<uint32_t*>(h->d_mbits), inlier_mask,
                                     h->d_rigid, s),
           "translation vote");
    RV_HIP(h, hipMemcpyAsync(h->h_rigid, h->d_rigid, sizeof(rv::RigidState), hipMemcpyDeviceToHost, s),
           "translation readback");
    RV_HIP(h, hipStreamSynchronize(s), "sync");
    const rv::RigidState& r = *h->h_rigid;
    std::memcpy(t_out, r.t, sizeof(r.t));
    *t_votes = (int64_t)r.votes;
    *inliers = (int64_t)r.inliers;
    return RV_OK;
}

RV_API rv_status rot_vote_solve_rigid(rv_handle* h, const float* x, const float* y, int64_t n,
                                      const rv_rigid_params* p, rv_rigid_result* res,
                                      uint8_t* inlier_mask)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (!p || !res)
        return fail(h, RV_EINVAL, "rot_vote_solve_rigid: p and res must not be NULL");
    if (h->max_pairs == 0)
        return fail(h, RV_EUNSUPPORTED, "rot_vote_solve_rigid: the handle has no pair buffers (max_pairs 0)");
    if (p->grid < 1 || p->grid > h->max_grid)
        return fail(h, RV_EINVAL, "rot_vote_solve_rigid: grid outside 1..max_grid");
    if (!(p->eps_rad > 0.0f) || !(p->eps_rad <= (float)M_PI))
        return fail(h, RV_EINVAL, "rot_vote_solve_rigid: eps_rad outside (0, pi]");
    if (p->refine_rounds < 0 || p->refine_rounds > RV_MAX_REFINE_ROUNDS)
        return fail(h, RV_EINVAL, "rot_vote_solve_rigid: refine_rounds outside 0..64");
    if (!(p->mu >= 0.0f))
        return fail(h, RV_EINVAL, "rot_vote_solve_rigid: mu must be >= 0");
    if (!std::isfinite(p->t_min) || !(p->t_step > 0.0f) || !std::isfinite(p->t_step) ||
        p->t_cells < 1 || p->t_cells > RV_MAX_T_CELLS || !(p->t_inlier >= 0.0f) ||
        !std::isfinite(p->t_inlier))
        return fail(h, RV_EINVAL, "rot_vote_solve_rigid: translation domain or t_inlier invalid");
    if (n > 0 && (!inlier_mask || !is_device_memory(inlier_mask)))
        return fail(h, RV_EINVAL, "rot_vote_solve_rigid: inlier_mask must be device memory");
    rv_rigid_result r{};
    r.q[0] = 1.0f;
    if (rv_status st = rot_vote_pairs(h, x, y, n, p->mu, h->max_pairs, h->d_pm, h->d_pn, nullptr,
                                      &r.pairs)) {
        res->pairs = r.pairs;
        return st;
    }
    const int64_t P = r.pairs;
    if (P > 0) {
        // the pair buffers hold [3][P] with stride P
        if (rv_status st = rot_vote_solve(h, h->d_pm, h->d_pn, P, p->grid, p->eps_rad, r.q,
                                          &r.rot_inliers, h->d_pmask))
            return st;
        if (p->refine_rounds > 0)
            if (rv_status st = rot_vote_refine(h, h->d_pm, h->d_pn, P, p->eps_rad, p->refine_rounds,
                                               r.q, &r.rot_inliers, h->d_pmask, &r.refine_rounds_run))
                return st;
    }
    if (rv_status st = rot_vote_translation(h, x, y, n, r.q, p->t_min, p->t_step, p->t_cells,
                                            p->t_inlier, r.t, &r.t_votes, &r.inliers, inlier_mask))
        return st;
    *res = r;
    return RV_OK;
}

RV_API rv_status rot_vote_solve_batch(rv_handle* h, const float* x, const float* y,
                                      const int64_t* offsets, int32_t B, int32_t grid, float eps_rad,
                                      float* q_out, int64_t* inlier_count, uint8_t* inlier_mask)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (h->max_batch == 0)
        return fail(h, RV_EUNSUPPORTED, "rot_vote_solve_batch: handle created with max_batch = 0");
    if (B < 0 || B > h->max_batch)
        return fail(h, RV_EINVAL, "rot_vote_solve_batch: B outside 0..max_batch");
    if (B == 0)
        return RV_OK;
    if (!offsets || !q_out || !inlier_count)
        return fail(h, RV_EINVAL, "rot_vote_solve_batch: offsets, q_out and inlier_count must not be NULL");
    if (grid < 1 || grid > h->batch_grid)
        return fail(h, RV_EINVAL, "rot_vote_solve_batch: grid outside 1..min(max_grid, 64)");
    if (!(eps_rad > 0.0f) || !(eps_rad <= (float)M_PI))
        return fail(h, RV_EINVAL, "rot_vote_solve_batch: eps_rad outside (0, pi]");
    const int32_t J = h->cfg.samples_per_circle > 0 ? h->cfg.samples_per_circle : 8 * grid;
    if (J > h->max_J)
        return fail(h, RV_EINVAL, "rot_vote_solve_batch: J = 8*grid exceeds the table sized at create");
    if (offsets[0] != 0)
        return fail(h, RV_EINVAL, "rot_vote_solve_batch: offsets[0] must be 0");
    for (int32_t b = 0; b < B; ++b) {
        const int64_t nb = offsets[b + 1] - offsets[b];
        if (nb < 0)
            return fail(h, RV_EINVAL, "rot_vote_solve_batch: offsets must be nondecreasing");
        if (offsets[b + 1] > h->max_n)
            return fail(h, RV_EINVAL, "rot_vote_solve_batch: offsets[B] exceeds the handle's max_n");
        if (nb * (int64_t)J > (int64_t)INT32_MAX)
            return fail(h, RV_EUNSUPPORTED, "rot_vote_solve_batch: an instance's n*J exceeds int32 vote counts");
    }
    const int64_t n = offsets[B];
    if (n > 0) {
        if (!x || !y || !inlier_mask)
            return fail(h, RV_EINVAL, "rot_vote_solve_batch: x, y and inlier_mask must not be NULL");
        if (!is_device_memory(x) || !is_device_memory(y) || !is_device_memory(inlier_mask))
            return fail(h, RV_EINVAL, "rot_vote_solve_batch: x, y and inlier_mask must be device memory");
    }
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    hipStream_t s = h->stream;
    const float T2 = residual_bound(eps_rad);
    // brick edge: fixed by the config, else measured by rot_vote_tune_batch, else 32
    const int edge_log2 = h->cfg.batch_brick_edge == 16   ? 4
                          : h->cfg.batch_brick_edge == 32 ? 5
                          : h->batch_edge_log2[grid]      ? h->batch_edge_log2[grid]
                                                          : 5;
    const int nba = rv::brick_axis(grid, edge_log2);
    const int nb = nba * nba * nba;
    const int64_t nq = (int64_t)B * nb;
    // slack per queue: smaller bricks, more queues per instance, less slack each
    const uint64_t slack = (uint64_t)std::min(256, std::max(64, 2048 / nb));

    // The staging buffers are reused: nothing of an earlier call may still read them.
    RV_HIP(h, hipStreamSynchronize(s), "sync before batch plan");
    if (h->table_J != J) {
        fill_table(h->h_table, J);
        RV_HIP(h, hipMemcpyAsync(h->d_table, h->h_table, (size_t)J * sizeof(float2),
                                 hipMemcpyHostToDevice, s),
               "table upload");
        h->table_J = J;
    }
    // Host plan: work units of up to kUnitSize correspondences, and queue
    // capacities from each instance's expected runs (overflowing runs go to
    // the instance's overflow grid, so the plan bounds speed, not results).
    const double share = kBatchCapFactor * (double)runs_per_circle(grid, J) / (double)nb;
    uint32_t* cap = h->h_bplan;
    uint32_t* qbase = h->h_bplan + nq;
    uint64_t total = 0;
    int64_t nunits = 0;
    for (int32_t b = 0; b < B; ++b) {
        const int64_t lo = offsets[b], hi = offsets[b + 1];
        for (int64_t f = lo; f < hi; f += rv::kUnitSize)
            h->h_units[nunits++] = rv::Unit{b, (int32_t)std::min<int64_t>(rv::kUnitSize, hi - f), f};
        const uint64_t c = hi > lo ? (((uint64_t)std::ceil(share * (double)(hi - lo)) + slack + 63u) & ~63ull)
                                   : 0u;
        for (int k = 0; k < nb; ++k)
            cap[(int64_t)b * nb + k] = (uint32_t)std::min<uint64_t>(c, 0x7FFFFFC0u);
        total += c * (uint64_t)nb;
    }
    if (total > h->bin.pool_runs) {  // cannot happen within max_n; keep every queue inside the pool
        const double f = (double)h->bin.pool_runs / (double)total;
        for (int64_t k = 0; k < nq; ++k)
            cap[k] = (uint32_t)((uint64_t)((double)cap[k] * f) & ~63ull);
    }
    uint64_t at = 0;
    for (int64_t k = 0; k < nq; ++k) {
        qbase[k] = (uint32_t)at;
        at += cap[k];
    }
    for (int32_t b = 0; b <= B; ++b)
        h->h_offsets[b] = offsets[b];

    const bool tm = h->timing;
    h->batched = true;
    h->last_batch_edge = 1 << edge_log2;
    h->last_B = B;
    h->last_bgrid = grid;
    h->last_J = J;
    h->last_strategy = RV_VOTE_BRICK;
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[0], s), "event");
    if (nunits > 0)
        RV_HIP(h, hipMemcpyAsync(h->d_units, h->h_units, (size_t)nunits * sizeof(rv::Unit),
                                 hipMemcpyHostToDevice, s),
               "unit upload");
    RV_HIP(h, hipMemcpyAsync(h->d_bplan, h->h_bplan, (size_t)(2 * nq) * sizeof(uint32_t),
                             hipMemcpyHostToDevice, s),
           "plan upload");
    RV_HIP(h, hipMemcpyAsync(h->d_offsets, h->h_offsets, (size_t)(B + 1) * sizeof(int64_t),
                             hipMemcpyHostToDevice, s),
           "offsets upload");
    RV_HIP(h, rv::launch_fill((int32_t*)h->d_bfill, nq, 0, s), "clear queue fills");
    RV_HIP(h, rv::launch_fill((int32_t*)h->d_bflags, nq, 0, s), "clear overflow flags");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[1], s), "event");

    rv::BinArgs a = h->bin;
    a.fill = h->d_bfill;
    a.qbase = h->d_bplan + nq;
    a.cap = h->d_bplan;
    a.flags = h->d_bflags;
    a.ovf = h->d_bovf;
    a.units = h->d_units;
    a.nsets = 1;
    a.qstride = (int32_t)nq;
    a.batch = B;
    RV_HIP(h, rv::launch_bin_vote_batch(x, y, n, grid, J, edge_log2, h->d_table, a, (int)nunits, s),
           "batch vote");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[2], s), "event");
    RV_HIP(h, rv::launch_brick_accum(grid, h->K, edge_log2, h->batch_grids ? h->d_bgrids : nullptr,
                                     h->d_bpartial, a, s),
           "batch brick accumulate");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[3], s), "event");
    const rv::Candidates c{h->d_bcand_q, h->d_bcand_votes, h->d_bcand_idx, h->d_bcand_inl, h->d_bresult};
    RV_HIP(h, rv::launch_batch_finish(x, y, n, T2, B, nb, h->K, grid, h->d_bpartial, h->d_units,
                                      (int)nunits, h->d_offsets, c, inlier_mask, s,
                                      tm ? h->ev[4] : nullptr, tm ? h->ev[5] : nullptr),
           "batch top-K, rescore and mask");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[6], s), "event");
    RV_HIP(h, hipMemcpyAsync(h->h_bresult, h->d_bresult, (size_t)B * sizeof(rv::Result),
                             hipMemcpyDeviceToHost, s),
           "result readback");
    RV_HIP(h, hipStreamSynchronize(s), "sync");
    h->events_recorded = tm;
    for (int32_t b = 0; b < B; ++b) {
        const rv::Result& r = h->h_bresult[b];
        std::memcpy(q_out + 4 * (int64_t)b, r.q, sizeof(r.q));
        inlier_count[b] = r.count;
    }
    return RV_OK;
}

RV_API rv_status rot_vote_tune_batch(rv_handle* h, const float* x, const float* y,
                                     const int64_t* offsets, int32_t B, int32_t grid, float eps_rad,
                                     int32_t reps, uint8_t* mask_scratch, int32_t* edge_out,
                                     float ms_out[2])
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (reps < 1 || reps > 1000)
        return fail(h, RV_EINVAL, "rot_vote_tune_batch: reps outside 1..1000");
    if (B < 1 || B > h->max_batch)
        return fail(h, RV_EINVAL, "rot_vote_tune_batch: B outside 1..max_batch");
    if (h->cfg.batch_brick_edge != 0)
        return fail(h, RV_EINVAL, "rot_vote_tune_batch: the config fixes batch_brick_edge");
    if (grid < 1 || grid > h->batch_grid)
        return fail(h, RV_EINVAL, "rot_vote_tune_batch: grid outside 1..min(max_grid, 64)");
    std::vector<float> q(4 * (size_t)B);
    std::vector<int64_t> cnt(B);
    const int edges[2] = {5, 4};
    float ms[2] = {-1.0f, -1.0f};
    const int8_t saved = h->batch_edge_log2[grid];
    for (int c = 0; c < 2; ++c) {
        h->batch_edge_log2[grid] = (int8_t)edges[c];
        rv_status st = rot_vote_solve_batch(h, x, y, offsets, B, grid, eps_rad, q.data(), cnt.data(),
                                            mask_scratch);  // warm-up (and argument checks)
        const auto t0 = std::chrono::steady_clock::now();
        for (int r = 0; st == RV_OK && r < reps; ++r)
            st = rot_vote_solve_batch(h, x, y, offsets, B, grid, eps_rad, q.data(), cnt.data(),
                                      mask_scratch);
        const auto t1 = std::chrono::steady_clock::now();
        if (st != RV_OK) {
            h->batch_edge_log2[grid] = saved;
            return st;
        }
        ms[c] = (float)(std::chrono::duration<double, std::milli>(t1 - t0).count() / reps);
    }
    const int best = ms[1] < ms[0] ? 4 : 5;
    h->batch_edge_log2[grid] = (int8_t)best;
    if (edge_out)
        *edge_out = 1 << best;
    if (ms_out) {
        ms_out[0] = ms[0];
        ms_out[1] = ms[1];
    }
    return RV_OK;
}

RV_API rv_status rot_vote_get_batch_histogram(rv_handle* h, int32_t b, int32_t* dst_device)
{
    if (!h)
        return RV_EINVAL;
    if (!h->batched)
        return fail(h, RV_EINVAL, "rot_vote_get_batch_histogram: no batch yet");
    if (!h->batch_grids)
        return fail(h, RV_EINVAL, "rot_vote_get_batch_histogram: create with RV_FLAG_BATCH_GRIDS");
    if (b < 0 || b >= h->last_B)
        return fail(h, RV_EINVAL, "rot_vote_get_batch_histogram: b outside the last batch");
    if (!dst_device || !is_device_memory(dst_device))
        return fail(h, RV_EINVAL, "rot_vote_get_batch_histogram: dst must be device memory");
    const int64_t g = h->last_bgrid;
    const size_t cells = (size_t)(g * g * g);
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    RV_HIP(h, hipMemcpyAsync(dst_device, h->d_bgrids + (size_t)b * cells, cells * sizeof(int32_t),
                             hipMemcpyDeviceToDevice, h->stream),
           "histogram copy");
    RV_HIP(h, hipStreamSynchronize(h->stream), "sync");
    return RV_OK;
}

RV_API rv_status rot_vote_get_batch_topk(rv_handle* h, int32_t b, int32_t* n_cand, int32_t* votes,
                                         int32_t* cell_idx, int64_t* inliers, int32_t* winner)
{
    if (!h)
        return RV_EINVAL;
    if (!h->batched)
        return fail(h, RV_EINVAL, "rot_vote_get_batch_topk: no batch yet");
    if (b < 0 || b >= h->last_B)
        return fail(h, RV_EINVAL, "rot_vote_get_batch_topk: b outside the last batch");
    if (!n_cand || !votes || !cell_idx || !inliers || !winner)
        return fail(h, RV_EINVAL, "rot_vote_get_batch_topk: NULL argument");
    const rv::Result& r = h->h_bresult[b];
    const int m = r.n_cand;
    if (m > 0) {
        int32_t v[64], ix[64];
        uint32_t in[64];
        const size_t o = (size_t)b * 64;
        RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
        RV_HIP(h, hipMemcpy(v, h->d_bcand_votes + o, m * sizeof(int32_t), hipMemcpyDeviceToHost), "copy");
        RV_HIP(h, hipMemcpy(ix, h->d_bcand_idx + o, m * sizeof(int32_t), hipMemcpyDeviceToHost), "copy");
        RV_HIP(h, hipMemcpy(in, h->d_bcand_inl + o, m * sizeof(uint32_t), hipMemcpyDeviceToHost), "copy");
        for (int k = 0; k < m; ++k) {
            votes[k] = v[k];
            cell_idx[k] = ix[k];
            inliers[k] = in[k];
        }
    }
    *n_cand = m;
    *winner = r.winner;
    return RV_OK;
}

RV_API rv_status rot_vote_get_histogram(rv_handle* h, int32_t* dst_device)
{
    if (!h)
        return RV_EINVAL;
    if (!h->solved)
        return fail(h, RV_EINVAL, "rot_vote_get_histogram: no solve yet");
    if (!dst_device || !is_device_memory(dst_device))
        return fail(h, RV_EINVAL, "rot_vote_get_histogram: dst must be device memory");
    const size_t bytes = (size_t)h->last_grid * h->last_grid * h->last_grid * sizeof(int32_t);
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    RV_HIP(h, hipMemcpyAsync(dst_device, h->d_hist, bytes, hipMemcpyDeviceToDevice, h->stream),
           "histogram copy");
    RV_HIP(h, hipStreamSynchronize(h->stream), "sync");
    return RV_OK;
}

RV_API rv_status rot_vote_get_topk(rv_handle* h, int32_t* n_cand, int32_t* votes, int32_t* cell_idx,
                                   int64_t* inliers, int32_t* winner)
{
    if (!h)
        return RV_EINVAL;
    if (!h->solved)
        return fail(h, RV_EINVAL, "rot_vote_get_topk: no solve yet");
    if (!n_cand || !votes || !cell_idx || !inliers || !winner)
        return fail(h, RV_EINVAL, "rot_vote_get_topk: NULL argument");
    if (h->last_async) {
        RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
        RV_HIP(h, hipMemcpyAsync(h->h_result, h->d_result, sizeof(rv::Result),
                                 hipMemcpyDeviceToHost, h->stream),
               "result readback");
        RV_HIP(h, hipStreamSynchronize(h->stream), "sync");
        h->last_ncand = h->h_result->n_cand;
        h->last_winner = h->h_result->winner;
        h->last_count = h->h_result->count;
        h->last_async = false;
    }
    const int m = h->last_ncand;
    if (m > 0) {
        int32_t v[64], ix[64];
        uint32_t in[64];
        RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
        RV_HIP(h, hipMemcpy(v, h->d_cand_votes, m * sizeof(int32_t), hipMemcpyDeviceToHost), "copy");
        RV_HIP(h, hipMemcpy(ix, h->d_cand_idx, m * sizeof(int32_t), hipMemcpyDeviceToHost), "copy");
        RV_HIP(h, hipMemcpy(in, h->d_cand_inl, m * sizeof(uint32_t), hipMemcpyDeviceToHost), "copy");
        for (int k = 0; k < m; ++k) {
            votes[k] = v[k];
            cell_idx[k] = ix[k];
            inliers[k] = in[k];
        }
    }
    *n_cand = m;
    *winner = h->last_winner;
    return RV_OK;
}

RV_API rv_status rot_vote_get_footprint(const rv_handle* h, int64_t* device_bytes)
{
    if (!h || !device_bytes)
        return RV_EINVAL;
    *device_bytes = h->device_bytes;
    return RV_OK;
}

RV_API rv_status rot_vote_get_plan(rv_handle* h, int32_t* samples_per_circle, int32_t* vote_strategy)
{
    if (!h)
        return RV_EINVAL;
    if (!h->solved)
        return fail(h, RV_EINVAL, "rot_vote_get_plan: no solve yet");
    if (!samples_per_circle || !vote_strategy)
        return fail(h, RV_EINVAL, "rot_vote_get_plan: NULL argument");
    *samples_per_circle = h->last_J;
    *vote_strategy = h->last_strategy;
    return RV_OK;
}

RV_API rv_status rot_vote_get_timings(rv_handle* h, float* ms)
{
    if (!h)
        return RV_EINVAL;
    if (!ms)
        return fail(h, RV_EINVAL, "rot_vote_get_timings: NULL argument");
    if (!h->timing || !h->events_recorded)
        return fail(h, RV_EINVAL, "rot_vote_get_timings: no timed solve (create with RV_FLAG_TIMING)");
    // stages: prepare, vote, reduce, top-K, rescore, mask (an asynchronous
    // solve may still be running)
    RV_HIP(h, hipEventSynchronize(h->ev[kStages]), "hipEventSynchronize");
    for (int k = 0; k < kStages; ++k)
        RV_HIP(h, hipEventElapsedTime(&ms[k], h->ev[k], h->ev[k + 1]), "hipEventElapsedTime");
    return RV_OK;
}
