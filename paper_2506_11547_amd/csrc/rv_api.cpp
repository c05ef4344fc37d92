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
// At and below this many samples per grid step (J <= kKeysMaxRatio * G) the
// automatic choice among the binned strategies takes keys: the circle then
// crosses a new cell at nearly every sample, so run merging saves nothing.
constexpr int kKeysMaxRatio = 2;
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
    int64_t* d_offsets = nullptr;       // max_batch + 1
    int64_t* h_offsets = nullptr;       // pinned staging
    rv::InstPlan* d_iplan = nullptr;    // max_batch
    int32_t* d_bcounts = nullptr;       // the plan's counts (8)
    rv::Unit* d_units_all = nullptr;    // max_units
    // per brick-size class (0: 16^3 bricks, 1: 32^3)
    int32_t cls_nb[2] = {0, 0};         // largest bricks per instance of the class
    rv::Unit* d_cunits[2] = {};         // max_units each
    int32_t* d_inst_of[2] = {};         // max_batch each
    uint32_t* d_cq[2] = {};             // cap | qbase | fill | flags, 4 * max_batch * cls_nb
    uint64_t* d_cpartial[2] = {};       // max_batch * cls_nb * 64
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
    hipEvent_t ev_switch = nullptr;      // orders a stream change (rot_vote_set_stream)
    bool timing = false;
    bool keep_hist = false;             // RV_FLAG_KEEP_HISTOGRAM: brick solves write the grid
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
    bool last_batch_async = false;      // h_bresult is read back on demand
    int32_t last_bgrid = 0;

    int64_t device_bytes = 0;           // sum of the handle's device allocations
    // A server lane: the grid and the run pool are not the handle's but bound
    // per solve from the server's arena (rv::lane_bind); never freed here.
    bool lane = false;
    int8_t tuned[RV_MAX_GRID + 1] = {};  // per grid: strategy chosen by rot_vote_tune (0: none)
    // per grid and instance-size bucket: brick edge (log2) of a batch's
    // instances, set by rot_vote_tune_batch, rot_vote_set_batch_schedule or a
    // loaded tuning file (0: not set)
    int8_t sched[RV_MAX_BATCH_GRID + 1][rv::kBatchBuckets] = {};
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
    if (!h->lane)
        (void)hipFree(h->d_hist);
    (void)hipFree(h->d_table);
    (void)hipFree(h->d_partial);
    (void)hipFree(h->d_cand_q);
    (void)hipFree(h->d_cand_votes);
    (void)hipFree(h->d_cand_idx);
    (void)hipFree(h->d_cand_inl);
    (void)hipFree(h->d_result);
    (void)hipFree(h->d_empty);
    if (!h->lane)
        (void)hipFree(h->bin.pool);
    (void)hipFree(h->bin.fill);
    (void)hipFree(h->bin.qbase);
    (void)hipFree(h->bin.cap);
    (void)hipFree(h->bin.est);
    (void)hipFree(h->bin.flags);
    (void)hipFree(h->bin.order);
    (void)hipFree(h->d_ovf);
    (void)hipFree(h->d_offsets);
    (void)hipFree(h->d_iplan);
    (void)hipFree(h->d_bcounts);
    (void)hipFree(h->d_units_all);
    for (int c = 0; c < 2; ++c) {
        (void)hipFree(h->d_cunits[c]);
        (void)hipFree(h->d_inst_of[c]);
        (void)hipFree(h->d_cq[c]);
        (void)hipFree(h->d_cpartial[c]);
    }
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
    (void)hipHostFree(h->h_offsets);
    (void)hipHostFree(h->h_bresult);
    (void)hipHostFree(h->h_result);
    (void)hipHostFree(h->h_table);
    for (auto& e : h->ev)
        if (e)
            (void)hipEventDestroy(e);
    if (h->ev_switch)
        (void)hipEventDestroy(h->ev_switch);
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

namespace {

rv_status create_impl(rv_handle** out, const rv_config* cfg, bool lane)
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
    if (cfg->vote_strategy < RV_VOTE_AUTO || cfg->vote_strategy > RV_VOTE_KEYS)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: unknown vote_strategy");
    if (cfg->flags & ~(uint32_t)(RV_FLAG_TIMING | RV_FLAG_BATCH_GRIDS | RV_FLAG_KEEP_HISTOGRAM))
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
    h->lane = lane;
    h->device = cfg->device;
    h->stream = static_cast<hipStream_t>(cfg->stream);
    h->max_n = cfg->max_n;
    h->max_grid = cfg->max_grid;
    h->K = cfg->topk;
    h->max_J = cfg->samples_per_circle > 0 ? cfg->samples_per_circle : 8 * cfg->max_grid;
    h->timing = (cfg->flags & RV_FLAG_TIMING) != 0;
    h->keep_hist = (cfg->flags & RV_FLAG_KEEP_HISTOGRAM) != 0;

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
    if (!lane && (e = dev_alloc(h, &h->d_hist, ncell * sizeof(int32_t))) != hipSuccess)
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
    if ((e = hipEventCreateWithFlags(&h->ev_switch, hipEventDisableTiming)) != hipSuccess)
        return bail(e, "events");
    if ((e = dev_alloc(h, &h->d_rstate, sizeof(rv::RefineState))) != hipSuccess ||
        (e = dev_alloc(h, &h->d_rpartial,
                       (size_t)rv::kRefineMaxBlocks * rv::kRefineSums * sizeof(double))) != hipSuccess)
        return bail(e, "refinement scratch");
    if ((e = hipHostMalloc(&h->h_rstate, sizeof(rv::RefineState), hipHostMallocDefault)) != hipSuccess)
        return bail(e, "pinned refinement state");
    if ((e = dev_alloc(h, &h->d_mbits,
                       (size_t)std::max<int64_t>(1, lane ? 1 : h->max_n) * sizeof(uint64_t))) !=
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
        // One solve: about 1.7 G runs per circle are expected at J = 8 G, and
        // up to J (every sample, the key strategy) when J is small; room for
        // 1.25 x min(J, 3 G) per circle, since the plan asks for 1.15 x its
        // estimate (a pool without that margin scales every queue down, and a
        // few percent of the entries then take the overflow atomics), plus the
        // per-queue slack.
        const uint64_t per_circle = (uint64_t)std::ceil(
            1.25 * (double)std::min<int64_t>(h->max_J, 3 * (int64_t)h->max_grid));
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
    if (lane)
        runs = 0;  // bound per solve
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
        const int64_t bg = h->batch_grid;
        const size_t gcells = (size_t)B * (size_t)(bg * bg * bg);
        h->max_units = (h->max_n + rv::kUnitSize - 1) / rv::kUnitSize + B;
        for (int c = 0; c < 2; ++c) {
            const int nba = rv::brick_axis((int)bg, c == 0 ? 4 : 5);
            h->cls_nb[c] = nba * nba * nba;
            const size_t q = (size_t)B * h->cls_nb[c];
            if ((e = dev_alloc(h, &h->d_cunits[c], (size_t)h->max_units * sizeof(rv::Unit))) !=
                    hipSuccess ||
                (e = dev_alloc(h, &h->d_inst_of[c], (size_t)B * sizeof(int32_t))) != hipSuccess ||
                (e = dev_alloc(h, &h->d_cq[c], 4 * q * sizeof(uint32_t))) != hipSuccess ||
                (e = dev_alloc(h, &h->d_cpartial[c], q * 64 * sizeof(uint64_t))) != hipSuccess)
                return bail(e, "batch class scratch");
        }
        if ((e = dev_alloc(h, &h->d_units_all, (size_t)h->max_units * sizeof(rv::Unit))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_offsets, (size_t)(B + 1) * sizeof(int64_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_iplan, (size_t)B * sizeof(rv::InstPlan))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bcounts, 8 * sizeof(int32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bcand_q, (size_t)B * 64 * sizeof(float4))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bcand_votes, (size_t)B * 64 * sizeof(int32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bcand_idx, (size_t)B * 64 * sizeof(int32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bcand_inl, (size_t)B * 64 * sizeof(uint32_t))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bresult, (size_t)B * sizeof(rv::Result))) != hipSuccess ||
            (e = dev_alloc(h, &h->d_bovf, gcells * sizeof(int32_t))) != hipSuccess)
            return bail(e, "batch scratch");
        if (h->batch_grids && (e = dev_alloc(h, &h->d_bgrids, gcells * sizeof(int32_t))) != hipSuccess)
            return bail(e, "batch grids");
        if ((e = hipHostMalloc(&h->h_offsets, (size_t)(B + 1) * sizeof(int64_t),
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

// The vote strategy a solve at this grid uses.
int pick_strategy(const rv_handle* h, int grid)
{
    int strategy = h->forced_strategy ? h->forced_strategy : h->cfg.vote_strategy;
    if (strategy == RV_VOTE_AUTO && h->tuned[grid] != 0)
        strategy = h->tuned[grid];  // measured by rot_vote_tune
    if (strategy == RV_VOTE_AUTO) {
        const int J = h->cfg.samples_per_circle > 0 ? h->cfg.samples_per_circle : 8 * grid;
        strategy = !(h->brick_ok && grid >= kBrickMinGrid && grid <= rv::kMaxBrickGrid)
                       ? RV_VOTE_GLOBAL
                       : (J <= kKeysMaxRatio * grid ? RV_VOTE_KEYS : RV_VOTE_BRICK);
    }
    return strategy;
}

int64_t align256(int64_t b) { return (b + 255) & ~(int64_t)255; }

// Brick edge (log2) of a batch instance in size bucket k at this grid: fixed
// by the config, else the schedule (tuned, set or loaded), else 32.
int batch_edge_log2(const rv_handle* h, int grid, int k)
{
    return h->cfg.batch_brick_edge == 16   ? 4
           : h->cfg.batch_brick_edge == 32 ? 5
           : h->sched[grid][k]             ? h->sched[grid][k]
                                           : 5;
}

}  // namespace

RV_API rv_status rot_vote_create(rv_handle** out, const rv_config* cfg)
{
    return create_impl(out, cfg, false);
}

rv_status rv::create_lane(rv_handle** out, const rv_config* cfg)
{
    if (cfg && cfg->max_pairs != 0)
        return fail(nullptr, RV_EINVAL, "server lane: no pair buffers");
    if (cfg && (cfg->flags & RV_FLAG_BATCH_GRIDS))
        return fail(nullptr, RV_EINVAL, "server lane: no kept batch grids");
    return create_impl(out, cfg, true);
}

int64_t rv::lane_solve_bytes(const rv_handle* h, int64_t n, int32_t grid)
{
    if (grid < 1 || grid > h->max_grid || n < 0)
        return -1;
    const int64_t G = grid;
    const int64_t gbytes = align256(G * G * G * (int64_t)sizeof(int32_t));
    const int strategy = pick_strategy(h, grid);
    if (n == 0 || strategy == RV_VOTE_GLOBAL)
        return gbytes;
    const int J = h->cfg.samples_per_circle > 0 ? h->cfg.samples_per_circle : 8 * grid;
    const bool keys = strategy == RV_VOTE_KEYS;
    const int nba = rv::brick_axis(grid, keys ? 5 : rv::solve_edge_log2(grid));
    const int64_t nb = (int64_t)nba * nba * nba;
    // the plan asks for 1.15 x the estimated runs (keys: samples) plus 256..319
    // per queue
    const int64_t per_circle =
        (int64_t)std::ceil(1.25 * (double)(keys ? J : runs_per_circle(grid, J)));
    const int64_t runs = std::min<int64_t>(n * per_circle + rv::kQueueSets * nb * 320,
                                           (int64_t)0xFFFFFFFFll - 64);
    return gbytes + align256(runs * (int64_t)sizeof(uint32_t));
}

int64_t rv::lane_batch_bytes(const rv_handle* h, int64_t cols, int32_t B, int32_t grid)
{
    if (grid < 1 || grid > h->batch_grid || B < 1 || B > h->max_batch || cols < 0)
        return -1;
    const int J = h->cfg.samples_per_circle > 0 ? h->cfg.samples_per_circle : 8 * grid;
    // the batch plan: ceil(share * n_b) + slack, rounded up to 64, per (instance,
    // brick), with the more queues of the two brick sizes
    const int nba = rv::brick_axis(grid, 4);
    const int64_t nb = (int64_t)nba * nba * nba;
    const int64_t runs = std::min<int64_t>(
        (int64_t)std::ceil(kBatchCapFactor * (double)runs_per_circle(grid, J) * (double)cols) +
            (int64_t)B * nb * (256 + 64 + 1),
        (int64_t)0xFFFFFFFFll - 64);
    return align256(runs * (int64_t)sizeof(uint32_t));
}

void rv::lane_bind(rv_handle* h, int32_t* grid, uint32_t* pool, uint64_t pool_runs)
{
    h->d_hist = grid;
    h->bin.pool = pool;
    h->bin.pool_runs = std::min<uint64_t>(pool_runs, 0xFFFFFFFFull - 64);
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
    h->err.clear();
    hipStream_t next = static_cast<hipStream_t>(stream);
    if (next != h->stream) {
        // the handle's scratch may still be in use by work on the old stream
        RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
        RV_HIP(h, hipEventRecord(h->ev_switch, h->stream), "event on the old stream");
        RV_HIP(h, hipStreamWaitEvent(next, h->ev_switch, 0), "wait on the new stream");
        h->stream = next;
    }
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
    const int strategy = pick_strategy(h, grid);
    if (strategy != RV_VOTE_GLOBAL && !(h->brick_ok && grid <= rv::kMaxBrickGrid))
        return fail(h, RV_EUNSUPPORTED,
                    f + ": the brick and key strategies need grid <= 384 and a handle created "
                        "for them");

    if (h->table_J != J) {
        RV_HIP(h, hipStreamSynchronize(s), "sync before table upload");
        fill_table(h->h_table, J);
        RV_HIP(h, hipMemcpyAsync(h->d_table, h->h_table, (size_t)J * sizeof(float2),
                                 hipMemcpyHostToDevice, s),
               "table upload");
        h->table_J = J;
    }

    const bool tm = h->timing;
    const bool keys = strategy == RV_VOTE_KEYS;
    const bool brick = strategy == RV_VOTE_BRICK || keys;
    h->solved = true;
    h->last_async = false;
    h->last_grid = grid;
    h->last_J = J;
    h->last_strategy = strategy;
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[0], s), "event");
    const int edge = keys ? 5 : rv::solve_edge_log2(grid);
    if (brick)
        RV_HIP(h, rv::launch_bin_prepare(x, y, n, grid, J, edge, h->d_table, h->bin, s, keys),
               "brick plan");
    else
        RV_HIP(h, rv::launch_fill(h->d_hist, ncell, 0, s), "clear grid");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[1], s), "event");
    if (keys)
        RV_HIP(h, rv::launch_key_vote(x, y, n, grid, J, h->d_table, h->bin, s), "key vote");
    else if (brick)
        RV_HIP(h, rv::launch_bin_vote(x, y, n, grid, J, edge, h->d_table, h->bin, s),
               "binned vote");
    else
        RV_HIP(h, rv::launch_vote_global(x, y, n, grid, J, h->d_table, h->d_hist, 0, s), "vote");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[2], s), "event");
    int nlists;
    if (brick) {
        // the whole grid only for the histogram hook: the top-K needs the
        // bricks' lists alone
        const rv::QueueFormat fmt = keys ? rv::QueueFormat::kKeys
                                    : grid <= rv::kNarrowGrid ? rv::QueueFormat::kNarrow
                                                              : rv::QueueFormat::kWide;
        RV_HIP(h, rv::launch_brick_accum(grid, h->K, edge, fmt, h->keep_hist ? h->d_hist : nullptr,
                                         h->d_partial, h->bin, s),
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
    // the mask kernel also writes the result record into the pinned host copy
    RV_HIP(h, rv::launch_mask(x, y, n, T2, c, inlier_mask, s, h->h_result), "mask");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[6], s), "event");
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
                               int32_t* strategy_out, float ms_out[3])
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
    const int cand[3] = {RV_VOTE_GLOBAL, RV_VOTE_BRICK, RV_VOTE_KEYS};
    float ms[3] = {-1.0f, -1.0f, -1.0f};
    float q[4];
    int64_t cnt = 0;
    for (int c = 0; c < 3; ++c) {
        if (cand[c] != RV_VOTE_GLOBAL && !brick_ok)
            continue;
        // keys write every sample; beyond J = 2 kKeysMaxRatio G the circle
        // stays in a cell for several samples and keys cannot win (they then
        // outnumber the run pool's room), so they are not timed
        if (cand[c] == RV_VOTE_KEYS && J > 2 * kKeysMaxRatio * grid)
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
    int best = RV_VOTE_GLOBAL;
    for (int c = 1; c < 3; ++c)
        if (ms[c] >= 0.0f && ms[c] < ms[best - 1])
            best = cand[c];
    h->tuned[grid] = (int8_t)best;
    if (strategy_out)
        *strategy_out = best;
    if (ms_out)
        std::memcpy(ms_out, ms, sizeof(ms));
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

namespace {

// Argument checks shared by the batch entry points (offsets are checked by
// the caller where they live on the host).
rv_status check_batch(rv_handle* h, const char* fn, int32_t B, int32_t grid, float eps_rad,
                      int32_t* J)
{
    const std::string f(fn);
    if (h->max_batch == 0)
        return fail(h, RV_EUNSUPPORTED, f + ": handle created with max_batch = 0");
    if (B < 0 || B > h->max_batch)
        return fail(h, RV_EINVAL, f + ": B outside 0..max_batch");
    if (grid < 1 || grid > h->batch_grid)
        return fail(h, RV_EINVAL, f + ": grid outside 1..min(max_grid, 64)");
    if (!(eps_rad > 0.0f) || !(eps_rad <= (float)M_PI))
        return fail(h, RV_EINVAL, f + ": eps_rad outside (0, pi]");
    *J = h->cfg.samples_per_circle > 0 ? h->cfg.samples_per_circle : 8 * grid;
    if (*J > h->max_J)
        return fail(h, RV_EINVAL, f + ": J = 8*grid exceeds the table sized at create");
    return RV_OK;
}

// The whole batch on the handle's stream, from offsets in device memory:
// plan, then per brick-size class the binned vote and the accumulation, then
// the per-instance top-K, rescoring and masks.  Results go to `results`
// (device, B records).  No host synchronisation (except a sample-table upload
// at a new J).
rv_status enqueue_batch(rv_handle* h, const float* x, const float* y, int64_t n_cols,
                        const int64_t* d_offsets, int32_t B, int32_t grid, int32_t J, float T2,
                        rv::Result* results, uint8_t* mask, const char* fn)
{
    hipStream_t s = h->stream;
    if (h->table_J != J) {
        RV_HIP(h, hipStreamSynchronize(s), "sync before table upload");
        fill_table(h->h_table, J);
        RV_HIP(h, hipMemcpyAsync(h->d_table, h->h_table, (size_t)J * sizeof(float2),
                                 hipMemcpyHostToDevice, s),
               "table upload");
        h->table_J = J;
    }
    rv::BatchPlanArgs p{};
    p.offsets = d_offsets;
    p.B = B;
    p.J = J;
    p.n_cols = n_cols;
    bool use[2] = {false, false};
    for (int k = 0; k < rv::kBatchBuckets; ++k) {
        p.bucket_edge[k] = (int8_t)batch_edge_log2(h, grid, k);
        use[p.bucket_edge[k] == 4 ? 0 : 1] = true;
    }
    const int edge[2] = {4, 5};
    int nb[2];
    for (int c = 0; c < 2; ++c) {
        const int nba = rv::brick_axis(grid, edge[c]);
        nb[c] = nba * nba * nba;
        p.nb[c] = nb[c];
        p.share[c] = kBatchCapFactor * (double)runs_per_circle(grid, J) / (double)nb[c];
        // slack per queue: smaller bricks, more queues per instance, less slack each
        p.slack[c] = (uint32_t)std::min(256, std::max(64, 2048 / nb[c]));
        const size_t q = (size_t)h->max_batch * h->cls_nb[c];
        p.cap[c] = h->d_cq[c];
        p.qbase[c] = h->d_cq[c] + q;
        p.fill[c] = h->d_cq[c] + 2 * q;
        p.flags[c] = h->d_cq[c] + 3 * q;
        p.inst_of[c] = h->d_inst_of[c];
        p.units[c] = h->d_cunits[c];
    }
    p.pool_runs = h->bin.pool_runs;
    p.inst = h->d_iplan;
    p.counts = h->d_bcounts;
    p.units_all = h->d_units_all;
    p.results = results;

    const bool tm = h->timing;
    h->batched = true;
    h->last_B = B;
    h->last_bgrid = grid;
    h->last_J = J;
    h->last_strategy = RV_VOTE_BRICK;
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[0], s), "event");
    RV_HIP(h, rv::launch_batch_plan(p, s), (std::string(fn) + ": plan").c_str());
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[1], s), "event");
    // launched for upper bounds: sum over instances of ceil(n_b / 512) units
    const int64_t max_units = n_cols / rv::kUnitSize + B;
    rv::BinArgs a[2];
    for (int c = 0; c < 2; ++c) {
        a[c] = h->bin;
        a[c].fill = p.fill[c];
        a[c].qbase = p.qbase[c];
        a[c].cap = p.cap[c];
        a[c].flags = p.flags[c];
        a[c].ovf = h->d_bovf;
        a[c].units = h->d_cunits[c];
        a[c].counts = h->d_bcounts + 2 * c;
        a[c].inst_of = h->d_inst_of[c];
        a[c].nsets = 1;
        a[c].qstride = B * nb[c];
        a[c].batch = B;
    }
    for (int c = 1; c >= 0; --c)
        if (use[c])
            RV_HIP(h, rv::launch_bin_vote_batch(x, y, n_cols, grid, J, edge[c], h->d_table, a[c],
                                                (int)max_units, s),
                   "batch vote");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[2], s), "event");
    for (int c = 1; c >= 0; --c)
        if (use[c])
            RV_HIP(h, rv::launch_brick_accum(grid, h->K, edge[c], rv::QueueFormat::kNarrow,
                                             h->batch_grids ? h->d_bgrids : nullptr,
                                             h->d_cpartial[c], a[c], s),
                   "batch brick accumulate");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[3], s), "event");
    const rv::Candidates cand{h->d_bcand_q, h->d_bcand_votes, h->d_bcand_idx, h->d_bcand_inl,
                              results};
    for (int c = 1; c >= 0; --c)
        if (use[c])
            RV_HIP(h, rv::launch_batch_topk(h->d_cpartial[c], B, nb[c], h->K, grid,
                                            h->d_bcounts + 2 * c, h->d_inst_of[c], cand, s),
                   "batch top-K");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[4], s), "event");
    RV_HIP(h, rv::launch_batch_rescore_mask(x, y, n_cols, T2, h->d_units_all, (int)max_units,
                                            h->d_bcounts + 4, d_offsets, cand, mask, s,
                                            tm ? h->ev[5] : nullptr),
           "batch rescore and mask");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[6], s), "event");
    return RV_OK;
}

}  // namespace

RV_API rv_status rot_vote_solve_batch(rv_handle* h, const float* x, const float* y,
                                      const int64_t* offsets, int32_t B, int32_t grid,
                                      float eps_rad, float* q_out, int64_t* inlier_count,
                                      uint8_t* inlier_mask)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    int32_t J = 0;
    if (rv_status st = check_batch(h, "rot_vote_solve_batch", B, grid, eps_rad, &J))
        return st;
    if (B == 0)
        return RV_OK;
    if (!offsets || !q_out || !inlier_count)
        return fail(h, RV_EINVAL, "rot_vote_solve_batch: offsets, q_out and inlier_count must not be NULL");
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
    // the pinned staging of the offsets is reused: nothing earlier may still read it
    RV_HIP(h, hipStreamSynchronize(s), "sync before batch");
    std::memcpy(h->h_offsets, offsets, (size_t)(B + 1) * sizeof(int64_t));
    RV_HIP(h, hipMemcpyAsync(h->d_offsets, h->h_offsets, (size_t)(B + 1) * sizeof(int64_t),
                             hipMemcpyHostToDevice, s),
           "offsets upload");
    if (rv_status st = enqueue_batch(h, x, y, n, h->d_offsets, B, grid, J, residual_bound(eps_rad),
                                     h->d_bresult, inlier_mask, "rot_vote_solve_batch"))
        return st;
    RV_HIP(h, hipMemcpyAsync(h->h_bresult, h->d_bresult, (size_t)B * sizeof(rv::Result),
                             hipMemcpyDeviceToHost, s),
           "result readback");
    RV_HIP(h, hipStreamSynchronize(s), "sync");
    h->events_recorded = h->timing;
    h->last_batch_async = false;
    for (int32_t b = 0; b < B; ++b) {
        const rv::Result& r = h->h_bresult[b];
        std::memcpy(q_out + 4 * (int64_t)b, r.q, sizeof(r.q));
        inlier_count[b] = r.count;
    }
    return RV_OK;
}

RV_API rv_status rot_vote_solve_batch_async(rv_handle* h, const float* x, const float* y,
                                            int64_t n_cols, const int64_t* offsets_device,
                                            int32_t B, int32_t grid, float eps_rad,
                                            rv_result* results_device, uint8_t* inlier_mask)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    int32_t J = 0;
    if (rv_status st = check_batch(h, "rot_vote_solve_batch_async", B, grid, eps_rad, &J))
        return st;
    if (B == 0)
        return RV_OK;
    if (n_cols < 0 || n_cols > h->max_n)
        return fail(h, RV_EINVAL, "rot_vote_solve_batch_async: n_cols outside 0..max_n");
    if (!offsets_device || !is_device_memory(offsets_device) ||
        reinterpret_cast<uintptr_t>(offsets_device) % alignof(int64_t) != 0)
        return fail(h, RV_EINVAL, "rot_vote_solve_batch_async: offsets must be aligned device memory");
    if (!results_device || !is_device_memory(results_device) ||
        reinterpret_cast<uintptr_t>(results_device) % alignof(rv_result) != 0)
        return fail(h, RV_EINVAL, "rot_vote_solve_batch_async: results must be aligned device memory");
    if (n_cols > 0 && (!x || !y || !inlier_mask || !is_device_memory(x) || !is_device_memory(y) ||
                       !is_device_memory(inlier_mask)))
        return fail(h, RV_EINVAL, "rot_vote_solve_batch_async: x, y and inlier_mask must be device memory");
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    if (rv_status st = enqueue_batch(h, x, y, n_cols, offsets_device, B, grid, J,
                                     residual_bound(eps_rad), h->d_bresult, inlier_mask,
                                     "rot_vote_solve_batch_async"))
        return st;
    RV_HIP(h, hipMemcpyAsync(results_device, h->d_bresult, (size_t)B * sizeof(rv::Result),
                             hipMemcpyDeviceToDevice, h->stream),
           "result copy");
    h->events_recorded = h->timing;
    h->last_batch_async = true;
    return RV_OK;
}

RV_API rv_status rot_vote_set_batch_schedule(rv_handle* h, int32_t grid, const int32_t* edges)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (h->max_batch == 0)
        return fail(h, RV_EUNSUPPORTED, "rot_vote_set_batch_schedule: handle created with max_batch = 0");
    if (grid < 1 || grid > h->batch_grid)
        return fail(h, RV_EINVAL, "rot_vote_set_batch_schedule: grid outside 1..min(max_grid, 64)");
    if (h->cfg.batch_brick_edge != 0)
        return fail(h, RV_EINVAL, "rot_vote_set_batch_schedule: the config fixes batch_brick_edge");
    if (!edges)
        return fail(h, RV_EINVAL, "rot_vote_set_batch_schedule: NULL edges");
    for (int k = 0; k < rv::kBatchBuckets; ++k)
        if (edges[k] != 16 && edges[k] != 32)
            return fail(h, RV_EINVAL, "rot_vote_set_batch_schedule: every edge must be 16 or 32");
    for (int k = 0; k < rv::kBatchBuckets; ++k)
        h->sched[grid][k] = (int8_t)(edges[k] == 16 ? 4 : 5);
    return RV_OK;
}

RV_API rv_status rot_vote_get_batch_schedule(rv_handle* h, int32_t grid, int32_t* edges)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (grid < 1 || grid > RV_MAX_BATCH_GRID || !edges)
        return fail(h, RV_EINVAL, "rot_vote_get_batch_schedule: grid outside 1..64 or NULL edges");
    for (int k = 0; k < rv::kBatchBuckets; ++k)
        edges[k] = 1 << batch_edge_log2(h, grid, k);
    return RV_OK;
}

RV_API rv_status rot_vote_tune_batch(rv_handle* h, const float* x, const float* y,
                                     const int64_t* offsets, int32_t B, int32_t grid, float eps_rad,
                                     int32_t reps, uint8_t* mask_scratch, int32_t* edges_out,
                                     float* ms_out)
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
    int8_t saved[rv::kBatchBuckets];
    std::memcpy(saved, h->sched[grid], sizeof(saved));
    auto timed = [&](float* ms) -> rv_status {
        rv_status st = rot_vote_solve_batch(h, x, y, offsets, B, grid, eps_rad, q.data(), cnt.data(),
                                            mask_scratch);  // warm-up (and argument checks)
        const auto t0 = std::chrono::steady_clock::now();
        for (int r = 0; st == RV_OK && r < reps; ++r)
            st = rot_vote_solve_batch(h, x, y, offsets, B, grid, eps_rad, q.data(), cnt.data(),
                                      mask_scratch);
        const auto t1 = std::chrono::steady_clock::now();
        *ms = (float)(std::chrono::duration<double, std::milli>(t1 - t0).count() / reps);
        return st;
    };
    // coordinate descent over the size buckets: from 32^3 bricks everywhere,
    // each bucket (with instances in this batch) in turn takes 16^3 bricks if
    // that times faster; results are the same whatever the schedule
    bool present[rv::kBatchBuckets] = {};
    for (int32_t b = 0; b < B; ++b) {
        const int64_t n = offsets[b + 1] - offsets[b];
        int k = 0;
        for (int i = 0; i < rv::kBatchBuckets - 1; ++i)
            k += n >= rv::kBucketBound[i] ? 1 : 0;
        present[k] = true;
    }
    float ms[rv::kBatchBuckets + 1];
    for (auto& v : ms)
        v = -1.0f;
    for (int k = 0; k < rv::kBatchBuckets; ++k)
        h->sched[grid][k] = 5;
    if (rv_status st = timed(&ms[0])) {
        std::memcpy(h->sched[grid], saved, sizeof(saved));
        return st;
    }
    float best = ms[0];
    for (int k = 0; k < rv::kBatchBuckets; ++k) {
        if (!present[k])
            continue;
        h->sched[grid][k] = 4;
        if (rv_status st = timed(&ms[k + 1])) {
            std::memcpy(h->sched[grid], saved, sizeof(saved));
            return st;
        }
        if (ms[k + 1] < best)
            best = ms[k + 1];
        else
            h->sched[grid][k] = 5;
    }
    if (edges_out)
        for (int k = 0; k < rv::kBatchBuckets; ++k)
            edges_out[k] = 1 << h->sched[grid][k];
    if (ms_out)
        std::memcpy(ms_out, ms, sizeof(ms));
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
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    if (h->last_batch_async) {
        RV_HIP(h, hipMemcpyAsync(h->h_bresult, h->d_bresult, (size_t)h->last_B * sizeof(rv::Result),
                                 hipMemcpyDeviceToHost, h->stream),
               "result readback");
        RV_HIP(h, hipStreamSynchronize(h->stream), "sync");
        h->last_batch_async = false;
    }
    const rv::Result& r = h->h_bresult[b];
    const int m = r.n_cand;
    if (m > 0) {
        int32_t v[64], ix[64];
        uint32_t in[64];
        const size_t o = (size_t)b * 64;
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

// ------------------------------------------------------------ tuning file
//
// The choices made by measurement (rot_vote_tune's vote strategy per grid,
// rot_vote_tune_batch's brick edge per grid and instance-size bucket) kept
// in a small JSON file, keyed by (GPU architecture, grid, J, size bucket):
//   {"format": "rotvote-tuning", "version": 1, "entries": [
//     {"arch": "gfx950", "kind": "solve", "grid": 256, "J": 2048, "n_lo": 0, "n_hi": -1,
//      "strategy": 2},
//     {"arch": "gfx950", "kind": "batch", "grid": 64, "J": 512, "n_lo": 0, "n_hi": 512,
//      "edge": 16}, ...]}
// n_hi = -1 means no upper bound.

namespace {

struct TuneEntry {
    std::string arch, kind;
    int64_t grid = 0, J = 0, n_lo = 0, n_hi = -1, value = 0;  // strategy or edge
};

std::string device_arch(int device)
{
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) != hipSuccess)
        return "unknown";
    std::string a = prop.gcnArchName;
    const size_t c = a.find(':');
    return c == std::string::npos ? a : a.substr(0, c);
}

// Parses the entries of a tuning file (objects of string and integer
// fields); false if the text is not one.
bool parse_tuning(const std::string& t, std::vector<TuneEntry>* out)
{
    if (t.find("\"rotvote-tuning\"") == std::string::npos)
        return false;
    size_t at = t.find("\"entries\"");
    if (at == std::string::npos)
        return false;
    at = t.find('[', at);
    if (at == std::string::npos)
        return false;
    for (;;) {
        const size_t open = t.find_first_of("{]", at);
        if (open == std::string::npos)
            return false;
        if (t[open] == ']')
            return true;
        const size_t close = t.find('}', open);
        if (close == std::string::npos)
            return false;
        TuneEntry e;
        size_t k = open + 1;
        while (k < close) {
            const size_t q0 = t.find('"', k);
            if (q0 == std::string::npos || q0 >= close)
                break;
            const size_t q1 = t.find('"', q0 + 1);
            const size_t colon = t.find(':', q1);
            if (q1 == std::string::npos || colon == std::string::npos || colon >= close)
                return false;
            const std::string key = t.substr(q0 + 1, q1 - q0 - 1);
            size_t v = t.find_first_not_of(" \t\r\n", colon + 1);
            if (v == std::string::npos || v >= close)
                return false;
            std::string sval;
            int64_t ival = 0;
            if (t[v] == '"') {
                const size_t v1 = t.find('"', v + 1);
                if (v1 == std::string::npos || v1 >= close)
                    return false;
                sval = t.substr(v + 1, v1 - v - 1);
                k = v1 + 1;
            } else {
                char* end = nullptr;
                ival = std::strtoll(t.c_str() + v, &end, 10);
                if (end == t.c_str() + v)
                    return false;
                k = (size_t)(end - t.c_str());
            }
            if (key == "arch") e.arch = sval;
            else if (key == "kind") e.kind = sval;
            else if (key == "grid") e.grid = ival;
            else if (key == "J") e.J = ival;
            else if (key == "n_lo") e.n_lo = ival;
            else if (key == "n_hi") e.n_hi = ival;
            else if (key == "strategy" || key == "edge") e.value = ival;
        }
        out->push_back(e);
        at = close + 1;
    }
}

bool read_file(const char* path, std::string* text)
{
    FILE* f = std::fopen(path, "rb");
    if (!f)
        return false;
    char buf[4096];
    size_t r;
    while ((r = std::fread(buf, 1, sizeof(buf), f)) > 0)
        text->append(buf, r);
    std::fclose(f);
    return true;
}

int handle_J(const rv_handle* h, int grid)
{
    return h->cfg.samples_per_circle > 0 ? h->cfg.samples_per_circle : 8 * grid;
}

}  // namespace

RV_API rv_status rot_vote_save_tuning(rv_handle* h, const char* path)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (!path)
        return fail(h, RV_EINVAL, "rot_vote_save_tuning: NULL path");
    const std::string arch = device_arch(h->device);
    std::vector<TuneEntry> mine;
    for (int g = 1; g <= h->max_grid && g <= RV_MAX_GRID; ++g)
        if (h->tuned[g])
            mine.push_back({arch, "solve", g, handle_J(h, g), 0, -1, h->tuned[g]});
    for (int g = 1; g <= RV_MAX_BATCH_GRID; ++g) {
        if (!h->sched[g][0])
            continue;
        for (int k = 0; k < rv::kBatchBuckets; ++k)
            mine.push_back({arch, "batch", g, handle_J(h, g), k ? rv::kBucketBound[k - 1] : 0,
                            k < rv::kBatchBuckets - 1 ? rv::kBucketBound[k] : -1,
                            (int64_t)1 << h->sched[g][k]});
    }
    // keep the file's other entries (other GPUs, grids, J or kinds)
    std::vector<TuneEntry> all;
    std::string text;
    if (read_file(path, &text) && !parse_tuning(text, &all))
        return fail(h, RV_EINVAL, "rot_vote_save_tuning: the file exists and is not a tuning file");
    std::vector<TuneEntry> keep;
    for (const TuneEntry& e : all) {
        bool replaced = false;
        for (const TuneEntry& m : mine)
            replaced |= e.arch == m.arch && e.kind == m.kind && e.grid == m.grid && e.J == m.J &&
                        e.n_lo == m.n_lo;
        if (!replaced)
            keep.push_back(e);
    }
    keep.insert(keep.end(), mine.begin(), mine.end());
    const std::string tmp = std::string(path) + ".tmp";
    FILE* f = std::fopen(tmp.c_str(), "wb");
    if (!f)
        return fail(h, RV_EINVAL, "rot_vote_save_tuning: cannot write " + tmp);
    std::fprintf(f, "{\"format\": \"rotvote-tuning\", \"version\": 1, \"entries\": [\n");
    for (size_t i = 0; i < keep.size(); ++i) {
        const TuneEntry& e = keep[i];
        std::fprintf(f,
                     "  {\"arch\": \"%s\", \"kind\": \"%s\", \"grid\": %lld, \"J\": %lld, "
                     "\"n_lo\": %lld, \"n_hi\": %lld, \"%s\": %lld}%s\n",
                     e.arch.c_str(), e.kind.c_str(), (long long)e.grid, (long long)e.J,
                     (long long)e.n_lo, (long long)e.n_hi, e.kind == "solve" ? "strategy" : "edge",
                     (long long)e.value, i + 1 < keep.size() ? "," : "");
    }
    std::fprintf(f, "]}\n");
    const bool ok = std::fclose(f) == 0;
    if (!ok || std::rename(tmp.c_str(), path) != 0)
        return fail(h, RV_EINVAL, std::string("rot_vote_save_tuning: cannot write ") + path);
    return RV_OK;
}

RV_API rv_status rot_vote_load_tuning(rv_handle* h, const char* path, int32_t* applied)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (!path)
        return fail(h, RV_EINVAL, "rot_vote_load_tuning: NULL path");
    std::string text;
    if (!read_file(path, &text))
        return fail(h, RV_EINVAL, std::string("rot_vote_load_tuning: cannot read ") + path);
    std::vector<TuneEntry> all;
    if (!parse_tuning(text, &all))
        return fail(h, RV_EINVAL, "rot_vote_load_tuning: not a tuning file");
    const std::string arch = device_arch(h->device);
    int32_t n = 0;
    for (const TuneEntry& e : all) {
        if (e.arch != arch || e.grid < 1 || e.grid > h->max_grid || e.J != handle_J(h, (int)e.grid))
            continue;
        if (e.kind == "solve" && (e.value == RV_VOTE_GLOBAL ||
                                  ((e.value == RV_VOTE_BRICK || e.value == RV_VOTE_KEYS) &&
                                   h->brick_ok &&
                                   e.grid <= rv::kMaxBrickGrid))) {
            h->tuned[e.grid] = (int8_t)e.value;
            ++n;
        } else if (e.kind == "batch" && e.grid <= RV_MAX_BATCH_GRID && h->max_batch > 0 &&
                   h->cfg.batch_brick_edge == 0 && (e.value == 16 || e.value == 32)) {
            for (int k = 0; k < rv::kBatchBuckets; ++k)
                if ((k ? rv::kBucketBound[k - 1] : 0) == e.n_lo) {
                    // a schedule entry sets its bucket; the others keep 32 until set
                    for (int j = 0; j < rv::kBatchBuckets; ++j)
                        if (!h->sched[e.grid][j])
                            h->sched[e.grid][j] = 5;
                    h->sched[e.grid][k] = (int8_t)(e.value == 16 ? 4 : 5);
                    ++n;
                }
        }
    }
    if (applied)
        *applied = n;
    return RV_OK;
}

RV_API rv_status rot_vote_get_histogram(rv_handle* h, int32_t* dst_device)
{
    if (!h)
        return RV_EINVAL;
    if (!h->solved)
        return fail(h, RV_EINVAL, "rot_vote_get_histogram: no solve yet");
    if (!h->keep_hist)
        return fail(h, RV_EINVAL, "rot_vote_get_histogram: create with RV_FLAG_KEEP_HISTOGRAM");
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
