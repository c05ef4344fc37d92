// C-ABI of the rotation-voting library: argument checks, scratch ownership,
// stage sequencing on one HIP stream, and the two small readbacks.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "rotvote.h"
#include "rv_internal.h"

#define RV_API extern "C" __attribute__((visibility("default")))

namespace {

constexpr int kStages = RV_NUM_STAGES;
// Below this grid the whole int32 grid (<= 1.4 MiB at 72^3) sits in every
// XCD's L2 and run-coalesced atomics straight into it beat binning.
constexpr int kBrickMinGrid = 72;

std::string g_create_error;  // reason of the last failed create (NULL handle)

}  // namespace

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
    float2* h_table = nullptr;          // pinned staging for the table
    int32_t table_J = -1;               // J the device table holds

    // brick strategy scratch (allocated when the config allows that strategy)
    bool brick_ok = false;
    rv::BinArgs bin{};
    int32_t* d_ovf = nullptr;           // max_grid^3, zero between solves

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

    std::string err;
};

namespace {

rv_status fail(rv_handle* h, rv_status st, const std::string& msg)
{
    if (h)
        h->err = msg;
    else
        g_create_error = msg;
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

bool is_device_memory(const void* p)
{
    hipPointerAttribute_t attr;
    if (hipPointerGetAttributes(&attr, p) != hipSuccess) {
        (void)hipGetLastError();  // clear the sticky "invalid value" for host pointers
        return false;
    }
    return attr.type == hipMemoryTypeDevice || attr.type == hipMemoryTypeManaged;
}

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
    (void)hipFree(h->bin.pool);
    (void)hipFree(h->bin.fill);
    (void)hipFree(h->bin.qbase);
    (void)hipFree(h->bin.cap);
    (void)hipFree(h->bin.est);
    (void)hipFree(h->bin.flags);
    (void)hipFree(h->bin.order);
    (void)hipFree(h->d_ovf);
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

// |L q|^2 = 4 sin^2(psi / 2) for the angle psi between R(q) a and b.
float residual_bound(float eps)
{
    const double s = std::sin(0.5 * (double)eps);
    return (float)(4.0 * s * s);
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
    if (cfg->flags & ~(uint32_t)RV_FLAG_TIMING)
        return fail(nullptr, RV_EINVAL, "rot_vote_create: unknown flags");
    for (int r : cfg->reserved)
        if (r != 0)
            return fail(nullptr, RV_EINVAL, "rot_vote_create: reserved fields must be 0");
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
    if ((e = hipMalloc(&h->d_hist, ncell * sizeof(int32_t))) != hipSuccess)
        return bail(e, "vote grid");
    if ((e = hipMalloc(&h->d_table, (size_t)h->max_J * sizeof(float2))) != hipSuccess)
        return bail(e, "sample table");
    if ((e = hipMalloc(&h->d_partial, (size_t)rv::kTopkMaxBlocks * 64 * sizeof(uint64_t))) !=
        hipSuccess)
        return bail(e, "top-K scratch");
    if ((e = hipMalloc(&h->d_cand_q, 64 * sizeof(float4))) != hipSuccess ||
        (e = hipMalloc(&h->d_cand_votes, 64 * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&h->d_cand_idx, 64 * sizeof(int32_t))) != hipSuccess ||
        (e = hipMalloc(&h->d_cand_inl, 64 * sizeof(uint32_t))) != hipSuccess ||
        (e = hipMalloc(&h->d_result, sizeof(rv::Result))) != hipSuccess)
        return bail(e, "candidate buffers");
    if ((e = hipHostMalloc(&h->h_result, sizeof(rv::Result), hipHostMallocDefault)) != hipSuccess)
        return bail(e, "pinned result");
    if ((e = hipHostMalloc(&h->h_table, (size_t)h->max_J * sizeof(float2), hipHostMallocDefault)) !=
        hipSuccess)
        return bail(e, "pinned table");
    for (auto& ev : h->ev)
        if ((e = hipEventCreate(&ev)) != hipSuccess)
            return bail(e, "events");
    if (cfg->vote_strategy != RV_VOTE_GLOBAL && h->max_grid <= rv::kMaxBrickGrid) {
        // Run pool: about 1.7 G runs per circle are expected at J = 8 G (at
        // most J); room for 3 G per circle plus the per-queue slack.
        const uint64_t per_circle = (uint64_t)std::min<int64_t>(h->max_J, 3 * (int64_t)h->max_grid);
        uint64_t runs = (uint64_t)h->max_n * per_circle +
                        (uint64_t)rv::kQueueSets * rv::kMaxBricks * 320u;
        runs = std::min<uint64_t>(runs, 0xFFFFFFFFull - 64);
        h->bin.pool_runs = runs;
        const size_t nq = (size_t)rv::kQueueSets * rv::kMaxBricks;
        if ((e = hipMalloc(&h->bin.pool, runs * sizeof(uint32_t))) != hipSuccess)
            return bail(e, "brick run pool");
        if ((e = hipMalloc(&h->bin.fill, nq * sizeof(uint32_t))) != hipSuccess ||
            (e = hipMalloc(&h->bin.qbase, nq * sizeof(uint32_t))) != hipSuccess ||
            (e = hipMalloc(&h->bin.cap, rv::kMaxBricks * sizeof(uint32_t))) != hipSuccess ||
            (e = hipMalloc(&h->bin.est, rv::kMaxBricks * sizeof(uint32_t))) != hipSuccess ||
            (e = hipMalloc(&h->bin.flags, rv::kMaxBricks * sizeof(uint32_t))) != hipSuccess ||
            (e = hipMalloc(&h->bin.order, rv::kMaxBricks * sizeof(uint32_t))) != hipSuccess ||
            (e = hipMalloc(&h->d_ovf, ncell * sizeof(int32_t))) != hipSuccess)
            return bail(e, "brick scratch");
        if ((e = hipMemset(h->bin.est, 0, rv::kMaxBricks * sizeof(uint32_t))) != hipSuccess ||
            (e = hipMemset(h->d_ovf, 0, ncell * sizeof(int32_t))) != hipSuccess ||
            (e = hipDeviceSynchronize()) != hipSuccess)
            return bail(e, "brick scratch init");
        h->bin.ovf = h->d_ovf;
        h->brick_ok = true;
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
    return h ? h->err.c_str() : g_create_error.c_str();
}

RV_API rv_status rot_vote_set_stream(rv_handle* h, void* stream)
{
    if (!h)
        return RV_EINVAL;
    h->stream = static_cast<hipStream_t>(stream);
    h->err.clear();
    return RV_OK;
}

RV_API rv_status rot_vote_solve(rv_handle* h, const float* x, const float* y, int64_t n,
                                int32_t grid, float eps_rad, float q_out[4],
                                int64_t* inlier_count, uint8_t* inlier_mask)
{
    if (!h)
        return RV_EINVAL;
    h->err.clear();
    if (!q_out || !inlier_count)
        return fail(h, RV_EINVAL, "rot_vote_solve: q_out and inlier_count must not be NULL");
    if (n < 0)
        return fail(h, RV_EINVAL, "rot_vote_solve: n < 0");
    if (n > h->max_n)
        return fail(h, RV_EINVAL, "rot_vote_solve: n exceeds the handle's max_n");
    if (grid < 1 || grid > h->max_grid)
        return fail(h, RV_EINVAL, "rot_vote_solve: grid outside 1..max_grid");
    if (!(eps_rad > 0.0f) || !(eps_rad <= (float)M_PI))
        return fail(h, RV_EINVAL, "rot_vote_solve: eps_rad outside (0, pi]");
    const int32_t J = h->cfg.samples_per_circle > 0 ? h->cfg.samples_per_circle : 8 * grid;
    if (J > h->max_J)
        return fail(h, RV_EINVAL, "rot_vote_solve: J = 8*grid exceeds the table sized at create");
    if ((int64_t)J * n > (int64_t)INT32_MAX)
        return fail(h, RV_EUNSUPPORTED, "rot_vote_solve: n*J exceeds int32 vote counts");
    if (n > 0) {
        if (!x || !y || !inlier_mask)
            return fail(h, RV_EINVAL, "rot_vote_solve: x, y and inlier_mask must not be NULL");
        if (!is_device_memory(x) || !is_device_memory(y) || !is_device_memory(inlier_mask))
            return fail(h, RV_EINVAL, "rot_vote_solve: x, y and inlier_mask must be device memory");
    }
    RV_HIP(h, hipSetDevice(h->device), "hipSetDevice");
    hipStream_t s = h->stream;
    const int64_t ncell = (int64_t)grid * grid * grid;
    const float T2 = residual_bound(eps_rad);
    int strategy = h->cfg.vote_strategy;
    if (strategy == RV_VOTE_AUTO)
        strategy = (h->brick_ok && grid >= kBrickMinGrid && grid <= rv::kMaxBrickGrid)
                       ? RV_VOTE_BRICK : RV_VOTE_GLOBAL;
    if (strategy == RV_VOTE_BRICK && !(h->brick_ok && grid <= rv::kMaxBrickGrid))
        return fail(h, RV_EUNSUPPORTED,
                    "rot_vote_solve: the brick strategy needs grid <= 256 and a handle created for it");

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
    h->last_grid = grid;
    h->last_J = J;
    h->last_strategy = strategy;
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[0], s), "event");
    if (brick)
        RV_HIP(h, rv::launch_bin_prepare(x, y, n, grid, J, h->d_table, h->bin, s), "brick plan");
    else
        RV_HIP(h, rv::launch_fill(h->d_hist, ncell, 0, s), "clear grid");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[1], s), "event");
    if (brick)
        RV_HIP(h, rv::launch_bin_vote(x, y, n, grid, J, h->d_table, h->bin, s), "binned vote");
    else
        RV_HIP(h, rv::launch_vote_global(x, y, n, grid, J, h->d_table, h->d_hist, 0, s), "vote");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[2], s), "event");
    int nlists;
    if (brick) {
        RV_HIP(h, rv::launch_brick_accum(grid, h->d_hist, h->d_partial, h->bin, s), "brick accumulate");
        const int nba = rv::brick_axis(grid);
        nlists = nba * nba * nba;
    } else {
        nlists = rv::topk_blocks(ncell);
        RV_HIP(h, rv::launch_topk_partial(h->d_hist, ncell, nlists, h->d_partial, s), "top-K partial");
    }
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[3], s), "event");
    if (n == 0) {
        RV_HIP(h, hipStreamSynchronize(s), "sync");
        q_out[0] = 1.0f;
        q_out[1] = q_out[2] = q_out[3] = 0.0f;
        *inlier_count = 0;
        h->last_ncand = 0;
        h->last_winner = -1;
        h->last_count = 0;
        h->events_recorded = false;
        return RV_OK;
    }
    const rv::Candidates c = candidates(h);
    RV_HIP(h, rv::launch_topk_final(h->d_partial, nlists, h->K, grid, c, s), "top-K final");
    if (tm)
        RV_HIP(h, hipEventRecord(h->ev[4], s), "event");
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
    // stages: prepare, vote, reduce, top-K, rescore, mask
    for (int k = 0; k < kStages; ++k)
        RV_HIP(h, hipEventElapsedTime(&ms[k], h->ev[k], h->ev[k + 1]), "hipEventElapsedTime");
    return RV_OK;
}
