// Request server over the C-ABI: one FIFO queue, admission by each request's
// device-memory footprint, lanes (a thread, a stream and a handle each) that
// run the admitted work concurrently, continuous batching of small requests.
// Host code only; every solve runs through the library's kernels.
//
// Admission.  A request's footprint is the scratch its solve needs bound:
// the G^3 int32 vote grid (1, 8 or 64 MiB at G = 64, 128, 256) plus, for the
// brick strategy, the run pool sized for its n; a fused batch needs its run
// pool and the gathered columns.  The scratch comes from one device arena of
// hbm_budget bytes allocated at create.  The dispatcher admits the oldest
// queued request (with the small requests it fuses) as soon as a lane is
// free and its footprint fits in the arena's free space, and hands it to the
// lane; when a lane finishes, its footprint returns to the arena and the
// next requests are admitted.  So the work in flight is bounded by memory
// (and by the lanes), not by a fixed count of worst-case slots: many small
// requests overlap on the device while one large one runs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <thread>
#include <unordered_map>
#include <vector>

#include "rotvote.h"
#include "rv_internal.h"

#define RV_API extern "C" __attribute__((visibility("default")))

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

constexpr int kMaxLanes = 64;
constexpr int64_t kAlign = 256;

int64_t align_up(int64_t b) { return (b + kAlign - 1) & ~(kAlign - 1); }

std::string g_server_create_error;

static_assert(sizeof(rv_request) == 56 && sizeof(rv_reply) == 72, "request and reply layouts");

struct Job {
    rv_request req;
    rv_reply reply{};
    hipEvent_t ready = nullptr;  // recorded on the caller's stream at submit (or null)
    int64_t solo_bytes = 0;      // footprint when run alone
    bool done = false;
};

// First-fit allocator over byte offsets of the device arena (host
// bookkeeping only; the arena itself is one hipMalloc at create).
struct Arena {
    char* base = nullptr;
    int64_t bytes = 0;
    std::map<int64_t, int64_t> free;  // offset -> size, coalesced
    int64_t in_use = 0;
    int64_t peak = 0;

    void reset()
    {
        free.clear();
        if (bytes > 0)
            free.emplace(0, bytes);
        in_use = peak = 0;
    }
    bool alloc(int64_t size, int64_t* off)
    {
        size = align_up(std::max<int64_t>(size, kAlign));
        for (auto it = free.begin(); it != free.end(); ++it) {
            if (it->second < size)
                continue;
            *off = it->first;
            const int64_t rest = it->second - size;
            const int64_t at = it->first + size;
            free.erase(it);
            if (rest > 0)
                free.emplace(at, rest);
            in_use += size;
            peak = std::max(peak, in_use);
            return true;
        }
        return false;
    }
    void release(int64_t off, int64_t size)
    {
        size = align_up(std::max<int64_t>(size, kAlign));
        in_use -= size;
        auto it = free.emplace(off, size).first;
        auto next = std::next(it);
        if (next != free.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free.erase(next);
        }
        if (it != free.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free.erase(it);
            }
        }
    }
};

struct Lane {
    int index = 0;
    hipStream_t stream = nullptr;
    rv_handle* h = nullptr;
    // gather/scatter descriptors of a fused batch (lane-owned, small)
    rv::GatherItem* d_items = nullptr;
    rv::Unit* d_units = nullptr;
    rv::GatherItem* h_items = nullptr;  // pinned
    rv::Unit* h_units = nullptr;        // pinned
    std::vector<int64_t> offsets;
    std::vector<float> q;
    std::vector<int64_t> counts;
    // the admitted work (guarded by the server mutex)
    std::vector<Job*> group;
    int64_t off = 0, bytes = 0;
    bool busy = false;
    bool stop = false;
    std::condition_variable cv;
    std::thread thread;
};

}  // namespace

struct rv_server {
    rv_server_config cfg{};
    int64_t max_units = 0;
    std::vector<std::unique_ptr<Lane>> lanes;
    int64_t device_bytes = 0;  // lanes' own scratch plus the arena
    Arena arena;

    std::mutex mu;
    std::condition_variable cv_admit;  // the dispatcher: work, a free lane or memory
    std::condition_variable cv_done;   // waiters
    std::deque<Job*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
    std::vector<hipEvent_t> events;    // free ready-events
    uint64_t next_ticket = 1;
    int64_t in_flight = 0;
    int64_t peak_in_flight = 0;
    bool paused = false;
    bool stopping = false;
    std::thread dispatcher;
    std::string err;
};

namespace {

rv_status sfail(rv_server* s, rv_status st, const std::string& msg)
{
    if (s) {
        std::lock_guard<std::mutex> lk(s->mu);
        s->err = msg;
    } else {
        g_server_create_error = msg;
    }
    return st;
}

bool batchable(const rv_server* s, const rv_request& r)
{
    return s->cfg.max_batch > 1 && r.grid <= RV_MAX_BATCH_GRID && r.n > 0 &&
           r.n <= s->cfg.batch_max_n && r.refine_rounds == 0;
}

bool same_solve(const rv_request& a, const rv_request& b)
{
    return a.grid == b.grid && std::memcmp(&a.eps_rad, &b.eps_rad, sizeof(float)) == 0;
}

// A fused batch's footprint: the run pool, then the gathered x, y (float32
// [3][cols] each) and mask (cols bytes).
int64_t batch_bytes(const rv_server* s, int64_t cols, int B, int grid, int64_t* pool_bytes)
{
    const int64_t pb = rv::lane_batch_bytes(s->lanes[0]->h, cols, B, grid);
    if (pb < 0)
        return -1;
    *pool_bytes = pb;
    return pb + 2 * align_up(3 * cols * (int64_t)sizeof(float)) + align_up(cols);
}

void release_lane(Lane* w)
{
    if (w->h)
        (void)rot_vote_destroy(w->h);
    (void)hipFree(w->d_items);
    (void)hipFree(w->d_units);
    (void)hipHostFree(w->h_items);
    (void)hipHostFree(w->h_units);
    if (w->stream)
        (void)hipStreamDestroy(w->stream);
}

// One request alone on the lane's bound scratch: solve (and refine).
void run_single(rv_server* s, Lane* w, Job* j)
{
    rv_request& r = j->req;
    rv_reply& out = j->reply;
    out.batched = 1;
    char* base = s->arena.base + w->off;
    const int64_t G = r.grid;
    const int64_t gbytes = align_up(G * G * G * (int64_t)sizeof(int32_t));
    rv::lane_bind(w->h, reinterpret_cast<int32_t*>(base), reinterpret_cast<uint32_t*>(base + gbytes),
                  (uint64_t)std::max<int64_t>(0, w->bytes - gbytes) / sizeof(uint32_t));
    rv_status st = rot_vote_solve(w->h, r.x, r.y, r.n, r.grid, r.eps_rad, out.q, &out.inlier_count,
                                  r.inlier_mask);
    if (st == RV_OK && r.refine_rounds > 0 && r.n > 0) {
        int32_t ran = 0;
        st = rot_vote_refine(w->h, r.x, r.y, r.n, r.eps_rad, r.refine_rounds, out.q,
                             &out.inlier_count, r.inlier_mask, &ran);
        out.refine_rounds_run = ran;
    }
    out.status = st;
}

// Several requests of one grid and eps as one batched solve: their columns
// gathered into the bound scratch, the batch's masks scattered back.
void run_batch(rv_server* s, Lane* w, const std::vector<Job*>& group)
{
    const int B = (int)group.size();
    w->offsets.assign(B + 1, 0);
    int64_t nu = 0;
    for (int b = 0; b < B; ++b) {
        const rv_request& r = group[b]->req;
        w->offsets[b + 1] = w->offsets[b] + r.n;
        w->h_items[b] = rv::GatherItem{r.x, r.y, r.inlier_mask, r.n, w->offsets[b]};
        for (int64_t f = 0; f < r.n; f += rv::kUnitSize)
            w->h_units[nu++] = rv::Unit{b, (int32_t)std::min<int64_t>(rv::kUnitSize, r.n - f), f};
    }
    const int64_t total = w->offsets[B];
    const rv_request& r0 = group[0]->req;
    int64_t pool_bytes = 0;
    (void)batch_bytes(s, total, B, r0.grid, &pool_bytes);
    char* base = s->arena.base + w->off;
    float* dx = reinterpret_cast<float*>(base + pool_bytes);
    float* dy = reinterpret_cast<float*>(base + pool_bytes + align_up(3 * total * (int64_t)sizeof(float)));
    uint8_t* dmask =
        reinterpret_cast<uint8_t*>(base + pool_bytes + 2 * align_up(3 * total * (int64_t)sizeof(float)));
    rv::lane_bind(w->h, nullptr, reinterpret_cast<uint32_t*>(base),
                  (uint64_t)pool_bytes / sizeof(uint32_t));
    rv_status st = RV_OK;
    hipError_t e = hipMemcpyAsync(w->d_items, w->h_items, (size_t)B * sizeof(rv::GatherItem),
                                  hipMemcpyHostToDevice, w->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w->d_units, w->h_units, (size_t)nu * sizeof(rv::Unit),
                           hipMemcpyHostToDevice, w->stream);
    if (e == hipSuccess)
        e = rv::launch_gather(w->d_items, w->d_units, (int)nu, dx, dy, total, w->stream);
    if (e != hipSuccess)
        st = RV_EDEVICE;
    if (st == RV_OK) {
        w->q.assign(4 * (size_t)B, 0.0f);
        w->counts.assign(B, 0);
        st = rot_vote_solve_batch(w->h, dx, dy, w->offsets.data(), B, r0.grid, r0.eps_rad,
                                  w->q.data(), w->counts.data(), dmask);
    }
    if (st == RV_OK) {
        e = rv::launch_scatter_masks(w->d_items, w->d_units, (int)nu, dmask, w->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(w->stream);
        if (e != hipSuccess)
            st = RV_EDEVICE;
    } else {
        (void)hipStreamSynchronize(w->stream);  // the scratch must be idle before it is freed
    }
    for (int b = 0; b < B; ++b) {
        rv_reply& out = group[b]->reply;
        out.batched = B;
        out.status = st;
        if (st == RV_OK) {
            std::memcpy(out.q, &w->q[4 * (size_t)b], 4 * sizeof(float));
            out.inlier_count = w->counts[b];
        }
    }
}

void lane_loop(rv_server* s, Lane* w)
{
    (void)hipSetDevice(s->cfg.device);
    for (;;) {
        std::vector<Job*> group;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            w->cv.wait(lk, [&] { return w->busy || w->stop; });
            if (!w->busy)
                return;  // stopping, nothing assigned
            group = w->group;
        }
        // the caller's stream produced x and y: wait for it on the lane's stream
        bool waited = false;
        for (Job* j : group)
            if (j->ready) {
                (void)hipStreamWaitEvent(w->stream, j->ready, 0);
                waited = true;
            }
        if (waited) {
            std::lock_guard<std::mutex> lk(s->mu);
            for (Job* j : group)
                if (j->ready) {
                    s->events.push_back(j->ready);  // re-recordable once the wait is enqueued
                    j->ready = nullptr;
                }
        }
        const double t0 = now_s();
        if (group.size() == 1)
            run_single(s, w, group[0]);
        else
            run_batch(s, w, group);
        const double t1 = now_s();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (Job* j : group) {
                j->reply.t_start = t0;
                j->reply.t_end = t1;
                j->reply.worker = w->index;
                j->reply.scratch_bytes = w->bytes;
                j->done = true;
            }
            s->arena.release(w->off, w->bytes);
            s->in_flight -= (int64_t)group.size();
            w->group.clear();
            w->busy = false;
        }
        s->cv_done.notify_all();
        s->cv_admit.notify_one();
    }
}

// Admits queued work (under the lock): the oldest request, with the small
// requests of the same grid and eps it fuses, on a free lane once its
// footprint fits in the arena.  Returns true if something was admitted.
bool admit_one(rv_server* s)
{
    if (s->paused || s->queue.empty())
        return false;
    Lane* lane = nullptr;
    for (auto& w : s->lanes)
        if (!w->busy) {
            lane = w.get();
            break;
        }
    if (!lane)
        return false;
    Job* head = s->queue.front();
    std::vector<Job*> group{head};
    int64_t cols = head->req.n;
    if (batchable(s, head->req)) {
        for (auto it = std::next(s->queue.begin());
             it != s->queue.end() && (int)group.size() < s->cfg.max_batch; ++it) {
            const rv_request& r = (*it)->req;
            if (batchable(s, r) && same_solve(r, head->req) && cols + r.n <= s->cfg.max_n) {
                cols += r.n;
                group.push_back(*it);
            }
        }
    }
    int64_t bytes = 0, off = 0, pool = 0;
    if (group.size() > 1) {
        bytes = batch_bytes(s, cols, (int)group.size(), head->req.grid, &pool);
        if (bytes < 0 || !s->arena.alloc(bytes, &off)) {
            group.resize(1);  // the head alone may still fit
            bytes = 0;
        }
    }
    if (group.size() == 1) {
        bytes = head->solo_bytes;
        if (!s->arena.alloc(bytes, &off))
            return false;  // wait for memory: the queue is served in order
    }
    for (Job* j : group) {
        auto it = std::find(s->queue.begin(), s->queue.end(), j);
        s->queue.erase(it);
    }
    lane->group = std::move(group);
    lane->off = off;
    lane->bytes = bytes;
    lane->busy = true;
    s->in_flight += (int64_t)lane->group.size();
    s->peak_in_flight = std::max(s->peak_in_flight, s->in_flight);
    lane->cv.notify_one();
    return true;
}

void dispatcher_loop(rv_server* s)
{
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        while (admit_one(s)) {
        }
        if (s->stopping && s->queue.empty())
            return;
        s->cv_admit.wait(lk);
    }
}

rv_status start_lane(rv_server* s, int index, std::unique_ptr<Lane>& out, int64_t* bytes)
{
    auto w = std::make_unique<Lane>();
    w->index = index;
    const rv_server_config& c = s->cfg;
    auto bail = [&](rv_status st, const std::string& m) {
        release_lane(w.get());
        return sfail(nullptr, st, m);
    };
    if (hipStreamCreateWithFlags(&w->stream, hipStreamNonBlocking) != hipSuccess)
        return bail(RV_EDEVICE, "rot_vote_server_create: stream");
    rv_config hc;
    rot_vote_default_config(&hc);
    hc.device = c.device;
    hc.stream = w->stream;
    hc.max_n = c.max_n;
    hc.max_grid = c.max_grid;
    hc.topk = c.topk;
    hc.samples_per_circle = c.samples_per_circle;
    const bool batching = c.max_batch > 1;
    hc.max_batch = batching ? c.max_batch : 0;
    rv_status st = rv::create_lane(&w->h, &hc);
    if (st != RV_OK)
        return bail(st, std::string("rot_vote_server_create: lane handle: ") +
                            rot_vote_last_error(nullptr));
    int64_t hb = 0;
    (void)rot_vote_get_footprint(w->h, &hb);
    if (batching) {
        if (hipMalloc(&w->d_items, (size_t)c.max_batch * sizeof(rv::GatherItem)) != hipSuccess ||
            hipMalloc(&w->d_units, (size_t)s->max_units * sizeof(rv::Unit)) != hipSuccess)
            return bail(RV_ENOMEM, "rot_vote_server_create: batch descriptors");
        if (hipHostMalloc(&w->h_items, (size_t)c.max_batch * sizeof(rv::GatherItem),
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&w->h_units, (size_t)s->max_units * sizeof(rv::Unit),
                          hipHostMallocDefault) != hipSuccess)
            return bail(RV_ENOMEM, "rot_vote_server_create: pinned staging");
        hb += (int64_t)(c.max_batch * sizeof(rv::GatherItem) + s->max_units * sizeof(rv::Unit));
    }
    *bytes = hb;
    out = std::move(w);
    return RV_OK;
}

void destroy_all(rv_server* s)
{
    for (auto& w : s->lanes)
        release_lane(w.get());
    for (hipEvent_t e : s->events)
        (void)hipEventDestroy(e);
    (void)hipFree(s->arena.base);
}

}  // namespace

RV_API void rot_vote_server_default_config(rv_server_config* cfg)
{
    if (!cfg)
        return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->device = 0;
    cfg->workers = 4;
    cfg->max_n = 1 << 20;
    cfg->max_grid = 256;
    cfg->topk = 16;
    cfg->samples_per_circle = 0;
    cfg->max_batch = 64;
    cfg->batch_max_n = 65536;
    cfg->max_queue = 1 << 20;
    cfg->hbm_budget = 0;
}

RV_API rv_status rot_vote_server_create(rv_server** out, const rv_server_config* cfg)
{
    if (!out || !cfg)
        return sfail(nullptr, RV_EINVAL, "rot_vote_server_create: NULL argument");
    if (cfg->workers < 1 || cfg->workers > kMaxLanes)
        return sfail(nullptr, RV_EINVAL, "rot_vote_server_create: workers outside 1..64");
    if (cfg->max_batch < 0 || cfg->max_batch > 4096 || cfg->batch_max_n < 0 || cfg->max_queue < 1 ||
        cfg->hbm_budget < 0 || cfg->max_n < 1)
        return sfail(nullptr, RV_EINVAL, "rot_vote_server_create: batch, queue, budget or max_n out of range");
    for (int r : cfg->reserved)
        if (r != 0)
            return sfail(nullptr, RV_EINVAL, "rot_vote_server_create: reserved fields must be 0");
    auto s = std::unique_ptr<rv_server>(new (std::nothrow) rv_server());
    if (!s)
        return sfail(nullptr, RV_ENOMEM, "rot_vote_server_create: out of host memory");
    s->cfg = *cfg;
    s->max_units = (cfg->max_n + rv::kUnitSize - 1) / rv::kUnitSize + std::max(1, cfg->max_batch);
    if (hipSetDevice(cfg->device) != hipSuccess)
        return sfail(nullptr, RV_EINVAL, "rot_vote_server_create: no such HIP device");
    for (int k = 0; k < cfg->workers; ++k) {
        std::unique_ptr<Lane> w;
        int64_t bytes = 0;
        rv_status st = start_lane(s.get(), k, w, &bytes);
        if (st != RV_OK) {
            destroy_all(s.get());
            return st;
        }
        s->device_bytes += bytes;
        s->lanes.push_back(std::move(w));
    }
    // the arena: hbm_budget bytes, or room for `workers` requests of the
    // largest size (so that memory never holds a request back)
    const rv_handle* h0 = s->lanes[0]->h;
    const int64_t largest = rv::lane_solve_bytes(h0, cfg->max_n, cfg->max_grid);
    int64_t arena = cfg->hbm_budget;
    if (arena == 0) {
        int64_t big = largest;
        if (cfg->max_batch > 1) {
            int64_t pool = 0;
            big = std::max(big, batch_bytes(s.get(), cfg->max_n, cfg->max_batch,
                                            std::min<int32_t>(cfg->max_grid, RV_MAX_BATCH_GRID), &pool));
        }
        arena = align_up(big) * cfg->workers;
    }
    arena = align_up(arena);
    if (hipMalloc(&s->arena.base, (size_t)arena) != hipSuccess) {
        (void)hipGetLastError();
        s->arena.base = nullptr;
        destroy_all(s.get());
        return sfail(nullptr, RV_ENOMEM, "rot_vote_server_create: the scratch arena does not fit");
    }
    s->arena.bytes = arena;
    s->arena.reset();
    s->device_bytes += arena;
    rv_server* raw = s.release();
    for (auto& w : raw->lanes)
        w->thread = std::thread(lane_loop, raw, w.get());
    raw->dispatcher = std::thread(dispatcher_loop, raw);
    *out = raw;
    return RV_OK;
}

RV_API rv_status rot_vote_server_destroy(rv_server* s)
{
    if (!s)
        return RV_OK;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stopping = true;
        s->paused = false;  // queued work is served before the server goes
    }
    s->cv_admit.notify_all();
    if (s->dispatcher.joinable())
        s->dispatcher.join();  // returns once the queue is empty
    {
        std::lock_guard<std::mutex> lk(s->mu);
        for (auto& w : s->lanes)
            w->stop = true;
    }
    for (auto& w : s->lanes) {
        w->cv.notify_all();
        if (w->thread.joinable())
            w->thread.join();  // a lane finishes its admitted work first
    }
    for (auto& kv : s->jobs)
        if (kv.second->ready)
            s->events.push_back(kv.second->ready);
    destroy_all(s);
    delete s;
    return RV_OK;
}

RV_API rv_status rot_vote_server_submit(rv_server* s, const rv_request* req, uint64_t* ticket)
{
    if (!s)
        return RV_EINVAL;
    if (!req || !ticket)
        return sfail(s, RV_EINVAL, "rot_vote_server_submit: NULL argument");
    const rv_request& r = *req;
    if (r.n < 0 || r.n > s->cfg.max_n)
        return sfail(s, RV_EINVAL, "rot_vote_server_submit: n outside 0..max_n");
    if (r.grid < 1 || r.grid > s->cfg.max_grid)
        return sfail(s, RV_EINVAL, "rot_vote_server_submit: grid outside 1..max_grid");
    if (!(r.eps_rad > 0.0f) || !(r.eps_rad <= 3.14159265f))
        return sfail(s, RV_EINVAL, "rot_vote_server_submit: eps_rad outside (0, pi]");
    if (r.refine_rounds < 0 || r.refine_rounds > RV_MAX_REFINE_ROUNDS)
        return sfail(s, RV_EINVAL, "rot_vote_server_submit: refine_rounds outside 0..64");
    if (r.flags & ~(uint32_t)RV_REQ_AFTER_STREAM)
        return sfail(s, RV_EINVAL, "rot_vote_server_submit: unknown request flags");
    if (r.n > 0 && (!r.x || !r.y || !r.inlier_mask))
        return sfail(s, RV_EINVAL, "rot_vote_server_submit: x, y and inlier_mask must not be NULL");
    auto j = std::make_unique<Job>();
    j->req = r;
    j->solo_bytes = rv::lane_solve_bytes(s->lanes[0]->h, r.n, r.grid);
    if (j->solo_bytes < 0 || align_up(j->solo_bytes) > s->arena.bytes)
        return sfail(s, RV_ENOMEM,
                     "rot_vote_server_submit: the request's scratch exceeds the server's hbm_budget");
    j->reply.t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int64_t)s->queue.size() >= s->cfg.max_queue) {
            s->err = "rot_vote_server_submit: queue full";
            return RV_EAGAIN;
        }
        if (r.flags & RV_REQ_AFTER_STREAM) {
            hipEvent_t ev = nullptr;
            if (!s->events.empty()) {
                ev = s->events.back();
                s->events.pop_back();
            } else if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
                s->err = "rot_vote_server_submit: event";
                return RV_EDEVICE;
            }
            if (hipEventRecord(ev, static_cast<hipStream_t>(r.stream)) != hipSuccess) {
                s->events.push_back(ev);
                s->err = "rot_vote_server_submit: recording on the request's stream failed";
                return RV_EDEVICE;
            }
            j->ready = ev;
        }
        const uint64_t t = s->next_ticket++;
        s->queue.push_back(j.get());
        s->jobs.emplace(t, std::move(j));
        *ticket = t;
    }
    s->cv_admit.notify_one();
    return RV_OK;
}

RV_API rv_status rot_vote_server_wait(rv_server* s, uint64_t ticket, int32_t timeout_ms,
                                      rv_reply* out)
{
    if (!s)
        return RV_EINVAL;
    if (!out)
        return sfail(s, RV_EINVAL, "rot_vote_server_wait: NULL argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) {
        s->err = "rot_vote_server_wait: unknown or collected ticket";
        return RV_EINVAL;
    }
    Job* j = it->second.get();
    auto ready = [&] { return j->done; };
    if (timeout_ms < 0) {
        s->cv_done.wait(lk, ready);
    } else if (!s->cv_done.wait_for(lk, std::chrono::milliseconds(timeout_ms), ready)) {
        return RV_ETIMEDOUT;
    }
    *out = j->reply;
    s->jobs.erase(it);
    return RV_OK;
}

RV_API rv_status rot_vote_server_stats(rv_server* s, int32_t* workers, int64_t* device_bytes,
                                       int64_t* queued, int64_t* in_flight)
{
    if (!s)
        return RV_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (workers)
        *workers = (int32_t)s->lanes.size();
    if (device_bytes)
        *device_bytes = s->device_bytes;
    if (queued)
        *queued = (int64_t)s->queue.size();
    if (in_flight)
        *in_flight = s->in_flight;
    return RV_OK;
}

RV_API rv_status rot_vote_server_memory(rv_server* s, int64_t* arena_bytes, int64_t* in_use,
                                        int64_t* peak_in_use, int64_t* peak_in_flight)
{
    if (!s)
        return RV_EINVAL;
    std::lock_guard<std::mutex> lk(s->mu);
    if (arena_bytes)
        *arena_bytes = s->arena.bytes;
    if (in_use)
        *in_use = s->arena.in_use;
    if (peak_in_use)
        *peak_in_use = s->arena.peak;
    if (peak_in_flight)
        *peak_in_flight = s->peak_in_flight;
    return RV_OK;
}

RV_API rv_status rot_vote_server_pause(rv_server* s, int32_t paused)
{
    if (!s)
        return RV_EINVAL;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->paused = paused != 0;
    }
    s->cv_admit.notify_all();
    return RV_OK;
}

RV_API rv_status rot_vote_server_request_bytes(rv_server* s, int64_t n, int32_t grid, int64_t* bytes)
{
    if (!s || !bytes)
        return RV_EINVAL;
    if (n < 0 || n > s->cfg.max_n || grid < 1 || grid > s->cfg.max_grid)
        return sfail(s, RV_EINVAL, "rot_vote_server_request_bytes: n or grid outside the server's limits");
    *bytes = align_up(rv::lane_solve_bytes(s->lanes[0]->h, n, grid));
    return RV_OK;
}

RV_API const char* rot_vote_server_last_error(const rv_server* s)
{
    return s ? s->err.c_str() : g_server_create_error.c_str();
}
