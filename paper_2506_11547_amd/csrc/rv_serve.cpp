// Request server over the C-ABI: one FIFO queue, worker threads with their own
// stream and handle, continuous batching of small requests.  Host code only;
// every solve runs through the library's entry points and kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
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

std::string g_server_create_error;

struct Job {
    rv_request req;
    rv_reply reply{};
    bool done = false;
};

struct Worker {
    int index = 0;
    hipStream_t stream = nullptr;
    rv_handle* h = nullptr;
    // batch staging (when batching is on)
    float* dx = nullptr;
    float* dy = nullptr;
    uint8_t* dmask = nullptr;
    rv::GatherItem* d_items = nullptr;
    rv::Unit* d_units = nullptr;
    rv::GatherItem* h_items = nullptr;  // pinned
    rv::Unit* h_units = nullptr;        // pinned
    std::vector<int64_t> offsets;
    std::vector<float> q;
    std::vector<int64_t> counts;
    std::thread thread;
};

}  // namespace

struct rv_server {
    rv_server_config cfg{};
    int64_t max_units = 0;
    std::vector<std::unique_ptr<Worker>> workers;
    int64_t device_bytes = 0;

    std::mutex mu;
    std::condition_variable cv_work;
    std::condition_variable cv_done;
    std::deque<Job*> queue;
    std::unordered_map<uint64_t, std::unique_ptr<Job>> jobs;
    uint64_t next_ticket = 1;
    int64_t in_flight = 0;
    bool stopping = false;
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

void release_worker(Worker* w)
{
    if (w->h)
        (void)rot_vote_destroy(w->h);
    (void)hipFree(w->dx);
    (void)hipFree(w->dy);
    (void)hipFree(w->dmask);
    (void)hipFree(w->d_items);
    (void)hipFree(w->d_units);
    (void)hipHostFree(w->h_items);
    (void)hipHostFree(w->h_units);
    if (w->stream)
        (void)hipStreamDestroy(w->stream);
}

// One request alone: solve (and refine), reply filled.
void run_single(Worker* w, Job* j)
{
    rv_request& r = j->req;
    rv_reply& out = j->reply;
    out.batched = 1;
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

// Several requests of one grid and eps as one batched solve.
void run_batch(rv_server* s, Worker* w, const std::vector<Job*>& group)
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
    rv_status st = RV_OK;
    hipError_t e = hipMemcpyAsync(w->d_items, w->h_items, (size_t)B * sizeof(rv::GatherItem),
                                  hipMemcpyHostToDevice, w->stream);
    if (e == hipSuccess)
        e = hipMemcpyAsync(w->d_units, w->h_units, (size_t)nu * sizeof(rv::Unit),
                           hipMemcpyHostToDevice, w->stream);
    if (e == hipSuccess)
        e = rv::launch_gather(w->d_items, w->d_units, (int)nu, w->dx, w->dy, total, w->stream);
    if (e != hipSuccess)
        st = RV_EDEVICE;
    if (st == RV_OK) {
        w->q.assign(4 * (size_t)B, 0.0f);
        w->counts.assign(B, 0);
        const rv_request& r0 = group[0]->req;
        st = rot_vote_solve_batch(w->h, w->dx, w->dy, w->offsets.data(), B, r0.grid, r0.eps_rad,
                                  w->q.data(), w->counts.data(), w->dmask);
    }
    if (st == RV_OK) {
        e = rv::launch_scatter_masks(w->d_items, w->d_units, (int)nu, w->dmask, w->stream);
        if (e == hipSuccess)
            e = hipStreamSynchronize(w->stream);
        if (e != hipSuccess)
            st = RV_EDEVICE;
    } else {
        (void)hipStreamSynchronize(w->stream);  // the staging must be idle before reuse
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
    (void)s;
}

void worker_loop(rv_server* s, Worker* w)
{
    (void)hipSetDevice(s->cfg.device);
    std::vector<Job*> group;
    for (;;) {
        group.clear();
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv_work.wait(lk, [&] { return s->stopping || !s->queue.empty(); });
            if (s->queue.empty())
                return;  // stopping and drained
            Job* head = s->queue.front();
            s->queue.pop_front();
            group.push_back(head);
            if (batchable(s, head->req)) {
                int64_t cols = head->req.n;
                for (auto it = s->queue.begin();
                     it != s->queue.end() && (int)group.size() < s->cfg.max_batch;) {
                    const rv_request& r = (*it)->req;
                    if (batchable(s, r) && same_solve(r, head->req) && cols + r.n <= s->cfg.max_n) {
                        cols += r.n;
                        group.push_back(*it);
                        it = s->queue.erase(it);
                    } else {
                        ++it;
                    }
                }
            }
            s->in_flight += (int64_t)group.size();
        }
        const double t0 = now_s();
        if (group.size() == 1)
            run_single(w, group[0]);
        else
            run_batch(s, w, group);
        const double t1 = now_s();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            for (Job* j : group) {
                j->reply.t_start = t0;
                j->reply.t_end = t1;
                j->reply.worker = w->index;
                j->done = true;
            }
            s->in_flight -= (int64_t)group.size();
        }
        s->cv_done.notify_all();
    }
}

rv_status start_worker(rv_server* s, int index, std::unique_ptr<Worker>& out, int64_t* bytes)
{
    auto w = std::make_unique<Worker>();
    w->index = index;
    const rv_server_config& c = s->cfg;
    auto bail = [&](rv_status st, const std::string& m) {
        release_worker(w.get());
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
    rv_status st = rot_vote_create(&w->h, &hc);
    if (st != RV_OK)
        return bail(st, std::string("rot_vote_server_create: worker handle: ") +
                            rot_vote_last_error(nullptr));
    int64_t hb = 0;
    (void)rot_vote_get_footprint(w->h, &hb);
    if (batching) {
        const size_t cols = (size_t)std::max<int64_t>(1, c.max_n);
        if (hipMalloc(&w->dx, 3 * cols * sizeof(float)) != hipSuccess ||
            hipMalloc(&w->dy, 3 * cols * sizeof(float)) != hipSuccess ||
            hipMalloc(&w->dmask, cols) != hipSuccess ||
            hipMalloc(&w->d_items, (size_t)c.max_batch * sizeof(rv::GatherItem)) != hipSuccess ||
            hipMalloc(&w->d_units, (size_t)s->max_units * sizeof(rv::Unit)) != hipSuccess)
            return bail(RV_ENOMEM, "rot_vote_server_create: batch staging");
        if (hipHostMalloc(&w->h_items, (size_t)c.max_batch * sizeof(rv::GatherItem),
                          hipHostMallocDefault) != hipSuccess ||
            hipHostMalloc(&w->h_units, (size_t)s->max_units * sizeof(rv::Unit),
                          hipHostMallocDefault) != hipSuccess)
            return bail(RV_ENOMEM, "rot_vote_server_create: pinned staging");
        hb += (int64_t)(6 * cols * sizeof(float) + cols + c.max_batch * sizeof(rv::GatherItem) +
                        s->max_units * sizeof(rv::Unit));
    }
    *bytes = hb;
    out = std::move(w);
    return RV_OK;
}

}  // namespace

RV_API void rot_vote_server_default_config(rv_server_config* cfg)
{
    if (!cfg)
        return;
    std::memset(cfg, 0, sizeof(*cfg));
    cfg->device = 0;
    cfg->workers = 2;
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
    if (cfg->workers < 1 || cfg->workers > 16)
        return sfail(nullptr, RV_EINVAL, "rot_vote_server_create: workers outside 1..16");
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
        std::unique_ptr<Worker> w;
        int64_t bytes = 0;
        rv_status st = start_worker(s.get(), k, w, &bytes);
        if (st != RV_OK) {
            if (k > 0 && st == RV_ENOMEM && cfg->hbm_budget > 0)
                break;  // fewer workers fit
            for (auto& v : s->workers)
                release_worker(v.get());
            return st;
        }
        if (cfg->hbm_budget > 0 && s->device_bytes + bytes > cfg->hbm_budget) {
            release_worker(w.get());
            if (k == 0) {
                return sfail(nullptr, RV_ENOMEM,
                             "rot_vote_server_create: one worker needs more than hbm_budget");
            }
            break;
        }
        s->device_bytes += bytes;
        s->workers.push_back(std::move(w));
    }
    rv_server* raw = s.release();
    for (auto& w : raw->workers)
        w->thread = std::thread(worker_loop, raw, w.get());
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
    }
    s->cv_work.notify_all();
    for (auto& w : s->workers)
        if (w->thread.joinable())
            w->thread.join();
    for (auto& w : s->workers)
        release_worker(w.get());
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
    if (r.refine_rounds < 0 || r.refine_rounds > RV_MAX_REFINE_ROUNDS || r.reserved != 0)
        return sfail(s, RV_EINVAL, "rot_vote_server_submit: refine_rounds outside 0..64");
    if (r.n > 0 && (!r.x || !r.y || !r.inlier_mask))
        return sfail(s, RV_EINVAL, "rot_vote_server_submit: x, y and inlier_mask must not be NULL");
    auto j = std::make_unique<Job>();
    j->req = r;
    j->reply.t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if ((int64_t)s->queue.size() >= s->cfg.max_queue) {
            s->err = "rot_vote_server_submit: queue full";
            return RV_EAGAIN;
        }
        const uint64_t t = s->next_ticket++;
        s->queue.push_back(j.get());
        s->jobs.emplace(t, std::move(j));
        *ticket = t;
    }
    s->cv_work.notify_one();
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
        *workers = (int32_t)s->workers.size();
    if (device_bytes)
        *device_bytes = s->device_bytes;
    if (queued)
        *queued = (int64_t)s->queue.size();
    if (in_flight)
        *in_flight = s->in_flight;
    return RV_OK;
}

RV_API const char* rot_vote_server_last_error(const rv_server* s)
{
    return s ? s->err.c_str() : g_server_create_error.c_str();
}
