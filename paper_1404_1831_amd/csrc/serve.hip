// Served form of the search: continuous batching over concurrent lanes.
//
// A server owns `nlanes` lanes, each a handle over the same index arrays with
// its own HIP stream and workspace. Requests (one query, its L and k) are
// queued by fbpq_server_submit from any host thread. Each lane has a worker
// thread that, whenever its previous batch is done, takes every pending
// request up to max_batch and searches them as one batch on its stream; the
// lanes' batches overlap on the GPU. Finished requests carry their submit,
// start and finish times and are collected with fbpq_server_poll.
#include <hip/hip_runtime.h>

#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "fbpq.h"
#include "fbpq_dev.h"

using namespace fbpq;

namespace {

double now_s()
{
    return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct Req {
    int64_t tag, L;
    int32_t k;
    double t_submit;
    std::vector<float> q;
};

struct Done {
    int64_t tag;
    int32_t rc;
    double t_submit, t_start, t_done;
    std::vector<int64_t> ids;
    std::vector<float> d;
};

}  // namespace

struct fbpq_server {
    fbpq_index *ix = nullptr;
    int32_t max_batch = 0, k_max = 0, D = 0;
    std::vector<fbpq_index *> lanes;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Req> pending;
    std::deque<Done> done;
    bool stop = false;
    int64_t batches = 0, batched = 0;
    std::string last_err;  // message of the first failed batch
};

namespace {

void worker(fbpq_server *s, fbpq_index *lane)
{
    (void)hipSetDevice(lane_device(lane));
    std::vector<Req> batch;
    std::vector<float> Q;
    std::vector<int64_t> L, ids;
    std::vector<int32_t> k;
    std::vector<float> d;
    for (;;) {
        {
            std::unique_lock<std::mutex> lk(s->mu);
            s->cv.wait(lk, [&] { return s->stop || !s->pending.empty(); });
            if (s->pending.empty()) return;  // stopping and drained
            batch.clear();
            while (!s->pending.empty() && (int32_t)batch.size() < s->max_batch) {
                batch.push_back(std::move(s->pending.front()));
                s->pending.pop_front();
            }
            s->batches += 1;
            s->batched += (int64_t)batch.size();
        }
        const double t_start = now_s();
        const int64_t n = (int64_t)batch.size();
        Q.resize((size_t)n * s->D);
        L.resize(n);
        k.resize(n);
        for (int64_t i = 0; i < n; ++i) {
            std::copy(batch[i].q.begin(), batch[i].q.end(), Q.begin() + i * s->D);
            L[i] = batch[i].L;
            k[i] = batch[i].k;
        }
        ids.assign((size_t)n * s->k_max, -1);
        d.assign((size_t)n * s->k_max, 0.f);
        const int rc = fbpq_search_uneven(lane, Q.data(), n, L.data(), k.data(), s->k_max, ids.data(), d.data());
        const double t_done = now_s();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            if (rc && s->last_err.empty()) s->last_err = fbpq_last_error();
            for (int64_t i = 0; i < n; ++i) {
                Done r;
                r.tag = batch[i].tag;
                // CAPACITY marks only the rows it could not serve
                r.rc = rc == FBPQ_E_CAPACITY ? (ids[i * s->k_max] == -2 ? rc : FBPQ_OK) : rc;
                r.t_submit = batch[i].t_submit;
                r.t_start = t_start;
                r.t_done = t_done;
                r.ids.assign(ids.begin() + i * s->k_max, ids.begin() + (i + 1) * s->k_max);
                r.d.assign(d.begin() + i * s->k_max, d.begin() + (i + 1) * s->k_max);
                s->done.push_back(std::move(r));
            }
        }
        s->cv.notify_all();
    }
}

}  // namespace

extern "C" {

int fbpq_server_create(fbpq_index *ix, int32_t max_batch, int32_t nlanes, int32_t k_max, fbpq_server **out)
{
    if (!ix || !out || max_batch < 1 || nlanes < 1 || nlanes > 16 || k_max < 1 || k_max > FBPQ_K_MAX)
        return FBPQ_E_INVALID;
    fbpq_server *s = new fbpq_server();
    s->ix = ix;
    s->max_batch = max_batch;
    s->k_max = k_max;
    s->D = lane_dim(ix);
    for (int i = 0; i < nlanes; ++i) {
        fbpq_index *lane = nullptr;
        const int rc = lane_create(ix, &lane);
        if (rc) {
            for (fbpq_index *l : s->lanes) fbpq_free_index(l);
            delete s;
            return rc;
        }
        s->lanes.push_back(lane);
    }
    for (fbpq_index *lane : s->lanes) s->workers.emplace_back(worker, s, lane);
    *out = s;
    return FBPQ_OK;
}

int fbpq_server_submit(fbpq_server *s, const float *q, int64_t L, int32_t k, int64_t tag)
{
    if (!s || !q || L < 1 || k < 1 || k > s->k_max) return FBPQ_E_INVALID;
    Req r;
    r.tag = tag;
    r.L = L;
    r.k = k;
    r.q.assign(q, q + s->D);
    r.t_submit = now_s();
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return FBPQ_E_STATE;
        s->pending.push_back(std::move(r));
    }
    s->cv.notify_one();
    return FBPQ_OK;
}

int fbpq_server_poll(fbpq_server *s, int32_t max_n, double wait_s, int64_t *tags, int64_t *ids, float *dists,
                     double *times, int32_t *status, int32_t *n_out)
{
    if (!s || max_n < 0 || !n_out || (max_n > 0 && (!tags || !ids || !dists || !times || !status)))
        return FBPQ_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    if (s->done.empty() && wait_s > 0)
        s->cv.wait_for(lk, std::chrono::duration<double>(wait_s), [&] { return !s->done.empty(); });
    int32_t n = 0;
    while (n < max_n && !s->done.empty()) {
        Done &r = s->done.front();
        tags[n] = r.tag;
        status[n] = r.rc;
        std::copy(r.ids.begin(), r.ids.end(), ids + (int64_t)n * s->k_max);
        std::copy(r.d.begin(), r.d.end(), dists + (int64_t)n * s->k_max);
        times[3 * n] = r.t_submit;
        times[3 * n + 1] = r.t_start;
        times[3 * n + 2] = r.t_done;
        s->done.pop_front();
        ++n;
    }
    *n_out = n;
    return FBPQ_OK;
}

int fbpq_server_counts(fbpq_server *s, int64_t *pending, int64_t *batches, int64_t *batched)
{
    if (!s || !pending || !batches || !batched) return FBPQ_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    *pending = (int64_t)s->pending.size();
    *batches = s->batches;
    *batched = s->batched;
    return FBPQ_OK;
}

const char *fbpq_server_first_error(fbpq_server *s)
{
    if (!s) return "";
    std::lock_guard<std::mutex> lk(s->mu);
    thread_local std::string copy;
    copy = s->last_err;
    return copy.c_str();
}

void fbpq_server_destroy(fbpq_server *s)
{
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
    }
    s->cv.notify_all();
    for (std::thread &t : s->workers) t.join();
    for (fbpq_index *lane : s->lanes) fbpq_free_index(lane);
    delete s;
}

}  // extern "C"
