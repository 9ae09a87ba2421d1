// Served form of the search: continuous batching over concurrent lanes.
//
// A server owns `nlanes` lanes, each a handle over the same index arrays with
// its own HIP stream and workspace, and one host worker thread per lane.
// Requests (one query, its L and k) are queued by fbpq_server_submit from any
// host thread. A lane that is free takes the oldest pending request and, in
// arrival order, the pending requests of the same candidate-budget class
// (floor(log2(min(L, N)))) that fit its batch size and its share of the
// workspace budget, and searches them as one batch on its stream; the lanes'
// batches overlap on the GPU. Grouping by budget class keeps a short request
// out of a batch that waits for a long one, and taking the oldest request
// first keeps the queue fair.
//
// Admission: every request reserves an estimate of the workspace its search
// needs (a fixed part per query plus bytes per candidate, from the buffer
// sizes of the search pipeline, search_ws_estimate). A lane's batch reserves
// at most budget / nlanes, so the workspace the lanes can grow to stays within
// the budget. A request whose reservation alone exceeds a lane's share, or
// that arrives while max_pending requests are queued, is refused at submit
// with FBPQ_E_CAPACITY. A request still queued past its deadline completes
// with FBPQ_E_TIMEOUT without being searched; fbpq_server_cancel takes a
// queued request out (FBPQ_E_CANCELLED). A batch already on the GPU runs to
// the end.
//
// With a null index and cfg->fake_ns_per_cand > 0 the lanes run a host test
// backend instead of the GPU (for scheduler tests on machines without a GPU):
// it sleeps fake_ns_per_cand per candidate of the batch and answers request
// (q, k) with ids j + 1000 * round(q[0]) and distances q[1] + j, j < k.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
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
    int bucket;
    int64_t reserve;  // workspace bytes reserved while its batch runs
    double t_submit, deadline;
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
    fbpq_index *ix = nullptr;  // null: host test backend
    fbpq_server_config cfg{};
    int64_t N = 0;             // points of the index (caps the candidate budget)
    int64_t lane_budget = 0;   // workspace bytes one lane's batch may reserve
    std::vector<fbpq_index *> lanes;
    std::vector<std::thread> workers;
    std::mutex mu;
    std::condition_variable cv_work;  // workers: a request was queued, or the server stops
    std::condition_variable cv_done;  // pollers: a request completed
    std::deque<Req> pending;
    std::deque<Done> done;
    bool stop = false;
    int64_t reserved = 0;  // workspace reserved by the batches running now
    int64_t st[FBPQ_SERVER_NUM_STATS] = {0};
    std::string last_err;  // message of the first failed batch
};

namespace {

int lbucket(int64_t L, int64_t N)
{
    const int64_t e = std::max<int64_t>(1, std::min(L, N));
    return 63 - __builtin_clzll((unsigned long long)e);
}

void finish_unrun(fbpq_server *s, const Req &r, int32_t rc, double t)
{
    Done d;
    d.tag = r.tag;
    d.rc = rc;
    d.t_submit = r.t_submit;
    d.t_start = t;
    d.t_done = t;
    d.ids.assign((size_t)s->cfg.k_max, -1);
    d.d.assign((size_t)s->cfg.k_max, __builtin_huge_valf());
    s->done.push_back(std::move(d));
}

// Completes (TIMEOUT) the queued requests whose deadline has passed. Caller holds mu.
bool expire_locked(fbpq_server *s, double t)
{
    bool any = false;
    for (auto it = s->pending.begin(); it != s->pending.end();) {
        if (it->deadline > 0 && it->deadline <= t) {
            finish_unrun(s, *it, FBPQ_E_TIMEOUT, t);
            ++s->st[FBPQ_SERVER_STAT_TIMEOUT];
            it = s->pending.erase(it);
            any = true;
        } else {
            ++it;
        }
    }
    return any;
}

int fake_batch(const fbpq_server *s, const std::vector<float> &Q, const std::vector<int64_t> &L,
               const std::vector<int32_t> &k, std::vector<int64_t> &ids, std::vector<float> &d)
{
    const int64_t n = (int64_t)L.size();
    double cand = 0.0;
    for (int64_t i = 0; i < n; ++i) cand += (double)std::min(L[i], s->N);
    std::this_thread::sleep_for(std::chrono::duration<double>(cand * s->cfg.fake_ns_per_cand * 1e-9));
    for (int64_t i = 0; i < n; ++i) {
        const int64_t base = 1000 * (int64_t)std::llround(Q[(size_t)i * s->cfg.D]);
        const float d0 = Q[(size_t)i * s->cfg.D + (s->cfg.D > 1 ? 1 : 0)];
        for (int32_t j = 0; j < k[i]; ++j) {
            ids[(size_t)i * s->cfg.k_max + j] = base + j;
            d[(size_t)i * s->cfg.k_max + j] = d0 + (float)j;
        }
    }
    return FBPQ_OK;
}

void worker(fbpq_server *s, fbpq_index *lane)
{
    if (lane) (void)hipSetDevice(lane_device(lane));
    const int D = s->cfg.D, kmax = s->cfg.k_max;
    std::vector<Req> batch;
    std::vector<float> Q, d;
    std::vector<int64_t> L, ids;
    std::vector<int32_t> k;
    for (;;) {
        int64_t res = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            for (;;) {
                if (expire_locked(s, now_s())) s->cv_done.notify_all();
                if (!s->pending.empty() || s->stop) break;
                s->cv_work.wait(lk);
            }
            if (s->pending.empty()) return;  // stopping and drained
            // the oldest request, then same-class requests in arrival order
            batch.clear();
            const int b = s->pending.front().bucket;
            for (auto it = s->pending.begin(); it != s->pending.end() && (int32_t)batch.size() < s->cfg.max_batch;) {
                if (it->bucket == b && (batch.empty() || res + it->reserve <= s->lane_budget)) {
                    res += it->reserve;
                    batch.push_back(std::move(*it));
                    it = s->pending.erase(it);
                } else {
                    ++it;
                }
            }
            s->reserved += res;
            s->st[FBPQ_SERVER_STAT_PEAK_RESERVED] = std::max(s->st[FBPQ_SERVER_STAT_PEAK_RESERVED], s->reserved);
            s->st[FBPQ_SERVER_STAT_PEAK_BATCH_RESERVED] =
                std::max(s->st[FBPQ_SERVER_STAT_PEAK_BATCH_RESERVED], res);
            s->st[FBPQ_SERVER_STAT_BATCHES] += 1;
            s->st[FBPQ_SERVER_STAT_BATCHED] += (int64_t)batch.size();
        }
        const double t_start = now_s();
        const int64_t n = (int64_t)batch.size();
        Q.resize((size_t)n * D);
        L.resize(n);
        k.resize(n);
        for (int64_t i = 0; i < n; ++i) {
            std::copy(batch[i].q.begin(), batch[i].q.end(), Q.begin() + i * D);
            L[i] = batch[i].L;
            k[i] = batch[i].k;
        }
        ids.assign((size_t)n * kmax, -1);
        d.assign((size_t)n * kmax, __builtin_huge_valf());
        std::string err;
        int rc;
        if (lane) {
            rc = fbpq_search_uneven(lane, Q.data(), n, L.data(), k.data(), kmax, ids.data(), d.data());
            if (rc) err = fbpq_last_error();
        } else {
            rc = fake_batch(s, Q, L, k, ids, d);
        }
        const double t_done = now_s();
        {
            std::lock_guard<std::mutex> lk(s->mu);
            s->reserved -= res;
            if (rc && s->last_err.empty()) s->last_err = err;
            for (int64_t i = 0; i < n; ++i) {
                Done r;
                r.tag = batch[i].tag;
                // CAPACITY marks only the rows it could not serve
                r.rc = rc == FBPQ_E_CAPACITY ? (ids[i * kmax] == -2 ? rc : FBPQ_OK) : rc;
                ++s->st[r.rc == FBPQ_OK ? FBPQ_SERVER_STAT_COMPLETED : FBPQ_SERVER_STAT_FAILED];
                r.t_submit = batch[i].t_submit;
                r.t_start = t_start;
                r.t_done = t_done;
                r.ids.assign(ids.begin() + i * kmax, ids.begin() + (i + 1) * kmax);
                r.d.assign(d.begin() + i * kmax, d.begin() + (i + 1) * kmax);
                s->done.push_back(std::move(r));
            }
        }
        s->cv_done.notify_all();
    }
}

}  // namespace

extern "C" {

int fbpq_server_create2(fbpq_index *ix, const fbpq_server_config *cfg, fbpq_server **out)
{
    if (!out || !cfg) return FBPQ_E_INVALID;
    *out = nullptr;
    const fbpq_server_config &c = *cfg;
    if (c.max_batch < 1 || c.nlanes < 1 || c.nlanes > 16 || c.k_max < 1 || c.k_max > FBPQ_K_MAX ||
        c.ws_budget < 0 || c.max_pending < 0 || !(c.timeout_s >= 0) || !(c.fake_ns_per_cand >= 0))
        return FBPQ_E_INVALID;
    if (!ix && !(c.fake_ns_per_cand > 0 && c.D > 0)) return FBPQ_E_INVALID;
    fbpq_server *s = new fbpq_server();
    s->ix = ix;
    s->cfg = c;
    if (s->cfg.ws_budget == 0) s->cfg.ws_budget = (int64_t)16 << 30;
    if (s->cfg.max_pending == 0) s->cfg.max_pending = (int64_t)1 << 20;
    s->lane_budget = s->cfg.ws_budget / s->cfg.nlanes;
    if (ix) {
        s->cfg.D = lane_dim(ix);
        s->N = lane_points(ix);
        for (int i = 0; i < c.nlanes; ++i) {
            fbpq_index *lane = nullptr;
            const int rc = lane_create(ix, &lane);
            if (rc) {
                for (fbpq_index *l : s->lanes) fbpq_free_index(l);
                delete s;
                return rc;
            }
            s->lanes.push_back(lane);
        }
    } else {
        s->N = INT64_MAX;
        s->lanes.assign((size_t)c.nlanes, nullptr);
    }
    s->st[FBPQ_SERVER_STAT_BUDGET] = s->cfg.ws_budget;
    for (fbpq_index *lane : s->lanes) s->workers.emplace_back(worker, s, lane);
    *out = s;
    return FBPQ_OK;
}

int fbpq_server_create(fbpq_index *ix, int32_t max_batch, int32_t nlanes, int32_t k_max, fbpq_server **out)
{
    if (!ix) return FBPQ_E_INVALID;
    fbpq_server_config c{};
    c.max_batch = max_batch;
    c.nlanes = nlanes;
    c.k_max = k_max;
    return fbpq_server_create2(ix, &c, out);
}

int fbpq_server_submit(fbpq_server *s, const float *q, int64_t L, int32_t k, int64_t tag)
{
    if (!s || !q || L < 1 || k < 1 || k > s->cfg.k_max) return FBPQ_E_INVALID;
    Req r;
    r.tag = tag;
    r.L = L;
    r.k = k;
    r.bucket = lbucket(L, s->N);
    r.reserve = s->ix ? search_ws_estimate(s->ix, L, k) : 64 * std::min(L, (int64_t)1 << 40) + 4096;
    r.q.assign(q, q + s->cfg.D);
    r.t_submit = now_s();
    r.deadline = s->cfg.timeout_s > 0 ? r.t_submit + s->cfg.timeout_s : 0.0;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return FBPQ_E_STATE;
        if (r.reserve > s->lane_budget || (int64_t)s->pending.size() >= s->cfg.max_pending) {
            ++s->st[FBPQ_SERVER_STAT_REJECTED];
            return FBPQ_E_CAPACITY;
        }
        ++s->st[FBPQ_SERVER_STAT_SUBMITTED];
        s->pending.push_back(std::move(r));
    }
    s->cv_work.notify_one();
    return FBPQ_OK;
}

int fbpq_server_cancel(fbpq_server *s, int64_t tag)
{
    if (!s) return FBPQ_E_INVALID;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        auto it = std::find_if(s->pending.begin(), s->pending.end(), [&](const Req &r) { return r.tag == tag; });
        if (it == s->pending.end()) return FBPQ_E_STATE;  // running, finished or unknown
        finish_unrun(s, *it, FBPQ_E_CANCELLED, now_s());
        ++s->st[FBPQ_SERVER_STAT_CANCELLED];
        s->pending.erase(it);
    }
    s->cv_done.notify_all();
    return FBPQ_OK;
}

int fbpq_server_poll(fbpq_server *s, int32_t max_n, double wait_s, int64_t *tags, int64_t *ids, float *dists,
                     double *times, int32_t *status, int32_t *n_out)
{
    if (!s || max_n < 0 || !n_out || (max_n > 0 && (!tags || !ids || !dists || !times || !status)))
        return FBPQ_E_INVALID;
    std::unique_lock<std::mutex> lk(s->mu);
    expire_locked(s, now_s());
    if (s->done.empty() && wait_s > 0) {
        const auto until = std::chrono::steady_clock::now() + std::chrono::duration<double>(wait_s);
        while (s->done.empty()) {
            // wake at the earliest queued deadline too, so timeouts complete while lanes are busy
            auto wake = until;
            for (const Req &r : s->pending)
                if (r.deadline > 0) {
                    const auto t = std::chrono::steady_clock::time_point(std::chrono::duration_cast<
                        std::chrono::steady_clock::duration>(std::chrono::duration<double>(r.deadline)));
                    if (t < wake) wake = t;
                }
            if (s->cv_done.wait_until(lk, wake) == std::cv_status::timeout) {
                expire_locked(s, now_s());
                if (std::chrono::steady_clock::now() >= until) break;
            }
        }
    }
    int32_t n = 0;
    const int32_t km = s->cfg.k_max;
    while (n < max_n && !s->done.empty()) {
        Done &r = s->done.front();
        tags[n] = r.tag;
        status[n] = r.rc;
        std::copy(r.ids.begin(), r.ids.end(), ids + (int64_t)n * km);
        std::copy(r.d.begin(), r.d.end(), dists + (int64_t)n * km);
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
    *batches = s->st[FBPQ_SERVER_STAT_BATCHES];
    *batched = s->st[FBPQ_SERVER_STAT_BATCHED];
    return FBPQ_OK;
}

int fbpq_server_stats(fbpq_server *s, int64_t *out, int32_t n)
{
    if (!s || !out || n < 0) return FBPQ_E_INVALID;
    std::lock_guard<std::mutex> lk(s->mu);
    s->st[FBPQ_SERVER_STAT_PENDING] = (int64_t)s->pending.size();
    s->st[FBPQ_SERVER_STAT_LANE_BUDGET] = s->lane_budget;
    for (int32_t i = 0; i < n && i < FBPQ_SERVER_NUM_STATS; ++i) out[i] = s->st[i];
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
    s->cv_work.notify_all();
    s->cv_done.notify_all();
    for (std::thread &t : s->workers) t.join();
    for (fbpq_index *lane : s->lanes)
        if (lane) fbpq_free_index(lane);
    delete s;
}

}  // extern "C"
