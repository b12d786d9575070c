// Counting service with continuous batching (host side of bbc_server_*).
//
// Jobs are signed bipartite graphs submitted at any time.  Worker threads,
// each with its own context (device workspace and HIP stream, default
// priority), run them while more arrive:
//   * one batching worker takes every small job waiting at the moment it
//     becomes free and counts them with one bbc_count_batch call (one union
//     graph, one persistent wedge launch); jobs that arrive meanwhile form the
//     next batch;
//   * large-graph workers run one bbc_count each, concurrently on their own
//     streams, so their kernels overlap on the device with the batches.
// Admission against the device memory the workers really hold.  Each worker's
// context keeps its arenas between jobs (no allocation for a job that fits
// them), so the server reserves, per worker, what its arenas hold when idle and,
// while it runs jobs, the larger of that and the jobs' estimated footprint
// (input copy plus bbc_workspace_bytes) -- its grant.  The context's arenas
// are capped at the grant for the run, so they can never outgrow it.  A worker
// starts jobs only while the sum of the reservations stays within the memory
// budget.  A job whose estimate turns out too small (the planner's work lists
// grow with the graph's wedges, which the estimate cannot see) fails inside
// the grant and is queued again with its footprint raised to what it asked
// for.  A worker whose job waits for memory, or that finishes while another
// job waits, releases its arenas.  A job larger than the whole budget fails
// with BBC_ERR_OUT_OF_MEMORY.
#include <hip/hip_runtime.h>
#include <string.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <vector>

#include "bbc.h"
#include "bbc_internal.h"

namespace {

using Clock = std::chrono::steady_clock;

struct Job {
    uint64_t id = 0;
    int32_t n_u = 0, n_v = 0;
    std::vector<int32_t> eu, ev;
    std::vector<int8_t> sg;
    uint64_t footprint = 0;
    Clock::time_point t_submit, t_start, t_done;
    bbc_result res = {0, 0, 0};
    int32_t status = BBC_OK;
    bool done = false;
    bool batched = false;
};

}  // namespace

struct bbc_server {
    bbc_server_config cfg;
    std::mutex mu;
    std::condition_variable cv_work;  // queues changed or memory freed
    std::condition_variable cv_done;  // a job finished
    std::deque<Job*> q_small, q_large;
    std::unordered_map<uint64_t, Job*> jobs;
    uint64_t next_id = 1;
    uint64_t budget = 0, reserved = 0, peak_reserved = 0;
    std::vector<uint64_t> held;  // per worker: bytes reserved for it (see the top of this file)
    std::vector<char> idle;      // per worker: waiting for jobs
    bool mem_blocked = false;    // a queued job is waiting for memory
    int64_t trims = 0, retries = 0;
    int running = 0, peak_running = 0;
    int64_t submitted = 0, completed = 0, batches = 0, batched_jobs = 0, max_batch = 0;
    bool stop = false;
    std::vector<bbc_context*> ctx;
    std::vector<std::thread> workers;
};

namespace {

int64_t elapsed_us(Clock::time_point a, Clock::time_point b) {
    return std::chrono::duration_cast<std::chrono::microseconds>(b - a).count();
}

// Take jobs from q (front first) for worker w while the reservations fit the
// budget; at most max_jobs and max_edges.  Jobs that can never fit fail here.
// On success the worker's reservation becomes its grant, returned in *grant.
std::vector<Job*> take_jobs(bbc_server* s, std::deque<Job*>& q, size_t max_jobs, uint64_t max_edges,
                            int w, uint64_t* grant) {
    std::vector<Job*> out;
    uint64_t fp = 0, edges = 0;
    while (!q.empty() && out.size() < max_jobs) {
        Job* j = q.front();
        if (j->footprint > s->budget) {  // larger than the whole budget
            q.pop_front();
            j->status = BBC_ERR_OUT_OF_MEMORY;
            j->t_start = j->t_done = Clock::now();
            j->done = true;
            s->completed++;
            s->cv_done.notify_all();
            continue;
        }
        const uint64_t m = j->eu.size();
        if (!out.empty() && edges + m > max_edges) break;
        const uint64_t g = std::max(s->held[w], fp + j->footprint);
        if (s->reserved - s->held[w] + g > s->budget) {  // wait for memory
            s->mem_blocked = true;
            break;
        }
        q.pop_front();
        out.push_back(j);
        fp += j->footprint;
        edges += m;
    }
    if (!out.empty()) {
        const uint64_t g = std::max(s->held[w], fp);
        s->reserved += g - s->held[w];
        s->held[w] = g;
        *grant = g;
        s->peak_reserved = std::max(s->peak_reserved, s->reserved);
        s->running += (int)out.size();
        s->peak_running = std::max(s->peak_running, s->running);
        const auto now = Clock::now();
        for (Job* j : out) j->t_start = now;
    }
    return out;
}

// Wait (with the lock held) until worker w's queue yields jobs; an idle worker
// releases its arenas while a job waits for memory.  Returns no jobs once the
// server stops and the queue is empty.
std::vector<Job*> next_jobs(bbc_server* s, std::unique_lock<std::mutex>& lk, std::deque<Job*>& q,
                            size_t max_jobs, uint64_t max_edges, int w, bbc_context* ctx,
                            uint64_t* grant) {
    for (;;) {
        if (!q.empty()) {
            std::vector<Job*> js = take_jobs(s, q, max_jobs, max_edges, w, grant);
            if (!js.empty()) {
                s->idle[w] = 0;
                return js;
            }
            // blocked on memory: wake idle workers that hold arenas, so they release them
            bool holder = false;
            for (size_t x = 0; x < s->held.size(); ++x)
                holder = holder || ((int)x != w && s->idle[x] && s->held[x] > 0);
            if (s->mem_blocked && holder) s->cv_work.notify_all();
        }
        s->idle[w] = 1;
        if (s->stop && q.empty()) return {};
        if (s->mem_blocked && s->held[w] > 0) {
            lk.unlock();
            const bool ok = bbc::context_trim(ctx);
            lk.lock();
            if (ok) {
                s->reserved -= s->held[w];
                s->held[w] = 0;
                s->trims++;
            }
            s->mem_blocked = false;  // the waiting jobs look again
            s->cv_work.notify_all();
            continue;
        }
        s->cv_work.wait(lk);
    }
}

// After worker w ran `js` within `grant` (call status rc): jobs that failed only
// because their estimate was below what the count asked for go back to the
// front of their queue with a raised footprint; the rest are done.  The
// worker's reservation becomes what its arenas now hold, or zero when it
// releases them because a job waits for memory.
void finish(bbc_server* s, std::vector<Job*>& js, bbc_context* ctx, int w, uint64_t grant,
            bbc_status rc, std::deque<Job*>& q) {
    const uint64_t need = bbc::context_last_need(ctx);
    const bool retry = rc == BBC_ERR_OUT_OF_MEMORY && need > grant && grant > 0;
    bbc::context_set_budget(ctx, 0);
    uint64_t resident = bbc::context_resident_bytes(ctx);
    bool trim;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        trim = s->mem_blocked || retry;
    }
    if (trim && bbc::context_trim(ctx)) resident = 0;
    std::lock_guard<std::mutex> lk(s->mu);
    const auto now = Clock::now();
    if (trim && resident == 0) s->trims++;
    s->reserved = s->reserved - s->held[w] + resident;
    s->held[w] = resident;
    s->running -= (int)js.size();
    if (retry) {
        s->retries++;
        for (auto it = js.rbegin(); it != js.rend(); ++it) {
            Job* j = *it;
            j->footprint = (uint64_t)((double)j->footprint * (double)need / (double)grant) + 1;
            j->status = BBC_OK;
            q.push_front(j);
        }
    } else {
        for (Job* j : js) {
            j->t_done = now;
            j->done = true;
            s->completed++;
        }
    }
    s->mem_blocked = false;  // memory changed: waiting jobs look again
    s->cv_done.notify_all();
    s->cv_work.notify_all();
}

void batch_worker(bbc_server* s, bbc_context* ctx) {
    std::vector<int32_t> nu, nv, eu, ev;
    std::vector<int8_t> sg;
    std::vector<int64_t> off;
    std::vector<bbc_result> res;
    std::vector<int32_t> st;
    for (;;) {
        std::vector<Job*> js;
        uint64_t grant = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            js = next_jobs(s, lk, s->q_small, (size_t)s->cfg.max_batch_graphs, 1ull << 30, 0, ctx,
                           &grant);
            if (js.empty()) return;
            s->batches++;
            s->batched_jobs += (int64_t)js.size();
            s->max_batch = std::max<int64_t>(s->max_batch, (int64_t)js.size());
        }
        const size_t G = js.size();
        nu.resize(G);
        nv.resize(G);
        off.assign(G + 1, 0);
        for (size_t i = 0; i < G; ++i) {
            nu[i] = js[i]->n_u;
            nv[i] = js[i]->n_v;
            off[i + 1] = off[i] + (int64_t)js[i]->eu.size();
        }
        eu.resize((size_t)off[G]);
        ev.resize((size_t)off[G]);
        sg.resize((size_t)off[G]);
        for (size_t i = 0; i < G; ++i) {
            const size_t m = js[i]->eu.size();
            if (!m) continue;
            memcpy(eu.data() + off[i], js[i]->eu.data(), 4 * m);
            memcpy(ev.data() + off[i], js[i]->ev.data(), 4 * m);
            memcpy(sg.data() + off[i], js[i]->sg.data(), m);
        }
        res.assign(G, bbc_result{0, 0, 0});
        st.assign(G, BBC_OK);
        bbc::context_set_budget(ctx, grant);
        const bbc_status rc = bbc_count_batch(ctx, (int32_t)G, nu.data(), nv.data(), off.data(),
                                              eu.data(), ev.data(), sg.data(), 0, res.data(),
                                              st.data());
        const bool retry = rc == BBC_ERR_OUT_OF_MEMORY && bbc::context_last_need(ctx) > grant;
        for (size_t i = 0; i < G && !retry; ++i) {
            js[i]->status = rc == BBC_OK ? st[i] : rc;
            js[i]->res = rc == BBC_OK ? res[i] : bbc_result{0, 0, 0};
            js[i]->batched = true;
            js[i]->eu.clear();
            js[i]->eu.shrink_to_fit();
            js[i]->ev.clear();
            js[i]->ev.shrink_to_fit();
            js[i]->sg.clear();
            js[i]->sg.shrink_to_fit();
        }
        finish(s, js, ctx, 0, grant, rc, s->q_small);
    }
}

void large_worker(bbc_server* s, bbc_context* ctx, int w) {
    for (;;) {
        std::vector<Job*> js;
        uint64_t grant = 0;
        {
            std::unique_lock<std::mutex> lk(s->mu);
            js = next_jobs(s, lk, s->q_large, 1, ~0ull, w, ctx, &grant);
            if (js.empty()) return;
        }
        Job* j = js[0];
        bbc_result r = {0, 0, 0};
        bbc::context_set_budget(ctx, grant);
        const bbc_status rc = bbc_count(ctx, j->n_u, j->n_v, (int64_t)j->eu.size(), j->eu.data(),
                                        j->ev.data(), j->sg.data(), 0, &r, nullptr);
        const bool retry = rc == BBC_ERR_OUT_OF_MEMORY && bbc::context_last_need(ctx) > grant;
        if (!retry) {
            j->status = rc;
            j->res = rc == BBC_OK ? r : bbc_result{0, 0, 0};
            j->eu.clear();
            j->eu.shrink_to_fit();
            j->ev.clear();
            j->ev.shrink_to_fit();
            j->sg.clear();
            j->sg.shrink_to_fit();
        }
        finish(s, js, ctx, w, grant, rc, s->q_large);
    }
}

}  // namespace

extern "C" {

bbc_status bbc_server_create(const bbc_server_config* cfg, bbc_server** out) {
    if (!out) return BBC_ERR_INVALID_ARG;
    *out = nullptr;
    bbc_server_config c = {0, 2, 0, 0, 0};
    if (cfg) c = *cfg;
    if (c.large_workers < 0 || c.large_workers > 16 || c.memory_budget < 0 || c.small_side < 0 ||
        c.small_side > 16384 || c.max_batch_graphs < 0)
        return BBC_ERR_INVALID_ARG;
    if (c.large_workers == 0) c.large_workers = 2;
    if (c.small_side == 0) c.small_side = 16384;
    if (c.max_batch_graphs == 0) c.max_batch_graphs = 65536;
    bbc_server* s = new bbc_server();
    s->cfg = c;
    if (hipSetDevice(c.device) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return BBC_ERR_DEVICE;
    }
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) {
        (void)hipGetLastError();
        delete s;
        return BBC_ERR_DEVICE;
    }
    s->budget = c.memory_budget ? (uint64_t)c.memory_budget : (uint64_t)(free_b * 0.9);
    for (int i = 0; i < 1 + c.large_workers; ++i) {
        bbc_context* ctx = nullptr;
        const bbc_status rc = bbc_create(c.device, nullptr, &ctx);
        if (rc != BBC_OK) {
            for (bbc_context* x : s->ctx) bbc_destroy(x);
            delete s;
            return rc;
        }
        s->ctx.push_back(ctx);
    }
    s->held.assign(s->ctx.size(), 0);
    s->idle.assign(s->ctx.size(), 1);
    s->workers.emplace_back(batch_worker, s, s->ctx[0]);
    for (int i = 0; i < c.large_workers; ++i)
        s->workers.emplace_back(large_worker, s, s->ctx[1 + i], 1 + i);
    *out = s;
    return BBC_OK;
}

bbc_status bbc_server_submit(bbc_server* s, int32_t n_u, int32_t n_v, int64_t n_edges,
                             const int32_t* edge_u, const int32_t* edge_v,
                             const int8_t* edge_sign, uint64_t* ticket) {
    if (!s || !ticket || n_u < 0 || n_v < 0 || n_edges < 0) return BBC_ERR_INVALID_ARG;
    if (n_edges > 0 && (!edge_u || !edge_v || !edge_sign)) return BBC_ERR_INVALID_ARG;
    const int64_t fp = bbc_workspace_bytes(n_u, n_v, n_edges);
    if (fp < 0) return BBC_ERR_TOO_LARGE;
    Job* j = new Job();
    j->t_submit = Clock::now();  // arrival: the input copy below counts toward latency
    j->n_u = n_u;
    j->n_v = n_v;
    j->eu.assign(edge_u, edge_u + n_edges);
    j->ev.assign(edge_v, edge_v + n_edges);
    j->sg.assign(edge_sign, edge_sign + n_edges);
    // input copy on the device, plus the workspace
    j->footprint = (uint64_t)fp + 9ull * (uint64_t)n_edges;
    std::lock_guard<std::mutex> lk(s->mu);
    if (s->stop) {
        delete j;
        return BBC_ERR_INVALID_ARG;
    }
    j->id = s->next_id++;
    s->jobs[j->id] = j;
    s->submitted++;
    if (n_u <= s->cfg.small_side && n_v <= s->cfg.small_side)
        s->q_small.push_back(j);
    else
        s->q_large.push_back(j);
    *ticket = j->id;
    s->cv_work.notify_all();
    return BBC_OK;
}

bbc_status bbc_server_poll(bbc_server* s, uint64_t ticket, int32_t wait_ms, bbc_result* out,
                           int32_t* job_status, double* latency_ms) {
    if (!s || !out || !job_status) return BBC_ERR_INVALID_ARG;
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->jobs.find(ticket);
    if (it == s->jobs.end()) return BBC_ERR_INVALID_ARG;
    Job* j = it->second;
    if (!j->done && wait_ms != 0) {
        auto pred = [&] { return j->done; };
        if (wait_ms < 0)
            s->cv_done.wait(lk, pred);
        else
            s->cv_done.wait_for(lk, std::chrono::milliseconds(wait_ms), pred);
    }
    if (!j->done) return BBC_PENDING;
    *out = j->res;
    *job_status = j->status;
    if (latency_ms) *latency_ms = (double)elapsed_us(j->t_submit, j->t_done) / 1000.0;
    s->jobs.erase(it);
    delete j;
    return BBC_OK;
}

bbc_status bbc_server_stats(bbc_server* s, int64_t* stats, int n) {
    if (!s || !stats || n < 0) return BBC_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(s->mu);
    const int64_t v[12] = {s->submitted,
                           s->completed,
                           s->batches,
                           s->batched_jobs,
                           s->max_batch,
                           (int64_t)s->peak_reserved,
                           s->peak_running,
                           (int64_t)s->budget,
                           (int64_t)(s->q_small.size() + s->q_large.size()),
                           (int64_t)s->reserved,
                           s->trims,
                           s->retries};
    for (int i = 0; i < n && i < 12; ++i) stats[i] = v[i];
    return BBC_OK;
}

void bbc_server_destroy(bbc_server* s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        s->cv_work.notify_all();
    }
    for (std::thread& t : s->workers) t.join();
    for (bbc_context* c : s->ctx) bbc_destroy(c);
    for (auto& kv : s->jobs) delete kv.second;
    delete s;
}

}  // extern "C"
