// server.cpp -- the query server (imm_server_*): continuous batching of IMM
// queries on one device. A worker thread owns an AsyncRunner: every admitted
// query runs its own pipeline (sampling round, selection, theta decision) on
// one of the server's streams, so queries overlap on the GPU and none waits
// for another's rounds. Between polls of the runner the worker admits queued
// queries (slots and device memory permitting), drops cancelled ones and
// hands finished results to pollers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <deque>
#include <map>
#include <memory>
#include <new>
#include <string>
#include <thread>
#include <vector>

#include "engine.hpp"

using namespace imm;

namespace {

constexpr uint32_t kServerStreams = 8;

struct Entry {
    imm_graph* g = nullptr;
    imm_params p{};
    uint64_t reserve = 0;
    double t_submit = 0, t_admit = 0;
    Query* q = nullptr;  // once started
    bool cancel = false;
    bool finished = false;
    imm_status status = IMM_OK;
    std::string err;
    imm_result* r = nullptr;
};

uint64_t estimate_bytes(const imm_graph* g, const imm_params& p) {
    uint64_t e = g->peak_bytes.load();
    if (e == 0) e = (uint64_t)g->n * 64 + (1ull << 30);
    if (p.max_device_bytes && p.max_device_bytes < e) e = p.max_device_bytes;
    return e;
}

}  // namespace

struct imm_server {
    int device = 0;
    uint64_t budget = 0;
    uint32_t max_slots = 1;
    std::thread worker;
    std::mutex mu;
    std::condition_variable wake;      // the worker: new work or stop
    std::condition_variable finished;  // pollers
    bool stop = false;
    uint64_t next_ticket = 1;
    std::map<uint64_t, Entry> entries;
    std::deque<uint64_t> queue;  // submitted, not admitted
    uint32_t running = 0;
    uint64_t reserved = 0;
    std::vector<imm_graph*> graphs;  // every graph a query was submitted on

    void run();
    void complete(uint64_t t, Entry& e, imm_status st, const std::string& err, imm_result* r);
};

// Under mu.
void imm_server::complete(uint64_t, Entry& e, imm_status st, const std::string& err,
                          imm_result* r) {
    const double t = now_ms();
    e.status = st;
    e.err = err;
    e.r = r;
    if (r) {
        r->stats.ms_total = t - e.t_submit;
        r->stats.ms_queue = e.t_admit - e.t_submit;
    }
    e.finished = true;
    e.q = nullptr;
    finished.notify_all();
}

void imm_server::run() {
    (void)hipSetDevice(device);
    hipStream_t st[kServerStreams] = {};
    bool ok = true;
    for (uint32_t i = 0; ok && i < kServerStreams; ++i)
        ok = hipStreamCreateWithFlags(&st[i], hipStreamNonBlocking) == hipSuccess;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    const uint32_t big_cap = max_slots > 1 ? std::max<uint32_t>(64u, (uint32_t)cus * 8u / max_slots) : 0u;
    std::unique_ptr<AsyncRunner> br(ok ? new AsyncRunner() : nullptr);
    std::map<Query*, uint64_t> owner;  // running query -> ticket
    uint32_t rr = 0;
    for (;;) {
        std::vector<uint64_t> admit;
        {
            std::unique_lock<std::mutex> lk(mu);
            for (;;) {
                if (stop) {
                    for (auto& kv : owner) entries[kv.second].cancel = true;
                }
                // admission at the iteration boundary: the running queries'
                // reservations and the idle workspaces cached on the server's
                // graphs must leave room for the query's estimate; the caches
                // are emptied first when they are what stands in the way
                while (!stop && !queue.empty() && running < max_slots) {
                    const uint64_t t = queue.front();
                    Entry& e = entries[t];
                    uint64_t cached = 0;
                    for (imm_graph* g : graphs) cached += cached_bytes(g);
                    if (reserved + cached + e.reserve > budget && cached) {
                        for (imm_graph* g : graphs) trim_cache(g);
                        cached = 0;
                    }
                    if (running > 0 && reserved + cached + e.reserve > budget) break;
                    queue.pop_front();
                    ++running;
                    reserved += e.reserve;
                    e.t_admit = now_ms();
                    admit.push_back(t);
                }
                if (!ok) {
                    // no streams: every query fails
                    for (uint64_t t : admit) {
                        complete(t, entries[t], IMM_EDEVICE, "server: stream creation failed", nullptr);
                        --running;
                        reserved -= entries[t].reserve;
                    }
                    admit.clear();
                }
                if (running > 0 || !admit.empty()) break;
                if (stop) break;
                wake.wait(lk);
            }
            if (stop && running == 0 && admit.empty()) break;
            // cancellations of running queries
            for (auto& kv : owner)
                if (entries[kv.second].cancel) br->cancel(kv.first);
        }
        // start what was admitted (tuning and allocation happen here)
        for (uint64_t t : admit) {
            imm_graph* g;
            imm_params p;
            {
                std::lock_guard<std::mutex> lk(mu);
                g = entries[t].g;
                p = entries[t].p;
            }
            Query* q = br->start(g, p, st[rr++ % kServerStreams], big_cap);
            if (BatchRunner::done(q)) {
                imm_status s;
                std::string err;
                imm_result* r = BatchRunner::take(q, &s, &err);
                std::lock_guard<std::mutex> lk(mu);
                Entry& e = entries[t];
                reserved -= e.reserve;
                --running;
                complete(t, e, s, err, r);
            } else {
                owner[q] = t;
                std::lock_guard<std::mutex> lk(mu);
                entries[t].q = q;
            }
        }
        bool advanced = false;
        try {
            advanced = br->poll();
        } catch (...) {
        }
        for (Query* q : br->drain()) {
            const uint64_t t = owner[q];
            owner.erase(q);
            const uint64_t bytes = BatchRunner::bytes(q);
            imm_status s;
            std::string err;
            imm_graph* g;
            {
                std::lock_guard<std::mutex> lk(mu);
                g = entries[t].g;
            }
            imm_result* r = BatchRunner::take(q, &s, &err);
            (void)g;
            (void)bytes;
            std::lock_guard<std::mutex> lk(mu);
            Entry& e = entries[t];
            reserved -= e.reserve;
            --running;
            complete(t, e, s, err, r);
            advanced = true;
        }
        // nothing finished on the GPU since the last look: let it work
        if (!advanced) std::this_thread::sleep_for(std::chrono::microseconds(20));
    }
    br.reset();
    for (auto s2 : st)
        if (s2) (void)hipStreamDestroy(s2);
}

extern "C" {

imm_status imm_server_create(uint64_t budget_bytes, uint32_t max_slots, imm_server** out) {
    if (!out || budget_bytes == 0 || max_slots == 0)
        return fail(IMM_EINVAL, "server_create: need budget > 0, max_slots >= 1, out");
    try {
        std::unique_ptr<imm_server> s(new imm_server());
        HIP_TRY(hipGetDevice(&s->device));
        s->budget = budget_bytes;
        s->max_slots = max_slots;
        imm_server* raw = s.get();
        s->worker = std::thread([raw] { raw->run(); });
        *out = s.release();
        return IMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(IMM_ENOMEM, "server_create: host allocation failed");
    } catch (...) {
        return fail(IMM_EDEVICE, "server_create: could not start the worker");
    }
}

imm_status imm_server_submit(imm_server* s, const imm_graph* g, const imm_params* p,
                             uint64_t* ticket) {
    if (!s || !g || !p || !ticket) return fail(IMM_EINVAL, "server_submit: null argument");
    if (g->device != s->device) return fail(IMM_EINVAL, "server_submit: graph on another device");
    if (p->k == 0 || p->k > g->n) return fail(IMM_EINVAL, "server_submit: need 1 <= k <= n");
    if (!(p->epsilon > 0.0) || !(p->ell > 0.0))
        return fail(IMM_EINVAL, "server_submit: need eps > 0, ell > 0");
    try {
        Entry e;
        e.g = const_cast<imm_graph*>(g);
        e.p = *p;
        e.reserve = estimate_bytes(g, *p);
        if (e.reserve > s->budget)
            return fail(IMM_ENOMEM, "server_submit: the query's estimated workspace exceeds the budget");
        e.t_submit = now_ms();
        std::lock_guard<std::mutex> lk(s->mu);
        if (s->stop) return fail(IMM_EINVAL, "server_submit: server is shutting down");
        const uint64_t t = s->next_ticket++;
        if (std::find(s->graphs.begin(), s->graphs.end(), e.g) == s->graphs.end())
            s->graphs.push_back(e.g);
        s->entries.emplace(t, std::move(e));
        s->queue.push_back(t);
        *ticket = t;
        s->wake.notify_one();
        return IMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(IMM_ENOMEM, "server_submit: host allocation failed");
    }
}

imm_status imm_server_poll(imm_server* s, uint64_t ticket, int wait, imm_result** out) {
    if (!s || !out) return fail(IMM_EINVAL, "server_poll: null argument");
    std::unique_lock<std::mutex> lk(s->mu);
    auto it = s->entries.find(ticket);
    if (it == s->entries.end()) return fail(IMM_EINVAL, "server_poll: unknown ticket");
    if (!it->second.finished) {
        if (!wait) return fail(IMM_EBUSY, "server_poll: query not finished");
        s->finished.wait(lk, [&] { return it->second.finished; });
    }
    Entry e = std::move(it->second);
    s->entries.erase(it);
    lk.unlock();
    if (e.status != IMM_OK) {
        delete e.r;
        return fail(e.status, e.err.empty() ? "server: query failed" : e.err);
    }
    *out = e.r;
    return IMM_OK;
}

imm_status imm_server_cancel(imm_server* s, uint64_t ticket) {
    if (!s) return fail(IMM_EINVAL, "server_cancel: null server");
    std::lock_guard<std::mutex> lk(s->mu);
    auto it = s->entries.find(ticket);
    if (it == s->entries.end()) return fail(IMM_EINVAL, "server_cancel: unknown ticket");
    Entry& e = it->second;
    if (e.finished) return IMM_OK;
    for (auto qi = s->queue.begin(); qi != s->queue.end(); ++qi) {
        if (*qi == ticket) {
            s->queue.erase(qi);
            s->complete(ticket, e, IMM_ECANCELLED, "cancelled", nullptr);
            return IMM_OK;
        }
    }
    e.cancel = true;  // running: dropped at the next iteration boundary
    s->wake.notify_one();
    return IMM_OK;
}

imm_status imm_server_info(imm_server* s, uint64_t* queued, uint32_t* running,
                           uint64_t* reserved_bytes) {
    if (!s) return fail(IMM_EINVAL, "server_info: null server");
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued) *queued = s->queue.size();
    if (running) *running = s->running;
    if (reserved_bytes) *reserved_bytes = s->reserved;
    return IMM_OK;
}

imm_status imm_server_destroy(imm_server* s) {
    if (!s) return fail(IMM_EINVAL, "server_destroy: null server");
    {
        std::lock_guard<std::mutex> lk(s->mu);
        s->stop = true;
        while (!s->queue.empty()) {
            const uint64_t t = s->queue.front();
            s->queue.pop_front();
            s->complete(t, s->entries[t], IMM_ECANCELLED, "cancelled", nullptr);
        }
        s->wake.notify_one();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto& kv : s->entries) delete kv.second.r;
    delete s;
    return IMM_OK;
}

}  // extern "C"
