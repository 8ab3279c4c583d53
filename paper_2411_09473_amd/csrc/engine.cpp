// engine.cpp -- libimm host engine and C ABI (include/imm.h).
//
// Owns device memory, sequences the kernels of one IMM run on the caller's
// stream and runs IMM's theta schedule (Algorithm 1 with the bounds of Tang
// et al. 2015) in FP64 on the host. Per sampling round the host reads back a
// handful of scalars (staging cursor, deferred/retried counts, pool size) and
// one coverage figure; everything else stays on the device.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "../../include/imm.h"
#include "imm_internal.hpp"

using namespace imm;

// ---------------------------------------------------------------- errors --

namespace {

thread_local std::string g_err;

imm_status fail(imm_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

struct Status {
    imm_status st = IMM_OK;
    bool ok() const { return st == IMM_OK; }
};

#define IMM_TRY(expr)                      \
    do {                                   \
        imm_status _s = (expr);            \
        if (_s != IMM_OK) return _s;       \
    } while (0)

#define HIP_TRY(expr)                                                                  \
    do {                                                                               \
        hipError_t _e = (expr);                                                        \
        if (_e != hipSuccess) {                                                        \
            return fail(_e == hipErrorOutOfMemory ? IMM_ENOMEM : IMM_EDEVICE,          \
                        std::string(#expr) + ": " + hipGetErrorString(_e));           \
        }                                                                              \
    } while (0)

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------ allocation --

// Device allocations of one owner, with an optional byte budget.
struct Arena {
    uint64_t budget = 0;  // 0: none
    uint64_t used = 0;
    std::vector<std::pair<void*, uint64_t>> live;

    imm_status alloc(void** p, uint64_t bytes, const char* what) {
        *p = nullptr;
        if (bytes == 0) bytes = 16;
        bytes = (bytes + 255) & ~uint64_t(255);
        if (budget && used + bytes > budget)
            return fail(IMM_ENOMEM, std::string("device budget exceeded allocating ") + what);
        hipError_t e = hipMalloc(p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            *p = nullptr;
            return fail(IMM_ENOMEM, std::string("hipMalloc failed for ") + what);
        }
        used += bytes;
        live.emplace_back(*p, bytes);
        return IMM_OK;
    }
    void release(void* p) {
        if (!p) return;
        for (size_t i = 0; i < live.size(); ++i) {
            if (live[i].first == p) {
                used -= live[i].second;
                (void)hipFree(p);
                live[i] = live.back();
                live.pop_back();
                return;
            }
        }
    }
    void release_all() {
        for (auto& x : live) (void)hipFree(x.first);
        live.clear();
        used = 0;
    }
    ~Arena() { release_all(); }
};

template <class T>
imm_status grow(Arena& a, T** p, uint64_t* cap, uint64_t need, uint64_t keep, hipStream_t st,
                const char* what) {
    if (*p && *cap >= need) return IMM_OK;
    uint64_t nc = std::max<uint64_t>(need, *cap + *cap / 2);
    if (nc < 64) nc = 64;
    T* q = nullptr;
    imm_status s = a.alloc(reinterpret_cast<void**>(&q), nc * sizeof(T), what);
    if (s != IMM_OK && nc > need) {
        nc = need;
        s = a.alloc(reinterpret_cast<void**>(&q), nc * sizeof(T), what);
    }
    IMM_TRY(s);
    if (*p && keep) HIP_TRY(hipMemcpyAsync(q, *p, keep * sizeof(T), hipMemcpyDeviceToDevice, st));
    if (*p) {
        HIP_TRY(hipStreamSynchronize(st));
        a.release(*p);
    }
    *p = q;
    *cap = nc;
    return IMM_OK;
}

// Upper bound on the device memory of the large-set kernels' scratch.
constexpr uint64_t kBigScratchBytes = 16ull << 30;

// Scalars the kernels update, in one device block.
struct DevScalars {
    unsigned long long cursor;
    uint32_t ticket_small, ticket_big, defer_n, retry_n, spare_n, big_flag;
    uint32_t err, pad;
    unsigned long long stats[kStCount];
};

// Phase timing with HIP events on the run's stream.
struct Timer {
    bool on = false;
    hipStream_t st = nullptr;
    struct Rec { int phase; hipEvent_t a, b; };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        (void)hipEventCreate(&e);
        return e;
    }
    int open(int phase) {
        if (!on) return -1;
        Rec r{phase, get(), get()};
        (void)hipEventRecord(r.a, st);
        recs.push_back(r);
        return (int)recs.size() - 1;
    }
    void close(int h) {
        if (h < 0) return;
        (void)hipEventRecord(recs[h].b, st);
    }
    // phases: 0 sample, 1 compact, 2 index, 3 select, 4 main sampling
    // kernel, 5 large-set sampling kernel
    void collect(double* ms, uint64_t* launches) {
        for (auto& r : recs) {
            float t = 0.f;
            if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&t, r.a, r.b) == hipSuccess)
                ms[r.phase] += t;
            if (r.phase >= 4) ++launches[r.phase - 4];
            pool.push_back(r.a);
            pool.push_back(r.b);
        }
        recs.clear();
    }
    ~Timer() {
        for (auto& r : recs) { (void)hipEventDestroy(r.a); (void)hipEventDestroy(r.b); }
        for (auto e : pool) (void)hipEventDestroy(e);
    }
};

}  // namespace

// ---------------------------------------------------------------- graph --

namespace {
struct Workspace;
}

struct imm_graph {
    uint32_t n = 0;
    uint64_t m = 0;
    imm_model model = IMM_IC;
    int device = 0;
    Arena arena;
    uint32_t* off = nullptr;
    uint32_t* thr = nullptr;
    uint32_t* src = nullptr;
    uint2* cs = nullptr;
    uint32_t* guide = nullptr;
    // workspace of the last run, reused by the next one
    std::mutex ws_mu;
    std::unique_ptr<Workspace> ws_cache;
};

namespace {

IcGraphDev ic_view(const imm_graph* g) {
    return IcGraphDev{g->off, g->thr, g->src, g->n, (uint32_t)g->m};
}
LtGraphDev lt_view(const imm_graph* g) {
    return LtGraphDev{g->off, g->cs, g->guide, g->n, (uint32_t)g->m};
}

// ------------------------------------------------------------- workspace --
//
// Device state of one IMM run (or of one imm_sample / imm_greedy call). A
// graph keeps the workspace of its last run and hands it to the next run, so
// repeated queries on a resident graph allocate nothing.
//
// The pool grows by whole sampling rounds. Its vertex->sets index is kept in
// segments, one per round, each indexing only that round's sets (segment r
// occupies inv_set positions [P_{r-1}, P_r), the same range its sets occupy
// in set_vtx), so no set is indexed twice.

struct Workspace {
    int device = 0;
    uint32_t n = 0;
    hipStream_t st = nullptr;
    Arena arena;
    DevScalars* sc = nullptr;
    DevScalars* hsc = nullptr;  // pinned mirror
    uint64_t* hp = nullptr;     // pinned: pool size
    uint32_t* herr = nullptr;   // pinned: error flag
    uint32_t* counts_acc = nullptr;   // occurrences over all sets so far
    uint32_t* counts_prev = nullptr;  // ... over the sets already indexed
    uint32_t* counts_work = nullptr;  // the greedy's working copy
    uint32_t* inv_cursor = nullptr;
    uint64_t* inv_offs = nullptr; uint64_t cap_offs = 0;  // nseg * (n+1)
    uint32_t nseg = 0;
    uint64_t indexed_sets = 0;
    uint64_t* set_off = nullptr; uint64_t cap_sets = 0;
    uint32_t* set_vtx = nullptr; uint64_t cap_entries = 0;
    uint32_t* inv_set = nullptr; uint64_t cap_inv = 0;
    uint32_t* covered = nullptr; uint64_t cap_cov = 0;
    uint32_t* stage = nullptr; uint64_t stage_cap = 0;
    uint64_t* stage_off = nullptr; uint64_t cap_so = 0;
    uint32_t* sizes = nullptr; uint64_t cap_sz = 0;
    uint32_t* defer = nullptr; uint64_t cap_df = 0;
    uint32_t* retry = nullptr; uint64_t cap_rt = 0;
    uint32_t* spare = nullptr; uint64_t cap_sp = 0;  // third list for retry passes
    uint64_t* scan_tmp = nullptr; uint64_t cap_scan = 0;
    unsigned long long* slots = nullptr;  // k * kArgSlots partial maxima
    uint32_t* chunk_n = nullptr;          // k queue lengths
    Chunk* chunks = nullptr; uint64_t cap_chunks = 0;
    uint32_t* seeds_d = nullptr; uint32_t* gains_d = nullptr; uint64_t cap_k = 0;
    uint32_t* gains_h = nullptr;
    uint32_t* big = nullptr; uint32_t big_slots = 0;
    uint64_t n_sets = 0;
    uint64_t p_exact = 0;  // pool size, exact as of the last synchronisation
    uint64_t p_ub = 0;     // upper bound on the pool size
    double mean_size = 0.0;  // mean set size of the last round (staging estimate)
    Timer timer;

    ~Workspace() {
        // kernels of a failed call may still be queued on the workspace's
        // buffers; the caller's stream may already be gone, so wait for the
        // whole device before the arena frees them
        if (sc) (void)hipDeviceSynchronize();
        if (hsc) (void)hipHostFree(hsc);
        if (hp) (void)hipHostFree(hp);
        if (herr) (void)hipHostFree(herr);
        if (gains_h) (void)hipHostFree(gains_h);
    }
};

imm_status ws_init(Workspace& w, uint32_t n, int device, hipStream_t st, uint64_t budget) {
    w.device = device;
    w.n = n;
    w.st = st;
    w.arena.budget = budget;
    IMM_TRY(w.arena.alloc((void**)&w.sc, sizeof(DevScalars), "scalars"));
    HIP_TRY(hipHostMalloc((void**)&w.hsc, sizeof(DevScalars), hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void**)&w.hp, 8, hipHostMallocDefault));
    HIP_TRY(hipHostMalloc((void**)&w.herr, 4, hipHostMallocDefault));
    IMM_TRY(w.arena.alloc((void**)&w.counts_acc, (uint64_t)n * 4, "counts"));
    IMM_TRY(w.arena.alloc((void**)&w.counts_prev, (uint64_t)n * 4, "counts (indexed)"));
    IMM_TRY(w.arena.alloc((void**)&w.counts_work, (uint64_t)n * 4 + 16, "counts_work"));
    IMM_TRY(w.arena.alloc((void**)&w.inv_cursor, (uint64_t)n * 4, "inv_cursor"));
    IMM_TRY(grow(w.arena, &w.set_off, &w.cap_sets, 1024, 0, st, "set_off"));
    return IMM_OK;
}

// Start a new run on an (initialised, possibly reused) workspace.
imm_status ws_reset(Workspace& w, hipStream_t st, bool timing) {
    w.st = st;
    w.timer.st = st;
    w.timer.on = timing;
    w.timer.recs.clear();
    w.n_sets = 0;
    w.p_exact = 0;
    w.p_ub = 0;
    w.nseg = 0;
    w.indexed_sets = 0;
    HIP_TRY(hipMemsetAsync(w.sc, 0, sizeof(DevScalars), st));
    HIP_TRY(hipMemsetAsync(w.counts_acc, 0, (uint64_t)w.n * 4, st));
    HIP_TRY(hipMemsetAsync(w.counts_prev, 0, (uint64_t)w.n * 4, st));
    HIP_TRY(hipMemsetAsync(w.set_off, 0, 8, st));
    return IMM_OK;
}

imm_status ws_read_scalars(Workspace& w) {
    HIP_TRY(hipMemcpyAsync(w.hsc, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, w.st));
    HIP_TRY(hipStreamSynchronize(w.st));
    return IMM_OK;
}

// Scratch of the large-set kernels: per slot a visited bitmap and a queue
// of n entries; enough slots to fill the GPU (IC) or a few per CU (LT, whose
// walks rarely outgrow a chunk), within kBigScratchBytes and the budget.
imm_status ws_big_scratch(Workspace& w, imm_model model) {
    if (w.big) return IMM_OK;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, w.device);
    const uint64_t words = ((uint64_t)w.n + 31) / 32;
    const uint64_t per = (words + w.n) * 4;
    uint64_t slots = model == IMM_IC ? (uint64_t)cus * 8 : (uint64_t)cus;
    uint64_t limit = kBigScratchBytes;
    if (w.arena.budget) {
        const uint64_t left = w.arena.budget > w.arena.used ? w.arena.budget - w.arena.used : 0;
        limit = std::min(limit, left / 4);
    }
    slots = std::min<uint64_t>(slots, std::max<uint64_t>(1, limit / per));
    IMM_TRY(w.arena.alloc((void**)&w.big, per * slots, "large-set scratch"));
    HIP_TRY(hipMemsetAsync(w.big, 0, words * slots * 4, w.st));
    w.big_slots = (uint32_t)slots;
    return IMM_OK;
}

BigScratch big_view(const Workspace& w) {
    const uint32_t words = (uint32_t)(((uint64_t)w.n + 31) / 32);
    return BigScratch{w.big, w.big + (uint64_t)words * w.big_slots, words, w.big_slots};
}

// Generate sample ids [id_lo, id_lo + count) into the pool at set index
// w.n_sets (Generate_RRRsets with fused counting), then compact them. One
// host synchronisation: after sampling, to learn whether any set is still
// waiting for staging space and how much staging was used.
imm_status ws_extend_once(Workspace& w, const imm_graph* g, uint64_t seed, uint64_t id_lo,
                          uint32_t count) {
    hipStream_t st = w.st;
    IMM_TRY(ws_big_scratch(w, g->model));
    IMM_TRY(grow(w.arena, &w.stage_off, &w.cap_so, count, 0, st, "stage_off"));
    IMM_TRY(grow(w.arena, &w.sizes, &w.cap_sz, count, 0, st, "sizes"));
    IMM_TRY(grow(w.arena, &w.defer, &w.cap_df, count, 0, st, "defer list"));
    IMM_TRY(grow(w.arena, &w.retry, &w.cap_rt, count, 0, st, "retry list"));
    IMM_TRY(grow(w.arena, &w.spare, &w.cap_sp, count, 0, st, "retry list"));
    {
        // expected entries plus the unused tails of every wave's (IC) or
        // lane's (LT) staging chunk
        const double mean = w.mean_size > 0 ? w.mean_size : 16.0;
        uint64_t tails;
        if (g->model == IMM_IC) {
            const uint64_t waves = std::min<uint64_t>(
                ic_small_grid(w.device), (count + kIcTicketChunk - 1) / kIcTicketChunk);
            tails = waves * kIcStageChunk;
        } else {
            const uint64_t lanes =
                std::min<uint64_t>((uint64_t)lt_small_grid(w.device) * 64u, count);
            tails = lanes * kLtChunk;
        }
        uint64_t want = (uint64_t)(mean * 1.5 * (double)count) + 2 * tails + 65536;
        // IMM_STAGE_SCALE (a factor, default 1) scales this first guess; small
        // values exercise the staging-growth path
        if (const char* e = std::getenv("IMM_STAGE_SCALE")) {
            const double f = std::atof(e);
            if (f > 0.0) want = std::max<uint64_t>(64, (uint64_t)((double)want * f));
        }
        IMM_TRY(grow(w.arena, &w.stage, &w.stage_cap, want, 0, st, "staging"));
    }
    HIP_TRY(hipMemsetAsync(w.sc, 0, offsetof(DevScalars, stats), st));

    // A pass runs the fast kernel over the range (list = nullptr) or over a
    // list of indices, then the large-set kernel over what it deferred.
    // Failures for lack of staging land in *fl; deferred sets in w.defer.
    auto pass = [&](const uint32_t* list, const uint32_t* list_n, uint32_t nitems, uint32_t* fl,
                    uint32_t* fl_n) -> imm_status {
        const SampleRange rg{seed, id_lo, nitems, list, list_n};
        const SampleRange rgl{seed, id_lo, count, nullptr, nullptr};
        const SampleOut o{w.stage, w.stage_cap, &w.sc->cursor, w.stage_off, w.sizes, w.counts_acc,
                          w.defer, &w.sc->defer_n, fl, fl_n, w.sc->stats};
        HIP_TRY(hipMemsetAsync(&w.sc->ticket_small, 0, 8, st));  // ticket_small, ticket_big
        HIP_TRY(hipMemsetAsync(&w.sc->defer_n, 0, 4, st));
        const int th = w.timer.open(0);
        const int tm = w.timer.open(4);
        if (g->model == IMM_IC)
            HIP_TRY(launch_ic_small(ic_view(g), rg, o, &w.sc->ticket_small, ic_small_grid(w.device), st));
        else
            HIP_TRY(launch_lt_small(lt_view(g), rg, o, &w.sc->ticket_small, lt_small_grid(w.device), st));
        w.timer.close(tm);
        const int t3 = w.timer.open(5);
        if (g->model == IMM_IC)
            HIP_TRY(launch_ic_large(ic_view(g), rgl, o, w.defer, &w.sc->defer_n, fl, fl_n,
                                    &w.sc->ticket_big, big_view(w), st));
        else
            HIP_TRY(launch_lt_large(lt_view(g), rgl, o, w.defer, &w.sc->defer_n, fl, fl_n,
                                    &w.sc->ticket_big, big_view(w), st));
        w.timer.close(t3);
        w.timer.close(th);
        return ws_read_scalars(w);
    };
    IMM_TRY(pass(nullptr, nullptr, count, w.retry, &w.sc->retry_n));

    // sets that found the staging buffer full: grow it (keeping what is
    // stored), continue at the old capacity, and redo just those sets
    uint32_t* in = w.retry;
    uint32_t* in_n = &w.sc->retry_n;
    uint32_t* out_l = w.spare;
    uint32_t* out_n = &w.sc->spare_n;
    uint32_t failed = w.hsc->retry_n;
    for (int guard = 0; failed; ++guard) {
        if (guard == 32) return fail(IMM_ENOMEM, "staging could not be grown enough");
        const uint64_t used = std::min<uint64_t>(w.hsc->cursor, w.stage_cap);
        const uint64_t old_cap = w.stage_cap;
        const double mean = w.mean_size > 0 ? w.mean_size : 64.0;
        uint64_t need = old_cap + (uint64_t)(mean * 2.0 * failed) + (uint64_t)failed * 64 + (1u << 20);
        need = std::max<uint64_t>(need, old_cap * 2);
        uint64_t cap = w.stage_cap;
        IMM_TRY(grow(w.arena, &w.stage, &cap, need, used, st, "staging"));
        w.stage_cap = cap;
        const unsigned long long cur = old_cap;
        HIP_TRY(hipMemcpyAsync(&w.sc->cursor, &cur, 8, hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemsetAsync(out_n, 0, 4, st));
        IMM_TRY(pass(in, in_n, failed, out_l, out_n));
        std::swap(in, out_l);
        std::swap(in_n, out_n);
        failed = (in == w.retry) ? w.hsc->retry_n : w.hsc->spare_n;
    }

    // compaction: set_off[n_sets .. n_sets+count] (based on the device copy of
    // set_off[n_sets]) and the copy into the pool
    const uint64_t stored_bound = std::min<uint64_t>(w.hsc->cursor, w.stage_cap);
    IMM_TRY(grow(w.arena, &w.set_off, &w.cap_sets, w.n_sets + count + 1, w.n_sets + 1, st, "set_off"));
    IMM_TRY(grow(w.arena, &w.set_vtx, &w.cap_entries, w.p_ub + stored_bound + 1,
                 std::min(w.p_ub, w.cap_entries), st, "set_vtx"));
    IMM_TRY(grow(w.arena, &w.scan_tmp, &w.cap_scan, scan_tmp_entries(count), 0, st, "scan tmp"));
    const int tc = w.timer.open(1);
    HIP_TRY(launch_scan_u32(w.sizes, nullptr, w.set_off + w.n_sets, count, 0, w.set_off + w.n_sets,
                            w.scan_tmp, st));
    HIP_TRY(launch_compact(w.stage, w.stage_off, w.set_off, w.n_sets, count, w.set_vtx, st));
    w.timer.close(tc);
    w.n_sets += count;
    w.p_ub += stored_bound;
    return IMM_OK;
}

imm_status ws_sync_pool(Workspace& w);
void ws_note_pool(Workspace& w, uint64_t sets_before);

// ws_extend_once for [id_lo, id_lo + count); when the workspace has no set
// size estimate yet, a pilot batch measures one before the rest is sized.
imm_status ws_extend(Workspace& w, const imm_graph* g, uint64_t seed, uint64_t id_lo,
                     uint64_t count64) {
    if (count64 == 0) return IMM_OK;
    if (count64 > 0xFFFFFFFFull) return fail(IMM_EOVERFLOW, "sampling round too large");
    uint32_t count = (uint32_t)count64;
    constexpr uint32_t kPilot = 1u << 16;
    if (w.mean_size <= 0.0 && count > 2 * kPilot) {
        const uint64_t before = w.n_sets;
        IMM_TRY(ws_extend_once(w, g, seed, id_lo, kPilot));
        IMM_TRY(ws_sync_pool(w));
        ws_note_pool(w, before);
        id_lo += kPilot;
        count -= kPilot;
    }
    return ws_extend_once(w, g, seed, id_lo, count);
}

// Read the exact pool size (and the device error flag) at a synchronisation.
imm_status ws_sync_pool(Workspace& w) {
    HIP_TRY(hipMemcpyAsync(w.hp, w.set_off + w.n_sets, 8, hipMemcpyDeviceToHost, w.st));
    HIP_TRY(hipMemcpyAsync(w.herr, &w.sc->err, 4, hipMemcpyDeviceToHost, w.st));
    HIP_TRY(hipStreamSynchronize(w.st));
    return IMM_OK;
}

void ws_note_pool(Workspace& w, uint64_t sets_before) {
    const uint64_t p = *w.hp;
    if (w.n_sets > sets_before)
        w.mean_size = (double)(p - w.p_exact) / (double)(w.n_sets - sets_before);
    w.p_exact = p;
    w.p_ub = p;
}

// Index the sets added since the last call as a new segment: its offsets are
// the scan of the count increase since then, based at the pool position of
// its first set.
imm_status ws_index_update(Workspace& w) {
    hipStream_t st = w.st;
    if (w.indexed_sets == w.n_sets) return IMM_OK;
    if (w.n_sets > 0xFFFFFFFFull) return fail(IMM_EOVERFLOW, "more than 2^32 sets");
    const uint64_t stride = (uint64_t)w.n + 1;
    IMM_TRY(grow(w.arena, &w.inv_offs, &w.cap_offs, (w.nseg + 1) * stride, w.nseg * stride, st,
                 "index offsets"));
    IMM_TRY(grow(w.arena, &w.inv_set, &w.cap_inv, w.p_ub + 1, std::min(w.p_ub, w.cap_inv), st,
                 "inv_set"));
    IMM_TRY(grow(w.arena, &w.scan_tmp, &w.cap_scan, scan_tmp_entries(w.n), 0, st, "scan tmp"));
    uint64_t* io = w.inv_offs + w.nseg * stride;
    const int ti = w.timer.open(2);
    HIP_TRY(launch_scan_u32(w.counts_acc, w.counts_prev, io, w.n, 0, w.set_off + w.indexed_sets,
                            w.scan_tmp, st));
    HIP_TRY(hipMemsetAsync(w.inv_cursor, 0, (uint64_t)w.n * 4, st));
    HIP_TRY(launch_inv_scatter(w.set_off, w.set_vtx, w.indexed_sets,
                               (uint32_t)(w.n_sets - w.indexed_sets), io, w.inv_cursor, w.inv_set,
                               &w.sc->err, st));
    HIP_TRY(hipMemcpyAsync(w.counts_prev, w.counts_acc, (uint64_t)w.n * 4,
                           hipMemcpyDeviceToDevice, st));
    w.timer.close(ti);
    ++w.nseg;
    w.indexed_sets = w.n_sets;
    return IMM_OK;
}

// Greedy selection over the whole pool: bring the index up to date, then k
// (argmax, claim, decrement) triples. Ends with the run's second
// synchronisation per round, which also reads the exact pool size.
imm_status ws_greedy(Workspace& w, uint32_t k, uint64_t sets_before, uint64_t* covered) {
    hipStream_t st = w.st;
    IMM_TRY(ws_index_update(w));
    IMM_TRY(grow(w.arena, &w.covered, &w.cap_cov, w.n_sets / 32 + 1, 0, st, "covered"));
    if (w.cap_k < k) {
        if (w.seeds_d) {
            HIP_TRY(hipStreamSynchronize(st));
            w.arena.release(w.seeds_d);
            w.arena.release(w.gains_d);
            w.arena.release(w.slots);
            w.arena.release(w.chunk_n);
            (void)hipHostFree(w.gains_h);
            w.gains_h = nullptr;
        }
        IMM_TRY(w.arena.alloc((void**)&w.seeds_d, (uint64_t)k * 4, "seeds"));
        IMM_TRY(w.arena.alloc((void**)&w.gains_d, (uint64_t)k * 4, "gains"));
        IMM_TRY(w.arena.alloc((void**)&w.slots, (uint64_t)k * kArgSlots * 8, "argmax slots"));
        IMM_TRY(w.arena.alloc((void**)&w.chunk_n, (uint64_t)k * 4, "chunk counts"));
        HIP_TRY(hipHostMalloc((void**)&w.gains_h, (uint64_t)k * 4, hipHostMallocDefault));
        w.cap_k = k;
    }
    // a seed's chunks: at most one per started 64 members of every set
    IMM_TRY(grow(w.arena, &w.chunks, &w.cap_chunks, w.n_sets + w.p_ub / 64 + 1, 0, st,
                 "chunk queue"));
    const int ts = w.timer.open(3);
    HIP_TRY(hipMemcpyAsync(w.counts_work, w.counts_acc, (uint64_t)w.n * 4, hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemsetAsync(w.covered, 0, (w.n_sets / 32 + 1) * 4, st));
    HIP_TRY(hipMemsetAsync(w.slots, 0, (uint64_t)k * kArgSlots * 8, st));
    HIP_TRY(hipMemsetAsync(w.chunk_n, 0, (uint64_t)k * 4, st));
    const uint32_t ag = argmax_grid(w.n), sg = select_grid(w.device);
    for (uint32_t i = 0; i < k; ++i) {
        unsigned long long* sl = w.slots + (uint64_t)i * kArgSlots;
        HIP_TRY(launch_argmax(w.counts_work, w.n, sl, ag, st));
        HIP_TRY(launch_claim(w.inv_offs, w.nseg, w.n, w.inv_set, w.set_off, w.covered,
                             w.counts_work, sl, w.seeds_d, w.gains_d, i, w.chunks, w.chunk_n + i,
                             sg, st));
        HIP_TRY(launch_decrement(w.chunks, w.chunk_n + i, w.set_vtx, w.counts_work, w.seeds_d, i,
                                 sg, st));
    }
    w.timer.close(ts);
    HIP_TRY(hipMemcpyAsync(w.gains_h, w.gains_d, (uint64_t)k * 4, hipMemcpyDeviceToHost, st));
    IMM_TRY(ws_sync_pool(w));
    if (*w.herr) return fail(IMM_EDEVICE, "internal error: occurrence counts disagree with the pool");
    ws_note_pool(w, sets_before);
    uint64_t c = 0;
    for (uint32_t i = 0; i < k; ++i) c += w.gains_h[i];
    *covered = c;
    return IMM_OK;
}

// Canonical pool on the host: every set sorted ascending, sets by sample id.
imm_status ws_export_pool(Workspace& w, std::vector<uint64_t>* so, std::vector<uint32_t>* sv,
                          std::vector<uint32_t>* counts) {
    hipStream_t st = w.st;
    if (w.n_sets > 0xFFFFFFFFull) return fail(IMM_EOVERFLOW, "more than 2^32 sets");
    IMM_TRY(ws_sync_pool(w));
    ws_note_pool(w, w.n_sets);
    uint32_t* big_list = nullptr;
    IMM_TRY(w.arena.alloc((void**)&big_list, (w.n_sets + 1) * 4, "sort list"));
    HIP_TRY(hipMemsetAsync(&w.sc->big_flag, 0, 4, st));
    HIP_TRY(launch_sort_small(w.set_off, (uint32_t)w.n_sets, w.set_vtx, big_list, &w.sc->big_flag, st));
    IMM_TRY(ws_read_scalars(w));
    const uint32_t nbig = w.hsc->big_flag;
    if (nbig) {
        std::vector<uint32_t> bl(nbig);
        HIP_TRY(hipMemcpy(bl.data(), big_list, (uint64_t)nbig * 4, hipMemcpyDeviceToHost));
        std::vector<uint64_t> o2(2);
        uint64_t maxn = 0;
        std::vector<uint32_t> np(nbig);
        for (uint32_t b = 0; b < nbig; ++b) {
            HIP_TRY(hipMemcpy(o2.data(), w.set_off + bl[b], 16, hipMemcpyDeviceToHost));
            uint64_t sz = o2[1] - o2[0], p2 = 1;
            while (p2 < sz) p2 <<= 1;
            np[b] = (uint32_t)p2;
            maxn = std::max(maxn, p2);
        }
        uint32_t* scratch = nullptr;
        IMM_TRY(w.arena.alloc((void**)&scratch, maxn * 4, "sort scratch"));
        for (uint32_t b = 0; b < nbig; ++b)
            HIP_TRY(launch_sort_big(w.set_off, w.set_vtx, bl[b], np[b], scratch, st));
        HIP_TRY(hipStreamSynchronize(st));
        w.arena.release(scratch);
    }
    HIP_TRY(hipStreamSynchronize(st));
    w.arena.release(big_list);
    if (so) {
        so->resize(w.n_sets + 1);
        HIP_TRY(hipMemcpy(so->data(), w.set_off, (w.n_sets + 1) * 8, hipMemcpyDeviceToHost));
    }
    if (sv) {
        sv->resize(w.p_exact);
        if (w.p_exact)
            HIP_TRY(hipMemcpy(sv->data(), w.set_vtx, w.p_exact * 4, hipMemcpyDeviceToHost));
    }
    if (counts) {
        counts->resize(w.n);
        HIP_TRY(hipMemcpy(counts->data(), w.counts_acc, (uint64_t)w.n * 4, hipMemcpyDeviceToHost));
    }
    return IMM_OK;
}

void fill_stats(Workspace& w, imm_stats* s) {
    double ms[6] = {0, 0, 0, 0, 0, 0};
    uint64_t launches[2] = {0, 0};
    w.timer.collect(ms, launches);
    s->ms_sample += ms[0];
    s->ms_compact += ms[1];
    s->ms_index += ms[2];
    s->ms_select += ms[3];
    s->ms_sample_main += ms[4];
    s->ms_sample_big += ms[5];
    s->main_launches += launches[0];
    s->big_launches += launches[1];
    const unsigned long long* t = w.hsc->stats;
    s->sets = t[kStMainSets] + t[kStBigSets];
    s->entries = t[kStMainEntries] + t[kStBigEntries];
    s->edges = t[kStMainEdges] + t[kStBigEdges];
    s->live = t[kStMainLive] + t[kStBigLive];
    s->deferred = t[kStBigSets];
    s->main_sets = t[kStMainSets];
    s->main_entries = t[kStMainEntries];
    s->main_edges = t[kStMainEdges];
    s->main_live = t[kStMainLive];
}

// ------------------------------------------------------------ theta math --
// FP64, no contraction, this exact order (kept identical to the IMM theta
// expressions of Tang et al. 2015: Eq. 9 lambda', Eq. 6 lambda*, with ell
// replaced by ell (1 + ln 2 / ln n)).

const double kLn2 = 0.69314718055994530942;
const double kInvE = 0.36787944117144232160;

double log_binom(uint32_t n, uint32_t k) {
    double acc = 0.0;
    for (uint32_t i = 1; i <= k; ++i) acc += std::log((double)(n - k + i) / (double)i);
    return acc;
}

uint32_t bitlen(uint32_t x) {
    uint32_t b = 0;
    while (x) { ++b; x >>= 1; }
    return b;
}

}  // namespace

struct imm_result {
    uint32_t k = 0;
    std::vector<uint32_t> seeds;
    std::vector<uint64_t> gains;
    uint64_t theta = 0;
    uint32_t rounds = 0;
    double lb = 0.0;
    uint64_t covered = 0;
    std::vector<uint64_t> targets, round_cov;
    bool has_pool = false;
    std::vector<uint64_t> set_off;
    std::vector<uint32_t> set_vtx;
    imm_stats stats{};
};

struct imm_pool {
    std::unique_ptr<Workspace> ws;
    imm_stats stats{};
};

// =================================================================== ABI ===

extern "C" {

const char* imm_last_error(void) { return g_err.c_str(); }

imm_status imm_theta_plan(uint32_t n, uint32_t k, double eps, double ell, double* lambda_prime,
                          double* lambda_star, uint32_t* i_max) {
    if (n < 2 || k == 0 || k > n || !(eps > 0.0) || !(ell > 0.0))
        return fail(IMM_EINVAL, "theta_plan: need n >= 2, 1 <= k <= n, eps > 0, ell > 0");
    if (!lambda_prime || !lambda_star || !i_max) return fail(IMM_EINVAL, "theta_plan: null output");
    const double ln_n = std::log((double)n);
    const double ell_p = ell * (1.0 + kLn2 / ln_n);
    const double logcnk = log_binom(n, k);
    const double eps_p = std::sqrt(2.0) * eps;
    const double lam_p = (2.0 + 2.0 / 3.0 * eps_p) *
                         (logcnk + ell_p * ln_n + std::log(std::log2((double)n))) * (double)n /
                         (eps_p * eps_p);
    const double one_m = 1.0 - kInvE;
    const double alpha = std::sqrt(ell_p * ln_n + kLn2);
    const double beta = std::sqrt(one_m * (logcnk + ell_p * ln_n + kLn2));
    const double t = one_m * alpha + beta;
    const double lam_s = 2.0 * (double)n * t * t / (eps * eps);
    *lambda_prime = lam_p;
    *lambda_star = lam_s;
    *i_max = bitlen(n - 1) - 1;
    return IMM_OK;
}

imm_status imm_graph_create(uint32_t n, uint64_t m, const uint64_t* col_off,
                            const uint32_t* row_src, const uint32_t* weight, imm_model model,
                            uint32_t flags, void* stream, imm_graph** out) {
    try {
        if (!out) return fail(IMM_EINVAL, "graph_create: null out");
        if (n < 2 || n > 0xFFFFFFFEu) return fail(IMM_EINVAL, "graph_create: need 2 <= n <= 2^32-2");
        if (m > 0xFFFFFFF0ull) return fail(IMM_EOVERFLOW, "graph_create: m must be < 2^32 - 16");
        if (model != IMM_IC && model != IMM_LT) return fail(IMM_EINVAL, "graph_create: bad model");
        if (!col_off || (m && (!row_src || !weight))) return fail(IMM_EINVAL, "graph_create: null array");
        hipStream_t st = (hipStream_t)stream;
        const bool dev = (flags & IMM_DEVICE_PTRS) != 0;
        std::vector<uint64_t> h_off;
        std::vector<uint32_t> h_src, h_w;
        const uint64_t* co = col_off;
        const uint32_t* rs = row_src;
        const uint32_t* wt = weight;
        if (dev) {
            h_off.resize((size_t)n + 1);
            h_src.resize(m);
            h_w.resize(m);
            HIP_TRY(hipMemcpyAsync(h_off.data(), col_off, ((size_t)n + 1) * 8, hipMemcpyDeviceToHost, st));
            if (m) {
                HIP_TRY(hipMemcpyAsync(h_src.data(), row_src, m * 4, hipMemcpyDeviceToHost, st));
                HIP_TRY(hipMemcpyAsync(h_w.data(), weight, m * 4, hipMemcpyDeviceToHost, st));
            }
            HIP_TRY(hipStreamSynchronize(st));
            co = h_off.data();
            rs = h_src.data();
            wt = h_w.data();
        }
        if (co[0] != 0 || co[n] != m) return fail(IMM_EINVAL, "graph_create: col_off[0] must be 0 and col_off[n] = m");
        for (uint32_t v = 0; v < n; ++v)
            if (co[v] > co[v + 1]) return fail(IMM_EINVAL, "graph_create: col_off decreases");
        for (uint64_t e = 0; e < m; ++e)
            if (rs[e] >= n) return fail(IMM_EINVAL, "graph_create: row_src out of range");
        if (model == IMM_LT) {
            for (uint32_t v = 0; v < n; ++v)
                for (uint64_t e = co[v] + 1; e < co[v + 1]; ++e)
                    if (wt[e] < wt[e - 1]) return fail(IMM_EINVAL, "graph_create: LT cumulative table decreases within a column");
        }
        std::unique_ptr<imm_graph> g(new imm_graph());
        g->n = n;
        g->m = m;
        g->model = model;
        HIP_TRY(hipGetDevice(&g->device));
        std::vector<uint32_t> off32((size_t)n + 1);
        for (size_t v = 0; v <= n; ++v) off32[v] = (uint32_t)co[v];
        IMM_TRY(g->arena.alloc((void**)&g->off, ((uint64_t)n + 1) * 4, "graph offsets"));
        HIP_TRY(hipMemcpyAsync(g->off, off32.data(), ((size_t)n + 1) * 4, hipMemcpyHostToDevice, st));
        if (model == IMM_IC) {
            const uint64_t mp = ((m + 3) & ~uint64_t(3)) + 4;
            IMM_TRY(g->arena.alloc((void**)&g->thr, mp * 4, "thresholds"));
            IMM_TRY(g->arena.alloc((void**)&g->src, (m ? m : 1) * 4, "sources"));
            HIP_TRY(hipMemsetAsync(g->thr, 0, mp * 4, st));
            if (m) {
                HIP_TRY(hipMemcpyAsync(g->thr, wt, m * 4, hipMemcpyHostToDevice, st));
                HIP_TRY(hipMemcpyAsync(g->src, rs, m * 4, hipMemcpyHostToDevice, st));
            }
            HIP_TRY(hipStreamSynchronize(st));
        } else {
            std::vector<uint2> cs(m ? m : 1);
            for (uint64_t e = 0; e < m; ++e) cs[e] = make_uint2(wt[e], rs[e]);
            IMM_TRY(g->arena.alloc((void**)&g->cs, (m ? m : 1) * 8, "cum/src pairs"));
            IMM_TRY(g->arena.alloc((void**)&g->guide, (m ? m : 1) * 4, "guide table"));
            if (m) HIP_TRY(hipMemcpyAsync(g->cs, cs.data(), m * 8, hipMemcpyHostToDevice, st));
            HIP_TRY(launch_lt_guide(g->off, g->cs, g->guide, n, st));
            HIP_TRY(hipStreamSynchronize(st));
        }
        *out = g.release();
        return IMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(IMM_ENOMEM, "graph_create: host allocation failed");
    } catch (...) {
        return fail(IMM_EDEVICE, "graph_create: unexpected exception");
    }
}

imm_status imm_graph_destroy(imm_graph* g) {
    if (!g) return fail(IMM_EINVAL, "graph_destroy: null graph");
    (void)hipSetDevice(g->device);
    delete g;
    return IMM_OK;
}

imm_status imm_graph_info(const imm_graph* g, uint32_t* n, uint64_t* m, imm_model* model,
                          uint64_t* device_bytes) {
    if (!g) return fail(IMM_EINVAL, "graph_info: null graph");
    if (n) *n = g->n;
    if (m) *m = g->m;
    if (model) *model = g->model;
    if (device_bytes) *device_bytes = g->arena.used;
    return IMM_OK;
}

static imm_status run_impl(imm_graph* g, const imm_params* p, hipStream_t st,
                           imm_result** out) {
    const double t0 = now_ms();
    double lam_p, lam_s;
    uint32_t i_max;
    IMM_TRY(imm_theta_plan(g->n, p->k, p->epsilon, p->ell, &lam_p, &lam_s, &i_max));
    HIP_TRY(hipSetDevice(g->device));
    // take the graph's cached workspace when it fits the budget
    std::unique_ptr<Workspace> w;
    {
        std::lock_guard<std::mutex> lk(g->ws_mu);
        w = std::move(g->ws_cache);
    }
    if (w && (p->max_device_bytes != w->arena.budget)) w.reset();
    if (!w) {
        w.reset(new Workspace());
        IMM_TRY(ws_init(*w, g->n, g->device, st, p->max_device_bytes));
    }
    IMM_TRY(ws_reset(*w, st, (p->flags & IMM_TIMING) != 0));
    std::unique_ptr<imm_result> r(new imm_result());
    r->k = p->k;
    const double eps_p = std::sqrt(2.0) * p->epsilon;
    double lb = 1.0;
    uint64_t cov = 0;
    for (uint32_t i = 1; i <= i_max; ++i) {
        const double x = std::ldexp((double)g->n, -(int)i);
        const double tf = std::ceil(lam_p / x);
        if (!(tf < 4294967296.0)) return fail(IMM_EOVERFLOW, "theta_i >= 2^32");
        const uint64_t target = (uint64_t)tf;
        if (r->targets.size() < 63) r->targets.push_back(target);
        const uint64_t before = w->n_sets;
        if (w->n_sets < target) IMM_TRY(ws_extend(*w, g, p->seed, w->n_sets, target - w->n_sets));
        IMM_TRY(ws_greedy(*w, p->k, before, &cov));
        r->round_cov.push_back(cov);
        r->rounds = i;
        const double frac = (double)cov / (double)w->n_sets;
        if ((double)g->n * frac >= (1.0 + eps_p) * x) {
            lb = (double)g->n * frac / (1.0 + eps_p);
            break;
        }
    }
    const double tf = std::ceil(lam_s / lb);
    if (!(tf < 4294967296.0)) return fail(IMM_EOVERFLOW, "theta >= 2^32");
    const uint64_t theta = (uint64_t)tf;
    r->targets.push_back(theta);
    const uint64_t before = w->n_sets;
    if (w->n_sets < theta) IMM_TRY(ws_extend(*w, g, p->seed, w->n_sets, theta - w->n_sets));
    IMM_TRY(ws_greedy(*w, p->k, before, &cov));
    r->seeds.resize(p->k);
    HIP_TRY(hipMemcpy(r->seeds.data(), w->seeds_d, (uint64_t)p->k * 4, hipMemcpyDeviceToHost));
    r->gains.assign(w->gains_h, w->gains_h + p->k);
    r->theta = w->n_sets;
    r->lb = lb;
    r->covered = cov;
    const double t1 = now_ms();
    IMM_TRY(ws_read_scalars(*w));
    fill_stats(*w, &r->stats);
    r->stats.ms_total = t1 - t0;
    r->stats.rounds = r->rounds;
    if (p->flags & IMM_KEEP_POOL) {
        IMM_TRY(ws_export_pool(*w, &r->set_off, &r->set_vtx, nullptr));
        r->has_pool = true;
    }
    {
        std::lock_guard<std::mutex> lk(g->ws_mu);
        g->ws_cache = std::move(w);
    }
    *out = r.release();
    return IMM_OK;
}

imm_status imm_run(const imm_graph* g, const imm_params* p, void* stream, imm_result** out) {
    if (!g || !p || !out) return fail(IMM_EINVAL, "run: null argument");
    if (p->k == 0 || p->k > g->n) return fail(IMM_EINVAL, "run: need 1 <= k <= n");
    if (!(p->epsilon > 0.0) || !(p->ell > 0.0)) return fail(IMM_EINVAL, "run: need eps > 0, ell > 0");
    try {
        return run_impl(const_cast<imm_graph*>(g), p, (hipStream_t)stream, out);
    } catch (const std::bad_alloc&) {
        return fail(IMM_ENOMEM, "run: host allocation failed");
    } catch (...) {
        return fail(IMM_EDEVICE, "run: unexpected exception");
    }
}

imm_status imm_result_info(const imm_result* r, uint64_t* theta, uint32_t* rounds, double* lb,
                           uint64_t* covered) {
    if (!r) return fail(IMM_EINVAL, "result_info: null result");
    if (theta) *theta = r->theta;
    if (rounds) *rounds = r->rounds;
    if (lb) *lb = r->lb;
    if (covered) *covered = r->covered;
    return IMM_OK;
}

imm_status imm_result_seeds(const imm_result* r, uint32_t* seeds, uint64_t* gains) {
    if (!r) return fail(IMM_EINVAL, "result_seeds: null result");
    if (seeds) std::memcpy(seeds, r->seeds.data(), r->seeds.size() * 4);
    if (gains) std::memcpy(gains, r->gains.data(), r->gains.size() * 8);
    return IMM_OK;
}

imm_status imm_result_targets(const imm_result* r, uint32_t* count, uint64_t* targets,
                              uint64_t* round_cov) {
    if (!r) return fail(IMM_EINVAL, "result_targets: null result");
    const size_t nt = std::min<size_t>(r->targets.size(), 64);
    if (count) *count = (uint32_t)nt;
    if (targets) std::memcpy(targets, r->targets.data(), nt * 8);
    if (round_cov) std::memcpy(round_cov, r->round_cov.data(), std::min<size_t>(r->round_cov.size(), 64) * 8);
    return IMM_OK;
}

imm_status imm_result_pool(const imm_result* r, uint64_t* n_sets, uint64_t* n_entries,
                           uint64_t* set_off, uint32_t* set_vtx) {
    if (!r) return fail(IMM_EINVAL, "result_pool: null result");
    if (!r->has_pool) return fail(IMM_EINVAL, "result_pool: run without IMM_KEEP_POOL");
    if (n_sets) *n_sets = r->set_off.size() - 1;
    if (n_entries) *n_entries = r->set_vtx.size();
    if (set_off) std::memcpy(set_off, r->set_off.data(), r->set_off.size() * 8);
    if (set_vtx && !r->set_vtx.empty()) std::memcpy(set_vtx, r->set_vtx.data(), r->set_vtx.size() * 4);
    return IMM_OK;
}

imm_status imm_result_stats(const imm_result* r, imm_stats* stats) {
    if (!r || !stats) return fail(IMM_EINVAL, "result_stats: null argument");
    *stats = r->stats;
    return IMM_OK;
}

void imm_result_destroy(imm_result* r) { delete r; }

imm_status imm_sample(const imm_graph* g, uint64_t seed, uint64_t first_id, uint64_t count,
                      uint32_t flags, void* stream, imm_pool** out) {
    if (!g || !out) return fail(IMM_EINVAL, "sample: null argument");
    if (count == 0 || first_id + count < first_id) return fail(IMM_EINVAL, "sample: bad id range");
    if (count > 0xFFFFFFFFull) return fail(IMM_EOVERFLOW, "sample: count >= 2^32");
    try {
        const double t0 = now_ms();
        hipStream_t st = (hipStream_t)stream;
        HIP_TRY(hipSetDevice(g->device));
        std::unique_ptr<imm_pool> p(new imm_pool());
        p->ws.reset(new Workspace());
        IMM_TRY(ws_init(*p->ws, g->n, g->device, st, 0));
        IMM_TRY(ws_reset(*p->ws, st, (flags & IMM_TIMING) != 0));
        IMM_TRY(ws_extend(*p->ws, g, seed, first_id, count));
        IMM_TRY(ws_sync_pool(*p->ws));
        ws_note_pool(*p->ws, 0);
        IMM_TRY(ws_read_scalars(*p->ws));
        p->stats.ms_total = now_ms() - t0;
        fill_stats(*p->ws, &p->stats);
        *out = p.release();
        return IMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(IMM_ENOMEM, "sample: host allocation failed");
    } catch (...) {
        return fail(IMM_EDEVICE, "sample: unexpected exception");
    }
}

imm_status imm_pool_info(const imm_pool* p, uint64_t* n_sets, uint64_t* n_entries,
                         imm_stats* stats) {
    if (!p) return fail(IMM_EINVAL, "pool_info: null pool");
    if (n_sets) *n_sets = p->ws->n_sets;
    if (n_entries) *n_entries = p->ws->p_exact;
    if (stats) *stats = p->stats;
    return IMM_OK;
}

imm_status imm_pool_export(const imm_pool* p, uint64_t* set_off, uint32_t* set_vtx,
                           uint32_t* counts) {
    if (!p) return fail(IMM_EINVAL, "pool_export: null pool");
    try {
        HIP_TRY(hipSetDevice(p->ws->device));
        std::vector<uint64_t> so;
        std::vector<uint32_t> sv, cn;
        IMM_TRY(ws_export_pool(*p->ws, set_off ? &so : nullptr, set_vtx ? &sv : nullptr,
                               counts ? &cn : nullptr));
        if (set_off) std::memcpy(set_off, so.data(), so.size() * 8);
        if (set_vtx && !sv.empty()) std::memcpy(set_vtx, sv.data(), sv.size() * 4);
        if (counts) std::memcpy(counts, cn.data(), cn.size() * 4);
        return IMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(IMM_ENOMEM, "pool_export: host allocation failed");
    }
}

void imm_pool_destroy(imm_pool* p) { delete p; }

imm_status imm_greedy(uint32_t n, const uint64_t* set_off, const uint32_t* set_vtx,
                      uint64_t n_sets, uint32_t k, uint32_t flags, void* stream, uint32_t* seeds,
                      uint64_t* gains, uint64_t* covered) {
    if (n < 1 || n > 0xFFFFFFFEu || k == 0 || k > n) return fail(IMM_EINVAL, "greedy: need 1 <= k <= n");
    if (n_sets >= 0xFFFFFFFFull) return fail(IMM_EINVAL, "greedy: n_sets must be < 2^32");
    if (!set_off || !seeds) return fail(IMM_EINVAL, "greedy: null argument");
    try {
        hipStream_t st = (hipStream_t)stream;
        const bool devp = (flags & IMM_DEVICE_PTRS) != 0;
        std::vector<uint64_t> h_off;
        const uint64_t* so = set_off;
        if (devp) {
            h_off.resize(n_sets + 1);
            HIP_TRY(hipMemcpy(h_off.data(), set_off, (n_sets + 1) * 8, hipMemcpyDeviceToHost));
            so = h_off.data();
        }
        if (so[0] != 0) return fail(IMM_EINVAL, "greedy: set_off[0] must be 0");
        for (uint64_t j = 0; j < n_sets; ++j)
            if (so[j] > so[j + 1]) return fail(IMM_EINVAL, "greedy: set_off decreases");
        const uint64_t P = so[n_sets];
        if (P && !set_vtx) return fail(IMM_EINVAL, "greedy: null set_vtx");
        if (!devp) {
            for (uint64_t t = 0; t < P; ++t)
                if (set_vtx[t] >= n) return fail(IMM_EINVAL, "greedy: vertex id out of range");
        }
        int dev = 0;
        HIP_TRY(hipGetDevice(&dev));
        Workspace w;
        IMM_TRY(ws_init(w, n, dev, st, 0));
        IMM_TRY(ws_reset(w, st, false));
        IMM_TRY(grow(w.arena, &w.set_off, &w.cap_sets, n_sets + 1, 0, st, "set_off"));
        IMM_TRY(grow(w.arena, &w.set_vtx, &w.cap_entries, P + 1, 0, st, "set_vtx"));
        const hipMemcpyKind kind = devp ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice;
        HIP_TRY(hipMemcpyAsync(w.set_off, set_off, (n_sets + 1) * 8, kind, st));
        if (P) HIP_TRY(hipMemcpyAsync(w.set_vtx, set_vtx, P * 4, kind, st));
        if (devp) {
            HIP_TRY(hipMemsetAsync(&w.sc->big_flag, 0, 4, st));
            HIP_TRY(launch_validate_pool(w.set_off, n_sets, w.set_vtx, n, &w.sc->big_flag, st));
            IMM_TRY(ws_read_scalars(w));
            if (w.hsc->big_flag) return fail(IMM_EINVAL, "greedy: vertex id out of range");
        }
        HIP_TRY(launch_count_entries(w.set_vtx, P, w.counts_acc, st));
        w.n_sets = n_sets;
        w.p_ub = P;
        uint64_t cov = 0;
        IMM_TRY(ws_greedy(w, k, n_sets, &cov));
        std::vector<uint32_t> s32(k);
        HIP_TRY(hipMemcpy(s32.data(), w.seeds_d, (uint64_t)k * 4, hipMemcpyDeviceToHost));
        std::memcpy(seeds, s32.data(), (size_t)k * 4);
        if (gains)
            for (uint32_t i = 0; i < k; ++i) gains[i] = w.gains_h[i];
        if (covered) *covered = cov;
        return IMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(IMM_ENOMEM, "greedy: host allocation failed");
    }
}

imm_status imm_philox4x32_10(const uint32_t* ctr, uint64_t count, uint64_t key, uint32_t flags,
                             void* stream, uint32_t* out) {
    if (!ctr || !out) return fail(IMM_EINVAL, "philox: null argument");
    if (count == 0) return IMM_OK;
    hipStream_t st = (hipStream_t)stream;
    const bool devp = (flags & IMM_DEVICE_PTRS) != 0;
    if (devp) {
        HIP_TRY(launch_philox(ctr, count, key, out, st));
        HIP_TRY(hipStreamSynchronize(st));
        return IMM_OK;
    }
    Arena a;
    uint32_t *dc = nullptr, *dout = nullptr;
    IMM_TRY(a.alloc((void**)&dc, count * 16, "philox counters"));
    IMM_TRY(a.alloc((void**)&dout, count * 16, "philox output"));
    HIP_TRY(hipMemcpyAsync(dc, ctr, count * 16, hipMemcpyHostToDevice, st));
    HIP_TRY(launch_philox(dc, count, key, dout, st));
    HIP_TRY(hipMemcpyAsync(out, dout, count * 16, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return IMM_OK;
}

}  // extern "C"
