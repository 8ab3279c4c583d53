// workspace.cpp -- the device workspace of one IMM query: allocation with a
// budget, the sampling pass with its retry loop and compaction (steps of
// Generate_RRRsets), the per-round index segment, and the per-instance half
// of the greedy selection (Find_Most_Influential_Set).
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>

#include "engine.hpp"

namespace imm {

namespace {
// a fixed buffer, so that reporting an error allocates nothing
thread_local char g_err[512];
}

imm_status fail(imm_status st, const char* msg) {
    std::strncpy(g_err, msg ? msg : "", sizeof(g_err) - 1);
    g_err[sizeof(g_err) - 1] = '\0';
    return st;
}

imm_status fail(imm_status st, const std::string& msg) { return fail(st, msg.c_str()); }

const char* last_error() { return g_err; }

double now_ms() {
    using namespace std::chrono;
    return duration<double, std::milli>(steady_clock::now().time_since_epoch()).count();
}

// ------------------------------------------------------------ allocation --

imm_status Arena::alloc(void** p, uint64_t bytes, const char* what) {
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

void Arena::release(void* p) {
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

void Arena::release_all() {
    for (auto& x : live) (void)hipFree(x.first);
    live.clear();
    used = 0;
}

// ---------------------------------------------------------------- timing --

hipEvent_t Timer::get() {
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    (void)hipEventCreate(&e);
    return e;
}

int Timer::open(int phase, hipStream_t st) {
    if (!on) return -1;
    Rec r{phase, get(), get()};
    (void)hipEventRecord(r.a, st);
    recs.push_back(r);
    return (int)recs.size() - 1;
}

void Timer::close(int h, hipStream_t st) {
    if (h < 0) return;
    (void)hipEventRecord(recs[h].b, st);
}

void Timer::collect(double* ms, uint64_t* launches) {
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

Timer::~Timer() {
    for (auto& r : recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (auto e : pool) (void)hipEventDestroy(e);
}

// ------------------------------------------------------------- workspace --

Workspace::~Workspace() {
    // kernels of a failed call may still be queued on these buffers and the
    // caller's stream may already be gone: wait for the whole device
    if (sc) (void)hipDeviceSynchronize();
    if (hsc) (void)hipHostFree(hsc);
    if (hp) (void)hipHostFree(hp);
    if (herr) (void)hipHostFree(herr);
    if (gains_h) (void)hipHostFree(gains_h);
    if (cand_h) (void)hipHostFree(cand_h);
    if (sel2.gains_h) (void)hipHostFree(sel2.gains_h);
    if (sel2.cand_h) (void)hipHostFree(sel2.cand_h);
    if (side_ev) (void)hipEventDestroy(side_ev);
    if (side_ev2) (void)hipEventDestroy(side_ev2);
    if (side) (void)hipStreamDestroy(side);
}

IcGraphDev ic_view(const imm_graph* g) {
    return IcGraphDev{g->off, g->thr, g->src, g->n, (uint32_t)g->m};
}

LtGraphDev lt_view(const imm_graph* g) {
    return LtGraphDev{g->off, g->cs, g->guide, g->gw, g->n, (uint32_t)g->m};
}

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
    IMM_TRY(w.arena.alloc((void**)&w.heavy, (uint64_t)n * 4 + 16, "heavy vertex list"));
    IMM_TRY(w.arena.alloc((void**)&w.inv_cursor, (uint64_t)n * 4, "inv_cursor"));
    IMM_TRY(w.arena.alloc((void**)&w.desc_d, sizeof(SelectDesc), "select descriptor"));
    IMM_TRY(w.arena.alloc((void**)&w.cand, (uint64_t)kCandMax * 4, "candidate list"));
    IMM_TRY(w.arena.alloc((void**)&w.cand_bits, ((uint64_t)n + 31) / 32 * 4 + 16,
                          "candidate bitmap"));
    IMM_TRY(w.arena.alloc((void**)&w.cand_state, (kCandHead + kCandBins) * 4, "candidate state"));
    HIP_TRY(hipHostMalloc((void**)&w.cand_h, kCandHead * 4, hipHostMallocDefault));
    IMM_TRY(grow(w.arena, &w.set_off, &w.cap_sets, 1024, 0, st, "set_off"));
    return IMM_OK;
}

imm_status ws_reset(Workspace& w, hipStream_t st, bool timing) {
    w.st = st;
    w.timer.on = timing;
    w.timer.recs.clear();
    w.n_sets = 0;
    w.p_exact = 0;
    w.p_ub = 0;
    w.nseg = 0;
    w.indexed_sets = 0;
    w.p_indexed = 0;
    w.pend_lo = w.pend_hi = 0;
    w.n_dense = 0;
    w.dense_entries = 0;
    w.ahead_n = 0;
    w.ahead_next = 0;
    w.list_only = false;
    w.cand_steps = 0;
    w.cand_halts = 0;
    w.spec = false;
    w.spec_rounds = 0;
    if (w.dense_counts) HIP_TRY(hipMemsetAsync(w.dense_counts, 0, (uint64_t)w.n * 4, st));
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

namespace {

// Scratch of the large-set kernels: per slot a visited bitmap and a queue.
// IC: enough slots for the 256-thread shape with queues of kGiantQueue
// entries, plus kHugeSlots slots with queues of n for the sets that outgrow
// those; LT: one slot per CU with queues of n (its walks rarely outgrow a
// chunk). All within kBigScratchBytes and the budget.
imm_status ws_big_scratch(Workspace& w, const imm_graph* g) {
    if (w.big) return IMM_OK;
    const bool ic = g->model == IMM_IC;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, w.device);
    const uint64_t words = ((uint64_t)w.n + 31) / 32;
    // A graph on which tuning saw sets outgrow the bounded queue (the frontier
    // of a set of hundreds of thousands of members) gets queues of n/4
    // entries (a power of two: a ring when the set is stored as a bitmap),
    // and a full-size slot per eight CUs-worth of threads instead of a few.
    const bool outgrow = ic && g->over_rate > kOverRate;
    uint32_t qcap = ic ? std::min<uint32_t>(w.n, kGiantQueue) : w.n;
    if (outgrow) {
        uint64_t q = kGiantQueue;
        while (q < (uint64_t)w.n / 4 && q < kGiantQueueMax) q <<= 1;
        qcap = (uint32_t)std::min<uint64_t>(w.n, q);
    }
    const uint64_t per = (words + qcap) * 4;
    const uint64_t per_huge = (words + w.n) * 4;
    uint64_t slots = ic ? ic_large_slots(w.device, 256) : (uint64_t)cus;
    if (w.big_cap) slots = std::min<uint64_t>(slots, w.big_cap);
    uint64_t limit = kBigScratchBytes;
    if (w.arena.budget) {
        const uint64_t left = w.arena.budget > w.arena.used ? w.arena.budget - w.arena.used : 0;
        limit = std::min(limit, left / 4);
    }
    uint64_t huge = ic && qcap < w.n ? kHugeSlots : 0;
    if (huge && outgrow)
        huge = std::max<uint64_t>(huge, std::min<uint64_t>(2ull * cus, limit / 2 / per_huge));
    const uint64_t huge_bytes = huge * per_huge;
    const uint64_t room = limit > huge_bytes ? limit - huge_bytes : 0;
    slots = std::min<uint64_t>(slots, std::max<uint64_t>(1, room / per));
    IMM_TRY(w.arena.alloc((void**)&w.big, per * slots, "large-set scratch"));
    HIP_TRY(hipMemsetAsync(w.big, 0, words * slots * 4, w.st));
    w.big_slots = (uint32_t)slots;
    w.big_qcap = qcap;
    if (huge) {
        IMM_TRY(w.arena.alloc((void**)&w.huge, huge_bytes, "huge-set scratch"));
        HIP_TRY(hipMemsetAsync(w.huge, 0, words * huge * 4, w.st));
        w.huge_slots = (uint32_t)huge;
    }
    return IMM_OK;
}

// The scratch slots, at most `want` of them.
BigScratch big_view(const Workspace& w, uint32_t want) {
    const uint32_t words = (uint32_t)(((uint64_t)w.n + 31) / 32);
    return BigScratch{w.big, w.big + (uint64_t)words * w.big_slots, words,
                      std::min(w.big_slots, want), w.big_qcap};
}

BigScratch huge_view(const Workspace& w) {
    const uint32_t words = (uint32_t)(((uint64_t)w.n + 31) / 32);
    return BigScratch{w.huge, w.huge + (uint64_t)words * w.huge_slots, words, w.huge_slots, w.n};
}

// Sets of at least this many members are stored as bitmaps (IC only; none
// when the workspace keeps lists only).
uint32_t dense_min_of(const Workspace& w, const imm_graph* g) {
    return (g->model == IMM_IC && !w.list_only) ? dense_threshold(w.n) : 0xFFFFFFFFu;
}

// Bitmap slots for at least `want` dense sets in all, keeping the first
// `keep` slots' contents: grown by half or more, within the budget; a
// shortfall only costs a retry of the sets that found no slot.
imm_status ws_dense_reserve(Workspace& w, uint64_t want, uint64_t keep) {
    if (w.dense_words == 0) w.dense_words = (uint32_t)(((uint64_t)w.n + 31) / 32);
    if (w.cap_dense >= want) return IMM_OK;
    hipStream_t st = w.st;
    uint64_t nc = std::max<uint64_t>(want, w.cap_dense + w.cap_dense / 2);
    const uint64_t per = (uint64_t)w.dense_words * 4 + 12;
    if (w.arena.budget) {
        const uint64_t left = w.arena.budget > w.arena.used ? w.arena.budget - w.arena.used : 0;
        nc = std::min<uint64_t>(nc, std::max<uint64_t>(want, left / 2 / per));
    }
    uint64_t cb = w.cap_dense * w.dense_words, cs = w.cap_dense, cz = w.cap_dense,
             cl = w.cap_dense;
    IMM_TRY(grow(w.arena, &w.dense_bits, &cb, nc * w.dense_words, keep * w.dense_words, st,
                 "dense set bitmaps"));
    IMM_TRY(grow(w.arena, &w.dense_sid, &cs, nc, keep, st, "dense set ids"));
    IMM_TRY(grow(w.arena, &w.dense_size, &cz, nc, keep, st, "dense set sizes"));
    IMM_TRY(grow(w.arena, &w.dense_list, &cl, nc, 0, st, "dense claims"));
    w.cap_dense = std::min(std::min(cb / w.dense_words, cs), std::min(cz, cl));
    if (!w.dense_counts) {
        IMM_TRY(w.arena.alloc((void**)&w.dense_counts, (uint64_t)w.n * 4, "dense counts"));
        HIP_TRY(hipMemsetAsync(w.dense_counts, 0, (uint64_t)w.n * 4, st));
    }
    return IMM_OK;
}

// Where a pass of w stores its sets; fl / fl_n take the samples to retry.
SampleOut sample_out(Workspace& w, const imm_graph* g, uint32_t* fl, uint32_t* fl_n) {
    SampleOut o{w.stage, w.stage_cap, &w.sc->cursor, w.stage_off, w.sizes, w.counts_acc,
                w.defer, &w.sc->defer_n, fl, fl_n, w.sc->stats};
    o.dense_bits = w.dense_bits;
    o.dense_cap = w.cap_dense;
    o.dense_cursor = &w.sc->dense_n;
    o.dense_sid = w.dense_sid;
    o.dense_size = w.dense_size;
    o.dense_entries = &w.sc->dense_entries;
    o.dense_min = dense_min_of(w, g);
    o.dense_words = w.dense_words;
    o.pool_base = w.n_sets;
    o.count_lim = w.pending_split ? (uint32_t)w.pending_split : 0xFFFFFFFFu;
    o.count_lim2 = o.count_lim;
    o.counts_next = w.counts_next;
    if (w.pending_next && w.counts_next) o.count_lim2 = (uint32_t)(w.pending_split + w.pending_next);
    return o;
}

// One sampling pass: the fast kernel over the range (list = nullptr) or over
// a list of indices, then the large-set kernel over what it deferred.
// Failures for lack of staging land in fl; deferred sets in w.defer. The
// scalars are copied to the pinned mirror; nothing waits.
imm_status sample_pass(Workspace& w, const imm_graph* g, uint64_t seed, uint64_t id_lo,
                       uint32_t count, const uint32_t* list, const uint32_t* list_n,
                       uint32_t nitems, uint32_t* fl, uint32_t* fl_n, bool fresh) {
    hipStream_t st = w.st;
    const SampleRange rg{seed, id_lo, nitems, list, list_n};
    const SampleRange rgl{seed, id_lo, count, nullptr, nullptr};
    const SampleOut o = sample_out(w, g, fl, fl_n);
    // tickets and list lengths (already zero right after ws_extend_launch's reset)
    if (!fresh) HIP_TRY(hipMemsetAsync(&w.sc->ticket_small, 0, 7 * sizeof(uint32_t), st));
    const int th = w.timer.open(0, st);
    if (g->model == IMM_IC) {
        const int tl = w.timer.open(6, st);
        HIP_TRY(launch_ic_lane(ic_view(g), rg, o, w.pend, &w.sc->pend_n, &w.sc->ticket_small,
                               ic_small_grid(w.device), st));
        w.timer.close(tl, st);
        const int tm = w.timer.open(4, st);
        const SampleRange rgp{seed, id_lo, nitems, nullptr, nullptr};
        HIP_TRY(launch_ic_bfs(ic_view(g), rgp, o, w.pend, &w.sc->pend_n, &w.sc->ticket_bfs,
                              g->ic_team, ic_bfs_grid(w.device, g->ic_team), st));
        w.timer.close(tm, st);
    } else {
        const int tm = w.timer.open(4, st);
        HIP_TRY(launch_lt_small(lt_view(g), rg, o, &w.sc->ticket_small, g->lt_bloom_bits,
                                g->lt_lanes, lt_small_grid(w.device, g->lt_bloom_bits, g->lt_lanes),
                                st));
        w.timer.close(tm, st);
    }
    const int t3 = w.timer.open(5, st);
    if (g->model == IMM_IC) {
        // the tuned giant-set shape, unless the pass is expected to defer
        // more sets than that shape has workgroups
        uint32_t block = g->ic_big_block;
        if (!g->big_forced && g->defer_rate * (double)nitems > ic_large_slots(w.device, block))
            block = 256;
        HIP_TRY(launch_ic_large(ic_view(g), rgl, o, w.defer, &w.sc->defer_n, fl, fl_n, w.over,
                                &w.sc->over_n, &w.sc->ticket_big,
                                big_view(w, ic_large_slots(w.device, block)), block, st));
        w.timer.close(t3, st);
        if (w.huge_slots) {
            const int t7 = w.timer.open(7, st);
            HIP_TRY(launch_ic_large(ic_view(g), rgl, o, w.over, &w.sc->over_n, fl, fl_n, nullptr,
                                    nullptr, &w.sc->ticket_huge, huge_view(w), 1024, st));
            w.timer.close(t7, st);
        }
    } else {
        HIP_TRY(launch_lt_large(lt_view(g), rgl, o, w.defer, &w.sc->defer_n, fl, fl_n,
                                &w.sc->ticket_big, big_view(w, w.big_slots), st));
        w.timer.close(t3, st);
    }
    w.timer.close(th, st);
    HIP_TRY(hipMemcpyAsync(w.hsc, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, st));
    return IMM_OK;
}

}  // namespace

// The next k of the sets the last pass drew ahead join the pool: their
// offsets, members and counts (the staging, per-sample offsets and sizes of
// that pass are still in place). The rest wait for a later call; the next
// pass or a restart of the pool drops them.
imm_status ws_take_ahead(Workspace& w, uint64_t k) {
    hipStream_t st = w.st;
    const uint64_t split = w.ahead_split;
    k = std::min(k, w.ahead_n);
    w.ahead_n -= k;
    w.ahead_split += k;
    if (k == 0) return IMM_OK;
    IMM_TRY(grow(w.arena, &w.set_off, &w.cap_sets, w.n_sets + k + 1, w.n_sets + 1, st,
                 "set_off"));
    IMM_TRY(grow(w.arena, &w.scan_tmp, &w.cap_scan, scan_tmp_entries(k), 0, st, "scan tmp"));
    const int tc = w.timer.open(1, st);
    HIP_TRY(launch_scan_u32(w.sizes + split, nullptr, w.set_off + w.n_sets, k, 0,
                            w.set_off + w.n_sets, w.scan_tmp, st));
    HIP_TRY(launch_compact(w.stage, w.stage_off + split, w.set_off, w.n_sets, (uint32_t)k,
                           w.set_vtx, st));
    if (w.ahead_next && k == w.ahead_next) {
        // exactly the ids the pass counted apart
        HIP_TRY(launch_add_counts(w.counts_next, w.counts_acc, w.n, st));
    } else if (w.n_dense == 0 && w.indexed_sets <= w.n_sets &&
               (w.pend_hi == w.pend_lo || w.pend_hi == w.n_sets)) {
        // counted by the next index update, from the sets themselves
        if (w.pend_hi == w.pend_lo) w.pend_lo = w.n_sets;
        w.pend_hi = w.n_sets + k;
    } else {
        HIP_TRY(launch_count_sets(w.set_off, w.n_sets, w.n_sets + k, w.set_vtx, w.counts_acc,
                                  st));
    }
    w.ahead_next = 0;
    w.timer.close(tc, st);
    // set_vtx already has room: the last pass's compaction reserved its whole
    // staging bound. The pool-size bound (which sizes the index and later
    // compactions) takes that bound back in: a selection in between has set
    // it to the exact size of the pool without these sets.
    w.n_sets += k;
    w.p_ub += w.ahead_bound;
    return IMM_OK;
}

imm_status ws_extend_launch(Workspace& w, const imm_graph* g, uint64_t seed, uint64_t id_lo,
                            uint64_t count64, bool multi, uint64_t ahead, uint64_t next) {
    w.lt = g->model == IMM_LT;
    w.pending_count = 0;
    w.pending_multi = false;
    w.pending_split = 0;
    w.pending_next = 0;
    if (w.ahead_n) {
        // sets drawn ahead by the last pass, as many as this call wants
        const uint64_t k = std::min<uint64_t>(w.ahead_n, count64);
        IMM_TRY(ws_take_ahead(w, k));
        id_lo += k;
        count64 -= k;
    }
    if (count64 == 0) return IMM_OK;
    if (count64 + ahead > 0xFFFFFFFFull) return fail(IMM_EOVERFLOW, "sampling round too large");
    uint32_t count = (uint32_t)count64;
    // a large batch with no set-size estimate yet takes the graph's tuning
    // mean (with a margin), else a pilot batch measures one first; smaller
    // batches keep the generous default
    constexpr uint32_t kPilot = 1u << 16;
    if (w.mean_size <= 0.0 && count > 2 * kPilot && g->mean_set_hint > 0.0)
        w.mean_size = 1.25 * g->mean_set_hint;
    if (w.mean_size <= 0.0 && count > 2 * kPilot) {
        const uint64_t before = w.n_sets;
        IMM_TRY(ws_extend_launch(w, g, seed, id_lo, kPilot));
        HIP_TRY(hipStreamSynchronize(w.st));
        IMM_TRY(ws_extend_finish(w, g, seed));
        IMM_TRY(ws_sync_pool(w));
        ws_note_pool(w, before);
        id_lo += kPilot;
        count -= kPilot;
    }
    // the ids drawn ahead follow this call's ids in the same pass; they are
    // staged but not counted, and stay out of the pool until a later call.
    // Every per-sample array and the staging estimate below cover them.
    const uint32_t split = count;
    count += (uint32_t)ahead;
    hipStream_t st = w.st;
    if (next && ahead && g->model == IMM_LT) {
        if (!w.counts_next)
            IMM_TRY(w.arena.alloc((void**)&w.counts_next, (uint64_t)w.n * 4,
                                  "counts (next round's ids)"));
        HIP_TRY(hipMemsetAsync(w.counts_next, 0, (uint64_t)w.n * 4, st));
        w.pending_next = std::min<uint64_t>(next, ahead);
    }
    // a pass of a multi-instance launch uses the launch's shared giant-set
    // slots; the workspace's own are made when a retry pass needs them
    if (!multi) IMM_TRY(ws_big_scratch(w, g));
    IMM_TRY(grow(w.arena, &w.stage_off, &w.cap_so, count, 0, st, "stage_off"));
    IMM_TRY(grow(w.arena, &w.sizes, &w.cap_sz, count, 0, st, "sizes"));
    IMM_TRY(grow(w.arena, &w.defer, &w.cap_df, count, 0, st, "defer list"));
    IMM_TRY(grow(w.arena, &w.retry, &w.cap_rt, count, 0, st, "retry list"));
    IMM_TRY(grow(w.arena, &w.spare, &w.cap_sp, count, 0, st, "retry list"));
    if (g->model == IMM_IC) {
        IMM_TRY(grow(w.arena, &w.pend, &w.cap_pd, count, 0, st, "pending list"));
        IMM_TRY(grow(w.arena, &w.over, &w.cap_ov, count, 0, st, "huge-set list"));
    }
    {
        // expected entries plus the unused tails of every wave's (IC) or
        // lane's (LT) staging chunk
        // with no measured mean yet, a generous guess (a shortfall costs a
        // retry pass, an excess only memory)
        const double mean = w.mean_size > 0 ? w.mean_size : 64.0;
        uint64_t tails;
        if (g->model == IMM_IC) {
            const uint64_t waves = std::min<uint64_t>(
                ic_small_grid(w.device), (count + kIcTicketChunk - 1) / kIcTicketChunk);
            tails = waves * kIcStageChunk;
        } else {
            const uint64_t walks = std::min<uint64_t>(
                (uint64_t)lt_small_grid(w.device, g->lt_bloom_bits, g->lt_lanes) * 64u / g->lt_lanes,
                count);
            tails = walks * kLtChunk;
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
    if (dense_min_of(w, g) != 0xFFFFFFFFu) {
        // the rate of dense sets seen while tuning, or among this pool's sets
        // once there are some
        double rate = g->dense_rate > 0.0 ? 1.2 * g->dense_rate : 0.0;
        if (w.n_sets >= 4096) rate = 1.2 * (double)w.n_dense / (double)w.n_sets;
        // IMM_DENSE_SCALE (a factor, default 1) scales this estimate; 0
        // exercises the path that adds slots and redoes the sets that found
        // none
        if (const char* e = std::getenv("IMM_DENSE_SCALE")) rate *= std::max(0.0, std::atof(e));
        IMM_TRY(ws_dense_reserve(w, w.n_dense + (uint64_t)(rate * (double)count) + 256,
                                 w.n_dense));
    }
    HIP_TRY(hipMemsetAsync(w.sc, 0, offsetof(DevScalars, stats), st));
    w.pending_count = count;
    w.pending_split = split;
    w.pending_lo = id_lo;
    if (multi) {
        w.pending_multi = true;
        return IMM_OK;
    }
    return sample_pass(w, g, seed, id_lo, count, nullptr, nullptr, count, w.retry,
                       &w.sc->retry_n, true);
}

IcTask ws_ic_task(Workspace& w, const imm_graph* g, uint64_t seed, uint32_t qcap) {
    IcTask t{};
    t.g = ic_view(g);
    t.rg = SampleRange{seed, w.pending_lo, (uint32_t)w.pending_count, nullptr, nullptr};
    t.o = sample_out(w, g, w.retry, &w.sc->retry_n);
    t.pend = w.pend;
    t.pend_n = &w.sc->pend_n;
    t.qcap = std::min<uint32_t>(w.n, qcap);
    return t;
}

imm_status ws_after_multi(Workspace& w) {
    HIP_TRY(hipMemcpyAsync(w.hsc, w.sc, sizeof(DevScalars), hipMemcpyDeviceToHost, w.st));
    return IMM_OK;
}

imm_status ws_extend_finish(Workspace& w, const imm_graph* g, uint64_t seed) {
    if (w.pending_count == 0) return IMM_OK;
    const uint32_t count = (uint32_t)w.pending_count;
    const uint32_t split = (uint32_t)w.pending_split;
    const uint64_t id_lo = w.pending_lo;
    w.pending_count = 0;
    hipStream_t st = w.st;
    // sets that found the staging buffer full: grow it (keeping what is
    // stored), continue at the old capacity, and redo just those sets
    uint32_t* in = w.retry;
    uint32_t* in_n = &w.sc->retry_n;
    uint32_t* out_l = w.spare;
    uint32_t* out_n = &w.sc->spare_n;
    uint32_t failed = w.hsc->retry_n;
    for (int guard = 0; failed; ++guard) {
        if (guard == 32) return fail(IMM_ENOMEM, "staging could not be grown enough");
        if (w.hsc->dense_n > w.cap_dense) {
            // dense sets that found no bitmap slot: more slots (every slot
            // below the old capacity holds a set), the cursor back at the
            // stored ones; w.n_dense stays the count before this pass, whose
            // new sets are all counted below
            const uint64_t stored = w.cap_dense;
            IMM_TRY(ws_dense_reserve(w, w.hsc->dense_n + w.hsc->dense_n / 4 + 256, stored));
            const uint32_t cur = (uint32_t)stored;
            HIP_TRY(hipMemcpyAsync(&w.sc->dense_n, &cur, 4, hipMemcpyHostToDevice, st));
        }
        if (w.hsc->cursor > w.stage_cap) {
            const uint64_t used = w.stage_cap;
            const uint64_t old_cap = w.stage_cap;
            const double mean = w.mean_size > 0 ? w.mean_size : 64.0;
            uint64_t need =
                old_cap + (uint64_t)(mean * 2.0 * failed) + (uint64_t)failed * 64 + (1u << 20);
            need = std::max<uint64_t>(need, old_cap * 2);
            uint64_t cap = w.stage_cap;
            IMM_TRY(grow(w.arena, &w.stage, &cap, need, used, st, "staging"));
            w.stage_cap = cap;
            // at a multiple of four: the LT walk kernel reads its chunks in
            // aligned 16-byte groups (cap >= 2 old_cap, so this stays in bounds)
            const unsigned long long cur = (old_cap + 3) & ~3ull;
            HIP_TRY(hipMemcpyAsync(&w.sc->cursor, &cur, 8, hipMemcpyHostToDevice, st));
        }
        HIP_TRY(hipMemsetAsync(out_n, 0, 4, st));
        IMM_TRY(ws_big_scratch(w, g));
        IMM_TRY(sample_pass(w, g, seed, id_lo, count, in, in_n, failed, out_l, out_n, false));
        HIP_TRY(hipStreamSynchronize(st));
        std::swap(in, out_l);
        std::swap(in_n, out_n);
        failed = (in == w.retry) ? w.hsc->retry_n : w.hsc->spare_n;
    }

    // the new dense sets' members in the dense counts (one bitmap column sum)
    {
        const uint64_t nd = std::min<uint64_t>(w.hsc->dense_n, w.cap_dense);
        if (nd > w.n_dense) {
            const int tc = w.timer.open(1, st);
            HIP_TRY(launch_dense_count(w.dense_bits, w.dense_words, (uint32_t)w.n_dense,
                                       (uint32_t)nd, w.n, w.dense_counts, st));
            w.timer.close(tc, st);
        }
        w.n_dense = nd;
        w.dense_entries = w.hsc->dense_entries;
    }
    // compaction: set_off[n_sets .. n_sets+count] (based on the device copy of
    // set_off[n_sets]) and the copy into the pool
    // (only the first `split` sets; the ones drawn ahead wait in staging)
    const uint64_t stored_bound = std::min<uint64_t>(w.hsc->cursor, w.stage_cap);
    IMM_TRY(grow(w.arena, &w.set_off, &w.cap_sets, w.n_sets + split + 1, w.n_sets + 1, st,
                 "set_off"));
    IMM_TRY(grow(w.arena, &w.set_vtx, &w.cap_entries, w.p_ub + stored_bound + 1,
                 std::min(w.p_ub, w.cap_entries), st, "set_vtx"));
    IMM_TRY(grow(w.arena, &w.scan_tmp, &w.cap_scan, scan_tmp_entries(split), 0, st, "scan tmp"));
    const int tc = w.timer.open(1, st);
    HIP_TRY(launch_scan_u32(w.sizes, nullptr, w.set_off + w.n_sets, split, 0,
                            w.set_off + w.n_sets, w.scan_tmp, st));
    HIP_TRY(launch_compact(w.stage, w.stage_off, w.set_off, w.n_sets, split, w.set_vtx, st));
    w.timer.close(tc, st);
    w.n_sets += split;
    w.p_ub += stored_bound;
    w.ahead_n = count - split;
    w.ahead_split = split;
    w.ahead_next = std::min<uint64_t>(w.pending_next, w.ahead_n);
    w.ahead_bound = w.ahead_n ? stored_bound : 0;
    return IMM_OK;
}

imm_status ws_extend(Workspace& w, const imm_graph* g, uint64_t seed, uint64_t id_lo,
                     uint64_t count) {
    IMM_TRY(ws_extend_launch(w, g, seed, id_lo, count));
    HIP_TRY(hipStreamSynchronize(w.st));
    return ws_extend_finish(w, g, seed);
}

// Read the exact pool size (and the device error flag) at a synchronisation.
imm_status ws_sync_pool(Workspace& w) {
    HIP_TRY(hipMemcpyAsync(w.hp, w.set_off + w.n_sets, 8, hipMemcpyDeviceToHost, w.st));
    HIP_TRY(hipMemcpyAsync(w.herr, &w.sc->err, 4, hipMemcpyDeviceToHost, w.st));
    HIP_TRY(hipStreamSynchronize(w.st));
    return IMM_OK;
}

imm_status ws_restart_pool(Workspace& w) {
    hipStream_t st = w.st;
    w.n_sets = 0;
    w.p_exact = 0;
    w.p_ub = 0;
    w.nseg = 0;
    w.indexed_sets = 0;
    w.p_indexed = 0;
    w.pend_lo = w.pend_hi = 0;
    HIP_TRY(hipMemsetAsync(w.counts_acc, 0, (uint64_t)w.n * 4, st));
    HIP_TRY(hipMemsetAsync(w.counts_prev, 0, (uint64_t)w.n * 4, st));
    HIP_TRY(hipMemsetAsync(w.set_off, 0, 8, st));
    w.n_dense = 0;
    w.dense_entries = 0;
    w.ahead_n = 0;
    w.ahead_next = 0;
    HIP_TRY(hipMemsetAsync(&w.sc->dense_n, 0, 16, st));
    if (w.dense_counts) HIP_TRY(hipMemsetAsync(w.dense_counts, 0, (uint64_t)w.n * 4, st));
    return IMM_OK;
}

imm_status ws_coverage(Workspace& w, const uint32_t* seeds, uint32_t k, uint64_t* out) {
    hipStream_t st = w.st;
    const uint64_t vwords = (uint64_t)w.n / 32 + 1;
    const uint64_t swords = w.n_sets / 32 + 1;
    IMM_TRY(grow(w.arena, &w.mark, &w.cap_mark, vwords + swords, 0, st, "coverage bitmaps"));
    if (!w.cov_count) IMM_TRY(w.arena.alloc((void**)&w.cov_count, 8, "coverage count"));
    HIP_TRY(hipMemsetAsync(w.mark, 0, (vwords + swords) * 4, st));
    HIP_TRY(hipMemsetAsync(w.cov_count, 0, 8, st));
    HIP_TRY(launch_cover_count(w.set_off, w.set_vtx, w.n_sets, seeds, k, w.mark,
                               w.mark + vwords, w.cov_count, st));
    unsigned long long c = 0;
    HIP_TRY(hipMemcpyAsync(&c, w.cov_count, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    *out = c;
    return IMM_OK;
}

void ws_note_pool(Workspace& w, uint64_t sets_before) {
    const uint64_t p = *w.hp;
    if (w.n_sets > sets_before)
        w.mean_size = (double)(p - w.p_exact) / (double)(w.n_sets - sets_before);
    w.p_exact = p;
    w.p_ub = p;
    if (w.indexed_sets == w.n_sets) w.p_indexed = p;
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
    const int ti = w.timer.open(2, st);
    const uint32_t count = (uint32_t)(w.n_sets - w.indexed_sets);
    const uint32_t shift = index_bucket_shift(w.n);
    // sets whose members are not counted yet
    const uint64_t pend_lo = w.pend_lo, pend_hi = w.pend_hi;
    const bool pending = pend_hi > pend_lo;
    w.pend_lo = w.pend_hi = 0;
    // IMM_INDEX_ATOMIC / IMM_INDEX_PARTITION force either build (comparisons
    // and tests); results do not depend on it
    const bool atomic_scatter = std::getenv("IMM_INDEX_ATOMIC") != nullptr;
    const bool force_partition = std::getenv("IMM_INDEX_PARTITION") != nullptr;
    // entries of the new sets: at most the pool bound less the indexed ones
    const uint64_t seg_ub = w.p_ub - std::min(w.p_indexed, w.p_ub);
    // the pairs take 8 bytes per entry of the segment: a segment too large
    // for kIndexPairsBytes (or a quarter of what the budget leaves) is
    // indexed by the atomic scatter instead
    uint64_t pair_room = kIndexPairsBytes;
    if (w.arena.budget)
        pair_room = std::min(pair_room, (w.arena.budget - std::min(w.arena.budget, w.arena.used)) / 4);
    const bool pairs_fit = w.cap_pairs > seg_ub || (seg_ub + 1) * 8 <= pair_room;
    // a small segment costs the scatter less than the partition's two extra
    // launches
    const bool partition = shift < 32 && !atomic_scatter && pairs_fit &&
                           (seg_ub >= kIndexPartitionMin || force_partition);
    // partition tiles of about 32 K entries (64 K ones were slower)
    const double mean = std::max(1.0, (double)seg_ub / (double)count);
    const uint32_t groups = (uint32_t)std::min(64.0, std::max(1.0, 32768.0 / (256.0 * mean)));
    if (partition) {
        IMM_TRY(grow(w.arena, &w.inv_pairs, &w.cap_pairs, seg_ub + 1, 0, st, "index pairs"));
        if (!w.iplan) IMM_TRY(w.arena.alloc((void**)&w.iplan, sizeof(IndexPlan), "index plan"));
    }
    if (partition && (pending || w.lt) && w.n_dense == 0) {
        // the segment and the counts from the sets themselves: no count pass
        // over the uncounted sets, no scan of the count increase. It takes
        // one workgroup per bucket, so it serves LT pools (walks spread
        // their members over the buckets) and segments with uncounted sets
        HIP_TRY(launch_inv_counting(w.set_off, w.set_vtx, w.indexed_sets, count, groups, w.n,
                                    shift, io, w.counts_prev, w.counts_acc, w.iplan, w.inv_pairs,
                                    w.cap_pairs, w.inv_set, &w.sc->err, w.device, st));
    } else {
        if (pending)
            HIP_TRY(launch_count_sets(w.set_off, pend_lo, pend_hi, w.set_vtx, w.counts_acc, st));
        HIP_TRY(launch_scan_u32(w.counts_acc, w.counts_prev, io, w.n, 0,
                                w.set_off + w.indexed_sets, w.scan_tmp, st));
        HIP_TRY(hipMemsetAsync(w.inv_cursor, 0, (uint64_t)w.n * 4, st));
        if (partition)
            HIP_TRY(launch_inv_partitioned(w.set_off, w.set_vtx, w.indexed_sets, count, groups,
                                           w.n, shift, io, w.iplan, w.inv_pairs, w.cap_pairs,
                                           w.inv_cursor, w.inv_set, &w.sc->err, w.device, st));
        else
            HIP_TRY(launch_inv_scatter(w.set_off, w.set_vtx, w.indexed_sets, count, io,
                                       w.inv_cursor, w.inv_set, &w.sc->err, st));
    }
    HIP_TRY(hipMemcpyAsync(w.counts_prev, w.counts_acc, (uint64_t)w.n * 4,
                           hipMemcpyDeviceToDevice, st));
    w.timer.close(ti, st);
    ++w.nseg;
    w.indexed_sets = w.n_sets;
    return IMM_OK;
}

namespace {

// The selection state of a pool of n_sets sets (entries bounded by p_ub,
// indexed in nseg segments, cacc[v] the length of v's index lists): the
// workspace's selection buffers grown and cleared, the working counts, the
// candidate list, and the descriptor, on stream st.
imm_status ws_select_state(Workspace& w, uint32_t k, SelectDesc* d, const uint32_t* cacc,
                           uint64_t n_sets, uint32_t nseg, uint64_t p_ub, hipStream_t st) {
    IMM_TRY(grow(w.arena, &w.covered, &w.cap_cov, n_sets / 32 + 1, 0, st, "covered"));
    if (w.cap_k < k) {
        if (w.seeds_d) {
            HIP_TRY(hipStreamSynchronize(st));
            w.arena.release(w.seeds_d);
            w.arena.release(w.gains_d);
            w.arena.release(w.slots);  // also holds chunk_n and cov_entries
            (void)hipHostFree(w.gains_h);
            w.gains_h = nullptr;
        }
        IMM_TRY(w.arena.alloc((void**)&w.seeds_d, (uint64_t)k * 4, "seeds"));
        IMM_TRY(w.arena.alloc((void**)&w.gains_d, (uint64_t)k * 4, "gains"));
        // per seed step: argmax slots, two queue lengths, covered total; one
        // block, cleared with one fill per selection
        IMM_TRY(w.arena.alloc((void**)&w.slots, (uint64_t)k * (kArgSlots * 8 + 16),
                              "seed-step state"));
        w.chunk_n = reinterpret_cast<uint32_t*>(w.slots + (uint64_t)k * kArgSlots);
        w.cov_entries = reinterpret_cast<unsigned long long*>(w.chunk_n + 2ull * k);
        HIP_TRY(hipHostMalloc((void**)&w.gains_h, (uint64_t)k * 4, hipHostMallocDefault));
        w.cap_k = k;
    }
    // a seed's queue entries: at most one per started 64 members of every set
    IMM_TRY(grow(w.arena, &w.chunks, &w.cap_chunks, n_sets + p_ub / 64 + 1, 0, st,
                 "chunk queue"));
    if (nseg > kMaxSegments) return fail(IMM_EOVERFLOW, "too many index segments");
    // the candidate list from the working counts (steps 1 .. k-1 may use it);
    // IMM_CAND_MAX bounds it (0: every step in full)
    uint32_t cand_max = kCandMax;
    if (const char* e = std::getenv("IMM_CAND_MAX"))
        cand_max = (uint32_t)std::min<long>(std::max<long>(std::atol(e), 0), (long)kCandMax);
    const bool cand = cand_max > 0 && k >= 2;
    // working counts, and the list of vertices whose index lists are long;
    // the same launch clears the covered bits, the seed-step block (its
    // layout follows the capacity cap_k, not this k) and the candidate state
    HIP_TRY(hipMemsetAsync(w.heavy + w.n, 0, 4, st));
    ZeroSpans z;
    z.p[0] = w.covered;
    z.words[0] = n_sets / 32 + 1;
    z.p[1] = reinterpret_cast<uint32_t*>(w.slots);
    z.words[1] = w.cap_k * (kArgSlots * 8 + 16) / 4;
    if (cand) {
        z.p[2] = w.cand_state;
        z.words[2] = kCandHead + kCandBins;
    }
    HIP_TRY(launch_select_init2(cacc, w.n_dense ? w.dense_counts : nullptr, w.counts_work, w.n,
                                w.heavy, w.heavy + w.n, st, z));
    // dense claims: per-step marks, then the claim cursor
    if (w.n_dense) {
        if (w.cap_mark_k < k) {
            if (w.dense_mark) {
                HIP_TRY(hipStreamSynchronize(st));
                w.arena.release(w.dense_mark);
                w.dense_mark = nullptr;
            }
            IMM_TRY(w.arena.alloc((void**)&w.dense_mark, ((uint64_t)k + 2) * 4, "dense marks"));
            w.cap_mark_k = k;
        }
        HIP_TRY(hipMemsetAsync(w.dense_mark, 0, (w.cap_mark_k + 2) * 4, st));
    }
    if (cand)
        HIP_TRY(launch_cand_build(w.counts_work, w.n, cand_max, w.cand, w.cand_bits,
                                  w.cand_state, st));
    *d = SelectDesc{w.counts_work, cacc,         w.heavy,     w.heavy + w.n, w.inv_offs,
                    w.inv_set,     w.set_off,    w.set_vtx,   w.covered,     w.slots,
                    w.seeds_d,     w.gains_d,    w.chunks,    w.chunk_n,     w.cap_chunks,
                    w.cov_entries, w.n,          k,           nseg,          (uint32_t)n_sets,
                    0,             0,            0,           0,             w.update_mode};
    if (w.n_dense) {
        d->dense_bits = w.dense_bits;
        d->dense_sid = w.dense_sid;
        d->dense_size = w.dense_size;
        d->dense_list = w.dense_list;
        d->dense_list_n = w.dense_mark + w.cap_mark_k + 1;
        d->dense_mark = w.dense_mark;
        d->dense_entries = w.dense_entries;
        d->n_dense = (uint32_t)w.n_dense;
        d->dense_words = w.dense_words;
    }
    if (cand) {
        d->cand = w.cand;
        d->cand_bits = w.cand_bits;
        d->cand_state = w.cand_state;
    }
    w.desc_last = *d;
    return IMM_OK;
}

}  // namespace

imm_status ws_select_prepare(Workspace& w, uint32_t k, SelectDesc* d) {
    IMM_TRY(ws_index_update(w));
    return ws_select_state(w, k, d, w.counts_acc, w.n_sets, w.nseg, w.p_ub, w.st);
}

imm_status ws_select_copy_out(Workspace& w, uint32_t k, hipStream_t st) {
    HIP_TRY(hipMemcpyAsync(w.gains_h, w.gains_d, (uint64_t)k * 4, hipMemcpyDeviceToHost, st));
    if (w.desc_last.cand_state)
        HIP_TRY(hipMemcpyAsync(w.cand_h, w.cand_state, kCandHead * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(w.hp, w.set_off + w.n_sets, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(w.herr, &w.sc->err, 4, hipMemcpyDeviceToHost, st));
    return IMM_OK;
}

// A selection that halted at step h (its best listed count fell below tau):
// every working count recounted exactly from the index and the covered sets,
// then steps h .. k-1 in full, on the workspace's stream, waited for.
imm_status ws_select_resume(Workspace& w, uint32_t k, uint32_t h) {
    hipStream_t st = w.st;
    SelectDesc d = w.desc_last;
    d.cand = nullptr;
    d.cand_bits = nullptr;
    d.cand_state = nullptr;
    d.arg_lo = 0;
    d.arg_cnt = argmax_blocks(w.n);
    d.sel_lo = 0;
    d.sel_cnt = select_blocks(w.device, w.n_sets, 1);
    d.dense_lo = 0;
    d.dense_cnt = dense_blocks(d.n_dense, d.dense_words);
    SelectDesc r = d;
    r.update = kUpdateRecount;
    const int ts = w.timer.open(3, st);
    HIP_TRY(hipMemcpyAsync(w.desc_d, &r, sizeof(r), hipMemcpyHostToDevice, st));
    HIP_TRY(launch_select_recount(w.desc_d, h - 1, d.sel_cnt, d.dense_cnt, st));
    HIP_TRY(hipStreamSynchronize(st));
    HIP_TRY(hipMemcpyAsync(w.desc_d, &d, sizeof(d), hipMemcpyHostToDevice, st));
    for (uint32_t t = h; t < k; ++t)
        HIP_TRY(launch_select_step(w.desc_d, 1, t, d.arg_cnt, d.sel_cnt, d.dense_cnt, st));
    w.timer.close(ts, st);
    HIP_TRY(hipMemcpyAsync(w.gains_h, w.gains_d, (uint64_t)k * 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    return IMM_OK;
}

imm_status ws_select_finish(Workspace& w, uint32_t k, uint64_t sets_before, uint64_t* covered) {
    if (*w.herr) return fail(IMM_EDEVICE, "internal error: occurrence counts disagree with the pool");
    if (w.desc_last.cand_state) {
        const uint32_t h = w.cand_h[1];
        if (w.cand_h[0] == 1u) w.cand_steps += (h ? h : k) - 1u;
        if (h) {
            ++w.cand_halts;
            IMM_TRY(ws_select_resume(w, k, h));
        }
    }
    ws_note_pool(w, sets_before);
    uint64_t c = 0;
    for (uint32_t i = 0; i < k; ++i) c += w.gains_h[i];
    *covered = c;
    return IMM_OK;
}

SelectGraph::~SelectGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
}

int SelectGraph::launch(const SelectDesc* d, uint32_t q, uint32_t km, uint32_t at, uint32_t stot,
                        uint32_t dtot, hipStream_t st, bool* captured) {
    *captured = false;
    if (!exec || d != descs || q != nq || km != kmax || at != arg_total || stot != sel_total ||
        dtot != dense_total) {
        // the kernels only: nothing in the captured sequence is a memset or
        // a copy (the descriptors are copied before each launch)
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        hipError_t le = hipSuccess;
        for (uint32_t t = 0; le == hipSuccess && t < km; ++t)
            le = launch_select_step(d, q, t, at, stot, dtot, st);
        hipGraph_t graph = nullptr;
        const hipError_t ce = hipStreamEndCapture(st, &graph);
        if (le != hipSuccess || ce != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            return 0;
        }
        bool have = false;
        if (exec) {
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult res = hipGraphExecUpdateError;
            have = hipGraphExecUpdate(exec, graph, &bad, &res) == hipSuccess &&
                   res == hipGraphExecUpdateSuccess;
            if (!have) {
                // a refused update (a different topology or launch shape) is
                // no failure: clear it so no later launch reports it, and
                // instantiate anew
                (void)hipGetLastError();
                (void)hipGraphExecDestroy(exec);
                exec = nullptr;
            }
        }
        if (!have) have = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        (void)hipGraphDestroy(graph);
        if (!have) {
            exec = nullptr;
            (void)hipGetLastError();
            return 0;
        }
        descs = d;
        nq = q;
        kmax = km;
        arg_total = at;
        sel_total = stot;
        dense_total = dtot;
        *captured = true;
    }
    return hipGraphLaunch(exec, st) == hipSuccess ? 1 : -1;
}

SampleGraph::~SampleGraph() {
    if (exec) (void)hipGraphExecDestroy(exec);
}

int SampleGraph::launch(const IcTask* t, uint32_t nt, const uint32_t* pre, uint32_t* tk,
                        uint32_t tm, uint32_t blk, const BigScratch& bs, int dev, hipStream_t st,
                        bool* captured) {
    *captured = false;
    const bool same = exec && t == tasks && nt == ntask && pre == prefix && tk == tickets &&
                      tm == team && blk == block && bs.bitmaps == b.bitmaps &&
                      bs.queues == b.queues && bs.words == b.words && bs.slots == b.slots &&
                      bs.qcap == b.qcap && dev == device;
    if (!same) {
        // kernels only: the task table and its tickets are copied to the
        // device before every launch of the graph
        if (hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal) != hipSuccess) {
            (void)hipGetLastError();
            return 0;
        }
        const hipError_t le = launch_ic_multi(t, nt, pre, tk, tm, blk, bs, dev, st);
        hipGraph_t graph = nullptr;
        const hipError_t ce = hipStreamEndCapture(st, &graph);
        if (le != hipSuccess || ce != hipSuccess || !graph) {
            if (graph) (void)hipGraphDestroy(graph);
            (void)hipGetLastError();
            return 0;
        }
        bool have = false;
        if (exec) {
            hipGraphNode_t bad = nullptr;
            hipGraphExecUpdateResult res = hipGraphExecUpdateError;
            have = hipGraphExecUpdate(exec, graph, &bad, &res) == hipSuccess &&
                   res == hipGraphExecUpdateSuccess;
            if (!have) {
                // a refused update is no failure: clear it and instantiate anew
                (void)hipGetLastError();
                (void)hipGraphExecDestroy(exec);
                exec = nullptr;
            }
        }
        if (!have) have = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess;
        (void)hipGraphDestroy(graph);
        if (!have) {
            exec = nullptr;
            (void)hipGetLastError();
            return 0;
        }
        tasks = t;
        ntask = nt;
        prefix = pre;
        tickets = tk;
        team = tm;
        block = blk;
        b = bs;
        device = dev;
        *captured = true;
    }
    return hipGraphLaunch(exec, st) == hipSuccess ? 1 : -1;
}

imm_status ws_select_launch(Workspace& w, uint32_t k, bool graph, int* graph_out) {
    hipStream_t st = w.st;
    SelectDesc& d = w.desc_h;
    IMM_TRY(ws_select_prepare(w, k, &d));
    d.arg_cnt = argmax_blocks(w.n);
    d.sel_cnt = select_blocks(w.device, w.n_sets, 1);
    d.dense_cnt = dense_blocks(d.n_dense, d.dense_words);
    HIP_TRY(hipMemcpyAsync(w.desc_d, &d, sizeof(d), hipMemcpyHostToDevice, st));
    const int ts = w.timer.open(3, st);
    int launched = 0;
    bool captured = false;
    if (graph) {
        launched = w.sel_graph.launch(w.desc_d, 1, k, d.arg_cnt, d.sel_cnt, d.dense_cnt, st,
                                      &captured);
        if (launched < 0) return fail(IMM_EDEVICE, "select: graph launch failed");
    }
    if (launched == 0)
        for (uint32_t t = 0; t < k; ++t)
            HIP_TRY(launch_select_step(w.desc_d, 1, t, d.arg_cnt, d.sel_cnt, d.dense_cnt, st));
    if (graph_out) *graph_out = launched == 0 ? 0 : (captured ? 2 : 1);
    w.timer.close(ts, st);
    return ws_select_copy_out(w, k, st);
}

imm_status ws_select(Workspace& w, uint32_t k, uint64_t sets_before, uint64_t* covered) {
    IMM_TRY(ws_select_launch(w, k));
    HIP_TRY(hipStreamSynchronize(w.st));
    return ws_select_finish(w, k, sets_before, covered);
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
    HIP_TRY(launch_sort_small(w.set_off, (uint32_t)w.n_sets, w.set_vtx, big_list, &w.sc->big_flag,
                              st));
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
    if (w.n_dense == 0) return IMM_OK;
    // dense sets: their bitmaps, in set order, replace their empty lists
    // (members ascending, as a bitmap lists them); their counts are added
    const uint64_t nd = w.n_dense, words = w.dense_words;
    std::vector<uint32_t> sid(nd), bits(nd * words);
    HIP_TRY(hipMemcpy(sid.data(), w.dense_sid, nd * 4, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(bits.data(), w.dense_bits, nd * words * 4, hipMemcpyDeviceToHost));
    if (counts) {
        std::vector<uint32_t> dc(w.n);
        HIP_TRY(hipMemcpy(dc.data(), w.dense_counts, (uint64_t)w.n * 4, hipMemcpyDeviceToHost));
        for (uint32_t v = 0; v < w.n; ++v) (*counts)[v] += dc[v];
    }
    if (!so && !sv) return IMM_OK;
    std::vector<uint64_t> lso(w.n_sets + 1);
    HIP_TRY(hipMemcpy(lso.data(), w.set_off, (w.n_sets + 1) * 8, hipMemcpyDeviceToHost));
    std::vector<int64_t> dense_of(w.n_sets, -1);
    for (uint64_t b = 0; b < nd; ++b) dense_of[sid[b]] = (int64_t)b;
    auto popc = [&](uint64_t b) {
        uint64_t c = 0;
        for (uint64_t x = 0; x < words; ++x) c += (uint64_t)__builtin_popcount(bits[b * words + x]);
        return c;
    };
    std::vector<uint64_t> off(w.n_sets + 1, 0);
    for (uint64_t j = 0; j < w.n_sets; ++j)
        off[j + 1] = off[j] + (dense_of[j] >= 0 ? popc((uint64_t)dense_of[j]) : lso[j + 1] - lso[j]);
    if (sv) {
        std::vector<uint32_t> out(off[w.n_sets]);
        for (uint64_t j = 0; j < w.n_sets; ++j) {
            uint64_t o = off[j];
            if (dense_of[j] < 0) {
                for (uint64_t t = lso[j]; t < lso[j + 1]; ++t) out[o++] = (*sv)[t];
                continue;
            }
            const uint32_t* bm = bits.data() + (uint64_t)dense_of[j] * words;
            for (uint64_t x = 0; x < words; ++x)
                for (uint32_t y = bm[x]; y; y &= y - 1)
                    out[o++] = (uint32_t)(32 * x + (uint64_t)__builtin_ctz(y));
        }
        sv->swap(out);
    }
    if (so) so->swap(off);
    return IMM_OK;
}

// ---------------------------------------------------------- speculation --

namespace {

void swap_sel(Workspace& w, SelBufs& b) {
    std::swap(w.counts_work, b.counts_work);
    std::swap(w.heavy, b.heavy);
    std::swap(w.covered, b.covered);
    std::swap(w.cap_cov, b.cap_cov);
    std::swap(w.slots, b.slots);
    std::swap(w.chunk_n, b.chunk_n);
    std::swap(w.cov_entries, b.cov_entries);
    std::swap(w.chunks, b.chunks);
    std::swap(w.cap_chunks, b.cap_chunks);
    std::swap(w.seeds_d, b.seeds_d);
    std::swap(w.gains_d, b.gains_d);
    std::swap(w.cap_k, b.cap_k);
    std::swap(w.gains_h, b.gains_h);
    std::swap(w.desc_d, b.desc_d);
    std::swap(w.desc_h, b.desc_h);
    std::swap(w.cand, b.cand);
    std::swap(w.cand_bits, b.cand_bits);
    std::swap(w.cand_state, b.cand_state);
    std::swap(w.cand_h, b.cand_h);
    std::swap(w.desc_last, b.desc_last);
}

// Whether a segment of at most seg_ub entries is indexed by the partition
// (as ws_index_update decides), given the capacity of the pair buffer it
// would use.
bool index_by_partition(const Workspace& w, uint64_t seg_ub, uint64_t cap_pairs) {
    if (index_bucket_shift(w.n) >= 32 || std::getenv("IMM_INDEX_ATOMIC")) return false;
    uint64_t pair_room = kIndexPairsBytes;
    if (w.arena.budget)
        pair_room = std::min(pair_room, (w.arena.budget - std::min(w.arena.budget, w.arena.used)) / 4);
    const bool fits = cap_pairs > seg_ub || (seg_ub + 1) * 8 <= pair_room;
    return fits && (seg_ub >= kIndexPartitionMin || std::getenv("IMM_INDEX_PARTITION"));
}

}  // namespace

bool ws_spec_possible(const Workspace& w) {
    // (its counts start from the pool's, which must hold every set's members)
    return w.ahead_next > 0 && w.ahead_n >= w.ahead_next && w.counts_next && w.n_dense == 0 &&
           w.pend_hi == w.pend_lo && w.n_sets + w.ahead_next <= 0xFFFFFFFFull;
}

imm_status ws_spec_reserve(Workspace& w, uint32_t k) {
    hipStream_t st = w.st;
    const uint64_t kk = w.ahead_next;
    const uint64_t lo = w.n_sets, hi = lo + kk;
    const uint64_t p_hi = w.p_ub + w.ahead_bound;
    const uint64_t stride = (uint64_t)w.n + 1;
    // the index segment this round's selection builds first, then the
    // speculative one
    const uint32_t nseg = w.nseg + (w.indexed_sets < w.n_sets ? 1u : 0u);
    if (nseg + 1 > kMaxSegments) return fail(IMM_EOVERFLOW, "too many index segments");
    IMM_TRY(grow(w.arena, &w.set_off, &w.cap_sets, hi + 1, lo + 1, st, "set_off"));
    IMM_TRY(grow(w.arena, &w.scan_tmp, &w.cap_scan, scan_tmp_entries(w.n), 0, st, "scan tmp"));
    IMM_TRY(grow(w.arena, &w.scan_tmp2, &w.cap_scan2,
                 std::max(scan_tmp_entries(kk), scan_tmp_entries(w.n)), 0, st,
                 "scan tmp (speculative)"));
    if (!w.inv_cursor2)
        IMM_TRY(w.arena.alloc((void**)&w.inv_cursor2, (uint64_t)w.n * 4,
                              "inv_cursor (speculative)"));
    IMM_TRY(grow(w.arena, &w.inv_offs, &w.cap_offs, ((uint64_t)nseg + 1) * stride,
                 (uint64_t)w.nseg * stride, st, "index offsets"));
    IMM_TRY(grow(w.arena, &w.inv_set, &w.cap_inv, p_hi + 1, std::min(w.p_ub, w.cap_inv), st,
                 "inv_set"));
    const uint64_t cur_ub = w.p_ub - std::min(w.p_indexed, w.p_ub);
    if (w.indexed_sets < w.n_sets && index_by_partition(w, cur_ub, w.cap_pairs)) {
        IMM_TRY(grow(w.arena, &w.inv_pairs, &w.cap_pairs, cur_ub + 1, 0, st, "index pairs"));
        if (!w.iplan) IMM_TRY(w.arena.alloc((void**)&w.iplan, sizeof(IndexPlan), "index plan"));
    }
    if (index_by_partition(w, w.ahead_bound, w.cap_pairs2)) {
        IMM_TRY(grow(w.arena, &w.inv_pairs2, &w.cap_pairs2, w.ahead_bound + 1, 0, st,
                     "index pairs (speculative)"));
        if (!w.iplan2)
            IMM_TRY(w.arena.alloc((void**)&w.iplan2, sizeof(IndexPlan), "index plan (speculative)"));
    }
    if (!w.counts_spec)
        IMM_TRY(w.arena.alloc((void**)&w.counts_spec, (uint64_t)w.n * 4, "counts (speculative)"));
    // the second selection buffers, at the sizes ws_select_state will ask for
    SelBufs& b = w.sel2;
    if (!b.counts_work) {
        IMM_TRY(w.arena.alloc((void**)&b.counts_work, (uint64_t)w.n * 4 + 16, "counts_work"));
        IMM_TRY(w.arena.alloc((void**)&b.heavy, (uint64_t)w.n * 4 + 16, "heavy vertex list"));
        IMM_TRY(w.arena.alloc((void**)&b.desc_d, sizeof(SelectDesc), "select descriptor"));
        IMM_TRY(w.arena.alloc((void**)&b.cand, (uint64_t)kCandMax * 4, "candidate list"));
        IMM_TRY(w.arena.alloc((void**)&b.cand_bits, ((uint64_t)w.n + 31) / 32 * 4 + 16,
                              "candidate bitmap"));
        IMM_TRY(w.arena.alloc((void**)&b.cand_state, (kCandHead + kCandBins) * 4,
                              "candidate state"));
        HIP_TRY(hipHostMalloc((void**)&b.cand_h, kCandHead * 4, hipHostMallocDefault));
    }
    IMM_TRY(grow(w.arena, &b.covered, &b.cap_cov, hi / 32 + 1, 0, st, "covered"));
    IMM_TRY(grow(w.arena, &b.chunks, &b.cap_chunks, hi + p_hi / 64 + 1, 0, st, "chunk queue"));
    if (b.cap_k < k) {
        if (b.seeds_d) {
            HIP_TRY(hipStreamSynchronize(st));
            w.arena.release(b.seeds_d);
            w.arena.release(b.gains_d);
            w.arena.release(b.slots);
            (void)hipHostFree(b.gains_h);
            b.gains_h = nullptr;
        }
        IMM_TRY(w.arena.alloc((void**)&b.seeds_d, (uint64_t)k * 4, "seeds"));
        IMM_TRY(w.arena.alloc((void**)&b.gains_d, (uint64_t)k * 4, "gains"));
        IMM_TRY(w.arena.alloc((void**)&b.slots, (uint64_t)k * (kArgSlots * 8 + 16),
                              "seed-step state"));
        b.chunk_n = reinterpret_cast<uint32_t*>(b.slots + (uint64_t)k * kArgSlots);
        b.cov_entries = reinterpret_cast<unsigned long long*>(b.chunk_n + 2ull * k);
        HIP_TRY(hipHostMalloc((void**)&b.gains_h, (uint64_t)k * 4, hipHostMallocDefault));
        b.cap_k = k;
    }
    if (!w.side) HIP_TRY(hipStreamCreateWithFlags(&w.side, hipStreamNonBlocking));
    if (!w.side_ev) HIP_TRY(hipEventCreateWithFlags(&w.side_ev, hipEventDisableTiming));
    if (!w.side_ev2) HIP_TRY(hipEventCreateWithFlags(&w.side_ev2, hipEventDisableTiming));
    return IMM_OK;
}

imm_status ws_spec_launch_index(Workspace& w, hipEvent_t after) {
    hipStream_t S = w.side;
    HIP_TRY(hipStreamWaitEvent(S, after, 0));
    const uint64_t kk = w.ahead_next, lo = w.n_sets, hi = lo + kk, split = w.ahead_split;
    const uint64_t stride = (uint64_t)w.n + 1;
    // the segment after the one this round's index update adds
    w.spec_seg = w.nseg + (w.indexed_sets < w.n_sets ? 1u : 0u);
    // the sets' offsets and members, after the pool's (as ws_take_ahead)
    HIP_TRY(launch_scan_u32(w.sizes + split, nullptr, w.set_off + lo, kk, 0, w.set_off + lo,
                            w.scan_tmp2, S));
    HIP_TRY(launch_compact(w.stage, w.stage_off + split, w.set_off, lo, (uint32_t)kk, w.set_vtx, S));
    // their index segment, and the pool's counts with them
    uint64_t* io = w.inv_offs + (uint64_t)w.spec_seg * stride;
    const uint32_t shift = index_bucket_shift(w.n);
    if (index_by_partition(w, w.ahead_bound, w.cap_pairs2)) {
        // from the sets themselves, as ws_index_update's counting build
        const double mean = std::max(1.0, (double)w.ahead_bound / (double)kk);
        const uint32_t groups =
            (uint32_t)std::min(64.0, std::max(1.0, 32768.0 / (256.0 * mean)));
        HIP_TRY(launch_inv_counting(w.set_off, w.set_vtx, lo, (uint32_t)kk, groups, w.n, shift,
                                    io, w.counts_acc, w.counts_spec, w.iplan2, w.inv_pairs2,
                                    w.cap_pairs2, w.inv_set, &w.sc->err, w.device, S));
    } else {
        // offsets from the scan of the counts kept apart (as ws_index_update,
        // with those counts as the increase)
        HIP_TRY(hipMemcpyAsync(w.counts_spec, w.counts_acc, (uint64_t)w.n * 4,
                               hipMemcpyDeviceToDevice, S));
        HIP_TRY(launch_add_counts(w.counts_next, w.counts_spec, w.n, S));
        HIP_TRY(launch_scan_u32(w.counts_next, nullptr, io, w.n, 0, w.set_off + lo, w.scan_tmp2,
                                S));
        HIP_TRY(hipMemsetAsync(w.inv_cursor2, 0, (uint64_t)w.n * 4, S));
        HIP_TRY(launch_inv_scatter(w.set_off, w.set_vtx, lo, (uint32_t)kk, io, w.inv_cursor2,
                                   w.inv_set, &w.sc->err, S));
    }
    w.spec_lo = lo;
    w.spec_hi = hi;
    return IMM_OK;
}

imm_status ws_spec_launch_select(Workspace& w, uint32_t k, hipEvent_t after) {
    hipStream_t S = w.side;
    if (w.nseg != w.spec_seg) return fail(IMM_EDEVICE, "internal error: speculative segment");
    HIP_TRY(hipStreamWaitEvent(S, after, 0));
    const uint64_t hi = w.spec_hi;
    // the selection over the pool with them, in the second buffers
    swap_sel(w, w.sel2);
    SelectDesc d{};
    imm_status s = ws_select_state(w, k, &d, w.counts_spec, hi, w.spec_seg + 1,
                                   w.p_ub + w.ahead_bound, S);
    hipError_t e = hipSuccess;
    if (s == IMM_OK) {
        d.arg_cnt = argmax_blocks(w.n);
        d.sel_cnt = select_blocks(w.device, hi, 1);
        w.desc_h = d;
        e = hipMemcpyAsync(w.desc_d, &w.desc_h, sizeof(d), hipMemcpyHostToDevice, S);
        for (uint32_t t = 0; e == hipSuccess && t < k; ++t)
            e = launch_select_step(w.desc_d, 1, t, d.arg_cnt, d.sel_cnt, 0, S);
        if (e == hipSuccess)
            e = hipMemcpyAsync(w.gains_h, w.gains_d, (uint64_t)k * 4, hipMemcpyDeviceToHost, S);
        if (e == hipSuccess && d.cand_state)
            e = hipMemcpyAsync(w.cand_h, w.cand_state, kCandHead * 4, hipMemcpyDeviceToHost, S);
    }
    swap_sel(w, w.sel2);
    IMM_TRY(s);
    HIP_TRY(e);
    w.spec = true;
    return IMM_OK;
}

imm_status ws_spec_commit(Workspace& w) {
    HIP_TRY(hipStreamSynchronize(w.side));
    const uint64_t kk = w.spec_hi - w.spec_lo;
    // the host state the next round's ws_extend_launch and ws_select_prepare
    // would have left
    w.ahead_n -= kk;
    w.ahead_split += kk;
    w.ahead_next = 0;
    w.n_sets = w.spec_hi;
    w.p_ub += w.ahead_bound;
    ++w.nseg;
    w.indexed_sets = w.n_sets;
    hipStream_t st = w.st;
    HIP_TRY(hipMemcpyAsync(w.counts_acc, w.counts_spec, (uint64_t)w.n * 4,
                           hipMemcpyDeviceToDevice, st));
    HIP_TRY(hipMemcpyAsync(w.counts_prev, w.counts_spec, (uint64_t)w.n * 4,
                           hipMemcpyDeviceToDevice, st));
    // the pool size and error flag, as the selection's copy-out leaves them
    HIP_TRY(hipMemcpyAsync(w.hp, w.set_off + w.n_sets, 8, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(w.herr, &w.sc->err, 4, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    swap_sel(w, w.sel2);
    w.spec = false;
    ++w.spec_rounds;
    return IMM_OK;
}

imm_status ws_spec_drop(Workspace& w) {
    w.spec = false;
    HIP_TRY(hipStreamSynchronize(w.side));
    return IMM_OK;
}

void fill_stats(Workspace& w, imm_stats* s) {
    double ms[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    uint64_t launches[4] = {0, 0, 0, 0};
    w.timer.collect(ms, launches);
    s->ms_sample += ms[0];
    s->ms_compact += ms[1];
    s->ms_index += ms[2];
    s->ms_select += ms[3];
    s->ms_sample_main += ms[4];
    s->ms_sample_big += ms[5];
    s->ms_sample_lane += ms[6];
    s->main_launches += launches[0];
    s->big_launches += launches[1];
    s->lane_launches += launches[2];
    const unsigned long long* t = w.hsc->stats;
    s->sets = t[kStMainSets] + t[kStBigSets] + t[kStLaneSets];
    s->entries = t[kStMainEntries] + t[kStBigEntries] + t[kStLaneSets];
    s->edges = t[kStMainEdges] + t[kStBigEdges] + t[kStLaneEdges];
    s->lane_sets = t[kStLaneSets];
    s->lane_edges = t[kStLaneEdges];
    s->live = t[kStMainLive] + t[kStBigLive];
    s->deferred = t[kStBigSets];
    s->main_sets = t[kStMainSets];
    s->main_entries = t[kStMainEntries];
    s->main_edges = t[kStMainEdges];
    s->main_live = t[kStMainLive];
    s->dense_sets = (uint32_t)std::min<uint64_t>(w.n_dense, 0xFFFFFFFFu);
    s->cand_steps = (uint32_t)std::min<uint64_t>(w.cand_steps, 0xFFFFFFFFu);
    s->cand_halts = (uint32_t)std::min<uint64_t>(w.cand_halts, 0xFFFFFFFFu);
    s->spec_rounds = (uint32_t)std::min<uint64_t>(w.spec_rounds, 0xFFFFFFFFu);
}

}  // namespace imm
