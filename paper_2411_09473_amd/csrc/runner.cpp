// runner.cpp -- IMM's sampling/selection driver (Algorithm 1) with the theta
// schedule of Tang et al. 2015, for one query or a batch of them.
//
// Each query is a state machine over iterations: sampling round i targets
// theta_i = ceil(lambda' 2^i / n) sets and ends with a greedy selection and
// the lower-bound test; after the break (or the last round) one final
// iteration targets theta = ceil(lambda* / LB) and its selection is the
// answer. A batch advances all its queries one iteration at a time: every
// query launches its sampling on its own stream, one synchronisation, then
// the selections of all queries run together (each launch of the selection
// kernels covers every query) and one more synchronisation; the FP64 theta
// decisions are taken on the host in between.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "engine.hpp"

namespace imm {

namespace {

// FP64, no contraction, this exact order (kept identical to IMM's theta
// expressions: Tang et al. 2015 Eq. 9 lambda', Eq. 6 lambda*, with ell
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
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}


}  // namespace

imm_status theta_plan(uint32_t n, uint32_t k, double eps, double ell, double* lambda_prime,
                      double* lambda_star, uint32_t* i_max) {
    if (n < 2 || k == 0 || k > n || !(eps > 0.0) || !(ell > 0.0))
        return fail(IMM_EINVAL, "theta_plan: need n >= 2, 1 <= k <= n, eps > 0, ell > 0");
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

imm_status early_plan(uint32_t n, uint32_t k, double eps, double ell, double* theta0,
                      uint32_t* i_max, double* a) {
    if (n < 2 || k == 0 || k > n || !(eps > 0.0) || !(ell > 0.0))
        return fail(IMM_EINVAL, "early_plan: need n >= 2, 1 <= k <= n, eps > 0, ell > 0");
    // IMM's lambda* (Tang et al. 2015, Eq. 6) at failure probability delta / 3,
    // delta = n^-ell, with OPT >= k: theta_max; the first pools hold
    // theta_max eps^2 k / n sets and double until they reach theta_max
    const double ln_n = std::log((double)n);
    const double logcnk = log_binom(n, k);
    const double one_m = 1.0 - kInvE;
    const double ln6d = std::log(6.0) + ell * ln_n;
    const double u = one_m * std::sqrt(ln6d) + std::sqrt(one_m * (logcnk + ln6d));
    const double theta_max = 2.0 * (double)n * u * u / (eps * eps * (double)k);
    *theta0 = theta_max * eps * eps * (double)k / (double)n;
    const double r = std::ceil(std::log2((double)n / (eps * eps * (double)k)));
    *i_max = r < 1.0 ? 1u : (uint32_t)r;
    // each of the 3 i_max bounds fails with probability at most exp(-a)
    *a = std::log(3.0 * (double)*i_max) + ell * ln_n;
    return IMM_OK;
}

namespace {
constexpr size_t kMaxCachedWorkspacesPerGraph = 8;
// sample ids of the early-stopping schedule's second pool start here
constexpr uint64_t kSecondPoolIds = 1ull << 32;
enum Schedule { kSchedImm = 0, kSchedFresh = 1, kSchedEarly = 2 };
}  // namespace

struct Query {
    imm_graph* g = nullptr;
    imm_params p{};
    hipStream_t st = nullptr;
    std::unique_ptr<Workspace> w;
    std::unique_ptr<Workspace> w2;  // early stopping: the second pool
    int sched = kSchedImm;
    double lam_p = 0, lam_s = 0, eps_p = 0, lb = 1.0;
    double theta0 = 0, a = 0, g_k = 0;  // early stopping
    uint32_t i_max = 0, i = 0;
    bool final = false, done = false;
    uint64_t before = 0, cov = 0;
    std::unique_ptr<imm_result> r;
    imm_status status = IMM_OK;
    std::string err;
    double t0 = 0, ms_select = 0;
    uint32_t select_graphs = 0, select_captures = 0;  // BatchRunner with IMM_GRAPH_SELECT
    uint32_t sample_graphs = 0, sample_captures = 0;  // ... with IMM_GRAPH_SAMPLE
    uint64_t bytes = 0;  // device bytes of the workspace when finished
    SelectDesc desc{};
    // AsyncRunner: the event that marks the end of the queued work, and
    // whether that work is a sampling round (0) or a selection (1)
    hipEvent_t ev = nullptr;
    int phase = 0;
    bool multi = false;  // BatchRunner: IC sampling passes join the multi-instance launch
    ~Query() {
        if (ev) (void)hipEventDestroy(ev);
    }
};

namespace {

imm_status acquire_workspace(Query& q, std::unique_ptr<Workspace>& slot, uint32_t big_cap) {
    {
        std::lock_guard<std::mutex> lk(q.g->ws_mu);
        auto& c = q.g->ws_cache;
        for (size_t j = 0; j < c.size(); ++j) {
            if (c[j]->arena.budget == q.p.max_device_bytes) {
                slot = std::move(c[j]);
                c.erase(c.begin() + (long)j);
                break;
            }
        }
    }
    if (!slot) {
        slot.reset(new Workspace());
        slot->big_cap = big_cap;
        IMM_TRY(ws_init(*slot, q.g->n, q.g->device, q.st, q.p.max_device_bytes));
    } else {
        // giant-set scratch narrower than this batch width wants (0: all the
        // GPU can use) is reallocated on use; wider scratch is kept
        Workspace& w = *slot;
        const uint32_t want = big_cap ? big_cap : 0xFFFFFFFFu;
        if (w.big && w.big_cap != big_cap && w.big_slots < want) {
            w.arena.release(w.big);
            w.arena.release(w.huge);
            w.big = nullptr;
            w.huge = nullptr;
            w.big_slots = 0;
            w.huge_slots = 0;
        }
        w.big_cap = big_cap;
    }
    return ws_reset(*slot, q.st, (q.p.flags & IMM_TIMING) != 0);
}

void release_workspace(Query& q) {
    std::lock_guard<std::mutex> lk(q.g->ws_mu);
    for (auto* slot : {&q.w, &q.w2}) {
        if (!*slot) continue;
        if (q.g->ws_cache.size() < kMaxCachedWorkspacesPerGraph)
            q.g->ws_cache.push_back(std::move(*slot));
        slot->reset();
    }
}

imm_status start_query(Query& q, uint32_t big_cap) {
    q.t0 = now_ms();
    if (q.p.k == 0 || q.p.k > q.g->n) return fail(IMM_EINVAL, "run: need 1 <= k <= n");
    if (!(q.p.epsilon > 0.0) || !(q.p.ell > 0.0)) return fail(IMM_EINVAL, "run: need eps > 0, ell > 0");
    const bool fresh = (q.p.flags & IMM_FRESH_FINAL) != 0;
    const bool early = (q.p.flags & IMM_EARLY_STOP) != 0;
    if (fresh && early) return fail(IMM_EINVAL, "run: IMM_FRESH_FINAL and IMM_EARLY_STOP exclude each other");
    q.sched = early ? kSchedEarly : (fresh ? kSchedFresh : kSchedImm);
    const bool dec = (q.p.flags & IMM_UPDATE_DECREMENT) != 0;
    const bool rec = (q.p.flags & IMM_UPDATE_RECOUNT) != 0;
    if (dec && rec)
        return fail(IMM_EINVAL, "run: IMM_UPDATE_DECREMENT and IMM_UPDATE_RECOUNT exclude each other");
    const uint32_t update = dec ? kUpdateDecrement : (rec ? kUpdateRecount : kUpdateAdaptive);
    IMM_TRY(theta_plan(q.g->n, q.p.k, q.p.epsilon, q.p.ell, &q.lam_p, &q.lam_s, &q.i_max));
    if (early) {
        IMM_TRY(early_plan(q.g->n, q.p.k, q.p.epsilon, q.p.ell, &q.theta0, &q.i_max, &q.a));
        q.g_k = 1.0 - std::pow(1.0 - 1.0 / (double)q.p.k, (double)q.p.k);
    }
    IMM_TRY(tune_graph(q.g, q.st));
    IMM_TRY(acquire_workspace(q, q.w, big_cap));
    if (early) IMM_TRY(acquire_workspace(q, q.w2, big_cap));
    q.w->update_mode = update;
    q.w->list_only = (q.p.flags & IMM_LIST_SETS) != 0;
    if (q.w2) q.w2->list_only = q.w->list_only;
    q.r.reset(new imm_result());
    q.r->k = q.p.k;
    q.eps_p = std::sqrt(2.0) * q.p.epsilon;
    q.lb = 1.0;
    q.i = 0;
    q.final = q.sched != kSchedEarly && q.i_max == 0;
    return IMM_OK;
}

// This iteration's target, and its sampling launched on the query's stream
// (for a query in the multi-instance launch, only prepared).
imm_status begin_iteration(Query& q) {
    double tf;
    if (q.sched == kSchedEarly) {
        // both pools grow to theta_0 2^(i-1) sets
        ++q.i;
        tf = std::ceil(std::ldexp(q.theta0, (int)q.i - 1));
        if (!(tf < 4294967296.0)) return fail(IMM_EOVERFLOW, "theta_i >= 2^32");
        const uint64_t target = (uint64_t)tf;
        if (q.r->targets.size() < 64) q.r->targets.push_back(target);
        Workspace& w = *q.w;
        Workspace& w2 = *q.w2;
        q.before = w.n_sets;
        IMM_TRY(ws_extend_launch(w, q.g, q.p.seed, w.n_sets,
                                 w.n_sets < target ? target - w.n_sets : 0));
        return ws_extend_launch(w2, q.g, q.p.seed, kSecondPoolIds + w2.n_sets,
                                w2.n_sets < target ? target - w2.n_sets : 0);
    }
    if (!q.final) {
        ++q.i;
        tf = std::ceil(q.lam_p / std::ldexp((double)q.g->n, -(int)q.i));
        if (!(tf < 4294967296.0)) return fail(IMM_EOVERFLOW, "theta_i >= 2^32");
        if (q.r->targets.size() < 63) q.r->targets.push_back((uint64_t)tf);
    } else {
        tf = std::ceil(q.lam_s / q.lb);
        if (!(tf < 4294967296.0)) return fail(IMM_EOVERFLOW, "theta >= 2^32");
        q.r->targets.push_back((uint64_t)tf);
    }
    const uint64_t target = (uint64_t)tf;
    Workspace& w = *q.w;
    if (q.final && q.sched == kSchedFresh) {
        // the final selection's theta sets are drawn afresh: sample ids after
        // the rounds' ids, into an emptied pool
        const uint64_t used = w.n_sets;
        IMM_TRY(ws_restart_pool(w));
        q.before = 0;
        return ws_extend_launch(w, q.g, q.p.seed, used, target, q.multi);
    }
    q.before = w.n_sets;
    const uint64_t count = w.n_sets < target ? target - w.n_sets : 0;
    // An LT round of a few walks per walk slot lasts as long as its longest
    // walk, whatever its size: such a round also draws ids ahead (up to about
    // four walks per slot in all), which then need no launch of their own.
    // It draws up to lam* 2^(i+1) / n: the next round's target (lam' < lam*)
    // and, should this round or the next one pass its test (LB >= n / 2^(i+1)),
    // the final theta = lam* / LB. Ids drawn ahead are counted and pooled only
    // when a later iteration asks for them; what the run never asks for is
    // dropped, so results do not change.
    uint64_t ahead = 0, next = 0;
    if (!q.final && q.sched == kSchedImm && q.g->model == IMM_LT && q.i < q.i_max && count) {
        const double nf = std::ceil(q.lam_s / std::ldexp((double)q.g->n, -(int)(q.i + 1)));
        const uint64_t slots = (uint64_t)lt_small_grid(q.g->device, q.g->lt_bloom_bits,
                                                       q.g->lt_lanes) * 64u / q.g->lt_lanes / 2u;
        const uint64_t cap = 4 * slots;
        if (nf < 4294967296.0 && (uint64_t)nf > target && count < cap)
            ahead = std::min<uint64_t>((uint64_t)nf - target, cap - count);
        // should this round fail its test, the next one asks for the ids up
        // to its own target: those are counted apart in the same pass
        const double tn = std::ceil(q.lam_p / std::ldexp((double)q.g->n, -(int)(q.i + 1)));
        if (ahead && tn < 4294967296.0 && (uint64_t)tn > target)
            next = std::min<uint64_t>((uint64_t)tn - target, ahead);
    }
    return ws_extend_launch(w, q.g, q.p.seed, w.n_sets, count, q.multi, ahead, next);
}

// After the round's sampling: retries and compaction of the pool (pools).
imm_status finish_sampling(Query& q) {
    IMM_TRY(ws_extend_finish(*q.w, q.g, q.p.seed));
    if (q.w2) IMM_TRY(ws_extend_finish(*q.w2, q.g, q.p.seed));
    return IMM_OK;
}

// After the theta decision of this iteration's coverage.
imm_status end_iteration(Query& q) {
    Workspace& w = *q.w;
    IMM_TRY(ws_select_finish(w, q.p.k, q.before, &q.cov));
    imm_result& r = *q.r;
    if (q.sched == kSchedEarly) {
        // the seeds' coverage in the second pool, then both bounds: an upper
        // bound on OPT from the first pool's coverage (at least g_k of the
        // best possible there), a lower bound on the seeds' spread from the
        // second's (Chernoff bounds, each failing with probability <= e^-a)
        uint64_t cov2 = 0;
        IMM_TRY(ws_coverage(*q.w2, w.seeds_d, q.p.k, &cov2));
        r.round_cov.push_back(q.cov);
        r.round_cov2.push_back(cov2);
        r.rounds = q.i;
        const double scale = (double)q.g->n / (double)w.n_sets;
        const double su = std::sqrt((double)q.cov / q.g_k + q.a / 2.0) + std::sqrt(q.a / 2.0);
        const double up = su * su * scale;
        const double sl = std::sqrt((double)cov2 + 2.0 * q.a / 9.0) - std::sqrt(q.a / 2.0);
        double lo = sl > 0.0 ? (sl * sl - q.a / 18.0) * scale : 0.0;
        if (lo < 0.0) lo = 0.0;
        r.sigma_up = up;
        r.alpha = lo / up;
        q.lb = lo;
        if (!(lo / up >= (1.0 - kInvE) - q.p.epsilon) && q.i < q.i_max) return IMM_OK;
    } else if (!q.final) {
        r.round_cov.push_back(q.cov);
        r.rounds = q.i;
        const double x = std::ldexp((double)q.g->n, -(int)q.i);
        const double frac = (double)q.cov / (double)w.n_sets;
        if ((double)q.g->n * frac >= (1.0 + q.eps_p) * x) {
            q.lb = (double)q.g->n * frac / (1.0 + q.eps_p);
            q.final = true;
        } else if (q.i == q.i_max) {
            q.final = true;
        }
        return IMM_OK;
    }
    r.seeds.resize(q.p.k);
    HIP_TRY(hipMemcpyAsync(r.seeds.data(), w.seeds_d, (uint64_t)q.p.k * 4, hipMemcpyDeviceToHost,
                           w.st));
    HIP_TRY(hipStreamSynchronize(w.st));
    r.gains.assign(w.gains_h, w.gains_h + q.p.k);
    r.theta = w.n_sets;
    r.lb = q.lb;
    r.covered = q.cov;
    const double t1 = now_ms();
    IMM_TRY(ws_read_scalars(w));
    fill_stats(w, &r.stats);
    r.stats.ms_select += q.ms_select;
    r.stats.ms_total = t1 - q.t0;
    r.stats.rounds = r.rounds;
    r.stats.team = q.g->model == IMM_IC ? q.g->ic_team : 0;
    r.stats.device_bytes = w.arena.used;
    r.stats.big_block = q.g->model == IMM_IC ? q.g->ic_big_block : 0;
    r.stats.bloom_bits = q.g->model == IMM_LT ? q.g->lt_bloom_bits : 0;
    r.stats.walk_lanes = q.g->model == IMM_LT ? q.g->lt_lanes : 0;
    r.stats.select_graphs = q.select_graphs;
    r.stats.select_captures = q.select_captures;
    r.stats.sample_graphs = q.sample_graphs;
    r.stats.sample_captures = q.sample_captures;
    if (q.p.flags & IMM_KEEP_POOL) {
        IMM_TRY(ws_export_pool(w, &r.set_off, &r.set_vtx, nullptr));
        r.has_pool = true;
    }
    q.done = true;
    q.bytes = w.arena.used + (q.w2 ? q.w2->arena.used : 0);
    // the largest workspace a query on this graph has needed (the server's
    // admission estimate)
    uint64_t prev = q.g->peak_bytes.load();
    while (q.bytes > prev && !q.g->peak_bytes.compare_exchange_weak(prev, q.bytes)) {
    }
    return IMM_OK;
}

}  // namespace

// ------------------------------------------------------------ BatchRunner --

BatchRunner::BatchRunner(hipStream_t main, bool multi) : main_(main), multi_(multi) {}

BatchRunner::~BatchRunner() {
    for (auto* q : active_) delete q;
    if (multi_buf_) (void)hipFree(multi_buf_);
    if (tasks_h_) (void)hipHostFree(tasks_h_);
    if (tasks_d_) (void)hipFree(tasks_d_);
    if (descs_h_) (void)hipHostFree(descs_h_);
    if (descs_d_) (void)hipFree(descs_d_);
    if (ev_a_) (void)hipEventDestroy(ev_a_);
    if (ev_b_) (void)hipEventDestroy(ev_b_);
}

Query* BatchRunner::start(imm_graph* g, const imm_params& p, hipStream_t st, uint32_t big_cap) {
    Query* q = new Query();
    q->g = g;
    q->p = p;
    q->st = st;
    // IC queries sample together in one multi-instance launch on the main
    // stream (an early-stopping query's second pool keeps the plain path)
    if (multi_ && g->model == IMM_IC && !(p.flags & IMM_EARLY_STOP)) {
        q->st = main_;
        q->multi = true;
    }
    const imm_status s = start_query(*q, big_cap);
    if (s != IMM_OK) {
        q->status = s;
        q->err = last_error();
        q->done = true;
        q->w.reset();
        return q;
    }
    active_.push_back(q);
    return q;
}

void BatchRunner::finish_err(Query* q, imm_status s) {
    q->status = s;
    q->err = last_error();
    q->done = true;
    q->w.reset();  // a failed workspace is not reused
    q->w2.reset();
}

void BatchRunner::cancel(Query* q) {
    if (q->done) return;
    q->status = IMM_ECANCELLED;
    q->err = "cancelled";
    q->done = true;
    release_workspace(*q);
}

bool BatchRunner::step() {
    {
        // queries cancelled since the last step leave first
        std::vector<Query*> keep;
        for (auto* q : active_) {
            if (q->done) finished_.push_back(q);
            else keep.push_back(q);
        }
        active_.swap(keep);
    }
    if (active_.empty()) return false;
    bool timing = false;
    for (auto* q : active_) timing |= (q->p.flags & IMM_TIMING) != 0;
    if (timing && !ev_a_) {
        (void)hipEventCreate(&ev_a_);
        (void)hipEventCreate(&ev_b_);
    }
    // sampling, each query on its stream; the IC queries' passes prepared
    // and then run by one multi-instance launch on the main stream
    std::vector<Query*> live;
    for (auto* q : active_) {
        const imm_status s = begin_iteration(*q);
        if (s != IMM_OK) finish_err(q, s);
        else live.push_back(q);
    }
    {
        std::vector<Query*> group;
        for (auto* q : live)
            if (q->multi && q->w->pending_multi) group.push_back(q);
        for (size_t a = 0; a < group.size(); a += kMaxTasks) {
            std::vector<Query*> part(group.begin() + (long)a,
                                     group.begin() + (long)std::min(group.size(), a + kMaxTasks));
            // the host task table is rewritten only after its last copy ran
            if (a > 0) (void)hipStreamSynchronize(main_);
            const imm_status s = multi_pass(part);
            if (s != IMM_OK)
                for (auto* q : part) finish_err(q, s);
        }
        std::vector<Query*> keep;
        for (auto* q : live)
            if (!q->done) keep.push_back(q);
        live.swap(keep);
    }
    // one wait per stream, then retries, compaction, index, selection state
    std::vector<hipStream_t> synced;
    for (auto* q : live) {
        if (std::find(synced.begin(), synced.end(), q->st) == synced.end()) {
            (void)hipStreamSynchronize(q->st);
            synced.push_back(q->st);
        }
    }
    std::vector<Query*> ready;
    // a lone LT query whose round drew the next round's ids ahead runs that
    // round speculatively beside this one's index update and selection (its
    // own stream, scratch and selection buffers): kept if this round fails
    // its test
    Query* spec_q = nullptr;
    for (auto* q : live) {
        imm_status s = finish_sampling(*q);
        if (s == IMM_OK && live.size() == 1 && active_.size() == 1 && q->st == main_ &&
            q->sched == kSchedImm && !q->final && q->i < q->i_max && q->g->model == IMM_LT &&
            ws_spec_possible(*q->w)) {
            const char* e = std::getenv("IMM_SPEC");
            // without the memory for it the round runs alone
            if (!(e && std::strcmp(e, "0") == 0) && ws_spec_reserve(*q->w, q->p.k) == IMM_OK) {
                spec_q = q;
                // its compaction and index segment, once the pool's compaction is queued
                s = hipEventRecord(q->w->side_ev, q->st) == hipSuccess
                        ? ws_spec_launch_index(*q->w, q->w->side_ev)
                        : fail(IMM_EDEVICE, "speculative round: event record failed");
                // its selection reads every segment: it waits for this round's
                if (s == IMM_OK) s = ws_index_update(*q->w);
                if (s == IMM_OK && hipEventRecord(q->w->side_ev2, q->st) != hipSuccess)
                    s = fail(IMM_EDEVICE, "speculative round: event record failed");
            }
        }
        if (s == IMM_OK) s = ws_select_prepare(*q->w, q->p.k, &q->desc);
        if (s != IMM_OK) {
            finish_err(q, s);
            if (q == spec_q) {
                (void)ws_spec_drop(*q->w);  // waits for what it queued
                spec_q = nullptr;
            }
        } else {
            ready.push_back(q);
        }
    }
    // the selections of all queries together, on the main stream
    if (!ready.empty()) {
        std::vector<SelectDesc> descs;
        uint32_t arg_total = 0, sel_total = 0, dense_total = 0, kmax = 0;
        for (auto* q : ready) {
            SelectDesc d = q->desc;
            d.arg_lo = arg_total;
            d.arg_cnt = argmax_blocks(d.n);
            d.sel_lo = sel_total;
            d.sel_cnt = select_blocks(q->g->device, q->w->n_sets, (uint32_t)ready.size());
            d.dense_lo = dense_total;
            d.dense_cnt = dense_blocks(d.n_dense, d.dense_words);
            arg_total += d.arg_cnt;
            sel_total += d.sel_cnt;
            dense_total += d.dense_cnt;
            kmax = std::max(kmax, d.k);
            descs.push_back(d);
        }
        bool ok = true;
        // a lone query uses its workspace's descriptor (allocated with the
        // cached workspace); a batch, the runner's buffers
        SelectDesc* dd = nullptr;
        if (ready.size() == 1) {
            Workspace& w1 = *ready[0]->w;
            w1.desc_h = descs[0];
            dd = w1.desc_d;
        } else if (cap_descs_ < descs.size()) {
            if (descs_h_) (void)hipHostFree(descs_h_);
            if (descs_d_) (void)hipFree(descs_d_);
            descs_h_ = nullptr;
            descs_d_ = nullptr;
            cap_descs_ = descs.size() * 2;
            ok = hipHostMalloc((void**)&descs_h_, cap_descs_ * sizeof(SelectDesc),
                               hipHostMallocDefault) == hipSuccess &&
                 hipMalloc((void**)&descs_d_, cap_descs_ * sizeof(SelectDesc)) == hipSuccess;
            if (!ok) cap_descs_ = 0;
        }
        if (ok && !dd) dd = descs_d_;
        std::vector<hipEvent_t> joins;
        if (ok) {
            const void* src = descs.size() == 1 ? (const void*)&ready[0]->w->desc_h
                                                : (const void*)descs_h_;
            if (descs.size() > 1)
                std::memcpy(descs_h_, descs.data(), descs.size() * sizeof(SelectDesc));
            for (auto* q : ready) {
                if (q->st == main_) continue;
                hipEvent_t e = nullptr;
                (void)hipEventCreateWithFlags(&e, hipEventDisableTiming);
                (void)hipEventRecord(e, q->st);
                (void)hipStreamWaitEvent(main_, e, 0);
                joins.push_back(e);
            }
            ok = hipMemcpyAsync(dd, src, descs.size() * sizeof(SelectDesc),
                                hipMemcpyHostToDevice, main_) == hipSuccess;
            bool graph = false;
            for (auto* q : ready) graph |= (q->p.flags & IMM_GRAPH_SELECT) != 0;
            if (timing) (void)hipEventRecord(ev_a_, main_);
            int launched = 0;
            if (graph && ok) {
                bool captured = false;
                launched = graph_.launch(dd, (uint32_t)descs.size(), kmax, arg_total,
                                         sel_total, dense_total, main_, &captured);
                ok = launched >= 0;
                for (auto* q : ready) {
                    q->select_graphs += launched > 0 ? 1u : 0u;
                    q->select_captures += launched > 0 && captured ? 1u : 0u;
                }
            }
            if (launched == 0) {
                for (uint32_t t = 0; ok && t < kmax; ++t)
                    ok = launch_select_step(dd, (uint32_t)descs.size(), t, arg_total,
                                            sel_total, dense_total, main_) == hipSuccess;
            }
            if (timing) (void)hipEventRecord(ev_b_, main_);
            if (spec_q && ok)
                ok = ws_spec_launch_select(*spec_q->w, spec_q->p.k, spec_q->w->side_ev2) == IMM_OK;
            for (auto* q : ready)
                if (ok) ok = ws_select_copy_out(*q->w, q->p.k, main_) == IMM_OK;
            if (ok) ok = hipStreamSynchronize(main_) == hipSuccess;
            for (auto e : joins) (void)hipEventDestroy(e);
            if (ok && timing) {
                float msf = 0.f;
                (void)hipEventElapsedTime(&msf, ev_a_, ev_b_);
                for (auto* q : ready) q->ms_select += msf;
            }
        }
        for (auto* q : ready) {
            const imm_status s = ok ? end_iteration(*q)
                                    : fail(IMM_EDEVICE, "batched selection failed");
            if (s != IMM_OK) finish_err(q, s);
        }
        if (spec_q) {
            Query* q = spec_q;
            Workspace& w = *q->w;
            if (w.spec && !q->done && !q->final) {
                // this round failed its test: the next round is the one run
                // speculatively; its θ decision is taken now
                imm_status s = ws_spec_commit(w);
                if (s == IMM_OK) s = begin_iteration(*q);
                if (s == IMM_OK) {
                    q->before = w.spec_lo;
                    s = end_iteration(*q);
                }
                if (s != IMM_OK) finish_err(q, s);
            } else {
                (void)ws_spec_drop(w);
            }
        }
    }
    std::vector<Query*> next;
    for (auto* q : active_) {
        if (q->done) finished_.push_back(q);
        else next.push_back(q);
    }
    active_.swap(next);
    return true;
}

// One multi-instance launch of the prepared IC passes of qs (<= kMaxTasks),
// on the main stream: the task table and the lane pass's position prefix
// (each range rounded up to whole tickets), shared giant-set slots sized for
// the largest graph, the three kernels, then every workspace's scalar copy.
imm_status BatchRunner::multi_pass(const std::vector<Query*>& qs) {
    const uint32_t nt = (uint32_t)qs.size();
    uint32_t words = 1, team = 2;
    uint64_t biggest = 0;
    for (auto* q : qs) {
        words = std::max(words, (q->g->n + 31) / 32);
        if (q->w->pending_count > biggest) {
            biggest = q->w->pending_count;
            team = q->g->ic_team;
        }
    }
    const int dev = qs[0]->g->device;
    const uint32_t slots = ic_large_slots(dev, 256);
    const uint64_t need = (uint64_t)slots * ((uint64_t)words + kGiantQueue) * 4 + 256;
    if (multi_cap_ < need || multi_words_ < words) {
        if (multi_buf_) {
            HIP_TRY(hipStreamSynchronize(main_));
            (void)hipFree(multi_buf_);
            multi_buf_ = nullptr;
        }
        multi_cap_ = 0;
        HIP_TRY(hipMalloc(&multi_buf_, need));
        // the bitmaps start clear; the kernels leave them clear
        HIP_TRY(hipMemsetAsync(multi_buf_, 0, (uint64_t)slots * words * 4, main_));
        multi_cap_ = need;
        multi_words_ = words;
    }
    if (!tasks_h_) {
        HIP_TRY(hipHostMalloc((void**)&tasks_h_, kTaskBytes, hipHostMallocDefault));
        HIP_TRY(hipMalloc((void**)&tasks_d_, kTaskBytes));
    }
    IcTask* th = reinterpret_cast<IcTask*>(tasks_h_);
    uint32_t* pre = reinterpret_cast<uint32_t*>(tasks_h_ + kMaxTasks * sizeof(IcTask));
    uint32_t* tk = pre + kMaxTasks + 1;
    uint64_t acc = 0;
    for (uint32_t j = 0; j < nt; ++j) {
        Query* q = qs[j];
        th[j] = ws_ic_task(*q->w, q->g, q->p.seed, kGiantQueue);
        pre[j] = (uint32_t)acc;
        acc += (q->w->pending_count + kLaneTicket - 1) / kLaneTicket * kLaneTicket;
        if (acc > 0xFFFF0000ull) return fail(IMM_EOVERFLOW, "batched sampling round too large");
        q->w->pending_multi = false;
    }
    pre[nt] = (uint32_t)acc;
    tk[0] = tk[1] = tk[2] = 0;
    HIP_TRY(hipMemcpyAsync(tasks_d_, tasks_h_, kTaskBytes, hipMemcpyHostToDevice, main_));
    const IcTask* td = reinterpret_cast<const IcTask*>(tasks_d_);
    const uint32_t* pd = reinterpret_cast<const uint32_t*>(tasks_d_ + kMaxTasks * sizeof(IcTask));
    uint32_t* tkd = const_cast<uint32_t*>(pd) + kMaxTasks + 1;
    uint32_t* bits = static_cast<uint32_t*>(multi_buf_);
    const BigScratch b{bits, bits + (uint64_t)slots * words, words, slots, kGiantQueue};
    bool graph = false;
    for (auto* q : qs) graph |= (q->p.flags & IMM_GRAPH_SAMPLE) != 0;
    int launched = 0;
    if (graph) {
        bool captured = false;
        launched = sgraph_.launch(td, nt, pd, tkd, team, 256, b, dev, main_, &captured);
        if (launched < 0) return fail(IMM_EDEVICE, "batched sampling: graph launch failed");
        for (auto* q : qs) {
            q->sample_graphs += launched > 0 ? 1u : 0u;
            q->sample_captures += launched > 0 && captured ? 1u : 0u;
        }
    }
    if (launched == 0) HIP_TRY(launch_ic_multi(td, nt, pd, tkd, team, 256, b, dev, main_));
    for (auto* q : qs) IMM_TRY(ws_after_multi(*q->w));
    // the host table is rewritten by the next launch only after main_ has
    // been synchronised (step waits for it before the selections)
    return IMM_OK;
}

std::vector<Query*> BatchRunner::drain() {
    std::vector<Query*> out;
    out.swap(finished_);
    return out;
}

uint64_t BatchRunner::bytes(const Query* q) { return q->bytes; }
bool BatchRunner::done(const Query* q) { return q->done; }

imm_result* BatchRunner::take(Query* q, imm_status* status, std::string* err) {
    *status = q->status;
    if (err) *err = q->err;
    imm_result* r = nullptr;
    if (q->status == IMM_OK && q->r) {
        r = q->r.release();
        release_workspace(*q);
    }
    q->w.reset();
    q->w2.reset();
    delete q;
    return r;
}

// ------------------------------------------------------------ AsyncRunner --

AsyncRunner::~AsyncRunner() {
    for (auto* q : active_) delete q;
}

void AsyncRunner::finish_err(Query* q, imm_status s) {
    q->status = s;
    q->err = last_error();
    q->done = true;
    if (q->w) (void)hipStreamSynchronize(q->w->st);
    q->w.reset();
    q->w2.reset();
}

Query* AsyncRunner::start(imm_graph* g, const imm_params& p, hipStream_t st, uint32_t big_cap) {
    Query* q = new Query();
    q->g = g;
    q->p = p;
    q->st = st;
    imm_status s = start_query(*q, big_cap);
    if (s == IMM_OK && hipEventCreateWithFlags(&q->ev, hipEventDisableTiming) != hipSuccess)
        s = fail(IMM_EDEVICE, "run: event creation failed");
    if (s == IMM_OK) s = begin_iteration(*q);
    if (s == IMM_OK && hipEventRecord(q->ev, q->st) != hipSuccess)
        s = fail(IMM_EDEVICE, "run: event record failed");
    if (s != IMM_OK) {
        finish_err(q, s);
        return q;
    }
    q->phase = 0;
    active_.push_back(q);
    return q;
}

void AsyncRunner::cancel(Query* q) {
    if (q->done) return;
    if (q->w) (void)hipStreamSynchronize(q->w->st);
    q->status = IMM_ECANCELLED;
    q->err = "cancelled";
    q->done = true;
    release_workspace(*q);
}

bool AsyncRunner::poll() {
    bool advanced = false;
    for (auto* q : active_) {
        if (q->done) continue;
        const hipError_t e = hipEventQuery(q->ev);
        if (e == hipErrorNotReady) continue;
        advanced = true;
        imm_status s = e == hipSuccess ? IMM_OK : fail(IMM_EDEVICE, "run: device work failed");
        if (s == IMM_OK && q->phase == 0) {
            // sampling round done: finish it, launch the selection
            s = finish_sampling(*q);
            int gs = 0;
            if (s == IMM_OK)
                s = ws_select_launch(*q->w, q->p.k, (q->p.flags & IMM_GRAPH_SELECT) != 0, &gs);
            q->select_graphs += gs > 0 ? 1u : 0u;
            q->select_captures += gs == 2 ? 1u : 0u;
            q->phase = 1;
        } else if (s == IMM_OK) {
            // selection done: theta decision, then the next round (if any)
            s = end_iteration(*q);
            if (s == IMM_OK && !q->done) {
                s = begin_iteration(*q);
                q->phase = 0;
            }
        }
        if (s == IMM_OK && !q->done && hipEventRecord(q->ev, q->st) != hipSuccess)
            s = fail(IMM_EDEVICE, "run: event record failed");
        if (s != IMM_OK) finish_err(q, s);
    }
    std::vector<Query*> keep;
    for (auto* q : active_) {
        if (q->done) finished_.push_back(q);
        else keep.push_back(q);
    }
    active_.swap(keep);
    return advanced;
}

std::vector<Query*> AsyncRunner::drain() {
    std::vector<Query*> out;
    out.swap(finished_);
    return out;
}

uint64_t cached_bytes(imm_graph* g) {
    std::lock_guard<std::mutex> lk(g->ws_mu);
    uint64_t b = 0;
    for (auto& w : g->ws_cache) b += w->arena.used;
    return b;
}

uint64_t trim_cache(imm_graph* g) {
    std::vector<std::unique_ptr<Workspace>> drop;
    {
        std::lock_guard<std::mutex> lk(g->ws_mu);
        drop.swap(g->ws_cache);
    }
    uint64_t b = 0;
    for (auto& w : drop) b += w->arena.used;
    drop.clear();  // frees the device memory (each workspace waits for its device first)
    return b;
}

void run_queries(imm_graph* const* graphs, const imm_params* params, uint32_t count,
                 hipStream_t main, const hipStream_t* streams, imm_result** out,
                 imm_status* status, std::string* errors) {
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, graphs[0]->device);
    const uint32_t big_cap = count > 1 ? std::max<uint32_t>(64u, (uint32_t)cus * 8u / count) : 0u;
    // lock-step: one set of selection launches per seed step serves every
    // query (measured faster than independent pipelines for many small
    // queries; the server, whose queries arrive over time, uses those)
    std::vector<Query*> qs(count);
    BatchRunner br(main, count > 1);
    for (uint32_t j = 0; j < count; ++j) qs[j] = br.start(graphs[j], params[j], streams[j], big_cap);
    while (br.step()) {
    }
    (void)br.drain();
    for (uint32_t j = 0; j < count; ++j)
        out[j] = BatchRunner::take(qs[j], &status[j], errors ? &errors[j] : nullptr);
}

}  // namespace imm
