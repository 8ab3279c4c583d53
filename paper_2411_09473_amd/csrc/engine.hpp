// engine.hpp -- host-side structures of libimm shared by workspace.cpp,
// runner.cpp and api.cpp: error reporting, device allocation with a byte
// budget, the per-query device workspace, and the resident graph.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <chrono>
#include <cstdint>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/imm.h"
#include "imm_internal.hpp"

namespace imm {

// ---------------------------------------------------------------- errors --

imm_status fail(imm_status st, const std::string& msg);
imm_status fail(imm_status st, const char* msg);  // copies msg; allocates nothing
const char* last_error();  // this thread's last message
double now_ms();

#define IMM_TRY(expr)                \
    do {                             \
        imm_status _s = (expr);      \
        if (_s != IMM_OK) return _s; \
    } while (0)

#define HIP_TRY(expr)                                                                \
    do {                                                                             \
        hipError_t _e = (expr);                                                      \
        if (_e != hipSuccess) {                                                      \
            return ::imm::fail(_e == hipErrorOutOfMemory ? IMM_ENOMEM : IMM_EDEVICE, \
                               std::string(#expr) + ": " + hipGetErrorString(_e));  \
        }                                                                            \
    } while (0)

// ------------------------------------------------------------ allocation --

// Device allocations of one owner, with an optional byte budget (0: none).
struct Arena {
    uint64_t budget = 0;
    uint64_t used = 0;
    std::vector<std::pair<void*, uint64_t>> live;

    imm_status alloc(void** p, uint64_t bytes, const char* what);
    void release(void* p);
    void release_all();
    ~Arena() { release_all(); }
};

// Make *p hold at least `need` elements (growing by half or more), keeping
// its first `keep` elements; waits for `st` before freeing the old buffer.
template <class T>
imm_status grow(Arena& a, T** p, uint64_t* cap, uint64_t need, uint64_t keep, hipStream_t st,
                const char* what) {
    if (*p && *cap >= need) return IMM_OK;
    uint64_t nc = *cap + *cap / 2 > need ? *cap + *cap / 2 : need;
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

// Upper bound on the device memory of one workspace's large-set scratch,
// the queue entries of an IC giant-set slot, and the IC slots whose queues
// hold n entries (for the sets that outgrow the bounded ones).
constexpr uint64_t kBigScratchBytes = 16ull << 30;
constexpr uint32_t kGiantQueue = 1u << 16;
constexpr uint32_t kHugeSlots = 16;
constexpr uint32_t kGiantQueueMax = 1u << 20;
constexpr double kOverRate = 1.0 / 1024;  // outgrown queues per sample that enlarge them
// Largest pair buffer of the partitioned index build.
constexpr uint64_t kIndexPairsBytes = 8ull << 30;
// Smallest segment (in entries, by its bound) indexed by the partition.
constexpr uint64_t kIndexPartitionMin = 1ull << 20;

// Scalars the kernels update, in one device block.
struct DevScalars {
    unsigned long long cursor;
    // reset per pass: the seven words from ticket_small to defer_n
    uint32_t ticket_small, ticket_big, ticket_bfs, ticket_huge, pend_n, over_n, defer_n;
    uint32_t retry_n, spare_n, big_flag, err;
    unsigned long long stats[kStCount];
    // kept across passes (cleared with the workspace): the dense-set cursor
    // and the dense sets' total size
    uint32_t dense_n, dense_pad;
    unsigned long long dense_entries;
};

// Phase timing with HIP events (phases: 0 sample, 1 compact, 2 index,
// 3 select, 4 main sampling kernel, 5 large-set sampling kernel, 6 IC
// lane-per-root kernel, 7 IC pass over sets that outgrew the large-set
// queues).
struct Timer {
    bool on = false;
    struct Rec {
        int phase;
        hipEvent_t a, b;
    };
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;
    hipEvent_t get();
    int open(int phase, hipStream_t st);
    void close(int h, hipStream_t st);
    void collect(double* ms, uint64_t* launches);
    ~Timer();
};

// ------------------------------------------------------------- workspace --
//
// Device state of one IMM query (or of one imm_sample / imm_greedy call).
// The pool grows by whole sampling rounds; its vertex->sets index is kept in
// segments, one per round, each indexing only that round's sets (segment r
// occupies inv_set positions [P_{r-1}, P_r), the range its sets occupy in
// set_vtx), so no set is indexed twice.
// The kmax seed steps of nq runs (launch_select_step for t < kmax) as one
// captured hipGraph: launch() relaunches the executable graph while the
// shape (descriptor buffer, runs, steps, workgroup counts) repeats, else
// updates it in place or instantiates it anew; *captured tells whether it
// had to capture. Returns 1 when launched; 0 when no graph could be made
// (e.g. the legacy default stream cannot be captured): nothing was
// launched, the caller launches the steps itself; -1 when the launch failed.
struct SelectGraph {
    hipGraphExec_t exec = nullptr;
    const SelectDesc* descs = nullptr;
    uint32_t nq = 0, kmax = 0, arg_total = 0, sel_total = 0, dense_total = 0;
    int launch(const SelectDesc* descs, uint32_t nq, uint32_t kmax, uint32_t arg_total,
               uint32_t sel_total, uint32_t dense_total, hipStream_t st, bool* captured);
    SelectGraph() = default;
    SelectGraph(const SelectGraph&) = delete;
    SelectGraph& operator=(const SelectGraph&) = delete;
    ~SelectGraph();
};

// The multi-instance IC sampling launch of a batched round (three kernels
// over a task table in device memory) as an executable graph: relaunched
// while the launch's arguments repeat (they are device pointers and shape
// only; the table's contents change every round and are copied before each
// launch), else updated in place or instantiated anew.
struct SampleGraph {
    hipGraphExec_t exec = nullptr;
    const IcTask* tasks = nullptr;
    const uint32_t* prefix = nullptr;
    uint32_t* tickets = nullptr;
    uint32_t ntask = 0, team = 0, block = 0;
    BigScratch b{};
    int device = -1;
    // 1: the graph ran; 0: nothing launched (the caller launches directly);
    // -1: the graph launch failed
    int launch(const IcTask* tasks, uint32_t ntask, const uint32_t* prefix, uint32_t* tickets,
               uint32_t team, uint32_t block, const BigScratch& b, int device, hipStream_t st,
               bool* captured);
    SampleGraph() = default;
    SampleGraph(const SampleGraph&) = delete;
    SampleGraph& operator=(const SampleGraph&) = delete;
    ~SampleGraph();
};

// The buffers of one greedy selection. A workspace holds the active ones in
// its own fields; a second set lets the next round's selection run
// speculatively beside the current one (swap_sel exchanges them).
struct SelBufs {
    uint32_t* counts_work = nullptr;
    uint32_t* heavy = nullptr;
    uint32_t* covered = nullptr;
    uint64_t cap_cov = 0;
    unsigned long long* slots = nullptr;
    uint32_t* chunk_n = nullptr;
    unsigned long long* cov_entries = nullptr;
    Chunk* chunks = nullptr;
    uint64_t cap_chunks = 0;
    uint32_t* seeds_d = nullptr;
    uint32_t* gains_d = nullptr;
    uint64_t cap_k = 0;
    uint32_t* gains_h = nullptr;  // pinned
    SelectDesc* desc_d = nullptr;
    SelectDesc desc_h{};
    uint32_t* cand = nullptr;
    uint32_t* cand_bits = nullptr;
    uint32_t* cand_state = nullptr;
    uint32_t* cand_h = nullptr;  // pinned
    SelectDesc desc_last{};
};

struct Workspace {
    int device = 0;
    uint32_t n = 0;
    hipStream_t st = nullptr;  // the stream of the query using it
    uint32_t big_cap = 0;      // large-set scratch slots wanted (0: fill the GPU)
    Arena arena;
    DevScalars* sc = nullptr;
    DevScalars* hsc = nullptr;  // pinned mirror
    uint64_t* hp = nullptr;     // pinned: pool size
    uint32_t* herr = nullptr;   // pinned: error flag
    uint32_t* counts_acc = nullptr;   // occurrences over all sets so far
    uint32_t* counts_prev = nullptr;  // ... over the sets already indexed
    uint32_t* counts_work = nullptr;  // the greedy's working copy
    uint32_t* heavy = nullptr;  // vertices with long index lists; their count at [n]
    uint32_t* inv_cursor = nullptr;
    uint64_t* inv_offs = nullptr;
    uint64_t cap_offs = 0;
    uint32_t nseg = 0;
    uint64_t indexed_sets = 0;
    uint64_t* set_off = nullptr;
    uint64_t cap_sets = 0;
    uint32_t* set_vtx = nullptr;
    uint64_t cap_entries = 0;
    uint32_t* inv_set = nullptr;
    uint64_t cap_inv = 0;
    uint32_t* covered = nullptr;
    uint64_t cap_cov = 0;
    uint32_t* stage = nullptr;
    uint64_t stage_cap = 0;
    uint64_t* stage_off = nullptr;
    uint64_t cap_so = 0;
    uint32_t* sizes = nullptr;
    uint64_t cap_sz = 0;
    uint32_t* defer = nullptr;
    uint64_t cap_df = 0;
    uint32_t* retry = nullptr;
    uint64_t cap_rt = 0;
    uint32_t* spare = nullptr;
    uint64_t cap_sp = 0;
    uint32_t* pend = nullptr;  // IC: samples left for the BFS pass
    uint64_t cap_pd = 0;
    uint64_t* scan_tmp = nullptr;
    uint64_t cap_scan = 0;
    IndexPlan* iplan = nullptr;            // partitioned index build: bucket plan
    unsigned long long* inv_pairs = nullptr;  // ... and its (set, vertex) pairs
    uint64_t cap_pairs = 0;
    uint64_t p_indexed = 0;  // entries of the indexed sets (a lower bound)
    // sets [pend_lo, pend_hi) of the pool whose members counts_acc does not
    // hold yet (taken from the ids drawn ahead): the next index update counts
    // them, building its segment from the sets alone when it can
    uint64_t pend_lo = 0, pend_hi = 0;
    bool lt = false;  // the pool holds LT sets (set by each sampling call)
    // one allocation: k * kArgSlots partial maxima, then 2k queue lengths,
    // then k covered-member totals
    unsigned long long* slots = nullptr;
    uint32_t* chunk_n = nullptr;
    unsigned long long* cov_entries = nullptr;
    Chunk* chunks = nullptr;
    uint64_t cap_chunks = 0;
    uint32_t* seeds_d = nullptr;
    uint32_t* gains_d = nullptr;
    uint64_t cap_k = 0;
    uint32_t* gains_h = nullptr;  // pinned
    SelectDesc* desc_d = nullptr; // one descriptor, for selection run alone
    SelectDesc desc_h{};          // its host copy (kept while the copy is queued)
    SelectGraph sel_graph;        // its seed steps as a captured graph (IMM_GRAPH_SELECT)
    // candidate steps of the greedy (SelectDesc::cand): the list, its
    // bitmap, the state block and a pinned copy of the state's first words;
    // the last selection's descriptor (to finish a halted selection); list
    // bound (IMM_CAND_MAX, default kCandMax; 0: none); steps taken over the
    // list and halts since the last reset
    uint32_t* cand = nullptr;
    uint32_t* cand_bits = nullptr;
    uint32_t* cand_state = nullptr;
    uint32_t* cand_h = nullptr;
    SelectDesc desc_last{};
    uint64_t cand_steps = 0, cand_halts = 0;
    // A speculative round (LT, ids drawn ahead and counted apart): while the
    // current round's index update, selection state and selection run, the
    // next round's sets [spec_lo, spec_hi) are compacted after the pool,
    // indexed as segment spec_seg and selected over, on the side stream, with
    // scratch of their own (scan_tmp2, inv_cursor2, inv_pairs2, iplan2), the
    // second selection buffers (sel2) and counts_spec (the pool's counts with
    // those sets). Kept if the current round fails its test, dropped
    // otherwise; the workspace's host state changes only when it is kept.
    // side_ev orders the side stream after the pool's compaction, side_ev2
    // after the current round's index update.
    SelBufs sel2;
    uint32_t* counts_spec = nullptr;
    uint64_t* scan_tmp2 = nullptr;
    uint64_t cap_scan2 = 0;
    uint32_t* inv_cursor2 = nullptr;
    unsigned long long* inv_pairs2 = nullptr;
    uint64_t cap_pairs2 = 0;
    IndexPlan* iplan2 = nullptr;
    uint32_t spec_seg = 0;
    hipStream_t side = nullptr;
    hipEvent_t side_ev = nullptr, side_ev2 = nullptr;
    bool spec = false;
    uint64_t spec_lo = 0, spec_hi = 0;
    uint64_t spec_rounds = 0;  // speculative rounds kept since the last reset
    uint32_t* big = nullptr;   // giant-set slots: bitmap + bounded queue each
    uint32_t big_slots = 0;
    uint32_t big_qcap = 0;
    uint32_t* huge = nullptr;  // IC: a few slots with queues of n
    uint32_t huge_slots = 0;
    uint32_t* over = nullptr;  // IC: giant sets that outgrew a bounded queue
    uint64_t cap_ov = 0;
    // dense sets (IC sets of at least dense_threshold(n) members) as
    // bitmaps: cap_dense slots of dense_words words, their set ids and sizes,
    // n_dense in use (as of the last synchronisation); dense_counts[n] their
    // members' occurrences; dense_list / dense_mark the seed steps' claims.
    // list_only stores every set as a list.
    uint32_t* dense_bits = nullptr;
    uint32_t* dense_sid = nullptr;
    uint32_t* dense_size = nullptr;
    uint32_t* dense_list = nullptr;
    uint64_t cap_dense = 0;
    uint32_t dense_words = 0;
    uint64_t n_dense = 0;
    uint64_t dense_entries = 0;
    uint32_t* dense_counts = nullptr;
    uint32_t* dense_mark = nullptr;  // k + 1 entries, then the list cursor
    uint64_t cap_mark_k = 0;
    bool list_only = false;
    // coverage of a seed set in this pool (early stopping): a vertex bitmap
    // and a set bitmap (cap_mark words in all), and the count
    uint32_t* mark = nullptr;
    uint64_t cap_mark = 0;
    unsigned long long* cov_count = nullptr;
    uint64_t n_sets = 0;
    uint64_t p_exact = 0;    // pool size, exact as of the last synchronisation
    uint64_t p_ub = 0;       // upper bound on the pool size
    double mean_size = 0.0;  // mean set size of the last round (staging estimate)
    uint32_t update_mode = 0;    // SelectDesc::update of this workspace's selections
    bool pending_multi = false;  // the prepared pass waits for a multi-instance launch
    uint64_t pending_split = 0;  // ... of which the first pending_split join the pool now
    // sets the last pass drew ahead of the round (sample indices [ahead_split,
    // ahead_split + ahead_n) of that pass): staged, not counted, not pooled
    uint64_t ahead_n = 0, ahead_split = 0;
    uint64_t ahead_bound = 0;  // bound on their entries: that pass's staging bound
    // the first ahead_next of them are counted in counts_next (LT); a take of
    // exactly those adds counts_next to counts_acc
    uint32_t* counts_next = nullptr;
    uint64_t ahead_next = 0;
    uint64_t pending_next = 0;  // ... as asked of the pass in flight
    uint64_t pending_count = 0;  // sets of the sampling pass in flight
    uint64_t pending_lo = 0;
    Timer timer;

    ~Workspace();
};

}  // namespace imm

// ---------------------------------------------------------------- graph --

struct imm_graph {
    uint32_t n = 0;
    uint64_t m = 0;
    imm_model model = IMM_IC;
    int device = 0;
    // IC launch shapes picked by tune_graph on first use: waves per sample of
    // the BFS pass (IMM_IC_TEAM = 1, 2 or 4 forces it) and the giant-set
    // workgroup size (IMM_IC_BIG = 256 or 1024 forces it); for LT, the path
    // filter size (IMM_LT_BLOOM = 10, 11 or 12 forces it) and the lanes per
    // walk (IMM_LT_LANES = 1, 2 or 4 forces it)
    uint32_t ic_team = 1;
    uint32_t ic_big_block = 256;  // threads per giant set (256 or 1024)
    uint32_t lt_bloom_bits = 12;  // LT: log2 bits of the per-walk path filter
    uint32_t lt_lanes = 2;        // LT: lanes per walk
    bool team_forced = false, big_forced = false, bloom_forced = false, lanes_forced = false;
    double defer_rate = 0.0;  // giant sets per sample seen while tuning
    double dense_rate = 0.0;  // IC: dense (bitmap) sets per sample seen while tuning
    double over_rate = 0.0;   // IC: sets per sample that outgrew a bounded queue, ditto
    // mean set size seen while tuning: a fresh workspace's first staging
    // estimate, in place of a pilot batch (0 when tuning did not run)
    double mean_set_hint = 0.0;
    bool tuned = false;
    std::mutex tune_mu;
    imm::Arena arena;
    uint32_t* off = nullptr;
    uint32_t* thr = nullptr;
    uint32_t* src = nullptr;
    uint4* cs = nullptr;
    uint32_t* guide = nullptr;
    uint4* gw = nullptr;  // per guide bucket, the kLtWindow records from its guide entry
    // workspaces of finished queries, reused by later ones
    std::mutex ws_mu;
    // largest workspace a finished query on this graph held (server admission)
    std::atomic<uint64_t> peak_bytes{0};
    std::vector<std::unique_ptr<imm::Workspace>> ws_cache;
};

struct imm_result {
    uint32_t k = 0;
    std::vector<uint32_t> seeds;
    std::vector<uint64_t> gains;
    uint64_t theta = 0;
    uint32_t rounds = 0;
    double lb = 0.0;
    uint64_t covered = 0;
    std::vector<uint64_t> targets, round_cov;
    // early stopping: the last iteration's upper bound on OPT and ratio, and
    // each iteration's coverage of its seeds in the second pool
    double sigma_up = 0.0, alpha = 0.0;
    std::vector<uint64_t> round_cov2;
    bool has_pool = false;
    std::vector<uint64_t> set_off;
    std::vector<uint32_t> set_vtx;
    imm_stats stats{};
};

namespace imm {

IcGraphDev ic_view(const imm_graph* g);
LtGraphDev lt_view(const imm_graph* g);

// ---- workspace.cpp
imm_status ws_init(Workspace& w, uint32_t n, int device, hipStream_t st, uint64_t budget);
imm_status ws_reset(Workspace& w, hipStream_t st, bool timing);
imm_status ws_read_scalars(Workspace& w);
// Sampling of [id_lo, id_lo + count): the pass is launched without waiting
// (ws_extend_launch), then, after the stream is synchronised and the
// scalars read, completed (retries, compaction: ws_extend_finish).
// multi: everything but the pass itself, which a multi-instance launch then
// runs (ws_ic_task gives its task, ws_after_multi queues the scalar copy).
// ahead: that many more ids (after the count asked for) are drawn in the same
// pass but join the pool only when a later call asks for them (the rest of
// them are then dropped); results do not change. next (<= ahead): the first
// ids drawn ahead that the next call is expected to ask for; the pass counts
// their members apart, so that a call asking for exactly these ids adds one
// count vector instead of counting their members again.
imm_status ws_extend_launch(Workspace& w, const imm_graph* g, uint64_t seed, uint64_t id_lo,
                            uint64_t count, bool multi = false, uint64_t ahead = 0,
                            uint64_t next = 0);
IcTask ws_ic_task(Workspace& w, const imm_graph* g, uint64_t seed, uint32_t qcap);
imm_status ws_after_multi(Workspace& w);
imm_status ws_extend_finish(Workspace& w, const imm_graph* g, uint64_t seed);
// Speculative rounds. ws_spec_possible: the last pass drew the next round's
// ids ahead and counted them apart. ws_spec_reserve (after the pool's
// compaction, before ws_select_prepare, on the workspace's stream): every
// buffer that this round's index update or the speculative round writes is
// grown now, as a grow waits for the workspace's stream alone before it
// frees the old buffer. ws_spec_launch_index (then): the next round's
// compaction, counts and index segment on the side stream, ordered after the
// work queued on the workspace's stream before `after`, so that they run
// beside this round's index update and selection. ws_spec_launch_select
// (after ws_select_prepare): their selection of k seeds, ordered after
// `after`, which must follow this round's index update (the selection reads
// every segment). ws_spec_commit: the speculation becomes the workspace's
// next round (its sets, index segment and selection, as ws_extend_launch and
// ws_select_prepare would have left them); ws_spec_drop: it is discarded
// (both wait for the side stream).
bool ws_spec_possible(const Workspace& w);
imm_status ws_spec_reserve(Workspace& w, uint32_t k);
imm_status ws_spec_launch_index(Workspace& w, hipEvent_t after);
imm_status ws_spec_launch_select(Workspace& w, uint32_t k, hipEvent_t after);
imm_status ws_spec_commit(Workspace& w);
imm_status ws_spec_drop(Workspace& w);
// Both halves and the synchronisation in between.
imm_status ws_extend(Workspace& w, const imm_graph* g, uint64_t seed, uint64_t id_lo,
                     uint64_t count);
// Selection: index update and per-instance state for k seeds (on w.st);
// returns the descriptor with its block ranges left for the caller.
imm_status ws_select_prepare(Workspace& w, uint32_t k, SelectDesc* d);
// The index update alone (the new sets' segment, on w.st; nothing when every
// set is indexed), as ws_select_prepare begins.
imm_status ws_index_update(Workspace& w);
// Queue the copy-out of gains, pool size and error flag on stream st.
imm_status ws_select_copy_out(Workspace& w, uint32_t k, hipStream_t st);
// After st is synchronised: error check, exact pool size, coverage.
imm_status ws_select_finish(Workspace& w, uint32_t k, uint64_t sets_before, uint64_t* covered);
// The selection of this workspace alone, launched on w.st without waiting
// (then ws_select_finish once the stream is done).
// graph: launch the seed steps as w.sel_graph (IMM_GRAPH_SELECT); *graph_out
// (if given) is 0 when they were launched directly, 1 when a graph was
// relaunched, 2 when it had to be captured first.
imm_status ws_select_launch(Workspace& w, uint32_t k, bool graph = false,
                            int* graph_out = nullptr);
// Prepare, run and finish the selection of this workspace alone.
imm_status ws_select(Workspace& w, uint32_t k, uint64_t sets_before, uint64_t* covered);
imm_status ws_sync_pool(Workspace& w);
// Empty the pool (sets, counts, index) and keep the buffers, the scalars and
// the set-size estimate: the next sampling call starts a new pool.
imm_status ws_restart_pool(Workspace& w);
// The number of this pool's sets that hold one of seeds[0..k) (device
// array); waits for the stream.
imm_status ws_coverage(Workspace& w, const uint32_t* seeds, uint32_t k, uint64_t* out);
void ws_note_pool(Workspace& w, uint64_t sets_before);
imm_status ws_export_pool(Workspace& w, std::vector<uint64_t>* so, std::vector<uint32_t>* sv,
                          std::vector<uint32_t>* counts);
void fill_stats(Workspace& w, imm_stats* s);

// ---- tune.cpp
// Pick g's IC team size by timing one fixed sampling batch per candidate
// (sets do not depend on the choice). Once per graph; thread-safe.
imm_status tune_graph(imm_graph* g, hipStream_t st);

// ---- runner.cpp
// Theta constants (Tang et al. 2015, Eq. 9 and Eq. 6 with ell adjusted).
imm_status theta_plan(uint32_t n, uint32_t k, double eps, double ell, double* lambda_prime,
                      double* lambda_star, uint32_t* i_max);
// The early-stopping schedule's first pool size theta_0, its iteration count
// and the exponent a of each bound's failure probability e^-a.
imm_status early_plan(uint32_t n, uint32_t k, double eps, double ell, double* theta0,
                      uint32_t* i_max, double* a);

struct Query;  // one IMM query's state machine (runner.cpp)

// Advances a changing set of queries together, one iteration at a time: an
// iteration launches every active query's sampling round on its own stream,
// waits, finishes the rounds, then runs the greedy selections of all of them
// with one set of launches per seed step on the main stream. Queries may be
// started (and cancelled) between steps; each finishes independently.
class BatchRunner {
public:
    // multi: IC queries sample together in multi-instance launches
    explicit BatchRunner(hipStream_t main, bool multi = false);
    ~BatchRunner();
    BatchRunner(const BatchRunner&) = delete;
    BatchRunner& operator=(const BatchRunner&) = delete;
    // Start a query sampling on stream st; a query that fails to start is
    // returned already finished (and is not active).
    Query* start(imm_graph* g, const imm_params& p, hipStream_t st, uint32_t big_cap);
    // One iteration of every active query; false when none is active.
    bool step();
    // Finish q as cancelled; it leaves at the next step.
    void cancel(Query* q);
    // Queries that finished (result, error or cancellation) since the last call.
    std::vector<Query*> drain();
    size_t active() const { return active_.size(); }
    // The result of a finished query (null unless *status is IMM_OK); frees q.
    static imm_result* take(Query* q, imm_status* status, std::string* err);
    static bool done(const Query* q);
    static uint64_t bytes(const Query* q);  // workspace bytes at the end

private:
    void finish_err(Query* q, imm_status s);
    imm_status multi_pass(const std::vector<Query*>& qs);
    hipStream_t main_;
    bool multi_ = false;
    // the multi-instance launch: shared giant-set slots, and the task table,
    // lane-position prefix and tickets (pinned host copy, device copy)
    void* multi_buf_ = nullptr;
    uint64_t multi_cap_ = 0;
    uint32_t multi_words_ = 0;
    static constexpr size_t kTaskBytes =
        kMaxTasks * sizeof(IcTask) + (kMaxTasks + 1 + 3) * sizeof(uint32_t);
    char* tasks_h_ = nullptr;
    char* tasks_d_ = nullptr;
    std::vector<Query*> active_, finished_;
    SelectDesc* descs_h_ = nullptr;
    SelectDesc* descs_d_ = nullptr;
    size_t cap_descs_ = 0;
    hipEvent_t ev_a_ = nullptr, ev_b_ = nullptr;
    SelectGraph graph_;  // the batched seed steps (IMM_GRAPH_SELECT)
    SampleGraph sgraph_; // the multi-instance sampling launch (IMM_GRAPH_SAMPLE)
};

// Runs queries independently of each other, each on its own stream: the
// host never waits for one query's GPU work while another query's is ready
// to advance. poll() advances every query whose queued work has finished
// (finish its sampling round and launch its selection; or take its theta
// decision and launch its next round) and returns whether any did.
class AsyncRunner {
public:
    AsyncRunner() = default;
    ~AsyncRunner();
    AsyncRunner(const AsyncRunner&) = delete;
    AsyncRunner& operator=(const AsyncRunner&) = delete;
    Query* start(imm_graph* g, const imm_params& p, hipStream_t st, uint32_t big_cap);
    bool poll();
    void cancel(Query* q);
    std::vector<Query*> drain();
    size_t active() const { return active_.size(); }

private:
    void finish_err(Query* q, imm_status s);
    std::vector<Query*> active_, finished_;
};
// Device bytes held by the idle workspaces cached on g, and freeing them all
// (returns the bytes freed).
uint64_t cached_bytes(imm_graph* g);
uint64_t trim_cache(imm_graph* g);
// Run queries to completion, advancing them together round by round.
// streams[q] (may repeat) is the stream query q samples on; `main` carries
// the batched selection. out[q] receives a result or stays null with
// status[q] set.
void run_queries(imm_graph* const* graphs, const imm_params* params, uint32_t count,
                 hipStream_t main, const hipStream_t* streams, imm_result** out,
                 imm_status* status, std::string* errors);

}  // namespace imm
