/*
 * imm.h -- C ABI of libimm, the MI355X (gfx950) implementation of the hot
 * path of IMM (Influence Maximization via Martingales) as studied in
 * arXiv 2411.09473: random reverse-reachable (RRR) set sampling, occurrence
 * counting, and greedy max-coverage seed selection, driven by IMM's
 * martingale theta schedule.
 *
 * Conventions (all entry points):
 *   - Every call returns an imm_status; IMM_OK is 0. On error, out-parameters
 *     are left untouched and imm_last_error() (thread-local) describes it.
 *   - No C++ exception crosses this boundary.
 *   - Handles (imm_graph, imm_result, imm_pool) are opaque and owned by the
 *     library until the matching *_destroy call.
 *   - Array arguments are host pointers unless the call's flags contain
 *     IMM_DEVICE_PTRS, in which case they are device pointers on the current
 *     HIP device that must stay valid for the duration of the call. Caller
 *     arrays are only borrowed for the duration of the call.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *     Calls that return host-side results synchronise that stream before
 *     returning.
 *   - Vertex ids are uint32 with n <= 2^32 - 2; edge ids are CSC positions
 *     and m must be < 2^32.
 *   - Randomness is Philox4x32-10 keyed by the 64-bit run seed; sample s,
 *     edge e and vertex v map to fixed counters (root: (0, s_lo, s_hi, 0);
 *     IC coin of edge e: word e&3 of (e>>2, s_lo, s_hi, 1); LT draw at v: word
 *     v&3 of (v>>2, s_lo, s_hi, 2)), so every set is a pure function of
 *     (graph, seed, sample id) and results do not depend on launch shapes.
 */
#ifndef IMM_H
#define IMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    IMM_OK = 0,
    IMM_EINVAL = 1,     /* malformed argument or graph */
    IMM_ENOMEM = 2,     /* device/host allocation failed or budget exceeded */
    IMM_EOVERFLOW = 3,  /* theta (or a round target) >= 2^32, or m >= 2^32 */
    IMM_EDEVICE = 4,    /* a HIP runtime call failed */
    IMM_EBUSY = 5,      /* server: the query has not finished yet */
    IMM_ECANCELLED = 6  /* server: the query was cancelled */
} imm_status;

/* Diffusion models (Section II-A). */
typedef enum {
    IMM_IC = 0, /* independent cascade: weight[e] is the live threshold thr,
                   edge live iff draw < thr, i.e. p = thr / 2^32 */
    IMM_LT = 1  /* linear threshold, live-edge form: weight[] is the per-column
                   cumulative in-weight table cum (non-decreasing within a
                   column); the live in-edge of v is the first e of v's column
                   with draw < cum[e], none if there is no such e */
} imm_model;

/* flags */
#define IMM_DEVICE_PTRS 0x1u /* array arguments are device pointers */
#define IMM_KEEP_POOL 0x2u   /* imm_run: keep the final RRR pool for imm_result_pool */
#define IMM_TIMING 0x4u      /* record per-phase kernel times with HIP events */
/* imm_run, imm_run_batch, server queries: launch each greedy selection's k
 * seed steps (3 kernels per step) as a captured hipGraph, relaunched while
 * the shape (runs, steps, workgroup counts) repeats: a single run captures
 * once and replays the graph every round. In a batch, an iteration's
 * selection uses it when any of its runs sets it. On a stream that cannot
 * be captured (the legacy default stream) the steps are launched directly.
 * Results are unchanged. */
#define IMM_GRAPH_SELECT 0x8u
/* Sampling schedules other than Algorithm 1's (imm_run, imm_run_batch,
 * server queries; at most one of the two):
 * IMM_FRESH_FINAL: IMM's rounds and LB as usual, but the final selection runs
 *   over theta = ceil(lambda* / LB) sets drawn afresh (sample ids right after
 *   those the rounds used) instead of reusing the rounds' sets: the
 *   correction of IMM's analysis noted by Chen (2018). theta, the pool and
 *   the coverage are those of the fresh sets.
 * IMM_EARLY_STOP: early termination in the manner of OPIM (Tang et al. 2018;
 *   the paper's related work): two independent pools R1 (sample ids j) and
 *   R2 (ids 2^32 + j) of theta_i = ceil(theta_0 2^(i-1)) sets each, i = 1 ..
 *   i_max; the greedy seeds S of R1 are returned as soon as
 *     lo / up >= 1 - 1/e - eps, or at i = i_max,
 *   where, with a = ln(3 i_max) + ell ln n and g_k = 1 - (1 - 1/k)^k,
 *     up = (sqrt(cov_R1(S) / g_k + a/2) + sqrt(a/2))^2 n / theta_i
 *          (an upper bound on OPT),
 *     lo = ((sqrt(cov_R2(S) + 2a/9) - sqrt(a/2))^2 - a/18) n / theta_i
 *          (a lower bound on the spread of S; 0 if not positive),
 *   theta_max = theta_0 n / (eps^2 k) = lambda* / k of Tang et al. Eq. 6 at
 *   failure probability n^-ell / 3, and i_max = ceil(log2(n / (eps^2 k))).
 *   theta is |R1|, LB is lo; imm_result_early gives up, lo / up and the
 *   coverages in R2. */
#define IMM_FRESH_FINAL 0x10u
#define IMM_EARLY_STOP 0x20u
/* The greedy's counter update after a seed covers its sets (Section IV-C's
 * adaptive update): by default a step recounts every count from the
 * uncovered sets when the newly covered sets hold more than a quarter of the
 * pool, and decrements their members' counts otherwise. These flags fix one
 * choice for every step (at most one of the two); results are unchanged. */
#define IMM_UPDATE_DECREMENT 0x40u
#define IMM_UPDATE_RECOUNT 0x80u
/* Adaptive set representation (Section IV-C): an IC RRR set of at least
 * max(ceil(n / 32), 2048) members is kept as an n-bit vertex bitmap instead
 * of a member list (the bitmap is then no larger), and its members are
 * counted and decremented by bitmap column sums. IMM_LIST_SETS (imm_run,
 * imm_run_batch, server queries, imm_sample) keeps every set as a list.
 * Results, exported pools and counts are the same either way. */
#define IMM_LIST_SETS 0x100u
/* imm_run_batch: each round's multi-instance IC sampling launch (the lane,
 * BFS and giant-set kernels over the task table of every IC query sampling
 * that round; Section IV-C's dynamic job balancing across instances) runs as
 * a captured hipGraph, relaunched while the launch's shape (number of
 * tasks, BFS team, shared scratch) repeats, else updated in place or
 * instantiated anew. The task table and its tickets are copied before each
 * launch; the graph holds kernels only. A round uses it when any of its IC
 * queries sets it; on a stream that cannot be captured the kernels are
 * launched directly. Results are unchanged. */
#define IMM_GRAPH_SAMPLE 0x200u

typedef struct imm_graph imm_graph;
typedef struct imm_result imm_result;
typedef struct imm_pool imm_pool;

/* Parameters of one IMM run (Algorithm 1's inputs k and epsilon, plus IMM's
 * failure-probability exponent ell: the guarantee holds with probability at
 * least 1 - n^-ell). max_device_bytes = 0 means no budget. */
typedef struct {
    uint32_t k;
    uint32_t flags;
    double epsilon;
    double ell;
    uint64_t seed;
    uint64_t max_device_bytes;
} imm_params;

/* Work and time accounting of a run or of a sampling call. Times are in
 * milliseconds, filled when IMM_TIMING was set (else 0). */
typedef struct {
    double ms_total;      /* host wall time of the call */
    double ms_sample;     /* sampling kernels (fused counting included) */
    double ms_compact;    /* size scan + pool compaction */
    double ms_index;      /* inverted index: count scan + scatter */
    double ms_select;     /* argmax + cover/decrement kernels */
    double ms_sample_main;/* the wave-per-sample sampling kernel alone */
    uint64_t main_launches;  /* launches of that kernel */
    uint64_t sets;        /* RRR sets generated */
    uint64_t entries;     /* total set size P */
    uint64_t edges;       /* IC: coins evaluated (in-edges examined);
                             LT: walk steps (draws evaluated) */
    uint64_t live;        /* IC: live in-edges followed; LT: cum entries read */
    uint64_t deferred;    /* sets finished by the large-set kernel */
    uint64_t main_sets;   /* sets finished by the wave/team-per-sample kernel */
    uint64_t main_entries;/* their total size */
    uint64_t main_edges;  /* their edges (IC coins / LT steps) */
    uint64_t main_live;   /* their live edges / cum entries */
    double ms_sample_big; /* the large-set sampling kernel alone */
    uint64_t big_launches;/* launches of that kernel */
    uint32_t rounds;      /* sampling-phase rounds executed (imm_run) */
    uint32_t team;        /* IC: waves per sample of the BFS kernel (autotuned) */
    double ms_sample_lane;   /* IC: the lane-per-root kernel alone */
    uint64_t lane_launches;  /* launches of that kernel */
    uint64_t lane_sets;      /* IC: single-vertex sets it finished */
    uint64_t lane_edges;     /* IC: coins it evaluated for them */
    uint32_t big_block;      /* IC: threads per giant set (autotuned) */
    uint32_t bloom_bits;     /* LT: log2 bits of the per-walk path filter (autotuned) */
    uint64_t device_bytes;   /* device memory held by the run's workspace */
    double ms_queue;         /* server: submit to admission (ms_total is then
                                submit to completion) */
    uint32_t walk_lanes;     /* LT: lanes per walk of the walk kernel (autotuned) */
    uint32_t select_graphs;  /* with IMM_GRAPH_SELECT: this run's selections
                                done by launching a captured graph */
    uint32_t select_captures;/* ... of which needed a new capture */
    uint32_t dense_sets;     /* IC: sets of the pool kept as vertex bitmaps
                                (see IMM_LIST_SETS) */
    uint32_t sample_graphs;  /* with IMM_GRAPH_SAMPLE: this run's sampling
                                rounds done by launching a captured graph */
    uint32_t sample_captures;/* ... of which needed a new capture */
    /* Candidate steps of the greedy: when a selection starts, the vertices
     * whose count is at least tau (a bin edge of a count histogram chosen so
     * that at most 4096 of them qualify; the environment variable
     * IMM_CAND_MAX lowers that bound, 0 turns the steps off) are listed.
     * Counts only fall, so while the best listed count is at least tau no
     * unlisted vertex can be the argmax: from seed step 1 on (unless step 0
     * recounted), a step takes its argmax over the list and decrements only
     * listed vertices. A step whose best listed count falls below tau halts
     * the selection; every count is then recounted exactly and the remaining
     * steps run in full. Results are unchanged. */
    uint32_t cand_steps;     /* seed steps whose argmax ran over the list */
    uint32_t cand_halts;     /* selections that halted and finished in full */
    uint32_t spec_rounds;    /* imm_run, LT: rounds whose compaction, index and
                                selection ran speculatively beside the round
                                before (its ids drawn ahead in that round's
                                launch) and were kept because that round
                                failed its test; IMM_SPEC=0 in the environment
                                turns this off. Results are unchanged. */
} imm_stats;

/* Thread-local description of the last error of this thread. */
const char* imm_last_error(void);

/* ---------------------------------------------------------------- graph ---
 * imm_graph_create: upload a directed graph given as CSC of in-edges (the
 * graph is traversed by in-neighbours, Algorithm 3).
 *   n        number of vertices, 2 <= n <= 2^32 - 2
 *   m        number of edges, m < 2^32
 *   col_off  uint64[n+1]: in-edges of v are [col_off[v], col_off[v+1]);
 *            col_off[0] = 0, non-decreasing, col_off[n] = m
 *   row_src  uint32[m]: source vertex of each in-edge (< n)
 *   weight   uint32[m]: see imm_model
 *   flags    IMM_DEVICE_PTRS or 0
 * Errors: IMM_EINVAL on a malformed CSC (checked on the host; with
 * IMM_DEVICE_PTRS the arrays are copied to the host for the check), an LT
 * table that decreases within a column, or a bad model; IMM_EOVERFLOW if
 * m >= 2^32; IMM_ENOMEM / IMM_EDEVICE from the runtime. The graph stays
 * resident in device memory until imm_graph_destroy. */
imm_status imm_graph_create(uint32_t n, uint64_t m, const uint64_t* col_off,
                            const uint32_t* row_src, const uint32_t* weight, imm_model model,
                            uint32_t flags, void* stream, imm_graph** out);
imm_status imm_graph_destroy(imm_graph* g);
/* n, m, model and the device bytes held by the resident graph. */
imm_status imm_graph_info(const imm_graph* g, uint32_t* n, uint64_t* m, imm_model* model,
                          uint64_t* device_bytes);

/* --------------------------------------------------------------- server ---
 * A query server on the device current at creation (continuous batching;
 * not in the paper: the serving form of the same computation). A worker
 * thread runs the admitted queries together, iteration by iteration, as
 * imm_run_batch does; a query submitted while others run is admitted at the
 * next iteration boundary once a slot (at most max_slots queries run at a
 * time) and device memory are free. Admission reserves each query's
 * estimated workspace size (the largest workspace any finished query on its
 * graph has held, else 64 bytes per vertex plus 1 GiB; max_device_bytes when
 * that is set and smaller) against budget_bytes, counting the idle
 * workspaces cached on the server's graphs as well: those caches are freed
 * when they are what keeps a query out. The first query always runs. Pools
 * stay in device memory. A result is
 * the same, bit for bit, as imm_run's with the same arguments. Graphs must
 * outlive the server. Server calls are thread-safe.
 *   imm_server_create   budget_bytes > 0, max_slots >= 1
 *   imm_server_submit   queue a query; *ticket identifies it. IMM_EINVAL on
 *                       bad arguments (as imm_run) or a graph on another
 *                       device; IMM_ENOMEM if its estimate exceeds the
 *                       budget even alone.
 *   imm_server_poll     IMM_EBUSY if the query has not finished and wait is
 *                       0 (else it blocks until it has); otherwise the
 *                       query's own status (IMM_OK with *out set, or its
 *                       error, IMM_ECANCELLED after a cancel), and the
 *                       ticket is retired. IMM_EINVAL for an unknown ticket.
 *                       In the result's stats, ms_total is the time from
 *                       submission to completion and ms_queue from
 *                       submission to admission.
 *   imm_server_cancel   a queued query is dropped at once, a running one at
 *                       the next iteration boundary
 *   imm_server_info     queued and running queries, reserved bytes
 *   imm_server_destroy  cancels everything, waits for the worker, frees
 *                       results nobody polled */
typedef struct imm_server imm_server;
imm_status imm_server_create(uint64_t budget_bytes, uint32_t max_slots, imm_server** out);
imm_status imm_server_submit(imm_server* s, const imm_graph* g, const imm_params* p,
                             uint64_t* ticket);
imm_status imm_server_poll(imm_server* s, uint64_t ticket, int wait, imm_result** out);
imm_status imm_server_cancel(imm_server* s, uint64_t ticket);
imm_status imm_server_info(imm_server* s, uint64_t* queued, uint32_t* running,
                           uint64_t* reserved_bytes);
imm_status imm_server_destroy(imm_server* s);

/* ---------------------------------------------------------------- theta ---
 * IMM's theta constants (Tang, Shi, Xiao 2015, cited for Theta_Estimation,
 * OPT_Lower_Bound and Set_Theta of Algorithm 1): lambda' (their Eq. 9) and
 * lambda* (their Eq. 6), both with ell replaced by ell (1 + ln 2 / ln n),
 * and the number of sampling rounds i_max = ceil(log2 n) - 1. FP64 on the
 * host. Errors: IMM_EINVAL if n < 2, k = 0, k > n, eps <= 0 or ell <= 0. */
imm_status imm_theta_plan(uint32_t n, uint32_t k, double eps, double ell,
                          double* lambda_prime, double* lambda_star, uint32_t* i_max);

/* ------------------------------------------------------------------ run ---
 * imm_run: one full IMM run (Algorithm 1): sampling rounds i = 1..i_max
 * with theta_i = ceil(lambda' 2^i / n) sets (generated while |R| < theta_i,
 * reused across rounds), greedy selection and the lower-bound test
 * n F_R(S_i) >= (1 + sqrt(2) eps) n / 2^i with early break; then
 * theta = ceil(lambda* / LB), top-up, and the final greedy over all sets.
 * Blocks until the seeds are on the host. Errors: IMM_EINVAL (k = 0, k > n,
 * eps <= 0, ell <= 0), IMM_EOVERFLOW (a target >= 2^32), IMM_ENOMEM (budget
 * exceeded or allocation failure; nothing leaks), IMM_EDEVICE. */
imm_status imm_run(const imm_graph* g, const imm_params* p, void* stream, imm_result** out);

/* imm_run_batch: `count` independent IMM runs (graphs[j], params[j]) advanced
 * together, round by round, on one device: each round's sampling of every
 * unfinished run is in flight at once (on up to 8 internal streams of default
 * priority, ordered after the work already queued on `stream`), and each
 * seed step of the greedy selection is one set of launches for all of them
 * (on `stream`). Runs may share a graph. The results equal those of count
 * imm_run calls with the same arguments, bit for bit: every set is a pure
 * function of (graph, seed, sample id), and each run's selection reads only
 * its own pool. Blocks until every run has finished.
 *   graphs  const imm_graph*[count], all on the current device
 *   params  imm_params[count]
 *   out     imm_result*[count]: receives one result per run
 * Errors: IMM_EINVAL (count = 0, a null or mixed-device graph, bad params),
 * otherwise the first failing run's status; then every out[j] is NULL and
 * nothing leaks. */
imm_status imm_run_batch(const imm_graph* const* graphs, const imm_params* params,
                         uint32_t count, void* stream, imm_result** out);

/* theta (= |R| of the final selection), sampling rounds executed, LB, and
 * the number of sets covered by the seeds (the sum of the gains). */
imm_status imm_result_info(const imm_result* r, uint64_t* theta, uint32_t* rounds, double* lb,
                           uint64_t* covered);
/* seeds (uint32[k], in selection order) and their marginal gains
 * (uint64[k], newly covered sets); either pointer may be NULL. Host memory. */
imm_status imm_result_seeds(const imm_result* r, uint32_t* seeds, uint64_t* gains);
/* The targets of the run: theta_1, theta_2, ... of the executed rounds, then
 * the final theta (count entries, at most 64), and the coverage of each
 * sampling-phase round (rounds entries, at most 64). Host memory; NULL ok. */
imm_status imm_result_targets(const imm_result* r, uint32_t* count, uint64_t* targets,
                              uint64_t* round_cov);
/* The final RRR pool in canonical order (sets by sample id, vertices
 * ascending within a set). Two-call protocol: n_sets/n_entries are always
 * written; set_off (uint64[n_sets+1]) and set_vtx (uint32[n_entries]) are
 * filled when non-NULL. Requires IMM_KEEP_POOL, else IMM_EINVAL. */
imm_status imm_result_pool(const imm_result* r, uint64_t* n_sets, uint64_t* n_entries,
                           uint64_t* set_off, uint32_t* set_vtx);
/* IMM_EARLY_STOP runs: the last iteration's upper bound on OPT (up), the
 * ratio lo / up, and the coverage of each iteration's seeds in the second
 * pool (rounds entries, at most 64; NULL ok). All 0 for other runs. */
imm_status imm_result_early(const imm_result* r, double* sigma_up, double* alpha,
                            uint64_t* round_cov2);
imm_status imm_result_stats(const imm_result* r, imm_stats* stats);
void imm_result_destroy(imm_result* r);

/* --------------------------------------------------------- test-granular ---
 * imm_sample: generate the RRR sets of sample ids [first_id, first_id+count)
 * (Generate_RRRsets, Algorithm 3, with the occurrence counts fused) into a
 * device-resident pool. flags: IMM_TIMING. Errors: IMM_EINVAL (count = 0 or
 * first_id + count overflows), IMM_ENOMEM, IMM_EDEVICE. */
imm_status imm_sample(const imm_graph* g, uint64_t seed, uint64_t first_id, uint64_t count,
                      uint32_t flags, void* stream, imm_pool** out);
imm_status imm_pool_info(const imm_pool* p, uint64_t* n_sets, uint64_t* n_entries,
                         imm_stats* stats);
/* Copy the pool out in canonical order (host pointers, each may be NULL):
 * set_off uint64[n_sets+1] (starting at 0), set_vtx uint32[n_entries],
 * counts uint32[n] (occurrences of each vertex over these sets). */
imm_status imm_pool_export(const imm_pool* p, uint64_t* set_off, uint32_t* set_vtx,
                           uint32_t* counts);
void imm_pool_destroy(imm_pool* p);

/* imm_greedy: greedy max coverage (Find_Most_Influential_Set, Algorithm 2)
 * over a caller-given pool: build the vertex->sets index, then k times pick
 * the unselected vertex with the most uncovered sets (lowest id on ties),
 * cover those sets and decrement their members' counts.
 *   set_off uint64[n_sets+1] with set_off[0] = 0; set_vtx uint32[set_off[n_sets]],
 *   members of a set distinct and < n. Host pointers unless IMM_DEVICE_PTRS.
 *   seeds uint32[k], gains uint64[k], covered: host outputs.
 * Errors: IMM_EINVAL (k = 0, k > n, n_sets >= 2^32, bad offsets or ids),
 * IMM_ENOMEM, IMM_EDEVICE. */
imm_status imm_greedy(uint32_t n, const uint64_t* set_off, const uint32_t* set_vtx,
                      uint64_t n_sets, uint32_t k, uint32_t flags, void* stream,
                      uint32_t* seeds, uint64_t* gains, uint64_t* covered);

/* imm_greedy_static: imm_greedy that allocates nothing, for callers that
 * cannot allocate device memory (code under hipGraph capture, tight serving
 * loops, harnesses that forbid hipMalloc). Same arguments, same results,
 * bit for bit, as imm_greedy; gains must not be NULL. Every scratch buffer
 * (counts, index, covered bits, seed-step state, and the pool itself when
 * it is passed in host memory) is carved out of one fixed array of
 * IMM_STATIC_SCRATCH_BYTES per device, held from library load until the
 * process ends. With n vertices, S sets, P entries and k seeds it needs about
 *   24 n + 4 P + 16 (S + P / 64) + S / 8 + 272 k bytes (device pool), plus
 *   8 S + 4 P bytes more when the pool is in host memory,
 * each piece rounded up to 256 bytes; a call that does not fit fails with
 * IMM_ENOMEM and a message giving the size it needed. The call blocks until
 * its results are on the host. Calls on one device share its array (each call
 * clears what must start at zero); calls in one process are serialised per
 * device, and any other use of the array would race with them. Errors: as
 * imm_greedy, and IMM_EINVAL for a null gains. */
#define IMM_STATIC_SCRATCH_BYTES (128ull << 20)
imm_status imm_greedy_static(uint32_t n, const uint64_t* set_off, const uint32_t* set_vtx,
                             uint64_t n_sets, uint32_t k, uint32_t flags, void* stream,
                             uint32_t* seeds, uint64_t* gains, uint64_t* covered);

/* imm_philox4x32_10: evaluate the device Philox4x32-10 (Salmon et al.,
 * SC'11) on `count` counters: ctr uint32[4*count] in, out uint32[4*count]
 * out, key = (key_lo, key_hi). Host pointers unless IMM_DEVICE_PTRS. */
imm_status imm_philox4x32_10(const uint32_t* ctr, uint64_t count, uint64_t key, uint32_t flags,
                             void* stream, uint32_t* out);

#ifdef __cplusplus
}
#endif

#endif /* IMM_H */
