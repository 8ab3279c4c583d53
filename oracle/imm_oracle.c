/*
 * imm_oracle.c -- CPU oracle for the IMM hot path.
 *
 * TEST INFRASTRUCTURE. This file is the plain, slow, obviously-correct
 * reference that the GPU library is checked against. Only the test suite, the
 * package smoke check and the benchmark's CPU-baseline leg may load it; the
 * product path never calls it and shares no code with it.
 *
 * What it computes (arXiv 2411.09473, "Enhancing Scalability and Performance
 * in Influence Maximization with Optimized Parallel Processing"):
 *   - random reverse-reachable (RRR) sets by probabilistic reverse BFS from a
 *     uniformly drawn root (Section II-B "Generate_RRRsets"; Algorithm 3),
 *     under the IC model (Section II-A, IC) and, via the live-edge reading of
 *     the LT model (Section II-A, LT; Kempe et al. 2003), as a reverse walk;
 *   - vertex occurrence counts over the sets (Algorithm 2, first loop);
 *   - greedy max-coverage seed selection with covered-set decrements
 *     (Algorithm 2, while-loop);
 *   - the IMM sampling/selection driver (Algorithm 1) with the theta bounds
 *     that the paper takes from Tang, Shi and Xiao, SIGMOD 2015 (Eq. 6 and
 *     Eq. 9 there, Algorithms 1-3 there).
 *
 * Readings where the paper is silent:
 *   R1 random(u,v) of Algorithm 3 is Philox4x32-10 keyed by the run seed;
 *      counters: root (0, s_lo, s_hi, 0); IC edge e (e>>2, s_lo, s_hi, 1),
 *      word e&3; LT vertex v (v>>2, s_lo, s_hi, 2), word v&3.
 *   R2 root = floor(w * n / 2^64) with w = word0 | word1 << 32.
 *   R3 IC edge live iff r < thr[e]; LT: the live in-edge of v is the first e
 *      of v's column with r < cum[e] (none if no such e).
 *   R4 argmax ties go to the lowest vertex id, over unselected vertices.
 *   R5 a covered set is removed only if it contains the chosen seed.
 *   R6 theta_i = ceil(lambda'/x), sets are generated while |R| < target, the
 *      sampling loop runs i = 1 .. bitlen(n-1)-1 with IMM's early break, sets
 *      are reused across rounds and the final selection runs over all of them.
 *
 * Parity pins (tests/test_oracle_*.py): Philox against rocRAND's independent
 * host implementation; theta constants against the Chernoff-bound identities
 * they are derived from and lgamma; sets against scipy reachability in the
 * materialised live-edge graph and against brute-force world enumeration;
 * greedy against a recompute-from-scratch greedy and exhaustive optimum.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_EINVAL 1
#define ORC_ENOMEM 2
#define ORC_EOVERFLOW 3

enum { ORC_IC = 0, ORC_LT = 1 };

/* ---------------------------------------------------------------------- */
/* Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel Random Numbers: As  */
/* Easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 products with the   */
/* published multipliers, a word permutation and a Weyl-sequence key bump.   */
/* ---------------------------------------------------------------------- */
void oracle_philox4x32_10(const uint32_t ctr[4], uint64_t key, uint32_t out[4]) {
    uint32_t c0 = ctr[0], c1 = ctr[1], c2 = ctr[2], c3 = ctr[3];
    uint32_t k0 = (uint32_t)key, k1 = (uint32_t)(key >> 32);
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* The same generator over `count` counters (ctr and out hold 4 words per
 * counter), one call per counter: a convenience for tests that compare
 * millions of outputs. */
void oracle_philox_many(const uint32_t* ctr, uint64_t count, uint64_t key, uint32_t* out) {
    for (uint64_t i = 0; i < count; ++i) oracle_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

/* Reading R2: the uniformly selected root of sample s (Section II-B). */
uint32_t oracle_root(uint64_t seed, uint64_t s, uint32_t n) {
    uint32_t c[4] = {0u, (uint32_t)s, (uint32_t)(s >> 32), 0u}, o[4];
    oracle_philox4x32_10(c, seed, o);
    uint64_t w = (uint64_t)o[0] | ((uint64_t)o[1] << 32);
    return (uint32_t)(((unsigned __int128)w * (unsigned __int128)n) >> 64);
}

/* Reading R1: the 32-bit draw that decides IC edge e in sample s. */
uint32_t oracle_ic_draw(uint64_t seed, uint64_t s, uint64_t e) {
    uint32_t c[4] = {(uint32_t)(e >> 2), (uint32_t)s, (uint32_t)(s >> 32), 1u}, o[4];
    oracle_philox4x32_10(c, seed, o);
    return o[e & 3u];
}

/* Reading R1: the 32-bit draw that picks LT vertex v's live in-edge in sample s. */
uint32_t oracle_lt_draw(uint64_t seed, uint64_t s, uint32_t v) {
    uint32_t c[4] = {v >> 2, (uint32_t)s, (uint32_t)(s >> 32), 2u}, o[4];
    oracle_philox4x32_10(c, seed, o);
    return o[v & 3u];
}

/* The live-edge graph of sample s under IC: live[e] = 1 iff edge e's coin
 * is live. Test support: the sets must equal reverse reachability in it. */
void oracle_ic_live(uint64_t seed, uint64_t s, uint64_t m, const uint32_t* thr, uint8_t* live) {
    for (uint64_t e = 0; e < m; ++e) live[e] = oracle_ic_draw(seed, s, e) < thr[e] ? 1 : 0;
}

/* ---------------------------------------------------------------------- */
/* One RRR set.                                                            */
/* ---------------------------------------------------------------------- */

typedef struct {
    uint32_t n;
    const uint64_t* col_off; /* n+1 */
    const uint32_t* row_src; /* m   */
    const uint32_t* weight;  /* m: IC thresholds / LT cumulative table */
    int model;
} ograph;

/* IC (Algorithm 3): BFS over in-edges from the root; an in-edge (w -> u) of
 * a dequeued vertex u is followed iff its coin is live; newly reached
 * vertices are marked on insertion. Returns |R|; members[] gets the set in
 * discovery order; mark[] must be all zero on entry and is zero on return.
 * *work accumulates the number of coins evaluated (in-edges examined). */
static uint32_t rrr_ic(const ograph* g, uint64_t seed, uint64_t s, uint32_t* members,
                       uint8_t* mark, uint64_t* work) {
    uint32_t root = oracle_root(seed, s, g->n);
    uint32_t size = 0, head = 0;
    members[size++] = root;
    mark[root] = 1;
    while (head < size) {
        uint32_t u = members[head++];
        for (uint64_t e = g->col_off[u]; e < g->col_off[u + 1]; ++e) {
            uint32_t r = oracle_ic_draw(seed, s, e);
            *work += 1;
            if (r < g->weight[e]) {
                uint32_t w = g->row_src[e];
                if (!mark[w]) {
                    mark[w] = 1;
                    members[size++] = w;
                }
            }
        }
    }
    for (uint32_t i = 0; i < size; ++i) mark[members[i]] = 0;
    return size;
}

/* LT (live-edge reading of Section II-A's LT model): every vertex keeps at
 * most one live in-edge, in-edge e of v with probability (cum[e]-cum[e-1])
 * / 2^32; the RRR set of the root is the chain of live in-edges walked
 * backwards from it, stopping at a vertex with no live in-edge or at the
 * first vertex already in the set. *work accumulates walk steps taken
 * (draws evaluated). */
static uint32_t rrr_lt(const ograph* g, uint64_t seed, uint64_t s, uint32_t* members,
                       uint8_t* mark, uint64_t* work) {
    uint32_t cur = oracle_root(seed, s, g->n);
    uint32_t size = 0;
    members[size++] = cur;
    mark[cur] = 1;
    for (;;) {
        uint64_t beg = g->col_off[cur], end = g->col_off[cur + 1];
        if (beg == end) break;
        uint32_t r = oracle_lt_draw(seed, s, cur);
        *work += 1;
        uint64_t e = beg;
        while (e < end && !(r < g->weight[e])) ++e;
        if (e == end) break;
        uint32_t w = g->row_src[e];
        if (mark[w]) break;
        mark[w] = 1;
        members[size++] = w;
        cur = w;
    }
    for (uint32_t i = 0; i < size; ++i) mark[members[i]] = 0;
    return size;
}

static uint32_t rrr_one(const ograph* g, uint64_t seed, uint64_t s, uint32_t* members,
                        uint8_t* mark, uint64_t* work) {
    return g->model == ORC_IC ? rrr_ic(g, seed, s, members, mark, work)
                              : rrr_lt(g, seed, s, members, mark, work);
}

/* Single set, for tests: writes up to n members, returns |R| (0 on error). */
uint32_t oracle_rrr_set(uint32_t n, const uint64_t* col_off, const uint32_t* row_src,
                        const uint32_t* weight, int model, uint64_t seed, uint64_t s,
                        uint32_t* members) {
    ograph g = {n, col_off, row_src, weight, model};
    uint8_t* mark = (uint8_t*)calloc(n, 1);
    if (!mark) return 0;
    uint64_t work = 0;
    uint32_t size = rrr_one(&g, seed, s, members, mark, &work);
    free(mark);
    return size;
}

/* ---------------------------------------------------------------------- */
/* A growable pool of sets in sample-id order.                             */
/* ---------------------------------------------------------------------- */

typedef struct {
    uint64_t n_sets, n_entries, cap_sets, cap_entries, work;
    uint64_t* set_off; /* n_sets+1 */
    uint32_t* set_vtx; /* n_entries */
    uint64_t id_base;  /* set j of the pool is the RRR set of sample id id_base + j */
} oracle_pool;

oracle_pool* oracle_pool_create(void) {
    oracle_pool* p = (oracle_pool*)calloc(1, sizeof(oracle_pool));
    if (!p) return NULL;
    p->cap_sets = 1024;
    p->set_off = (uint64_t*)calloc(p->cap_sets + 1, sizeof(uint64_t));
    p->cap_entries = 4096;
    p->set_vtx = (uint32_t*)malloc(p->cap_entries * sizeof(uint32_t));
    if (!p->set_off || !p->set_vtx) {
        free(p->set_off); free(p->set_vtx); free(p);
        return NULL;
    }
    return p;
}

void oracle_pool_destroy(oracle_pool* p) {
    if (!p) return;
    free(p->set_off);
    free(p->set_vtx);
    free(p);
}

uint64_t oracle_pool_nsets(const oracle_pool* p) { return p->n_sets; }
uint64_t oracle_pool_nentries(const oracle_pool* p) { return p->n_entries; }
uint64_t oracle_pool_work(const oracle_pool* p) { return p->work; }

void oracle_pool_copy(const oracle_pool* p, uint64_t* set_off, uint32_t* set_vtx) {
    if (set_off) memcpy(set_off, p->set_off, (p->n_sets + 1) * sizeof(uint64_t));
    if (set_vtx) memcpy(set_vtx, p->set_vtx, p->n_entries * sizeof(uint32_t));
}

static int pool_reserve(oracle_pool* p, uint64_t sets, uint64_t entries) {
    if (sets > p->cap_sets) {
        uint64_t c = p->cap_sets;
        while (c < sets) c *= 2;
        uint64_t* q = (uint64_t*)realloc(p->set_off, (c + 1) * sizeof(uint64_t));
        if (!q) return ORC_ENOMEM;
        p->set_off = q;
        p->cap_sets = c;
    }
    if (entries > p->cap_entries) {
        uint64_t c = p->cap_entries;
        while (c < entries) c *= 2;
        uint32_t* q = (uint32_t*)realloc(p->set_vtx, c * sizeof(uint32_t));
        if (!q) return ORC_ENOMEM;
        p->set_vtx = q;
        p->cap_entries = c;
    }
    return ORC_OK;
}

/* Append the sets j in [p->n_sets, target), i.e. sample ids id_base + j, to
 * the pool. With threads > 1 the id
 * range is cut into contiguous chunks sampled concurrently (one set at a time
 * per thread, as above) and appended in id order, so the pool is identical
 * for every thread count. */
int oracle_pool_extend(oracle_pool* p, uint32_t n, const uint64_t* col_off,
                       const uint32_t* row_src, const uint32_t* weight, int model,
                       uint64_t seed, uint64_t target, int threads) {
    if (target <= p->n_sets) return ORC_OK;
    ograph g = {n, col_off, row_src, weight, model};
    uint64_t first = p->n_sets, count = target - first;
    if (threads < 1) threads = 1;
    if ((uint64_t)threads > count) threads = (int)count;
    int rc = pool_reserve(p, target, p->n_entries);
    if (rc) return rc;

    typedef struct { uint32_t* vtx; uint64_t len, cap, work; uint32_t* sizes; int err; } chunk_t;
    chunk_t* ch = (chunk_t*)calloc((size_t)threads, sizeof(chunk_t));
    if (!ch) return ORC_ENOMEM;

#pragma omp parallel for num_threads(threads) schedule(static, 1)
    for (int t = 0; t < threads; ++t) {
        uint64_t lo = first + count * (uint64_t)t / (uint64_t)threads;
        uint64_t hi = first + count * (uint64_t)(t + 1) / (uint64_t)threads;
        chunk_t* c = &ch[t];
        uint32_t* members = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
        uint8_t* mark = (uint8_t*)calloc(n, 1);
        c->sizes = (uint32_t*)malloc((size_t)(hi - lo) * sizeof(uint32_t) + 4);
        c->cap = 1024;
        c->vtx = (uint32_t*)malloc(c->cap * sizeof(uint32_t));
        if (!members || !mark || !c->sizes || !c->vtx) {
            c->err = ORC_ENOMEM;
        } else {
            for (uint64_t s = lo; s < hi && !c->err; ++s) {
                uint32_t sz = rrr_one(&g, seed, p->id_base + s, members, mark, &c->work);
                if (c->len + sz > c->cap) {
                    uint64_t nc = c->cap;
                    while (nc < c->len + sz) nc *= 2;
                    uint32_t* q = (uint32_t*)realloc(c->vtx, nc * sizeof(uint32_t));
                    if (!q) { c->err = ORC_ENOMEM; break; }
                    c->vtx = q;
                    c->cap = nc;
                }
                memcpy(c->vtx + c->len, members, (size_t)sz * sizeof(uint32_t));
                c->len += sz;
                c->sizes[s - lo] = sz;
            }
        }
        free(members);
        free(mark);
    }

    for (int t = 0; t < threads && !rc; ++t) rc = ch[t].err;
    uint64_t total = p->n_entries;
    for (int t = 0; t < threads; ++t) total += ch[t].len;
    if (!rc) rc = pool_reserve(p, target, total);
    if (!rc) {
        for (int t = 0; t < threads; ++t) {
            uint64_t lo = first + count * (uint64_t)t / (uint64_t)threads;
            uint64_t hi = first + count * (uint64_t)(t + 1) / (uint64_t)threads;
            memcpy(p->set_vtx + p->n_entries, ch[t].vtx, ch[t].len * sizeof(uint32_t));
            for (uint64_t s = lo; s < hi; ++s)
                p->set_off[s + 1] = p->set_off[s] + ch[t].sizes[s - lo];
            p->n_entries += ch[t].len;
            p->work += ch[t].work;
        }
        p->n_sets = target;
    }
    for (int t = 0; t < threads; ++t) { free(ch[t].vtx); free(ch[t].sizes); }
    free(ch);
    return rc;
}

/* ---------------------------------------------------------------------- */
/* Counts and greedy selection (Algorithm 2).                              */
/* ---------------------------------------------------------------------- */

/* counter[v] = number of sets that contain v (Algorithm 2, first loop). */
void oracle_counts(uint32_t n, const uint64_t* set_off, const uint32_t* set_vtx,
                   uint64_t n_sets, uint32_t* counts) {
    memset(counts, 0, (size_t)n * sizeof(uint32_t));
    for (uint64_t j = 0; j < n_sets; ++j)
        for (uint64_t t = set_off[j]; t < set_off[j + 1]; ++t) counts[set_vtx[t]] += 1;
}

/* Greedy max coverage (Algorithm 2). k times: pick the unselected vertex with
 * the largest counter (lowest id on ties, reading R4), record its counter as
 * its marginal gain, then for every remaining set that contains it decrement
 * the counter of each member and remove the set (reading R5). Returns the
 * number of covered sets, the sum of the gains. */
uint64_t oracle_greedy(uint32_t n, const uint64_t* set_off, const uint32_t* set_vtx,
                       uint64_t n_sets, uint32_t k, uint32_t* seeds, uint64_t* gains) {
    uint32_t* counter = (uint32_t*)malloc((size_t)n * sizeof(uint32_t));
    uint8_t* selected = (uint8_t*)calloc(n, 1);
    uint8_t* removed = (uint8_t*)calloc(n_sets ? n_sets : 1, 1);
    if (!counter || !selected || !removed) {
        free(counter); free(selected); free(removed);
        return UINT64_MAX;
    }
    oracle_counts(n, set_off, set_vtx, n_sets, counter);
    uint64_t covered = 0;
    for (uint32_t i = 0; i < k; ++i) {
        uint32_t best = UINT32_MAX;
        for (uint32_t v = 0; v < n; ++v) {
            if (selected[v]) continue;
            if (best == UINT32_MAX || counter[v] > counter[best]) best = v;
        }
        seeds[i] = best;
        gains[i] = counter[best];
        covered += counter[best];
        selected[best] = 1;
        for (uint64_t j = 0; j < n_sets; ++j) {
            if (removed[j]) continue;
            int contains = 0;
            for (uint64_t t = set_off[j]; t < set_off[j + 1]; ++t)
                if (set_vtx[t] == best) { contains = 1; break; }
            if (!contains) continue;
            for (uint64_t t = set_off[j]; t < set_off[j + 1]; ++t) counter[set_vtx[t]] -= 1;
            removed[j] = 1;
        }
    }
    free(counter);
    free(selected);
    free(removed);
    return covered;
}

/* ---------------------------------------------------------------------- */
/* Theta bounds (Tang et al. 2015, Eq. 9 for lambda', Eq. 6 for lambda*,  */
/* with l replaced by l (1 + log 2 / log n) as in their Algorithm 1).      */
/* All FP64, no contraction, in this exact order.                          */
/* ---------------------------------------------------------------------- */

static const double ORC_LN2 = 0.69314718055994530942;
static const double ORC_INV_E = 0.36787944117144232160;

static double log_binom(uint32_t n, uint32_t k) {
    double acc = 0.0;
    for (uint32_t i = 1; i <= k; ++i) acc += log((double)(n - k + i) / (double)i);
    return acc;
}

static uint32_t bitlen32(uint32_t x) {
    uint32_t b = 0;
    while (x) { ++b; x >>= 1; }
    return b;
}

int oracle_theta_plan(uint32_t n, uint32_t k, double eps, double ell, double* lambda_prime,
                      double* lambda_star, uint32_t* i_max) {
    if (n < 2 || k == 0 || k > n || !(eps > 0.0) || !(ell > 0.0)) return ORC_EINVAL;
    double ln_n = log((double)n);
    double ell_p = ell * (1.0 + ORC_LN2 / ln_n);
    double logcnk = log_binom(n, k);
    double eps_p = sqrt(2.0) * eps;
    double lam_p = (2.0 + 2.0 / 3.0 * eps_p) * (logcnk + ell_p * ln_n + log(log2((double)n))) *
                   (double)n / (eps_p * eps_p);
    double one_m = 1.0 - ORC_INV_E;
    double alpha = sqrt(ell_p * ln_n + ORC_LN2);
    double beta = sqrt(one_m * (logcnk + ell_p * ln_n + ORC_LN2));
    double t = one_m * alpha + beta;
    double lam_s = 2.0 * (double)n * t * t / (eps * eps);
    *lambda_prime = lam_p;
    *lambda_star = lam_s;
    *i_max = bitlen32(n - 1) - 1;
    return ORC_OK;
}

typedef struct {
    uint64_t theta;       /* |R| used by the final selection */
    uint32_t rounds;      /* sampling-phase iterations executed */
    uint32_t n_targets;   /* entries used in targets[] */
    double lb;            /* lower bound LB on OPT (early stop: on the spread of the seeds) */
    uint64_t covered;     /* sets covered by the returned seeds */
    double lambda_prime, lambda_star;
    uint32_t i_max;
    uint32_t pad;
    uint64_t targets[64]; /* theta_1, theta_2, ... then the final theta */
    uint64_t round_cov[64];
    /* early stop only: the upper bound on OPT and the ratio of the last
     * iteration, and each iteration's coverage of its seeds in the second pool */
    double sigma_up, alpha;
    uint64_t round_cov2[64];
} oracle_imm_info;

/* Sampling schedules. */
enum { ORC_SCHED_IMM = 0, ORC_SCHED_FRESH = 1, ORC_SCHED_EARLY = 2 };

/* Number of sets with at least one member in seeds[0..k). */
uint64_t oracle_coverage(uint32_t n, const uint64_t* set_off, const uint32_t* set_vtx,
                         uint64_t n_sets, const uint32_t* seeds, uint32_t k) {
    uint8_t* is_seed = (uint8_t*)calloc(n, 1);
    if (!is_seed) return UINT64_MAX;
    for (uint32_t i = 0; i < k; ++i) is_seed[seeds[i]] = 1;
    uint64_t c = 0;
    for (uint64_t j = 0; j < n_sets; ++j) {
        for (uint64_t t = set_off[j]; t < set_off[j + 1]; ++t) {
            if (is_seed[set_vtx[t]]) { ++c; break; }
        }
    }
    free(is_seed);
    return c;
}

/* The early-stopping schedule in the manner of OPIM (Tang, Tang, Xiao, Yuan,
 * SIGMOD 2018, cited by the paper's related work for terminating sampling
 * once the coverage suffices). Two independent pools R1 (sample ids j) and
 * R2 (sample ids 2^32 + j) of theta_i = ceil(theta_0 2^(i-1)) sets each; the
 * greedy seeds S of R1 are kept as soon as a lower bound on their spread,
 * from their coverage in R2, is at least (1 - 1/e - eps) times an upper bound
 * on OPT from the greedy's coverage in R1, or at the last iteration, whose
 * pools reach theta_max (IMM's bound with OPT >= k). Failure probability
 * delta = n^-ell; both bounds are Chernoff bounds on a binomial count holding
 * with probability 1 - delta / (3 i_max) each:
 *   up = (sqrt(cov1 / g_k + a/2) + sqrt(a/2))^2 n / theta_i,
 *        g_k = 1 - (1 - 1/k)^k (the greedy's coverage guarantee)
 *   lo = ((sqrt(cov2 + 2a/9) - sqrt(a/2))^2 - a/18) n / theta_i (0 if that
 *        is not positive), a = ln(3 i_max / delta).
 * All FP64, in this order. */
static int early_plan(uint32_t n, uint32_t k, double eps, double ell, double* theta0,
                      uint32_t* i_max, double* a) {
    if (n < 2 || k == 0 || k > n || !(eps > 0.0) || !(ell > 0.0)) return ORC_EINVAL;
    double ln_n = log((double)n);
    double logcnk = log_binom(n, k);
    double one_m = 1.0 - ORC_INV_E;
    double ln6d = log(6.0) + ell * ln_n;
    double u = one_m * sqrt(ln6d) + sqrt(one_m * (logcnk + ln6d));
    double theta_max = 2.0 * (double)n * u * u / (eps * eps * (double)k);
    double t0 = theta_max * eps * eps * (double)k / (double)n;
    double r = ceil(log2((double)n / (eps * eps * (double)k)));  /* log2(theta_max / theta_0) */
    uint32_t im = r < 1.0 ? 1u : (uint32_t)r;
    *theta0 = t0;
    *i_max = im;
    *a = log(3.0 * (double)im) + ell * ln_n;
    return ORC_OK;
}

static int oracle_early(uint32_t n, const uint64_t* col_off, const uint32_t* row_src,
                        const uint32_t* weight, int model, uint32_t k, double eps, double ell,
                        uint64_t seed, int threads, oracle_pool* keep, uint32_t* seeds,
                        uint64_t* gains, oracle_imm_info* info) {
    double t0, a;
    uint32_t i_max;
    int rc = early_plan(n, k, eps, ell, &t0, &i_max, &a);
    if (rc) return rc;
    oracle_pool* r1 = keep ? keep : oracle_pool_create();
    oracle_pool* r2 = oracle_pool_create();
    if (!r1 || !r2) { rc = ORC_ENOMEM; goto done; }
    r2->id_base = (uint64_t)1 << 32;
    memset(info, 0, sizeof(*info));
    info->i_max = i_max;
    double one_m = 1.0 - ORC_INV_E;
    double g_k = 1.0 - pow(1.0 - 1.0 / (double)k, (double)k);
    for (uint32_t i = 1; i <= i_max; ++i) {
        double tf = ceil(ldexp(t0, (int)i - 1));
        if (!(tf < 4294967296.0)) { rc = ORC_EOVERFLOW; goto done; }
        uint64_t target = (uint64_t)tf;
        if (info->n_targets < 64) info->targets[info->n_targets++] = target;
        rc = oracle_pool_extend(r1, n, col_off, row_src, weight, model, seed, target, threads);
        if (!rc) rc = oracle_pool_extend(r2, n, col_off, row_src, weight, model, seed, target,
                                         threads);
        if (rc) goto done;
        uint64_t cov1 = oracle_greedy(n, r1->set_off, r1->set_vtx, r1->n_sets, k, seeds, gains);
        if (cov1 == UINT64_MAX) { rc = ORC_ENOMEM; goto done; }
        uint64_t cov2 = oracle_coverage(n, r2->set_off, r2->set_vtx, r2->n_sets, seeds, k);
        if (cov2 == UINT64_MAX) { rc = ORC_ENOMEM; goto done; }
        info->round_cov[info->rounds] = cov1;
        info->round_cov2[info->rounds] = cov2;
        info->rounds = i;
        double scale = (double)n / (double)target;
        double su = sqrt((double)cov1 / g_k + a / 2.0) + sqrt(a / 2.0);
        double up = su * su * scale;
        double sl = sqrt((double)cov2 + 2.0 * a / 9.0) - sqrt(a / 2.0);
        double lo = sl > 0.0 ? (sl * sl - a / 18.0) * scale : 0.0;
        if (lo < 0.0) lo = 0.0;
        info->theta = target;
        info->lb = lo;
        info->sigma_up = up;
        info->alpha = lo / up;
        info->covered = cov1;
        if (lo / up >= one_m - eps) break;
    }
done:
    if (!keep) oracle_pool_destroy(r1);
    oracle_pool_destroy(r2);
    return rc;
}

/* IMM (Algorithm 1): sampling-phase rounds i = 1..i_max with the early break
 * of Tang et al.'s Algorithm 3, then theta = ceil(lambda_star / LB), top-up, and
 * the final selection over every generated set (reading R6). schedule
 * ORC_SCHED_FRESH instead draws the final selection's theta sets afresh, the
 * sample ids after those of the rounds (the correction of IMM's reuse of the
 * rounds' sets pointed out by Chen, 2018); ORC_SCHED_EARLY runs the early
 * stopping schedule above. keep (may be NULL) receives the pool of the final
 * selection. */
int oracle_imm_ex(uint32_t n, const uint64_t* col_off, const uint32_t* row_src,
                  const uint32_t* weight, int model, uint32_t k, double eps, double ell,
                  uint64_t seed, int threads, int schedule, oracle_pool* keep, uint32_t* seeds,
                  uint64_t* gains, oracle_imm_info* info) {
    if (schedule == ORC_SCHED_EARLY)
        return oracle_early(n, col_off, row_src, weight, model, k, eps, ell, seed, threads, keep,
                            seeds, gains, info);
    if (schedule != ORC_SCHED_IMM && schedule != ORC_SCHED_FRESH) return ORC_EINVAL;
    double lam_p, lam_s;
    uint32_t i_max;
    int rc = oracle_theta_plan(n, k, eps, ell, &lam_p, &lam_s, &i_max);
    if (rc) return rc;
    const int fresh = schedule == ORC_SCHED_FRESH;
    oracle_pool* pool = keep && !fresh ? keep : oracle_pool_create();
    if (!pool) return ORC_ENOMEM;
    memset(info, 0, sizeof(*info));
    info->lambda_prime = lam_p;
    info->lambda_star = lam_s;
    info->i_max = i_max;
    double eps_p = sqrt(2.0) * eps;
    double lb = 1.0;
    uint32_t* tmp_seeds = (uint32_t*)malloc((size_t)k * sizeof(uint32_t));
    uint64_t* tmp_gains = (uint64_t*)malloc((size_t)k * sizeof(uint64_t));
    if (!tmp_seeds || !tmp_gains) { rc = ORC_ENOMEM; goto done; }
    for (uint32_t i = 1; i <= i_max; ++i) {
        double x = ldexp((double)n, -(int)i);
        double tf = ceil(lam_p / x);
        if (!(tf < 4294967296.0)) { rc = ORC_EOVERFLOW; goto done; }
        uint64_t target = (uint64_t)tf;
        if (info->n_targets < 63) info->targets[info->n_targets++] = target;
        rc = oracle_pool_extend(pool, n, col_off, row_src, weight, model, seed, target, threads);
        if (rc) goto done;
        uint64_t cov = oracle_greedy(n, pool->set_off, pool->set_vtx, pool->n_sets, k,
                                     tmp_seeds, tmp_gains);
        if (cov == UINT64_MAX) { rc = ORC_ENOMEM; goto done; }
        info->round_cov[info->rounds] = cov;
        info->rounds = i;
        double frac = (double)cov / (double)pool->n_sets;
        if ((double)n * frac >= (1.0 + eps_p) * x) {
            lb = (double)n * frac / (1.0 + eps_p);
            break;
        }
    }
    {
        double tf = ceil(lam_s / lb);
        if (!(tf < 4294967296.0)) { rc = ORC_EOVERFLOW; goto done; }
        uint64_t theta = (uint64_t)tf;
        if (info->n_targets < 64) info->targets[info->n_targets++] = theta;
        oracle_pool* fin = pool;
        if (fresh) {
            /* theta new sets: sample ids after the rounds' ids */
            fin = keep ? keep : oracle_pool_create();
            if (!fin) { rc = ORC_ENOMEM; goto done; }
            fin->id_base = pool->n_sets;
        }
        if (fin->n_sets < theta) {
            rc = oracle_pool_extend(fin, n, col_off, row_src, weight, model, seed, theta, threads);
        }
        uint64_t cov = rc ? UINT64_MAX
                          : oracle_greedy(n, fin->set_off, fin->set_vtx, fin->n_sets, k, seeds,
                                          gains);
        if (!rc && cov == UINT64_MAX) rc = ORC_ENOMEM;
        if (!rc) {
            info->theta = fin->n_sets;
            info->lb = lb;
            info->covered = cov;
        }
        if (fin != pool && !keep) oracle_pool_destroy(fin);
    }
done:
    free(tmp_seeds);
    free(tmp_gains);
    if (pool != keep) oracle_pool_destroy(pool);
    return rc;
}

int oracle_imm(uint32_t n, const uint64_t* col_off, const uint32_t* row_src,
               const uint32_t* weight, int model, uint32_t k, double eps, double ell,
               uint64_t seed, int threads, oracle_pool* keep, uint32_t* seeds, uint64_t* gains,
               oracle_imm_info* info) {
    return oracle_imm_ex(n, col_off, row_src, weight, model, k, eps, ell, seed, threads,
                         ORC_SCHED_IMM, keep, seeds, gains, info);
}

/* The early-stopping schedule's constants: theta_0, i_max and a. */
int oracle_early_plan(uint32_t n, uint32_t k, double eps, double ell, double* theta0,
                      uint32_t* i_max, double* a) {
    return early_plan(n, k, eps, ell, theta0, i_max, a);
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
