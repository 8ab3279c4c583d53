// tune.cpp -- per-graph choice of the sampling launch shapes.
//
// LT: the size of each walk's path filter in LDS (1024, 2048 or 4096 bits):
// smaller filters leave more waves, hence more walks, in flight, at the cost
// of more false hits that a path rescan must clear.
//
// IC: two shapes matter and depend on the graph: the BFS team (waves per sample:
// one wave suits graphs whose sets are small and cheap; samples that sweep
// long in-edge lists of high in-degree hubs finish sooner, and fit LDS more
// often, with two or four) and the giant-set workgroup (256 threads and many
// sets in flight, or 1024 threads for fewer, wider BFS levels). The choice
// is made by timing: one fixed batch of sample ids is drawn with every
// candidate and the fastest BFS plus giant-set kernel time wins. A pass
// that will defer many more giant sets than the wide shape has workgroups
// uses the 256-thread shape regardless (see sample_pass). Every set is a pure
// function of (graph, seed, sample id), so the choice never changes a result.
#include <cstdio>
#include <cstdlib>
#include <cstring>

#include "engine.hpp"

namespace imm {

namespace {

constexpr uint64_t kTuneSeed = 0x7475E5EEDull;
constexpr uint64_t kTuneSamples = 1u << 16;
// A probe of kProbeSamples with the wide shapes comes first; a graph whose
// probe takes longer than kProbeMs (very deep or very large sets) keeps the
// wide shapes without the full search, which would cost seconds.
constexpr uint64_t kProbeSamples = 2048;
constexpr double kProbeMs = 20.0;

// LT: the per-lane path filter size, among 1024, 2048 and 4096 bits.
imm_status tune_lt(imm_graph* g, hipStream_t st) {
    if (g->bloom_forced) {
        g->tuned = true;
        return IMM_OK;
    }
    Workspace w;
    IMM_TRY(ws_init(w, g->n, g->device, st, 0));
    const bool log = std::getenv("IMM_TUNE_LOG") != nullptr;
    double best = -1.0;
    uint32_t pick = 12;
    for (int c = -1; c < 3; ++c) {
        g->lt_bloom_bits = c < 0 ? 10u : 12u - (uint32_t)c;
        IMM_TRY(ws_reset(w, st, true));
        IMM_TRY(ws_extend(w, g, kTuneSeed, 0, kTuneSamples));
        HIP_TRY(hipStreamSynchronize(st));
        imm_stats s;
        std::memset(&s, 0, sizeof(s));
        fill_stats(w, &s);
        if (c < 0) continue;
        const double ms = s.ms_sample_main + s.ms_sample_big;
        if (log)
            std::fprintf(stderr, "imm tune: n=%u m=%llu LT filter 2^%u bits: walks %.3f ms, long %.3f ms\n",
                         g->n, (unsigned long long)g->m, g->lt_bloom_bits, s.ms_sample_main,
                         s.ms_sample_big);
        if (best < 0.0 || ms < best) {
            best = ms;
            pick = g->lt_bloom_bits;
        }
    }
    g->lt_bloom_bits = pick;
    g->tuned = true;
    return IMM_OK;
}

}  // namespace

imm_status tune_graph(imm_graph* g, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g->tune_mu);
    if (g->tuned) return IMM_OK;
    if (g->model == IMM_LT) return tune_lt(g, st);
    struct Cand {
        uint32_t team, big;
    };
    Cand cands[6];
    int nc = 0;
    for (uint32_t team : {1u, 2u, 4u}) {
        if (g->team_forced && team != g->ic_team) continue;
        for (uint32_t big : {256u, 1024u}) {
            if (g->big_forced && big != g->ic_big_block) continue;
            cands[nc++] = Cand{team, big};
        }
    }
    Workspace w;
    IMM_TRY(ws_init(w, g->n, g->device, st, 0));
    const bool log = std::getenv("IMM_TUNE_LOG") != nullptr;
    {
        if (!g->team_forced) g->ic_team = 4;
        if (!g->big_forced) g->ic_big_block = 256;  // allocates the most slots
        IMM_TRY(ws_reset(w, st, true));
        IMM_TRY(ws_extend(w, g, kTuneSeed, 0, kProbeSamples));
        HIP_TRY(hipStreamSynchronize(st));
        imm_stats s;
        std::memset(&s, 0, sizeof(s));
        fill_stats(w, &s);
        const double ms = s.ms_sample;
        if (log) std::fprintf(stderr, "imm tune: n=%u probe %.3f ms\n", g->n, ms);
        if (ms > kProbeMs) {
            if (!g->big_forced) g->ic_big_block = 1024;
            g->tuned = true;
            return IMM_OK;
        }
    }
    double best = -1.0, pick_rate = 0.0;
    Cand pick = cands[0];
    // the first pass allocates the workspace (with the most giant-set slots
    // any candidate uses) and is not timed
    const uint32_t big0 = g->ic_big_block;
    for (int c = -1; c < nc; ++c) {
        g->ic_team = c < 0 ? cands[0].team : cands[c].team;
        g->ic_big_block = c < 0 ? (g->big_forced ? big0 : 256u) : cands[c].big;
        IMM_TRY(ws_reset(w, st, true));
        IMM_TRY(ws_extend(w, g, kTuneSeed, 0, kTuneSamples));
        HIP_TRY(hipStreamSynchronize(st));
        imm_stats s;
        std::memset(&s, 0, sizeof(s));
        fill_stats(w, &s);
        if (c < 0) continue;
        const double ms = s.ms_sample_main + s.ms_sample_big;
        if (log)
            std::fprintf(stderr, "imm tune: n=%u m=%llu team=%u big=%u: bfs %.3f ms, giant %.3f ms\n",
                         g->n, (unsigned long long)g->m, g->ic_team, g->ic_big_block,
                         s.ms_sample_main, s.ms_sample_big);
        if (best < 0.0 || ms < best) {
            best = ms;
            pick = cands[c];
            pick_rate = (double)s.deferred / (double)kTuneSamples;
        }
    }
    g->ic_team = pick.team;
    g->ic_big_block = pick.big;
    g->defer_rate = pick_rate;
    g->tuned = true;
    return IMM_OK;
}

}  // namespace imm
