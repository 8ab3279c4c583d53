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
// is made by timing, at a steady-state batch size (smaller batches favour
// the wider teams, which the full-size passes do not): one fixed batch of
// sample ids is drawn with each candidate, the team first (with the 256-thread
// giant-set shape) and then the giant-set shape with that team, and the
// fastest BFS plus giant-set kernel time wins. A pass
// that will defer many more giant sets than the wide shape has workgroups
// uses the 256-thread shape regardless (see sample_pass). Every set is a pure
// function of (graph, seed, sample id), so the choice never changes a result.
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <vector>

#include "engine.hpp"

namespace imm {

namespace {

constexpr uint64_t kTuneSeed = 0x7475E5EEDull;
// The IC batch is sized to about kTuneEntries set members (from the probe's
// mean set size), between 2^14 and 2^20 samples.
constexpr uint64_t kTuneSamples = 1u << 20;
constexpr uint64_t kTuneEntries = 16u << 20;
// The LT batch is sized to about kTuneLtSteps walk steps (from a probe of
// kLtProbeSamples walks), between 2^16 and 2^21 walks: a batch with fewer
// walks than the kernel has walk slots times only its longest walk.
constexpr uint64_t kLtProbeSamples = 1u << 14;
constexpr uint64_t kTuneLtSteps = 1ull << 28;
constexpr int kTuneReps = 2;  // each candidate is timed this often; the minimum counts
// A probe of kProbeSamples with the wide shapes comes first; a graph whose
// probe takes longer than kProbeMs (very deep or very large sets) keeps the
// wide shapes without the full search, which would cost seconds.
constexpr uint64_t kProbeSamples = 2048;
constexpr double kProbeMs = 20.0;

// LT: the lanes per walk (2 or 4) and the per-walk path filter size (1024,
// 2048 or 4096 bits), each unless forced. A probe with 4 lanes and 4096 bits
// comes first; a graph whose probe takes longer than kProbeMs (very long
// walks) keeps that shape.
imm_status tune_lt(imm_graph* g, hipStream_t st) {
    if (g->bloom_forced && g->lanes_forced) {
        g->tuned = true;
        return IMM_OK;
    }
    Workspace w;
    IMM_TRY(ws_init(w, g->n, g->device, st, 0));
    const bool log = std::getenv("IMM_TUNE_LOG") != nullptr;
    if (!g->lanes_forced) g->lt_lanes = 4;
    if (!g->bloom_forced) g->lt_bloom_bits = 12;
    uint64_t batch = 0;
    {
        IMM_TRY(ws_reset(w, st, true));
        IMM_TRY(ws_extend(w, g, kTuneSeed, 0, kLtProbeSamples));
        HIP_TRY(hipStreamSynchronize(st));
        imm_stats s;
        std::memset(&s, 0, sizeof(s));
        fill_stats(w, &s);
        const double probe_ms = s.ms_sample_main + s.ms_sample_big;
        const double steps = (double)s.edges / (double)kLtProbeSamples;
        if (s.sets) g->mean_set_hint = (double)s.entries / (double)s.sets;
        if (log)
            std::fprintf(stderr, "imm tune: n=%u m=%llu LT probe %.3f ms, %.1f steps per walk\n",
                         g->n, (unsigned long long)g->m, probe_ms, steps);
        if (probe_ms > kProbeMs) {
            g->tuned = true;
            return IMM_OK;
        }
        const double want = (double)kTuneLtSteps / (steps > 1.0 ? steps : 1.0);
        batch = (uint64_t)std::min(std::max(want, (double)(1u << 16)), (double)(1u << 21));
    }
    std::vector<uint32_t> lane_opts, bit_opts;
    if (g->lanes_forced) lane_opts = {g->lt_lanes}; else lane_opts = {4u, 2u};
    if (g->bloom_forced) bit_opts = {g->lt_bloom_bits}; else bit_opts = {12u, 11u, 10u};
    double best = -1.0;
    uint32_t pick_bits = bit_opts[0], pick_lanes = lane_opts[0];
    // the first candidate runs once untimed (first launches of the kernels)
    bool warm = false;
    for (uint32_t lanes : lane_opts) {
        for (uint32_t bits : bit_opts) {
            g->lt_lanes = lanes;
            g->lt_bloom_bits = bits;
            double ms = -1.0;
            imm_stats s;
            for (int rep = warm ? 0 : -1; rep < kTuneReps; ++rep) {
                IMM_TRY(ws_reset(w, st, true));
                IMM_TRY(ws_extend(w, g, kTuneSeed, 0, batch));
                HIP_TRY(hipStreamSynchronize(st));
                std::memset(&s, 0, sizeof(s));
                fill_stats(w, &s);
                const double t = s.ms_sample_main + s.ms_sample_big;
                if (rep >= 0 && (ms < 0.0 || t < ms)) ms = t;
                if (s.sets) g->mean_set_hint = (double)s.entries / (double)s.sets;
            }
            warm = true;
            if (log)
                std::fprintf(stderr,
                             "imm tune: n=%u m=%llu LT %u lanes per walk, filter 2^%u bits, %llu "
                             "walks: %.3f ms, long %.3f ms\n",
                             g->n, (unsigned long long)g->m, lanes, bits,
                             (unsigned long long)batch, s.ms_sample_main, s.ms_sample_big);
            if (best < 0.0 || ms < best) {
                best = ms;
                pick_bits = bits;
                pick_lanes = lanes;
            }
        }
    }
    g->lt_bloom_bits = pick_bits;
    g->lt_lanes = pick_lanes;
    g->tuned = true;
    return IMM_OK;
}

}  // namespace

imm_status tune_graph(imm_graph* g, hipStream_t st) {
    std::lock_guard<std::mutex> lk(g->tune_mu);
    if (g->tuned) return IMM_OK;
    if (g->model == IMM_LT) return tune_lt(g, st);
    Workspace w;
    IMM_TRY(ws_init(w, g->n, g->device, st, 0));
    const bool log = std::getenv("IMM_TUNE_LOG") != nullptr;
    uint64_t batch = kTuneSamples;
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
        if (s.sets) g->mean_set_hint = (double)s.entries / (double)s.sets;
        g->dense_rate = (double)w.n_dense / (double)kProbeSamples;
        g->over_rate = (double)w.hsc->over_n / (double)kProbeSamples;
        if (log)
            std::fprintf(stderr, "imm tune: n=%u probe %.3f ms, %u sets outgrew their queue\n",
                         g->n, ms, w.hsc->over_n);
        if (ms > kProbeMs) {
            if (!g->big_forced) g->ic_big_block = 1024;
            g->tuned = true;
            return IMM_OK;
        }
        const double per_set = (double)s.entries / (double)kProbeSamples;
        const double want = per_set > 0.0 ? (double)kTuneEntries / per_set : (double)kTuneSamples;
        batch = want >= (double)kTuneSamples ? kTuneSamples
                                             : (want <= 16384.0 ? 16384u : (uint64_t)want);
    }
    // one batch drawn with the shapes set on g; the fastest of kTuneReps
    // timings of the BFS plus giant-set kernels
    auto time_batch = [&](double* ms_out, double* defer_rate) -> imm_status {
        double ms = -1.0;
        for (int rep = 0; rep < kTuneReps; ++rep) {
            IMM_TRY(ws_reset(w, st, true));
            IMM_TRY(ws_extend(w, g, kTuneSeed, 0, batch));
            HIP_TRY(hipStreamSynchronize(st));
            imm_stats s;
            std::memset(&s, 0, sizeof(s));
            fill_stats(w, &s);
            const double t = s.ms_sample_main + s.ms_sample_big;
            if (ms < 0.0 || t < ms) ms = t;
            *defer_rate = (double)s.deferred / (double)batch;
            g->dense_rate = (double)w.n_dense / (double)batch;
            if (s.sets) g->mean_set_hint = (double)s.entries / (double)s.sets;
        }
        if (log)
            std::fprintf(stderr, "imm tune: n=%u m=%llu batch=%llu team=%u big=%u: %.3f ms\n",
                         g->n, (unsigned long long)g->m, (unsigned long long)batch, g->ic_team,
                         g->ic_big_block, ms);
        *ms_out = ms;
        return IMM_OK;
    };
    // the first pass allocates the workspace (with the most giant-set slots
    // any shape uses) and is not timed
    const uint32_t big0 = g->ic_big_block;
    if (!g->big_forced) g->ic_big_block = 256;
    IMM_TRY(ws_reset(w, st, true));
    IMM_TRY(ws_extend(w, g, kTuneSeed, 0, batch));
    HIP_TRY(hipStreamSynchronize(st));
    if (g->big_forced) g->ic_big_block = big0;
    // the BFS team first (with the 256-thread giant-set shape), then the
    // giant-set shape with that team
    double best = -1.0, rate = 0.0, pick_rate = 0.0;
    if (!g->team_forced) {
        uint32_t pick = 4;
        for (uint32_t team : {1u, 2u, 4u}) {
            g->ic_team = team;
            double ms = 0.0;
            IMM_TRY(time_batch(&ms, &rate));
            if (best < 0.0 || ms < best) {
                best = ms;
                pick = team;
                pick_rate = rate;
            }
        }
        g->ic_team = pick;
    }
    if (!g->big_forced) {
        uint32_t pick = 256;
        best = -1.0;
        for (uint32_t big : {256u, 1024u}) {
            g->ic_big_block = big;
            double ms = 0.0;
            IMM_TRY(time_batch(&ms, &rate));
            if (best < 0.0 || ms < best) {
                best = ms;
                pick = big;
                pick_rate = rate;
            }
        }
        g->ic_big_block = pick;
    } else if (g->team_forced) {
        double ms = 0.0;
        IMM_TRY(time_batch(&ms, &pick_rate));
    }
    g->defer_rate = pick_rate;
    g->tuned = true;
    return IMM_OK;
}

}  // namespace imm
