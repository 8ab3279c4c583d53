// api.cpp -- the C ABI of libimm (include/imm.h) over the engine: graph
// upload and validation, single and batched IMM runs, the test-granular
// sampling/greedy/Philox entry points, and result accessors. No exception
// crosses this boundary.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cstring>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "engine.hpp"

using namespace imm;

struct imm_pool {
    std::unique_ptr<Workspace> ws;
    imm_stats stats{};
};

extern "C" {

const char* imm_last_error(void) { return last_error(); }

imm_status imm_theta_plan(uint32_t n, uint32_t k, double eps, double ell, double* lambda_prime,
                          double* lambda_star, uint32_t* i_max) {
    if (!lambda_prime || !lambda_star || !i_max) return fail(IMM_EINVAL, "theta_plan: null output");
    return theta_plan(n, k, eps, ell, lambda_prime, lambda_star, i_max);
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
        // launch shapes forced from the environment (else autotuned)
        const char* et = std::getenv("IMM_IC_TEAM");
        const char* eb = std::getenv("IMM_IC_BIG");
        const int team = et ? std::atoi(et) : 0;
        const int big = eb ? std::atoi(eb) : 0;
        if (team == 1 || team == 2 || team == 4) g->ic_team = (uint32_t)team;
        const bool big_ok = big == 256 || big == 1024;
        if (big_ok) g->ic_big_block = (uint32_t)big;
        g->team_forced = team == 1 || team == 2 || team == 4;
        g->big_forced = big_ok;
        const char* el = std::getenv("IMM_LT_BLOOM");
        const int bloom = el ? std::atoi(el) : 0;
        if (bloom >= 10 && bloom <= 12) g->lt_bloom_bits = (uint32_t)bloom;
        g->bloom_forced = bloom >= 10 && bloom <= 12;
        const char* ew = std::getenv("IMM_LT_LANES");
        const int lanes = ew ? std::atoi(ew) : 0;
        g->lanes_forced = lanes == 1 || lanes == 2 || lanes == 4;
        if (g->lanes_forced) g->lt_lanes = (uint32_t)lanes;
        g->tuned = model == IMM_IC ? (g->team_forced && g->big_forced)
                                   : (g->bloom_forced && g->lanes_forced);
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
            std::vector<uint4> cs(m ? m : 1);
            for (uint64_t e = 0; e < m; ++e) {
                const uint32_t u = rs[e];
                cs[e] = make_uint4(wt[e], u, off32[u], off32[(size_t)u + 1]);
            }
            IMM_TRY(g->arena.alloc((void**)&g->cs, (m ? m : 1) * 16, "edge records"));
            IMM_TRY(g->arena.alloc((void**)&g->guide, (m ? m : 1) * 4, "guide table"));
            IMM_TRY(g->arena.alloc((void**)&g->gw, (m ? m : 1) * 16 * kLtWindow,
                                   "guide windows"));
            if (m) HIP_TRY(hipMemcpyAsync(g->cs, cs.data(), m * 16, hipMemcpyHostToDevice, st));
            HIP_TRY(launch_lt_guide(g->off, g->cs, g->guide, g->gw, n, st));
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

imm_status imm_run(const imm_graph* g, const imm_params* p, void* stream, imm_result** out) {
    if (!g || !p || !out) return fail(IMM_EINVAL, "run: null argument");
    if (p->k == 0 || p->k > g->n) return fail(IMM_EINVAL, "run: need 1 <= k <= n");
    if (!(p->epsilon > 0.0) || !(p->ell > 0.0)) return fail(IMM_EINVAL, "run: need eps > 0, ell > 0");
    try {
        if (hipSetDevice(g->device) != hipSuccess) return fail(IMM_EDEVICE, "run: hipSetDevice failed");
        imm_graph* gg = const_cast<imm_graph*>(g);
        hipStream_t st = (hipStream_t)stream;
        imm_result* r = nullptr;
        imm_status s = IMM_OK;
        std::string err;
        run_queries(&gg, p, 1, st, &st, &r, &s, &err);
        if (s != IMM_OK) return fail(s, err);
        *out = r;
        return IMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(IMM_ENOMEM, "run: host allocation failed");
    } catch (...) {
        return fail(IMM_EDEVICE, "run: unexpected exception");
    }
}

imm_status imm_run_batch(const imm_graph* const* graphs, const imm_params* params, uint32_t count,
                         void* stream, imm_result** out) {
    if (!graphs || !params || !out || count == 0) return fail(IMM_EINVAL, "run_batch: bad arguments");
    for (uint32_t j = 0; j < count; ++j) {
        out[j] = nullptr;
        if (!graphs[j]) return fail(IMM_EINVAL, "run_batch: null graph");
        if (graphs[j]->device != graphs[0]->device)
            return fail(IMM_EINVAL, "run_batch: graphs on different devices");
    }
    try {
        if (hipSetDevice(graphs[0]->device) != hipSuccess)
            return fail(IMM_EDEVICE, "run_batch: hipSetDevice failed");
        hipStream_t main = (hipStream_t)stream;
        // sampling streams (default priority), ordered after the caller's work
        const uint32_t ns = std::min<uint32_t>(count, 8);
        std::vector<hipStream_t> own(ns, nullptr);
        hipEvent_t ready = nullptr;
        if (hipEventCreateWithFlags(&ready, hipEventDisableTiming) != hipSuccess ||
            hipEventRecord(ready, main) != hipSuccess)
            return fail(IMM_EDEVICE, "run_batch: event setup failed");
        for (uint32_t i = 0; i < ns; ++i) {
            if (hipStreamCreateWithFlags(&own[i], hipStreamNonBlocking) != hipSuccess ||
                hipStreamWaitEvent(own[i], ready, 0) != hipSuccess) {
                for (auto s : own)
                    if (s) (void)hipStreamDestroy(s);
                (void)hipEventDestroy(ready);
                return fail(IMM_EDEVICE, "run_batch: stream setup failed");
            }
        }
        std::vector<hipStream_t> per(count);
        std::vector<imm_graph*> gs(count);
        for (uint32_t j = 0; j < count; ++j) {
            per[j] = own[j % ns];
            gs[j] = const_cast<imm_graph*>(graphs[j]);
        }
        std::vector<imm_status> st(count, IMM_OK);
        std::vector<std::string> errs(count);
        run_queries(gs.data(), params, count, main, per.data(), out, st.data(), errs.data());
        (void)hipDeviceSynchronize();
        for (auto s : own) (void)hipStreamDestroy(s);
        (void)hipEventDestroy(ready);
        for (uint32_t j = 0; j < count; ++j) {
            if (st[j] == IMM_OK) continue;
            for (uint32_t i = 0; i < count; ++i) {
                delete out[i];
                out[i] = nullptr;
            }
            return fail(st[j], "run_batch: query " + std::to_string(j) + ": " + errs[j]);
        }
        return IMM_OK;
    } catch (const std::bad_alloc&) {
        return fail(IMM_ENOMEM, "run_batch: host allocation failed");
    } catch (...) {
        return fail(IMM_EDEVICE, "run_batch: unexpected exception");
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
    if (round_cov)
        std::memcpy(round_cov, r->round_cov.data(), std::min<size_t>(r->round_cov.size(), 64) * 8);
    return IMM_OK;
}

imm_status imm_result_pool(const imm_result* r, uint64_t* n_sets, uint64_t* n_entries,
                           uint64_t* set_off, uint32_t* set_vtx) {
    if (!r) return fail(IMM_EINVAL, "result_pool: null result");
    if (!r->has_pool) return fail(IMM_EINVAL, "result_pool: run without IMM_KEEP_POOL");
    if (n_sets) *n_sets = r->set_off.size() - 1;
    if (n_entries) *n_entries = r->set_vtx.size();
    if (set_off) std::memcpy(set_off, r->set_off.data(), r->set_off.size() * 8);
    if (set_vtx && !r->set_vtx.empty())
        std::memcpy(set_vtx, r->set_vtx.data(), r->set_vtx.size() * 4);
    return IMM_OK;
}

imm_status imm_result_early(const imm_result* r, double* sigma_up, double* alpha,
                            uint64_t* round_cov2) {
    if (!r) return fail(IMM_EINVAL, "result_early: null result");
    if (sigma_up) *sigma_up = r->sigma_up;
    if (alpha) *alpha = r->alpha;
    if (round_cov2 && !r->round_cov2.empty())
        std::memcpy(round_cov2, r->round_cov2.data(),
                    std::min<size_t>(r->round_cov2.size(), 64) * 8);
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
        IMM_TRY(tune_graph(const_cast<imm_graph*>(g), st));
        std::unique_ptr<imm_pool> p(new imm_pool());
        p->ws.reset(new Workspace());
        IMM_TRY(ws_init(*p->ws, g->n, g->device, st, 0));
        IMM_TRY(ws_reset(*p->ws, st, (flags & IMM_TIMING) != 0));
        p->ws->list_only = (flags & IMM_LIST_SETS) != 0;
        IMM_TRY(ws_extend(*p->ws, g, seed, first_id, count));
        IMM_TRY(ws_sync_pool(*p->ws));
        ws_note_pool(*p->ws, 0);
        IMM_TRY(ws_read_scalars(*p->ws));
        p->stats.ms_total = now_ms() - t0;
        fill_stats(*p->ws, &p->stats);
        p->stats.team = g->model == IMM_IC ? g->ic_team : 0;
        p->stats.big_block = g->model == IMM_IC ? g->ic_big_block : 0;
        p->stats.bloom_bits = g->model == IMM_LT ? g->lt_bloom_bits : 0;
        p->stats.walk_lanes = g->model == IMM_LT ? g->lt_lanes : 0;
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
    // list members plus the members of the sets kept as bitmaps
    if (n_entries) *n_entries = p->ws->p_exact + p->ws->dense_entries;
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
        IMM_TRY(ws_select(w, k, n_sets, &cov));
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
