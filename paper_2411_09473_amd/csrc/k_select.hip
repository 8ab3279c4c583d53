// k_select.hip -- greedy max-coverage seed selection (Find_Most_Influential_Set,
// Algorithm 2) over device-resident pools, for one or many IMM instances.
//
// Seed step t of every instance in a batch costs three launches and no host
// round trip; each launch covers all instances, its workgroups split among
// them by a per-instance block range (SelectDesc):
//  * argmax: the two-step reduction of the paper's PARALLEL_REDUCTION. Each
//    workgroup reduces its part of the counts (regional maximum) and folds it
//    into one of kArgSlots partial slots with a 64-bit atomic max; the next
//    kernel reduces the slots (global maximum). A vertex is the packed key
//    count<<32 | ~id, so a plain max picks the largest count and, among equal
//    counts, the lowest id. A chosen vertex's count becomes a sentinel that
//    maps to key 0, which keeps it out of later picks.
//  * claim: the chosen vertex's inverted-index lists (one per index segment)
//    name exactly the sets that contain it ("if v in R" of Algorithm 2
//    without scanning all sets); each one not yet covered is claimed with an
//    atomic bit and queued: a small set as one entry, a larger one cut into
//    pieces of at most 64 members.
//  * decrement: the instance's threads take small sets one per lane and
//    pieces one per wave, and decrement the counts of the members (except
//    the chosen vertex), so both a flood of tiny sets and a few very large
//    ones spread over the GPU. When the queue is long, decrements are summed
//    per workgroup in LDS first. When the covered sets hold more than a
//    quarter of the pool, the step instead recounts every remaining count
//    from the uncovered sets (the paper's adaptive counter update, Section
//    IV-C), a gather without atomics. A descriptor can also fix the choice
//    (decrement always, or recount always) for measurement; every choice
//    gives the same counts.
#include <algorithm>

#include "device_common.hpp"
#include "imm_internal.hpp"

namespace imm {

namespace {

constexpr uint32_t kArgBS = 256;
constexpr uint32_t kArgLoads = 4;
constexpr uint32_t kClaimBS = 256;
constexpr uint32_t kDecBS = 256;

#define IMM_GLOBAL __attribute__((address_space(1)))

// A seed-step descriptor as the kernels use it: a register copy whose
// pointers are typed as global memory. Accesses through pointers loaded from
// memory would otherwise compile to flat instructions, which also count
// against the LDS wait counter, so every LDS wait in a loop would drain the
// loop's outstanding global loads as well.
struct SelView {
    IMM_GLOBAL uint32_t* cw;
    const IMM_GLOBAL uint32_t* cacc;
    const IMM_GLOBAL uint32_t* heavy;
    const IMM_GLOBAL uint32_t* n_heavy;
    const IMM_GLOBAL uint64_t* inv_offs;
    const IMM_GLOBAL uint32_t* inv_set;
    const IMM_GLOBAL uint64_t* set_off;
    const IMM_GLOBAL uint32_t* set_vtx;
    IMM_GLOBAL uint32_t* covered;
    IMM_GLOBAL unsigned long long* slots;
    IMM_GLOBAL uint32_t* seeds;
    IMM_GLOBAL uint32_t* gains;
    IMM_GLOBAL Chunk* chunks;
    IMM_GLOBAL uint32_t* chunk_n;
    uint64_t chunk_cap;
    IMM_GLOBAL unsigned long long* cov_entries;
    uint32_t n, k, nseg, n_sets;
    uint32_t arg_lo, arg_cnt, sel_lo, sel_cnt;
    uint32_t update;
    const IMM_GLOBAL uint32_t* dense_bits;
    const IMM_GLOBAL uint32_t* dense_sid;
    const IMM_GLOBAL uint32_t* dense_size;
    IMM_GLOBAL uint32_t* dense_list;
    IMM_GLOBAL uint32_t* dense_list_n;
    IMM_GLOBAL uint32_t* dense_mark;
    uint64_t dense_entries;
    uint32_t n_dense, dense_words;
    const IMM_GLOBAL uint32_t* cand;
    const IMM_GLOBAL uint32_t* cand_bits;
    IMM_GLOBAL uint32_t* cand_state;
};

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// 16-byte records through global pointers (one dwordx4 access each).
__device__ __forceinline__ uint4 load_u4(const IMM_GLOBAL uint4* p) {
    const u32x4 v = *(const IMM_GLOBAL u32x4*)p;
    return make_uint4(v.x, v.y, v.z, v.w);
}
__device__ __forceinline__ Chunk load_chunk(const IMM_GLOBAL Chunk* p) {
    const u32x4 v = *(const IMM_GLOBAL u32x4*)p;
    return Chunk{(uint64_t)v.x | ((uint64_t)v.y << 32), v.z, v.w};
}
__device__ __forceinline__ void store_chunk(IMM_GLOBAL Chunk* p, uint64_t off, uint32_t len) {
    *(IMM_GLOBAL u32x4*)p = u32x4{(uint32_t)off, (uint32_t)(off >> 32), len, 0u};
}

template <class T>
__device__ __forceinline__ IMM_GLOBAL T* glb(T* p) {
    return (IMM_GLOBAL T*)p;
}

__device__ __forceinline__ SelView view_of(const SelectDesc& d) {
    return SelView{glb(d.cw),      glb(d.cacc),    glb(d.heavy),   glb(d.n_heavy),
                   glb(d.inv_offs), glb(d.inv_set), glb(d.set_off), glb(d.set_vtx),
                   glb(d.covered), glb(d.slots),   glb(d.seeds),   glb(d.gains),
                   glb(d.chunks),  glb(d.chunk_n), d.chunk_cap,    glb(d.cov_entries),
                   d.n,            d.k,            d.nseg,         d.n_sets,
                   d.arg_lo,       d.arg_cnt,      d.sel_lo,       d.sel_cnt,
                   d.update,       glb(d.dense_bits), glb(d.dense_sid), glb(d.dense_size),
                   glb(d.dense_list), glb(d.dense_list_n), glb(d.dense_mark), d.dense_entries,
                   d.n_dense,      d.dense_words, glb(d.cand), glb(d.cand_bits),
                   glb(d.cand_state)};
}

// Candidate steps (SelectDesc::cand). A step at or after the halting step
// does nothing; the host finishes the selection.
__device__ __forceinline__ bool step_halted(const SelView& d, uint32_t t) {
    if (!d.cand_state) return false;
    const uint32_t h = d.cand_state[1];
    return h != 0u && t >= h;
}
// The first four state words (mode, halting step, tau, list length) as one
// load; zeros without a list.
__device__ __forceinline__ uint4 cand_head(const SelView& d) {
    return d.cand_state ? load_u4(reinterpret_cast<const IMM_GLOBAL uint4*>(d.cand_state))
                        : make_uint4(0u, 0u, 0u, 0u);
}
// Whether step t >= 1 takes its argmax over the list and filters its
// decrements (decided by step 1's argmax).
__device__ __forceinline__ bool cand_step(const SelView& d, uint32_t t) {
    return d.cand_state && t >= 1 && d.cand_state[0] == 1u;
}

// The count histogram's bin of c and the smallest count of bin b.
__device__ __forceinline__ uint32_t cand_bin(uint32_t c) {
    if (c < 16u) return c;
    const uint32_t e = 31u - (uint32_t)__clz(c);
    return 16u + 8u * (e - 4u) + ((c >> (e - 3u)) & 7u);
}
__device__ __forceinline__ uint32_t cand_edge(uint32_t b) {
    if (b < 16u) return b;
    const uint32_t e = 4u + (b - 16u) / 8u, sub = (b - 16u) % 8u;
    return (8u + sub) << (e - 3u);
}
__device__ __forceinline__ bool is_cand(const SelView& d, uint32_t u) {
    return (d.cand_bits[u >> 5] >> (u & 31u)) & 1u;
}

// Device-scope relaxed atomics on global memory (what atomicAdd and friends do).
__device__ __forceinline__ uint32_t g_add(IMM_GLOBAL uint32_t* p, uint32_t x) {
    return __hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_sub(IMM_GLOBAL uint32_t* p, uint32_t x) {
    (void)__hip_atomic_fetch_sub(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t g_or(IMM_GLOBAL uint32_t* p, uint32_t x) {
    return __hip_atomic_fetch_or(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_add64(IMM_GLOBAL unsigned long long* p, unsigned long long x) {
    (void)__hip_atomic_fetch_add(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void g_max64(IMM_GLOBAL unsigned long long* p, unsigned long long x) {
    (void)__hip_atomic_fetch_max(p, x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t vkey(uint32_t c, uint32_t v) {
    return c == kSelected ? 0ull : (((uint64_t)c << 32) | (uint64_t)(~v));
}

// The instance whose block range [lo, lo + cnt) holds block b (ranges are
// ascending and disjoint); nq when none does.
// kind: 0 the claim and decrement launches, 1 argmax, 2 the dense update.
__device__ __forceinline__ uint32_t find_inst(const SelectDesc* d, uint32_t nq, uint32_t b,
                                              int kind) {
    auto lo_of = [&](uint32_t q) {
        return kind == 1 ? d[q].arg_lo : (kind == 2 ? d[q].dense_lo : d[q].sel_lo);
    };
    uint32_t lo = 0, hi = nq;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (lo_of(mid) <= b) lo = mid; else hi = mid;
    }
    const uint32_t l = lo_of(lo);
    const uint32_t c = kind == 1 ? d[lo].arg_cnt : (kind == 2 ? d[lo].dense_cnt : d[lo].sel_cnt);
    return (b >= l && b < l + c) ? lo : nq;
}

__global__ __launch_bounds__(kArgBS) void argmax_kernel(const SelectDesc* descs, uint32_t nq,
                                                        uint32_t t) {
    __shared__ uint64_t s_w[kArgBS / kWave];
    const uint32_t q = find_inst(descs, nq, blockIdx.x, 1);
    if (q == nq) return;
    const SelView d = view_of(descs[q]);
    if (t >= d.k) return;
    const IMM_GLOBAL uint32_t* cw = d.cw;
    const uint32_t n = d.n;
    const uint32_t blk = blockIdx.x - d.arg_lo;
    const uint32_t tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    if (d.cand_state && t >= 1) {
        // the state words and this workgroup's first list entries load
        // together (the list buffer holds kCandMax entries; the ones past the
        // list's length are not used)
        const uint32_t first = blk * kArgBS * 4u;
        uint32_t v0[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint32_t i = first + u * kArgBS + tid;
            v0[u] = d.cand[i < kCandMax ? i : kCandMax - 1];
        }
        const uint4 cs = cand_head(d);
        if (cs.y != 0u && t >= cs.y) return;  // halted
        bool use;
        if (t == 1) {
            // the list serves steps 1.. unless it is empty, the update is
            // fixed, or step 0 recounted (its seed covered much of the pool)
            const uint64_t pool = d.set_off[d.n_sets] + d.dense_entries;
            use = cs.w != 0u && d.update == kUpdateAdaptive && d.cov_entries[0] * 4ull <= pool;
            if (blk == 0 && tid == 0) d.cand_state[0] = use ? 1u : 2u;
        } else {
            use = cs.x == 1u;
        }
        if (use) {
            // the list's counts, four per thread per round, spread over the
            // instance's workgroups (a small graph has one)
            const uint32_t nc = cs.w;
            if (first >= nc) {
                if (blk == 0 && tid == 0 && d.n_dense) d.dense_mark[t] = *d.dense_list_n;
                return;
            }
            uint64_t best = 0;
            for (uint32_t base = first; base < nc; base += d.arg_cnt * kArgBS * 4u) {
                uint32_t v[4];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) {
                    const uint32_t i = base + u * kArgBS + tid;
                    // entries past the length repeat the last one (a repeated
                    // vertex changes no maximum)
                    v[u] = base == first && i < nc ? v0[u] : d.cand[i < nc ? i : nc - 1];
                }
                uint32_t c[4];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) c[u] = cw[v[u]];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) {
                    const uint64_t k = vkey(c[u], v[u]);
                    best = k > best ? k : best;
                }
            }
            best = wave_max64(best);
            if (lane == 0) s_w[w] = best;
            __syncthreads();
            if (tid == 0) {
                uint64_t b = s_w[0];
                for (uint32_t x = 1; x < kArgBS / kWave; ++x) b = s_w[x] > b ? s_w[x] : b;
                g_max64(&d.slots[(uint64_t)t * kArgSlots + blk % kArgSlots], (unsigned long long)b);
                if (blk == 0 && d.n_dense) d.dense_mark[t] = *d.dense_list_n;
            }
            return;
        }
    }
    const uint32_t gtid = blk * kArgBS + tid, gthreads = d.arg_cnt * kArgBS;
    uint64_t best = 0;
    const uint32_t n4 = n >> 2;
    const IMM_GLOBAL uint4* cw4 = (const IMM_GLOBAL uint4*)cw;
    // kArgLoads 16-byte loads in flight per thread: unguarded, at clamped
    // positions (a repeated group changes no maximum)
    for (uint32_t x0 = gtid; x0 < n4; x0 += kArgLoads * gthreads) {
        uint4 c[kArgLoads];
#pragma unroll
        for (uint32_t u = 0; u < kArgLoads; ++u) {
            const uint32_t x = x0 + u * gthreads;
            c[u] = load_u4(cw4 + (x < n4 ? x : x0));
        }
#pragma unroll
        for (uint32_t u = 0; u < kArgLoads; ++u) {
            const uint32_t x = x0 + u * gthreads;
            const uint32_t v = (x < n4 ? x : x0) << 2;
            uint64_t k = vkey(c[u].x, v);
            uint64_t y = vkey(c[u].y, v + 1); k = y > k ? y : k;
            y = vkey(c[u].z, v + 2); k = y > k ? y : k;
            y = vkey(c[u].w, v + 3); k = y > k ? y : k;
            best = k > best ? k : best;
        }
    }
    if (gtid < (n & 3u)) {
        const uint32_t v = (n4 << 2) + gtid;
        const uint64_t k = vkey(cw[v], v);
        best = k > best ? k : best;
    }
    best = wave_max64(best);
    if (lane == 0) s_w[w] = best;
    __syncthreads();
    if (tid == 0) {
        uint64_t b = s_w[0];
        for (uint32_t x = 1; x < kArgBS / kWave; ++x) b = s_w[x] > b ? s_w[x] : b;
        g_max64(&d.slots[(uint64_t)t * kArgSlots + blk % kArgSlots], (unsigned long long)b);
        // the dense claims of step t start where those of the earlier steps end
        if (blk == 0 && d.n_dense) d.dense_mark[t] = *d.dense_list_n;
    }
}

__device__ __forceinline__ uint64_t slots_max(const IMM_GLOBAL unsigned long long* slots) {
    uint64_t m = 0;
#pragma unroll
    for (uint32_t x = 0; x < kArgSlots; ++x) m = slots[x] > m ? slots[x] : m;
    return m;
}

__global__ __launch_bounds__(kClaimBS) void claim_kernel(const SelectDesc* descs, uint32_t nq,
                                                         uint32_t t) {
    const uint32_t q = find_inst(descs, nq, blockIdx.x, 0);
    if (q == nq) return;
    const SelView d = view_of(descs[q]);
    if (t >= d.k) return;
    const uint32_t blk = blockIdx.x - d.sel_lo;
    // the step's partial maxima and the state words load together
    const uint64_t m = slots_max(d.slots + (uint64_t)t * kArgSlots);
    const uint4 cs = cand_head(d);
    if (cs.y != 0u && t >= cs.y) return;  // halted
    if (t >= 1 && cs.x == 1u && (uint32_t)(m >> 32) < cs.z) {
        // no listed vertex reaches tau: an unlisted one might now be the
        // argmax, so the selection halts here (every workgroup agrees)
        if (blk == 0 && threadIdx.x == 0) d.cand_state[1] = t;
        return;
    }
    const uint32_t v = ~(uint32_t)m;
    if (blk == 0 && threadIdx.x == 0) {
        d.seeds[t] = v;
        d.gains[t] = (uint32_t)(m >> 32);
        d.cw[v] = kSelected;
    }
    IMM_GLOBAL uint32_t* small_n = d.chunk_n + 2ull * t;
    IMM_GLOBAL uint32_t* big_n = small_n + 1;
    const uint64_t step = (uint64_t)d.sel_cnt * kClaimBS;
    const uint32_t lane = threadIdx.x % kWave;
    const uint64_t lane_mask = (1ull << lane) - 1ull;
    // v's list bounds in every segment, loaded at once (lane s: segment s)
    uint64_t my_lb = 0, my_len = 0;
    if (lane < d.nseg) {
        const IMM_GLOBAL uint64_t* io = d.inv_offs + (uint64_t)lane * ((uint64_t)d.n + 1);
        my_lb = io[v];
        my_len = io[v + 1] - my_lb;
    }
    // the lists of all segments as one range [0, total): no per-segment
    // round trips
    const uint64_t my_end = wave_incl_scan64(my_len);
    const uint64_t total = __shfl(my_end, kWave - 1, kWave);
    uint64_t cov = 0;  // members of the sets this thread claimed
    {
        for (uint64_t base = (uint64_t)blk * kClaimBS; base < total; base += step) {
            const uint64_t i = base + threadIdx.x;
            bool small = false;
            uint32_t nbig = 0;
            uint64_t a = 0, sz = 0;
            // segment of position i: the first whose running end exceeds i
            uint64_t pos = 0;
            for (uint32_t seg = 0; seg < d.nseg; ++seg) {
                const uint64_t e = __shfl(my_end, seg, kWave);
                const uint64_t l = __shfl(my_len, seg, kWave);
                const uint64_t b = __shfl(my_lb, seg, kWave);
                if (i < e && i >= e - l) pos = b + (i - (e - l));
            }
            if (i < total) {
                const uint32_t j = d.inv_set[pos];
                const uint32_t bit = 1u << (j & 31);
                const uint32_t old = g_or(&d.covered[j >> 5], bit);
                // the set's bounds load beside the claim, not after it (the
                // claim selects them rather than guarding their loads)
                const uint64_t a0 = d.set_off[j], a1 = d.set_off[j + 1];
                const bool claimed = !(old & bit);
                a = claimed ? a0 : 0;
                sz = claimed ? a1 - a0 : 0;
                cov += sz;
                // a set of one member is {v} itself: nothing to decrement
                small = sz > 1 && sz <= kSmallSet;
                nbig = sz > kSmallSet ? (uint32_t)((sz + kWave - 1) / kWave) : 0u;
            }
            // one reservation per wave and queue
            const uint64_t smask = __ballot(small);
            if (smask) {
                uint32_t sbase = 0;
                if (lane == 0) sbase = g_add(small_n, (uint32_t)__popcll(smask));
                sbase = __shfl(sbase, 0, kWave);
                if (small)
                    store_chunk(d.chunks + sbase + (uint32_t)__popcll(smask & lane_mask), a,
                                (uint32_t)sz);
            }
            const uint32_t incl = wave_incl_scan(nbig);
            const uint32_t tot = __shfl(incl, kWave - 1, kWave);
            if (tot) {
                uint32_t wbase = 0;
                if (lane == kWave - 1) wbase = g_add(big_n, tot);
                wbase = __shfl(wbase, kWave - 1, kWave);
                const uint32_t pos = wbase + incl - nbig;
                for (uint32_t c = 0; c < nbig; ++c) {
                    const uint64_t o = (uint64_t)c * kWave;
                    store_chunk(d.chunks + (d.chunk_cap - 1 - (pos + c)), a + o,
                                (uint32_t)(sz - o < kWave ? sz - o : kWave));
                }
            }
        }
    }
    // dense sets: one bit test per uncovered bitmap; the claimed ones are
    // listed for the dense update
    for (uint32_t b0 = blk * kClaimBS; b0 < d.n_dense; b0 += d.sel_cnt * kClaimBS) {
        const uint32_t b = b0 + threadIdx.x;
        bool claimed = false;
        if (b < d.n_dense) {
            const uint32_t wv = d.dense_bits[(size_t)b * d.dense_words + (v >> 5)];
            if ((wv >> (v & 31)) & 1u) {
                const uint32_t j = d.dense_sid[b];
                const uint32_t bit = 1u << (j & 31);
                claimed = !(g_or(&d.covered[j >> 5], bit) & bit);
            }
        }
        const uint64_t cm = __ballot(claimed);
        if (cm) {
            uint32_t base = 0;
            if (lane == 0) base = g_add(d.dense_list_n, (uint32_t)__popcll(cm));
            base = __shfl(base, 0, kWave);
            if (claimed) {
                d.dense_list[base + (uint32_t)__popcll(cm & lane_mask)] = b;
                cov += d.dense_size[b];
            }
        }
    }
    cov = wave_sum64(cov);
    if (lane == 0 && cov) g_add64(&d.cov_entries[t], (unsigned long long)cov);
}

// Decrements summed per workgroup in an LDS table (vertex -> count) are
// applied with one atomic per distinct vertex: the sets a seed covers share
// their high-degree vertices, which would otherwise take one global atomic
// per covering set. A vertex that finds no slot within a few probes is
// decremented directly.
constexpr uint32_t kAggBits = 12;
constexpr uint32_t kAggSize = 1u << kAggBits;
constexpr uint32_t kAggProbes = 8;

__device__ __forceinline__ void agg_dec(uint32_t u, bool agg, uint32_t* h_key, uint32_t* h_cnt,
                                        IMM_GLOBAL uint32_t* cw) {
    if (agg) {
        uint32_t slot = (u * 0x9E3779B1u) >> (32 - kAggBits);
        for (uint32_t p = 0; p < kAggProbes; ++p) {
            uint32_t cur = h_key[slot];
            if (cur == kEmpty) cur = atomicCAS(&h_key[slot], kEmpty, u);
            if (cur == kEmpty || cur == u) {
                atomicAdd(&h_cnt[slot], 1u);
                return;
            }
            slot = (slot + 1) & (kAggSize - 1);
        }
    }
    g_sub(&cw[u], 1u);
}

// The adaptive counter update: when a seed covers sets that hold a large
// part of the pool, rebuilding each remaining count from the uncovered sets
// (a gather over the index, no global atomics) is cheaper than decrementing
// once per member of every covered set. The work items are the vertices with
// long index lists (more than kHeavyList positions), one wave each, then
// tiles of 64 consecutive vertices, one wave each, which skip those vertices.
// A tile's lists are one contiguous position range per segment, swept
// coalesced, sixteen positions per lane per round, counting uncovered sets per
// vertex in LDS (the owner of a position by binary search over the 65 list
// bounds). The index is read once per recount with non-temporal loads, so
// the covered bitmap, looked up at random once per position, stays in L2.
// Selected vertices keep their sentinel and zero counts stay zero.
constexpr uint32_t kRecountUnroll = 16;

// Uncovered sets in the index lists of one vertex, summed over the wave.
__device__ uint32_t count_uncovered(const SelView& d, uint32_t u) {
    const uint32_t lane = threadIdx.x % kWave;
    uint32_t cnt = 0;
    for (uint32_t seg = 0; seg < d.nseg; ++seg) {
        const IMM_GLOBAL uint64_t* io = d.inv_offs + (uint64_t)seg * ((uint64_t)d.n + 1);
        const uint64_t b = io[u], e = io[u + 1];
        for (uint64_t q = b + lane; q < e; q += kWave * kRecountUnroll) {
            // unguarded loads at clamped positions (a guarded load becomes a
            // branch with a wait of its own); positions past e count nothing
            uint32_t sid[kRecountUnroll];
#pragma unroll
            for (uint32_t x = 0; x < kRecountUnroll; ++x) {
                const uint64_t r = q + x * kWave;
                sid[x] = __builtin_nontemporal_load(d.inv_set + (r < e ? r : e - 1));
            }
            uint32_t cw_[kRecountUnroll];  // all covered-bit words in flight together
#pragma unroll
            for (uint32_t x = 0; x < kRecountUnroll; ++x) cw_[x] = d.covered[sid[x] >> 5];
#pragma unroll
            for (uint32_t x = 0; x < kRecountUnroll; ++x)
                if (q + x * kWave < e) cnt += ((cw_[x] >> (sid[x] & 31)) & 1u) ^ 1u;
        }
    }
#pragma unroll
    for (uint32_t s = kWave / 2; s >= 1; s >>= 1) cnt += __shfl_xor(cnt, s, kWave);
    return cnt;
}

__device__ void recount_all(const SelView& d, uint32_t blk, uint32_t* lds_off,
                            uint32_t* lds_cnt) {
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t wpb = kDecBS / kWave;
    const uint32_t wv = threadIdx.x / kWave;
    const uint32_t wid = blk * wpb + wv;
    const uint32_t nw = d.sel_cnt * wpb;
    const uint32_t nh = *d.n_heavy;
    const uint64_t ntiles = ((uint64_t)d.n + kWave - 1) / kWave;
    uint32_t* s_off = lds_off + wv * (kWave + 1);  // this wave's 65 bounds
    uint32_t* s_cnt = lds_cnt + wv * kWave;        // this wave's 64 counters
    for (uint64_t item = wid; item < nh + ntiles; item += nw) {
        if (item < nh) {
            const uint32_t u = d.heavy[item];
            const uint32_t c = d.cw[u];
            if (c == 0u || c == kSelected) continue;
            const uint32_t cnt = count_uncovered(d, u);
            if (lane == 0) d.cw[u] = cnt;
            continue;
        }
        const uint64_t u0 = (item - nh) * kWave;
        const uint32_t u = (uint32_t)u0 + lane;
        const bool in = u < d.n;
        const uint32_t c = in ? d.cw[u] : 0u;
        const bool heavy = in && d.cacc[u] > kHeavyList;
        const bool act = c != 0u && c != kSelected && !heavy;
        if (!__ballot(act)) continue;
        const uint64_t hmask = __ballot(heavy);
        s_cnt[lane] = 0u;
        const uint32_t hi_v = u0 + kWave < d.n ? (uint32_t)(u0 + kWave) : d.n;
        for (uint32_t seg = 0; seg < d.nseg; ++seg) {
            const IMM_GLOBAL uint64_t* io = d.inv_offs + (uint64_t)seg * ((uint64_t)d.n + 1);
            const uint64_t base = io[u0];
            const uint64_t my = io[u < hi_v ? u : hi_v];
            const uint64_t top = io[hi_v];
            // bounds relative to the range start (a range of one segment
            // holds fewer than 2^32 positions)
            s_off[lane] = (uint32_t)(my - base);
            if (lane == 0) s_off[kWave] = (uint32_t)(top - base);
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            // sweep the runs of lanes between long-list vertices
            for (uint32_t l0 = 0; l0 < kWave;) {
                const uint64_t light_from = ~hmask & (~0ull << l0);
                if (!light_from) break;
                l0 = (uint32_t)__ffsll((long long)light_from) - 1u;
                const uint64_t heavy_after = hmask & (~0ull << l0);
                const uint32_t l1 =
                    heavy_after ? (uint32_t)__ffsll((long long)heavy_after) - 1u : kWave;
                const uint32_t lo_pos = s_off[l0], hi_pos = s_off[l1];
                for (uint32_t q0 = lo_pos; q0 < hi_pos; q0 += kWave * kRecountUnroll) {
                    // unguarded loads at clamped positions, as in
                    // count_uncovered; positions past hi_pos count nothing
                    uint32_t sid[kRecountUnroll];
#pragma unroll
                    for (uint32_t x = 0; x < kRecountUnroll; ++x) {
                        const uint32_t r = q0 + x * kWave + lane;
                        sid[x] = __builtin_nontemporal_load(d.inv_set + base +
                                                            (r < hi_pos ? r : hi_pos - 1));
                    }
                    uint32_t cw_[kRecountUnroll];  // all covered-bit words in flight together
#pragma unroll
                    for (uint32_t x = 0; x < kRecountUnroll; ++x) cw_[x] = d.covered[sid[x] >> 5];
#pragma unroll
                    for (uint32_t x = 0; x < kRecountUnroll; ++x) {
                        const uint32_t r = q0 + x * kWave + lane;
                        if (r < hi_pos && !((cw_[x] >> (sid[x] & 31)) & 1u)) {
                            // owner: the last lane whose list starts at or before r
                            uint32_t lo = l0, hi = l1;
                            while (hi - lo > 1) {
                                const uint32_t mid = (lo + hi) >> 1;
                                if (s_off[mid] <= r) lo = mid; else hi = mid;
                            }
                            atomicAdd(&s_cnt[lo], 1u);
                        }
                    }
                }
                l0 = l1;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        if (act) d.cw[u] = s_cnt[lane];
        __builtin_amdgcn_wave_barrier();
    }
}

// Small covered sets are taken one per lane (a flood of tiny sets keeps every
// lane busy), the 64-member pieces of larger ones one per wave.
__global__ __launch_bounds__(kDecBS) void decrement_kernel(const SelectDesc* descs, uint32_t nq,
                                                           uint32_t t) {
    __shared__ uint32_t h_key[kAggSize], h_cnt[kAggSize];
    const uint32_t q = find_inst(descs, nq, blockIdx.x, 0);
    if (q == nq) return;
    const SelView d = view_of(descs[q]);
    if (t >= d.k) return;
    const uint32_t blk = blockIdx.x - d.sel_lo;
    // the state words, the pool size, the step's covered total and its queue
    // lengths load together
    const uint4 cs = cand_head(d);
    const uint64_t pool = d.set_off[d.n_sets] + d.dense_entries;
    const uint64_t cov = d.cov_entries[t];
    const uint32_t ns = d.chunk_n[2ull * t], nb = d.chunk_n[2ull * t + 1];
    if (cs.y != 0u && t >= cs.y) return;  // halted
    if (d.update == kUpdateRecount || (d.update == kUpdateAdaptive && cov * 4ull > pool)) {
        recount_all(d, blk, h_key, h_cnt);
        return;
    }
    const uint32_t wpb = kDecBS / kWave;
    if (blk * kDecBS >= ns && blk * wpb >= nb) return;
    IMM_GLOBAL uint32_t* cw = d.cw;
    const uint32_t v = d.seeds[t];
    // a candidate step decrements only the listed vertices
    const bool filt = t >= 1 && cs.x == 1u;
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t threads = d.sel_cnt * kDecBS;
    const uint32_t nw = d.sel_cnt * wpb;
    const uint32_t wid = blk * wpb + threadIdx.x / kWave;
    // aggregate when a workgroup will see many decrements
    const bool agg = (uint64_t)ns * 4 + (uint64_t)nb * kWave >= 16ull * threads;
    if (agg) {
        for (uint32_t x = threadIdx.x; x < kAggSize; x += kDecBS) {
            h_key[x] = kEmpty;
            h_cnt[x] = 0;
        }
        __syncthreads();
    }
    for (uint32_t e = blk * kDecBS + threadIdx.x; e < ns; e += threads) {
        const Chunk ch = load_chunk(d.chunks + e);
        // members four at a time, loaded together (clamped to the set; a
        // repeated member is skipped)
        for (uint32_t x = 0; x < ch.len; x += 4) {
            uint32_t u[4];
#pragma unroll
            for (uint32_t y = 0; y < 4; ++y)
                u[y] = d.set_vtx[ch.off + (x + y < ch.len ? x + y : ch.len - 1)];
            bool keep[4];
            if (filt) {
#pragma unroll
                for (uint32_t y = 0; y < 4; ++y) keep[y] = is_cand(d, u[y]);
            } else {
#pragma unroll
                for (uint32_t y = 0; y < 4; ++y) keep[y] = true;
            }
#pragma unroll
            for (uint32_t y = 0; y < 4; ++y)
                if (x + y < ch.len && u[y] != v && keep[y]) agg_dec(u[y], agg, h_key, h_cnt, cw);
        }
    }
    for (uint32_t c = wid; c < nb; c += nw) {
        const Chunk ch = load_chunk(d.chunks + (d.chunk_cap - 1 - c));
        if (lane < ch.len) {
            const uint32_t u = d.set_vtx[ch.off + lane];
            if (u != v && (!filt || is_cand(d, u))) agg_dec(u, agg, h_key, h_cnt, cw);
        }
    }
    if (agg) {
        __syncthreads();
        for (uint32_t x = threadIdx.x; x < kAggSize; x += kDecBS) {
            const uint32_t c = h_cnt[x];
            if (c) g_sub(&cw[h_key[x]], c);
        }
    }
}

// The dense sets' part of seed step t's counter update, after the list part
// (decrement_kernel): when the step recounts, every count gains the bitmap
// sum of the uncovered dense sets; otherwise it loses that of the dense sets
// the step claimed. Workgroup (word block wb, bitmap chunk c) of the
// instance covers 2048 vertices and kColChunk bitmaps; chosen seeds keep
// their sentinel.
__global__ __launch_bounds__(kColBS) void dense_update_kernel(const SelectDesc* descs,
                                                              uint32_t nq, uint32_t t) {
    __shared__ uint32_t lds[4 * 2048];
    const uint32_t q = find_inst(descs, nq, blockIdx.x, 2);
    if (q == nq) return;
    const SelView d = view_of(descs[q]);
    if (t >= d.k || d.n_dense == 0) return;
    if (step_halted(d, t)) return;
    const uint32_t blk = blockIdx.x - descs[q].dense_lo;
    const uint32_t wblocks = (d.dense_words + 63) / 64;
    const uint32_t wb = blk % wblocks, c = blk / wblocks;
    const uint64_t pool = d.set_off[d.n_sets] + d.dense_entries;
    const bool recount = d.update == kUpdateRecount ||
                         (d.update == kUpdateAdaptive && d.cov_entries[t] * 4ull > pool);
    const uint32_t lo = recount ? 0u : d.dense_mark[t];
    const uint32_t hi = recount ? d.n_dense : *d.dense_list_n;
    const uint32_t i0 = lo + c * kColChunk;
    if (i0 >= hi) return;
    const uint32_t cnt = min(kColChunk, hi - i0);
    uint32_t out[8];
    if (recount) {
        col_sums((const uint32_t*)d.dense_bits, d.dense_words, 64u * wb, cnt,
                 [&](uint32_t i) {
                     const uint32_t b = i0 + i;
                     const uint32_t j = d.dense_sid[b];
                     return ((d.covered[j >> 5] >> (j & 31)) & 1u) ? kEmpty : b;
                 },
                 lds, out);
    } else {
        col_sums((const uint32_t*)d.dense_bits, d.dense_words, 64u * wb, cnt,
                 [&](uint32_t i) { return d.dense_list[i0 + i]; }, lds, out);
    }
#pragma unroll
    for (uint32_t x = 0; x < 8; ++x) {
        const uint32_t u = 2048u * wb + 8u * threadIdx.x + x;
        if (u >= d.n || out[x] == 0) continue;
        if (d.cw[u] == kSelected) continue;
        if (recount) g_add(&d.cw[u], out[x]);
        else g_sub(&d.cw[u], out[x]);
    }
}

// The histogram of the working counts over kCandBins bins (LDS per
// workgroup, then one global add per bin), zero counts left out.
__global__ __launch_bounds__(256) void cand_hist_kernel(const uint32_t* cw, uint32_t n,
                                                        uint32_t* hist) {
    __shared__ uint32_t s_h[kCandBins];
    for (uint32_t x = threadIdx.x; x < kCandBins; x += 256) s_h[x] = 0u;
    __syncthreads();
    const uint32_t stride = gridDim.x * 256;
    const uint32_t n4 = n >> 2;
    const uint4* cw4 = reinterpret_cast<const uint4*>(cw);
    // four 16-byte loads per thread in flight (clamped; a repeated group
    // is not counted)
    for (uint32_t x0 = blockIdx.x * 256 + threadIdx.x; x0 < n4; x0 += 4 * stride) {
        uint4 cc[4];
#pragma unroll
        for (uint32_t y = 0; y < 4; ++y) {
            const uint32_t x = x0 + y * stride;
            cc[y] = cw4[x < n4 ? x : x0];
        }
#pragma unroll
        for (uint32_t y = 0; y < 4; ++y) {
            if (x0 + y * stride >= n4) continue;
            const uint4 c = cc[y];
            if (c.x) atomicAdd(&s_h[cand_bin(c.x)], 1u);
            if (c.y) atomicAdd(&s_h[cand_bin(c.y)], 1u);
            if (c.z) atomicAdd(&s_h[cand_bin(c.z)], 1u);
            if (c.w) atomicAdd(&s_h[cand_bin(c.w)], 1u);
        }
    }
    const uint32_t tail = (n4 << 2) + blockIdx.x * 256 + threadIdx.x;
    if (tail < n && blockIdx.x * 256 + threadIdx.x < 4u) {
        const uint32_t c = cw[tail];
        if (c) atomicAdd(&s_h[cand_bin(c)], 1u);
    }
    __syncthreads();
    for (uint32_t x = threadIdx.x; x < kCandBins; x += 256)
        if (s_h[x]) atomicAdd(&hist[x], s_h[x]);
}

// tau, the lowest bin edge with at most cand_max vertices counting that much
// or more (never below 1; no list when even the top bin holds more), then
// the bitmap and the list. A wave takes 64 bitmap words (2048 vertices) as
// eight coalesced rows of 64 16-byte loads; the eight lanes of a word OR its
// 32 bits together. The workgroup reserves its list entries with one atomic
// (the list length is one counter for the whole launch: an atomic per wave
// would queue up on it).
constexpr uint32_t kListBS = 1024;
__global__ __launch_bounds__(kListBS) void cand_list_kernel(const uint32_t* cw, uint32_t n,
                                                            uint32_t cand_max, uint32_t* cand,
                                                            uint32_t* cand_bits,
                                                            uint32_t* state) {
    __shared__ uint32_t s_tau;
    __shared__ uint32_t s_wt[kListBS / kWave];
    __shared__ uint32_t s_base;
    __shared__ uint32_t s_hist[kCandBins];
    // the histogram staged in LDS by all threads at once (a walk down it
    // through global memory would be one dependent load per bin)
    for (uint32_t x = threadIdx.x; x < kCandBins; x += kListBS) s_hist[x] = state[kCandHead + x];
    __syncthreads();
    if (threadIdx.x == 0) {
        const uint32_t* hist = s_hist;
        uint32_t acc = 0, b = kCandBins;
        for (uint32_t x = kCandBins; x-- > 1;) {
            acc += hist[x];
            if (acc > cand_max) break;
            b = x;
        }
        const uint32_t tau = b < kCandBins ? cand_edge(b) : 0xFFFFFFFFu;
        s_tau = tau;
        if (blockIdx.x == 0) state[2] = tau;
    }
    __syncthreads();
    const uint32_t tau = s_tau;
    const uint32_t words = (n + 31) / 32;
    const uint32_t lane = lane_id(), wv = threadIdx.x / kWave;
    const uint32_t w0 = (blockIdx.x * (kListBS / kWave) + wv) * kWave;
    const bool live = w0 < words;  // (the whole wave alike)
    const uint32_t n4 = n / 4;
    const uint4* cw4 = reinterpret_cast<const uint4*>(cw);
    uint4 c[8];
#pragma unroll
    for (uint32_t r = 0; r < 8; ++r) {
        // row r, lane l: the four counts of 16-byte group 8 w0 + 64 r + l
        const uint32_t g = 8u * w0 + 64u * r + lane;
        if (!live) {
            c[r] = make_uint4(0u, 0u, 0u, 0u);
        } else if (g < n4) {
            c[r] = cw4[g];
        } else {
            const uint32_t v = 4u * g;
            c[r] = make_uint4(v < n ? cw[v] : 0u, v + 1 < n ? cw[v + 1] : 0u,
                              v + 2 < n ? cw[v + 2] : 0u, v + 3 < n ? cw[v + 3] : 0u);
        }
    }
    uint32_t bits[8], cnt = 0;
#pragma unroll
    for (uint32_t r = 0; r < 8; ++r) {
        uint32_t b = (uint32_t)(c[r].x >= tau) | ((uint32_t)(c[r].y >= tau) << 1) |
                     ((uint32_t)(c[r].z >= tau) << 2) | ((uint32_t)(c[r].w >= tau) << 3);
        b <<= 4u * (lane & 7u);
        b |= __shfl_xor(b, 1, kWave);
        b |= __shfl_xor(b, 2, kWave);
        b |= __shfl_xor(b, 4, kWave);
        // word w0 + 8 r + lane / 8, held by the first lane of its eight
        const uint32_t wd = w0 + 8u * r + lane / 8u;
        const bool own = live && (lane & 7u) == 0u && wd < words;
        bits[r] = own ? b : 0u;
        if (own) cand_bits[wd] = b;
        cnt += (uint32_t)__popc(bits[r]);
    }
    const uint32_t incl = wave_incl_scan(cnt);
    if (lane == kWave - 1) s_wt[wv] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t tot = 0;
        for (uint32_t x = 0; x < kListBS / kWave; ++x) {
            const uint32_t t = s_wt[x];
            s_wt[x] = tot;  // the waves' offsets within the workgroup
            tot += t;
        }
        s_base = tot ? atomicAdd(&state[3], tot) : 0u;
    }
    __syncthreads();
    if (cnt == 0) return;
    uint32_t pos = s_base + s_wt[wv] + incl - cnt;
#pragma unroll
    for (uint32_t r = 0; r < 8; ++r) {
        uint32_t b = bits[r];
        const uint32_t wd = w0 + 8u * r + lane / 8u;
        while (b) {
            const uint32_t j = (uint32_t)__ffs(b) - 1u;
            b &= b - 1u;
            if (pos < kCandMax) cand[pos] = wd * 32u + j;
            ++pos;
        }
    }
}

// cw = cacc (+ dc, the dense sets' counts); vertices with long index lists
// are appended to heavy (one atomic per wave).
__global__ __launch_bounds__(256) void select_init_kernel(const uint32_t* cacc, const uint32_t* dc,
                                                          uint32_t* cw, uint32_t n,
                                                          uint32_t* heavy, uint32_t* n_heavy,
                                                          ZeroSpans z) {
    // the selection's state blocks cleared on the way (no fill launches)
    {
        const uint64_t g = (uint64_t)blockIdx.x * 256 + threadIdx.x;
        const uint64_t stride = (uint64_t)gridDim.x * 256;
#pragma unroll
        for (uint32_t k = 0; k < ZeroSpans::kCount; ++k)
            for (uint64_t x = g; x < z.words[k]; x += stride) z.p[k][x] = 0u;
    }
    const uint32_t u = blockIdx.x * 256 + threadIdx.x;
    const uint32_t c = u < n ? cacc[u] : 0u;
    if (u < n) cw[u] = c + (dc ? dc[u] : 0u);
    const bool h = c > kHeavyList;
    const uint64_t m = __ballot(h);
    if (!m) return;
    const uint32_t lane = lane_id();
    uint32_t base = 0;
    if (lane == 0) base = atomicAdd(n_heavy, (uint32_t)__popcll(m));
    base = __shfl(base, 0, kWave);
    if (h) heavy[base + __popcll(m & ((1ull << lane) - 1ull))] = u;
}

}  // namespace

uint32_t argmax_blocks(uint32_t n) {
    uint32_t g = (n / 4 + kArgBS * kArgLoads - 1) / (kArgBS * kArgLoads);
    if (g < 1) g = 1;
    if (g > 1024) g = 1024;
    return g;
}

uint32_t select_blocks(int device, uint64_t n_sets, uint32_t batch) {
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    // a lone instance gets the whole GPU; in a batch, blocks follow pool size
    const uint64_t full = (uint64_t)cus * 4u;
    if (batch <= 1) return (uint32_t)full;
    return (uint32_t)std::min<uint64_t>(full, n_sets / 4096 + 8);
}

hipError_t launch_select_init(const uint32_t* cacc, uint32_t* cw, uint32_t n, uint32_t* heavy,
                              uint32_t* n_heavy, hipStream_t st) {
    return launch_select_init2(cacc, nullptr, cw, n, heavy, n_heavy, st);
}

hipError_t launch_select_init2(const uint32_t* cacc, const uint32_t* dc, uint32_t* cw,
                               uint32_t n, uint32_t* heavy, uint32_t* n_heavy, hipStream_t st,
                               const ZeroSpans& z) {
    uint64_t zw = 0;
    for (uint32_t k = 0; k < ZeroSpans::kCount; ++k) zw += z.p[k] ? z.words[k] : 0;
    if (n == 0 && zw == 0) return hipSuccess;
    ZeroSpans zz = z;
    for (uint32_t k = 0; k < ZeroSpans::kCount; ++k)
        if (!zz.p[k]) zz.words[k] = 0;
    hipLaunchKernelGGL(select_init_kernel, dim3(std::max(1u, (n + 255) / 256)), dim3(256), 0, st,
                       cacc, dc, cw, n, heavy, n_heavy, zz);
    return hipGetLastError();
}

hipError_t launch_cand_build(const uint32_t* cw, uint32_t n, uint32_t cand_max, uint32_t* cand,
                             uint32_t* cand_bits, uint32_t* cand_state, hipStream_t st) {
    if (n == 0 || cand_max == 0) return hipSuccess;
    if (cand_max > kCandMax) cand_max = kCandMax;
    const uint32_t hb = std::min<uint32_t>(256u, (n + 1023u) / 1024u);
    hipLaunchKernelGGL(cand_hist_kernel, dim3(hb), dim3(256), 0, st, cw, n,
                       cand_state + kCandHead);
    const uint32_t words = (n + 31) / 32;
    // sixteen waves of 64 words each per workgroup
    constexpr uint32_t kWordsPerBlock = kListBS / kWave * kWave;
    hipLaunchKernelGGL(cand_list_kernel, dim3((words + kWordsPerBlock - 1) / kWordsPerBlock),
                       dim3(kListBS), 0, st, cw, n, cand_max, cand, cand_bits, cand_state);
    return hipGetLastError();
}

hipError_t launch_select_recount(const SelectDesc* descs, uint32_t t, uint32_t sel_blocks,
                                 uint32_t dense_blocks, hipStream_t st) {
    hipLaunchKernelGGL(decrement_kernel, dim3(sel_blocks), dim3(kDecBS), 0, st, descs, 1u, t);
    if (dense_blocks)
        hipLaunchKernelGGL(dense_update_kernel, dim3(dense_blocks), dim3(kColBS), 0, st, descs,
                           1u, t);
    return hipGetLastError();
}

uint32_t dense_blocks(uint32_t n_dense, uint32_t words) {
    if (n_dense == 0) return 0;
    return ((words + 63) / 64) * ((n_dense + kColChunk - 1) / kColChunk);
}

hipError_t launch_select_step(const SelectDesc* descs, uint32_t nq, uint32_t t,
                              uint32_t arg_blocks, uint32_t sel_blocks, uint32_t dense_blocks,
                              hipStream_t st) {
    hipLaunchKernelGGL(argmax_kernel, dim3(arg_blocks), dim3(kArgBS), 0, st, descs, nq, t);
    hipLaunchKernelGGL(claim_kernel, dim3(sel_blocks), dim3(kClaimBS), 0, st, descs, nq, t);
    hipLaunchKernelGGL(decrement_kernel, dim3(sel_blocks), dim3(kDecBS), 0, st, descs, nq, t);
    if (dense_blocks)
        hipLaunchKernelGGL(dense_update_kernel, dim3(dense_blocks), dim3(kColBS), 0, st, descs,
                           nq, t);
    return hipGetLastError();
}

}  // namespace imm
