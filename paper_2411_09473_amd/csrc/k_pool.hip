// k_pool.hip -- RRR pool construction and the vertex->sets inverted index.
//
//  * scan: exclusive prefix sums of uint32 values into uint64 offsets
//    (reduce tiles, scan the tile sums in one block, rescan tiles with carry).
//  * compact: staged sets -> a CSR pool in sample-id order.
//  * inverted index: inv_off = scan(counts); each member v of set j writes j
//    into v's list, so covering the sets of a chosen seed (Algorithm 2,
//    "if v in R") touches only those sets instead of testing every set.
//  * canonical order for export: each set sorted ascending in place.
// Segmented loops give the entries of 64 consecutive sets to the 64 lanes of
// a wave, so the work stays balanced whatever the mix of set sizes.
#include "device_common.hpp"
#include "imm_internal.hpp"

namespace imm {

namespace {

constexpr uint32_t kScanBS = 256;
constexpr uint32_t kScanIPT = 8;
constexpr uint32_t kScanTile = kScanBS * kScanIPT;

__device__ __forceinline__ uint64_t block_sum64(uint64_t v, uint64_t* s_w) {
    const uint32_t w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    v = wave_sum64(v);
    if (lane == 0) s_w[w] = v;
    __syncthreads();
    uint64_t t = 0;
    for (uint32_t i = 0; i < blockDim.x / kWave; ++i) t += s_w[i];
    __syncthreads();
    return t;
}

// Exclusive scan of one uint64 per thread across the block; returns the total.
__device__ __forceinline__ uint64_t block_excl_scan64(uint64_t v, uint64_t* excl,
                                                      uint64_t* s_w) {
    const uint32_t w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const uint64_t incl = wave_incl_scan64(v);
    if (lane == kWave - 1) s_w[w] = incl;
    __syncthreads();
    uint64_t before = 0, total = 0;
    for (uint32_t i = 0; i < blockDim.x / kWave; ++i) {
        const uint64_t x = s_w[i];
        if (i < w) before += x;
        total += x;
    }
    __syncthreads();
    *excl = before + incl - v;
    return total;
}

// Scanned value of element i: in[i], or in[i] - sub[i] with SUB; 0 for
// i >= N. The loads are unguarded (at the clamped position N - 1, N >= 1): a
// guarded load compiles to a branch with a wait of its own, which would
// serialise a thread's loads.
template <bool SUB>
__device__ __forceinline__ uint32_t scan_val(const uint32_t* in, const uint32_t* sub, uint64_t i,
                                             uint64_t N) {
    const uint64_t c = i < N ? i : N - 1;
    const uint32_t x = SUB ? in[c] - sub[c] : in[c];
    return i < N ? x : 0u;
}

template <bool SUB>
__global__ __launch_bounds__(kScanBS) void scan_tiles_kernel(const uint32_t* in,
                                                             const uint32_t* sub, uint64_t N,
                                                             uint64_t* tile_sum) {
    __shared__ uint64_t s_w[kScanBS / kWave];
    const uint64_t base = (uint64_t)blockIdx.x * kScanTile;
    uint64_t acc = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanIPT; ++k) {
        const uint64_t i = base + (uint64_t)k * kScanBS + threadIdx.x;
        acc += scan_val<SUB>(in, sub, i, N);
    }
    const uint64_t t = block_sum64(acc, s_w);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = t;
}

__global__ __launch_bounds__(1024) void scan_sums_kernel(uint64_t* tile_sum, uint64_t tiles) {
    __shared__ uint64_t s_w[1024 / kWave];
    __shared__ uint64_t s_carry;
    if (threadIdx.x == 0) s_carry = 0;
    __syncthreads();
    for (uint64_t c = 0; c < tiles; c += 1024) {
        const uint64_t i = c + threadIdx.x;
        const uint64_t v = i < tiles ? tile_sum[i] : 0;
        uint64_t excl;
        const uint64_t total = block_excl_scan64(v, &excl, s_w);
        const uint64_t carry = s_carry;
        if (i < tiles) tile_sum[i] = carry + excl;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + total;
        __syncthreads();
    }
}

// base_dev, when given, supplies the base from device memory (it may alias
// out[0], which is rewritten with the same value).
template <bool SUB>
__global__ __launch_bounds__(kScanBS) void scan_apply_kernel(const uint32_t* in,
                                                             const uint32_t* sub, uint64_t N,
                                                             const uint64_t* tile_off,
                                                             uint64_t* out, uint64_t base,
                                                             const uint64_t* base_dev) {
    __shared__ uint64_t s_w[kScanBS / kWave];
    if (base_dev) base = *base_dev;
    const uint64_t tb = (uint64_t)blockIdx.x * kScanTile;
    const uint64_t my = tb + (uint64_t)threadIdx.x * kScanIPT;  // kScanIPT consecutive
    uint32_t v[kScanIPT];
    uint64_t acc = 0;
#pragma unroll
    for (uint32_t k = 0; k < kScanIPT; ++k) {
        v[k] = scan_val<SUB>(in, sub, my + k, N);
        acc += v[k];
    }
    uint64_t excl;
    block_excl_scan64(acc, &excl, s_w);
    uint64_t run = base + tile_off[blockIdx.x] + excl;
#pragma unroll
    for (uint32_t k = 0; k < kScanIPT; ++k) {
        run += v[k];
        if (my + k < N) out[my + k + 1] = run;
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[0] = base;
}

// A wave copies the members of 64 sets as one flattened range, eight loads
// per lane in flight before their stores (one at a time, each copy waited
// for its load: a wave of LJ-shaped sets, 6,000 members, took 95 round trips).
__global__ __launch_bounds__(64) void compact_kernel(const uint32_t* stage,
                                                     const uint64_t* stage_off,
                                                     const uint64_t* set_off, uint64_t lo,
                                                     uint32_t count, uint32_t* set_vtx) {
    __shared__ uint64_t s_base[kWave], s_src[kWave], s_dst[kWave];
    const uint32_t lane = threadIdx.x;
    const uint64_t i = (uint64_t)blockIdx.x * kWave + lane;
    uint32_t sz = 0;
    uint64_t src = 0, dst = 0;
    if (i < count) {
        dst = set_off[lo + i];
        sz = (uint32_t)(set_off[lo + i + 1] - dst);
        src = stage_off[i];
    }
    const uint64_t incl = wave_incl_scan64(sz);
    const uint64_t T = __shfl(incl, kWave - 1, kWave);
    s_base[lane] = incl - sz;
    s_src[lane] = src;
    s_dst[lane] = dst;
    __syncthreads();
    constexpr uint32_t kB = 8;
    uint32_t ow = 0;
    for (uint64_t t0 = 0; t0 < T; t0 += (uint64_t)kWave * kB) {
        uint32_t v[kB];
        uint64_t d[kB];
#pragma unroll
        for (uint32_t x = 0; x < kB; ++x) {
            const uint64_t t = t0 + (uint64_t)x * kWave + lane;
            const uint64_t tc = t < T ? t : T - 1;
            ow = owner_from(s_base, kWave, tc, ow);
            const uint64_t k = tc - s_base[ow];
            v[x] = stage[s_src[ow] + k];
            d[x] = s_dst[ow] + k;
        }
#pragma unroll
        for (uint32_t x = 0; x < kB; ++x)
            if (t0 + (uint64_t)x * kWave + lane < T) set_vtx[d[x]] = v[x];
    }
}

// A member beyond its vertex's counted occurrences would mean the counts and
// the pool disagree; it is not written and raises *err instead.
//
// A wave takes 64 sets and walks their members as one flattened range. Full
// rounds of kScatterBatch members per lane issue their loads, then their
// cursor atomics and list bounds, together, so a round costs two round trips
// however many members it holds (a wave that owns a giant set walks hundreds
// of thousands of members; one member at a time, its round trips would set
// the launch's duration). The rest goes one member per lane at a time.
constexpr uint32_t kScatterBatch = 8;

__global__ __launch_bounds__(64) void inv_scatter_kernel(const uint64_t* set_off,
                                                         const uint32_t* set_vtx, uint64_t lo,
                                                         uint32_t count, const uint64_t* inv_off,
                                                         uint32_t* cursor, uint32_t* inv_set,
                                                         uint32_t* err) {
    __shared__ uint64_t s_base[kWave], s_a[kWave];
    const uint32_t lane = threadIdx.x;
    const uint64_t j0 = lo + (uint64_t)blockIdx.x * kWave;
    const uint64_t j = j0 + lane;
    const uint64_t jl = j < lo + count ? j : lo + count - 1;
    const uint64_t a = set_off[jl];
    const uint32_t sz = j < lo + count ? (uint32_t)(set_off[jl + 1] - a) : 0u;
    const uint64_t incl = wave_incl_scan64(sz);
    const uint64_t T = __shfl(incl, kWave - 1, kWave);
    s_base[lane] = incl - sz;
    s_a[lane] = a;
    __syncthreads();
    uint32_t hint = 0;
    bool bad = false;
    constexpr uint64_t kRound = (uint64_t)kWave * kScatterBatch;
    uint64_t t0 = 0;
    for (; t0 + kRound <= T; t0 += kRound) {
        uint32_t ow[kScatterBatch], u[kScatterBatch];
#pragma unroll
        for (uint32_t x = 0; x < kScatterBatch; ++x) {
            const uint64_t t = t0 + (uint64_t)x * kWave + lane;
            hint = owner_from(s_base, kWave, t, hint);
            ow[x] = hint;
            u[x] = set_vtx[s_a[hint] + (t - s_base[hint])];
        }
        uint32_t r[kScatterBatch];
        uint64_t b[kScatterBatch], e[kScatterBatch];
#pragma unroll
        for (uint32_t x = 0; x < kScatterBatch; ++x) {
            r[x] = atomicAdd(&cursor[u[x]], 1u);
            b[x] = inv_off[u[x]];
            e[x] = inv_off[u[x] + 1];
        }
#pragma unroll
        for (uint32_t x = 0; x < kScatterBatch; ++x) {
            if (b[x] + r[x] < e[x]) inv_set[b[x] + r[x]] = (uint32_t)(j0 + ow[x]);
            else bad = true;
        }
    }
    for (uint64_t t = t0 + lane; t < T; t += kWave) {
        hint = owner_from(s_base, kWave, t, hint);
        const uint32_t u = set_vtx[s_a[hint] + (t - s_base[hint])];
        const uint32_t r = atomicAdd(&cursor[u], 1u);
        const uint64_t b = inv_off[u];
        if (b + r < inv_off[u + 1]) inv_set[b + r] = (uint32_t)(j0 + hint);
        else bad = true;
    }
    if (__any(bad) && lane == 0) atomicOr(err, 1u);
}

// ---- index build by radix partition
//
// The per-entry cursor atomic above goes to the memory side (the L2 caches of
// the XCDs are not coherent with each other), and a hub vertex's cursor takes
// one such atomic per occurrence. The partitioned build needs none per entry:
//  1. plan: buckets of 2^shift consecutive vertices; bucket b's entries occupy
//     [off[b], off[b+1]) of the segment, the list space of its vertices, so
//     its bounds come from the segment offsets already scanned. Each bucket
//     is cut into slices of kSlice entries, numbered across buckets.
//  2. partition: a workgroup takes a tile of sets, counts its members per
//     bucket in LDS, reserves each bucket's share with one atomic, and writes
//     (set << 32 | vertex) pairs into the bucket's range.
//  3. place: a workgroup takes a slice of one bucket and ranks its pairs per
//     vertex with LDS counters; when the bucket has more than one slice, one
//     atomic per vertex and slice reserves the slice's share of that
//     vertex's list.
// Ranks within a list depend on timing, as with the atomic scatter: the
// selection only counts and tests a list's members, never its order.
constexpr uint32_t kPartBS = 1024;
constexpr uint32_t kPartTile = 256;  // sets per tile group
constexpr uint32_t kPlaceBS = 1024;
constexpr uint32_t kPlaceBatch = 4;

__global__ __launch_bounds__(1024) void inv_plan_kernel(const uint64_t* io, uint32_t n,
                                                        uint32_t shift, uint32_t nb,
                                                        uint64_t cap, IndexPlan* pl,
                                                        uint32_t* err) {
    __shared__ uint64_t s_w[1024 / kWave];
    __shared__ uint64_t s_carry;
    const uint64_t base = io[0];
    const uint64_t total = io[n] - base;
    const bool fits = total <= cap;
    if (threadIdx.x == 0) {
        s_carry = 0;
        if (!fits) atomicOr(err, 1u);
    }
    __syncthreads();
    for (uint32_t c = 0; c <= nb; c += 1024) {
        const uint32_t b = c + threadIdx.x;
        uint64_t ns = 0;
        // a segment beyond the pair buffer gets empty buckets: every
        // reservation then fails, and no pair is written or placed
        if (b < nb) {
            const uint64_t v1 = min((uint64_t)(b + 1) << shift, (uint64_t)n);
            const uint64_t a0 = io[(uint64_t)b << shift] - base, a1 = io[v1] - base;
            pl->off[b] = fits ? a0 : 0;
            pl->cur[b] = 0;
            ns = fits ? (a1 - a0 + kSlice - 1) / kSlice : 0;
        } else if (b == nb) {
            pl->off[nb] = fits ? total : 0;
        }
        uint64_t excl;
        const uint64_t tot = block_excl_scan64(ns, &excl, s_w);
        const uint64_t carry = s_carry;
        if (b <= nb) pl->sl_pre[b] = (uint32_t)(carry + excl);
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
}

// The members of the sets [j0, min(j0 + kPartBS, jend)), walked by the
// whole workgroup: f(u, j) for each member u of set j, up to eight loads per
// thread in flight.
template <class F>
__device__ __forceinline__ void block_members(const uint64_t* set_off, const uint32_t* set_vtx,
                                              uint64_t j0, uint64_t jend, uint64_t* s_sb,
                                              uint64_t* s_sa, uint64_t* s_w, F f) {
    const uint64_t j = j0 + threadIdx.x;
    const uint64_t jl = j < jend ? j : jend - 1;
    const uint64_t a = set_off[jl];
    const uint64_t sz = j < jend ? set_off[jl + 1] - a : 0;
    uint64_t excl;
    const uint64_t T = block_excl_scan64(sz, &excl, s_w);
    s_sb[threadIdx.x] = excl;
    s_sa[threadIdx.x] = a;
    __syncthreads();
    constexpr uint32_t kB = 8;
    uint32_t ow = 0;
    for (uint64_t t0 = 0; t0 < T; t0 += (uint64_t)kPartBS * kB) {
        uint32_t u[kB], o[kB];
#pragma unroll
        for (uint32_t x = 0; x < kB; ++x) {
            const uint64_t t = t0 + (uint64_t)x * kPartBS + threadIdx.x;
            const uint64_t tc = t < T ? t : T - 1;
            ow = owner_from(s_sb, kPartBS, tc, ow);
            o[x] = ow;
            u[x] = set_vtx[s_sa[ow] + (tc - s_sb[ow])];
        }
#pragma unroll
        for (uint32_t x = 0; x < kB; ++x)
            if (t0 + (uint64_t)x * kPartBS + threadIdx.x < T) f(u[x], j0 + o[x]);
    }
    __syncthreads();
}

__global__ __launch_bounds__(kPartBS) void inv_part_kernel(const uint64_t* set_off,
                                                           const uint32_t* set_vtx, uint64_t lo,
                                                           uint32_t count, uint32_t tile_groups,
                                                           uint32_t shift, uint32_t nb,
                                                           IndexPlan* pl, unsigned long long* tmp,
                                                           uint32_t* err) {
    __shared__ uint32_t s_cnt[kBktMax], s_res[kBktMax];
    __shared__ uint64_t s_base[kBktMax];
    __shared__ uint64_t s_sb[kPartBS], s_sa[kPartBS], s_w[kPartBS / kWave];
    for (uint32_t b = threadIdx.x; b < nb; b += kPartBS) s_cnt[b] = 0;
    __syncthreads();
    const uint64_t jend = lo + count;
    const uint64_t g0 = lo + (uint64_t)blockIdx.x * tile_groups * kPartTile;
    const uint64_t g1 = min(g0 + (uint64_t)tile_groups * kPartTile, jend);
    // the tile's members are one contiguous range of the pool: the histogram
    // reads it flat, eight coalesced loads per thread in flight
    {
        const uint64_t a0 = set_off[g0], a1 = set_off[g1];
        constexpr uint32_t kB = 8;
        for (uint64_t e0 = a0; e0 < a1; e0 += (uint64_t)kPartBS * kB) {
            uint32_t u[kB];
#pragma unroll
            for (uint32_t x = 0; x < kB; ++x) {
                const uint64_t e = e0 + (uint64_t)x * kPartBS + threadIdx.x;
                u[x] = set_vtx[e < a1 ? e : a1 - 1];
            }
#pragma unroll
            for (uint32_t x = 0; x < kB; ++x) {
                const uint32_t b = u[x] >> shift;
                if (e0 + (uint64_t)x * kPartBS + threadIdx.x < a1 && b < nb)
                    atomicAdd(&s_cnt[b], 1u);
            }
        }
    }
    __syncthreads();
    // one reservation per bucket, a thread's all in flight together; a
    // bucket whose range would overflow keeps its pairs out and raises *err
    static_assert(kBktMax % kPartBS == 0, "buckets per thread");
    constexpr uint32_t kResPer = kBktMax / kPartBS;
    unsigned long long got[kResPer];
#pragma unroll
    for (uint32_t x = 0; x < kResPer; ++x) {
        const uint32_t b = threadIdx.x + x * kPartBS;
        const uint32_t c = b < nb ? s_cnt[b] : 0u;
        got[x] = 0ull;
        if (c) got[x] = atomicAdd(&pl->cur[b], (unsigned long long)c);
    }
    bool bad = false;
#pragma unroll
    for (uint32_t x = 0; x < kResPer; ++x) {
        const uint32_t b = threadIdx.x + x * kPartBS;
        if (b < nb) {
            const uint32_t c = s_cnt[b];
            uint64_t at = ~0ull;
            if (c) {
                at = pl->off[b] + got[x];
                if (at + c > pl->off[b + 1]) {
                    at = ~0ull;
                    bad = true;
                }
            }
            s_base[b] = at;
            s_res[b] = c;
            s_cnt[b] = 0;
        }
    }
    __syncthreads();
    for (uint64_t j0 = g0; j0 < g1; j0 += kPartBS)
        block_members(set_off, set_vtx, j0, g1, s_sb, s_sa, s_w, [&](uint32_t u, uint64_t j) {
            const uint32_t b = u >> shift;
            if (b >= nb) {  // not a vertex: the pool is corrupt
                bad = true;
                return;
            }
            const uint32_t r = atomicAdd(&s_cnt[b], 1u);
            const uint64_t at = s_base[b];
            // both walks see the same members, so r < s_res[b]; checked all
            // the same, as a write past the reservation would land in
            // another tile's range
            if (at != ~0ull && r < s_res[b]) tmp[at + r] = (unsigned long long)j << 32 | u;
            else bad = true;
        });
    if (bad) atomicOr(err, 1u);
}

__global__ __launch_bounds__(kPlaceBS) void inv_place_kernel(const unsigned long long* tmp,
                                                             const IndexPlan* pl, uint32_t nb,
                                                             uint32_t shift, uint32_t n,
                                                             const uint64_t* io, uint32_t* cursor,
                                                             uint32_t* inv_set, uint32_t* err) {
    __shared__ uint32_t s_cnt[kBktVtxMax];
    __shared__ uint32_t s_base[kBktVtxMax];
    __shared__ uint32_t s_pre[kBktMax + 1];  // the plan's first slice per bucket
    __shared__ uint32_t s_b;
    for (uint32_t b = threadIdx.x; b <= nb; b += kPlaceBS) s_pre[b] = pl->sl_pre[b];
    __syncthreads();
    const uint32_t nsl = s_pre[nb];
    // Workgroups go to the eight XCDs in turn (workgroup i to XCD i mod 8),
    // each with its own L2. With a grid of a multiple of eight, the slices
    // (in bucket order) are cut into eight ranges, one per XCD, so that the
    // list writes of a bucket meet in one L2 instead of eight partial lines.
    uint32_t t0 = blockIdx.x, tstep = gridDim.x, tend = nsl;
    if ((gridDim.x & 7u) == 0) {
        const uint32_t x = blockIdx.x & 7u;
        t0 = (uint32_t)((uint64_t)nsl * x / 8) + (blockIdx.x >> 3);
        tend = (uint32_t)((uint64_t)nsl * (x + 1) / 8);
        tstep = gridDim.x >> 3;
    }
    bool bad = false;
    for (uint32_t t = t0; t < tend; t += tstep) {
        if (threadIdx.x == 0) {  // the bucket of slice t: the last b with sl_pre[b] <= t
            uint32_t a = 0, z = nb;
            while (z - a > 1) {
                const uint32_t mid = (a + z) >> 1;
                if (s_pre[mid] <= t) a = mid; else z = mid;
            }
            s_b = a;
        }
        __syncthreads();
        const uint32_t b = s_b;
        const uint64_t bo = pl->off[b], be = pl->off[b + 1];
        const uint64_t e0 = bo + (uint64_t)(t - s_pre[b]) * kSlice;
        const uint64_t e1 = min(be, e0 + kSlice);
        const bool whole = be - bo <= kSlice;
        const uint32_t v0 = b << shift;
        const uint32_t wn = min(1u << shift, n - v0);
        for (uint32_t i = threadIdx.x; i < wn; i += kPlaceBS) s_cnt[i] = 0;
        __syncthreads();
        if (!whole) {
            for (uint64_t e = e0 + threadIdx.x; e < e1; e += kPlaceBS) {
                const uint32_t ul = (uint32_t)tmp[e] - v0;
                if (ul < wn) atomicAdd(&s_cnt[ul], 1u);
            }
            __syncthreads();
            for (uint32_t i = threadIdx.x; i < wn; i += kPlaceBS) {
                const uint32_t c = s_cnt[i];
                s_base[i] = c ? atomicAdd(&cursor[v0 + i], c) : 0u;
                s_cnt[i] = 0;
            }
            __syncthreads();
        }
        constexpr uint64_t kRound = (uint64_t)kPlaceBS * kPlaceBatch;
        for (uint64_t r0 = e0; r0 < e1; r0 += kRound) {
            unsigned long long p[kPlaceBatch];
#pragma unroll
            for (uint32_t x = 0; x < kPlaceBatch; ++x) {
                const uint64_t e = r0 + (uint64_t)x * kPlaceBS + threadIdx.x;
                p[x] = tmp[e < e1 ? e : e1 - 1];
            }
            uint64_t d[kPlaceBatch], de[kPlaceBatch];
            bool ok[kPlaceBatch];
#pragma unroll
            for (uint32_t x = 0; x < kPlaceBatch; ++x) {
                const uint32_t u = (uint32_t)p[x];
                const uint32_t ul = u - v0;
                ok[x] = r0 + (uint64_t)x * kPlaceBS + threadIdx.x < e1;
                bad |= ok[x] && ul >= wn;
                ok[x] = ok[x] && ul < wn;
                const uint32_t uc = ok[x] ? u : v0;
                const uint32_t r = ok[x] ? atomicAdd(&s_cnt[ul], 1u) + (whole ? 0u : s_base[ul])
                                         : 0u;
                d[x] = io[uc] + r;
                de[x] = io[uc + 1];
            }
#pragma unroll
            for (uint32_t x = 0; x < kPlaceBatch; ++x) {
                if (!ok[x]) continue;
                if (d[x] < de[x]) inv_set[d[x]] = (uint32_t)(p[x] >> 32);
                else bad = true;
            }
        }
        __syncthreads();
    }
    if (bad) atomicOr(err, 1u);
}

// ---- index build from the sets alone (the counting build)
//
// For a segment whose sets' counts are not all known, the bucket ranges come
// from a histogram of the entries instead of the scanned offsets, and every
// bucket is one slice: its workgroup sees all the entries of its vertices,
// counts them, scans them into list offsets, writes the offsets and counts
// of its vertices and places their lists (ranks from LDS counters, no
// global atomic per entry).
constexpr uint32_t kHistBS = 1024;

__global__ __launch_bounds__(kHistBS) void inv_hist_kernel(const uint64_t* set_off, uint64_t lo,
                                                           uint64_t hi, const uint32_t* set_vtx,
                                                           uint32_t shift, uint32_t nb,
                                                           IndexPlan* pl) {
    __shared__ uint32_t s_h[kBktMax];
    for (uint32_t b = threadIdx.x; b < nb; b += kHistBS) s_h[b] = 0u;
    __syncthreads();
    const uint64_t a0 = set_off[lo], a1 = set_off[hi];
    const uint64_t stride = (uint64_t)gridDim.x * kHistBS;
    constexpr uint32_t kB = 8;
    for (uint64_t e0 = a0 + (uint64_t)blockIdx.x * kHistBS + threadIdx.x; e0 < a1;
         e0 += stride * kB) {
        uint32_t u[kB];
#pragma unroll
        for (uint32_t x = 0; x < kB; ++x) {
            const uint64_t e = e0 + x * stride;
            u[x] = set_vtx[e < a1 ? e : e0];
        }
#pragma unroll
        for (uint32_t x = 0; x < kB; ++x) {
            const uint32_t b = u[x] >> shift;
            if (e0 + x * stride < a1 && b < nb) atomicAdd(&s_h[b], 1u);
        }
    }
    __syncthreads();
    for (uint32_t b = threadIdx.x; b < nb; b += kHistBS)
        if (s_h[b]) atomicAdd(&pl->tot[b], s_h[b]);
}

// Bucket ranges as the exclusive scan of the totals, one slice per bucket
// (empty ones too: their vertices still get offsets). A segment beyond the
// pair buffer gets empty buckets and raises *err, as in inv_plan_kernel.
__global__ __launch_bounds__(1024) void inv_plan_counts_kernel(uint32_t nb, uint64_t cap,
                                                               IndexPlan* pl, uint32_t* err) {
    __shared__ uint64_t s_w[1024 / kWave];
    __shared__ uint64_t s_carry;
    uint64_t part = 0;
    for (uint32_t b = threadIdx.x; b < nb; b += 1024) part += pl->tot[b];
    uint64_t excl;
    const uint64_t total = block_excl_scan64(part, &excl, s_w);
    const bool fits = total <= cap;
    if (threadIdx.x == 0) {
        s_carry = 0;
        if (!fits) atomicOr(err, 1u);
    }
    __syncthreads();
    for (uint32_t c = 0; c <= nb; c += 1024) {
        const uint32_t b = c + threadIdx.x;
        const uint64_t t = b < nb && fits ? pl->tot[b] : 0;
        const uint64_t tot = block_excl_scan64(t, &excl, s_w);
        const uint64_t carry = s_carry;
        if (b <= nb) {
            pl->off[b] = carry + excl;
            pl->sl_pre[b] = b;
        }
        if (b < nb) pl->cur[b] = 0;
        __syncthreads();
        if (threadIdx.x == 0) s_carry = carry + tot;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kPlaceBS) void inv_place_counts_kernel(
    const unsigned long long* tmp, const IndexPlan* pl, uint32_t nb, uint32_t shift, uint32_t n,
    const uint64_t* seg_base, uint64_t* io, const uint32_t* base, uint32_t* counts,
    uint32_t* inv_set, uint32_t* err) {
    static_assert(kBktVtxMax == 4 * kPlaceBS, "four vertices per thread");
    __shared__ uint32_t s_cnt[kBktVtxMax];  // counts, then ranks
    __shared__ uint32_t s_ex[kBktVtxMax];   // list offsets within the bucket
    __shared__ uint64_t s_w[kPlaceBS / kWave];
    const uint64_t sb = *seg_base;
    // buckets in eight ranges, one per XCD, as in inv_place_kernel
    uint32_t t0 = blockIdx.x, tstep = gridDim.x, tend = nb;
    if ((gridDim.x & 7u) == 0) {
        const uint32_t x = blockIdx.x & 7u;
        t0 = (uint32_t)((uint64_t)nb * x / 8) + (blockIdx.x >> 3);
        tend = (uint32_t)((uint64_t)nb * (x + 1) / 8);
        tstep = gridDim.x >> 3;
    }
    bool bad = false;
    for (uint32_t b = t0; b < tend; b += tstep) {
        const uint64_t bo = pl->off[b], be = pl->off[b + 1];
        const uint32_t v0 = b << shift;
        const uint32_t wn = min(1u << shift, n - v0);
        for (uint32_t i = threadIdx.x; i < kBktVtxMax; i += kPlaceBS) s_cnt[i] = 0u;
        __syncthreads();
        constexpr uint64_t kRound = (uint64_t)kPlaceBS * kPlaceBatch;
        for (uint64_t r0 = bo; r0 < be; r0 += kRound) {
            uint32_t u[kPlaceBatch];
#pragma unroll
            for (uint32_t x = 0; x < kPlaceBatch; ++x) {
                const uint64_t e = r0 + (uint64_t)x * kPlaceBS + threadIdx.x;
                u[x] = (uint32_t)tmp[e < be ? e : be - 1];
            }
#pragma unroll
            for (uint32_t x = 0; x < kPlaceBatch; ++x) {
                const uint32_t ul = u[x] - v0;
                if (r0 + (uint64_t)x * kPlaceBS + threadIdx.x < be) {
                    if (ul < wn) atomicAdd(&s_cnt[ul], 1u);
                    else bad = true;
                }
            }
        }
        __syncthreads();
        // the counts' exclusive scan, four vertices per thread
        const uint32_t i0 = 4u * threadIdx.x;
        uint32_t c[4], sum = 0;
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            c[j] = i0 + j < wn ? s_cnt[i0 + j] : 0u;
            sum += c[j];
        }
        uint64_t excl;
        (void)block_excl_scan64(sum, &excl, s_w);
        uint32_t run = (uint32_t)excl;
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            const uint32_t i = i0 + j;
            if (i < wn) {
                s_ex[i] = run;
                io[v0 + i] = sb + bo + run;
                counts[v0 + i] = base[v0 + i] + c[j];
            }
            run += c[j];
        }
        if (b == nb - 1 && threadIdx.x == 0) io[n] = sb + be;
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) s_cnt[i0 + j] = 0u;
        __syncthreads();
        // the lists: rank within the vertex's list from the LDS counters
        for (uint64_t r0 = bo; r0 < be; r0 += kRound) {
            unsigned long long p[kPlaceBatch];
#pragma unroll
            for (uint32_t x = 0; x < kPlaceBatch; ++x) {
                const uint64_t e = r0 + (uint64_t)x * kPlaceBS + threadIdx.x;
                p[x] = tmp[e < be ? e : be - 1];
            }
#pragma unroll
            for (uint32_t x = 0; x < kPlaceBatch; ++x) {
                const uint32_t ul = (uint32_t)p[x] - v0;
                if (r0 + (uint64_t)x * kPlaceBS + threadIdx.x < be && ul < wn) {
                    const uint64_t at = bo + s_ex[ul] + atomicAdd(&s_cnt[ul], 1u);
                    if (at < be) inv_set[sb + at] = (uint32_t)(p[x] >> 32);
                    else bad = true;
                }
            }
        }
        __syncthreads();
    }
    if (bad) atomicOr(err, 1u);
}

__global__ __launch_bounds__(256) void count_entries_kernel(const uint32_t* set_vtx, uint64_t P,
                                                            uint32_t* counts) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P; t += stride)
        atomicAdd(&counts[set_vtx[t]], 1u);
}

// counts[v] += the number of bitmaps b in [b_lo, b_hi) holding v: workgroup
// (word block wb, bitmap chunk c) sums the 2048 vertices of word block wb over
// kColChunk bitmaps of chunk c, then one atomic per vertex with a nonzero sum.
__global__ __launch_bounds__(kColBS) void dense_count_kernel(const uint32_t* bits, uint32_t words,
                                                             uint32_t b_lo, uint32_t b_hi,
                                                             uint32_t n, uint32_t* counts) {
    __shared__ uint32_t lds[4 * 2048];
    const uint32_t wblocks = (words + 63) / 64;
    const uint32_t wb = blockIdx.x % wblocks, c = blockIdx.x / wblocks;
    const uint32_t i0 = b_lo + c * kColChunk;
    const uint32_t cnt = min(kColChunk, b_hi - i0);
    uint32_t out[8];
    col_sums(bits, words, 64u * wb, cnt, [&](uint32_t i) { return i0 + i; }, lds, out);
#pragma unroll
    for (uint32_t q = 0; q < 8; ++q) {
        const uint32_t v = 2048u * wb + 8u * threadIdx.x + q;
        if (v < n && out[q]) atomicAdd(&counts[v], out[q]);
    }
}

// Seeds' bits in a vertex bitmap.
__global__ __launch_bounds__(256) void mark_seeds_kernel(const uint32_t* seeds, uint32_t k,
                                                         uint32_t* mark) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < k) atomicOr(&mark[seeds[i] >> 5], 1u << (seeds[i] & 31));
}

// Sets holding a marked vertex: an entry of a marked vertex finds its set j
// (the last j with set_off[j] <= t, so empty sets are never chosen), sets
// j's bit in hit, and counts j the first time that bit is set.
__global__ __launch_bounds__(256) void cover_count_kernel(const uint64_t* set_off,
                                                          const uint32_t* set_vtx,
                                                          uint64_t n_sets, const uint32_t* mark,
                                                          uint32_t* hit,
                                                          unsigned long long* count) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t P = set_off[n_sets];
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P; t += stride) {
        const uint32_t v = set_vtx[t];
        if (!((mark[v >> 5] >> (v & 31)) & 1u)) continue;
        uint64_t a = 0, z = n_sets;  // first j in [0, n_sets] with set_off[j] > t, minus one
        while (a < z) {
            const uint64_t mid = a + ((z - a) >> 1);
            if (set_off[mid] > t) z = mid; else a = mid + 1;
        }
        const uint64_t j = a - 1;
        const uint32_t bit = 1u << (j & 31);
        if (!(atomicOr(&hit[j >> 5], bit) & bit)) atomicAdd(count, 1ull);
    }
}

__global__ __launch_bounds__(256) void count_sets_kernel(const uint64_t* set_off, uint64_t lo,
                                                         uint64_t hi, const uint32_t* set_vtx,
                                                         uint32_t* counts) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t a = set_off[lo], b = set_off[hi];
    // eight loads per thread in flight before their atomics
    constexpr uint32_t kB = 8;
    for (uint64_t t0 = a + (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t0 < b;
         t0 += stride * kB) {
        uint32_t u[kB];
#pragma unroll
        for (uint32_t x = 0; x < kB; ++x) {
            const uint64_t t = t0 + x * stride;
            u[x] = set_vtx[t < b ? t : t0];
        }
#pragma unroll
        for (uint32_t x = 0; x < kB; ++x)
            if (t0 + x * stride < b) atomicAdd(&counts[u[x]], 1u);
    }
}

// dst[v] += src[v] for v < n, four at a time where they fit.
__global__ __launch_bounds__(256) void add_counts_kernel(const uint32_t* src, uint32_t* dst,
                                                         uint32_t n) {
    const uint32_t stride = gridDim.x * 256;
    const uint32_t n4 = n >> 2;
    for (uint32_t x = blockIdx.x * 256 + threadIdx.x; x < n4; x += stride) {
        const uint4 a = reinterpret_cast<const uint4*>(src)[x];
        uint4 b = reinterpret_cast<const uint4*>(dst)[x];
        b.x += a.x;
        b.y += a.y;
        b.z += a.z;
        b.w += a.w;
        reinterpret_cast<uint4*>(dst)[x] = b;
    }
    const uint32_t v = (n4 << 2) + blockIdx.x * 256 + threadIdx.x;
    if (blockIdx.x * 256 + threadIdx.x < 4u && v < n) dst[v] += src[v];
}

__global__ __launch_bounds__(256) void validate_kernel(const uint64_t* set_off, uint64_t n_sets,
                                                       const uint32_t* set_vtx, uint32_t n,
                                                       uint32_t* flag) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    const uint64_t P = set_off[n_sets];
    for (uint64_t j = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; j < n_sets; j += stride)
        if (set_off[j] > set_off[j + 1]) atomicOr(flag, 1u);
    for (uint64_t t = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; t < P; t += stride)
        if (set_vtx[t] >= n) atomicOr(flag, 2u);
}

// Bitonic sort of buf[0..N) (N a power of two) by one wave; ascending.
__device__ __forceinline__ void wave_bitonic(uint32_t* buf, uint32_t N) {
    const uint32_t lane = threadIdx.x;
    for (uint32_t k = 2; k <= N; k <<= 1) {
        for (uint32_t j = k >> 1; j > 0; j >>= 1) {
            for (uint32_t i = lane; i < N; i += kWave) {
                const uint32_t p = i ^ j;
                if (p > i) {
                    const uint32_t a = buf[i], b = buf[p];
                    const bool asc = (i & k) == 0;
                    if ((a > b) == asc) {
                        buf[i] = b;
                        buf[p] = a;
                    }
                }
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(64) void sort_small_kernel(const uint64_t* set_off, uint32_t n_sets,
                                                        uint32_t* set_vtx, uint32_t* big_list,
                                                        uint32_t* big_n) {
    __shared__ uint32_t buf[kSortSmallMax];
    const uint32_t lane = threadIdx.x;
    for (uint32_t j = blockIdx.x; j < n_sets; j += gridDim.x) {
        const uint64_t a = set_off[j];
        const uint32_t sz = (uint32_t)(set_off[j + 1] - a);
        if (sz <= 1) continue;
        if (sz > kSortSmallMax) {
            if (lane == 0) big_list[atomicAdd(big_n, 1u)] = j;
            continue;
        }
        uint32_t N = 2;
        while (N < sz) N <<= 1;
        for (uint32_t i = lane; i < N; i += kWave) buf[i] = i < sz ? set_vtx[a + i] : kEmpty;
        __syncthreads();
        wave_bitonic(buf, N);
        for (uint32_t i = lane; i < sz; i += kWave) set_vtx[a + i] = buf[i];
        __syncthreads();
    }
}

// One block per big set, bitonic network over a padded copy in scratch.
__global__ __launch_bounds__(1024) void sort_big_kernel(const uint64_t* set_off,
                                                        uint32_t* set_vtx, uint32_t j,
                                                        uint32_t* scratch, uint32_t N) {
    const uint64_t a = set_off[j];
    const uint32_t sz = (uint32_t)(set_off[j + 1] - a);
    for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) scratch[i] = i < sz ? set_vtx[a + i] : kEmpty;
    __threadfence_block();
    __syncthreads();
    for (uint32_t k = 2; k <= N; k <<= 1) {
        for (uint32_t jj = k >> 1; jj > 0; jj >>= 1) {
            for (uint32_t i = threadIdx.x; i < N; i += blockDim.x) {
                const uint32_t p = i ^ jj;
                if (p > i) {
                    const uint32_t x = scratch[i], y = scratch[p];
                    const bool asc = (i & k) == 0;
                    if ((x > y) == asc) {
                        scratch[i] = y;
                        scratch[p] = x;
                    }
                }
            }
            __threadfence_block();
            __syncthreads();
        }
    }
    for (uint32_t i = threadIdx.x; i < sz; i += blockDim.x) set_vtx[a + i] = scratch[i];
}

__global__ __launch_bounds__(256) void philox_kernel(const uint32_t* ctr, uint64_t count,
                                                     uint64_t key, uint32_t* out) {
    const uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const uint4 c = reinterpret_cast<const uint4*>(ctr)[i];
    const Philox4 r = philox10(c.x, c.y, c.z, c.w, (uint32_t)key, (uint32_t)(key >> 32));
    reinterpret_cast<uint4*>(out)[i] = make_uint4(r.x, r.y, r.z, r.w);
}

uint32_t grid_for(uint64_t work, uint32_t per_block, uint32_t cap) {
    uint64_t g = (work + per_block - 1) / per_block;
    if (g == 0) g = 1;
    if (g > cap) g = cap;
    return (uint32_t)g;
}

}  // namespace

uint64_t scan_tmp_entries(uint64_t N) { return (N + kScanTile - 1) / kScanTile + 1; }

hipError_t launch_scan_u32(const uint32_t* in, const uint32_t* sub, uint64_t* out, uint64_t N,
                           uint64_t base, const uint64_t* base_dev, uint64_t* tile_tmp,
                           hipStream_t st) {
    if (N == 0) return hipErrorInvalidValue;
    const uint64_t tiles = (N + kScanTile - 1) / kScanTile;
    if (tiles > 0x7FFFFFFFull) return hipErrorInvalidValue;
    if (sub) {
        hipLaunchKernelGGL(scan_tiles_kernel<true>, dim3((uint32_t)tiles), dim3(kScanBS), 0, st,
                           in, sub, N, tile_tmp);
    } else {
        hipLaunchKernelGGL(scan_tiles_kernel<false>, dim3((uint32_t)tiles), dim3(kScanBS), 0, st,
                           in, sub, N, tile_tmp);
    }
    hipLaunchKernelGGL(scan_sums_kernel, dim3(1), dim3(1024), 0, st, tile_tmp, tiles);
    if (sub) {
        hipLaunchKernelGGL(scan_apply_kernel<true>, dim3((uint32_t)tiles), dim3(kScanBS), 0, st,
                           in, sub, N, tile_tmp, out, base, base_dev);
    } else {
        hipLaunchKernelGGL(scan_apply_kernel<false>, dim3((uint32_t)tiles), dim3(kScanBS), 0, st,
                           in, sub, N, tile_tmp, out, base, base_dev);
    }
    return hipGetLastError();
}

hipError_t launch_compact(const uint32_t* stage, const uint64_t* stage_off,
                          const uint64_t* set_off, uint64_t lo, uint32_t count,
                          uint32_t* set_vtx, hipStream_t st) {
    if (count == 0) return hipSuccess;
    const uint32_t blocks = (count + kWave - 1) / kWave;
    hipLaunchKernelGGL(compact_kernel, dim3(blocks), dim3(kWave), 0, st, stage, stage_off,
                       set_off, lo, count, set_vtx);
    return hipGetLastError();
}

hipError_t launch_inv_scatter(const uint64_t* set_off, const uint32_t* set_vtx, uint64_t lo,
                              uint32_t count, const uint64_t* inv_off, uint32_t* cursor,
                              uint32_t* inv_set, uint32_t* err, hipStream_t st) {
    if (count == 0) return hipSuccess;
    const uint32_t blocks = (count + kWave - 1) / kWave;
    hipLaunchKernelGGL(inv_scatter_kernel, dim3(blocks), dim3(kWave), 0, st, set_off, set_vtx, lo,
                       count, inv_off, cursor, inv_set, err);
    return hipGetLastError();
}

uint32_t index_bucket_shift(uint32_t n) {
    uint32_t shift = 0;
    while ((((uint64_t)n + (1ull << shift) - 1) >> shift) > kBktMax) ++shift;
    return (1u << shift) <= kBktVtxMax ? shift : 32u;
}

hipError_t launch_inv_partitioned(const uint64_t* set_off, const uint32_t* set_vtx, uint64_t lo,
                                  uint32_t count, uint32_t tile_groups, uint32_t n,
                                  uint32_t shift, const uint64_t* inv_off, IndexPlan* pl,
                                  unsigned long long* tmp, uint64_t cap, uint32_t* cursor,
                                  uint32_t* inv_set, uint32_t* err, int device, hipStream_t st) {
    if (count == 0) return hipSuccess;
    if (shift >= 32 || tile_groups == 0) return hipErrorInvalidValue;
    const uint32_t nb = (uint32_t)(((uint64_t)n + (1ull << shift) - 1) >> shift);
    hipLaunchKernelGGL(inv_plan_kernel, dim3(1), dim3(1024), 0, st, inv_off, n, shift, nb, cap, pl,
                       err);
    const uint64_t tile = (uint64_t)tile_groups * kPartTile;
    const uint64_t tiles = (count + tile - 1) / tile;
    hipLaunchKernelGGL(inv_part_kernel, dim3((uint32_t)tiles), dim3(kPartBS), 0, st, set_off,
                       set_vtx, lo, count, tile_groups, shift, nb, pl, tmp, err);
    // slices: at most cap / kSlice + nb; the grid strides over them
    const uint64_t sl_ub = cap / kSlice + nb;
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    uint64_t grid = std::min<uint64_t>(sl_ub, (uint64_t)cus * 8);
    if (grid >= 8) grid &= ~7ull;  // a multiple of the XCD count
    hipLaunchKernelGGL(inv_place_kernel, dim3((uint32_t)std::max<uint64_t>(grid, 1)),
                       dim3(kPlaceBS), 0, st, tmp, pl, nb, shift, n, inv_off, cursor, inv_set,
                       err);
    return hipGetLastError();
}

hipError_t launch_inv_counting(const uint64_t* set_off, const uint32_t* set_vtx, uint64_t lo,
                               uint32_t count, uint32_t tile_groups, uint32_t n, uint32_t shift,
                               uint64_t* inv_off, const uint32_t* base, uint32_t* counts,
                               IndexPlan* pl, unsigned long long* tmp, uint64_t cap,
                               uint32_t* inv_set, uint32_t* err, int device, hipStream_t st) {
    if (count == 0) return hipSuccess;
    if (shift >= 32 || tile_groups == 0) return hipErrorInvalidValue;
    const uint32_t nb = (uint32_t)(((uint64_t)n + (1ull << shift) - 1) >> shift);
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    hipError_t e = hipMemsetAsync(pl->tot, 0, (uint64_t)nb * 4, st);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(inv_hist_kernel, dim3((uint32_t)cus * 2), dim3(kHistBS), 0, st, set_off,
                       lo, lo + count, set_vtx, shift, nb, pl);
    hipLaunchKernelGGL(inv_plan_counts_kernel, dim3(1), dim3(1024), 0, st, nb, cap, pl, err);
    const uint64_t tile = (uint64_t)tile_groups * kPartTile;
    const uint64_t tiles = (count + tile - 1) / tile;
    hipLaunchKernelGGL(inv_part_kernel, dim3((uint32_t)tiles), dim3(kPartBS), 0, st, set_off,
                       set_vtx, lo, count, tile_groups, shift, nb, pl, tmp, err);
    uint64_t grid = std::min<uint64_t>(nb, (uint64_t)cus * 8);
    if (grid >= 8) grid &= ~7ull;  // a multiple of the XCD count
    hipLaunchKernelGGL(inv_place_counts_kernel, dim3((uint32_t)std::max<uint64_t>(grid, 1)),
                       dim3(kPlaceBS), 0, st, tmp, pl, nb, shift, n, set_off + lo, inv_off, base,
                       counts, inv_set, err);
    return hipGetLastError();
}

hipError_t launch_count_entries(const uint32_t* set_vtx, uint64_t P, uint32_t* counts,
                                hipStream_t st) {
    if (P == 0) return hipSuccess;
    hipLaunchKernelGGL(count_entries_kernel, dim3(grid_for(P, 256 * 8, 8192)), dim3(256), 0, st,
                       set_vtx, P, counts);
    return hipGetLastError();
}

hipError_t launch_add_counts(const uint32_t* src, uint32_t* dst, uint32_t n, hipStream_t st) {
    if (n == 0) return hipSuccess;
    const uint32_t n4 = (n + 3) / 4;
    hipLaunchKernelGGL(add_counts_kernel, dim3(std::min<uint32_t>((n4 + 255) / 256, 4096u)),
                       dim3(256), 0, st, src, dst, n);
    return hipGetLastError();
}

hipError_t launch_count_sets(const uint64_t* set_off, uint64_t lo, uint64_t hi,
                             const uint32_t* set_vtx, uint32_t* counts, hipStream_t st) {
    if (hi <= lo) return hipSuccess;
    hipLaunchKernelGGL(count_sets_kernel, dim3(2048), dim3(256), 0, st, set_off, lo, hi, set_vtx,
                       counts);
    return hipGetLastError();
}

hipError_t launch_dense_count(const uint32_t* bits, uint32_t words, uint32_t b_lo, uint32_t b_hi,
                              uint32_t n, uint32_t* counts, hipStream_t st) {
    if (b_hi <= b_lo) return hipSuccess;
    const uint32_t wblocks = (words + 63) / 64;
    const uint32_t chunks = (b_hi - b_lo + kColChunk - 1) / kColChunk;
    hipLaunchKernelGGL(dense_count_kernel, dim3(wblocks * chunks), dim3(kColBS), 0, st, bits,
                       words, b_lo, b_hi, n, counts);
    return hipGetLastError();
}

hipError_t launch_cover_count(const uint64_t* set_off, const uint32_t* set_vtx, uint64_t n_sets,
                              const uint32_t* seeds, uint32_t k, uint32_t* mark, uint32_t* hit,
                              unsigned long long* count, hipStream_t st) {
    hipLaunchKernelGGL(mark_seeds_kernel, dim3((k + 255) / 256), dim3(256), 0, st, seeds, k, mark);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || n_sets == 0) return e;
    hipLaunchKernelGGL(cover_count_kernel, dim3(2048), dim3(256), 0, st, set_off, set_vtx, n_sets,
                       mark, hit, count);
    return hipGetLastError();
}

hipError_t launch_validate_pool(const uint64_t* set_off, uint64_t n_sets, const uint32_t* set_vtx,
                                uint32_t n, uint32_t* flag, hipStream_t st) {
    hipLaunchKernelGGL(validate_kernel, dim3(2048), dim3(256), 0, st, set_off, n_sets, set_vtx, n,
                       flag);
    return hipGetLastError();
}

hipError_t launch_sort_small(const uint64_t* set_off, uint32_t n_sets, uint32_t* set_vtx,
                             uint32_t* big_list, uint32_t* big_n, hipStream_t st) {
    if (n_sets == 0) return hipSuccess;
    hipLaunchKernelGGL(sort_small_kernel, dim3(grid_for(n_sets, 1, 16384)), dim3(kWave), 0, st,
                       set_off, n_sets, set_vtx, big_list, big_n);
    return hipGetLastError();
}

hipError_t launch_sort_big(const uint64_t* set_off, uint32_t* set_vtx, uint32_t j,
                           uint32_t n_pow2, uint32_t* scratch, hipStream_t st) {
    hipLaunchKernelGGL(sort_big_kernel, dim3(1), dim3(1024), 0, st, set_off, set_vtx, j, scratch,
                       n_pow2);
    return hipGetLastError();
}

hipError_t launch_philox(const uint32_t* ctr, uint64_t count, uint64_t key, uint32_t* out,
                         hipStream_t st) {
    if (count == 0) return hipSuccess;
    hipLaunchKernelGGL(philox_kernel, dim3((uint32_t)((count + 255) / 256)), dim3(256), 0, st, ctr,
                       count, key, out);
    return hipGetLastError();
}

}  // namespace imm
