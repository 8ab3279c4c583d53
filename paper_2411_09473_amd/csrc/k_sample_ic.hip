// k_sample_ic.hip -- IC reverse-BFS RRR sampling with fused occurrence counts
// (Generate_RRRsets with in-place counter updates, Algorithm 3; IC model,
// Section II-A).
//
// Three kernels share the work of one sampling round:
//  * ic_lane: a wave takes 4 x 64 sample ids at a time. Each lane draws the root
//    of its own sample and flips the coins of the root's in-edges (roots of
//    in-degree <= kLaneDegCap); a root with no live in-edge is a complete set
//    {root}, stored at once (at low edge probabilities that is most samples).
//    Every other sample index goes to a pending list.
//  * ic_bfs<TEAM>: a team of TEAM waves (one workgroup) takes one pending
//    sample at a time, so samples of very different cost spread evenly over
//    the GPU. The set doubles as the BFS queue and lives in LDS together with
//    an open-addressing hash of visited vertices. Each BFS level takes up to
//    64*TEAM queued vertices and the team sweeps their in-edges in aligned
//    groups of four: one Philox call yields the four coins of a group and one
//    16-byte load its four thresholds; sources are read only for live edges,
//    which each wave collects and follows in batches.
//    A set that outgrows LDS is abandoned (no side effects) and its sample
//    index deferred.
//  * ic_large<BS>: one workgroup of BS (256 or 1024) threads per deferred
//    sample (a giant set, whose BFS levels are wide), with a visited bitmap and a
//    queue in device memory (one slot per workgroup, reset sparsely). Queues
//    hold a bounded number of members; the rare set that outgrows one is
//    redone by a second launch over a few slots with queues of n. A slot
//    is only ever touched by its own workgroup, so workgroup barriers order
//    every access; no device-scope fence is used (on this GPU such a fence
//    writes back and invalidates the L2 of the whole XCD).
// Finished sets are staged in chunks reserved from a bump cursor; their
// members' counts are incremented right away. A set that finds the staging
// buffer full is listed for a retry after the host grows it.
#include "device_common.hpp"
#include "imm_internal.hpp"

namespace imm {

namespace {

constexpr uint32_t kLaneDegCap = 32;  // roots tried one per lane up to this in-degree
constexpr uint32_t kStageChunk = kIcStageChunk;
constexpr uint32_t kLargePage = 1u << 16;  // groups per start-bitmap page of a giant-set workgroup
constexpr uint32_t kBfsLiveBuf = 64;       // buffered live edges per wave, BFS team
constexpr uint32_t kLargeLiveBuf = 256;    // ... giant-set workgroup

// LDS shape of a BFS team of TEAM waves: members kept on chip and a visited
// hash of twice that many slots (load factor <= 1/2).
template <uint32_t TEAM>
struct Team {
    static constexpr uint32_t BS = kWave * TEAM;
    static constexpr uint32_t CAP = 256 * TEAM;
    static constexpr uint32_t HBITS = TEAM == 1 ? 9 : (TEAM == 2 ? 10 : 11);
    static constexpr uint32_t HSIZE = 1u << HBITS;
    static constexpr uint32_t PAGE = 4096 * TEAM;  // groups per start-bitmap page
    static_assert(2 * CAP == HSIZE, "hash holds twice the member capacity");
    static_assert(CAP <= kStageChunk, "a set fits one staging chunk");
};

__device__ __forceinline__ uint32_t lds_load(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The task whose positions hold pos: the last q with pre[q] <= pos
// (pre[0] = 0, non-decreasing, ntask + 1 entries).
__device__ __forceinline__ uint32_t task_of(const uint32_t* pre, uint32_t ntask, uint32_t pos) {
    uint32_t lo = 0, hi = ntask;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (pre[mid] <= pos) lo = mid; else hi = mid;
    }
    return lo;
}

// Staging space of one workgroup: the rest of its current chunk.
struct Stager {
    uint64_t base = 0;
    uint32_t left = 0;
};

// Reserve `need` (<= kStageChunk) staging entries; called by the whole
// workgroup alike. False when the staging buffer is full.
__device__ __forceinline__ bool stage_reserve(Stager& c, uint32_t need, uint64_t* off,
                                              unsigned long long* s_chunk, const SampleOut& o) {
    if (need > c.left) {
        if (threadIdx.x == 0) *s_chunk = atomicAdd(o.cursor, (unsigned long long)kStageChunk);
        __syncthreads();
        c.base = *s_chunk;
        c.left = kStageChunk;
        __syncthreads();
        if (c.base + kStageChunk > o.stage_cap) {
            c.left = 0;
            return false;
        }
    }
    *off = c.base + (kStageChunk - c.left);
    c.left -= need;
    return true;
}

// One chunk of a BFS level: up to BS queued vertices, one per thread. Their
// in-edges are swept in aligned groups of four edges (one Philox call gives
// the four coins of a group). The chunk's groups are numbered 0 .. G-1; the
// k-th entry with in-edges (rank k) owns groups [a_k, a_k + ng_k), which are
// edge groups g0_k, g0_k + 1, ... of its column [beg_k, end_k), and its layout
// record is s_ent[k] = (a_k, g0_k, beg_k, end_k).
//
// Owner lookup without a search per group: the groups are swept in pages of
// PAGE groups, and an LDS bitmap holds one bit per group of the page, set
// where an entry starts. A page is split into one contiguous span per wave (a
// multiple of 64 groups); the wave finds the owner of its span's first group
// once (a wave-wide search over the entries' first groups), and from there
// the owner of any group is that rank plus the starts between: one 64-bit
// popcount per row of 64 groups.
struct LevelChunk {
    uint32_t G;   // groups of the chunk
    uint32_t ne;  // entries with at least one in-edge
    uint32_t a;   // this thread's entry: first group ...
    uint32_t ng;  // ... and group count (0 past the chunk's entries)
};

// Span of each wave's share of a page of pn groups (a multiple of 64).
template <uint32_t BS>
__device__ __forceinline__ uint32_t page_span(uint32_t pn) {
    constexpr uint32_t NW = BS / kWave;
    return (((pn + NW - 1u) / NW) + kWave - 1u) & ~(kWave - 1u);
}

// Block-wide layout scan: the exclusive prefix sum of ng over the threads
// (*a), and the rank of the thread among threads with ng > 0 (*rank, from a
// ballot). Returns (sum of ng, count with ng > 0). s_wsum holds 2 * BS / 64
// words.
template <uint32_t BS>
__device__ __forceinline__ uint2 block_layout_scan(uint32_t ng, uint32_t* a, uint32_t* rank,
                                                   uint32_t* s_wsum) {
    constexpr uint32_t NW = BS / kWave;
    const uint32_t tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const uint32_t incl = wave_incl_scan(ng);
    const uint64_t nz = __ballot(ng != 0u);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(nz >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)nz, 0u));
    const uint32_t wcount = (uint32_t)__popcll(nz);
    if (NW == 1) {
        *a = incl - ng;
        *rank = below;
        return make_uint2(__shfl(incl, kWave - 1, kWave), wcount);
    }
    if (lane == kWave - 1) {
        s_wsum[w] = incl;
        s_wsum[NW + w] = wcount;
    }
    __syncthreads();
    if (NW <= 4) {
        uint32_t bu = 0, bv = 0, tu = 0, tv = 0;
#pragma unroll
        for (uint32_t i = 0; i < NW; ++i) {
            const uint32_t x = s_wsum[i], y = s_wsum[NW + i];
            if (i < w) {
                bu += x;
                bv += y;
            }
            tu += x;
            tv += y;
        }
        *a = bu + incl - ng;
        *rank = bv + below;
        return make_uint2(tu, tv);
    }
    // many waves: scan the wave totals across the lanes of every wave
    const uint32_t su = wave_incl_scan(lane < NW ? s_wsum[lane] : 0u);
    const uint32_t sv = wave_incl_scan(lane < NW ? s_wsum[NW + lane] : 0u);
    const uint32_t bu = __shfl(su, (int)(w ? w - 1 : 0), kWave);
    const uint32_t bv = __shfl(sv, (int)(w ? w - 1 : 0), kWave);
    *a = (w ? bu : 0u) + incl - ng;
    *rank = (w ? bv : 0u) + below;
    return make_uint2(__shfl(su, NW - 1, kWave), __shfl(sv, NW - 1, kWave));
}

// Lay out the chunk of queue entries [head, head + nb) (nb <= BS) and set the
// start bits of its first page (the bitmap must be all zero on entry). Adds
// the entries' in-degrees to *edges. The caller synchronises before the sweep.
template <uint32_t BS, uint32_t PAGE>
__device__ __forceinline__ LevelChunk level_layout(const IcGraphDev& g, const uint32_t* queue,
                                                   uint32_t head, uint32_t nb, uint4* s_ent,
                                                   uint32_t* s_start, uint32_t* s_wsum,
                                                   uint32_t* edges,
                                                   uint32_t qmask = 0xFFFFFFFFu) {
    const uint32_t tid = threadIdx.x;
    uint32_t beg = 0, end = 0;
    if (tid < nb) {
        const uint32_t v = queue[(head + tid) & qmask];
        beg = g.off[v];
        end = g.off[v + 1];
    }
    const uint32_t ng = end > beg ? ((end + 3) >> 2) - (beg >> 2) : 0u;
    uint32_t a, rank;
    const uint2 tot = block_layout_scan<BS>(ng, &a, &rank, s_wsum);
    if (ng) {
        s_ent[rank] = make_uint4(a, beg >> 2, beg, end);
        if (a < PAGE) atomicOr(&s_start[a >> 5], 1u << (a & 31));
    }
    *edges += end - beg;
    return LevelChunk{tot.x, tot.y, a, ng};
}

// Rank of the entry owning group t: the last k < ne with s_ent[k].x <= t
// (ne <= 64 * 64, s_ent[0].x == 0). The whole wave searches: 64 candidates
// per step, two steps at most.
__device__ __forceinline__ uint32_t owner_rank(const uint4* s_ent, uint32_t ne, uint32_t t) {
    const uint32_t lane = lane_id();
    uint32_t base = 0;
    if (ne > kWave) {
        const uint32_t i = lane * kWave;
        const bool le = i < ne && s_ent[i].x <= t;
        base = ((uint32_t)__popcll(__ballot(le)) - 1u) * kWave;
    }
    const uint32_t i = base + lane;
    const bool le = i < ne && s_ent[i].x <= t;
    return base + (uint32_t)__popcll(__ballot(le)) - 1u;
}

// Bits j of the edges 4*grp + j that lie in the column [beg, end).
__device__ __forceinline__ uint32_t column_bits(uint32_t grp, uint32_t beg, uint32_t end) {
    const uint32_t e0 = grp << 2;
    const uint32_t lo = beg > e0 ? beg - e0 : 0u;
    const uint32_t hi = end - e0 < 4u ? end - e0 : 4u;
    return (0xFu >> (4u - hi)) & (0xFu << lo);
}

// Bits j of the four coins of a group that come up live.
__device__ __forceinline__ uint32_t coin_bits(const Philox4& r, const uint4& th) {
    return (r.x < th.x ? 1u : 0u) | (r.y < th.y ? 2u : 0u) | (r.z < th.z ? 4u : 0u) |
           (r.w < th.w ? 8u : 0u);
}

// Read and clear the 64 start bits of the row at page position r (r % 64 == 0).
__device__ __forceinline__ uint64_t take_row(uint32_t* s_start, uint32_t r) {
    uint2* p = reinterpret_cast<uint2*>(s_start + (r >> 5));
    const uint2 v = *p;
    __builtin_amdgcn_wave_barrier();
    if (lane_id() == 0) *p = make_uint2(0u, 0u);
    return (uint64_t)v.x | ((uint64_t)v.y << 32);
}

// Flip the coins of a chunk laid out by level_layout (first page's start bits
// set, and synchronised). Each wave sweeps its span of every page two rows of
// 64 groups at a time (both threshold loads and both Philox chains in flight)
// and clears the start bits it read, so the bitmap is all zero again on
// return. Live in-edges are not followed one at a time: each wave appends
// their edge ids to its LDS buffer s_lbuf (LBUF entries) and, when the buffer
// is full and at the end of its span, loads the sources of up to 4 x 64
// buffered edges at once and hands them to on_live(u[4]) (kEmpty marks an
// unused entry). After a wave has seen a live edge it asks stop() whether to
// abandon the chunk; the whole block takes the stop at the next page
// boundary.
template <uint32_t BS, uint32_t PAGE, bool PAIR, uint32_t LBUF, class OnLive, class Stop>
__device__ __forceinline__ void level_sweep(const IcGraphDev& g, uint32_t slo, uint32_t shi,
                                            uint32_t k0, uint32_t k1, const uint4* s_ent,
                                            uint32_t* s_start, uint32_t* s_lbuf,
                                            const LevelChunk& ch, uint32_t* live_n,
                                            OnLive on_live, Stop stop) {
    static_assert(PAGE % BS == 0, "wave spans of whole rows stay inside the page");
    static_assert(LBUF >= kWave, "a row of live edges always fits an empty buffer");
    constexpr uint32_t STEP = PAIR ? 2 * kWave : kWave;
    const uint32_t w = threadIdx.x / kWave, lane = lane_id();
    const uint64_t upto = ~0ull >> (kWave - 1u - lane);  // row bits 0 .. lane
    for (uint32_t p = 0; p < ch.G;) {
        const uint32_t pn = ch.G - p < PAGE ? ch.G - p : PAGE;
        const uint32_t span = page_span<BS>(pn);
        const uint32_t w0 = w * span;
        const uint32_t w1 = w0 + span < pn ? w0 + span : pn;
        if (w0 < w1) {
            // rank o owns the last group looked at; cur is its record and
            // [cur.x, cur_hi) its groups. A row that lies inside that range
            // after its start holds no start bit and needs no LDS access.
            uint32_t o = p + w0 ? owner_rank(s_ent, ch.ne, p + w0) : 0u;
            uint4 cur = s_ent[o];
            uint32_t cur_hi = cur.x + (((cur.w + 3u) >> 2) - cur.y);
            // groups and in-column edge bits of the lanes of the row at page position rr
            auto row = [&](uint32_t rr, uint32_t* grp, uint32_t* cbits) {
                const uint32_t pos = p + rr;
                const bool valid = rr + lane < w1;
                if (cur.x < pos && pos + kWave <= cur_hi) {
                    *grp = cur.y + (pos + lane - cur.x);
                    *cbits = valid ? column_bits(*grp, cur.z, cur.w) : 0u;
                    return;
                }
                uint64_t bits = take_row(s_start, rr);
                if (rr == w0) bits &= ~1ull;  // a start on the span's first group is o's own
                const uint32_t ol = o + (uint32_t)__popcll(bits & upto);
                o += (uint32_t)__popcll(bits);
                const uint4 e = s_ent[ol];
                *grp = e.y + (pos + lane - e.x);
                *cbits = valid ? column_bits(*grp, e.z, e.w) : 0u;
                // lane 63 is owned by rank o
                cur = make_uint4((uint32_t)__builtin_amdgcn_readlane((int)e.x, 63),
                                 (uint32_t)__builtin_amdgcn_readlane((int)e.y, 63),
                                 (uint32_t)__builtin_amdgcn_readlane((int)e.z, 63),
                                 (uint32_t)__builtin_amdgcn_readlane((int)e.w, 63));
                cur_hi = cur.x + (((cur.w + 3u) >> 2) - cur.y);
            };
            uint32_t lcount = 0;  // entries in this wave's live-edge buffer (wave-uniform)
            auto flush = [&]() {
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                for (uint32_t base = 0; base < lcount; base += 4 * kWave) {
                    uint32_t e[4], u[4];
#pragma unroll
                    for (uint32_t x = 0; x < 4; ++x) {
                        const uint32_t i = base + x * kWave + lane;
                        e[x] = i < lcount ? s_lbuf[i] : kEmpty;
                    }
#pragma unroll
                    for (uint32_t x = 0; x < 4; ++x) u[x] = e[x] != kEmpty ? g.src[e[x]] : kEmpty;
                    on_live(u);
                }
                __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
                lcount = 0;
            };
            uint32_t r = w0;
            bool quit = false;
            for (; r < w1; r += STEP) {
                const bool two = PAIR && r + kWave < w1;  // wave-uniform
                uint32_t ga, ca, gb = 0u, cb = 0u;
                row(r, &ga, &ca);
                if (two) row(r + kWave, &gb, &cb);
                const bool va = ca != 0u, vb = cb != 0u;
                const uint4 tha = va ? *reinterpret_cast<const uint4*>(g.thr + 4ull * ga)
                                     : make_uint4(0u, 0u, 0u, 0u);
                const uint4 thb = vb ? *reinterpret_cast<const uint4*>(g.thr + 4ull * gb)
                                     : make_uint4(0u, 0u, 0u, 0u);
                const Philox4 ra = philox10(ga, slo, shi, 1u, k0, k1);
                const Philox4 rb = philox10(gb, slo, shi, 1u, k0, k1);
                // live edges of both groups: bits 0-3 of group a, 4-7 of group b
                const uint32_t live =
                    (coin_bits(ra, tha) & ca) | ((coin_bits(rb, thb) & cb) << 4);
                const bool any = live != 0u;
                if (__ballot(any)) {
                    const uint32_t nl = (uint32_t)__popc(live);
                    *live_n += nl;
                    // this lane's slots in the buffer: a wave prefix sum of the counts
                    const uint32_t incl = wave_incl_scan(nl);
                    const uint32_t total = (uint32_t)__builtin_amdgcn_readlane((int)incl, 63);
                    if (lcount + total > LBUF) flush();
                    if (total > LBUF) {
                        // more than a buffer's worth in one iteration (edges
                        // that are almost surely live): followed in place
                        for (uint32_t rest = live; __ballot(rest != 0u);) {
                            uint32_t u[4];  // up to four of this lane's live edges per round
#pragma unroll
                            for (uint32_t x = 0; x < 4; ++x) {
                                u[x] = kEmpty;
                                if (rest) {
                                    const uint32_t j = (uint32_t)__ffs(rest) - 1u;
                                    rest &= rest - 1u;
                                    u[x] = g.src[j < 4u ? (ga << 2) + j : (gb << 2) + (j - 4u)];
                                }
                            }
                            on_live(u);
                        }
                    } else {
                        uint32_t slot = lcount + incl - nl;
                        for (uint32_t rest = live; rest; rest &= rest - 1u) {
                            const uint32_t j = (uint32_t)__ffs(rest) - 1u;
                            s_lbuf[slot++] = j < 4u ? (ga << 2) + j : (gb << 2) + (j - 4u);
                        }
                        lcount += total;
                    }
                    if (stop()) {
                        quit = true;
                        break;
                    }
                }
            }
            if (!quit) flush();
            if (quit) {
                // the rows up to r + STEP are cleared; clear the rest of the span
                for (uint32_t q = r + STEP; q < w1; q += kWave)
                    if (lane < 2u) s_start[(q >> 5) + lane] = 0u;
            }
        }
        p += PAGE;
        if (p >= ch.G) break;
        __syncthreads();  // every wave is done with this page's bits
        if (stop()) break;
        if (ch.ng && ch.a >= p && ch.a - p < PAGE)
            atomicOr(&s_start[(ch.a - p) >> 5], 1u << ((ch.a - p) & 31));
        __syncthreads();
    }
}

// ----------------------------------------------------------------- ic_lane

// A wave claims kLaneRounds batches of 64 ids per ticket and appends its
// pending samples once per ticket: the ticket and the pending-list length
// are single counters that every wave of the launch updates.
constexpr uint32_t kLaneRounds = 4;

static_assert(kWave * kLaneRounds == kLaneTicket, "lane tickets");

__device__ __forceinline__ void lane_flush(const SampleOut& o, uint64_t* sets, uint64_t* edges) {
    const uint64_t a = wave_sum64(*sets), b = wave_sum64(*edges);
    if (lane_id() == 0) {
        atomicAdd(&o.stats[kStLaneSets], (unsigned long long)a);
        atomicAdd(&o.stats[kStLaneEdges], (unsigned long long)b);
    }
    *sets = 0;
    *edges = 0;
}

// MULTI = false: one instance (the arguments). Otherwise the tasks'
// positions follow each other (prefix), every ticket inside one task. The
// single-instance form is compiled apart: its arguments stay in scalar
// registers, where a task switch would move them into vector registers and
// halve the waves that fit.
template <bool MULTI>
__global__ __launch_bounds__(kWave) void ic_lane_kernel(IcGraphDev g, SampleRange rg,
                                                        SampleOut o, uint32_t* pend,
                                                        uint32_t* pend_n, uint32_t* ticket,
                                                        const IcTask* tasks, uint32_t ntask_in,
                                                        const uint32_t* prefix) {
    const uint32_t ntask = MULTI ? ntask_in : 0u;
    __shared__ uint32_t s_tk, s_np;
    __shared__ uint32_t s_pend[kWave * kLaneRounds];
    __shared__ unsigned long long s_chunk;
    const uint32_t lane = threadIdx.x;
    uint32_t k0 = (uint32_t)rg.seed, k1 = (uint32_t)(rg.seed >> 32);
    Stager sg;
    uint64_t st_sets = 0, st_edges = 0;  // lane-partial
    uint32_t total = ntask ? 0u : (rg.list ? *rg.list_n : rg.count);
    const uint32_t end = ntask ? prefix[ntask] : total;
    uint32_t cur = ntask, base = 0;  // the task in hand (ntask: none yet)
    for (;;) {
        if (lane == 0) {
            s_tk = atomicAdd(ticket, kWave * kLaneRounds);
            s_np = 0;
        }
        __syncthreads();
        const uint32_t ticket_pos = s_tk;
        __syncthreads();
        if (ticket_pos >= end) break;
        if (ntask) {
            const uint32_t q = task_of(prefix, ntask, ticket_pos);
            if (q != cur) {
                if (cur != ntask) lane_flush(o, &st_sets, &st_edges);
                cur = q;
                g = tasks[q].g;
                rg = tasks[q].rg;
                o = tasks[q].o;
                pend = tasks[q].pend;
                pend_n = tasks[q].pend_n;
                k0 = (uint32_t)rg.seed;
                k1 = (uint32_t)(rg.seed >> 32);
                sg = Stager{};
                base = prefix[q];
                total = rg.count;
            }
        }

        for (uint32_t round = 0; round < kLaneRounds; ++round) {
            const uint32_t base_pos = ticket_pos - base + round * kWave;
            if (base_pos >= total) break;
            const uint32_t my_pos = base_pos + lane;
            const bool valid = my_pos < total;
            const uint32_t my_idx = valid ? (rg.list ? rg.list[my_pos] : my_pos) : 0u;
            const uint64_t ms = rg.id_lo + my_idx;
            uint32_t root = 0, rbeg = 0, rend = 0;
            bool single = false;
            if (valid) {
                root = sample_root(rg.seed, ms, g.n);
                rbeg = g.off[root];
                rend = g.off[root + 1];
                single = rend - rbeg <= kLaneDegCap;
                for (uint32_t grp = rbeg >> 2; single && (grp << 2) < rend; ++grp) {
                    const uint4 th = *reinterpret_cast<const uint4*>(g.thr + 4ull * grp);
                    const Philox4 r = philox10(grp, (uint32_t)ms, (uint32_t)(ms >> 32), 1u, k0, k1);
                    const uint32_t e0 = grp << 2;
                    if ((r.x < th.x && e0 >= rbeg && e0 < rend) ||
                        (r.y < th.y && e0 + 1 >= rbeg && e0 + 1 < rend) ||
                        (r.z < th.z && e0 + 2 >= rbeg && e0 + 2 < rend) ||
                        (r.w < th.w && e0 + 3 >= rbeg && e0 + 3 < rend))
                        single = false;
                }
            }
            const uint64_t smask = __ballot(single);
            const uint32_t nsingle = (uint32_t)__popcll(smask);
            if (nsingle) {
                uint64_t off = 0;
                const bool ok = stage_reserve(sg, nsingle, &off, &s_chunk, o);
                const uint32_t rank = (uint32_t)__popcll(smask & ((1ull << lane) - 1ull));
                if (single) {
                    if (ok) {
                        o.stage[off + rank] = root;
                        atomicAdd(&o.counts[root], 1u);
                        o.stage_off[my_idx] = off + rank;
                        o.sizes[my_idx] = 1;
                        st_sets += 1;
                        st_edges += rend - rbeg;
                    } else {
                        o.retry[atomicAdd(o.retry_n, 1u)] = my_idx;
                    }
                }
            }
            // pending samples wait in LDS until the ticket is done
            const bool pending = valid && !single;
            const uint64_t pmask = __ballot(pending);
            const uint32_t np = s_np;
            if (pending) s_pend[np + (uint32_t)__popcll(pmask & ((1ull << lane) - 1ull))] = my_idx;
            __syncthreads();
            if (lane == 0) s_np = np + (uint32_t)__popcll(pmask);
            __syncthreads();
        }
        const uint32_t np = s_np;
        if (np) {
            uint32_t pbase = 0;
            if (lane == 0) pbase = atomicAdd(pend_n, np);
            pbase = __shfl(pbase, 0, kWave);
            for (uint32_t i = lane; i < np; i += kWave) pend[pbase + i] = s_pend[i];
        }
        __syncthreads();
    }
    if (cur != ntask || ntask == 0) lane_flush(o, &st_sets, &st_edges);
}

// ------------------------------------------------------------------ ic_bfs

// Insert u into the LDS visited hash; append it to the member list when new.
template <uint32_t TEAM>
__device__ __forceinline__ void team_insert(uint32_t u, uint32_t* hash, uint32_t* members,
                                            uint32_t* s_size, uint32_t* s_over) {
    using T = Team<TEAM>;
    uint32_t slot = (u * 0x9E3779B1u) >> (32 - T::HBITS);
    for (uint32_t probe = 0; probe < T::HSIZE; ++probe) {
        const uint32_t cur = lds_load(&hash[slot]);
        if (cur == u) return;
        if (cur == kEmpty) {
            if (lds_load(s_size) >= T::CAP) {
                *s_over = 1u;
                return;
            }
            const uint32_t old = atomicCAS(&hash[slot], kEmpty, u);
            if (old == kEmpty) {
                const uint32_t pos = atomicAdd(s_size, 1u);
                if (pos < T::CAP) members[pos] = u; else *s_over = 1u;
                return;
            }
            if (old == u) return;
        }
        slot = (slot + 1) & (T::HSIZE - 1);
    }
    *s_over = 1u;
}

// Work-item lists of several tasks as one: s_pre[q] = the items of tasks
// before q (list lengths read on the device), s_pre[ntask] = all of them.
__device__ __forceinline__ void list_prefix(const IcTask* tasks, uint32_t ntask, bool deferred,
                                            uint32_t* s_pre) {
    if (threadIdx.x == 0) {
        uint32_t a = 0;
        for (uint32_t q = 0; q < ntask; ++q) {
            s_pre[q] = a;
            a += deferred ? *tasks[q].o.defer_n : *tasks[q].pend_n;
        }
        s_pre[ntask] = a;
    }
    __syncthreads();
}

// Per-thread partial statistics of a sampling pass, flushed into a task's
// counters (every thread of the workgroup calls it alike).
__device__ __forceinline__ void stats_flush(const SampleOut& o, bool big, uint64_t* sets,
                                            uint64_t* entries, uint64_t* edges, uint64_t* live) {
    const uint64_t a = wave_sum64(*sets), b = wave_sum64(*entries), c = wave_sum64(*edges),
                   d = wave_sum64(*live);
    if (threadIdx.x % kWave == 0) {
        atomicAdd(&o.stats[big ? kStBigSets : kStMainSets], (unsigned long long)a);
        atomicAdd(&o.stats[big ? kStBigEntries : kStMainEntries], (unsigned long long)b);
        atomicAdd(&o.stats[big ? kStBigEdges : kStMainEdges], (unsigned long long)c);
        atomicAdd(&o.stats[big ? kStBigLive : kStMainLive], (unsigned long long)d);
    }
    *sets = *entries = *edges = *live = 0;
}

// MULTI = false: one instance (the arguments). Otherwise the pending lists
// of the tasks, one after another.
template <uint32_t TEAM, bool MULTI>
__global__ __launch_bounds__(kWave * TEAM) void ic_bfs_kernel(IcGraphDev g, SampleRange rg,
                                                              SampleOut o, const uint32_t* pend,
                                                              const uint32_t* pend_n,
                                                              uint32_t* ticket,
                                                              const IcTask* tasks,
                                                              uint32_t ntask_in) {
    const uint32_t ntask = MULTI ? ntask_in : 0u;
    using T = Team<TEAM>;
    constexpr uint32_t BS = T::BS;
    __shared__ uint32_t hash[T::HSIZE];
    __shared__ uint32_t members[T::CAP];
    __shared__ uint4 s_ent[BS];
    __shared__ uint32_t s_start[T::PAGE / 32];
    __shared__ uint32_t s_lbuf[TEAM * kBfsLiveBuf];
    __shared__ uint32_t s_wsum[2 * TEAM];
    __shared__ uint32_t s_size, s_over, s_tk;
    __shared__ unsigned long long s_chunk;
    __shared__ uint32_t s_pre[kMaxTasks + 1];

    const uint32_t tid = threadIdx.x;
    uint32_t k0 = (uint32_t)rg.seed, k1 = (uint32_t)(rg.seed >> 32);
    for (uint32_t i = tid; i < T::HSIZE; i += BS) hash[i] = kEmpty;
    for (uint32_t i = tid; i < T::PAGE / 32; i += BS) s_start[i] = 0u;
    Stager sg;
    uint64_t st_sets = 0, st_entries = 0, st_edges = 0, st_live = 0;  // thread-partial
    if (ntask) list_prefix(tasks, ntask, false, s_pre);
    const uint32_t total = ntask ? s_pre[ntask] : *pend_n;
    uint32_t cur = ntask;  // the task in hand (ntask: none yet)

    for (;;) {
        if (tid == 0) s_tk = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t pos = s_tk;
        __syncthreads();
        if (pos >= total) break;
        uint32_t lpos = pos;
        if (ntask) {
            const uint32_t q = task_of(s_pre, ntask, pos);
            if (q != cur) {
                if (cur != ntask) stats_flush(o, false, &st_sets, &st_entries, &st_edges, &st_live);
                cur = q;
                g = tasks[q].g;
                rg = tasks[q].rg;
                o = tasks[q].o;
                pend = tasks[q].pend;
                k0 = (uint32_t)rg.seed;
                k1 = (uint32_t)(rg.seed >> 32);
                sg = Stager{};
            }
            lpos = pos - s_pre[q];
        }
        const uint32_t idx = pend[lpos];
        const uint64_t s = rg.id_lo + idx;
        const uint32_t slo = (uint32_t)s, shi = (uint32_t)(s >> 32);
        if (tid == 0) {
            const uint32_t r0 = sample_root(rg.seed, s, g.n);
            members[0] = r0;
            hash[(r0 * 0x9E3779B1u) >> (32 - T::HBITS)] = r0;
            s_size = 1;
            s_over = 0;
        }
        __syncthreads();

        uint32_t head = 0, size = 1, my_edges = 0, my_live = 0;
        bool over = false;
        while (head < size) {
            const uint32_t nb = min(BS, size - head);
            const LevelChunk ch = level_layout<BS, T::PAGE>(g, members, head, nb, s_ent, s_start,
                                                            s_wsum, &my_edges);
            __syncthreads();
            level_sweep<BS, T::PAGE, true, kBfsLiveBuf>(
                g, slo, shi, k0, k1, s_ent, s_start, s_lbuf + (tid / kWave) * kBfsLiveBuf, ch,
                &my_live,
                [&](const uint32_t(&u)[4]) {
#pragma unroll
                    for (uint32_t x = 0; x < 4; ++x)
                        if (u[x] != kEmpty) team_insert<TEAM>(u[x], hash, members, &s_size, &s_over);
                },
                [&]() { return lds_load(&s_over) != 0u; });
            __syncthreads();
            head += nb;
            size = s_size;
            over = s_over != 0u;
            __syncthreads();
            if (over) break;
        }

        if (over) {
            if (tid == 0) o.defer[atomicAdd(o.defer_n, 1u)] = idx;
        } else {
            uint64_t off = 0;
            if (stage_reserve(sg, size, &off, &s_chunk, o)) {
                for (uint32_t i = tid; i < size; i += BS) {
                    const uint32_t u = members[i];
                    o.stage[off + i] = u;
                    atomicAdd(&o.counts[u], 1u);
                }
                if (tid == 0) {
                    o.stage_off[idx] = off;
                    o.sizes[idx] = size;
                    st_sets += 1;
                    st_entries += size;
                }
                st_edges += my_edges;
                st_live += my_live;
            } else if (tid == 0) {
                o.retry[atomicAdd(o.retry_n, 1u)] = idx;
            }
        }
        // reset the hash slots this sample used (all members are listed)
        const uint32_t used = min(size, T::CAP);
        __syncthreads();
        if (over) {
            // an abandoned set may have hashed vertices beyond the list
            for (uint32_t i = tid; i < T::HSIZE; i += BS) hash[i] = kEmpty;
        } else {
            for (uint32_t i = tid; i < used; i += BS) {
                const uint32_t u = members[i];
                uint32_t slot = (u * 0x9E3779B1u) >> (32 - T::HBITS);
                for (uint32_t probe = 0; probe < T::HSIZE; ++probe) {
                    if (hash[slot] == u) {
                        hash[slot] = kEmpty;
                        break;
                    }
                    slot = (slot + 1) & (T::HSIZE - 1);
                }
            }
        }
        __syncthreads();
    }
    if (cur != ntask || ntask == 0)
        stats_flush(o, false, &st_sets, &st_entries, &st_edges, &st_live);
}

// ---------------------------------------------------------------- ic_large

// MULTI = false: one instance (the arguments). Otherwise the deferred lists
// of the tasks, one after another, with b's slots sized for the largest
// task; a set that overflows its queue goes to its task's retry list.
template <uint32_t kBigBlock, bool MULTI>
__global__ __launch_bounds__(kBigBlock, kBigBlock == 1024 ? 8 : 1) void ic_large_kernel(IcGraphDev g, SampleRange rg,
                                                             SampleOut o, const uint32_t* list,
                                                             const uint32_t* list_n,
                                                             uint32_t* fail, uint32_t* fail_n,
                                                             uint32_t* over, uint32_t* over_n,
                                                             uint32_t* ticket, BigScratch b,
                                                             const IcTask* tasks, uint32_t ntask_in) {
    const uint32_t ntask = MULTI ? ntask_in : 0u;
    __shared__ uint4 s_ent[kBigBlock];
    __shared__ uint32_t s_start[kLargePage / 32];
    __shared__ uint32_t s_lbuf[kBigBlock / kWave * kLargeLiveBuf];
    __shared__ uint32_t s_wsum[2 * kBigBlock / kWave];
    __shared__ uint32_t s_size, s_i, s_b, s_ovf;
    __shared__ unsigned long long s_off;
    __shared__ uint32_t s_pre[kMaxTasks + 1];

    const uint32_t tid = threadIdx.x;
    uint32_t k0 = (uint32_t)rg.seed, k1 = (uint32_t)(rg.seed >> 32);
    uint32_t* bm = b.bitmaps + (size_t)blockIdx.x * b.words;
    uint32_t* q = b.queues + (size_t)blockIdx.x * b.qcap;
    // this instance's bitmap words and queue capacity (the slot may be larger)
    uint32_t words = b.words, qcap = b.qcap;
    // A bounded queue of a power-of-two size is used as a ring when a set
    // too large for it can still be stored: as a bitmap, whose members need
    // no list. The BFS then only needs its frontier (the entries not yet
    // swept) to fit; a set that ends larger than the queue must be dense,
    // else it goes to the full-size pass like one whose frontier overflows.
    bool ring = o.dense_min != 0xFFFFFFFFu && qcap < g.n && (qcap & (qcap - 1)) == 0;
    uint32_t qmask = ring ? qcap - 1 : 0xFFFFFFFFu;
    if (ntask) list_prefix(tasks, ntask, true, s_pre);
    const uint32_t cnt = ntask ? s_pre[ntask] : *list_n;
    uint32_t cur = ntask;  // the task in hand (ntask: none yet)
    uint64_t st_sets = 0, st_entries = 0, st_edges = 0, st_live = 0;
    for (uint32_t i = tid; i < kLargePage / 32; i += kBigBlock) s_start[i] = 0u;

    for (;;) {
        if (tid == 0) s_i = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t li = s_i;
        __syncthreads();
        if (li >= cnt) break;
        uint32_t lpos = li;
        if (ntask) {
            const uint32_t tq = task_of(s_pre, ntask, li);
            if (tq != cur) {
                if (cur != ntask) stats_flush(o, true, &st_sets, &st_entries, &st_edges, &st_live);
                cur = tq;
                g = tasks[tq].g;
                rg = tasks[tq].rg;
                o = tasks[tq].o;
                list = o.defer;
                fail = o.retry;
                fail_n = o.retry_n;
                over = o.retry;
                over_n = o.retry_n;
                k0 = (uint32_t)rg.seed;
                k1 = (uint32_t)(rg.seed >> 32);
                words = (g.n + 31) / 32;
                qcap = tasks[tq].qcap;
                ring = o.dense_min != 0xFFFFFFFFu && qcap < g.n && (qcap & (qcap - 1)) == 0;
                qmask = ring ? qcap - 1 : 0xFFFFFFFFu;
            }
            lpos = li - s_pre[tq];
        }
        const uint32_t idx = list[lpos];
        const uint64_t s = rg.id_lo + idx;
        const uint32_t slo = (uint32_t)s, shi = (uint32_t)(s >> 32);
        if (tid == 0) {
            const uint32_t root = sample_root(rg.seed, s, g.n);
            q[0] = root;
            atomicOr(&bm[root >> 5], 1u << (root & 31));
            s_size = 1;
            s_ovf = 0;
        }
        __syncthreads();

        uint32_t head = 0, size = 1, my_edges = 0, my_live = 0;
        bool overflow = false;
        while (head < size) {
            const uint32_t nb = min(kBigBlock, size - head);
            const LevelChunk ch = level_layout<kBigBlock, kLargePage>(
                g, q, head, nb, s_ent, s_start, s_wsum, &my_edges, qmask);
            __syncthreads();
            level_sweep<kBigBlock, kLargePage, (kBigBlock < 1024), kLargeLiveBuf>(
                g, slo, shi, k0, k1, s_ent, s_start, s_lbuf + (tid / kWave) * kLargeLiveBuf, ch,
                &my_live,
                [&](const uint32_t(&u)[4]) {
                    // all four visited-bit atomics in flight before any result is used
                    uint32_t old[4];
#pragma unroll
                    for (uint32_t x = 0; x < 4; ++x)
                        old[x] = u[x] != kEmpty ? atomicOr(&bm[u[x] >> 5], 1u << (u[x] & 31))
                                                : 0xFFFFFFFFu;
#pragma unroll
                    for (uint32_t x = 0; x < 4; ++x) {
                        if (!((old[x] >> (u[x] & 31)) & 1u)) {
                            const uint32_t pos = atomicAdd(&s_size, 1u);
                            // ring: the chunk being swept is already in LDS,
                            // so positions up to head + qcap - 1 are free
                            if (ring) {
                                if (pos - head < qcap) q[pos & qmask] = u[x];
                                else s_ovf = 1u;
                            } else if (pos < qcap) {
                                q[pos] = u[x];
                            }
                        }
                    }
                },
                []() { return false; });
            __syncthreads();
            head += nb;
            size = s_size;
            overflow = ring ? s_ovf != 0u : size > qcap;
            __syncthreads();
            if (overflow) break;
        }
        // a ring that wrapped lists only its last entries: such a set is
        // stored as a bitmap, or else redone with a full-size queue
        if (!overflow && size > qcap && size < o.dense_min) overflow = true;

        if (overflow) {
            // the queue no longer lists every visited vertex: clear the whole
            // bitmap, and leave the sample to the pass with full-size queues
            for (uint32_t i = tid; i < words; i += kBigBlock)
                __hip_atomic_store(&bm[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (tid == 0) over[atomicAdd(over_n, 1u)] = idx;
            __syncthreads();
            continue;
        }

        if (size >= o.dense_min) {
            // a dense set: its visited bitmap is the set; it goes to a bitmap
            // slot (read with device-scope loads, which skip the CU cache the
            // atomics never updated) and the slot's bitmap is cleared whole
            if (tid == 0) s_b = atomicAdd(o.dense_cursor, 1u);
            __syncthreads();
            const uint32_t slot = s_b;
            const bool ok = slot < o.dense_cap;
            uint32_t* dst = o.dense_bits + (ok ? (size_t)slot * o.dense_words : 0);
            for (uint32_t i = tid; i < words; i += kBigBlock) {
                if (ok)
                    dst[i] = __hip_atomic_load(&bm[i], __ATOMIC_RELAXED,
                                               __HIP_MEMORY_SCOPE_AGENT);
                __hip_atomic_store(&bm[i], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            }
            if (tid == 0) {
                if (ok) {
                    o.dense_sid[slot] = (uint32_t)(o.pool_base + idx);
                    o.dense_size[slot] = size;
                    atomicAdd(o.dense_entries, (unsigned long long)size);
                    o.stage_off[idx] = 0;
                    o.sizes[idx] = 0;
                    st_sets += 1;
                    st_entries += size;
                } else {
                    fail[atomicAdd(fail_n, 1u)] = idx;
                }
            }
            if (ok) {
                st_edges += my_edges;
                st_live += my_live;
            }
            __syncthreads();
            continue;
        }

        if (tid == 0) s_off = atomicAdd(o.cursor, (unsigned long long)size);
        __syncthreads();
        const uint64_t off = s_off;
        const bool fits = off + size <= o.stage_cap;
        for (uint32_t i = tid; i < size; i += kBigBlock) {
            const uint32_t u = q[i];
            if (fits) {
                o.stage[off + i] = u;
                atomicAdd(&o.counts[u], 1u);
            }
            __hip_atomic_store(&bm[u >> 5], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (tid == 0) {
            if (fits) {
                o.stage_off[idx] = off;
                o.sizes[idx] = size;
                st_sets += 1;
                st_entries += size;
            } else {
                fail[atomicAdd(fail_n, 1u)] = idx;
            }
        }
        if (fits) {
            st_edges += my_edges;
            st_live += my_live;
        }
        __syncthreads();
    }
    if (cur != ntask || ntask == 0)
        stats_flush(o, true, &st_sets, &st_entries, &st_edges, &st_live);
}

int cu_count(int device) {
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    return cus;
}

}  // namespace

uint32_t ic_small_grid(int device) { return (uint32_t)cu_count(device) * 24u; }

uint32_t ic_bfs_grid(int device, uint32_t team) {
    // enough workgroups for 8 waves per SIMD
    return (uint32_t)cu_count(device) * 32u / team;
}

hipError_t launch_ic_lane(const IcGraphDev& g, const SampleRange& r, const SampleOut& o,
                          uint32_t* pend, uint32_t* pend_n, uint32_t* ticket, uint32_t grid,
                          hipStream_t st) {
    const uint32_t per = kWave * kLaneRounds;
    const uint32_t need = (r.count + per - 1) / per;
    if (grid > need) grid = need;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(ic_lane_kernel<false>, dim3(grid), dim3(kWave), 0, st, g, r, o, pend,
                       pend_n,
                       ticket, (const IcTask*)nullptr, 0u, (const uint32_t*)nullptr);
    return hipGetLastError();
}

hipError_t launch_ic_bfs(const IcGraphDev& g, const SampleRange& r, const SampleOut& o,
                         const uint32_t* pend, const uint32_t* pend_n, uint32_t* ticket,
                         uint32_t team, uint32_t grid, hipStream_t st) {
    // r.count bounds the pending list (its length is read on the device)
    if (grid > r.count) grid = r.count;
    if (grid == 0) return hipSuccess;
    switch (team) {
        case 1:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(ic_bfs_kernel<1, false>), dim3(grid), dim3(kWave), 0, st, g, r, o, pend,
                               pend_n, ticket, (const IcTask*)nullptr, 0u);
            break;
        case 2:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(ic_bfs_kernel<2, false>), dim3(grid), dim3(2 * kWave), 0, st, g, r, o,
                               pend, pend_n, ticket, (const IcTask*)nullptr, 0u);
            break;
        case 4:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(ic_bfs_kernel<4, false>), dim3(grid), dim3(4 * kWave), 0, st, g, r, o,
                               pend, pend_n, ticket, (const IcTask*)nullptr, 0u);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

uint32_t ic_large_slots(int device, uint32_t block) {
    // the same 2048 threads per CU either way: many giant sets in flight
    // (256 threads each) or fewer, wider ones (1024)
    return (uint32_t)cu_count(device) * (block == 256 ? 8u : 2u);
}

hipError_t launch_ic_large(const IcGraphDev& g, const SampleRange& r, const SampleOut& o,
                           const uint32_t* list, const uint32_t* list_n, uint32_t* fail,
                           uint32_t* fail_n, uint32_t* over, uint32_t* over_n,
                           uint32_t* ticket, const BigScratch& b, uint32_t block,
                           hipStream_t st) {
    if (b.slots == 0 || b.qcap == 0 || b.qcap > g.n) return hipErrorInvalidValue;
    if (b.qcap < g.n && (over == nullptr || over_n == nullptr)) return hipErrorInvalidValue;
    if (block == 256)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(ic_large_kernel<256, false>), dim3(b.slots), dim3(256), 0, st, g, r, o, list,
                           list_n, fail, fail_n, over, over_n, ticket, b, (const IcTask*)nullptr,
                           0u);
    else if (block == 1024)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(ic_large_kernel<1024, false>), dim3(b.slots), dim3(1024), 0, st, g, r, o,
                           list, list_n, fail, fail_n, over, over_n, ticket, b,
                           (const IcTask*)nullptr, 0u);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

hipError_t launch_ic_multi(const IcTask* tasks, uint32_t ntask, const uint32_t* prefix,
                           uint32_t* tickets, uint32_t team, uint32_t block, const BigScratch& b,
                           int device, hipStream_t st) {
    if (ntask == 0 || ntask > kMaxTasks || b.slots == 0 || b.qcap == 0) return hipErrorInvalidValue;
    // the per-task arguments come from the table; these only fill the slots
    const IcGraphDev g{};
    const SampleRange r{};
    const SampleOut o{};
    hipLaunchKernelGGL(ic_lane_kernel<true>, dim3(ic_small_grid(device)), dim3(kWave), 0, st, g, r, o,
                       (uint32_t*)nullptr, (uint32_t*)nullptr, tickets, tasks, ntask, prefix);
    const uint32_t grid = ic_bfs_grid(device, team);
    switch (team) {
        case 1:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(ic_bfs_kernel<1, true>), dim3(grid), dim3(kWave), 0, st, g, r, o,
                               (const uint32_t*)nullptr, (const uint32_t*)nullptr, tickets + 1,
                               tasks, ntask);
            break;
        case 2:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(ic_bfs_kernel<2, true>), dim3(grid), dim3(2 * kWave), 0, st, g, r, o,
                               (const uint32_t*)nullptr, (const uint32_t*)nullptr, tickets + 1,
                               tasks, ntask);
            break;
        case 4:
            hipLaunchKernelGGL(HIP_KERNEL_NAME(ic_bfs_kernel<4, true>), dim3(grid), dim3(4 * kWave), 0, st, g, r, o,
                               (const uint32_t*)nullptr, (const uint32_t*)nullptr, tickets + 1,
                               tasks, ntask);
            break;
        default:
            return hipErrorInvalidValue;
    }
    if (block == 256)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(ic_large_kernel<256, true>), dim3(b.slots), dim3(256), 0, st, g, r, o,
                           (const uint32_t*)nullptr, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                           (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr,
                           tickets + 2, b, tasks, ntask);
    else if (block == 1024)
        hipLaunchKernelGGL(HIP_KERNEL_NAME(ic_large_kernel<1024, true>), dim3(b.slots), dim3(1024), 0, st, g, r, o,
                           (const uint32_t*)nullptr, (const uint32_t*)nullptr, (uint32_t*)nullptr,
                           (uint32_t*)nullptr, (uint32_t*)nullptr, (uint32_t*)nullptr,
                           tickets + 2, b, tasks, ntask);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace imm
