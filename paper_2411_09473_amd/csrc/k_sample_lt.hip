// k_sample_lt.hip -- LT RRR sampling as reverse live-edge walks, with fused
// occurrence counts (Generate_RRRsets, Algorithm 3; LT model of Section II-A
// in its live-edge form: every vertex keeps at most one live in-edge).
//
// A walk is a chain of dependent loads. A group of P lanes (2 or 4, picked
// per graph by the autotuner) runs one walk, so a wave keeps 64/P walks in
// flight: the lanes split each step's eight-record line read, and a wave load
// instruction then touches 64/P lines instead of 64, which the vector memory
// pipeline serves several times faster than 64 lines of one record each. A
// group whose walk ends takes the next sample at once (wave-aggregated
// tickets), which keeps the memory system busy.
//  * The live in-edge of v is the first e of v's column with r < cum[e]. The
//    guide table jumps to the first candidate of r's bucket j = floor(r d /
//    2^32), from where a short forward scan over the edge records finds the
//    same edge the plain search would. Each bucket keeps a copy of the four
//    records from its candidate on (a 64-byte window), which holds the answer
//    unless more than three of the column's edges end inside the bucket
//    (about one step in 1300 on a LiveJournal-shaped graph); the scan then
//    goes on in the column itself. A record also holds the bounds of its
//    source's column, so the next step needs no offset load.
//  * The path is written straight into the walk's staging chunk. A per-walk
//    Bloom filter of 1024 to 4096 bits (three hashes, size picked per graph
//    by the autotuner) in LDS answers "not on the path" for most vertices; a
//    hit is confirmed by rescanning the path (vectorised), so the test is
//    exact.
//  * Counts are incremented as vertices join the path (only for samples
//    below the pass's count limit: later ones are drawn ahead for the next
//    round and counted when they join the pool); a walk that has to move to
//    the large-walk kernel (path longer than a chunk) or to a retry (staging
//    full) gives its increments back first. The large-walk kernel
//    picks a walk up where it stopped: the draw at a vertex depends only on
//    the sample and the vertex, so the chunk's path and the next vertex are
//    all it needs.
#include "device_common.hpp"
#include "imm_internal.hpp"

namespace imm {

namespace {

constexpr uint32_t kNone = 0xFFFFFFFFu;
constexpr uint32_t kWin = kLtWindow;   // records per guide window
constexpr uint32_t kScanLoads = 2;     // 16-byte path groups per lane per rescan round

// The three filter positions of v in a 2^BB-bit filter (multiplicative hashes).
template <uint32_t BB>
__device__ __forceinline__ void bloom_pos(uint32_t v, uint32_t h[3]) {
    h[0] = (v * 0x9E3779B1u) >> (32 - BB);
    h[1] = (v * 0x85EBCA77u) >> (32 - BB);
    h[2] = (v * 0xC2B2AE3Du) >> (32 - BB);
}

// mb points at the walk's filter (2^BB / 32 consecutive words).
template <uint32_t BB>
__device__ __forceinline__ void bloom_set(uint32_t* mb, uint32_t v) {
    uint32_t h[3];
    bloom_pos<BB>(v, h);
#pragma unroll
    for (uint32_t j = 0; j < 3; ++j) mb[h[j] >> 5] |= 1u << (h[j] & 31);
}

template <uint32_t BB>
__device__ __forceinline__ bool bloom_test(const uint32_t* mb, uint32_t v) {
    uint32_t h[3];
    bloom_pos<BB>(v, h);
    bool all = true;
#pragma unroll
    for (uint32_t j = 0; j < 3; ++j) all &= ((mb[h[j] >> 5] >> (h[j] & 31)) & 1u) != 0;
    return all;
}

// The live in-edge of the column [beg, end) for draw r, for a walk run by a
// single lane (the long-walk kernel): its record (src in .y, src's column
// bounds in .z/.w), or .y = kNone. *reads counts the records inspected. The
// lane reads the window of r's bucket in one round trip; the answer lies
// further on only when more than three edges of the column end inside the
// bucket, and then the scan goes on in the column, four records per round
// trip. Needs beg < end.
__device__ __forceinline__ uint4 lt_pick(const LtGraphDev& g, uint32_t beg, uint32_t end,
                                         uint32_t r, uint32_t* reads) {
    const uint32_t d = end - beg;
    const uint32_t jb = (uint32_t)(((uint64_t)r * (uint64_t)d) >> 32);
    const uint4* w = g.gw + (uint64_t)kWin * (beg + jb);
    uint4 p[kWin];
#pragma unroll
    for (uint32_t j = 0; j < kWin; ++j) p[j] = w[j];
    uint4 res = make_uint4(0u, kNone, 0u, 0u);
    bool ended = false;
#pragma unroll
    for (uint32_t j = 0; j < kWin; ++j) {
        if (res.y == kNone && !ended) {
            if (p[j].y == kNone) {
                ended = true;
            } else {
                ++*reads;
                if (r < p[j].x) res = p[j];
            }
        }
    }
    if (res.y != kNone || ended) return res;
    for (uint32_t e = g.guide[beg + jb] + kWin; e < end; e += 4) {
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j)
            p[j] = e + j < end ? g.cs[e + j] : make_uint4(0xFFFFFFFFu, kNone, 0u, 0u);
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            if (res.y == kNone && e + j < end) {
                ++*reads;
                if (r < p[j].x) res = p[j];
            }
        }
        if (res.y != kNone) break;
    }
    return res;
}

// The lanes of one walk: P consecutive lanes of a wave (P = 1, 2 or 4), the
// group starting at lane `lead`. Its bits of a wave ballot.
template <uint32_t P>
__device__ __forceinline__ uint32_t group_bits(uint64_t ballot, uint32_t lead) {
    return (uint32_t)(ballot >> lead) & ((1u << P) - 1u);
}

// Sum of x over the group (every lane gets it).
template <uint32_t P>
__device__ __forceinline__ uint32_t group_sum(uint32_t x) {
#pragma unroll
    for (uint32_t o = 1; o < P; o <<= 1) x += __shfl_xor(x, o, kWave);
    return x;
}

// The live in-edge of a column for a walk run by a group of P lanes, in two
// parts so that a step's window read can be in flight while the walk does
// other work. window_issue: each lane loads kWin/P of the window's records
// (a wave load instruction then touches 64/P windows instead of 64, which the
// memory pipeline serves several times faster). Needs beg < end.
template <uint32_t P>
__device__ __forceinline__ void window_issue(const LtGraphDev& g, uint32_t beg, uint32_t end,
                                             uint32_t r, uint32_t sub, uint4 (&p)[kWin / P]) {
    constexpr uint32_t R = kWin / P;
    const uint32_t d = end - beg;
    const uint32_t jb = (uint32_t)(((uint64_t)r * (uint64_t)d) >> 32);
    const uint4* w = g.gw + (uint64_t)kWin * (beg + jb) + sub * R;
#pragma unroll
    for (uint32_t j = 0; j < R; ++j) p[j] = w[j];
}

// window_pick: the first lane of the group with a hit supplies the record
// (src in .y, src's column bounds in .z/.w; .y = kNone for no live edge).
// Records past the column's end are empty (src = kNone): a window that
// reaches one without a hit has no live edge. Every lane returns the same
// record and count; the caller's control flow is uniform across the group.
// The answer lies past the window only when more than three edges of the
// column end inside r's bucket; the scan then goes on in the column, four
// records per lane per round trip.
template <uint32_t P>
__device__ __forceinline__ uint4 window_pick(const LtGraphDev& g, uint32_t beg, uint32_t end,
                                             uint32_t r, uint32_t* reads, uint32_t sub,
                                             uint32_t lead, const uint4 (&p)[kWin / P]) {
    constexpr uint32_t R = kWin / P;
    // this lane's first hit or column end (R: neither), and records
    // inspected up to it
    uint32_t hj = R, used = 0;
    bool hit = false;
    uint4 mine = make_uint4(0u, kNone, 0u, 0u);
#pragma unroll
    for (uint32_t j = 0; j < R; ++j) {
        if (hj == R) {
            if (p[j].y == kNone) {
                hj = j;
            } else {
                ++used;
                if (r < p[j].x) {
                    hj = j;
                    hit = true;
                    mine = p[j];
                }
            }
        }
    }
    uint32_t gb = group_bits<P>(__ballot(hj < R), lead);
    uint4 res = make_uint4(0u, kNone, 0u, 0u);
    if (gb) {
        // the lanes before the first stop hold R inspected records each
        const uint32_t src = lead + (uint32_t)__ffs(gb) - 1u;
        if (__shfl((uint32_t)hit, src, kWave)) {
            res.y = __shfl(mine.y, src, kWave);
            res.z = __shfl(mine.z, src, kWave);
            res.w = __shfl(mine.w, src, kWave);
        }
        *reads += (src - lead) * R + __shfl(used, src, kWave);
        return res;
    }
    *reads += kWin;
    const uint32_t d = end - beg;
    const uint32_t jb = (uint32_t)(((uint64_t)r * (uint64_t)d) >> 32);
    for (uint32_t e = g.guide[beg + jb] + kWin; e < end; e += 4 * P) {
        const uint32_t e0 = e + 4 * sub;
        uint4 q[4];
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) q[j] = g.cs[e0 + j < end ? e0 + j : end - 1];
        uint32_t h = 4, u = 0;
#pragma unroll
        for (uint32_t j = 0; j < 4; ++j) {
            if (h == 4 && e0 + j < end) {
                ++u;
                if (r < q[j].x) {
                    h = j;
                    mine = q[j];
                }
            }
        }
        gb = group_bits<P>(__ballot(h < 4), lead);
        if (gb) {
            const uint32_t src = lead + (uint32_t)__ffs(gb) - 1u;
            res.y = __shfl(mine.y, src, kWave);
            res.z = __shfl(mine.z, src, kWave);
            res.w = __shfl(mine.w, src, kWave);
            *reads += (src - lead) * 4 + __shfl(u, src, kWave);
            break;
        }
        *reads += group_sum<P>(u);
    }
    return res;
}

// Is w among the len entries of the path that starts at stage[pos]? The
// walk's P lanes take turns over the path's aligned 16-byte groups, sixteen
// independent loads per lane per round; words of a group outside [pos, pos +
// len) are ignored. A group never crosses the end of the walk's chunk: every
// pass starts the staging cursor at a multiple of four, and the kernel
// reserves whole chunks of kLtChunk entries.
template <uint32_t P>
__device__ __forceinline__ bool on_path_group(const uint32_t* stage, uint64_t pos, uint32_t len,
                                              uint32_t w, uint32_t sub, uint32_t lead) {
    const uint64_t end = pos + len;
    const uint64_t last = (end - 1) & ~3ull;  // the group of the path's last entry
    for (uint64_t q = pos & ~3ull; q < end; q += 4 * kScanLoads * P) {
        bool hit = false;
        // kScanLoads loads in flight at once: groups past the end read the
        // path's last group again and count for nothing
        uint4 v[kScanLoads];
#pragma unroll
        for (uint32_t j = 0; j < kScanLoads; ++j) {
            const uint64_t b = q + 4 * (j * P + sub);
            v[j] = *reinterpret_cast<const uint4*>(stage + (b < end ? b : last));
        }
#pragma unroll
        for (uint32_t j = 0; j < kScanLoads; ++j) {
            const uint64_t b = q + 4 * (j * P + sub);
            if (b < end) {
                hit |= (v[j].x == w) & (b >= pos);
                hit |= (v[j].y == w) & (b + 1 >= pos) & (b + 1 < end);
                hit |= (v[j].z == w) & (b + 2 >= pos) & (b + 2 < end);
                hit |= (v[j].w == w) & (b + 3 >= pos) & (b + 3 < end);
            }
        }
        if (group_bits<P>(__ballot(hit), lead)) return true;
    }
    return false;
}

// BB: log2 of the per-walk path filter size in bits (10..12); P: lanes per
// walk. A wave runs 64/P walks. Every lane of a walk's group holds the same
// walk state and takes the same branches; the group's first lane alone does
// what must happen once per walk (count atomics, filter updates, ticket and
// chunk reservations, list appends), and every lane writes the path entries
// it later rescans. A smaller filter leaves more waves resident (more walks
// in flight) at the price of more false hits, each confirmed by a path
// rescan. The launch bounds hold the kernel to 96 VGPRs, five waves per SIMD
// (the LDS of 16 walks' 4096-bit filters allows five as well).
template <uint32_t BB, uint32_t P>
__global__ __launch_bounds__(64, 5) void lt_small_kernel(LtGraphDev g, SampleRange rg,
                                                         SampleOut o, uint32_t* ticket) {
    constexpr uint32_t kBloomWords = (1u << BB) / 32;
    constexpr uint32_t kWalks = kWave / P;
    __shared__ uint32_t bloom[kBloomWords * kWalks];
    const uint32_t lane = threadIdx.x;
    const uint32_t sub = lane % P, lead = lane - sub;
    const bool first = sub == 0;
    uint32_t* mb = bloom + (lane / P) * kBloomWords;  // this walk's filter
    // the wave's reservoir of sample positions [res_pos, res_end), claimed
    // from the ticket 64 at a time, and one per walk slot for the last
    // round of claims (uniform across the wave)
    uint32_t res_pos = 0, res_end = 0;

    constexpr uint32_t R = kWin / P;
    bool has = false, done = false, fresh = false, primed = false;
    // where the walk's members are counted: counts (sample index below
    // count_lim), counts_next (below count_lim2: the ids the next round will
    // take) or nowhere (drawn further ahead)
    uint32_t* cnt = nullptr;
    uint32_t idx = 0, cur = 0, len = 0, wstart = 0, chunk_used = kLtChunk;
    uint32_t cbeg = 0, cend = 0;  // cur's column
    uint32_t nbeg = 0, nend = 0;  // a new root's column, in flight
    uint32_t wr = 0;              // the draw at cur ...
    uint4 win[R];                 // ... and this lane's part of its window, in flight
#pragma unroll
    for (uint32_t j = 0; j < R; ++j) win[j] = make_uint4(0u, kNone, 0u, 0u);
    uint64_t s = 0, chunk_base = 0;
    uint32_t w_steps = 0, w_reads = 0;
    uint64_t st_sets = 0, st_entries = 0, st_steps = 0, st_reads = 0;

    const uint32_t total = rg.list ? *rg.list_n : rg.count;
    for (;;) {
        const bool need = !has && !done;
        const uint64_t mask = __ballot(need && first);
        if (mask) {
            const uint32_t want = (uint32_t)__popcll(mask);
            const uint32_t rank = (uint32_t)__popcll(mask & ((1ull << lead) - 1ull));
            const uint32_t have = res_end - res_pos;
            uint32_t pos;
            if (have >= want) {
                pos = res_pos + rank;
                res_pos += want;
            } else {
                // near the end of the positions (within one round of 64-wide
                // claims by every wave, judged by this wave's last claim) a
                // claim covers one walk per slot: a last wide claim would
                // leave a few waves with several walks per slot to run while
                // the rest of the GPU idles (want <= walk slots <= claim)
                const uint32_t claim =
                    (uint64_t)res_end + (uint64_t)gridDim.x * kWave >= total ? kWave / P : kWave;
                uint32_t nb = 0;
                if (lane == 0) nb = atomicAdd(ticket, claim);
                nb = __shfl(nb, 0, kWave);
                pos = rank < have ? res_pos + rank : nb + (rank - have);
                res_pos = nb + (want - have);
                res_end = nb + claim;
            }
            bool start = false;
            if (need) {
                if (pos >= total) {
                    done = true;
                } else {
                    idx = rg.list ? rg.list[pos] : pos;
                    s = rg.id_lo + idx;
                    cur = sample_root(rg.seed, s, g.n);
                    nbeg = g.off[cur];
                    nend = g.off[cur + 1];
                    bool ok = true;
                    if (chunk_used >= kLtChunk) {
                        unsigned long long nb = 0;
                        if (first) nb = atomicAdd(o.cursor, (unsigned long long)kLtChunk);
                        nb = __shfl(nb, lead, kWave);
                        if (nb + kLtChunk > o.stage_cap) {
                            if (first) o.retry[atomicAdd(o.retry_n, 1u)] = idx;
                            ok = false;
                        } else {
                            chunk_base = nb;
                            chunk_used = 0;
                        }
                    }
                    start = ok;
                }
            }
            // the whole wave clears each starting walk's filter in turn
            uint64_t smask = __ballot(start && first);
            while (smask) {
                const uint32_t l = (uint32_t)__ffsll((unsigned long long)smask) - 1u;
                smask &= smask - 1ull;
                for (uint32_t wd = lane; wd < kBloomWords; wd += kWave)
                    bloom[(l / P) * kBloomWords + wd] = 0u;
            }
            if (start) {
                wstart = chunk_used;
                o.stage[chunk_base + wstart] = cur;
                cnt = idx < o.count_lim ? o.counts
                                        : (idx < o.count_lim2 ? o.counts_next : nullptr);
                if (first) {
                    if (cnt) atomicAdd(&cnt[cur], 1u);
                    bloom_set<BB>(mb, cur);
                }
                len = 1;
                w_steps = 0;
                w_reads = 0;
                has = true;
                fresh = true;
                primed = false;
            }
        }
        // a walk slot whose start failed (staging full) takes the next
        // position: the wave leaves only when every slot has run past the
        // end, so no position it claimed from the ticket goes unprocessed
        if (!__any(has || !done)) break;
        // The step is software-pipelined: a walk's window for its current
        // vertex was issued in the previous iteration. As soon as the pick
        // names the next vertex, that vertex's draw and window go out, ahead
        // of the path check and of this step's writes (a load issued after a
        // store waits for the store too), and are dropped if the walk ends.
        // A walk started in an iteration draws at its root in the next one
        // (its column bounds load meanwhile) and picks in the one after.
        if (has && !fresh && !primed) {
            if (cbeg < cend) {
                wr = lt_draw(rg.seed, s, cur);
                ++w_steps;
                window_issue<P>(g, cbeg, cend, wr, sub, win);
            }
            primed = true;
        } else if (has && !fresh) {
            uint4 pk = make_uint4(0u, kNone, 0u, 0u);
            if (cbeg < cend) pk = window_pick<P>(g, cbeg, cend, wr, &w_reads, sub, lead, win);
            const uint32_t nxt = pk.y;
            bool finish = nxt == kNone;
            if (!finish) {
                // the pick has consumed wr and win: they take nxt's draw and
                // window (meaningless if the walk ends here)
                if (pk.z < pk.w) {
                    wr = lt_draw(rg.seed, s, nxt);
                    window_issue<P>(g, pk.z, pk.w, wr, sub, win);
                }
                if (bloom_test<BB>(mb, nxt) &&
                    on_path_group<P>(o.stage, chunk_base + wstart, len, nxt, sub, lead))
                    finish = true;
                if (!finish) {
                    bool keep = true;
                    if (wstart + len == kLtChunk) {
                        bool moved = false;
                        if (wstart != 0) {
                            unsigned long long nb = 0;
                            if (first) nb = atomicAdd(o.cursor, (unsigned long long)kLtChunk);
                            nb = __shfl(nb, lead, kWave);
                            if (nb + kLtChunk <= o.stage_cap) {
                                for (uint32_t t = 0; t < len; ++t)
                                    o.stage[nb + t] = o.stage[chunk_base + wstart + t];
                                chunk_base = nb;
                                wstart = 0;
                                moved = true;
                            } else if (first) {
                                o.retry[atomicAdd(o.retry_n, 1u)] = idx;
                            }
                        } else if (first) {
                            // the large-walk kernel resumes at nxt (checked
                            // to be off the path): the path stays in this
                            // chunk, whose offset and nxt go in the sample's
                            // slots; the steps taken so far count here
                            o.stage_off[idx] = chunk_base;
                            o.sizes[idx] = nxt;
                            st_steps += w_steps;
                            st_reads += w_reads;
                            o.defer[atomicAdd(o.defer_n, 1u)] = idx;
                        }
                        if (!moved) {
                            if (first && cnt)
                                for (uint32_t t = 0; t < len; ++t)
                                    atomicSub(&cnt[o.stage[chunk_base + wstart + t]], 1u);
                            // a deferred path keeps its chunk
                            chunk_used = wstart == 0 ? kLtChunk : wstart;
                            has = false;
                            keep = false;
                        }
                    }
                    if (keep) {
                        o.stage[chunk_base + wstart + len] = nxt;
                        if (first) {
                            if (cnt) atomicAdd(&cnt[nxt], 1u);
                            bloom_set<BB>(mb, nxt);
                        }
                        ++len;
                        cur = nxt;
                        cbeg = pk.z;
                        cend = pk.w;
                        if (cbeg < cend) ++w_steps;
                    }
                }
            }
            if (finish) {
                if (first) {
                    o.stage_off[idx] = chunk_base + wstart;
                    o.sizes[idx] = len;
                    st_sets += 1;
                    st_entries += len;
                    st_steps += w_steps;
                    st_reads += w_reads;
                }
                chunk_used = wstart + len;
                has = false;
            }
        }
        if (fresh) {
            cbeg = nbeg;
            cend = nend;
            fresh = false;
        }
    }
    st_sets = wave_sum64(st_sets);
    st_entries = wave_sum64(st_entries);
    st_steps = wave_sum64(st_steps);
    st_reads = wave_sum64(st_reads);
    if (lane == 0) {
        atomicAdd(&o.stats[kStMainSets], (unsigned long long)st_sets);
        atomicAdd(&o.stats[kStMainEntries], (unsigned long long)st_entries);
        atomicAdd(&o.stats[kStMainEdges], (unsigned long long)st_steps);
        atomicAdd(&o.stats[kStMainLive], (unsigned long long)st_reads);
    }
}

// Walks handed over by lt_small_kernel, one per wave: the wave marks the
// kLtChunk members it left staged in an exact visited bitmap in device memory
// (slot per workgroup) and copies them to the workgroup's queue, lane 0
// continues the walk from the vertex it was about to add, then the wave
// stages the whole path and counts it.
__global__ __launch_bounds__(64) void lt_large_kernel(LtGraphDev g, SampleRange rg, SampleOut o,
                                                      const uint32_t* list, const uint32_t* list_n,
                                                      uint32_t* fail, uint32_t* fail_n,
                                                      uint32_t* ticket, BigScratch b) {
    __shared__ uint32_t s_i, s_len;
    __shared__ unsigned long long s_off, s_steps, s_reads;
    const uint32_t lane = threadIdx.x;
    uint32_t* bm = b.bitmaps + (size_t)blockIdx.x * b.words;
    uint32_t* q = b.queues + (size_t)blockIdx.x * b.qcap;
    const uint32_t cnt = *list_n;
    uint64_t st_sets = 0, st_entries = 0, st_steps = 0, st_reads = 0;
    for (;;) {
        if (lane == 0) s_i = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t li = s_i;
        __syncthreads();
        if (li >= cnt) break;
        const uint32_t idx = list[li];
        const uint64_t s = rg.id_lo + idx;
        const uint64_t pre = o.stage_off[idx];
        for (uint32_t i = lane; i < kLtChunk; i += kWave) {
            const uint32_t u = o.stage[pre + i];
            q[i] = u;
            atomicOr(&bm[u >> 5], 1u << (u & 31));
        }
        __threadfence();
        __syncthreads();
        if (lane == 0) {
            uint32_t cur = o.sizes[idx];
            uint32_t beg = g.off[cur], end = g.off[cur + 1];
            uint32_t len = kLtChunk, steps = 0, reads = 0;
            q[len++] = cur;
            atomicOr(&bm[cur >> 5], 1u << (cur & 31));
            for (;;) {
                if (beg == end) break;
                const uint32_t r = lt_draw(rg.seed, s, cur);
                ++steps;
                const uint4 pk = lt_pick(g, beg, end, r, &reads);
                const uint32_t nxt = pk.y;
                if (nxt == kNone) break;
                const uint32_t bit = 1u << (nxt & 31);
                if (atomicOr(&bm[nxt >> 5], bit) & bit) break;
                q[len++] = nxt;
                cur = nxt;
                beg = pk.z;
                end = pk.w;
            }
            s_len = len;
            s_steps = steps;
            s_reads = reads;
            s_off = atomicAdd(o.cursor, (unsigned long long)len);
        }
        __syncthreads();
        const uint32_t len = s_len;
        const uint64_t off = s_off;
        const bool fits = off + len <= o.stage_cap;
        for (uint32_t i = lane; i < len; i += kWave) {
            const uint32_t u = q[i];
            if (fits) {
                o.stage[off + i] = u;
                if (idx < o.count_lim) atomicAdd(&o.counts[u], 1u);
                else if (idx < o.count_lim2) atomicAdd(&o.counts_next[u], 1u);
            }
            __hip_atomic_store(&bm[u >> 5], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        if (lane == 0) {
            if (fits) {
                o.stage_off[idx] = off;
                o.sizes[idx] = len;
                st_sets += 1;
                st_entries += len;
                st_steps += s_steps;
                st_reads += s_reads;
            } else {
                fail[atomicAdd(fail_n, 1u)] = idx;
            }
        }
        __syncthreads();
    }
    if (lane == 0) {
        atomicAdd(&o.stats[kStBigSets], (unsigned long long)st_sets);
        atomicAdd(&o.stats[kStBigEntries], (unsigned long long)st_entries);
        atomicAdd(&o.stats[kStBigEdges], (unsigned long long)st_steps);
        atomicAdd(&o.stats[kStBigLive], (unsigned long long)st_reads);
    }
}

// guide[beg + j] = first e in [beg, end) with cum[e] > ceil(j 2^32 / d) - 1,
// or end if there is none, and the window gw[kWin (beg + j) + k] =
// cs[guide[beg + j] + k] (k < kWin; an empty record, src = kNone, past the
// column), for every column (64 columns per wave).
__global__ __launch_bounds__(64) void lt_guide_kernel(const uint32_t* off, const uint4* cs,
                                                      uint32_t* guide, uint4* gw, uint32_t n) {
    const uint64_t v = (uint64_t)blockIdx.x * kWave + threadIdx.x;
    uint32_t sz = 0;
    uint64_t beg = 0;
    if (v < n) {
        beg = off[v];
        sz = off[v + 1] - (uint32_t)beg;
    }
    wave_segments(sz, beg, sz, [&](uint32_t, uint64_t b0, uint64_t d, uint32_t j) {
        const uint64_t lo = (((uint64_t)j << 32) + d - 1) / d;  // smallest r in bucket j
        uint32_t a = (uint32_t)b0, z = (uint32_t)(b0 + d);      // first e with cum[e] > lo
        while (a < z) {
            const uint32_t mid = a + ((z - a) >> 1);
            if ((uint64_t)cs[mid].x > lo) z = mid; else a = mid + 1;
        }
        guide[b0 + j] = a;
#pragma unroll
        for (uint32_t k = 0; k < kWin; ++k)
            gw[(uint64_t)kWin * (b0 + j) + k] =
                a + k < b0 + d ? cs[a + k] : make_uint4(0u, kNone, 0u, 0u);
    });
}

}  // namespace

uint32_t lt_small_grid(int device, uint32_t bloom_bits, uint32_t lanes) {
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    // resident waves per CU as LDS allows (64 / lanes walks x 2^bits bits
    // each, 160 KB per CU), twice over
    const uint32_t lds = (1u << bloom_bits) / 8 * (kWave / lanes);
    uint32_t per_cu = (160u * 1024u) / lds;
    if (per_cu > 32) per_cu = 32;
    return (uint32_t)cus * per_cu * 2u;
}

template <uint32_t P>
hipError_t launch_lt_small_p(const LtGraphDev& g, const SampleRange& r, const SampleOut& o,
                             uint32_t* ticket, uint32_t bloom_bits, uint32_t grid, hipStream_t st) {
    switch (bloom_bits) {
        case 10:
            hipLaunchKernelGGL((lt_small_kernel<10, P>), dim3(grid), dim3(kWave), 0, st, g, r, o,
                               ticket);
            break;
        case 11:
            hipLaunchKernelGGL((lt_small_kernel<11, P>), dim3(grid), dim3(kWave), 0, st, g, r, o,
                               ticket);
            break;
        case 12:
            hipLaunchKernelGGL((lt_small_kernel<12, P>), dim3(grid), dim3(kWave), 0, st, g, r, o,
                               ticket);
            break;
        default:
            return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_lt_small(const LtGraphDev& g, const SampleRange& r, const SampleOut& o,
                           uint32_t* ticket, uint32_t bloom_bits, uint32_t lanes, uint32_t grid,
                           hipStream_t st) {
    const uint32_t walks = kWave / (lanes ? lanes : 1u);
    const uint32_t need = (r.count + walks - 1) / walks;
    if (grid > need) grid = need;
    if (grid == 0) return hipSuccess;
    switch (lanes) {
        case 1: return launch_lt_small_p<1>(g, r, o, ticket, bloom_bits, grid, st);
        case 2: return launch_lt_small_p<2>(g, r, o, ticket, bloom_bits, grid, st);
        case 4: return launch_lt_small_p<4>(g, r, o, ticket, bloom_bits, grid, st);
        default: return hipErrorInvalidValue;
    }
}

hipError_t launch_lt_large(const LtGraphDev& g, const SampleRange& r, const SampleOut& o,
                           const uint32_t* list, const uint32_t* list_n, uint32_t* fail,
                           uint32_t* fail_n, uint32_t* ticket, const BigScratch& b,
                           hipStream_t st) {
    if (b.slots == 0 || b.qcap != g.n) return hipErrorInvalidValue;
    hipLaunchKernelGGL(lt_large_kernel, dim3(b.slots), dim3(kWave), 0, st, g, r, o, list, list_n,
                       fail, fail_n, ticket, b);
    return hipGetLastError();
}

hipError_t launch_lt_guide(const uint32_t* off, const uint4* cs, uint32_t* guide, uint4* gw,
                           uint32_t n, hipStream_t st) {
    const uint32_t blocks = (n + kWave - 1) / kWave;
    hipLaunchKernelGGL(lt_guide_kernel, dim3(blocks), dim3(kWave), 0, st, off, cs, guide, gw, n);
    return hipGetLastError();
}

}  // namespace imm
