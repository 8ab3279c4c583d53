// k_sample_ic.hip -- IC reverse-BFS RRR sampling with fused occurrence counts
// (Generate_RRRsets with in-place counter updates, Algorithm 3; IC model,
// Section II-A).
//
// Two kernels share the work of one sampling round:
//  * ic_small: a wave takes 64 sample ids at a time. First each lane draws
//    the root of its own sample and flips the coins of the root's in-edges
//    (roots of in-degree <= kLaneDegCap); a root with no live in-edge is a
//    complete set {root}, stored at once (at low edge probabilities that is
//    most samples). The other samples of the batch then run one at a time,
//    one wave per sample: the set doubles as the BFS queue and lives in LDS
//    together with an open-addressing hash of visited vertices.
//    Each BFS level takes up to 64 queued vertices, and the wave walks their
//    in-edges in aligned groups of four: one Philox call yields the four
//    coins of a group and one 16-byte load its four thresholds; sources are
//    gathered only for live edges. A set that outgrows LDS is abandoned
//    (no side effects) and its sample index deferred.
//  * ic_large: one workgroup per deferred sample, with a visited bitmap and a
//    queue in device memory (one slot per workgroup, reset sparsely). A slot
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

constexpr uint32_t kSmallCap = 256;     // members kept in LDS
constexpr uint32_t kHashBits = 10;      // 1024-slot LDS hash (load < 0.32)
constexpr uint32_t kHashSize = 1u << kHashBits;
constexpr uint32_t kTicketChunk = kIcTicketChunk;  // one sample id per lane
constexpr uint32_t kLaneDegCap = 32;  // roots tried one per lane up to this in-degree
constexpr uint32_t kStageChunk = kIcStageChunk;
constexpr uint32_t kBigBlock = 256;

__device__ __forceinline__ uint32_t hslot(uint32_t v) { return (v * 0x9E3779B1u) >> (32 - kHashBits); }

__device__ __forceinline__ uint32_t lds_load(const uint32_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Insert u into the LDS visited hash; append it to the member list when new.
__device__ __forceinline__ void small_insert(uint32_t u, uint32_t* hash, uint32_t* members,
                                             uint32_t* s_size, uint32_t* s_over) {
    uint32_t slot = hslot(u);
    for (uint32_t probe = 0; probe < kHashSize; ++probe) {
        const uint32_t cur = lds_load(&hash[slot]);
        if (cur == u) return;
        if (cur == kEmpty) {
            if (lds_load(s_size) >= kSmallCap) {
                *s_over = 1u;
                return;
            }
            const uint32_t old = atomicCAS(&hash[slot], kEmpty, u);
            if (old == kEmpty) {
                const uint32_t pos = atomicAdd(s_size, 1u);
                if (pos < kSmallCap) members[pos] = u; else *s_over = 1u;
                return;
            }
            if (old == u) return;
        }
        slot = (slot + 1) & (kHashSize - 1);
    }
    *s_over = 1u;
}

__global__ __launch_bounds__(64) void ic_small_kernel(IcGraphDev g, SampleRange rg, SampleOut o,
                                                      uint32_t* ticket) {
    __shared__ uint32_t hash[kHashSize];
    __shared__ uint32_t members[kSmallCap];
    __shared__ uint32_t s_base[kWave], s_g0[kWave], s_beg[kWave], s_end[kWave];
    __shared__ uint32_t s_pend[kWave];
    __shared__ uint32_t s_size, s_over, s_tk;
    __shared__ unsigned long long s_chunk;

    const uint32_t lane = threadIdx.x;
    const uint32_t k0 = (uint32_t)rg.seed, k1 = (uint32_t)(rg.seed >> 32);
    for (uint32_t i = lane; i < kHashSize; i += kWave) hash[i] = kEmpty;

    uint64_t chunk_base = 0;
    uint32_t chunk_left = 0;  // uniform across the wave
    uint64_t st_sets = 0, st_entries = 0, st_edges = 0, st_live = 0;  // lane-partial

    // Reserve `need` staging entries from the wave's chunk (a new chunk when
    // the current one is too short); false when the staging buffer is full.
    auto reserve = [&](uint32_t need, uint64_t* off) -> bool {
        if (need > chunk_left) {
            if (lane == 0) s_chunk = atomicAdd(o.cursor, (unsigned long long)kStageChunk);
            __syncthreads();
            chunk_base = s_chunk;
            chunk_left = kStageChunk;
            __syncthreads();
            if (chunk_base + kStageChunk > o.stage_cap) {
                chunk_left = 0;
                return false;
            }
        }
        *off = chunk_base + (kStageChunk - chunk_left);
        chunk_left -= need;
        return true;
    };

    const uint32_t total = rg.list ? *rg.list_n : rg.count;
    for (;;) {
        if (lane == 0) s_tk = atomicAdd(ticket, kTicketChunk);
        __syncthreads();
        const uint32_t base_pos = s_tk;
        __syncthreads();
        if (base_pos >= total) break;

        // ---- one sample per lane: a root without a live in-edge is a
        // complete set {root}; the others go to the wave-per-sample BFS
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
                const uint32_t rr[4] = {r.x, r.y, r.z, r.w};
                const uint32_t tt[4] = {th.x, th.y, th.z, th.w};
#pragma unroll
                for (uint32_t j = 0; j < 4; ++j) {
                    const uint32_t e = e0 + j;
                    if (e >= rbeg && e < rend && rr[j] < tt[j]) single = false;
                }
            }
        }
        const uint64_t smask = __ballot(single);
        const uint32_t nsingle = (uint32_t)__popcll(smask);
        if (nsingle) {
            uint64_t off = 0;
            const bool ok = reserve(nsingle, &off);
            const uint32_t rank = (uint32_t)__popcll(smask & ((1ull << lane) - 1ull));
            if (single) {
                if (ok) {
                    o.stage[off + rank] = root;
                    atomicAdd(&o.counts[root], 1u);
                    o.stage_off[my_idx] = off + rank;
                    o.sizes[my_idx] = 1;
                    st_sets += 1;
                    st_entries += 1;
                    st_edges += rend - rbeg;
                } else {
                    o.retry[atomicAdd(o.retry_n, 1u)] = my_idx;
                }
            }
        }
        const uint64_t pmask = __ballot(valid && !single);
        const uint32_t npend = (uint32_t)__popcll(pmask);
        if (valid && !single) s_pend[__popcll(pmask & ((1ull << lane) - 1ull))] = my_idx;
        __syncthreads();

        // ---- wave-per-sample BFS for the remaining samples of this batch
        for (uint32_t pi = 0; pi < npend; ++pi) {
            const uint32_t idx = s_pend[pi];
            const uint64_t s = rg.id_lo + idx;
            const uint32_t slo = (uint32_t)s, shi = (uint32_t)(s >> 32);
            if (lane == 0) {
                const uint32_t r0 = sample_root(rg.seed, s, g.n);
                members[0] = r0;
                hash[hslot(r0)] = r0;
                s_size = 1;
                s_over = 0;
            }
            __syncthreads();

            uint32_t head = 0, size = 1;
            uint32_t my_edges = 0, my_live = 0;
            while (head < size) {
                const uint32_t nb = min(kWave, size - head);
                uint32_t beg = 0, end = 0;
                if (lane < nb) {
                    const uint32_t v = members[head + lane];
                    beg = g.off[v];
                    end = g.off[v + 1];
                }
                const uint32_t ng = end > beg ? ((end + 3) >> 2) - (beg >> 2) : 0u;
                const uint32_t incl = wave_incl_scan(ng);
                const uint32_t G = __shfl(incl, kWave - 1, kWave);
                s_base[lane] = incl - ng;
                s_g0[lane] = beg >> 2;
                s_beg[lane] = beg;
                s_end[lane] = end;
                my_edges += end - beg;
                __syncthreads();
                uint32_t ow = 0;
                for (uint32_t base = 0; base < G; base += kWave) {
                    if (lds_load(&s_over)) break;
                    const uint32_t t = base + lane;
                    if (t < G) {
                        ow = owner_from(s_base, nb, t, ow);
                        const uint32_t grp = s_g0[ow] + (t - s_base[ow]);
                        const uint32_t eb = s_beg[ow], ee = s_end[ow];
                        const uint4 th = *reinterpret_cast<const uint4*>(g.thr + 4ull * grp);
                        const Philox4 r = philox10(grp, slo, shi, 1u, k0, k1);
                        const uint32_t e0 = grp << 2;
                        const uint32_t rr[4] = {r.x, r.y, r.z, r.w};
                        const uint32_t tt[4] = {th.x, th.y, th.z, th.w};
#pragma unroll
                        for (uint32_t j = 0; j < 4; ++j) {
                            const uint32_t e = e0 + j;
                            if (e >= eb && e < ee && rr[j] < tt[j]) {
                                ++my_live;
                                small_insert(g.src[e], hash, members, &s_size, &s_over);
                            }
                        }
                    }
                }
                __syncthreads();
                head += nb;
                size = s_size;
                const uint32_t over = s_over;
                __syncthreads();
                if (over) break;
            }

            const bool over = s_over != 0u;
            if (over) {
                if (lane == 0) o.defer[atomicAdd(o.defer_n, 1u)] = idx;
            } else {
                uint64_t off = 0;
                if (reserve(size, &off)) {
                    for (uint32_t i = lane; i < size; i += kWave) {
                        const uint32_t u = members[i];
                        o.stage[off + i] = u;
                        atomicAdd(&o.counts[u], 1u);
                    }
                    if (lane == 0) {
                        o.stage_off[idx] = off;
                        o.sizes[idx] = size;
                        st_sets += 1;
                        st_entries += size;
                    }
                    st_edges += my_edges;
                    st_live += my_live;
                } else if (lane == 0) {
                    o.retry[atomicAdd(o.retry_n, 1u)] = idx;
                }
            }
            // reset the hash slots this sample used (all members are present)
            const uint32_t used = min(size, kSmallCap);
            __syncthreads();
            for (uint32_t i = lane; i < used; i += kWave) {
                const uint32_t u = members[i];
                uint32_t slot = hslot(u);
                for (uint32_t probe = 0; probe < kHashSize; ++probe) {
                    if (hash[slot] == u) { hash[slot] = kEmpty; break; }
                    slot = (slot + 1) & (kHashSize - 1);
                }
            }
            if (over) {
                // an abandoned set may have hashed vertices beyond the list
                for (uint32_t i = lane; i < kHashSize; i += kWave) hash[i] = kEmpty;
            }
            __syncthreads();
        }
    }
    st_sets = wave_sum64(st_sets);
    st_entries = wave_sum64(st_entries);
    st_edges = wave_sum64(st_edges);
    st_live = wave_sum64(st_live);
    if (lane == 0) {
        atomicAdd(&o.stats[kStMainSets], (unsigned long long)st_sets);
        atomicAdd(&o.stats[kStMainEntries], (unsigned long long)st_entries);
        atomicAdd(&o.stats[kStMainEdges], (unsigned long long)st_edges);
        atomicAdd(&o.stats[kStMainLive], (unsigned long long)st_live);
    }
}

// Block-wide exclusive scan of one uint32 per thread; returns the total.
template <uint32_t BS>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* excl_out,
                                                    uint32_t* s_wsum) {
    const uint32_t tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const uint32_t incl = wave_incl_scan(v);
    if (lane == kWave - 1) s_wsum[w] = incl;
    __syncthreads();
    uint32_t before = 0, total = 0;
#pragma unroll
    for (uint32_t i = 0; i < BS / kWave; ++i) {
        const uint32_t x = s_wsum[i];
        if (i < w) before += x;
        total += x;
    }
    *excl_out = before + incl - v;
    return total;
}

__global__ __launch_bounds__(kBigBlock) void ic_large_kernel(IcGraphDev g, SampleRange rg,
                                                             SampleOut o, const uint32_t* list,
                                                             const uint32_t* list_n,
                                                             uint32_t* fail, uint32_t* fail_n,
                                                             uint32_t* ticket, BigScratch b) {
    __shared__ uint32_t s_base[kBigBlock], s_g0[kBigBlock], s_beg[kBigBlock], s_end[kBigBlock];
    __shared__ uint32_t s_wsum[kBigBlock / kWave];
    __shared__ uint32_t s_size, s_i;
    __shared__ unsigned long long s_off;

    const uint32_t tid = threadIdx.x;
    const uint32_t k0 = (uint32_t)rg.seed, k1 = (uint32_t)(rg.seed >> 32);
    uint32_t* bm = b.bitmaps + (size_t)blockIdx.x * b.words;
    uint32_t* q = b.queues + (size_t)blockIdx.x * g.n;
    const uint32_t cnt = *list_n;
    uint64_t st_sets = 0, st_entries = 0, st_edges = 0, st_live = 0;

    for (;;) {
        if (tid == 0) s_i = atomicAdd(ticket, 1u);
        __syncthreads();
        const uint32_t li = s_i;
        __syncthreads();
        if (li >= cnt) break;
        const uint32_t idx = list[li];
        const uint64_t s = rg.id_lo + idx;
        const uint32_t slo = (uint32_t)s, shi = (uint32_t)(s >> 32);
        if (tid == 0) {
            const uint32_t root = sample_root(rg.seed, s, g.n);
            q[0] = root;
            atomicOr(&bm[root >> 5], 1u << (root & 31));
            s_size = 1;
        }
        __syncthreads();

        uint32_t head = 0, size = 1;
        uint32_t my_edges = 0, my_live = 0;
        while (head < size) {
            const uint32_t nb = min(kBigBlock, size - head);
            uint32_t beg = 0, end = 0;
            if (tid < nb) {
                const uint32_t v = q[head + tid];
                beg = g.off[v];
                end = g.off[v + 1];
            }
            const uint32_t ng = end > beg ? ((end + 3) >> 2) - (beg >> 2) : 0u;
            uint32_t excl;
            const uint32_t G = block_excl_scan<kBigBlock>(ng, &excl, s_wsum);
            s_base[tid] = excl;
            s_g0[tid] = beg >> 2;
            s_beg[tid] = beg;
            s_end[tid] = end;
            my_edges += end - beg;
            __syncthreads();
            uint32_t ow = 0;
            for (uint32_t base = 0; base < G; base += kBigBlock) {
                const uint32_t t = base + tid;
                if (t < G) {
                    ow = owner_from(s_base, nb, t, ow);
                    const uint32_t grp = s_g0[ow] + (t - s_base[ow]);
                    const uint32_t eb = s_beg[ow], ee = s_end[ow];
                    const uint4 th = *reinterpret_cast<const uint4*>(g.thr + 4ull * grp);
                    const Philox4 r = philox10(grp, slo, shi, 1u, k0, k1);
                    const uint32_t e0 = grp << 2;
                    const uint32_t rr[4] = {r.x, r.y, r.z, r.w};
                    const uint32_t tt[4] = {th.x, th.y, th.z, th.w};
#pragma unroll
                    for (uint32_t j = 0; j < 4; ++j) {
                        const uint32_t e = e0 + j;
                        if (e >= eb && e < ee && rr[j] < tt[j]) {
                            ++my_live;
                            const uint32_t u = g.src[e];
                            const uint32_t bit = 1u << (u & 31);
                            const uint32_t old = atomicOr(&bm[u >> 5], bit);
                            if (!(old & bit)) q[atomicAdd(&s_size, 1u)] = u;
                        }
                    }
                }
            }
            __syncthreads();
            head += nb;
            size = s_size;
            __syncthreads();
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
    st_edges = wave_sum64(st_edges);
    st_live = wave_sum64(st_live);
    if (tid % kWave == 0) {
        atomicAdd(&o.stats[kStBigEdges], (unsigned long long)st_edges);
        atomicAdd(&o.stats[kStBigLive], (unsigned long long)st_live);
    }
    if (tid == 0) {
        atomicAdd(&o.stats[kStBigSets], (unsigned long long)st_sets);
        atomicAdd(&o.stats[kStBigEntries], (unsigned long long)st_entries);
    }
}

}  // namespace

uint32_t ic_small_grid(int device) {
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    return (uint32_t)cus * 24u;
}

hipError_t launch_ic_small(const IcGraphDev& g, const SampleRange& r, const SampleOut& o,
                           uint32_t* ticket, uint32_t grid, hipStream_t st) {
    const uint32_t need = (r.count + kTicketChunk - 1) / kTicketChunk;
    if (grid > need) grid = need;
    if (grid == 0) return hipSuccess;
    hipLaunchKernelGGL(ic_small_kernel, dim3(grid), dim3(kWave), 0, st, g, r, o, ticket);
    return hipGetLastError();
}

hipError_t launch_ic_large(const IcGraphDev& g, const SampleRange& r, const SampleOut& o,
                           const uint32_t* list, const uint32_t* list_n, uint32_t* fail,
                           uint32_t* fail_n, uint32_t* ticket, const BigScratch& b,
                           hipStream_t st) {
    if (b.slots == 0) return hipErrorInvalidValue;
    hipLaunchKernelGGL(ic_large_kernel, dim3(b.slots), dim3(kBigBlock), 0, st, g, r, o, list,
                       list_n, fail, fail_n, ticket, b);
    return hipGetLastError();
}

}  // namespace imm
