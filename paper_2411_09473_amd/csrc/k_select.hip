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
//    atomic bit and cut into chunks of at most 64 members on a work queue.
//  * decrement: the instance's waves take chunks from its queue and
//    decrement the counts of the members (except the chosen vertex), so a
//    few very large covered sets are spread over many waves. When the queue
//    is long, decrements are summed per workgroup in LDS first.
#include <algorithm>

#include "device_common.hpp"
#include "imm_internal.hpp"

namespace imm {

namespace {

constexpr uint32_t kArgBS = 256;
constexpr uint32_t kClaimBS = 256;
constexpr uint32_t kDecBS = 256;

__device__ __forceinline__ uint64_t vkey(uint32_t c, uint32_t v) {
    return c == kSelected ? 0ull : (((uint64_t)c << 32) | (uint64_t)(~v));
}

// The instance whose block range [lo, lo + cnt) holds block b (ranges are
// ascending and disjoint); nq when none does.
__device__ __forceinline__ uint32_t find_inst(const SelectDesc* d, uint32_t nq, uint32_t b,
                                              bool argmax) {
    uint32_t lo = 0, hi = nq;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((argmax ? d[mid].arg_lo : d[mid].sel_lo) <= b) lo = mid; else hi = mid;
    }
    const uint32_t l = argmax ? d[lo].arg_lo : d[lo].sel_lo;
    const uint32_t c = argmax ? d[lo].arg_cnt : d[lo].sel_cnt;
    return (b >= l && b < l + c) ? lo : nq;
}

__global__ __launch_bounds__(kArgBS) void argmax_kernel(const SelectDesc* descs, uint32_t nq,
                                                        uint32_t t) {
    __shared__ uint64_t s_w[kArgBS / kWave];
    const uint32_t q = find_inst(descs, nq, blockIdx.x, true);
    if (q == nq) return;
    const SelectDesc& d = descs[q];
    if (t >= d.k) return;
    const uint32_t* cw = d.cw;
    const uint32_t n = d.n;
    const uint32_t blk = blockIdx.x - d.arg_lo;
    const uint32_t tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const uint32_t gtid = blk * kArgBS + tid, gthreads = d.arg_cnt * kArgBS;
    uint64_t best = 0;
    const uint32_t n4 = n >> 2;
    const uint4* cw4 = reinterpret_cast<const uint4*>(cw);
    for (uint32_t x = gtid; x < n4; x += gthreads) {
        const uint4 c = cw4[x];
        const uint32_t v = x << 2;
        uint64_t k = vkey(c.x, v);
        uint64_t y = vkey(c.y, v + 1); k = y > k ? y : k;
        y = vkey(c.z, v + 2); k = y > k ? y : k;
        y = vkey(c.w, v + 3); k = y > k ? y : k;
        best = k > best ? k : best;
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
        atomicMax(&d.slots[(uint64_t)t * kArgSlots + blk % kArgSlots], (unsigned long long)b);
    }
}

__device__ __forceinline__ uint64_t slots_max(const unsigned long long* slots) {
    uint64_t m = 0;
#pragma unroll
    for (uint32_t x = 0; x < kArgSlots; ++x) m = slots[x] > m ? slots[x] : m;
    return m;
}

__global__ __launch_bounds__(kClaimBS) void claim_kernel(const SelectDesc* descs, uint32_t nq,
                                                         uint32_t t) {
    const uint32_t q = find_inst(descs, nq, blockIdx.x, false);
    if (q == nq) return;
    const SelectDesc& d = descs[q];
    if (t >= d.k) return;
    const uint32_t blk = blockIdx.x - d.sel_lo;
    const uint64_t m = slots_max(d.slots + (uint64_t)t * kArgSlots);
    const uint32_t v = ~(uint32_t)m;
    if (blk == 0 && threadIdx.x == 0) {
        d.seeds[t] = v;
        d.gains[t] = (uint32_t)(m >> 32);
        d.cw[v] = kSelected;
    }
    uint32_t* chunk_n = d.chunk_n + t;
    const uint64_t step = (uint64_t)d.sel_cnt * kClaimBS;
    const uint32_t lane = threadIdx.x % kWave;
    for (uint32_t seg = 0; seg < d.nseg; ++seg) {
        const uint64_t* io = d.inv_offs + (uint64_t)seg * ((uint64_t)d.n + 1);
        const uint64_t lb = io[v], len = io[v + 1] - lb;
        for (uint64_t base = (uint64_t)blk * kClaimBS; base < len; base += step) {
            const uint64_t i = base + threadIdx.x;
            uint32_t nch = 0;
            uint64_t a = 0, sz = 0;
            if (i < len) {
                const uint32_t j = d.inv_set[lb + i];
                const uint32_t bit = 1u << (j & 31);
                const uint32_t old = atomicOr(&d.covered[j >> 5], bit);
                if (!(old & bit)) {
                    a = d.set_off[j];
                    sz = d.set_off[j + 1] - a;
                    nch = (uint32_t)((sz + kWave - 1) / kWave);
                }
            }
            // one queue reservation per wave
            const uint32_t incl = wave_incl_scan(nch);
            const uint32_t tot = __shfl(incl, kWave - 1, kWave);
            uint32_t wbase = 0;
            if (lane == kWave - 1 && tot) wbase = atomicAdd(chunk_n, tot);
            wbase = __shfl(wbase, kWave - 1, kWave);
            const uint32_t pos = wbase + incl - nch;
            for (uint32_t c = 0; c < nch; ++c) {
                const uint64_t o = (uint64_t)c * kWave;
                d.chunks[pos + c] = Chunk{a + o, (uint32_t)(sz - o < kWave ? sz - o : kWave), 0u};
            }
        }
    }
}

// Decrements summed per workgroup in an LDS table (vertex -> count) are
// applied with one atomic per distinct vertex: the sets a seed covers share
// their high-degree vertices, which would otherwise take one global atomic
// per covering set. A vertex that finds no slot within a few probes is
// decremented directly.
constexpr uint32_t kAggBits = 12;
constexpr uint32_t kAggSize = 1u << kAggBits;
constexpr uint32_t kAggProbes = 8;

__global__ __launch_bounds__(kDecBS) void decrement_kernel(const SelectDesc* descs, uint32_t nq,
                                                           uint32_t t) {
    __shared__ uint32_t h_key[kAggSize], h_cnt[kAggSize];
    const uint32_t q = find_inst(descs, nq, blockIdx.x, false);
    if (q == nq) return;
    const SelectDesc& d = descs[q];
    if (t >= d.k) return;
    const uint32_t blk = blockIdx.x - d.sel_lo;
    const uint32_t nchunks = d.chunk_n[t];
    const uint32_t wpb = kDecBS / kWave;
    if (blk * wpb >= nchunks) return;
    uint32_t* cw = d.cw;
    const uint32_t v = d.seeds[t];
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t wid = blk * wpb + threadIdx.x / kWave;
    const uint32_t nw = d.sel_cnt * wpb;
    const bool agg = nchunks >= 4 * nw;
    if (agg) {
        for (uint32_t x = threadIdx.x; x < kAggSize; x += kDecBS) {
            h_key[x] = kEmpty;
            h_cnt[x] = 0;
        }
        __syncthreads();
    }
    for (uint32_t c = wid; c < nchunks; c += nw) {
        const Chunk ch = d.chunks[c];
        if (lane < ch.len) {
            const uint32_t u = d.set_vtx[ch.off + lane];
            if (u != v) {
                bool done = false;
                if (agg) {
                    uint32_t slot = (u * 0x9E3779B1u) >> (32 - kAggBits);
                    for (uint32_t p = 0; p < kAggProbes; ++p) {
                        uint32_t cur = h_key[slot];
                        if (cur == kEmpty) cur = atomicCAS(&h_key[slot], kEmpty, u);
                        if (cur == kEmpty || cur == u) {
                            atomicAdd(&h_cnt[slot], 1u);
                            done = true;
                            break;
                        }
                        slot = (slot + 1) & (kAggSize - 1);
                    }
                }
                if (!done) atomicSub(&cw[u], 1u);
            }
        }
    }
    if (agg) {
        __syncthreads();
        for (uint32_t x = threadIdx.x; x < kAggSize; x += kDecBS) {
            const uint32_t c = h_cnt[x];
            if (c) atomicSub(&cw[h_key[x]], c);
        }
    }
}

}  // namespace

uint32_t argmax_blocks(uint32_t n) {
    uint32_t g = (n / 4 + kArgBS * 4 - 1) / (kArgBS * 4);
    if (g < 1) g = 1;
    if (g > 512) g = 512;
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

hipError_t launch_select_step(const SelectDesc* descs, uint32_t nq, uint32_t t,
                              uint32_t arg_blocks, uint32_t sel_blocks, hipStream_t st) {
    hipLaunchKernelGGL(argmax_kernel, dim3(arg_blocks), dim3(kArgBS), 0, st, descs, nq, t);
    hipLaunchKernelGGL(claim_kernel, dim3(sel_blocks), dim3(kClaimBS), 0, st, descs, nq, t);
    hipLaunchKernelGGL(decrement_kernel, dim3(sel_blocks), dim3(kDecBS), 0, st, descs, nq, t);
    return hipGetLastError();
}

}  // namespace imm
