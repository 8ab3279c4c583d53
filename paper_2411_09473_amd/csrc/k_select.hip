// k_select.hip -- greedy max-coverage seed selection (Find_Most_Influential_Set,
// Algorithm 2) over the device-resident pool.
//
// One seed costs three launches and no host round trip:
//  * argmax: the two-step reduction of the paper's PARALLEL_REDUCTION. Each
//    workgroup reduces its part of the counts (regional maximum) and folds it
//    into one of kArgSlots partial slots with a 64-bit atomic max; the next
//    kernel reduces the slots (global maximum). A vertex is the packed key
//    count<<32 | ~id, so a plain max picks the largest count and, among equal
//    counts, the lowest id. A chosen vertex's count becomes a sentinel that
//    maps to key 0, which keeps it out of later picks.
//  * claim: the chosen vertex's inverted-index list names exactly the sets
//    that contain it ("if v in R" of Algorithm 2 without scanning all sets);
//    each one not yet covered is claimed with an atomic bit and cut into
//    chunks of at most 64 members appended to a work queue.
//  * decrement: all waves of the GPU take chunks from the queue and decrement
//    the counts of the members (except the chosen vertex), so a few very
//    large covered sets are spread over the whole device.
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

__global__ __launch_bounds__(kArgBS) void argmax_kernel(const uint32_t* cw, uint32_t n,
                                                        unsigned long long* slots) {
    __shared__ uint64_t s_w[kArgBS / kWave];
    const uint32_t tid = threadIdx.x, w = tid / kWave, lane = tid % kWave;
    const uint32_t gtid = blockIdx.x * kArgBS + tid, gthreads = gridDim.x * kArgBS;
    uint64_t best = 0;
    const uint32_t n4 = n >> 2;
    const uint4* cw4 = reinterpret_cast<const uint4*>(cw);
    for (uint32_t q = gtid; q < n4; q += gthreads) {
        const uint4 c = cw4[q];
        const uint32_t v = q << 2;
        uint64_t k = vkey(c.x, v);
        uint64_t t = vkey(c.y, v + 1); k = t > k ? t : k;
        t = vkey(c.z, v + 2); k = t > k ? t : k;
        t = vkey(c.w, v + 3); k = t > k ? t : k;
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
        atomicMax(&slots[blockIdx.x % kArgSlots], (unsigned long long)b);
    }
}

__device__ __forceinline__ uint64_t slots_max(const unsigned long long* slots) {
    uint64_t m = 0;
#pragma unroll
    for (uint32_t x = 0; x < kArgSlots; ++x) m = slots[x] > m ? slots[x] : m;
    return m;
}

__global__ __launch_bounds__(kClaimBS) void claim_kernel(const uint64_t* inv_off, uint32_t nseg,
                                                         uint32_t n, const uint32_t* inv_set,
                                                         const uint64_t* set_off,
                                                         uint32_t* covered, uint32_t* cw,
                                                         const unsigned long long* slots,
                                                         uint32_t* seeds, uint32_t* gains,
                                                         uint32_t i, Chunk* chunks,
                                                         uint32_t* chunk_n) {
    const uint64_t m = slots_max(slots);
    const uint32_t v = ~(uint32_t)m;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        seeds[i] = v;
        gains[i] = (uint32_t)(m >> 32);
        cw[v] = kSelected;
    }
    const uint64_t step = (uint64_t)gridDim.x * kClaimBS;
    const uint32_t lane = threadIdx.x % kWave;
    for (uint32_t seg = 0; seg < nseg; ++seg) {
        const uint64_t* io = inv_off + (uint64_t)seg * ((uint64_t)n + 1);
        const uint64_t lb = io[v], len = io[v + 1] - lb;
        for (uint64_t base = (uint64_t)blockIdx.x * kClaimBS; base < len; base += step) {
            const uint64_t t = base + threadIdx.x;
            uint32_t nch = 0;
            uint64_t a = 0, sz = 0;
            if (t < len) {
                const uint32_t j = inv_set[lb + t];
                const uint32_t bit = 1u << (j & 31);
                const uint32_t old = atomicOr(&covered[j >> 5], bit);
                if (!(old & bit)) {
                    a = set_off[j];
                    sz = set_off[j + 1] - a;
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
                chunks[pos + c] = Chunk{a + o, (uint32_t)(sz - o < kWave ? sz - o : kWave), 0u};
            }
        }
    }
}

// When the queue is long (a seed covering many sets), decrements are first
// summed per workgroup in an LDS table (vertex -> count) and applied with one
// atomic per distinct vertex: covered sets share their high-degree vertices,
// which would otherwise take one global atomic per covering set. A vertex
// that finds no slot within a few probes is decremented directly.
constexpr uint32_t kAggBits = 12;
constexpr uint32_t kAggSize = 1u << kAggBits;
constexpr uint32_t kAggProbes = 8;

__global__ __launch_bounds__(kDecBS) void decrement_kernel(const Chunk* chunks,
                                                           const uint32_t* chunk_n,
                                                           const uint32_t* set_vtx, uint32_t* cw,
                                                           const uint32_t* seeds, uint32_t i) {
    __shared__ uint32_t h_key[kAggSize], h_cnt[kAggSize];
    const uint32_t nchunks = *chunk_n;
    const uint32_t wpb = kDecBS / kWave;
    if (blockIdx.x * wpb >= nchunks) return;
    const uint32_t v = seeds[i];
    const uint32_t lane = threadIdx.x % kWave;
    const uint32_t wid = blockIdx.x * wpb + threadIdx.x / kWave;
    const uint32_t nw = gridDim.x * wpb;
    const bool agg = nchunks >= 4 * nw;
    if (agg) {
        for (uint32_t x = threadIdx.x; x < kAggSize; x += kDecBS) {
            h_key[x] = kEmpty;
            h_cnt[x] = 0;
        }
        __syncthreads();
    }
    for (uint32_t c = wid; c < nchunks; c += nw) {
        const Chunk ch = chunks[c];
        if (lane < ch.len) {
            const uint32_t u = set_vtx[ch.off + lane];
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

uint32_t argmax_grid(uint32_t n) {
    uint32_t g = (n / 4 + kArgBS * 4 - 1) / (kArgBS * 4);
    if (g < 1) g = 1;
    if (g > 512) g = 512;
    return g;
}

uint32_t select_grid(int device) {
    int cus = 256;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    return (uint32_t)cus * 4u;
}

hipError_t launch_argmax(const uint32_t* counts_work, uint32_t n, unsigned long long* slots,
                         uint32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(argmax_kernel, dim3(grid), dim3(kArgBS), 0, st, counts_work, n, slots);
    return hipGetLastError();
}

hipError_t launch_claim(const uint64_t* inv_off, uint32_t nseg, uint32_t n,
                        const uint32_t* inv_set, const uint64_t* set_off, uint32_t* covered,
                        uint32_t* counts_work, const unsigned long long* slots, uint32_t* seeds,
                        uint32_t* gains, uint32_t i, Chunk* chunks, uint32_t* chunk_n,
                        uint32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(claim_kernel, dim3(grid), dim3(kClaimBS), 0, st, inv_off, nseg, n, inv_set,
                       set_off, covered, counts_work, slots, seeds, gains, i, chunks, chunk_n);
    return hipGetLastError();
}

hipError_t launch_decrement(const Chunk* chunks, const uint32_t* chunk_n, const uint32_t* set_vtx,
                            uint32_t* counts_work, const uint32_t* seeds, uint32_t i,
                            uint32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(decrement_kernel, dim3(grid), dim3(kDecBS), 0, st, chunks, chunk_n, set_vtx,
                       counts_work, seeds, i);
    return hipGetLastError();
}

}  // namespace imm
