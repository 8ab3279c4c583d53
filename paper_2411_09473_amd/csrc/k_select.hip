// k_select.hip -- greedy max-coverage seed selection (Find_Most_Influential_Set,
// Algorithm 2) over the device-resident pool.
//
// One seed costs two launches and no host round trip:
//  * argmax: the two-step reduction of the paper's PARALLEL_REDUCTION
//    (regional maxima per workgroup, then the global maximum by the last
//    workgroup to finish). Each vertex is a packed key count<<32 | ~id, so a
//    plain 64-bit max picks the largest count and, among equal counts, the
//    lowest id. A chosen vertex's count is replaced by a sentinel that maps
//    to key 0, which keeps it out of later picks.
//  * cover: the chosen vertex's inverted-index list names exactly the sets
//    that contain it; each uncovered one is claimed with an atomic bit and
//    the counts of its other members are decremented atomically.
#include "device_common.hpp"
#include "imm_internal.hpp"

namespace imm {

namespace {

constexpr uint32_t kArgBS = 256;

__device__ __forceinline__ uint64_t vkey(uint32_t c, uint32_t v) {
    return c == kSelected ? 0ull : (((uint64_t)c << 32) | (uint64_t)(~v));
}

__global__ __launch_bounds__(kArgBS) void argmax_kernel(uint32_t* cw, uint32_t n,
                                                        unsigned long long* partials,
                                                        uint32_t* ticket, uint32_t* seeds,
                                                        uint32_t* gains, uint32_t i) {
    __shared__ uint64_t s_w[kArgBS / kWave];
    __shared__ uint32_t s_last;
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
        partials[blockIdx.x] = b;
        __threadfence();
        s_last = atomicAdd(ticket, 1u) == gridDim.x - 1 ? 1u : 0u;
    }
    __syncthreads();
    if (!s_last) return;
    uint64_t b = 0;
    for (uint32_t x = tid; x < gridDim.x; x += kArgBS) {
        const uint64_t p = __hip_atomic_load(&partials[x], __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        b = p > b ? p : b;
    }
    b = wave_max64(b);
    if (lane == 0) s_w[w] = b;
    __syncthreads();
    if (tid == 0) {
        uint64_t m = s_w[0];
        for (uint32_t x = 1; x < kArgBS / kWave; ++x) m = s_w[x] > m ? s_w[x] : m;
        const uint32_t v = ~(uint32_t)m;
        seeds[i] = v;
        gains[i] = (uint32_t)(m >> 32);
        cw[v] = kSelected;
        *ticket = 0;
    }
}

__global__ __launch_bounds__(64) void cover_kernel(const uint64_t* inv_off, const uint32_t* inv_set,
                                                   const uint64_t* set_off,
                                                   const uint32_t* set_vtx, uint32_t* covered,
                                                   uint32_t* cw, const uint32_t* seeds,
                                                   uint32_t i) {
    const uint32_t v = seeds[i];
    const uint64_t lb = inv_off[v], len = inv_off[v + 1] - lb;
    const uint64_t step = (uint64_t)gridDim.x * kWave;
    for (uint64_t base = (uint64_t)blockIdx.x * kWave; base < len; base += step) {
        const uint64_t t = base + threadIdx.x;
        uint32_t sz = 0;
        uint64_t a = 0;
        if (t < len) {
            const uint32_t j = inv_set[lb + t];
            const uint32_t bit = 1u << (j & 31);
            const uint32_t old = atomicOr(&covered[j >> 5], bit);
            if (!(old & bit)) {
                a = set_off[j];
                sz = (uint32_t)(set_off[j + 1] - a);
            }
        }
        wave_segments(sz, a, 0, [&](uint32_t, uint64_t a0, uint64_t, uint32_t k) {
            const uint32_t u = set_vtx[a0 + k];
            if (u != v) atomicSub(&cw[u], 1u);
        });
    }
}

}  // namespace

uint32_t argmax_grid(uint32_t n) {
    uint32_t g = (n / 4 + kArgBS * 4 - 1) / (kArgBS * 4);
    if (g < 1) g = 1;
    if (g > 1024) g = 1024;
    return g;
}

uint32_t cover_grid(int device) {
    int cus = 256;
    hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    return (uint32_t)cus * 8u;
}

hipError_t launch_argmax(uint32_t* counts_work, uint32_t n, unsigned long long* partials,
                         uint32_t* ticket, uint32_t* seeds, uint32_t* gains, uint32_t i,
                         uint32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(argmax_kernel, dim3(grid), dim3(kArgBS), 0, st, counts_work, n, partials,
                       ticket, seeds, gains, i);
    return hipGetLastError();
}

hipError_t launch_cover(const uint64_t* inv_off, const uint32_t* inv_set, const uint64_t* set_off,
                        const uint32_t* set_vtx, uint32_t* covered, uint32_t* counts_work,
                        const uint32_t* seeds, uint32_t i, uint32_t grid, hipStream_t st) {
    hipLaunchKernelGGL(cover_kernel, dim3(grid), dim3(kWave), 0, st, inv_off, inv_set, set_off,
                       set_vtx, covered, counts_work, seeds, i);
    return hipGetLastError();
}

}  // namespace imm
