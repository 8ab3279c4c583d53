// probe_chase.hip -- a measurement probe, not part of the IMM path: the
// memory pattern of the LT walk kernel without its arithmetic. Chains of
// dependent reads of random 64-byte rows, each chain run by a group of four
// lanes (16 bytes each), as a walk reads its guide window; the next row is a
// hash of the words just loaded, so every read waits for the one before.
// Optionally each step also adds one to a random counter (a walk's count
// atomic). bench.py --chase-probe times it on tables the size of the
// LiveJournal-shaped window table and of the Infinity Cache, at several
// numbers of chains in flight (set by the workgroups' LDS share).
#include <hip/hip_runtime.h>

#include <cstdint>

namespace {

constexpr uint32_t kWave = 64;

__device__ __forceinline__ uint32_t mix32(uint32_t x) {
    x ^= x >> 16;
    x *= 0x7FEB352Du;
    x ^= x >> 15;
    x *= 0x846CA68Bu;
    x ^= x >> 16;
    return x;
}

__global__ __launch_bounds__(256) void fill_kernel(uint4* t, uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) {
        const uint32_t a = (uint32_t)i, b = (uint32_t)(i >> 32);
        t[i] = make_uint4(mix32(a ^ 0x9E3779B9u), mix32(a + b * 0x85EBCA6Bu), mix32(~a),
                          mix32(a * 0xC2B2AE35u + 1u));
    }
}

// Four waves per workgroup (one per SIMD); dynamic LDS (unused) limits the
// workgroups per CU, hence the waves per SIMD.
template <bool kCount>
__global__ __launch_bounds__(256) void chase_kernel(const uint4* t, uint64_t rows, uint32_t steps,
                                                   uint32_t* counts, uint32_t ncounts,
                                                   unsigned long long* sink) {
    extern __shared__ uint32_t pad[];
    const uint32_t lane = threadIdx.x % kWave, sub = lane & 3u;
    const uint32_t chain = blockIdx.x * 64u + threadIdx.x / 4;
    uint32_t h = mix32(chain * 0x9E3779B1u + 12345u);
    uint64_t r = ((uint64_t)h * rows) >> 32;
    uint32_t acc = 0;
    for (uint32_t s = 0; s < steps; ++s) {
        const uint4 v = t[r * 4 + sub];
        uint32_t x = v.x ^ v.y ^ v.z ^ v.w;
        x ^= __shfl_xor(x, 1, kWave);
        x ^= __shfl_xor(x, 2, kWave);
        h = mix32(x ^ (s * 0x27D4EB2Du) ^ chain);
        r = ((uint64_t)h * rows) >> 32;
        if (kCount && sub == 0) atomicAdd(&counts[((uint64_t)h * ncounts) >> 32], 1u);
        acc += x;
    }
    if (sub == 0 && acc == 0x12345678u) atomicAdd(sink, 1ull);  // keeps the loads live
    if (threadIdx.x == 0 && blockIdx.x == 0) pad[0] = acc;
}

}  // namespace

// Chains of dependent random 64-byte row reads: a table of `rows` rows,
// `wg_per_cu` four-wave workgroups (64 chains each; one wave per SIMD) per
// compute unit held resident by `lds_bytes` of LDS each, `steps` reads per
// chain, and with
// count != 0 one atomic add per step into a table of `ncounts` counters.
// Writes the kernel time (HIP events) and the number of chain steps.
// Returns 0, or a HIP error code.
extern "C" int imm_probe_chase(uint64_t rows, uint32_t wg_per_cu, uint32_t lds_bytes,
                               uint32_t steps, int count, uint32_t ncounts, double* ms,
                               uint64_t* total_steps) {
    int dev = 0, cus = 256;
    if (rows == 0 || steps == 0 || wg_per_cu == 0 || (count && ncounts == 0)) return 1;
    if (lds_bytes < 16) lds_bytes = 16;  // the kernel writes its first word
    if (hipGetDevice(&dev) != hipSuccess) return 1;
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    uint4* t = nullptr;
    uint32_t* c = nullptr;
    unsigned long long* sink = nullptr;
    hipEvent_t a = nullptr, b = nullptr;
    hipError_t e = hipMalloc((void**)&t, rows * 64);
    if (e == hipSuccess) e = hipMalloc((void**)&c, (uint64_t)(ncounts ? ncounts : 1) * 4);
    if (e == hipSuccess) e = hipMalloc((void**)&sink, 8);
    if (e == hipSuccess) e = hipMemset(c, 0, (uint64_t)(ncounts ? ncounts : 1) * 4);
    if (e == hipSuccess) {
        hipLaunchKernelGGL(fill_kernel, dim3(4096), dim3(256), 0, 0, t, rows * 4);
        e = hipGetLastError();
    }
    const uint32_t grid = (uint32_t)cus * wg_per_cu;
    if (e == hipSuccess) e = hipEventCreate(&a);
    if (e == hipSuccess) e = hipEventCreate(&b);
    if (e == hipSuccess) {
        // one untimed pass (first launch), then the timed one
        for (int pass = 0; pass < 2 && e == hipSuccess; ++pass) {
            if (pass == 1) (void)hipEventRecord(a, 0);
            if (count)
                hipLaunchKernelGGL(chase_kernel<true>, dim3(grid), dim3(256), lds_bytes, 0, t,
                                   rows, pass ? steps : 64u, c, ncounts, sink);
            else
                hipLaunchKernelGGL(chase_kernel<false>, dim3(grid), dim3(256), lds_bytes, 0, t,
                                   rows, pass ? steps : 64u, c, ncounts, sink);
            e = hipGetLastError();
        }
        if (e == hipSuccess) e = hipEventRecord(b, 0);
        if (e == hipSuccess) e = hipEventSynchronize(b);
        float f = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&f, a, b);
        *ms = f;
        *total_steps = (uint64_t)grid * 64u * steps;
    }
    if (a) (void)hipEventDestroy(a);
    if (b) (void)hipEventDestroy(b);
    if (t) (void)hipFree(t);
    if (c) (void)hipFree(c);
    if (sink) (void)hipFree(sink);
    return e == hipSuccess ? 0 : (int)e;
}
