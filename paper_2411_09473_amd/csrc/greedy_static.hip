// greedy_static.hip -- imm_greedy_static: the greedy selection of imm_greedy
// (Find_Most_Influential_Set, Algorithm 2) with every scratch buffer carved
// out of one fixed device array, so that a call allocates nothing: for
// callers that cannot allocate device memory (code under hipGraph capture,
// serving loops, harnesses that forbid hipMalloc).
//
// The array lives in this library's code object, one copy per device, from
// module load until the process ends. Host code never uses its name as an
// address: on each device's first call the device address is looked up once
// (hipGetSymbolAddress) and kept, and kernels receive pointers into it.
// Every call on a device shares that device's array and leaves its contents
// behind; a call clears what must start at zero. Calls in one process are
// serialised per device by a lock held until the call's work has finished;
// calls issued from outside this entry point that touch the array would race.
#include <cstdio>
#include <cstring>
#include <mutex>

#include "engine.hpp"

// The whole scratch of one device (see imm.h for the size limits it implies).
static __device__ __align__(256) unsigned char scratch[IMM_STATIC_SCRATCH_BYTES];

namespace imm {

namespace {

constexpr int kMaxDevices = 64;

std::mutex g_mu[kMaxDevices];
unsigned char* g_ptr[kMaxDevices] = {};

// Byte offsets of the pieces inside the scratch, each aligned to 256 bytes.
struct StaticLayout {
    uint64_t sc, counts, work, heavy, cursor, inv_offs, scan, inv_set, covered, slots, chunks,
        seeds, gains, desc, set_off, set_vtx, total;
};

uint64_t take(uint64_t* at, uint64_t bytes) {
    const uint64_t o = *at;
    *at = (o + bytes + 255) & ~uint64_t(255);
    return o;
}

// host_pool: the pool arrives in host memory and is copied into the scratch.
StaticLayout layout_for(uint32_t n, uint64_t n_sets, uint64_t P, uint32_t k, bool host_pool) {
    StaticLayout L{};
    uint64_t at = 0;
    L.sc = take(&at, sizeof(DevScalars));
    L.counts = take(&at, (uint64_t)n * 4);
    L.work = take(&at, (uint64_t)n * 4 + 16);  // read by 16-byte loads
    L.heavy = take(&at, (uint64_t)n * 4 + 16);
    L.cursor = take(&at, (uint64_t)n * 4);
    L.inv_offs = take(&at, ((uint64_t)n + 1) * 8);
    L.scan = take(&at, scan_tmp_entries(n) * 8);
    L.inv_set = take(&at, (P + 1) * 4);
    L.covered = take(&at, (n_sets / 32 + 1) * 4);
    L.slots = take(&at, (uint64_t)k * (kArgSlots * 8 + 16));
    L.chunks = take(&at, (n_sets + P / 64 + 1) * sizeof(Chunk));
    L.seeds = take(&at, (uint64_t)k * 4);
    L.gains = take(&at, (uint64_t)k * 4);
    L.desc = take(&at, sizeof(SelectDesc));
    L.set_off = host_pool ? take(&at, (n_sets + 1) * 8) : 0;
    L.set_vtx = host_pool ? take(&at, (P + 1) * 4) : 0;
    L.total = at;
    return L;
}

#define HIP_STATIC(expr, what)                                                       \
    do {                                                                             \
        const hipError_t _e = (expr);                                                \
        if (_e != hipSuccess) {                                                      \
            (void)hipGetLastError();                                                 \
            return fail(_e == hipErrorOutOfMemory ? IMM_ENOMEM : IMM_EDEVICE, what); \
        }                                                                            \
    } while (0)

// The device address of this device's scratch, looked up on its first call.
imm_status scratch_of(int dev, unsigned char** out) {
    if (!g_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(IMM_EDEVICE, "greedy_static: hipGetSymbolAddress of the scratch failed");
        }
        g_ptr[dev] = static_cast<unsigned char*>(p);
    }
    *out = g_ptr[dev];
    return IMM_OK;
}

imm_status run(uint32_t n, const uint64_t* set_off, const uint32_t* set_vtx, uint64_t n_sets,
               uint32_t k, uint32_t flags, hipStream_t st, int dev, unsigned char* base,
               uint32_t* seeds, uint64_t* gains, uint64_t* covered) {
    const bool devp = (flags & IMM_DEVICE_PTRS) != 0;
    // the pool size and the first offset (host memory, or read from the device)
    uint64_t first = 0, P = 0;
    if (devp) {
        HIP_STATIC(hipMemcpyAsync(&first, set_off, 8, hipMemcpyDeviceToHost, st),
                   "greedy_static: reading set_off failed");
        HIP_STATIC(hipMemcpyAsync(&P, set_off + n_sets, 8, hipMemcpyDeviceToHost, st),
                   "greedy_static: reading set_off failed");
        HIP_STATIC(hipStreamSynchronize(st), "greedy_static: reading set_off failed");
    } else {
        first = set_off[0];
        P = set_off[n_sets];
    }
    if (first != 0) return fail(IMM_EINVAL, "greedy_static: set_off[0] must be 0");
    if (P && !set_vtx) return fail(IMM_EINVAL, "greedy_static: null set_vtx");
    if (P >= 0xFFFFFFFFull) return fail(IMM_EINVAL, "greedy_static: more than 2^32 - 2 entries");
    const StaticLayout L = layout_for(n, n_sets, P, k, !devp);
    if (L.total > IMM_STATIC_SCRATCH_BYTES) {
        char msg[256];
        std::snprintf(msg, sizeof(msg),
                      "greedy_static: n = %u, %llu sets, %llu entries, k = %u need %llu bytes "
                      "of scratch, more than the fixed %llu",
                      n, (unsigned long long)n_sets, (unsigned long long)P, k,
                      (unsigned long long)L.total,
                      (unsigned long long)IMM_STATIC_SCRATCH_BYTES);
        return fail(IMM_ENOMEM, msg);
    }
    auto at = [&](uint64_t o) { return base + o; };
    DevScalars* sc = reinterpret_cast<DevScalars*>(at(L.sc));
    uint32_t* counts = reinterpret_cast<uint32_t*>(at(L.counts));
    uint32_t* work = reinterpret_cast<uint32_t*>(at(L.work));
    uint32_t* heavy = reinterpret_cast<uint32_t*>(at(L.heavy));
    uint32_t* cursor = reinterpret_cast<uint32_t*>(at(L.cursor));
    uint64_t* inv_offs = reinterpret_cast<uint64_t*>(at(L.inv_offs));
    uint64_t* scan = reinterpret_cast<uint64_t*>(at(L.scan));
    uint32_t* inv_set = reinterpret_cast<uint32_t*>(at(L.inv_set));
    uint32_t* cov = reinterpret_cast<uint32_t*>(at(L.covered));
    unsigned long long* slots = reinterpret_cast<unsigned long long*>(at(L.slots));
    uint32_t* chunk_n = reinterpret_cast<uint32_t*>(slots + (uint64_t)k * kArgSlots);
    unsigned long long* cov_entries = reinterpret_cast<unsigned long long*>(chunk_n + 2ull * k);
    Chunk* chunks = reinterpret_cast<Chunk*>(at(L.chunks));
    uint32_t* seeds_d = reinterpret_cast<uint32_t*>(at(L.seeds));
    uint32_t* gains_d = reinterpret_cast<uint32_t*>(at(L.gains));
    SelectDesc* desc_d = reinterpret_cast<SelectDesc*>(at(L.desc));
    const uint64_t* so = set_off;
    const uint32_t* sv = set_vtx;
    if (!devp) {
        uint64_t* so_d = reinterpret_cast<uint64_t*>(at(L.set_off));
        uint32_t* sv_d = reinterpret_cast<uint32_t*>(at(L.set_vtx));
        HIP_STATIC(hipMemcpyAsync(so_d, set_off, (n_sets + 1) * 8, hipMemcpyHostToDevice, st),
                   "greedy_static: copying set_off failed");
        if (P)
            HIP_STATIC(hipMemcpyAsync(sv_d, set_vtx, P * 4, hipMemcpyHostToDevice, st),
                       "greedy_static: copying set_vtx failed");
        so = so_d;
        sv = sv_d;
    }
    // the previous call's contents are left in place: clear what starts at zero
    HIP_STATIC(hipMemsetAsync(sc, 0, sizeof(DevScalars), st), "greedy_static: clear failed");
    HIP_STATIC(launch_validate_pool(so, n_sets, sv, n, &sc->big_flag, st),
               "greedy_static: pool check launch failed");
    uint32_t bad = 0;
    HIP_STATIC(hipMemcpyAsync(&bad, &sc->big_flag, 4, hipMemcpyDeviceToHost, st),
               "greedy_static: pool check failed");
    HIP_STATIC(hipStreamSynchronize(st), "greedy_static: pool check failed");
    if (bad & 1u) return fail(IMM_EINVAL, "greedy_static: set_off decreases");
    if (bad) return fail(IMM_EINVAL, "greedy_static: vertex id out of range");
    // occurrence counts, then the vertex -> sets index as one segment
    HIP_STATIC(hipMemsetAsync(counts, 0, (uint64_t)n * 4, st), "greedy_static: clear failed");
    HIP_STATIC(launch_count_entries(sv, P, counts, st), "greedy_static: count launch failed");
    HIP_STATIC(launch_scan_u32(counts, nullptr, inv_offs, n, 0, nullptr, scan, st),
               "greedy_static: scan launch failed");
    HIP_STATIC(hipMemsetAsync(cursor, 0, (uint64_t)n * 4, st), "greedy_static: clear failed");
    if (n_sets)
        HIP_STATIC(launch_inv_scatter(so, sv, 0, (uint32_t)n_sets, inv_offs, cursor, inv_set,
                                      &sc->err, st),
                   "greedy_static: index launch failed");
    // selection state
    HIP_STATIC(hipMemsetAsync(heavy + n, 0, 4, st), "greedy_static: clear failed");
    HIP_STATIC(launch_select_init(counts, work, n, heavy, heavy + n, st),
               "greedy_static: select init launch failed");
    HIP_STATIC(hipMemsetAsync(cov, 0, (n_sets / 32 + 1) * 4, st), "greedy_static: clear failed");
    HIP_STATIC(hipMemsetAsync(slots, 0, (uint64_t)k * (kArgSlots * 8 + 16), st),
               "greedy_static: clear failed");
    SelectDesc d{work,   counts,   heavy,  heavy + n,   inv_offs, inv_set,     so, sv,
                 cov,    slots,    seeds_d, gains_d,    chunks,   chunk_n,
                 n_sets + P / 64 + 1,       cov_entries, n,        k,           1u,
                 (uint32_t)n_sets,          0u,          0u,       0u,          0u};
    d.arg_cnt = argmax_blocks(n);
    d.sel_cnt = select_blocks(dev, n_sets, 1);
    HIP_STATIC(hipMemcpyAsync(desc_d, &d, sizeof(d), hipMemcpyHostToDevice, st),
               "greedy_static: descriptor copy failed");
    for (uint32_t t = 0; t < k; ++t)
        HIP_STATIC(launch_select_step(desc_d, 1, t, d.arg_cnt, d.sel_cnt, 0, st),
                   "greedy_static: seed step launch failed");
    // results: gains land in the first half of the caller's uint64 array
    uint32_t err = 0;
    HIP_STATIC(hipMemcpyAsync(seeds, seeds_d, (uint64_t)k * 4, hipMemcpyDeviceToHost, st),
               "greedy_static: copying seeds failed");
    HIP_STATIC(hipMemcpyAsync(gains, gains_d, (uint64_t)k * 4, hipMemcpyDeviceToHost, st),
               "greedy_static: copying gains failed");
    HIP_STATIC(hipMemcpyAsync(&err, &sc->err, 4, hipMemcpyDeviceToHost, st),
               "greedy_static: copying the error flag failed");
    HIP_STATIC(hipStreamSynchronize(st), "greedy_static: selection failed");
    if (err) return fail(IMM_EDEVICE, "greedy_static: internal error: index overflow");
    // widen in place from the back: entry i reads 4-byte slot i, which no
    // wider entry written before it (those at i' > i cover slots >= 2i' > i)
    // has touched
    const uint32_t* g32 = reinterpret_cast<const uint32_t*>(gains);
    uint64_t c = 0;
    for (uint32_t i = k; i-- > 0;) {
        const uint32_t v = g32[i];
        gains[i] = v;
        c += v;
    }
    if (covered) *covered = c;
    return IMM_OK;
}

}  // namespace

}  // namespace imm

using namespace imm;

extern "C" imm_status imm_greedy_static(uint32_t n, const uint64_t* set_off,
                                        const uint32_t* set_vtx, uint64_t n_sets, uint32_t k,
                                        uint32_t flags, void* stream, uint32_t* seeds,
                                        uint64_t* gains, uint64_t* covered) {
    if (n < 1 || n > 0xFFFFFFFEu || k == 0 || k > n)
        return fail(IMM_EINVAL, "greedy_static: need 1 <= k <= n");
    if (n_sets >= 0xFFFFFFFFull) return fail(IMM_EINVAL, "greedy_static: n_sets must be < 2^32");
    if (!set_off || !seeds || !gains) return fail(IMM_EINVAL, "greedy_static: null argument");
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) {
        (void)hipGetLastError();
        return fail(IMM_EDEVICE, "greedy_static: no usable current device");
    }
    std::lock_guard<std::mutex> lk(g_mu[dev]);
    unsigned char* base = nullptr;
    IMM_TRY(scratch_of(dev, &base));
    const imm_status s = run(n, set_off, set_vtx, n_sets, k, flags, (hipStream_t)stream, dev, base,
                             seeds, gains, covered);
    // nothing of a failed call may still be running when the lock is released
    if (s != IMM_OK) (void)hipStreamSynchronize((hipStream_t)stream);
    return s;
}
