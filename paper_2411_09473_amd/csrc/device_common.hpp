// device_common.hpp -- device helpers shared by the libimm kernels (gfx950):
// the Philox4x32-10 stream that defines every random decision, and wave64
// scan/reduction primitives.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imm {

constexpr uint32_t kWave = 64;
constexpr uint32_t kEmpty = 0xFFFFFFFFu;
constexpr uint32_t kSelected = 0xFFFFFFFFu;  // counts_work value of a chosen seed

// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, each two
// 32x32->64 products by the published multipliers, an xor with the other two
// counter words and the round key, a word permutation, and a Weyl key bump.
// The key is wave-uniform (the run seed) so the key schedule stays scalar.
struct Philox4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ Philox4 philox10(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3,
                                            uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
        const uint32_t n0 = (uint32_t)(p1 >> 32) ^ c1 ^ k0;
        const uint32_t n2 = (uint32_t)(p0 >> 32) ^ c3 ^ k1;
        c1 = (uint32_t)p1;
        c3 = (uint32_t)p0;
        c0 = n0;
        c2 = n2;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return Philox4{c0, c1, c2, c3};
}

__device__ __forceinline__ uint32_t pick(const Philox4& r, uint32_t j) {
    return j == 0 ? r.x : (j == 1 ? r.y : (j == 2 ? r.z : r.w));
}

// Root of sample s: floor(w * n / 2^64), w = word0 | word1 << 32.
__device__ __forceinline__ uint32_t sample_root(uint64_t seed, uint64_t s, uint32_t n) {
    const Philox4 r = philox10(0u, (uint32_t)s, (uint32_t)(s >> 32), 0u, (uint32_t)seed,
                               (uint32_t)(seed >> 32));
    const uint64_t w = (uint64_t)r.x | ((uint64_t)r.y << 32);
    return (uint32_t)__umul64hi(w, (uint64_t)n);
}

// LT draw at vertex v in sample s: word v&3 of counter (v>>2, s_lo, s_hi, 2).
__device__ __forceinline__ uint32_t lt_draw(uint64_t seed, uint64_t s, uint32_t v) {
    const Philox4 r = philox10(v >> 2, (uint32_t)s, (uint32_t)(s >> 32), 2u, (uint32_t)seed,
                               (uint32_t)(seed >> 32));
    return pick(r, v & 3u);
}

__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Inclusive wave64 prefix sum of a uint32, with DPP lane moves (no LDS
// round trips): shifts by 1, 2, 4 and 8 lanes inside each row of 16 (zeros
// shifted in), then lane 15 of rows 0 and 2 is added to rows 1 and 3, and
// lane 31 to rows 2 and 3.
__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x111, 0xF, 0xF, true);  // row_shr:1
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x112, 0xF, 0xF, true);  // row_shr:2
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x114, 0xF, 0xF, true);  // row_shr:4
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x118, 0xF, 0xF, true);  // row_shr:8
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x142, 0xA, 0xF, false); // row_bcast:15
    v += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, 0x143, 0xC, 0xF, false); // row_bcast:31
    return v;
}

__device__ __forceinline__ uint64_t wave_incl_scan64(uint64_t v) {
    const uint32_t lane = lane_id();
#pragma unroll
    for (uint32_t d = 1; d < kWave; d <<= 1) {
        const uint64_t t = __shfl_up(v, d, kWave);
        if (lane >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_max64(uint64_t v) {
#pragma unroll
    for (uint32_t d = kWave / 2; d >= 1; d >>= 1) {
        const uint64_t t = __shfl_xor(v, d, kWave);
        v = t > v ? t : v;
    }
    return v;
}

__device__ __forceinline__ uint64_t wave_sum64(uint64_t v) {
#pragma unroll
    for (uint32_t d = kWave / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, kWave);
    return v;
}

// Largest index o in [0, cnt) with base[o] <= t (base non-decreasing, base[0] = 0).
template <class T>
__device__ __forceinline__ uint32_t owner_of(const T* base, uint32_t cnt, T t) {
    uint32_t lo = 0, hi = cnt;  // invariant: base[lo] <= t, answer in [lo, hi)
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (base[mid] <= t) lo = mid; else hi = mid;
    }
    return lo;
}

// Like owner_of, for a thread whose t only grows: search forward from its
// previous answer `ow` (base[ow] <= t must hold), galloping then bisecting.
template <class T>
__device__ __forceinline__ uint32_t owner_from(const T* base, uint32_t cnt, T t, uint32_t ow) {
    uint32_t step = 1;
    while (ow + step < cnt && base[ow + step] <= t) {
        ow += step;
        step <<= 1;
    }
    uint32_t hi = ow + step < cnt ? ow + step : cnt;
    while (hi - ow > 1) {
        const uint32_t mid = (ow + hi) >> 1;
        if (base[mid] <= t) ow = mid; else hi = mid;
    }
    return ow;
}

// Enumerate the (segment, k) pairs of the 64 segments held one per lane;
// f(owner_lane, a_owner, b_owner, k) runs once for every k < size_owner.
// Requires blockDim.x == 64 (one wave per block).
template <class F>
__device__ __forceinline__ void wave_segments(uint32_t sz, uint64_t a, uint64_t b, F f) {
    __shared__ uint64_t s_base[kWave];
    __shared__ uint64_t s_a[kWave], s_b[kWave];
    const uint32_t lane = threadIdx.x;
    const uint64_t incl = wave_incl_scan64(sz);
    const uint64_t T = __shfl(incl, kWave - 1, kWave);
    s_base[lane] = incl - sz;
    s_a[lane] = a;
    s_b[lane] = b;
    __syncthreads();
    uint32_t ow = 0;
    for (uint64_t t = lane; t < T; t += kWave) {
        ow = owner_from(s_base, kWave, t, ow);
        f(ow, s_a[ow], s_b[ow], (uint32_t)(t - s_base[ow]));
    }
    __syncthreads();
}

// Column sums of a group of vertex bitmaps ("vertical popcount"), by one
// workgroup of kColBS threads: the 64 words (2048 vertices) from word w0 on,
// over the bitmaps src(i) names for i in [0, cnt), cnt <= kColChunk (src
// returns kEmpty to skip one; it is called alike by a whole wave). Wave s
// takes i = s, s + 4, ...: each lane adds its word of each bitmap into 11
// bit-planes (a ripple-carry add of 32 one-bit counts at once, 33 operations
// instead of 96 for 32 separate counts), and the four waves' counts are
// summed in LDS (lds: 4 * 2048 words). Thread x gets the sums of the
// vertices 32 w0 + 8x .. 32 w0 + 8x + 7 in out.
constexpr uint32_t kColBS = 256;
constexpr uint32_t kColChunk = 4096;  // at most 1024 bitmaps per wave: 11 planes
constexpr uint32_t kColPlanes = 11;
template <class Src>
__device__ __forceinline__ void col_sums(const uint32_t* bits, uint32_t words, uint32_t w0,
                                         uint32_t cnt, Src src, uint32_t* lds, uint32_t out[8]) {
    const uint32_t lane = threadIdx.x % kWave, s = threadIdx.x / kWave;
    const uint32_t w = w0 + lane;
    const bool in = w < words;
    uint32_t pl[kColPlanes];
#pragma unroll
    for (uint32_t p = 0; p < kColPlanes; ++p) pl[p] = 0u;
    // four bitmaps' words in flight per lane
    for (uint32_t i = s; i < cnt; i += 4 * 4) {
        uint32_t x[4];
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            const uint32_t ii = i + 4 * u;
            const uint32_t b = ii < cnt ? src(ii) : kEmpty;
            x[u] = (b != kEmpty && in) ? bits[(size_t)b * words + w] : 0u;
        }
#pragma unroll
        for (uint32_t u = 0; u < 4; ++u) {
            uint32_t c = x[u];
#pragma unroll
            for (uint32_t p = 0; p < kColPlanes; ++p) {
                const uint32_t t = pl[p] & c;
                pl[p] ^= c;
                c = t;
            }
        }
    }
    // bit j of this lane's word: vertex 32 lane + j, at lds[s * 2048 + 64 j + lane]
#pragma unroll
    for (uint32_t j = 0; j < 32; ++j) {
        uint32_t c = 0;
#pragma unroll
        for (uint32_t p = 0; p < kColPlanes; ++p) c |= ((pl[p] >> j) & 1u) << p;
        lds[s * 2048u + 64u * j + lane] = c;
    }
    __syncthreads();
#pragma unroll
    for (uint32_t q = 0; q < 8; ++q) {
        const uint32_t v = 8u * threadIdx.x + q;
        const uint32_t a = 64u * (v & 31u) + (v >> 5);
        out[q] = lds[a] + lds[2048u + a] + lds[4096u + a] + lds[6144u + a];
    }
}

}  // namespace imm
