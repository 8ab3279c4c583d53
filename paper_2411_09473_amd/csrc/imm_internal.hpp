// imm_internal.hpp -- host-side declarations shared by the libimm translation
// units: device views of a resident graph, sampling outputs, and the kernel
// launchers each .hip file provides.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace imm {

// Resident IC graph: CSC offsets, live thresholds padded to a multiple of 4
// (+4) entries so a 16-byte load of edge group e>>2 stays in bounds, sources.
struct IcGraphDev {
    const uint32_t* off;  // n+1
    const uint32_t* thr;  // round_up(m,4)+4
    const uint32_t* src;  // m
    uint32_t n;
    uint32_t m;
};

// Resident LT graph: offsets, one 16-byte record per in-edge (cum, src and
// the bounds of src's own column, so a walk that follows the edge needs no
// further offset load), and the guide table: for column v of in-degree d,
// guide[off[v]+j] is the first edge e of the column with cum[e] > ceil(j
// 2^32 / d) - 1, i.e. the answer for the smallest draw in bucket j =
// floor(r d / 2^32). gw holds per bucket a copy of the kLtWindow records
// from its guide entry on (64 bytes; entries past the column are records
// with src = 0xFFFFFFFF and cum = 0), so a walk step almost always finds its
// edge with one window read.
constexpr uint32_t kLtWindow = 4;
struct LtGraphDev {
    const uint32_t* off;   // n+1
    const uint4* cs;       // m (x = cum, y = src, z = off[src], w = off[src+1])
    const uint32_t* guide; // m
    const uint4* gw;       // kLtWindow * m
    uint32_t n;
    uint32_t m;
};

// Work granules of the sampling kernels: sample ids claimed per ticket by a
// wave of the IC kernel, staging entries it reserves at a time, and staging
// entries an LT lane reserves at a time (also the longest walk it keeps).
constexpr uint32_t kIcTicketChunk = 64;
constexpr uint32_t kIcStageChunk = 4096;
constexpr uint32_t kLtChunk = 1024;

// Samples of run seed `seed`: sample id = id_lo + index, for the indices
// [0, count), or, when `list` is given, for list[0 .. *list_n) (a retry pass).
struct SampleRange {
    uint64_t seed;
    uint64_t id_lo;
    uint32_t count;
    const uint32_t* list;
    const uint32_t* list_n;
};

// Stats slots (uint64 counters in device memory).
// Main: the wave/team-per-sample kernels; Big: the large-set kernels; Lane:
// the IC lane-per-root kernel (its sets are single vertices).
enum StatSlot : int {
    kStMainSets = 0, kStMainEntries, kStMainEdges, kStMainLive,
    kStBigSets, kStBigEntries, kStBigEdges, kStBigLive,
    kStLaneSets, kStLaneEdges, kStCount
};

// Where sampled sets go: a staging buffer with a bump cursor, per-sample
// (stage offset, size), the accumulated occurrence counts, and the lists of
// sample indices that must be redone by the large-set kernel (defer: the set
// outgrew the on-chip structures; retry: the staging buffer was full).
struct SampleOut {
    uint32_t* stage;
    uint64_t stage_cap;
    unsigned long long* cursor;
    // [count] each: a finished set's staging offset and size; for an LT walk
    // handed to the long-walk kernel, its chunk's offset and the next vertex
    uint64_t* stage_off;
    uint32_t* sizes;
    uint32_t* counts;      // [n]
    uint32_t* defer;       // [count]
    uint32_t* defer_n;
    uint32_t* retry;       // [count]
    uint32_t* retry_n;
    unsigned long long* stats;  // [kStCount]
    // IC sets of at least dense_min members are stored as vertex bitmaps
    // (dense_words words each) instead of member lists: bitmap slot b =
    // atomicAdd(dense_cursor) (< dense_cap, else the set is listed for a
    // retry), dense_sid[b] = pool_base + sample index, dense_size[b] = its
    // size, *dense_entries += its size; its list is empty and its members'
    // counts are left to a bitmap count after the pass. dense_min =
    // 0xFFFFFFFF stores every set as a list.
    uint32_t* dense_bits;
    uint64_t dense_cap;
    uint32_t* dense_cursor;
    uint32_t* dense_sid;
    uint32_t* dense_size;
    unsigned long long* dense_entries;
    uint32_t dense_min;
    uint32_t dense_words;
    uint64_t pool_base;
    // LT: only samples with index < count_lim add to counts (the others are
    // drawn ahead of the round that needs them; 0xFFFFFFFF: all count);
    // those with count_lim <= index < count_lim2, the ids the next round
    // would take, add to counts_next instead
    uint32_t count_lim;
    uint32_t count_lim2;
    uint32_t* counts_next;
};
// Sets of at least max(ceil(n / 32), kDenseMinSize) members are dense: a
// bitmap of n bits then takes no more room than the member list. Every set
// that large comes from the large-set kernel (the team kernel's sets hold at
// most 1024 members), which has the set's bitmap at hand.
constexpr uint32_t kDenseMinSize = 2048;
inline uint32_t dense_threshold(uint32_t n) {
    const uint32_t t = (uint32_t)(((uint64_t)n + 31) / 32);
    return t > kDenseMinSize ? t : kDenseMinSize;
}

// Scratch of the large-set kernels: per slot a visited bitmap of `words`
// uint32 (all zero between samples) and a queue of qcap (<= n) uint32.
struct BigScratch {
    uint32_t* bitmaps;
    uint32_t* queues;
    uint32_t words;
    uint32_t slots;
    uint32_t qcap;
};

// One instance of a multi-instance IC sampling pass: its graph, its range
// of sample ids (no list), its outputs (SampleOut: staging, counts, deferred
// and retry lists), its pending list, and the logical queue capacity of its
// giant sets (min(n, the shared slots' queue length)). A launch over several
// tasks numbers their work items one after another; a workgroup that moves
// to another task's items flushes its statistics and staging chunk first.
struct IcTask {
    IcGraphDev g;
    SampleRange rg;
    SampleOut o;
    uint32_t* pend;
    uint32_t* pend_n;
    uint32_t qcap;
    uint32_t pad;
};
// Tasks of one multi-instance launch at most.
constexpr uint32_t kMaxTasks = 64;

// ---- sampling (k_sample_ic.hip, k_sample_lt.hip)
// IC, first pass: lane-per-root tries over the range (or list); samples that
// are not a single vertex are appended to pend (*pend_n entries).
hipError_t launch_ic_lane(const IcGraphDev& g, const SampleRange& r, const SampleOut& o,
                          uint32_t* pend, uint32_t* pend_n, uint32_t* ticket, uint32_t grid,
                          hipStream_t st);
// IC, second pass: BFS of the pending samples, one team of `team` (1, 2 or
// 4) waves per sample; r.count bounds *pend_n.
hipError_t launch_ic_bfs(const IcGraphDev& g, const SampleRange& r, const SampleOut& o,
                         const uint32_t* pend, const uint32_t* pend_n, uint32_t* ticket,
                         uint32_t team, uint32_t grid, hipStream_t st);
uint32_t ic_bfs_grid(int device, uint32_t team);
// IC, giant sets: one workgroup of `block` (256 or 1024) threads per listed
// sample, b.slots workgroups (each owns one scratch slot). A set with more
// than b.qcap members is abandoned and its index appended to over (which may
// be null only when b.qcap = n).
hipError_t launch_ic_large(const IcGraphDev& g, const SampleRange& r, const SampleOut& o,
                           const uint32_t* list, const uint32_t* list_n, uint32_t* fail,
                           uint32_t* fail_n, uint32_t* over, uint32_t* over_n,
                           uint32_t* ticket, const BigScratch& b, uint32_t block,
                           hipStream_t st);
uint32_t ic_large_slots(int device, uint32_t block);
// The same three passes over ntask (<= kMaxTasks) tasks at once: the lane
// pass over their id ranges (task q's positions are [prefix[q], prefix[q+1]),
// each range rounded up to whole tickets of kLaneTicket ids), the BFS pass
// over their pending lists, the giant-set pass over their deferred lists
// with shared scratch slots b (words and queues sized for the largest task).
// A giant set whose queue overflows is listed in its task's retry list (to be
// redone alone). Every list length is read on the device.
constexpr uint32_t kLaneTicket = 256;
hipError_t launch_ic_multi(const IcTask* tasks, uint32_t ntask, const uint32_t* prefix,
                           uint32_t* tickets /* 3, zeroed */, uint32_t team, uint32_t block,
                           const BigScratch& b, int device, hipStream_t st);
// LT: one walk per group of `lanes` (1, 2 or 4) lanes; bloom_bits (10, 11 or
// 12) sizes the per-walk path filter in LDS.
hipError_t launch_lt_small(const LtGraphDev& g, const SampleRange& r, const SampleOut& o,
                           uint32_t* ticket, uint32_t bloom_bits, uint32_t lanes, uint32_t grid,
                           hipStream_t st);
hipError_t launch_lt_large(const LtGraphDev& g, const SampleRange& r, const SampleOut& o,
                           const uint32_t* list, const uint32_t* list_n, uint32_t* fail,
                           uint32_t* fail_n, uint32_t* ticket, const BigScratch& b,
                           hipStream_t st);
hipError_t launch_lt_guide(const uint32_t* off, const uint4* cs, uint32_t* guide, uint4* gw,
                           uint32_t n,
                           hipStream_t st);
uint32_t ic_small_grid(int device);
uint32_t lt_small_grid(int device, uint32_t bloom_bits, uint32_t lanes);

// ---- pool, index, canonical order (k_pool.hip)
// out[0] = B; out[i+1] = B + x[0] + ... + x[i] for N >= 1 entries, where
// x[i] = in[i] - (sub ? sub[i] : 0) and B = base_dev ? *base_dev : base.
hipError_t launch_scan_u32(const uint32_t* in, const uint32_t* sub, uint64_t* out, uint64_t N,
                           uint64_t base, const uint64_t* base_dev, uint64_t* tile_tmp,
                           hipStream_t st);
uint64_t scan_tmp_entries(uint64_t N);
// Copy staged sets [lo, lo+count) to set_vtx at set_off[lo..lo+count].
hipError_t launch_compact(const uint32_t* stage, const uint64_t* stage_off,
                          const uint64_t* set_off, uint64_t lo, uint32_t count,
                          uint32_t* set_vtx, hipStream_t st);
// For the sets j in [lo, lo+count): inv_set[inv_off[v] + rank] = j for each
// member v of set j (rank by atomic cursor); *err |= 1 if a vertex has more
// members than inv_off allows.
hipError_t launch_inv_scatter(const uint64_t* set_off, const uint32_t* set_vtx, uint64_t lo,
                              uint32_t count, const uint64_t* inv_off, uint32_t* cursor,
                              uint32_t* inv_set, uint32_t* err, hipStream_t st);
// The same index segment built by radix partition (no atomic per entry):
// buckets of 2^shift consecutive vertices, at most kBktMax of them and at
// most kBktVtxMax vertices each (so n <= kBktMax * kBktVtxMax); tmp holds
// cap (set, vertex) pairs, at least the segment's entries (else *err |= 1
// and nothing is indexed); tile_groups: sets per partition tile, in units of
// 256. cursor: n zeros. pl: one IndexPlan of device memory.
constexpr uint32_t kBktMax = 2048;
constexpr uint32_t kBktVtxMax = 4096;
constexpr uint32_t kSlice = 16384;
struct IndexPlan {
    uint64_t off[kBktMax + 1];          // bucket ranges in the segment
    unsigned long long cur[kBktMax];    // partition cursors
    uint32_t sl_pre[kBktMax + 1];       // first slice of each bucket
    uint32_t tot[kBktMax];              // the counting build's bucket totals
};
uint32_t index_bucket_shift(uint32_t n);  // 32 when n is too large for the partition
hipError_t launch_inv_partitioned(const uint64_t* set_off, const uint32_t* set_vtx, uint64_t lo,
                                  uint32_t count, uint32_t tile_groups, uint32_t n,
                                  uint32_t shift, const uint64_t* inv_off, IndexPlan* pl,
                                  unsigned long long* tmp, uint64_t cap, uint32_t* cursor,
                                  uint32_t* inv_set, uint32_t* err, int device, hipStream_t st);
// The same segment built from the sets alone, when the counts of some of
// them are not known yet: the entries per bucket are counted first (one
// pass, LDS histograms), the partition follows, and each bucket's workgroup
// counts its vertices' entries, scans them into the segment's list offsets
// inv_off (n + 1 of them, based at set_off[lo]), places the lists, and sets
// counts[v] = base[v] + v's entries in the segment for every vertex. One
// workgroup per bucket: meant for segments whose buckets hold a modest
// number of entries each.
hipError_t launch_inv_counting(const uint64_t* set_off, const uint32_t* set_vtx, uint64_t lo,
                               uint32_t count, uint32_t tile_groups, uint32_t n, uint32_t shift,
                               uint64_t* inv_off, const uint32_t* base, uint32_t* counts,
                               IndexPlan* pl, unsigned long long* tmp, uint64_t cap,
                               uint32_t* inv_set, uint32_t* err, int device, hipStream_t st);
// counts[v] += occurrences of v in set_vtx[0..P).
hipError_t launch_count_entries(const uint32_t* set_vtx, uint64_t P, uint32_t* counts,
                                hipStream_t st);
// dst[v] += src[v] for v < n.
hipError_t launch_add_counts(const uint32_t* src, uint32_t* dst, uint32_t n, hipStream_t st);
// counts[v] += occurrences of v in the sets [lo, hi) of a pool (their entry
// range read from set_off on the device).
hipError_t launch_count_sets(const uint64_t* set_off, uint64_t lo, uint64_t hi,
                             const uint32_t* set_vtx, uint32_t* counts, hipStream_t st);
// counts[u] += number of bitmaps b in [b_lo, b_hi) with bit u set (each
// bitmap `words` words long, counts over n = 32 * words vertices at most).
hipError_t launch_dense_count(const uint32_t* bits, uint32_t words, uint32_t b_lo, uint32_t b_hi,
                              uint32_t n, uint32_t* counts, hipStream_t st);
// *count += number of sets of the pool holding one of seeds[0..k); mark
// (one bit per vertex) and hit (one bit per set) must be zero before.
hipError_t launch_cover_count(const uint64_t* set_off, const uint32_t* set_vtx, uint64_t n_sets,
                              const uint32_t* seeds, uint32_t k, uint32_t* mark, uint32_t* hit,
                              unsigned long long* count, hipStream_t st);
// Check a caller pool: offsets non-decreasing, ids < n. flag[0] set on error.
hipError_t launch_validate_pool(const uint64_t* set_off, uint64_t n_sets, const uint32_t* set_vtx,
                                uint32_t n, uint32_t* flag, hipStream_t st);
// Sort every set ascending in place; big_list/big_n get the sets too large
// for the on-chip sort, which launch_sort_big then sorts one at a time.
hipError_t launch_sort_small(const uint64_t* set_off, uint32_t n_sets, uint32_t* set_vtx,
                             uint32_t* big_list, uint32_t* big_n, hipStream_t st);
// Sort set j (size <= n_pow2, a power of two) using scratch[n_pow2].
hipError_t launch_sort_big(const uint64_t* set_off, uint32_t* set_vtx, uint32_t j,
                           uint32_t n_pow2, uint32_t* scratch, hipStream_t st);
constexpr uint32_t kSortSmallMax = 4096;

// ---- greedy selection (k_select.hip)
// A run of at most 64 members of one covered set, queued for decrementing.
struct Chunk {
    uint64_t off;  // position of the first member in set_vtx
    uint32_t len;  // 1..64
    uint32_t pad;
};
// Partial maxima slots per seed step (argmax spreads its atomics over these).
constexpr uint32_t kArgSlots = 32;

// One instance's greedy state, as the batched selection kernels see it.
// Its index has nseg segments; segment r's offsets are
// inv_offs[r * (n + 1) .. r * (n + 1) + n], absolute in inv_set. slots holds
// k * kArgSlots zeroed entries, chunk_n 2k zeroed counters: seed step t
// queues the small covered sets (one entry each) at chunks[0 ..
// chunk_n[2t]) and the 64-member pieces of the others at chunks[chunk_cap -
// chunk_n[2t+1] .. chunk_cap). A step whose covered sets hold more than a
// quarter of all pool entries recounts every count from the index instead of
// decrementing. Workgroups
// [arg_lo, arg_lo + arg_cnt) of the argmax launch and [sel_lo, sel_lo +
// sel_cnt) of the claim and decrement launches belong to this instance;
// ranges ascend with the instance index.
struct SelectDesc {
    uint32_t* cw;
    const uint32_t* cacc;     // index list length of every vertex (over all segments)
    const uint32_t* heavy;    // vertices with cacc > kHeavyList ...
    const uint32_t* n_heavy;  // ... and their number
    const uint64_t* inv_offs;
    const uint32_t* inv_set;
    const uint64_t* set_off;
    const uint32_t* set_vtx;
    uint32_t* covered;
    unsigned long long* slots;
    uint32_t* seeds;
    uint32_t* gains;
    Chunk* chunks;
    uint32_t* chunk_n;
    uint64_t chunk_cap;
    unsigned long long* cov_entries;  // k zeroed: members of the sets step t covers
    uint32_t n, k, nseg;              // nseg <= kMaxSegments
    uint32_t n_sets;
    uint32_t arg_lo, arg_cnt, sel_lo, sel_cnt;
    // counter update after a seed's sets are covered: kUpdateAdaptive
    // (recount when they hold more than a quarter of the pool, else
    // decrement), kUpdateDecrement or kUpdateRecount (always that one)
    uint32_t update = 0;
    // dense sets (bitmaps): n_dense of them, dense_words words each, with
    // their set ids and sizes; dense_entries their total size. Seed step t
    // claims the uncovered ones holding its seed and appends them to
    // dense_list (cursor *dense_list_n; dense_mark[t] is the cursor before
    // step t's claims). Workgroups [dense_lo, dense_lo + dense_cnt) of the
    // dense update launch belong to this instance.
    const uint32_t* dense_bits = nullptr;
    const uint32_t* dense_sid = nullptr;
    const uint32_t* dense_size = nullptr;
    uint32_t* dense_list = nullptr;
    uint32_t* dense_list_n = nullptr;
    uint32_t* dense_mark = nullptr;
    uint64_t dense_entries = 0;
    uint32_t n_dense = 0, dense_words = 0;
    uint32_t dense_lo = 0, dense_cnt = 0;
    // Candidate steps (null cand: none). The vertices whose working count is
    // at least tau when the selection starts (at most kCandMax of them, tau
    // a bin edge of a count histogram) are listed in cand and flagged in
    // cand_bits. Counts only fall, so a vertex outside the list never counts
    // tau or more. From step 1 on, if step 0 did not recount, a step takes
    // its argmax over the list alone, and the decrements skip the vertices
    // outside it: while the best listed count is at least tau, it beats
    // every unlisted vertex, whose stale count is never read. A step whose
    // best listed count falls below tau halts the selection there; the host
    // then recounts every count exactly and runs the remaining steps in full.
    // cand_state: [0] 1 when steps 1.. use the list (decided by step 1's
    // argmax), 2 when they do not; [1] the halting step (0: none); [2] tau;
    // [3] the list length; [4 ..] the histogram (kCandBins bins).
    const uint32_t* cand = nullptr;
    const uint32_t* cand_bits = nullptr;
    uint32_t* cand_state = nullptr;
};
// Candidate list bound, and the count histogram's bins: counts 0..15 one bin
// each, then eight bins per octave (bins ascend with the count).
constexpr uint32_t kCandMax = 4096;
constexpr uint32_t kCandBins = 240;
constexpr uint32_t kCandHead = 4;
enum : uint32_t { kUpdateAdaptive = 0, kUpdateDecrement = 1, kUpdateRecount = 2 };
constexpr uint32_t kMaxSegments = 64;
// A recount gives a vertex with a longer index list a wave of its own.
constexpr uint32_t kHeavyList = 4096;
// Covered sets of at most this many members are decremented one per lane.
constexpr uint32_t kSmallSet = 16;
uint32_t argmax_blocks(uint32_t n);
uint32_t select_blocks(int device, uint64_t n_sets, uint32_t batch);
// cw = cacc, and the list of vertices with cacc > kHeavyList (*n_heavy zeroed).
hipError_t launch_select_init(const uint32_t* cacc, uint32_t* cw, uint32_t n, uint32_t* heavy,
                              uint32_t* n_heavy, hipStream_t st);
// Seed step t (argmax, claim, decrement, and with dense_blocks > 0 the
// bitmap update of the dense sets) of every instance with t < k.
hipError_t launch_select_step(const SelectDesc* descs, uint32_t nq, uint32_t t,
                              uint32_t arg_blocks, uint32_t sel_blocks, uint32_t dense_blocks,
                              hipStream_t st);
// Workgroups of the dense update for n_dense bitmaps of `words` words.
uint32_t dense_blocks(uint32_t n_dense, uint32_t words);
// cw = cacc (+ dc, the dense sets' counts, when given), and the list of
// vertices with cacc > kHeavyList (*n_heavy zeroed).
// The candidate list of a selection whose working counts cw are in place:
// the histogram of cw (cand_state[kCandHead ..], zeroed before), then tau,
// the list and the bitmap (cand_state[3] zeroed before). cand_max <= kCandMax
// bounds the list (0: no list, every step in full).
hipError_t launch_cand_build(const uint32_t* cw, uint32_t n, uint32_t cand_max, uint32_t* cand,
                             uint32_t* cand_bits, uint32_t* cand_state, hipStream_t st);
// An exact recount of every working count from the index and the covered
// sets (descs[0]; its update field must be kUpdateRecount), as a recounting
// seed step does; chosen seeds keep their sentinel.
hipError_t launch_select_recount(const SelectDesc* descs, uint32_t t, uint32_t sel_blocks,
                                 uint32_t dense_blocks, hipStream_t st);
// Word ranges zeroed by launch_select_init2 on the way (the selection's
// covered bits, seed-step block and candidate state; empty ones skipped).
struct ZeroSpans {
    static constexpr uint32_t kCount = 3;
    uint32_t* p[kCount] = {nullptr, nullptr, nullptr};
    uint64_t words[kCount] = {0, 0, 0};
};
hipError_t launch_select_init2(const uint32_t* cacc, const uint32_t* dc, uint32_t* cw,
                               uint32_t n, uint32_t* heavy, uint32_t* n_heavy, hipStream_t st,
                               const ZeroSpans& z = ZeroSpans{});

// ---- misc
hipError_t launch_philox(const uint32_t* ctr, uint64_t count, uint64_t key, uint32_t* out,
                         hipStream_t st);

}  // namespace imm
