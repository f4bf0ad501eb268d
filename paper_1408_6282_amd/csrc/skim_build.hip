// skim_build.hip -- combined bottom-k reachability sketches on gfx950.
//
// What is computed (Section 3, eq. combinedrs): X_v = the k smallest ranks
// r(u, i) over all pairs (u, i) that v reaches in live-edge instance G^(i).
// How (Section 5.2, Algorithm 2, re-organised for the GPU):
//
//  1. Live lists.  One coalesced pass over the edges evaluates every
//     instance's coin of each edge (a 64-bit instance mask per edge); the
//     live (pair, source) entries are written at per-edge prefix offsets
//     and radix-sorted by pair, so the live in-list of every node-instance
//     pair p = 64 v + i is one run, built without atomics.  Each pair's
//     16-byte record holds its search state word next to its list word
//     (the source itself when the list has one entry), so a claim reads
//     both in one cache line.  Every expansion later reads only live
//     in-edges of its own instance, and pairs without any are never put on
//     a frontier.
//  2. Rank windows.  All pairs are bucketed by the bit length of their
//     rank (a stable counting sort, so every bucket is in pair order):
//     bucket 0 holds about k/2 ranks per instance and each later bucket
//     doubles the rank range.  A window is a run of buckets: the first
//     five (a pair is pruned only once it has received k ranks, so merging
//     early buckets costs few extra visits and saves search levels); if
//     that window overflows, the build restarts with bucket 0 alone and
//     then as many buckets as keep the arrivals per pair (measured on
//     bucket 0) below k.  Later windows take window_span buckets, or one
//     after a window with many visits per pair, and the last bucket alone.
//     Windows are processed in increasing order.
//  3. Pruned reverse searches, window by window.  Every source pair (u, i)
//     of the window runs a reverse search in G^(i).  A visited pair (w, i)
//     is pruned when it received k ranks in earlier windows (the paper's
//     rule: its instance-local sketch is full).  Because every pair on a
//     path to an unpruned pair reaches a subset of what it reaches, an
//     unpruned pair receives every rank of its instance in the window, so
//     the rule is exact whatever order the window's searches run in.  All
//     searches of a window advance together, level by level: one
//     whole-grid launch per level (frontiers in batches of levels launched
//     without reading their sizes back); once the frontier is small it is
//     split over many workgroups that each run the remaining levels of their
//     part in LDS, without waiting for each other (the window's result does
//     not depend on the order of its visits).  Visits are
//     deduplicated per source exactly: the first visitor of a pair in the
//     window claims the pair's state word; later visitors go through a
//     hash set keyed by (pair, source).  The same word counts the pair's
//     arrivals (up to k, all pruning needs).  A visit that could neither
//     expand nor record (no live in-edge, node no longer recording) is
//     skipped.
//  4. Records.  A visit of node v is recorded while v held fewer than k
//     ranks at the window start; windows go up in rank, so the k smallest
//     records of v are its sketch.
//  5. Merge.  Records are sorted by node (radix sort on the node bits) and
//     each node keeps its k smallest ranks in LDS (bitonic sort), written
//     ascending.
//
// Device atomics from different waves on one 128-byte line are serialised
// by the hardware, so shared counters sit on lines of their own and are
// added to once per workgroup.
#include "skim_internal.h"

#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <chrono>
#include <cstdlib>
#include <mutex>
#include <string>
#include <cstring>

namespace skim {


namespace {

constexpr uint32_t kOvfHash = 2u, kOvfRecords = 4u, kOvfSpill = 8u;
constexpr uint32_t kOvfFirst = 16u;  // the optimistic first window overflowed
// Buckets of the first window: about 8k ranks per instance, which on graphs
// with modest reach sets is still below where pruning starts; graphs where
// it overflows restart with bucket 0 alone.
constexpr uint32_t kFirstSpan = 5;
constexpr int kBlock = 256;

// Thrown inside the build when a buffer was too small; the windows restart
// from scratch with larger buffers.
struct Retry {
    uint32_t flags;
};

// Device control block read back by the host at synchronisation points.
// Level L of a window's search reads front[L % 2] (size[L % 3] entries) and
// appends level L + 1 to front[(L + 1) % 2], counting in size[(L + 1) % 3];
// it also clears size[(L + 2) % 3] for the level after.
// Every counter has a 128-byte line of its own: device atomics on one line
// are serialised (about 12 ns each on the MI355X, whichever word of the
// line they hit), so counters sharing a line would queue behind each other.
struct alignas(128) Ctl {
    unsigned long long size[3 * 16];  // frontier sizes, ring over levels: size[16 j]
    unsigned long long scans;         // live in-edges scanned (work counter)
    char pad0[120];
    unsigned long long hinserts;      // hash-set insertions in this window
    char pad1[120];
    unsigned long long records;       // records appended (all windows)
    char pad2[120];
    unsigned long long full;          // nodes holding k records
    char pad3[120];
    unsigned long long visits;        // accepted visits (work counter)
    char pad4[120];
    uint32_t flags;                   // overflow bits
    uint32_t level;                   // level reached by the tail kernel
    char pad5[120];
    unsigned long long budget;        // visits reserved by the workgroup tails (k_tails)
    char pad6[120];
    unsigned long long hsize[2 * 16];  // long-list entries of level L: hsize[16 (L % 2)]
};

// ------------------------------------------------------- 2. rank windows

// Rank bucket: bucket 0 holds the ranks of at most `b0` bits, bucket j >= 1
// the ranks of exactly b0 + j bits (each bucket doubles the rank range seen
// so far).  A window is a run of one or two consecutive buckets.
__device__ __forceinline__ uint32_t bucket_of(uint64_t r, uint32_t b0) {
    const int bits = r ? 64 - __clzll((long long)r) : 0;
    return bits <= (int)b0 ? 0u : (uint32_t)(bits - (int)b0);
}

// Rank of pair p: the hashed rank r(v, i), or the pair's entry of a rank
// table (structured permutation positions).
__device__ __forceinline__ uint64_t rank_of(uint64_t seed, const uint64_t *table, uint32_t p) {
    return table ? table[p] : pair_rank(seed, p);
}

constexpr int kRankPer = 8;  // pairs per thread in the bucketing kernels

// Bucketing is a stable counting sort: each block counts its pairs per
// bucket (bcount is bucket-major, so one exclusive scan gives every block
// its place inside every bucket), then writes its pairs in pair order.
// Every bucket of the sources array is therefore in increasing pair order,
// and a window's pair records are visited in memory order.
// Pairs whose rank exceeds `limit` can enter no sketch and are left out.
__global__ void k_rank_hist(uint32_t n, uint32_t ell, uint64_t seed, const uint64_t *table,
                            uint64_t limit, uint32_t W, uint32_t b0, uint32_t *bcount,
                            uint32_t nblocks) {
    __shared__ uint32_t h[64];
    if (threadIdx.x < 64) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t total = (uint64_t)n * ell;
    const uint64_t base = (uint64_t)blockIdx.x * kBlock * kRankPer;
    for (int j = 0; j < kRankPer; ++j) {
        const uint64_t t = base + (uint64_t)j * kBlock + threadIdx.x;
        if (t < total) {
            const uint32_t v = (uint32_t)(t / ell), i = (uint32_t)(t % ell);
            const uint64_t r = rank_of(seed, table, v * kPairStride + i);
            if (r <= limit) atomicAdd(&h[bucket_of(r, b0)], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < W) bcount[(uint64_t)threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x];
}

// Bucket b starts at boff[b * nblocks] (b = W: the total).
__global__ void k_bucket_bases(const uint64_t *boff, uint32_t nblocks, uint32_t W,
                               unsigned long long *wb) {
    if (threadIdx.x <= W) wb[threadIdx.x] = boff[(uint64_t)threadIdx.x * nblocks];
}

// Pairs base + j * kBlock + tid, in that order (j outer): within each round
// j every wave ranks its lanes per bucket by ballots, and the waves of the
// block and the earlier rounds are added in order.
__global__ void __launch_bounds__(kBlock) k_rank_scatter(uint32_t n, uint32_t ell, uint64_t seed,
                                                         const uint64_t *table, uint64_t limit,
                                                         uint32_t W, uint32_t b0,
                                                         const uint64_t *boff, uint32_t nblocks,
                                                         uint32_t *sources) {
    constexpr int kWaves = kBlock / 64;
    __shared__ uint32_t wcnt[kWaves][64];  // lanes per bucket of every wave, this round
    __shared__ uint32_t run[64];           // pairs per bucket of the earlier rounds
    const uint32_t tid = threadIdx.x, wave = tid / 64, lane = tid % 64;
    if (tid < 64) run[tid] = 0;
    const uint64_t total = (uint64_t)n * ell;
    const uint64_t base = (uint64_t)blockIdx.x * kBlock * kRankPer;
    for (int j = 0; j < kRankPer; ++j) {
        wcnt[wave][lane] = 0;
        __syncthreads();
        const uint64_t t = base + (uint64_t)j * kBlock + tid;
        uint32_t b = 0xFFFFFFFFu, pid = 0, rank = 0;
        if (t < total) {
            const uint32_t v = (uint32_t)(t / ell), i = (uint32_t)(t % ell);
            pid = v * kPairStride + i;
            const uint64_t r = rank_of(seed, table, pid);
            if (r <= limit) b = bucket_of(r, b0);
        }
        bool todo = b != 0xFFFFFFFFu;
        for (;;) {  // one bucket of this wave per pass (wave-uniform loop)
            const unsigned long long act = __ballot(todo);
            if (!act) break;
            const int leader = __ffsll((long long)act) - 1;
            const uint32_t bb = __shfl(b, leader);
            const bool mine = todo && b == bb;
            const unsigned long long m = __ballot(mine);
            if (mine) {
                rank = (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                todo = false;
            }
            if ((int)lane == leader) wcnt[wave][bb] = (uint32_t)__popcll(m);
        }
        __syncthreads();
        if (b != 0xFFFFFFFFu) {
            uint32_t before = run[b] + rank;
            for (uint32_t w2 = 0; w2 < wave; ++w2) before += wcnt[w2][b];
            sources[boff[(uint64_t)b * nblocks + blockIdx.x] + before] = pid;
        }
        __syncthreads();
        if (tid < 64)
            for (int w2 = 0; w2 < kWaves; ++w2) run[tid] += wcnt[w2][tid];
        __syncthreads();
    }
}

// --------------------------------------------------- pair state words
// One 64-bit word per pair p = 64 v + i:
//   bits  0..31  stamp: source pair of the first visitor in window `tag`
//   bits 32..39  tag:   window of the last visit (0xFF: never visited)
//   bits 40..51  arr:   sources that visited the pair in window `tag`
//   bits 52..63  cnt:   sources that visited it before window `tag`
// Counts are at most 4095 (> every k); see claim() for arrivals beyond.  The
// pair's count of received ranks at the start of window w is cnt, plus arr
// when tag < w.
constexpr uint64_t kWordInit = 0xFFull << 32;
constexpr uint32_t kSat = 4095;

__device__ __forceinline__ uint32_t w_tag(uint64_t w) { return (uint32_t)(w >> 32) & 0xFFu; }
__device__ __forceinline__ uint32_t w_arr(uint64_t w) { return (uint32_t)(w >> 40) & 0xFFFu; }
__device__ __forceinline__ uint32_t w_cnt(uint64_t w) { return (uint32_t)(w >> 52); }

__device__ __forceinline__ uint32_t prior_count(uint64_t w, uint32_t win) {
    const uint32_t c = w_cnt(w) + (w_tag(w) != win ? w_arr(w) : 0u);
    return c < kSat ? c : kSat;
}

__device__ __forceinline__ uint64_t hmix(uint64_t x) {
    x ^= x >> 31;
    x *= 0xD6E8FEB86659FD93ull;
    x ^= x >> 32;
    return x;
}

// Hash-set keys (pair, source).  When pair ids fit in 28 bits, a window
// tag (1..239) rides in the top nibbles of both halves; keys of earlier
// windows then count as empty slots and the set needs no clearing between
// windows.  Tag 0: untagged keys, every non-empty slot is live.
__device__ __forceinline__ uint64_t hkey(uint32_t q, uint32_t src, uint32_t tag) {
    return ((uint64_t)(q | ((tag >> 4) << 28)) << 32) | (src | ((tag & 0xFu) << 28));
}
__device__ __forceinline__ uint32_t hkey_tag(uint64_t key) {
    return (uint32_t)(key >> 60) << 4 | ((uint32_t)(key >> 28) & 0xFu);
}
__device__ __forceinline__ bool hslot_free(uint64_t cur, uint32_t tag) {
    return cur == kNone || (tag && hkey_tag(cur) != tag);
}

// 1 = inserted, 0 = already present, -1 = table full.  Slots only go from
// free to live within a window, so a probe chain never loses a key.
// Each probe starts with a CAS that expects an empty slot (the common case
// when most keys are new): its return value is the slot's content, so no
// load precedes it.  With look_first (graphs whose dense cores bring the
// same (pair, source) key back many times) a plain load comes first, so a
// key already present costs no atomic: atomics on one line are serialised,
// loads are not.
__device__ int hset_insert(uint64_t *T, uint32_t logcap, uint64_t key, uint32_t tag,
                           bool look_first = false) {
    const uint64_t mask = (1ull << logcap) - 1;
    uint64_t h = hmix(key) & mask;
    for (int probe = 0; probe < 256; ++probe) {
        if (look_first) {
            const uint64_t seen = load_relaxed(T + h);
            if (seen == key) return 0;
            if (!hslot_free(seen, tag)) {
                h = (h + 1) & mask;
                continue;
            }
        }
        uint64_t cur = atomicCAS((unsigned long long *)(T + h), kNone, key);
        if (cur == kNone) return 1;
        if (cur == key) return 0;
        if (hslot_free(cur, tag)) {
            const uint64_t prev = atomicCAS((unsigned long long *)(T + h), cur, key);
            if (prev == cur) return 1;
            if (prev == key) return 0;  // else a live key of this window took it
        }
        h = (h + 1) & mask;
    }
    return -1;
}

// Move every live key of a hash set into a larger, cleared one.
__global__ void k_rehash(const uint64_t *old, uint64_t old_size, uint64_t *T, uint32_t logcap,
                         uint32_t tag, uint32_t *flags) {
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < old_size;
         j += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t key = old[j];
        if (!hslot_free(key, tag) && hset_insert(T, logcap, key, tag) < 0)
            atomicOr(flags, kOvfHash);
    }
}

// Per-pair record, 16 bytes, in one array: the state word (above) and the
// pair's live in-list, read by the claim in the same cache line.  The list
// word is 0 for no live in-edge, bit 63 | u for the single source u, else
// begin << 24 | count into the live-source array.

struct WinArgs {
    uint64_t *prec;        // [2 * 64 n] state word, live-list word per pair
    const uint32_t *lsrc;  // live sources of lists with two or more entries
    uint64_t *hset;
    uint32_t logcap;
    uint32_t htag;         // hash-key tag of this window (0: untagged)
    uint32_t win;          // window id (tag)
    uint32_t k;
    uint32_t last;         // last window: its arrivals are never read
    const uint8_t *want;   // node records its visits in this window (fewer than k so far)
    uint64_t *rec;         // records: (node << 32) | source pair
    uint64_t rec_cap;
    uint64_t *fkey[2];     // current / next level: (pair << 32) | source pair
    uint64_t *flive[2];    // the pair's live-list word
    uint64_t front_cap;
    Ctl *ctl;
    uint64_t *heavy;       // [2 kHeavyMax] entries with long lists (key, list word), for
                           // k_expand_heavy; set only on graphs with such lists, which also
                           // probe the hash set load-first
};

// Visit of pair q by the search of source pair src: 1 if it is a new visit
// (and counts as one more rank received by q), 0 if pruned or repeated.
// `live` receives q's live-list word.  A pair without live in-edges whose
// node records nothing more (`want` false) is skipped outright: the visit
// would neither expand nor record, and its count serves nothing (such a
// pair never expands, and its node's recording never resumes).
__device__ __forceinline__ int claim(const WinArgs &A, uint32_t q, uint32_t src, bool want,
                                     uint32_t &hashed, uint64_t &live) {
    uint64_t *rq = A.prec + 2 * (uint64_t)q;
    uint64_t old = load_relaxed(rq);
    live = rq[1];  // read-only during the searches
    if (!live && !want) return 0;
    for (;;) {
        if (prior_count(old, A.win) >= A.k) return 0;  // instance-local sketch full: prune
        if (w_tag(old) != A.win) {
            const uint64_t nw = (uint64_t)src | ((uint64_t)A.win << 32) | (1ull << 40) |
                                ((uint64_t)prior_count(old, A.win) << 52);
            const uint64_t prev = atomicCAS((unsigned long long *)rq, old, nw);
            if (prev == old) return 1;
            old = prev;
            continue;
        }
        if ((uint32_t)old == src) return 0;
        const int r =
            hset_insert(A.hset, A.logcap, hkey(q, src, A.htag), A.htag, A.heavy != nullptr);
        if (r <= 0) {
            if (r < 0) atomicOr(&A.ctl->flags, kOvfHash);
            return 0;
        }
        // One more source reached q in this window.  A carry out of the
        // 12-bit arrival field (4096 arrivals) turns into +1 on cnt, and cnt
        // itself can wrap: both only ever undercount, which can only weaken
        // pruning, never make it wrong.  Arrivals only serve later windows,
        // and only until the pair holds k (the word read above may be older
        // than the pair's count, never newer).
        if (!A.last && w_cnt(old) + w_arr(old) < A.k) atomicAdd((unsigned long long *)rq, 1ull << 40);
        ++hashed;
        return 1;
    }
}

// Record a visit of node v when v held fewer than k ranks at the window start.
__device__ __forceinline__ bool wants_record(const WinArgs &A, uint32_t v) {
    return A.want[v] != 0;
}

// ------------------------------------ 3. level-synchronous window search
// Block-aggregated appends: threads stage new entries in LDS; one global
// reservation per flush moves them to the output arrays (coalesced).
constexpr uint32_t kChunk = 1024;   // frontier entries per block per round
constexpr uint32_t kStageF = 1024;  // staged frontier entries per round (16 bytes each)
constexpr uint32_t kStageR = 1912;  // staged records per round (5 workgroups fit in LDS)
constexpr uint32_t kHeavyCap = 256;  // long live lists per round expanded by the whole block
constexpr uint32_t kSerialEdges = 16;  // longer lists go to the block
// Still longer lists (hubs) are deferred to k_expand_heavy, which spreads
// their entries over every workgroup (at most kHeavyMax per level; more are
// expanded by their block).
constexpr uint32_t kSplitLive = 4096;
constexpr uint32_t kHeavyMax = 1u << 20;

struct StageF {
    uint64_t key[kStageF];
    uint64_t live[kStageF];
    uint32_t n;
    unsigned long long base;
};

struct StageR {
    uint64_t buf[kStageR];
    uint32_t n;
    unsigned long long base;
};

// Stage slots are handed out per wave (one LDS atomic for all lanes that
// push at once); when a stage is full the overflowing lanes reserve their
// output slots per wave as well, so a burst of outputs (a hub's in-edges)
// does not serialise on one global counter.
__device__ __forceinline__ uint32_t stage_slots(uint32_t *n) {
    const unsigned long long act = __ballot(1);
    const int leader = __ffsll((long long)act) - 1;
    const uint32_t lane = lane_id();
    uint32_t pos0 = 0;
    if ((int)lane == leader) pos0 = atomicAdd(n, (uint32_t)__popcll(act));
    return __shfl(pos0, leader) + (uint32_t)__popcll(act & ((1ull << lane) - 1ull));
}

// Frontier entries carry the pair's live-list word; pairs without live
// in-edges have nothing to expand and are not appended.
__device__ __forceinline__ void push_front(StageF &S, uint64_t key, uint64_t live, uint64_t *okey,
                                           uint64_t *olive, uint64_t cap,
                                           unsigned long long *count, uint32_t *flags) {
    const uint32_t pos = stage_slots(&S.n);
    if (pos < kStageF) {
        S.key[pos] = key;
        S.live[pos] = live;
        return;
    }
    const uint64_t g = wave_reserve(count, true);  // stage full
    if (g < cap) {
        okey[g] = key;
        olive[g] = live;
    } else {
        atomicOr(flags, kOvfSpill);
    }
}

__device__ __forceinline__ void push_record(StageR &S, uint64_t v, uint64_t *out, uint64_t cap,
                                            unsigned long long *count, uint32_t *flags) {
    const uint32_t pos = stage_slots(&S.n);
    if (pos < kStageR) {
        S.buf[pos] = v;
        return;
    }
    const uint64_t g = wave_reserve(count, true);  // stage full
    if (g < cap) out[g] = v;
    else atomicOr(flags, kOvfRecords);
}

// Flush both stages; the two reservations are issued by different waves so
// they are in flight together.  Called by every thread of the block.
__device__ __forceinline__ void stage_flush2(StageF &F, uint64_t *okey, uint64_t *olive,
                                             uint64_t fcap, unsigned long long *fcount, StageR &R,
                                             uint64_t *rout, uint64_t rcap,
                                             unsigned long long *rcount, uint32_t *flags,
                                             uint32_t *heavy_n = nullptr) {
    __syncthreads();
    const uint32_t mf = F.n < kStageF ? F.n : kStageF;
    const uint32_t mr = R.n < kStageR ? R.n : kStageR;
    if (threadIdx.x == 0) F.base = mf ? atomicAdd(fcount, (unsigned long long)mf) : 0;
    if (threadIdx.x == 64) R.base = mr ? atomicAdd(rcount, (unsigned long long)mr) : 0;
    __syncthreads();
    const unsigned long long fb = F.base, rb = R.base;
    if (threadIdx.x == 0 && mf && fb + mf > fcap) atomicOr(flags, kOvfSpill);
    if (threadIdx.x == 64 && mr && rb + mr > rcap) atomicOr(flags, kOvfRecords);
    for (uint32_t j = threadIdx.x; j < mf; j += blockDim.x) {
        if (fb + j < fcap) {
            okey[fb + j] = F.key[j];
            olive[fb + j] = F.live[j];
        }
    }
    for (uint32_t j = threadIdx.x; j < mr; j += blockDim.x)
        if (rb + j < rcap) rout[rb + j] = R.buf[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        F.n = R.n = 0;
        if (heavy_n) *heavy_n = 0;
    }
    __syncthreads();
}

__device__ __forceinline__ uint32_t live_count(uint64_t live) {
    return (uint32_t)(live & ((1u << kLiveCountBits) - 1));
}

struct ExpandShared {
    StageF F;
    StageR R;
    uint32_t heavy[kHeavyCap];  // frontier positions of this round's long lists
    uint32_t nheavy;
    uint32_t hex[kHeavyCap + 1];  // their starts when laid end to end
    uint64_t hkey[kHeavyCap], hlive[kHeavyCap];
    uint32_t hwsum[kBlock / 64];
};

__device__ __forceinline__ uint64_t shfl_u64(uint64_t x, uint32_t src) {
    const uint32_t lo = __shfl((uint32_t)x, (int)src), hi = __shfl((uint32_t)(x >> 32), (int)src);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_up_u64(uint64_t x, uint32_t d) {
    const uint32_t lo = __shfl_up((uint32_t)x, d), hi = __shfl_up((uint32_t)(x >> 32), d);
    return ((uint64_t)hi << 32) | lo;
}

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t x, int m) {
    const uint32_t lo = __shfl_xor((uint32_t)x, m), hi = __shfl_xor((uint32_t)(x >> 32), m);
    return ((uint64_t)hi << 32) | lo;
}

// Adds this workgroup's sums of up to three counters with one device atomic
// each (per-wave atomics at the end of a launch would all queue on the
// counters' lines).  Called by every thread; `scratch` holds 3 words per
// wave of LDS that is free at this point.
__device__ __forceinline__ void block_add3(uint64_t *scratch, unsigned long long *c0, uint32_t x0,
                                           unsigned long long *c1, uint32_t x1,
                                           unsigned long long *c2, uint32_t x2) {
    unsigned long long v[3] = {x0, x1, x2};
    for (int j = 0; j < 3; ++j)
        for (int off = 32; off > 0; off >>= 1) v[j] += shfl_xor_u64(v[j], off);
    const uint32_t wave = threadIdx.x / 64, waves = (blockDim.x + 63) / 64;
    __syncthreads();
    if (lane_id() == 0)
        for (int j = 0; j < 3; ++j) scratch[3 * wave + j] = v[j];
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long *c[3] = {c0, c1, c2};
        for (int j = 0; j < 3; ++j) {
            unsigned long long t = 0;
            for (uint32_t w = 0; w < waves; ++w) t += scratch[3 * w + j];
            if (t && c[j]) atomicAdd(c[j], t);
        }
    }
}

// One live in-edge w -> v of the expanded pair (v, i), taken by the search
// of source pair src.
__device__ __forceinline__ void visit_edge(const WinArgs &A, uint32_t w, uint32_t i, uint32_t src,
                                           uint64_t *nkey, uint64_t *nlive,
                                           unsigned long long *next_count, ExpandShared &X,
                                           uint32_t &scans, uint32_t &hashed, uint32_t &visits) {
    const uint32_t q = w * kPairStride + i;
    ++scans;
    const bool want = wants_record(A, w);
    uint64_t live;
    if (claim(A, q, src, want, hashed, live) == 1) {
        ++visits;
        if (live)
            push_front(X.F, ((uint64_t)q << 32) | src, live, nkey, nlive, A.front_cap, next_count,
                       &A.ctl->flags);
        if (want)
            push_record(X.R, ((uint64_t)w << 32) | src, A.rec, A.rec_cap, &A.ctl->records,
                        &A.ctl->flags);
    }
}

// Expand the current level's entries [0, b) (already claimed and recorded)
// over their live in-edges; new visits are recorded and appended to the
// next level (counted in *next_count).
__device__ __forceinline__ void expand_range(const WinArgs &A, uint32_t L,
                                             unsigned long long *next_count, uint64_t b,
                                             uint32_t chunk, ExpandShared &X, uint32_t &scans,
                                             uint32_t &hashed, uint32_t &visits) {
    const uint64_t *ckey = A.fkey[L & 1], *clive = A.flive[L & 1];
    uint64_t *nkey = A.fkey[(L + 1) & 1], *nlive = A.flive[(L + 1) & 1];
    const uint64_t stride = (uint64_t)gridDim.x * chunk;
    for (uint64_t c = (uint64_t)blockIdx.x * chunk; c < b; c += stride) {
        const uint64_t end = c + chunk < b ? c + chunk : b;
        // Each wave lays the short lists of its 64 entries end to end and
        // takes them 64 entries at a time (a lane finds the entry of its
        // position by binary lifting over the wave's prefix sums), so one
        // lane's longer list does not hold the others.
        const uint32_t lane = lane_id();
        for (uint64_t tb = c; tb < end; tb += blockDim.x) {
            const uint64_t t = tb + threadIdx.x;
            uint64_t it = 0, live = 0;
            uint32_t nwork = 0;
            if (t < end) {
                it = ckey[t];
                live = clive[t];
                const uint32_t cnt = (live & kLiveOne) ? 1u : live_count(live);
                nwork = cnt;
                if (cnt > kSplitLive && A.heavy) {  // a hub's list: the whole grid, next launch
                    const unsigned long long slot =
                        atomicAdd(&A.ctl->hsize[16 * (L % 2)], 1ull);
                    if (slot < kHeavyMax) {
                        A.heavy[2 * slot] = it;
                        A.heavy[2 * slot + 1] = live;
                        nwork = 0;
                    }
                }
                if (nwork > kSerialEdges) {  // a long list: the whole block takes it below
                    const uint32_t slot = stage_slots(&X.nheavy);
                    if (slot < kHeavyCap) {
                        X.heavy[slot] = (uint32_t)(t - c);
                        nwork = 0;
                    }
                }
            }
            if (__all(nwork <= 1)) {  // the common case: at most one edge per entry
                if (nwork) {
                    const uint32_t w =
                        (live & kLiveOne) ? (uint32_t)live : A.lsrc[live >> kLiveCountBits];
                    visit_edge(A, w, (uint32_t)(it >> 32) % kPairStride, (uint32_t)it, nkey,
                               nlive, next_count, X, scans, hashed, visits);
                }
                continue;
            }
            uint32_t incl = nwork;  // inclusive prefix over the wave
            for (uint32_t off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off);
                if (lane >= off) incl += y;
            }
            const uint32_t total = __shfl(incl, 63);
            for (uint32_t base = 0; base < total; base += 64) {
                const uint32_t j = base + lane;
                uint32_t r = 0;  // lanes whose entries end at or before position j
                for (uint32_t step = 32; step > 0; step >>= 1) {
                    const uint32_t v = __shfl(incl, (int)(r + step - 1));
                    if (v <= j) r += step;
                }
                const uint32_t rr = r & 63u;
                const uint32_t first = __shfl(incl, (int)rr) - __shfl(nwork, (int)rr);
                const uint64_t rit = shfl_u64(it, rr), rlive = shfl_u64(live, rr);
                if (j < total) {
                    const uint32_t w = (rlive & kLiveOne)
                                           ? (uint32_t)rlive
                                           : A.lsrc[(rlive >> kLiveCountBits) + (j - first)];
                    visit_edge(A, w, (uint32_t)(rit >> 32) % kPairStride, (uint32_t)rit, nkey,
                               nlive, next_count, X, scans, hashed, visits);
                }
            }
        }
        __syncthreads();
        // Long live lists (up to 4096 sources) laid end to end and spread
        // over all threads of the block, instead of one thread walking each.
        const uint32_t nh = X.nheavy < kHeavyCap ? X.nheavy : kHeavyCap;
        if (nh) {  // uniform: read after the barrier
            static_assert(kHeavyCap == kBlock, "one long list per thread");
            const uint32_t tid = threadIdx.x, wave = tid >> 6;
            uint32_t cnt = 0;
            if (tid < nh) {
                const uint64_t t = c + X.heavy[tid];
                X.hkey[tid] = ckey[t];
                X.hlive[tid] = clive[t];
                cnt = live_count(X.hlive[tid]);
            }
            uint32_t incl = cnt;
            for (uint32_t off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off);
                if (lane >= off) incl += y;
            }
            if (lane == 63u) X.hwsum[wave] = incl;
            __syncthreads();
            uint32_t before = 0, H = 0;
            for (uint32_t w = 0; w < kBlock / 64; ++w) {
                before += w < wave ? X.hwsum[w] : 0u;
                H += X.hwsum[w];
            }
            X.hex[tid] = before + incl - cnt;
            if (tid == 0) X.hex[kHeavyCap] = H;
            __syncthreads();
            for (uint32_t p = tid; p < H; p += blockDim.x) {
                uint32_t lo = 0, hi = kHeavyCap;  // hex[lo] <= p < hex[hi]
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (X.hex[mid] <= p) lo = mid;
                    else hi = mid;
                }
                const uint64_t it = X.hkey[lo];
                const uint64_t e = (X.hlive[lo] >> kLiveCountBits) + (p - X.hex[lo]);
                visit_edge(A, A.lsrc[e], (uint32_t)(it >> 32) % kPairStride, (uint32_t)it, nkey,
                           nlive, next_count, X, scans, hashed, visits);
            }
        }
        stage_flush2(X.F, nkey, nlive, A.front_cap, next_count, X.R, A.rec, A.rec_cap,
                     &A.ctl->records, &A.ctl->flags, &X.nheavy);
    }
}

// Level 0: the window's sources visit their own pairs.  Each source pair is
// reached only by its own source at this point, so the claim is a store.
__global__ void __launch_bounds__(kBlock) k_seed_window(WinArgs A, const uint32_t *sources,
                                                        uint64_t ws, uint64_t we) {
    __shared__ ExpandShared X;
    if (threadIdx.x == 0) X.F.n = X.R.n = 0;
    __syncthreads();
    uint32_t visits = 0;
    for (uint64_t c = ws + (uint64_t)blockIdx.x * kChunk; c < we;
         c += (uint64_t)gridDim.x * kChunk) {
        const uint64_t end = c + kChunk < we ? c + kChunk : we;
        for (uint64_t t = c + threadIdx.x; t < end; t += blockDim.x) {
            const uint32_t p = sources[t];
            uint64_t *rp = A.prec + 2 * (uint64_t)p;
            const uint64_t old = rp[0], live = rp[1];
            const uint32_t prior = prior_count(old, A.win);
            if (prior >= A.k) continue;  // pruned
            const uint32_t v = p / kPairStride;
            const bool want = wants_record(A, v);
            if (!live && !want) continue;  // would neither expand nor record (see claim)
            rp[0] = (uint64_t)p | ((uint64_t)A.win << 32) | (1ull << 40) | ((uint64_t)prior << 52);
            ++visits;
            if (live)
                push_front(X.F, ((uint64_t)p << 32) | p, live, A.fkey[0], A.flive[0], A.front_cap,
                           &A.ctl->size[16 * (0)], &A.ctl->flags);
            if (want)
                push_record(X.R, ((uint64_t)v << 32) | p, A.rec, A.rec_cap, &A.ctl->records,
                            &A.ctl->flags);
        }
        stage_flush2(X.F, A.fkey[0], A.flive[0], A.front_cap, &A.ctl->size[16 * (0)], X.R, A.rec,
                     A.rec_cap, &A.ctl->records, &A.ctl->flags);
    }
    block_add3(X.R.buf, &A.ctl->visits, visits, nullptr, 0, nullptr, 0);
}

// Level L of the window's search, on the whole grid; each block takes
// `chunk` (<= kChunk) frontier entries per round.
__global__ void __launch_bounds__(kBlock) k_expand(WinArgs A, uint32_t L, uint32_t chunk) {
    __shared__ ExpandShared X;
    __shared__ uint32_t s_flags;
    __shared__ unsigned long long s_size;
    if (threadIdx.x == 0) {
        X.F.n = X.R.n = X.nheavy = 0;
        s_flags = __hip_atomic_load(&A.ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_size = A.ctl->size[16 * (L % 3)];
        if (blockIdx.x == 0) {
            A.ctl->size[16 * ((L + 2) % 3)] = 0;  // counter of level L + 2
            A.ctl->hsize[16 * ((L + 1) % 2)] = 0;  // long lists of level L + 1
        }
    }
    __syncthreads();
    uint32_t scans = 0, hashed = 0, visits = 0;
    if (!s_flags && s_size) {  // after an overflow the windows are redone with more room
        expand_range(A, L, &A.ctl->size[16 * ((L + 1) % 3)], s_size, chunk, X, scans, hashed, visits);
    }
    block_add3(X.R.buf, &A.ctl->scans, scans, &A.ctl->hinserts, hashed, &A.ctl->visits, visits);
}

// The long live lists that level L deferred (hubs), their entries spread
// evenly over every workgroup: kBlock lists at a time, each workgroup taking
// an equal range of their entries laid end to end.  Visits, appends and
// records are those of k_expand for level L.
__global__ void __launch_bounds__(kBlock) k_expand_heavy(WinArgs A, uint32_t L) {
    __shared__ ExpandShared X;
    __shared__ uint64_t ex[kBlock + 1], wsum[kBlock / 64], hk[kBlock], hl[kBlock];
    __shared__ uint32_t s_flags;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wave = tid >> 6;
    if (tid == 0) {
        X.F.n = X.R.n = X.nheavy = 0;
        s_flags = __hip_atomic_load(&A.ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    const unsigned long long hc = A.ctl->hsize[16 * (L % 2)];  // final: level L has ended
    const uint32_t nh = hc < kHeavyMax ? (uint32_t)hc : kHeavyMax;
    if (s_flags || nh == 0) return;  // uniform
    uint64_t *nkey = A.fkey[(L + 1) & 1], *nlive = A.flive[(L + 1) & 1];
    unsigned long long *next_count = &A.ctl->size[16 * ((L + 1) % 3)];
    uint32_t scans = 0, hashed = 0, visits = 0;
    for (uint32_t h0 = 0; h0 < nh; h0 += kBlock) {
        uint64_t key = 0, live = 0, cnt = 0;
        if (h0 + tid < nh) {
            key = A.heavy[2 * (h0 + tid)];
            live = A.heavy[2 * (h0 + tid) + 1];
            cnt = live_count(live);
        }
        // exclusive prefix of the list lengths over the block
        uint64_t x = cnt;
        for (uint32_t off = 1; off < 64; off <<= 1) {
            const uint64_t y = shfl_up_u64(x, off);
            if (lane >= off) x += y;
        }
        if (lane == 63u) wsum[wave] = x;
        __syncthreads();
        uint64_t before = 0, tot = 0;
        for (uint32_t w = 0; w < kBlock / 64; ++w) {
            before += w < wave ? wsum[w] : 0;
            tot += wsum[w];
        }
        ex[tid] = before + x - cnt;
        hk[tid] = key;
        hl[tid] = live;
        if (tid == 0) ex[kBlock] = tot;
        __syncthreads();
        const uint64_t a = tot * blockIdx.x / gridDim.x, b = tot * (blockIdx.x + 1) / gridDim.x;
        for (uint64_t base = a; base < b; base += kBlock) {
            const uint64_t t = base + tid;
            if (t < b) {
                uint32_t lo = 0, hi = kBlock;  // ex[lo] <= t < ex[hi]
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (ex[mid] <= t) lo = mid;
                    else hi = mid;
                }
                const uint64_t it = hk[lo];
                const uint32_t i = (uint32_t)(it >> 32) % kPairStride;
                const uint64_t e = (hl[lo] >> kLiveCountBits) + (t - ex[lo]);
                visit_edge(A, A.lsrc[e], i, (uint32_t)it, nkey, nlive, next_count, X, scans,
                           hashed, visits);
            }
            // flush the stages before they can overflow (the test is uniform:
            // the counts are read between two barriers)
            __syncthreads();
            const bool full = X.F.n > kStageF - kBlock || X.R.n > kStageR - kBlock;
            __syncthreads();
            if (full)
                stage_flush2(X.F, nkey, nlive, A.front_cap, next_count, X.R, A.rec, A.rec_cap,
                             &A.ctl->records, &A.ctl->flags);
        }
        __syncthreads();  // ex, hk, hl are reused
    }
    stage_flush2(X.F, nkey, nlive, A.front_cap, next_count, X.R, A.rec, A.rec_cap,
                 &A.ctl->records, &A.ctl->flags);
    block_add3(X.R.buf, &A.ctl->scans, scans, &A.ctl->hinserts, hashed, &A.ctl->visits, visits);
}

// ------------------------------------------- level by pull (other side)
// A level can also be taken from the visited side: every pair q = (u, i)
// reads its live out-list and, for each out-neighbour pair p = (w, i) with
// entries in the level's frontier, makes the visit of q by each of their
// sources.  These are the (q, source) attempts the push makes for the level,
// met in another order; since a level's outcome does not depend on that
// order (see claim), neither does the build's.  `skey` is the frontier
// sorted by pair; for a pair p with entries, skey[fidx[p] - 1 .. fend[p])
// are they (fidx[p] = 0 for a pair without entries; fend is then unused).
__global__ void k_pull_index(const uint64_t *skey, uint64_t f, uint32_t *fidx, uint32_t *fend) {
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < f;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t p = skey[t] >> 32;
        if (t == 0 || (skey[t - 1] >> 32) != p) fidx[p] = (uint32_t)(t + 1);
        if (t + 1 == f || (skey[t + 1] >> 32) != p) fend[p] = (uint32_t)(t + 1);
    }
}

// Level L by pull over the n l actual pairs, node by node (pair 64 u + i for
// i < l), kChunk pairs per workgroup per round.  The out-lists of a round's
// kBlock pairs are laid end to end over the workgroup (a hub's lists do not
// hold one lane), and the sources of the frontier pairs that a wave's edges
// meet are laid end to end over the wave.  Counters, appends and records are
// those of k_expand for the level.
__global__ void __launch_bounds__(kBlock) k_pull(WinArgs A, uint32_t L, uint32_t n, uint32_t ell,
                                                 const uint64_t *skey, const uint32_t *fidx,
                                                 const uint32_t *fend, const uint64_t *fptr,
                                                 const uint32_t *fadj) {
    __shared__ ExpandShared X;
    __shared__ uint64_t s_ex[kBlock + 1];  // starts of the round's out-lists laid end to end
    __shared__ uint64_t s_e0[kBlock];      // their offsets in fadj
    __shared__ uint64_t s_wsum[kBlock / 64];
    __shared__ uint32_t s_flags;
    __shared__ unsigned long long s_size;
    if (threadIdx.x == 0) {
        X.F.n = X.R.n = X.nheavy = 0;
        s_flags = __hip_atomic_load(&A.ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        s_size = A.ctl->size[16 * (L % 3)];
        if (blockIdx.x == 0) {
            A.ctl->size[16 * ((L + 2) % 3)] = 0;  // counter of level L + 2
            A.ctl->hsize[16 * ((L + 1) % 2)] = 0;  // long lists of level L + 1
        }
    }
    __syncthreads();
    uint32_t scans = 0, hashed = 0, visits = 0;
    if (!s_flags && s_size) {
        uint64_t *nkey = A.fkey[(L + 1) & 1], *nlive = A.flive[(L + 1) & 1];
        unsigned long long *next_count = &A.ctl->size[16 * ((L + 1) % 3)];
        const uint32_t tid = threadIdx.x, lane = lane_id(), wave = tid >> 6;
        const uint64_t nv = (uint64_t)n * ell;
        for (uint64_t c = (uint64_t)blockIdx.x * kChunk; c < nv;
             c += (uint64_t)gridDim.x * kChunk) {
            const uint64_t end = c + kChunk < nv ? c + kChunk : nv;
            for (uint64_t tb = c; tb < end; tb += kBlock) {
                const uint64_t v = tb + tid;
                uint64_t e0 = 0, cnt = 0;
                if (v < end) {
                    // a pair that every claim of this window turns away (its
                    // count at the window start is k already, or it neither
                    // expands nor records) pulls nothing: that count and
                    // `want` do not change within a window
                    const uint64_t q = (v / ell) * kPairStride + v % ell;
                    const uint64_t w = load_relaxed(A.prec + 2 * q);
                    const bool idle = prior_count(w, A.win) >= A.k ||
                                      (!A.prec[2 * q + 1] && !wants_record(A, (uint32_t)(v / ell)));
                    if (!idle) {
                        e0 = fptr[q];
                        cnt = fptr[q + 1] - e0;
                    }
                }
                uint64_t incl = cnt;  // inclusive prefix over the wave
                for (uint32_t off = 1; off < 64; off <<= 1) {
                    const uint64_t y = shfl_up_u64(incl, off);
                    if (lane >= off) incl += y;
                }
                if (lane == 63u) s_wsum[wave] = incl;
                s_e0[tid] = e0;
                __syncthreads();
                uint64_t before = 0, T = 0;
                for (uint32_t w = 0; w < kBlock / 64; ++w) {
                    before += w < wave ? s_wsum[w] : 0;
                    T += s_wsum[w];
                }
                s_ex[tid] = before + incl - cnt;
                if (tid == 0) s_ex[kBlock] = T;
                __syncthreads();
                for (uint64_t b0 = 0; b0 < T; b0 += kBlock) {  // uniform over the workgroup
                    const uint64_t pos = b0 + tid;
                    uint64_t s0 = 0, S = 0;
                    uint32_t u = 0, i = 0;
                    if (pos < T) {
                        uint32_t lo = 0, hi = kBlock;  // s_ex[lo] <= pos < s_ex[hi]
                        while (hi - lo > 1) {
                            const uint32_t mid = (lo + hi) >> 1;
                            if (s_ex[mid] <= pos) lo = mid;
                            else hi = mid;
                        }
                        const uint64_t vv = tb + lo;
                        u = (uint32_t)(vv / ell);
                        i = (uint32_t)(vv % ell);
                        const uint64_t p =
                            (uint64_t)fadj[s_e0[lo] + (pos - s_ex[lo])] * kPairStride + i;
                        const uint32_t at = fidx[p];
                        if (at) {
                            s0 = at - 1;
                            S = fend[p] - s0;
                        }
                    }
                    uint64_t sincl = S;  // the wave's sources, 64 at a time
                    for (uint32_t off = 1; off < 64; off <<= 1) {
                        const uint64_t y = shfl_up_u64(sincl, off);
                        if (lane >= off) sincl += y;
                    }
                    const uint64_t ST = shfl_u64(sincl, 63);
                    for (uint64_t sb = 0; sb < ST; sb += 64) {
                        const uint64_t jj = sb + lane;
                        uint32_t r = 0;  // lanes whose sources end at or before position jj
                        for (uint32_t step = 32; step > 0; step >>= 1) {
                            const uint64_t y = shfl_u64(sincl, r + step - 1);
                            if (y <= jj) r += step;
                        }
                        const uint32_t rr = r & 63u;
                        const uint64_t first = shfl_u64(sincl, rr) - shfl_u64(S, rr);
                        const uint64_t rs0 = shfl_u64(s0, rr);
                        const uint32_t ru = __shfl(u, (int)rr), ri = __shfl(i, (int)rr);
                        if (jj < ST)
                            visit_edge(A, ru, ri, (uint32_t)skey[rs0 + (jj - first)], nkey, nlive,
                                       next_count, X, scans, hashed, visits);
                    }
                }
                __syncthreads();  // s_ex, s_e0 and s_wsum are refilled next round
            }
            stage_flush2(X.F, nkey, nlive, A.front_cap, next_count, X.R, A.rec, A.rec_cap,
                         &A.ctl->records, &A.ctl->flags);
        }
    }
    block_add3(X.R.buf, &A.ctl->scans, scans, &A.ctl->hinserts, hashed, &A.ctl->visits, visits);
}

// Pair records at the start of a build: the initial state word and the
// pair's live-list word.
__global__ void k_pair_init(const uint64_t *live, uint64_t npairs, uint64_t *prec) {
    for (uint64_t q = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; q < npairs;
         q += (uint64_t)gridDim.x * blockDim.x) {
        prec[2 * q] = kWordInit;
        prec[2 * q + 1] = live[q];
    }
}

constexpr uint64_t kTailRecords = 1ull << 20;  // record room the host adds before the tails

// ------------------------------------- tails in many independent workgroups
// The last levels of a window, once its frontier is small, in many
// workgroups that never wait for each other: the frontier is split between
// them and each runs its own level-synchronous search over its part, its
// frontier in LDS, until that part dies out.  A window's result does not
// depend on the order of its visits (pruning reads only counts from before
// the window, and every (pair, source) visit is claimed exactly once, on
// the device), so workgroups at different levels stay exact.  A workgroup
// hands its frontier back to global memory (appended to the next level's
// array, which the host then continues level by level) when its next level
// could outgrow its LDS frontier or the visits reserved by all tails could
// outgrow the room for records or hash-set inserts that the host gave.
// There is no inter-workgroup barrier: every workgroup leaves its loop on
// its own.
constexpr uint32_t kTailsCap = 512;    // frontier entries per workgroup (LDS)
constexpr int kTailsBlock = 256;
constexpr uint32_t kTailsGrid = 1024;  // workgroups that fit on the device at once (4 per CU)
constexpr uint32_t kTailsPer = 16;     // entries per workgroup at the start, or more
constexpr uint64_t kTailsMax = (uint64_t)kTailsGrid * 192;  // frontiers handed to the tails

struct TailsShared {
    uint64_t key[2][kTailsCap];
    uint64_t live[2][kTailsCap];
    uint32_t n[2];
    StageR R;
    uint32_t ex[kTailsCap + 1];  // the level's live edges laid end to end: entry starts
    uint32_t wsum[kTailsBlock / 64];
    uint32_t hashed;
    uint32_t spilled;
    unsigned long long work;
    uint32_t dump;
    unsigned long long rbase;
};

__device__ __forceinline__ void tails_visit(const WinArgs &A, TailsShared &T, uint32_t nxt,
                                            uint32_t w, uint32_t i, uint32_t src,
                                            uint32_t &scans, uint32_t &hashed, uint32_t &visits) {
    const uint32_t q = w * kPairStride + i;
    ++scans;
    const bool want = wants_record(A, w);
    uint64_t live;
    if (claim(A, q, src, want, hashed, live) == 1) {
        ++visits;
        if (live) {  // room: the level's visits were bounded by kTailsCap before it ran
            const uint32_t pos = stage_slots(&T.n[nxt]);
            T.key[nxt][pos] = ((uint64_t)q << 32) | src;
            T.live[nxt][pos] = live;
        }
        if (want) {
            const uint32_t pos = stage_slots(&T.R.n);
            if (pos < kStageR) {
                T.R.buf[pos] = ((uint64_t)w << 32) | src;
            } else {  // stage full: straight to global memory
                atomicAdd(&T.spilled, 1u);
                const uint64_t g = wave_reserve(&A.ctl->records, true);
                if (g < A.rec_cap) A.rec[g] = ((uint64_t)w << 32) | src;
                else atomicOr(&A.ctl->flags, kOvfRecords);
            }
        }
    }
}

// The frontier of level L (nin entries at fkey/flive[L & 1]) split over the
// grid; entries handed back go to level L + 1's arrays, counted in
// ctl->size[(L + 1) % 3] (zero at launch).  room: visits all tails may
// reserve in total (bounded by the free records and hash-set room).
__global__ void __launch_bounds__(kTailsBlock) k_tails(WinArgs A, uint32_t L, uint64_t nin,
                                                       unsigned long long room) {
    __shared__ TailsShared T;
    const uint32_t tid = threadIdx.x;
    const uint64_t a = nin * blockIdx.x / gridDim.x, b = nin * (blockIdx.x + 1) / gridDim.x;
    const uint32_t n0 = (uint32_t)(b - a);  // <= kTailsCap (the host sizes the grid)
    if (tid == 0) {
        T.n[0] = n0;
        T.R.n = 0;
    }
    for (uint32_t t = tid; t < n0; t += blockDim.x) {
        T.key[0][t] = A.fkey[L & 1][a + t];
        T.live[0][t] = A.flive[L & 1][a + t];
    }
    uint32_t scans = 0, visits = 0, cur = 0;
    uint64_t *okey = A.fkey[(L + 1) & 1], *olive = A.flive[(L + 1) & 1];
    unsigned long long *ocount = &A.ctl->size[16 * ((L + 1) % 3)];
    for (;;) {
        if (tid == 0) {
            T.n[cur ^ 1] = 0;
            T.hashed = 0;
            T.spilled = 0;
            T.work = 0;
            T.dump = 0;
        }
        __syncthreads();
        const uint32_t nc = T.n[cur];
        if (nc == 0) break;  // uniform: read after the barrier
        {   // the level's live in-edges bound its visits, records and inserts
            unsigned long long wk = 0;
            for (uint32_t t = tid; t < nc; t += blockDim.x) {
                const uint64_t live = T.live[cur][t];
                wk += (live & kLiveOne) ? 1u : live_count(live);
            }
            if (wk) atomicAdd(&T.work, wk);
        }
        __syncthreads();
        if (tid == 0) {
            const unsigned long long W = T.work;
            const uint32_t fl =
                __hip_atomic_load(&A.ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            if (fl || W > kTailsCap) {
                T.dump = 1;
            } else if (atomicAdd(&A.ctl->budget, W) + W > room) {
                T.dump = 1;  // the reservation stays: it only makes later tails stop sooner
            }
        }
        __syncthreads();
        if (T.dump) {  // hand the level's entries back to global memory
            if (tid == 0) T.rbase = atomicAdd(ocount, (unsigned long long)nc);
            __syncthreads();
            const unsigned long long base = T.rbase;
            if (tid == 0 && base + nc > A.front_cap) atomicOr(&A.ctl->flags, kOvfSpill);
            for (uint32_t t = tid; t < nc; t += blockDim.x) {
                if (base + t < A.front_cap) {
                    okey[base + t] = T.key[cur][t];
                    olive[base + t] = T.live[cur][t];
                }
            }
            break;
        }
        const uint32_t nxt = cur ^ 1;
        uint32_t hashed = 0;
        {   // the level's live edges (at most kTailsCap) laid end to end and
            // taken kTailsBlock at a time: thread t owns entries 2t and 2t + 1
            uint32_t c[2] = {0, 0};
            for (uint32_t h = 0; h < 2; ++h) {
                const uint32_t e = 2 * tid + h;
                if (e < nc) {
                    const uint64_t lv = T.live[cur][e];
                    c[h] = (lv & kLiveOne) ? 1u : live_count(lv);
                }
            }
            const uint32_t lane = lane_id(), wave = tid >> 6;
            uint32_t incl = c[0] + c[1];
            for (uint32_t off = 1; off < 64; off <<= 1) {
                const uint32_t y = __shfl_up(incl, off);
                if (lane >= off) incl += y;
            }
            if (lane == 63u) T.wsum[wave] = incl;
            __syncthreads();
            uint32_t before = 0, W = 0;
            for (uint32_t w = 0; w < kTailsBlock / 64; ++w) {
                before += w < wave ? T.wsum[w] : 0u;
                W += T.wsum[w];
            }
            const uint32_t start = before + incl - c[0] - c[1];
            T.ex[2 * tid] = start;
            T.ex[2 * tid + 1] = start + c[0];
            if (tid == 0) T.ex[kTailsCap] = W;
            __syncthreads();
            for (uint32_t p = tid; p < W; p += kTailsBlock) {
                uint32_t lo = 0, hi = kTailsCap;  // ex[lo] <= p < ex[hi]
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) >> 1;
                    if (T.ex[mid] <= p) lo = mid;
                    else hi = mid;
                }
                const uint64_t it = T.key[cur][lo], lv = T.live[cur][lo];
                const uint32_t w = (lv & kLiveOne) ? (uint32_t)lv
                                                   : A.lsrc[(lv >> kLiveCountBits) + (p - T.ex[lo])];
                tails_visit(A, T, nxt, w, (uint32_t)(it >> 32) % kPairStride, (uint32_t)it, scans,
                            hashed, visits);
            }
        }
        if (hashed) atomicAdd(&T.hashed, hashed);
        __syncthreads();
        // the level's staged records to global memory, one reservation
        const uint32_t mr = T.R.n < kStageR ? T.R.n : kStageR;
        if (tid == 0) {
            T.rbase = mr ? atomicAdd(&A.ctl->records, (unsigned long long)mr) : 0;
            if (mr && T.rbase + mr > A.rec_cap) atomicOr(&A.ctl->flags, kOvfRecords);
            if (T.hashed) atomicAdd(&A.ctl->hinserts, (unsigned long long)T.hashed);
        }
        __syncthreads();
        const unsigned long long rb = T.rbase;
        for (uint32_t j = tid; j < mr; j += blockDim.x)
            if (rb + j < A.rec_cap) A.rec[rb + j] = T.R.buf[j];
        __syncthreads();
        if (tid == 0) T.R.n = 0;
        cur = nxt;
    }
    block_add3((uint64_t *)T.R.buf, &A.ctl->scans, scans, &A.ctl->visits, visits, nullptr, 0);
}

// Before the tails at level L: the counter of the entries they hand back
// (level L + 1) and that of the level after it (L + 2, which the next
// expansion appends to; it still holds level L - 1's size) start at zero.
__global__ void k_tails_begin(Ctl *ctl, uint32_t L) {
    ctl->size[16 * ((L + 1) % 3)] = 0;
    ctl->size[16 * ((L + 2) % 3)] = 0;
    ctl->hsize[16 * ((L + 1) % 2)] = 0;  // the level after the tails may defer long lists
    ctl->budget = 0;
}

// Start of a window (or of its redo): clear the per-window fields and set
// the running counters to their values at the window start.
__global__ void k_ctl_begin(Ctl *ctl, unsigned long long visits, unsigned long long scans,
                            unsigned long long records) {
    ctl->size[16 * (0)] = ctl->size[16 * (1)] = ctl->size[16 * (2)] = 0;
    ctl->hsize[0] = ctl->hsize[16] = 0;
    ctl->hinserts = 0;
    ctl->flags = 0;
    ctl->visits = visits;
    ctl->scans = scans;
    ctl->records = records;
}

// ---------------------------------------------------------- 4. records

// After a window: want[v] = 1 while node v has received fewer than k ranks
// in all, summed over its 64 pairs (each pair's count undercounts at worst,
// so a node never stops recording too early); ctl->full counts the others.
// Eight lanes per node, each summing the state words of eight consecutive
// pairs.
__global__ void k_want(const uint64_t *prec, uint32_t n, uint32_t k, uint8_t *want, Ctl *ctl) {
    __shared__ uint64_t scratch[3 * (kBlock / 64)];
    uint32_t full = 0;
    const uint64_t lanes = (uint64_t)n * 8;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < ((lanes + 63) & ~63ull);
         t += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t c = 0;
        // a node that stopped recording never records again: skip its words
        const bool open = t < lanes && want[t >> 3];
        if (open) {
            const uint64_t *wv = prec + t * 16;
            for (int j = 0; j < 8; ++j) c += prior_count(wv[2 * j], 0xFEu);
        }
        c += __shfl_xor(c, 1);
        c += __shfl_xor(c, 2);
        c += __shfl_xor(c, 4);
        if (t < lanes && (t & 7) == 0) {
            const bool w = open && c < k;
            if (open) want[t >> 3] = w;
            full += !w;
        }
    }
    block_add3(scratch, &ctl->full, full, nullptr, 0, nullptr, 0);
}

// Segment [start[v], end[v]) of node v in the records sorted by node.
__global__ void k_bounds(const uint64_t *seg, uint64_t nrec, uint64_t *start, uint64_t *end) {
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < nrec;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)(seg[t] >> 32);
        if (t == 0 || (uint32_t)(seg[t - 1] >> 32) != v) start[v] = t;
        if (t + 1 == nrec || (uint32_t)(seg[t + 1] >> 32) != v) end[v] = t + 1;
    }
}

// ------------------------------------------------------------- 5. merge

// LDS written by some lanes of a wave, then read by others of the same wave.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Bitonic sort of 64 R keys held in registers by one wave: key r of lane l
// is element r * 64 + l.  Strides below 64 pair lanes (shuffles), larger
// strides pair the registers of one lane.  Ascending on return.
template <int R>
__device__ __forceinline__ void wave_bitonic(uint64_t (&x)[R], uint32_t lane) {
#pragma unroll
    for (uint32_t size = 2; size <= 64u * R; size <<= 1) {
#pragma unroll
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            if (stride >= 64) {
                const uint32_t rs = stride / 64;
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    if ((r & rs) == 0) {
                        const bool up = ((r * 64u + lane) & size) == 0;
                        const uint64_t a = x[r], b = x[r | rs];
                        const bool swap = (a > b) == up;
                        x[r] = swap ? b : a;
                        x[r | rs] = swap ? a : b;
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < R; ++r) {
                    const uint64_t o = shfl_xor_u64(x[r], (int)stride);
                    const bool up = ((r * 64u + lane) & size) == 0;
                    const bool low = (lane & stride) == 0;
                    x[r] = (low == up) ? (x[r] < o ? x[r] : o) : (x[r] < o ? o : x[r]);
                }
            }
        }
    }
}

// The k smallest of the S <= 64 R ranks of segment `a` (records sorted by
// node), written ascending to `row` with kNone padding.
template <int R>
__device__ __forceinline__ void select_regs(const uint64_t *seg, uint64_t a, uint64_t S,
                                            uint32_t k, uint64_t seed, const uint64_t *table,
                                            uint64_t *row, uint32_t lane) {
    uint64_t x[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint64_t j = r * 64u + lane;
        x[r] = j < S ? rank_of(seed, table, (uint32_t)seg[a + j]) : kNone;
    }
    wave_bitonic<R>(x, lane);
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t j = r * 64u + lane;
        if (j < k) row[j] = x[r];  // positions at or past S hold kNone
    }
    for (uint32_t j = 64u * R + lane; j < k; j += 64) row[j] = kNone;  // k above 64 R
}

// One wave per node: keep the k smallest ranks of the node's records
// seg[start[v], end[v]).  Up to 512 records are sorted in registers; a
// longer segment goes through LDS in chunks of 256, keeping the 256
// smallest so far (k <= 256).
__global__ void __launch_bounds__(256) k_select(const uint64_t *start, const uint64_t *end,
                                                const uint64_t *seg, uint32_t n, uint32_t k,
                                                uint64_t seed, const uint64_t *table,
                                                uint64_t *ranks, uint32_t *size) {
    __shared__ uint64_t lbuf[4][512];
    const uint32_t lane = lane_id(), wave = threadIdx.x / 64;
    uint64_t *buf = lbuf[wave];
    const uint64_t waves = (uint64_t)gridDim.x * 4;
    for (uint64_t v = blockIdx.x * 4ull + wave; v < n; v += waves) {
        const uint64_t a = start[v], b = end[v];
        const uint64_t S = b - a;
        uint64_t *row = ranks + v * k;
        if (S <= 64) select_regs<1>(seg, a, S, k, seed, table, row, lane);
        else if (S <= 128) select_regs<2>(seg, a, S, k, seed, table, row, lane);
        else if (S <= 256) select_regs<4>(seg, a, S, k, seed, table, row, lane);
        else if (S <= 512) select_regs<8>(seg, a, S, k, seed, table, row, lane);
        else {
            // buf[0, 256): the 256 smallest so far, ascending; buf[256, 256 + nc):
            // candidates since, the ranks below the k-th smallest so far (no
            // other can be among the k smallest).  The candidates are merged
            // in by one sort of the 512 slots once they may outgrow their room.
            for (uint32_t j = lane; j < 512; j += 64) buf[j] = kNone;
            wave_lds_sync();
            uint64_t tau = kNone;
            uint32_t nc = 0;
            for (uint64_t c = a; c < b; c += 64) {
                const uint64_t x =
                    c + lane < b ? rank_of(seed, table, (uint32_t)seg[c + lane]) : kNone;
                const bool cand = x < tau;
                const unsigned long long m = __ballot(cand);
                if (cand) buf[256 + nc + __popcll(m & ((1ull << lane) - 1ull))] = x;
                nc += (uint32_t)__popcll(m);
                if (nc > 192 || (c + 64 >= b && nc > 0)) {
                    wave_lds_sync();
                    uint64_t y[8];
#pragma unroll
                    for (int r = 0; r < 8; ++r) y[r] = buf[r * 64 + lane];
                    wave_bitonic<8>(y, lane);
#pragma unroll
                    for (int r = 0; r < 4; ++r) buf[r * 64 + lane] = y[r];
#pragma unroll
                    for (int r = 4; r < 8; ++r) buf[r * 64 + lane] = kNone;
                    wave_lds_sync();
                    tau = buf[k - 1];
                    nc = 0;
                }
            }
            for (uint32_t j = lane; j < k; j += 64) row[j] = buf[j];
            wave_lds_sync();  // buf is refilled for the wave's next node
        }
        if (lane == 0) size[v] = (uint32_t)(S < k ? S : k);
    }
}

// Bucket 0 holds about k/2 sources per instance (ranks of at most b0 bits,
// a fraction 2^(b0 - bits) of all, for ranks spread over `bits` bits: 64
// for hashed ranks, the bit length of n l for permutation positions); NB
// buckets in all.
void choose_buckets(uint32_t n, uint32_t k, uint32_t bits, uint32_t &NB, uint32_t &b0) {
    const double x = 2.0 * n / (double)k;  // 1 / (bucket-0 fraction)
    uint32_t lg = 0;
    while (lg + 1 < bits && (double)(1ull << lg) < x) ++lg;
    b0 = bits - lg;
    NB = 1 + lg;
}

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Launch shapes of the search (see skim_build_params).
struct Shapes {
    uint64_t small_frontier = 65536;
    int small_batch = 8;
    int large_batch = 3;
    uint64_t thread_frontier = (uint64_t)kBlock * 2048;
    double heavy = 4.0;
    uint64_t sort_frontier = 0;  // 0: never sort
    uint32_t window_span = 2;    // buckets per window after a light one
    uint32_t first_span = kFirstSpan;  // buckets of the first window
    uint64_t pull_frontier = 0;  // levels of at least this many entries by pull; 0: never
};

std::mutex g_shapes_mu;
skim_build_params g_params{65536, 8, 3, kBlock * 2048, 4, 0, 2, kFirstSpan, 0};

Shapes current_shapes() {
    std::lock_guard<std::mutex> lk(g_shapes_mu);
    Shapes sh;
    sh.small_frontier = g_params.small_frontier;
    sh.small_batch = (int)g_params.small_batch;
    sh.large_batch = (int)g_params.large_batch;
    sh.thread_frontier = g_params.thread_frontier;
    sh.heavy = (double)g_params.heavy_visits;
    sh.sort_frontier = g_params.sort_frontier;
    sh.window_span = g_params.window_span;
    sh.first_span = g_params.first_span;
    sh.pull_frontier = g_params.pull_frontier;
    return sh;
}

struct Capacity {
    uint64_t rec, front, hash;
    uint64_t hash_min;    // least hash-set size of a window (raised after an overflow)
    uint32_t first_span;  // buckets of window 0 (1 after an optimistic one overflowed)
};

}  // namespace

// Where the ranks come from: hashed r(v, i) (table NULL), or a table of
// structured permutation positions 1 .. n l, of which only those up to
// `limit` = min(k, l) n can enter a sketch.
struct RankSource {
    const uint64_t *table = nullptr;
    uint64_t limit = ~0ull;
    uint32_t bits = 64;    // bit length of the largest rank
    uint64_t perm_d = 0;   // n l for positions (the permutation estimator), 0 if hashed
};

// One attempt at the windows and the merge; throws Retry when a buffer was
// too small (the caller's outputs are written only by the merge).
static void run_windows(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed,
                        const RankSource &rs, const PairLists &live, const LiveLists *fwd,
                        const uint32_t *sources, const unsigned long long *wb, uint32_t W,
                        const Capacity &cap, const Shapes &sh, uint64_t *ranks_out,
                        uint32_t *size_out, uint64_t *work, Arena &A) {
    hipStream_t s = A.stream();
    const uint32_t n = g->n;
    const uint64_t npairs = (uint64_t)n * kPairStride;
    Ctl *ctl = A.alloc<Ctl>(1);
    fill_u64((uint64_t *)ctl, 0, sizeof(Ctl) / 8, s);
    uint64_t *prec = A.alloc<uint64_t>(2 * npairs);
    // hub lists for k_expand_heavy, only when some list is long enough
    uint64_t *heavy =
        live.maxlen > kSplitLive ? A.alloc<uint64_t>(2 * (uint64_t)kHeavyMax) : nullptr;
    k_pair_init<<<grid_for(npairs, kBlock, 65536), kBlock, 0, s>>>(live.live, npairs, prec);
    SKIM_LAUNCH_CHECK();
    uint8_t *want = A.alloc<uint8_t>((uint64_t)n + 4);
    fill_u32((uint32_t *)want, 0x01010101u, (n + 3) / 4, s);  // no records yet: all record
    uint64_t rec_cap = cap.rec, front_cap = cap.front;
    uint64_t *rec = A.alloc<uint64_t>(rec_cap);
    uint64_t *fkey[2] = {A.alloc<uint64_t>(front_cap), A.alloc<uint64_t>(front_cap)};
    uint64_t *flive[2] = {A.alloc<uint64_t>(front_cap), A.alloc<uint64_t>(front_cap)};
    // The hash set is allocated once for up to 2^29 entries (4 GiB) and only
    // reallocated by windows that need more.
    uint64_t hset_size = std::min<uint64_t>(cap.hash, 1ull << 29);
    uint64_t *hset = A.alloc<uint64_t>(hset_size);
    bool hset_clean = false;  // every slot kNone or a tagged key
    const bool tagged = npairs <= (1ull << 28);  // pair ids leave room for a window tag
    uint64_t *snap = nullptr;  // pair records at the start of a guarded window
    uint64_t *sort_key = nullptr, *sort_live = nullptr, sort_cap = 0;  // sort_frontier
    uint8_t *sort_tmp = nullptr;
    size_t sort_tmp_bytes = 0;
    uint64_t *pull_key = nullptr, pull_cap = 0;  // levels by pull (fwd given)
    uint32_t *fidx = nullptr, *fend = nullptr;
    uint8_t *pull_tmp = nullptr;
    size_t pull_tmp_bytes = 0;
    int pair_bits = 1;
    while (pair_bits < 32 && (1ull << pair_bits) < npairs) ++pair_bits;
    uint32_t levels_run = 0;
    uint64_t windows_done = 0, prev_hash = 0, prev_nw = 0;
    const bool debug = std::getenv("SKIM_DEBUG") != nullptr;
    const bool debug2 = debug && std::atoi(std::getenv("SKIM_DEBUG")) > 1;
    const auto t_start = std::chrono::steady_clock::now();
    auto elapsed_ms = [&]() {
        return std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t_start)
            .count();
    };
    // Buffers grow between levels when the next levels could outrun them
    // (a level's new visits are assumed to be at most kGrow times its
    // frontier; a level that breaks this overflows and the windows are
    // redone with more room).
    constexpr uint64_t kGrow = 3;
    const uint64_t kSmall = sh.small_frontier;  // frontiers handled in blind batches of levels
    auto grow_u64 = [&](uint64_t *&buf, uint64_t &capacity, uint64_t keep, uint64_t need) {
        if (need <= capacity && buf) return;
        uint64_t nc = std::max<uint64_t>(capacity, 1024);
        while (nc < need) nc *= 2;
        uint64_t *nb = A.alloc<uint64_t>(nc);
        if (keep) SKIM_HIP(hipMemcpyAsync(nb, buf, keep * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        if (buf) A.release(buf);
        buf = nb;
        capacity = nc;
    };
    Ctl h;
    // Window w covers buckets [bb, be): bucket 0 alone; then, unless that
    // was heavy, as many buckets as keep the arrivals per pair below k; then
    // sh.window_span buckets at a time, or one (twofold) after a window whose
    // visited pairs took more than kHeavy visits each on average (large
    // reach sets: a smaller step keeps the visits past k in check).
    const double kHeavy = sh.heavy;
    uint64_t prev_visits = 0;
    uint32_t span = 1, span_next = 2;
    bool merged = cap.first_span > 1;  // the current window gathers arrivals by design
    for (uint32_t w = 0, bb = 0; bb < W && w < 255; ++w, bb += span) {
        span = std::min<uint32_t>(w == 0 ? cap.first_span : span_next, W - bb);
        if (bb + span == W && span > 1) --span;  // the last bucket (half the ranks) alone
        const uint64_t ws = wb[bb], we = wb[bb + span];
        const uint32_t htag = tagged ? w + 1 : 0;
        const uint32_t last = bb + span >= W;
        read_back(&h, ctl, sizeof h, s);
        if (h.flags) throw Retry{h.flags};
        if (h.full >= n) break;  // every sketch holds k ranks: later ranks cannot enter
        if (ws == we) continue;
        const uint64_t nw = we - ws;
        // A pair is often visited by several sources of one window; every
        // visit after the first goes through the hash set.  Hashed visits
        // per source fall from window to window (pruning takes hold), so the
        // previous window's rate bounds this one's; window 0 assumes 16.
        const double pred = w == 0 || prev_nw == 0
                                ? 16.0 * (double)nw
                                : 1.5 * (double)prev_hash * (double)nw / (double)prev_nw + (double)nw;
        uint64_t hsize = std::min<uint64_t>(
            cap.hash, next_pow2(std::max<uint64_t>(cap.hash_min, (uint64_t)(2.5 * pred))));
        // The first window and windows after a heavy one can be redone: an
        // overflow there costs one redo of the window with more room instead
        // of a restart of all windows.  The first window restores the pair
        // records from scratch, the others from a copy taken here.
        const bool guard = w == 0 || span_next == 1;
        if (guard && w > 0) {
            if (!snap) snap = A.alloc<uint64_t>(2 * npairs);
            SKIM_HIP(hipMemcpyAsync(snap, prec, 2 * npairs * sizeof(uint64_t),
                                    hipMemcpyDeviceToDevice, s));
        }
        const Ctl base = h;  // counters at the window start
        for (int redo = 0;; ++redo) {
            uint32_t logcap = 0;
            while ((1ull << logcap) < hsize) ++logcap;
            if (hsize > hset_size) {
                if (hset) A.release(hset);
                hset = A.alloc<uint64_t>(hsize);
                hset_size = hsize;
                hset_clean = false;
            }
            // tagged keys of earlier windows are free slots: clear only a
            // set that never was (or a window being redone)
            if (!tagged) {
                fill_u64(hset, kNone, hsize, s);
            } else if (!hset_clean || redo > 0) {
                fill_u64(hset, kNone, hset_size, s);
                hset_clean = true;
            }
            k_ctl_begin<<<1, 1, 0, s>>>(ctl, base.visits, base.scans, base.records);
            SKIM_LAUNCH_CHECK();
            auto args = [&]() {
                return WinArgs{prec,    live.adj, hset,
                               logcap,  htag,     w,        k,
                               last,    want,     rec,      rec_cap,
                               {fkey[0], fkey[1]}, {flive[0], flive[1]}, front_cap,
                               ctl,     heavy};
            };
            {
                const WinArgs WA = args();
                LaunchTimer t("k_seed_window", s);
                k_seed_window<<<grid_for(nw, kChunk, 4096), kBlock, 0, s>>>(WA, sources, ws, we);
            }
            SKIM_LAUNCH_CHECK();
            uint32_t L = 0;
            uint32_t overflow = 0;
            uint64_t f_prev = 0;
            bool tails_ok = true;  // false right after the tails handed entries back
            for (;;) {
                read_back(&h, ctl, sizeof h, s);
                if (h.flags) {
                    overflow = h.flags;
                    if (debug)
                        std::fprintf(stderr, "skim window %u overflow %u: hashed %llu table %llu\n",
                                     w, h.flags, h.hinserts, (unsigned long long)hsize);
                    break;
                }
                const uint64_t f = h.size[16 * (L % 3)];
                if (f == 0) break;  // empty frontier: window done
                if (debug2)
                    std::fprintf(stderr, "skim window %u level %u: frontier %llu hashed %llu\n", w,
                                 L, (unsigned long long)f, h.hinserts);
                // Room for the next level: the frontier and the records are grown
                // to kGrow times the frontier, the hash set (rehashed) once it is
                // 40% full.  A level that still overflows is redone with the
                // window (guarded windows) or with all windows.
                {
                    uint64_t c[4] = {front_cap, front_cap, front_cap, front_cap};
                    grow_u64(fkey[L & 1], c[0], f, kGrow * f);
                    grow_u64(flive[L & 1], c[1], f, kGrow * f);
                    grow_u64(fkey[(L + 1) & 1], c[2], 0, kGrow * f);
                    grow_u64(flive[(L + 1) & 1], c[3], 0, kGrow * f);
                    front_cap = std::min(std::min(c[0], c[1]), std::min(c[2], c[3]));
                }
                grow_u64(rec, rec_cap, h.records, h.records + kGrow * f);
                if (5 * h.hinserts > 2 * hsize) {
                    const uint64_t ns = 2 * hsize;
                    uint32_t nlog = 0;
                    while ((1ull << nlog) < ns) ++nlog;
                    uint64_t *nt = A.alloc<uint64_t>(ns);
                    fill_u64(nt, kNone, ns, s);
                    k_rehash<<<grid_for(hsize, kBlock, 65536), kBlock, 0, s>>>(hset, hsize, nt, nlog,
                                                                               htag, &ctl->flags);
                    SKIM_LAUNCH_CHECK();
                    A.release(hset);
                    hset = nt;  // cleared, then only this window's keys
                    hset_size = hsize = ns;
                    logcap = nlog;
                    if (debug)
                        std::fprintf(stderr, "skim window %u: hash set grown to %llu\n", w,
                                     (unsigned long long)ns);
                }
                const bool after_tails = !tails_ok;
                if (fwd && sh.pull_frontier && f >= sh.pull_frontier && f < 0xFFFFFFFFull) {
                    // this level by pull: the frontier sorted by pair and
                    // indexed over pairs, then every pair reads its out-list
                    grow_u64(pull_key, pull_cap, 0, f);
                    size_t tb = 0;
                    SKIM_HIP(rocprim::radix_sort_keys(nullptr, tb, fkey[L & 1], pull_key, (size_t)f,
                                                      32, 32 + pair_bits, s));
                    if (tb > pull_tmp_bytes) {
                        if (pull_tmp) A.release(pull_tmp);
                        pull_tmp = A.alloc<uint8_t>(tb);
                        pull_tmp_bytes = tb;
                    }
                    SKIM_HIP(rocprim::radix_sort_keys(pull_tmp, tb, fkey[L & 1], pull_key, (size_t)f,
                                                      32, 32 + pair_bits, s));
                    if (!fidx) {
                        fidx = A.alloc<uint32_t>(npairs);
                        fend = A.alloc<uint32_t>(npairs);
                    }
                    fill_u32(fidx, 0, npairs, s);
                    k_pull_index<<<grid_for(f, kBlock, 65536), kBlock, 0, s>>>(pull_key, f, fidx,
                                                                               fend);
                    SKIM_LAUNCH_CHECK();
                    const WinArgs WA = args();
                    {
                        LaunchTimer t("k_pull", s);
                        k_pull<<<grid_for((uint64_t)n * ell, kChunk, 2048), kBlock, 0, s>>>(
                            WA, L, n, ell, pull_key, fidx, fend, fwd->ptr, fwd->adj);
                    }
                    SKIM_LAUNCH_CHECK();
                    ++L;
                    tails_ok = true;
                    f_prev = f;
                    continue;
                }
                if (f <= kTailsMax && tails_ok) {
                    // the rest of the window in independent workgroups (about
                    // kTailsPer entries each, as many as fit on the device at
                    // once), with room for the records of many levels; what
                    // they hand back continues here as level L + 1
                    const uint32_t G = (uint32_t)std::min<uint64_t>(
                        kTailsGrid, std::max<uint64_t>(1, (f + kTailsPer - 1) / kTailsPer));
                    const uint64_t per = (f + G - 1) / G;
                    if (per <= kTailsCap) {
                        grow_u64(rec, rec_cap, h.records,
                                 h.records + std::max<uint64_t>(kTailRecords, 4 * f));
                        {
                            uint64_t c[2] = {front_cap, front_cap};
                            grow_u64(fkey[(L + 1) & 1], c[0], 0, f);
                            grow_u64(flive[(L + 1) & 1], c[1], 0, f);
                            front_cap = std::min(front_cap, std::min(c[0], c[1]));
                        }
                        const uint64_t hroom = 2 * hsize / 5 > h.hinserts
                                                   ? 2 * hsize / 5 - h.hinserts : 0;
                        const uint64_t room = std::min<uint64_t>(rec_cap - h.records, hroom);
                        k_tails_begin<<<1, 1, 0, s>>>(ctl, L);
                        SKIM_LAUNCH_CHECK();
                        const WinArgs WA = args();
                        LaunchTimer t("k_tails", s);
                        k_tails<<<G, kTailsBlock, 0, s>>>(WA, L, f, room);
                        SKIM_LAUNCH_CHECK();
                        ++L;
                        tails_ok = false;  // at least one level by k_expand before the next
                        f_prev = 0;
                        continue;
                    }
                }
                tails_ok = true;
                // what the tails handed back grows past their LDS: one level
                // here, then back to the tails; a frontier a little above
                // what the tails take goes two levels at a time, so that it
                // reaches them without a long blind batch
                int batch = after_tails            ? 1
                            : f <= 4 * kTailsMax   ? 2
                            : f > kSmall           ? sh.large_batch
                                                   : sh.small_batch;
                if (sh.sort_frontier && f > sh.sort_frontier) {
                    // the frontier in pair order: live-list bounds and entries
                    // are then read nearly sequentially
                    uint64_t sc0 = sort_cap, sc1 = sort_cap;
                    grow_u64(sort_key, sc0, 0, front_cap);
                    grow_u64(sort_live, sc1, 0, front_cap);
                    size_t tb = 0;
                    SKIM_HIP(rocprim::radix_sort_pairs(nullptr, tb, fkey[L & 1], sort_key,
                                                       flive[L & 1], sort_live, (size_t)f, 32,
                                                       32 + pair_bits, s));
                    if (tb > sort_tmp_bytes) {
                        if (sort_tmp) A.release(sort_tmp);
                        sort_tmp = A.alloc<uint8_t>(tb);
                        sort_tmp_bytes = tb;
                    }
                    SKIM_HIP(rocprim::radix_sort_pairs(sort_tmp, tb, fkey[L & 1], sort_key,
                                                       flive[L & 1], sort_live, (size_t)f, 32,
                                                       32 + pair_bits, s));
                    std::swap(fkey[L & 1], sort_key);  // capacities >= front_cap
                    std::swap(flive[L & 1], sort_live);
                    sort_cap = front_cap;
                    batch = 1;
                }
                // room for 64-fold growth at a window's first level and after a
                // batch over which the frontier grew more than fourfold
                const bool growing = f_prev == 0 || f > 4 * f_prev;
                f_prev = f;
                // Small frontiers go in batches of 8 levels (a level that finds an
                // empty frontier does nothing) on a grid sized to the frontier,
                // or with room for 64-fold growth while it grows fast; large
                // ones in batches of 3.
                const WinArgs WA = args();
                const uint32_t chunk = f <= sh.thread_frontier ? kBlock : kChunk;
                for (int j = 0; j < batch; ++j, ++L) {
                    const unsigned grid =
                        f > kSmall ? (j == 0 ? grid_for(f, chunk, 2048) : 2048)
                                   : grid_for((growing ? 64 : 1) * f, chunk, 2048);
                    {
                        LaunchTimer t("k_expand", s);
                        k_expand<<<grid, kBlock, 0, s>>>(WA, L,
                                                         f > kSmall && j > 0 ? kChunk : chunk);
                    }
                    SKIM_LAUNCH_CHECK();
                    if (heavy) {
                        LaunchTimer t("k_expand_heavy", s);
                        k_expand_heavy<<<2048, kBlock, 0, s>>>(WA, L);
                        SKIM_LAUNCH_CHECK();
                    }
                }
            }
            if (!overflow) {
                levels_run = L;
                break;
            }
            // An optimistic wide first window that overflows is given up:
            // the build restarts with bucket 0 alone and the measured merge.
            if (w == 0 && span > 1) throw Retry{overflow | kOvfFirst};
            if (!guard || redo >= 6) throw Retry{overflow};
            // redo the window with more room
            if (overflow & kOvfHash) hsize = std::max(16 * hsize, next_pow2(4 * h.hinserts));
            if (overflow & kOvfSpill) {
                const uint64_t nc = 2 * front_cap;
                uint64_t c[4] = {front_cap, front_cap, front_cap, front_cap};
                grow_u64(fkey[0], c[0], 0, nc);
                grow_u64(fkey[1], c[1], 0, nc);
                grow_u64(flive[0], c[2], 0, nc);
                grow_u64(flive[1], c[3], 0, nc);
                front_cap = std::min(std::min(c[0], c[1]), std::min(c[2], c[3]));
            }
            if (overflow & kOvfRecords) grow_u64(rec, rec_cap, base.records, 2 * rec_cap);
            if (w == 0) {
                k_pair_init<<<grid_for(npairs, kBlock, 65536), kBlock, 0, s>>>(live.live, npairs,
                                                                              prec);
                SKIM_LAUNCH_CHECK();
            } else {
                SKIM_HIP(hipMemcpyAsync(prec, snap, 2 * npairs * sizeof(uint64_t),
                                        hipMemcpyDeviceToDevice, s));
            }
            if (debug) std::fprintf(stderr, "skim window %u: redo %d\n", w, redo + 1);
        }
        prev_hash = h.hinserts;
        prev_nw = nw;
        {   // the next window's step
            const uint64_t v = h.visits - prev_visits;
            const uint64_t distinct = v > h.hinserts ? v - h.hinserts : 1;
            const double per_pair = (double)v / (double)distinct;
            // heavy: more than kHeavy visits per visited pair (per two
            // buckets for the merged window, which gathers arrivals by design)
            const bool heavy =
                per_pair > kHeavy * (merged ? std::max(1.0, span / 2.0) : 1.0);
            uint32_t next = heavy ? 1u : sh.window_span;
            merged = false;
            if (w == 0 && span == 1 && !heavy) {
                // Bucket 0 gave each visited pair per_pair arrivals; with no
                // pruning yet they grow with the source count, which doubles
                // with every bucket.  While they stay below k nothing can be
                // pruned, so the buckets up to there form one window, cut so
                // that the windows after it end on the last bucket alone.
                uint32_t j = 0;
                while (j < 16 && per_pair * (double)(2u << j) <= (double)k) ++j;
                if (j > next) {
                    const uint32_t rest = W > 2 + j ? W - 2 - j : 0;
                    const uint32_t cut = rest % sh.window_span;
                    next = std::max(next, j - std::min(cut, j - 1));
                    merged = true;
                }
            }
            prev_visits = h.visits;
            span_next = next;
        }
        if (debug)
            std::fprintf(stderr, "skim window %u: sources %llu visits-so-far %llu hashed %llu "
                                 "table %llu levels %u records %llu at %.1f ms\n",
                         w, (unsigned long long)nw, h.visits, h.hinserts,
                         (unsigned long long)hsize, levels_run, h.records, elapsed_ms());
        if (!last) {
            fill_u64((uint64_t *)&ctl->full, 0, 1, s);
            k_want<<<grid_for((uint64_t)n * 8, kBlock, 8192), kBlock, 0, s>>>(prec, n, k, want,
                                                                              ctl);
            SKIM_LAUNCH_CHECK();
        }
        ++windows_done;
    }
    read_back(&h, ctl, sizeof h, s);
    if (h.flags) throw Retry{h.flags};
    const uint64_t nrec = h.records;

    // ---- 5. merge: group records by node, keep the k smallest
    A.release(prec);
    for (int j = 0; j < 2; ++j) {
        A.release(fkey[j]);
        A.release(flive[j]);
    }
    if (hset) A.release(hset);
    if (pull_key) A.release(pull_key);
    if (fidx) {
        A.release(fidx);
        A.release(fend);
    }
    uint64_t *seg = A.alloc<uint64_t>(nrec ? nrec : 1);
    uint64_t *gstart = A.alloc<uint64_t>(n), *gend = A.alloc<uint64_t>(n);
    fill_u64(gstart, 0, n, s);
    fill_u64(gend, 0, n, s);
    if (nrec) {
        // stable radix sort of the records on their node bits
        int nb = 1;
        while (nb < 32 && (1ull << nb) < n) ++nb;
        size_t tmp_bytes = 0;
        SKIM_HIP(rocprim::radix_sort_keys(nullptr, tmp_bytes, rec, seg, (size_t)nrec, 32, 32 + nb, s));
        void *tmp = A.get(tmp_bytes ? tmp_bytes : 1);
        LaunchTimer t("sort_records", s);
        SKIM_HIP(rocprim::radix_sort_keys(tmp, tmp_bytes, rec, seg, (size_t)nrec, 32, 32 + nb, s));
    }
    if (nrec) {
        k_bounds<<<grid_for(nrec, kBlock, 65536), kBlock, 0, s>>>(seg, nrec, gstart, gend);
        SKIM_LAUNCH_CHECK();
    }
    {
        LaunchTimer t("k_select", s);
        k_select<<<grid_for(n, 4, 65536), 256, 0, s>>>(gstart, gend, seg, n, k, seed, rs.table,
                                                      ranks_out, size_out);
    }
    SKIM_LAUNCH_CHECK();
    if (work) {
        work[0] = h.visits;
        work[1] = h.scans;
        work[2] = nrec;
        work[3] = windows_done;
    }
}

// Host orchestration of one sketch build.
static void build_sketches(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed,
                           uint64_t *ranks_out, uint32_t *size_out, double *est_out,
                           uint64_t *work, hipStream_t s, bool permutation = false) {
    const Shapes shapes = current_shapes();
    SKIM_REQUIRE(ell >= 1 && ell <= 64, "l must be in [1, 64]");
    SKIM_REQUIRE(k >= 2 && k <= 256, "k must be in [2, 256]");
    SKIM_REQUIRE(ranks_out && size_out, "ranks/size output is NULL");
    Arena A(s);
    const uint32_t n = g->n;
    const uint64_t m = g->m;
    uint32_t *esrc = A.alloc<uint32_t>(m ? m : 1);
    validate_graph(g, esrc, A);
    const uint64_t nsrc = (uint64_t)n * ell;  // actual pairs

    // ---- 1. live lists (reverse: in-edges of every pair)
    PairLists live = build_pair_lists(g, ell, seed, esrc, A);
    // out-lists of every pair, for levels taken by pull
    LiveLists fwd;
    if (shapes.pull_frontier) fwd = build_out_lists(g, ell, seed, esrc, A);
    A.release(esrc);
    if (live.nlive >> (64 - 1 - kLiveCountBits)) {
        set_error("%llu live edges exceed the pair records' list offsets",
                  (unsigned long long)live.nlive);
        throw Fail{SKIM_EUNSUPPORTED};
    }

    // ---- 2. rank buckets
    uint32_t W = 1, b0 = 64;  // W: number of buckets
    // ---- rank source: hashed, or structured permutation positions
    RankSource rs;
    if (permutation) {
        const uint64_t D = (uint64_t)n * ell;
        uint64_t *table = A.alloc<uint64_t>((uint64_t)n * kPairStride);
        perm_positions(n, ell, seed, table, A);
        rs.table = table;
        rs.limit = (uint64_t)n * std::min<uint32_t>(k, ell);
        rs.bits = 1;
        while (rs.bits < 64 && (1ull << rs.bits) <= D) ++rs.bits;
        rs.perm_d = D;
    }
    choose_buckets(n, k, rs.bits, W, b0);
    unsigned long long *wbuf = A.alloc<unsigned long long>(65);
    const unsigned rblocks = (unsigned)((nsrc + (uint64_t)kBlock * kRankPer - 1) /
                                        ((uint64_t)kBlock * kRankPer));
    uint32_t *bcount = A.alloc<uint32_t>((uint64_t)W * rblocks);
    k_rank_hist<<<rblocks, kBlock, 0, s>>>(n, ell, seed, rs.table, rs.limit, W, b0, bcount,
                                           rblocks);
    SKIM_LAUNCH_CHECK();
    uint64_t *boff = A.alloc<uint64_t>((uint64_t)W * rblocks + 1);
    exclusive_scan_u32(bcount, boff, (uint64_t)W * rblocks, A);
    A.release(bcount);
    k_bucket_bases<<<1, 128, 0, s>>>(boff, rblocks, W, wbuf);
    SKIM_LAUNCH_CHECK();
    unsigned long long wb[65] = {}, hw[64] = {};
    read_back(wb, wbuf, sizeof(unsigned long long) * (W + 1), s);
    for (uint32_t w = 0; w < W; ++w) hw[w] = wb[w + 1] - wb[w];
    uint32_t *sources = A.alloc<uint32_t>(nsrc);
    k_rank_scatter<<<rblocks, kBlock, 0, s>>>(n, ell, seed, rs.table, rs.limit, W, b0, boff,
                                              rblocks, sources);
    SKIM_LAUNCH_CHECK();
    A.release(boff);

    // ---- 3./4./5. windows and merge; restart with more room on overflow
    uint64_t biggest = 0, bucket_max = 0;  // largest possible window (two buckets), bucket
    for (uint32_t w = 0; w < W; ++w) {
        biggest = std::max<uint64_t>(biggest, hw[w] + (w + 1 < W ? hw[w + 1] : 0));
        bucket_max = std::max<uint64_t>(bucket_max, hw[w]);
    }
    Capacity cap{std::max<uint64_t>(1ull << 20, 3 * (uint64_t)n * k),
                 std::max<uint64_t>(1ull << 20, 3 * biggest),
                 next_pow2(std::max<uint64_t>(1ull << 16, 8 * bucket_max)), 1ull << 16,
                 shapes.first_span};
    uint32_t retry_flags = 0;
    int attempt = 0;
    for (;; ++attempt) {
        try {
            Arena B(s);
            run_windows(g, ell, k, seed, rs, live, shapes.pull_frontier ? &fwd : nullptr, sources, wb,
                        W, cap, shapes, ranks_out, size_out, work, B);
            break;
        } catch (const Retry &r) {
            retry_flags |= r.flags;
            if (std::getenv("SKIM_DEBUG"))
                std::fprintf(stderr, "skim restart %d: flags %u\n", attempt, r.flags);
            if (attempt >= 6) {
                set_error("sketch build buffers did not fit after %d attempts (flags %u)", attempt,
                          r.flags);
                throw Fail{SKIM_ENOMEM};
            }
            if (r.flags & kOvfFirst) {
                cap.first_span = 1;  // the wide first window was too much for this graph
            } else {
                if (r.flags & kOvfRecords) cap.rec *= 2;
                if (r.flags & kOvfSpill) cap.front *= 2;
                if (r.flags & kOvfHash) {
                    cap.hash_min *= 16;
                    cap.hash = std::max(cap.hash, cap.hash_min);
                }
            }
        }
    }
    if (work) {
        work[4] = (uint64_t)attempt;
        work[5] = retry_flags;
    }
    if (est_out) launch_estimates(ranks_out, size_out, n, k, ell, est_out, s, rs.perm_d);
    SKIM_HIP(hipStreamSynchronize(s));
    timing_resolve();
}

}  // namespace skim

extern "C" skim_status skim_build_sketches(const skim_graph *g, uint32_t ell, uint32_t k,
                                           uint64_t seed, uint64_t *ranks, uint32_t *size,
                                           double *est, uint64_t *work, void *stream) {
    skim::clear_error();
    try {
        skim::build_sketches(g, ell, k, seed, ranks, size, est, work, (hipStream_t)stream);
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        return f.st;
    }
}

extern "C" skim_status skim_build_sketches_perm(const skim_graph *g, uint32_t ell, uint32_t k,
                                                uint64_t seed, uint64_t *ranks, uint32_t *size,
                                                double *est, uint64_t *work, void *stream) {
    skim::clear_error();
    try {
        skim::build_sketches(g, ell, k, seed, ranks, size, est, work, (hipStream_t)stream, true);
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        return f.st;
    }
}

extern "C" skim_status skim_set_build_params(const skim_build_params *p) {
    skim::clear_error();
    skim_build_params v{65536, 8, 3, skim::kBlock * 2048, 4, 0, 2, skim::kFirstSpan};
    if (p) {
        if (p->small_frontier < 1 || p->small_batch < 1 || p->small_batch > 64 ||
            p->large_batch < 1 || p->large_batch > 64 || p->thread_frontier < 1 ||
            p->heavy_visits < 1 || p->window_span < 1 || p->window_span > 8 ||
            p->first_span < 1 || p->first_span > 16) {
            skim::set_error("build parameters out of range");
            return SKIM_EINVAL;
        }
        v = *p;
    }
    std::lock_guard<std::mutex> lk(skim::g_shapes_mu);
    skim::g_params = v;
    return SKIM_OK;
}

extern "C" void skim_get_build_params(skim_build_params *p) {
    if (!p) return;
    std::lock_guard<std::mutex> lk(skim::g_shapes_mu);
    *p = skim::g_params;
}

extern "C" skim_status skim_tune_build(const skim_graph *g, uint32_t ell, uint32_t k,
                                       uint64_t seed, uint64_t *ranks, uint32_t *size,
                                       uint32_t reps, skim_build_params *best, double *best_ms,
                                       double *start_ms, void *stream) {
    skim::clear_error();
    hipStream_t s = (hipStream_t)stream;
    if (reps < 1) reps = 1;
    skim_build_params cur;
    skim_get_build_params(&cur);
    const skim_build_params at_start = cur;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) {
        skim::set_error("hipEventCreate failed");
        if (a) (void)hipEventDestroy(a);
        return SKIM_EDEVICE;
    }
    // best of `reps` builds with the given parameters, in ms (< 0 on error)
    auto time_with = [&](const skim_build_params &p, skim_status &st) -> double {
        st = skim_set_build_params(&p);
        if (st != SKIM_OK) return -1.0;
        double t_best = 1e300;
        for (uint32_t r = 0; r < reps; ++r) {
            if (hipEventRecord(a, s) != hipSuccess) { st = SKIM_EDEVICE; return -1.0; }
            st = skim_build_sketches(g, ell, k, seed, ranks, size, nullptr, nullptr, stream);
            if (st != SKIM_OK) return -1.0;
            float ms = 0;
            if (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess ||
                hipEventElapsedTime(&ms, a, b) != hipSuccess) {
                st = SKIM_EDEVICE;
                return -1.0;
            }
            t_best = std::min(t_best, (double)ms);
        }
        return t_best;
    };
    skim_status st = skim_build_sketches(g, ell, k, seed, ranks, size, nullptr, nullptr, stream);
    double t_cur = st == SKIM_OK ? time_with(cur, st) : -1.0;
    const double t_start = t_cur;
    if (st == SKIM_OK) {
        const uint32_t sf[] = {16384, 65536, 262144};
        const uint32_t sb[] = {4, 8, 16};
        const uint32_t lb[] = {2, 3, 4};
        const uint32_t tf[] = {131072, 524288, 2097152};
        const uint32_t so[] = {0, 1u << 20, 1u << 22};
        const uint32_t fw[] = {2, 3, 4};
        const uint32_t fs[] = {3, 5, 7};
        const uint32_t pf[] = {0, 1u << 21, 1u << 23};
        for (int field = 0; field < 8 && st == SKIM_OK; ++field) {
            for (int c = 0; c < 3 && st == SKIM_OK; ++c) {
                skim_build_params p = cur;
                uint32_t *slot = field == 0   ? &p.small_frontier
                                 : field == 1 ? &p.small_batch
                                 : field == 2 ? &p.large_batch
                                 : field == 3 ? &p.thread_frontier
                                 : field == 4 ? &p.sort_frontier
                                 : field == 5 ? &p.window_span
                                 : field == 6 ? &p.first_span
                                              : &p.pull_frontier;
                const uint32_t v = field == 0   ? sf[c]
                                   : field == 1 ? sb[c]
                                   : field == 2 ? lb[c]
                                   : field == 3 ? tf[c]
                                   : field == 4 ? so[c]
                                   : field == 5 ? fw[c]
                                   : field == 6 ? fs[c]
                                                : pf[c];
                if (*slot == v) continue;
                *slot = v;
                const double t = time_with(p, st);
                if (st == SKIM_OK && t < t_cur) {
                    t_cur = t;
                    cur = p;
                }
            }
        }
    }
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    if (st != SKIM_OK) {
        const std::string msg = skim_last_error();
        (void)skim_set_build_params(&at_start);
        skim::set_error("%s", msg.c_str());
        return st;
    }
    st = skim_set_build_params(&cur);
    if (st != SKIM_OK) return st;
    if (best) *best = cur;
    if (best_ms) *best_ms = t_cur;
    if (start_ms) *start_ms = t_start;
    return SKIM_OK;
}
