// skim_internal.h -- shared device helpers and host plumbing of the gfx950
// library (kernels live in skim_build.hip, skim_query.hip, skim_greedy.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <vector>

#include "skim.h"

namespace skim {

// ---------------------------------------------------------------- randomness
// SplitMix64 (Steele, Lea, Flood 2014): output c of the stream seeded with s
// is mix(s + (c + 1) * golden), golden = odd integer nearest 2^64 / phi;
// mix is the variant-13 finaliser.  Ranks and live-edge coins of the paper
// (Section 3: a U[0,1] rank per node-instance pair; Section 1: a biased
// coin per edge and instance) are read off this stream.
constexpr uint64_t kGolden = 0x9E3779B97F4A7C15ull;
constexpr uint64_t kCoinBase = 1ull << 62;  // coins live above every rank counter
constexpr uint64_t kNone = ~0ull;
constexpr uint32_t kNoSrc = 0xFFFFFFFFu;
constexpr uint32_t kPairStride = 64;        // pair id p = 64 v + i

__device__ __forceinline__ uint64_t sm_mix(uint64_t z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__device__ __forceinline__ uint64_t sm_at(uint64_t seed, uint64_t c) {
    return sm_mix(seed + (c + 1) * kGolden);
}

// rank of pair p = 64 v + i
__device__ __forceinline__ uint64_t pair_rank(uint64_t seed, uint32_t p) { return sm_at(seed, p); }

// 64-bit mask of the instances (< ell) in which edge (u -> v) is live:
// coin of instance 2j is the high half, of 2j+1 the low half, of output
// kCoinBase + 32 (u n + v) + j; live iff coin <= thr.
__device__ __forceinline__ uint64_t live_mask(uint64_t seed, uint32_t n, uint32_t u, uint32_t v,
                                              uint32_t thr, uint32_t ell) {
    const uint64_t base = kCoinBase + ((uint64_t)u * n + v) * 32;
    uint64_t mask = 0;
    const uint32_t pairs = (ell + 1) >> 1;
    for (uint32_t j = 0; j < pairs; ++j) {
        const uint64_t h = sm_at(seed, base + j);
        const uint32_t hi = (uint32_t)(h >> 32), lo = (uint32_t)h;
        mask |= (uint64_t)(hi <= thr) << (2 * j);
        mask |= (uint64_t)(lo <= thr) << (2 * j + 1);
    }
    return ell == 64 ? mask : (mask & ((1ull << ell) - 1));
}

// Influence estimate from structured permutation positions (Section 3.1):
// the cardinality estimate 1 + (k - 1)(D - 1)/(T - 1), D = n l positions,
// divided by l; the exact count when the sketch holds fewer than k.
__device__ __forceinline__ double perm_estimate(uint64_t size, uint64_t T, uint32_t k, uint32_t ell,
                                                uint64_t D) {
    if (size < k) return (double)size / (double)ell;
    return (1.0 + ((double)(k - 1) * ((double)D - 1.0)) / (double)(T - 1)) / (double)ell;
}

// Real reading of a threshold rank: rho(T) = ((T >> 11) + 1) * 2^-53 in (0, 1].
__device__ __forceinline__ double rank_real(uint64_t T) {
    return (double)((T >> 11) + 1) * 0x1p-53;
}

// Bottom-k estimate divided by l (Section 3, eq. combinedthresh; Section 5.1).
__device__ __forceinline__ double bottomk_estimate(uint64_t size, uint64_t tau, uint32_t k,
                                                   uint32_t ell) {
    if (size < k) return (double)size / (double)ell;
    return ((double)(k - 1) / rank_real(tau)) / (double)ell;
}

// ------------------------------------------------------------- wave helpers
__device__ __forceinline__ uint32_t lane_id() { return __lane_id(); }

// Wave-aggregated append: every lane with `want` gets a distinct slot of
// `*counter`; one atomic per wave (ballot + prefix popcount).
__device__ __forceinline__ uint64_t wave_reserve(unsigned long long *counter, bool want) {
    const unsigned long long mask = __ballot(want);
    if (mask == 0) return 0;
    const int leader = __ffsll((long long)mask) - 1;
    const uint32_t lane = lane_id();
    unsigned long long base = 0;
    if ((int)lane == leader) base = atomicAdd(counter, (unsigned long long)__popcll(mask));
    const uint32_t lo = __shfl((uint32_t)base, leader);
    const uint32_t hi = __shfl((uint32_t)(base >> 32), leader);
    base = ((unsigned long long)hi << 32) | lo;
    return base + __popcll(mask & ((1ull << lane) - 1ull));
}

// Wave-aggregated counter add (one atomic per wave).
__device__ __forceinline__ void wave_add(unsigned long long *counter, uint32_t x) {
    unsigned long long s = x;
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)s, off);
        const uint32_t hi = __shfl_xor((uint32_t)(s >> 32), off);
        s += ((unsigned long long)hi << 32) | lo;
    }
    if (lane_id() == 0 && s) atomicAdd(counter, s);
}

__device__ __forceinline__ uint64_t load_relaxed(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// ------------------------------------------------------------ host plumbing
void set_error(const char *fmt, ...);
void clear_error();

// Host-side fault injection (skim_debug_inject): the next `count` device
// allocations (kFaultAlloc) or serving-loop copies and launches
// (kFaultServe) are treated as failed, or IC-model sketch builds take their
// counting path (kFaultIcRecords).  take_fault() consumes one.
enum FaultKind : uint32_t { kFaultAlloc = 1, kFaultServe = 2, kFaultIcRecords = 3 };
bool take_fault(FaultKind what);

struct Fail {
    skim_status st;
};

#define SKIM_HIP(expr)                                                                  \
    do {                                                                                \
        hipError_t e_ = (expr);                                                         \
        if (e_ != hipSuccess) {                                                         \
            ::skim::set_error("%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                              __FILE__, __LINE__);                                      \
            throw ::skim::Fail{e_ == hipErrorOutOfMemory ? SKIM_ENOMEM : SKIM_EDEVICE}; \
        }                                                                               \
    } while (0)

#define SKIM_LAUNCH_CHECK() SKIM_HIP(hipGetLastError())

#define SKIM_REQUIRE(cond, ...)           \
    do {                                  \
        if (!(cond)) {                    \
            ::skim::set_error(__VA_ARGS__); \
            throw ::skim::Fail{SKIM_EINVAL}; \
        }                                 \
    } while (0)

// Scratch of one call on one stream.  Blocks come from a per-device cache
// (hipMalloc on a miss) and return to it when the arena dies, after a
// synchronisation of the stream.  A persistent arena holds state that
// outlives a call (used by calls on any stream): its blocks go back to the
// cache after a synchronisation of the whole device.
class Arena {
  public:
    explicit Arena(hipStream_t s, bool persistent = false);
    ~Arena();
    void *get(size_t bytes);
    template <class T> T *alloc(size_t count) { return (T *)get(count * sizeof(T)); }
    void release(void *p);  // give one buffer back early (reused by this arena)
    hipStream_t stream() const { return s_; }

  private:
    struct Block {
        void *p;
        size_t bytes;
    };
    hipStream_t s_;
    bool persistent_;
    int dev_ = 0;
    std::vector<Block> bufs_, spare_;
};

// Small pinned host buffer per thread, for reading device counters.
void *pinned_scratch(size_t bytes);

// Device-side fills (no hipMemsetAsync: callers may capture these streams).
void fill_u32(uint32_t *p, uint32_t value, uint64_t count, hipStream_t s);
void fill_u64(uint64_t *p, uint64_t value, uint64_t count, hipStream_t s);

// Exclusive scan: out[0..n] with out[n] = total.  Uses arena scratch.
void exclusive_scan_u32(const uint32_t *in, uint64_t *out, uint64_t n, Arena &a);

// Copy `bytes` device -> pinned host and wait for the stream.
void read_back(void *host, const void *dev, size_t bytes, hipStream_t s);

inline unsigned grid_for(uint64_t work, unsigned block, unsigned cap = 65536) {
    uint64_t g = (work + block - 1) / block;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

// Live in- (or out-) lists of every pair p = 64 v + i, as one CSR over pair
// ids: adj[ptr[p] .. ptr[p+1]) = sources u of edges (u -> v) live in
// instance i (forward: heads v of edges (v -> w) live in i).
struct LiveLists {
    uint64_t *ptr = nullptr;  // [64 n + 1]
    uint32_t *adj = nullptr;
    uint64_t nlive = 0;
};
LiveLists build_live_lists(const skim_graph *g, uint32_t ell, uint64_t seed, const uint32_t *esrc,
                           bool forward, Arena &a, LiveLists *also_other = nullptr);

// Live-list word of a pair: 0 for no live in-edge, kLiveOne | u for the
// single source u, else begin << kLiveCountBits | count into the sources.
constexpr uint64_t kLiveOne = 1ull << 63;
constexpr uint32_t kLiveCountBits = 24;

// Live in-lists of every pair as runs of one array: the sources u of edges
// (u -> v) live in instance i, p = 64 v + i, in edge order, located by the
// pair's live-list word live[p].  Built with no atomics: per-edge prefix
// offsets and a radix sort by pair.  A list of 2^kLiveCountBits entries or
// more gives SKIM_EUNSUPPORTED.
struct PairLists {
    uint64_t *live = nullptr;  // [64 n]
    uint32_t *adj = nullptr;
    uint64_t nlive = 0;
    uint32_t maxlen = 0;  // longest live in-list (0 when none is longer than 16)
};
PairLists build_pair_lists(const skim_graph *g, uint32_t ell, uint64_t seed, const uint32_t *esrc,
                           Arena &a, Arena *out = nullptr);  // out: arena of the lists (else a)

// Live out-lists of every pair as one CSR over pair ids (as build_live_lists
// with forward set, entries in no particular order), by the chunked builder
// over the forward CSR's rows: no atomic per entry.
LiveLists build_out_lists(const skim_graph *g, uint32_t ell, uint64_t seed, const uint32_t *esrc,
                          Arena &a, Arena *out = nullptr);

// Optional per-kernel timing: while a kernel name is enabled, each launch of
// that kernel is bracketed by HIP events on its stream; durations are folded
// into the totals when the owning call resolves them after its final sync.
class LaunchTimer {
  public:
    LaunchTimer(const char *kernel, hipStream_t s);
    ~LaunchTimer();

  private:
    hipEvent_t a_ = nullptr;
    hipStream_t s_;
    const char *name_;
};
void timing_resolve();  // call after the stream has been synchronised

// Union queries (skim_query.hip): sketches, sets in CSR form, outputs.
struct QueryArgs {
    const uint64_t *ranks;
    const uint32_t *size;
    uint32_t n, k, ell;
    uint64_t q;  // sets in the batch (qoff has q + 1 entries)
    const uint64_t *qoff;
    const uint32_t *qnodes;
    double *est;
    int32_t *qstatus;
    uint32_t estimator;
    uint64_t nodes_cap = ~0ull;  // entries qnodes holds (a set reaching past them: status -3)
    uint64_t perm_d = 0;  // n l for sketches of permutation positions, 0 for hashed ranks
};
// Per-node estimates of sketches (perm_d = 0: hashed ranks; else sketches of
// permutation positions over perm_d = n l pairs), enqueued on `s`.
void launch_estimates(const uint64_t *ranks, const uint32_t *size, uint32_t n, uint32_t k,
                      uint32_t ell, double *est, hipStream_t s, uint64_t perm_d = 0);
// Structured permutation positions of every pair (table[64 v + i], 1-based;
// Section 3.1), computed on the stream of `a`.
void perm_positions(uint32_t n, uint32_t ell, uint64_t seed, uint64_t *table, Arena &a);

// Launch the persistent query kernel for q sets on `s` without waiting;
// `next` is a device work counter (zeroed here on the stream).
void launch_queries_async(const QueryArgs &Q, uint64_t q, unsigned long long *next, hipStream_t s);

// Validate a forward CSR on the device; throws Fail{SKIM_EINVAL} if invalid.
// On success writes esrc[m] (source node of every edge) when esrc != nullptr.
void validate_graph(const skim_graph *g, uint32_t *esrc, Arena &a);

}  // namespace skim
