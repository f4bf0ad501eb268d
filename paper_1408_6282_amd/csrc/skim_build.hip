// skim_build.hip -- combined bottom-k reachability sketches on gfx950.
//
// What is computed (Section 3, eq. combinedrs): X_v = the k smallest ranks
// r(u, i) over all pairs (u, i) that v reaches in live-edge instance G^(i).
// How (Section 5.2, Algorithm 2, re-organised for the GPU):
//
//  1. Live lists.  One coalesced pass over the edges evaluates every
//     instance's coin of each edge (a 64-bit instance mask per edge), and
//     the live in-lists of every node-instance pair p = 64 v + i are
//     materialised as one CSR (lptr / lsrc).  Every expansion later reads
//     only live in-edges of its own instance.
//  2. Rank windows.  All pairs are bucketed by rank into W windows: window 0
//     holds ranks below 2^(65-W), window j >= 1 the ranks in
//     [2^(64-W+j), 2^(65-W+j)).  Windows are processed in increasing order.
//  3. Pruned reverse searches, window by window.  Every source pair (u, i)
//     of the window starts a reverse search in G^(i).  A visited pair (w, i)
//     is pruned when it already received k ranks in earlier windows (the
//     paper's rule: its instance-local sketch is full); all sources of a
//     window run together, level-synchronously.  Because every pair on a
//     path to an unpruned pair reaches a subset of what it reaches, the
//     unpruned pair receives every rank of its instance in the window, so
//     the rule is exact.  Visits are deduplicated per source exactly: the
//     first visitor of a pair in the window claims its word; later visitors
//     go through a hash set keyed by (pair, source).
//  4. Records.  A visit of node v is recorded while v held fewer than k
//     ranks at the window start; windows go up in rank, so the first k
//     records (by rank) of v are its sketch.
//  5. Merge.  Records are grouped by node and each node keeps its k
//     smallest in LDS (bitonic sort), written ascending.
#include "skim_internal.h"

#include <algorithm>
#include <cstring>

namespace skim {

void launch_estimates(const uint64_t *ranks, const uint32_t *size, uint32_t n, uint32_t k,
                      uint32_t ell, double *est, hipStream_t s);

namespace {

constexpr uint32_t kOvfItems = 1u, kOvfHash = 2u, kOvfRecords = 4u;
constexpr int kBlock = 256;

// Device control block read back by the host at synchronisation points.
struct Ctl {
    unsigned long long lb[4];     // ring of level boundaries into items[]
    unsigned long long count;     // items appended in this window
    unsigned long long scans;     // live in-edges scanned (work counter)
    unsigned long long hinserts;  // hash-set insertions in this window
    unsigned long long records;   // records appended (all windows)
    unsigned long long full;      // nodes holding k records
    uint32_t flags;               // overflow bits
    uint32_t done_blocks;         // blocks finished in the current level
    uint32_t level;               // next level after a tail launch
    uint32_t pad;
};

// ------------------------------------------------------- 2. rank windows

__device__ __forceinline__ uint32_t window_of(uint64_t r, uint32_t W) {
    const int bits = r ? 64 - __clzll((long long)r) : 0;
    const int w = bits + (int)W - 65;
    return w < 0 ? 0u : (uint32_t)w;
}

constexpr int kRankPer = 8;  // pairs per thread in the bucketing kernels

__global__ void k_rank_hist(uint32_t n, uint32_t ell, uint64_t seed, uint32_t W,
                            unsigned long long *whist) {
    __shared__ uint32_t h[64];
    if (threadIdx.x < 64) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t total = (uint64_t)n * ell;
    const uint64_t base = (uint64_t)blockIdx.x * kBlock * kRankPer;
    for (int j = 0; j < kRankPer; ++j) {
        const uint64_t t = base + (uint64_t)j * kBlock + threadIdx.x;
        if (t < total) {
            const uint32_t v = (uint32_t)(t / ell), i = (uint32_t)(t % ell);
            atomicAdd(&h[window_of(pair_rank(seed, v * kPairStride + i), W)], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < W && h[threadIdx.x]) atomicAdd(&whist[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_rank_scatter(uint32_t n, uint32_t ell, uint64_t seed, uint32_t W,
                               const unsigned long long *wbase, unsigned long long *wfill,
                               uint32_t *sources) {
    __shared__ uint32_t h[64];
    __shared__ unsigned long long off[64];
    if (threadIdx.x < 64) h[threadIdx.x] = 0;
    __syncthreads();
    const uint64_t total = (uint64_t)n * ell;
    const uint64_t base = (uint64_t)blockIdx.x * kBlock * kRankPer;
    uint32_t pid[kRankPer], win[kRankPer], slot[kRankPer];
    for (int j = 0; j < kRankPer; ++j) {
        const uint64_t t = base + (uint64_t)j * kBlock + threadIdx.x;
        win[j] = 0xFFFFFFFFu;
        if (t < total) {
            const uint32_t v = (uint32_t)(t / ell), i = (uint32_t)(t % ell);
            pid[j] = v * kPairStride + i;
            win[j] = window_of(pair_rank(seed, pid[j]), W);
            slot[j] = atomicAdd(&h[win[j]], 1u);
        }
    }
    __syncthreads();
    if (threadIdx.x < W && h[threadIdx.x])
        off[threadIdx.x] = wbase[threadIdx.x] + atomicAdd(&wfill[threadIdx.x], h[threadIdx.x]);
    __syncthreads();
    for (int j = 0; j < kRankPer; ++j)
        if (win[j] != 0xFFFFFFFFu) sources[off[win[j]] + slot[j]] = pid[j];
}

// ------------------------------------------------ 3. pruned reverse search

__device__ __forceinline__ uint64_t hmix(uint64_t x) {
    x ^= x >> 31;
    x *= 0xD6E8FEB86659FD93ull;
    x ^= x >> 32;
    return x;
}

// 1 = inserted, 0 = already present, -1 = table full.
__device__ int hset_insert(uint64_t *T, uint32_t logcap, uint64_t key) {
    const uint64_t mask = (1ull << logcap) - 1;
    uint64_t h = hmix(key) & mask;
    for (int probe = 0; probe < 256; ++probe) {
        uint64_t cur = load_relaxed(T + h);
        if (cur == key) return 0;
        if (cur == kNone) {
            const uint64_t prev = atomicCAS((unsigned long long *)(T + h), kNone, key);
            if (prev == kNone) return 1;
            if (prev == key) return 0;
        }
        h = (h + 1) & mask;
    }
    return -1;
}

struct WinArgs {
    uint64_t *words;      // [64 n]: hi32 = ranks received so far, lo32 = first visitor
    uint64_t *items;      // visits of this window: (pair << 32) | source index
    uint64_t items_cap;
    uint64_t *hset;
    uint32_t logcap;
    uint32_t ws, we;      // sources [ws, we) of this window
    uint32_t k;
    Ctl *ctl;
};

// Visit of pair p by source s: 1 if new, 0 if pruned or already visited by s.
__device__ __forceinline__ int claim(const WinArgs &A, uint32_t p, uint32_t s, uint32_t &hashed) {
    uint64_t old = load_relaxed(A.words + p);
    for (;;) {
        if ((uint32_t)(old >> 32) >= A.k) return 0;  // instance-local sketch full: prune
        const uint32_t st = (uint32_t)old;
        if (st == s) return 0;
        if (st < A.ws || st >= A.we) {
            const uint64_t nw = (old & 0xFFFFFFFF00000000ull) | s;
            const uint64_t prev = atomicCAS((unsigned long long *)(A.words + p), old, nw);
            if (prev == old) return 1;
            old = prev;
            continue;
        }
        const int r = hset_insert(A.hset, A.logcap, ((uint64_t)p << 32) | s);
        if (r < 0) {
            atomicOr(&A.ctl->flags, kOvfHash);
            return 0;
        }
        hashed += r;
        return r;
    }
}

// Block-aggregated appends: threads stage new entries in LDS; one global
// reservation per flush moves them to the output array (coalesced).
constexpr uint32_t kChunk = 1024;        // input entries per block per round
constexpr uint32_t kStage = 4096;        // staged outputs per round (32 KiB)

struct Stage {
    uint64_t buf[kStage];
    uint32_t n;
    unsigned long long base;
};

__device__ __forceinline__ void stage_push(Stage &S, uint64_t v, uint64_t *out, uint64_t cap,
                                           unsigned long long *count, uint32_t *flags,
                                           uint32_t ovf_bit) {
    const uint32_t pos = atomicAdd(&S.n, 1u);
    if (pos < kStage) {
        S.buf[pos] = v;
        return;
    }
    const unsigned long long g = atomicAdd(count, 1ull);  // rare: stage full
    if (g < cap) out[g] = v;
    else atomicOr(flags, ovf_bit);
}

// Called by every thread of the block.
__device__ __forceinline__ void stage_flush(Stage &S, uint64_t *out, uint64_t cap,
                                            unsigned long long *count, uint32_t *flags,
                                            uint32_t ovf_bit) {
    __syncthreads();
    const uint32_t m = S.n < kStage ? S.n : kStage;
    if (threadIdx.x == 0) S.base = m ? atomicAdd(count, (unsigned long long)m) : 0;
    __syncthreads();
    const unsigned long long base = S.base;
    if (m && base + m > cap && threadIdx.x == 0) atomicOr(flags, ovf_bit);
    for (uint32_t j = threadIdx.x; j < m; j += blockDim.x)
        if (base + j < cap) out[base + j] = S.buf[j];
    __syncthreads();
    if (threadIdx.x == 0) S.n = 0;
    __syncthreads();
}

// Sources of the window start their searches.  Each source pair is claimed
// only by its own source here, so the claim is a plain store.
__global__ void __launch_bounds__(kBlock) k_seed_window(WinArgs A, const uint32_t *sources) {
    __shared__ Stage S;
    if (threadIdx.x == 0) S.n = 0;
    __syncthreads();
    for (uint64_t c = A.ws + (uint64_t)blockIdx.x * kChunk; c < A.we;
         c += (uint64_t)gridDim.x * kChunk) {
        const uint64_t end = c + kChunk < A.we ? c + kChunk : A.we;
        for (uint64_t t = c + threadIdx.x; t < end; t += blockDim.x) {
            const uint32_t s = (uint32_t)t;
            const uint32_t p = sources[s];
            const uint64_t w = A.words[p];
            if ((uint32_t)(w >> 32) >= A.k) continue;  // pruned
            reinterpret_cast<uint32_t *>(A.words + p)[0] = s;
            stage_push(S, ((uint64_t)p << 32) | s, A.items, A.items_cap, &A.ctl->count,
                       &A.ctl->flags, kOvfItems);
        }
        stage_flush(S, A.items, A.items_cap, &A.ctl->count, &A.ctl->flags, kOvfItems);
    }
}

// Expand the frontier items[a, b) over live in-edges of their instance.
__device__ __forceinline__ void expand_range(const WinArgs &A, const uint64_t *lptr,
                                             const uint32_t *lsrc, uint64_t a, uint64_t b,
                                             uint64_t first, uint64_t stride, Stage &S,
                                             uint32_t &scans, uint32_t &hashed) {
    for (uint64_t c = a + first; c < b; c += stride) {
        const uint64_t end = c + kChunk < b ? c + kChunk : b;
        for (uint64_t t = c + threadIdx.x; t < end; t += blockDim.x) {
            const uint64_t it = A.items[t];
            const uint32_t p = (uint32_t)(it >> 32);
            const uint32_t s = (uint32_t)it;
            const uint32_t i = p % kPairStride;
            const uint64_t e1 = lptr[p + 1];
            for (uint64_t e = lptr[p]; e < e1; ++e) {
                const uint32_t q = lsrc[e] * kPairStride + i;
                ++scans;
                if (claim(A, q, s, hashed) == 1)
                    stage_push(S, ((uint64_t)q << 32) | s, A.items, A.items_cap, &A.ctl->count,
                               &A.ctl->flags, kOvfItems);
            }
        }
        stage_flush(S, A.items, A.items_cap, &A.ctl->count, &A.ctl->flags, kOvfItems);
    }
}

// One level with the whole grid; the last block to finish publishes the
// next frontier boundary.
__global__ void __launch_bounds__(kBlock) k_expand(WinArgs A, const uint64_t *lptr,
                                                   const uint32_t *lsrc, uint32_t level) {
    __shared__ Stage S;
    __shared__ uint32_t s_flags;
    if (threadIdx.x == 0) {
        S.n = 0;
        s_flags = __hip_atomic_load(&A.ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    uint32_t scans = 0, hashed = 0;
    if (!s_flags) {  // after an overflow the window is redone with more room
        const uint64_t a = A.ctl->lb[level & 3], b = A.ctl->lb[(level + 1) & 3];
        expand_range(A, lptr, lsrc, a, b, (uint64_t)blockIdx.x * kChunk,
                     (uint64_t)gridDim.x * kChunk, S, scans, hashed);
    }
    wave_add(&A.ctl->scans, scans);
    wave_add(&A.ctl->hinserts, hashed);
    __syncthreads();
    if (threadIdx.x == 0) {
        __threadfence();
        const uint32_t prev = atomicAdd(&A.ctl->done_blocks, 1u);
        if (prev == gridDim.x - 1) {
            A.ctl->lb[(level + 2) & 3] =
                __hip_atomic_load(&A.ctl->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            A.ctl->done_blocks = 0;
            __threadfence();
        }
    }
}

// Small frontiers: one workgroup runs level after level until the frontier
// is empty, grows past `max_frontier`, or an overflow is flagged.
__global__ void __launch_bounds__(1024) k_expand_tail(WinArgs A, const uint64_t *lptr,
                                                      const uint32_t *lsrc, uint32_t level,
                                                      uint64_t max_frontier) {
    __shared__ Stage S;
    __shared__ unsigned long long s_a, s_b;
    __shared__ uint32_t s_stop;
    if (threadIdx.x == 0) S.n = 0;
    uint32_t scans = 0, hashed = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            s_a = A.ctl->lb[level & 3];
            s_b = A.ctl->lb[(level + 1) & 3];
            const uint32_t f =
                __hip_atomic_load(&A.ctl->flags, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_stop = f || s_a == s_b || s_b - s_a > max_frontier;
        }
        __syncthreads();
        if (s_stop) break;
        expand_range(A, lptr, lsrc, s_a, s_b, 0, kChunk, S, scans, hashed);
        if (threadIdx.x == 0) {
            __threadfence();
            A.ctl->lb[(level + 2) & 3] =
                __hip_atomic_load(&A.ctl->count, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        ++level;
        __syncthreads();
    }
    wave_add(&A.ctl->scans, scans);
    wave_add(&A.ctl->hinserts, hashed);
    if (threadIdx.x == 0) A.ctl->level = level;
}

// Start of an attempt at a window: clear the per-window fields.
__global__ void k_ctl_begin(Ctl *ctl) {
    ctl->lb[0] = ctl->lb[1] = ctl->lb[2] = ctl->lb[3] = 0;
    ctl->count = 0;
    ctl->scans = 0;
    ctl->hinserts = 0;
    ctl->flags = 0;
    ctl->done_blocks = 0;
    ctl->level = 0;
}

__global__ void k_seed_done(Ctl *ctl) { ctl->lb[1] = ctl->count; }

// Roll the record counter back (after growing the record buffer).
__global__ void k_ctl_records(Ctl *ctl, unsigned long long records) {
    ctl->records = records;
    ctl->flags = 0;
}

struct WinBases {
    unsigned long long b[64];
};

__global__ void k_set_bases(unsigned long long *dst, WinBases wb) {
    if (threadIdx.x < 64) dst[threadIdx.x] = wb.b[threadIdx.x];
}

// Undo the claims of an aborted attempt at window [ws, we).
__global__ void k_unclaim(uint64_t *words, uint64_t npairs, uint32_t ws, uint32_t we) {
    for (uint64_t p = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; p < npairs;
         p += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t w = words[p];
        const uint32_t st = (uint32_t)w;
        if (st >= ws && st < we) words[p] = (w & 0xFFFFFFFF00000000ull) | kNoSrc;
    }
}

// ---------------------------------------------------------- 4. records

// Keep a record of every visit of a node that held fewer than k ranks at the
// window start (xcnt is the node's record count before this window).
__global__ void __launch_bounds__(kBlock) k_records(const uint64_t *items, uint64_t count,
                                                    const uint32_t *xcnt, uint32_t *xadd,
                                                    uint32_t k, uint64_t *rec, uint64_t rec_cap,
                                                    Ctl *ctl) {
    __shared__ Stage S;
    if (threadIdx.x == 0) S.n = 0;
    __syncthreads();
    for (uint64_t c = (uint64_t)blockIdx.x * kChunk; c < count; c += (uint64_t)gridDim.x * kChunk) {
        const uint64_t end = c + kChunk < count ? c + kChunk : count;
        for (uint64_t t = c + threadIdx.x; t < end; t += blockDim.x) {
            const uint64_t it = items[t];
            const uint32_t v = (uint32_t)(it >> 32) / kPairStride;
            if (xcnt[v] < k) {
                atomicAdd(xadd + v, 1u);
                stage_push(S, ((uint64_t)v << 32) | (uint32_t)it, rec, rec_cap, &ctl->records,
                           &ctl->flags, kOvfRecords);
            }
        }
        stage_flush(S, rec, rec_cap, &ctl->records, &ctl->flags, kOvfRecords);
    }
}

__global__ void k_fold(uint32_t *xcnt, uint32_t *xadd, uint32_t n, uint32_t k, Ctl *ctl) {
    uint32_t crossed = 0;
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t add = xadd[v];
        if (add) {
            const uint32_t old = xcnt[v];
            xcnt[v] = old + add;
            xadd[v] = 0;
            crossed += (old < k && old + add >= k);
        }
    }
    wave_add(&ctl->full, crossed);
}

// Pair (v, i) received one more rank (its instance-local count).
__global__ void k_count_arrivals(const uint64_t *items, uint64_t count, uint64_t *words) {
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < count;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p = (uint32_t)(items[t] >> 32);
        atomicAdd((uint32_t *)(words + p) + 1, 1u);  // high half of the little-endian word
    }
}

// ------------------------------------------------------------- 5. merge

__global__ void k_group(const uint64_t *rec, uint64_t nrec, const uint32_t *sources,
                        uint64_t seed, const uint64_t *goff, uint32_t *gfill, uint64_t *seg) {
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < nrec;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t r = rec[t];
        const uint32_t v = (uint32_t)(r >> 32);
        const uint32_t s = (uint32_t)r;
        const uint64_t pos = goff[v] + atomicAdd(gfill + v, 1u);
        seg[pos] = pair_rank(seed, sources[s]);
    }
}

// Bitonic sort of P (power of two, <= 512) keys in LDS by one 64-lane block.
__device__ void lds_bitonic(uint64_t *x, uint32_t P) {
    for (uint32_t size = 2; size <= P; size <<= 1) {
        for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
            for (uint32_t t = threadIdx.x; t < P / 2; t += blockDim.x) {
                const uint32_t lo = 2 * t - (t & (stride - 1));
                const uint32_t hi = lo + stride;
                const bool up = (lo & size) == 0;
                const uint64_t a = x[lo], b = x[hi];
                if ((a > b) == up) {
                    x[lo] = b;
                    x[hi] = a;
                }
            }
            __syncthreads();
        }
    }
}

// One block (one wave) per node: keep the k smallest of the node's records.
__global__ void __launch_bounds__(64) k_select(const uint64_t *goff, const uint64_t *seg,
                                               uint32_t n, uint32_t k, uint64_t *ranks,
                                               uint32_t *size) {
    __shared__ uint64_t buf[512];
    for (uint32_t v = blockIdx.x; v < n; v += gridDim.x) {
        const uint64_t a = goff[v], b = goff[v + 1];
        const uint64_t S = b - a;
        uint32_t keep;
        if (S <= 512) {
            uint32_t P = 64;
            while (P < S) P <<= 1;
            for (uint32_t j = threadIdx.x; j < P; j += blockDim.x) buf[j] = j < S ? seg[a + j] : kNone;
            __syncthreads();
            if (S > 1) lds_bitonic(buf, P);
            keep = (uint32_t)(S < k ? S : k);
        } else {
            for (uint32_t j = threadIdx.x; j < 256; j += blockDim.x) buf[j] = kNone;
            for (uint64_t c = a; c < b; c += 256) {
                for (uint32_t j = threadIdx.x; j < 256; j += blockDim.x)
                    buf[256 + j] = c + j < b ? seg[c + j] : kNone;
                __syncthreads();
                lds_bitonic(buf, 512);
            }
            keep = k;
        }
        uint64_t *row = ranks + (uint64_t)v * k;
        for (uint32_t j = threadIdx.x; j < k; j += blockDim.x) row[j] = j < keep ? buf[j] : kNone;
        if (threadIdx.x == 0) size[v] = keep;
        __syncthreads();
    }
}

uint32_t choose_windows(uint32_t n, uint32_t k) {
    // window 0 holds about k/2 sources per instance; later windows double
    double x = 2.0 * n / (double)k;
    uint32_t W = 1;
    while (W < 48 && (double)(1ull << (W - 1)) < x) ++W;
    return W;
}

uint64_t next_pow2(uint64_t x) {
    uint64_t p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

// Host orchestration of one sketch build.
static void build_sketches(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed,
                           uint64_t *ranks_out, uint32_t *size_out, double *est_out,
                           uint64_t *work, hipStream_t s) {
    SKIM_REQUIRE(ell >= 1 && ell <= 64, "l must be in [1, 64]");
    SKIM_REQUIRE(k >= 2 && k <= 256, "k must be in [2, 256]");
    SKIM_REQUIRE(ranks_out && size_out, "ranks/size output is NULL");
    Arena A(s);
    const uint32_t n = g->n;
    const uint64_t m = g->m;
    uint32_t *esrc = A.alloc<uint32_t>(m ? m : 1);
    validate_graph(g, esrc, A);

    const uint64_t npairs = (uint64_t)n * kPairStride;  // pair-id space (stride 64)
    const uint64_t nsrc = (uint64_t)n * ell;            // actual pairs

    // ---- 1. live lists (reverse: in-edges of every pair)
    LiveLists live = build_live_lists(g, ell, seed, esrc, /*forward=*/false, A);
    const uint64_t *lptr = live.ptr;
    const uint32_t *lsrc = live.adj;
    A.release(esrc);

    // ---- 2. rank windows
    const uint32_t W = choose_windows(n, k);
    unsigned long long *wbuf = A.alloc<unsigned long long>(2 * 64);
    fill_u64((uint64_t *)wbuf, 0, 128, s);
    const unsigned rblocks = (unsigned)((nsrc + (uint64_t)kBlock * kRankPer - 1) /
                                        ((uint64_t)kBlock * kRankPer));
    k_rank_hist<<<rblocks, kBlock, 0, s>>>(n, ell, seed, W, wbuf);
    SKIM_LAUNCH_CHECK();
    unsigned long long hw[64] = {};
    read_back(hw, wbuf, sizeof(unsigned long long) * 64, s);
    unsigned long long wb[65] = {};
    for (uint32_t w = 0; w < W; ++w) wb[w + 1] = wb[w] + hw[w];
    WinBases bases;
    std::memcpy(bases.b, wb, sizeof bases.b);
    k_set_bases<<<1, 64, 0, s>>>(wbuf, bases);
    SKIM_LAUNCH_CHECK();
    fill_u64((uint64_t *)wbuf + 64, 0, 64, s);
    uint32_t *sources = A.alloc<uint32_t>(nsrc);
    k_rank_scatter<<<rblocks, kBlock, 0, s>>>(n, ell, seed, W, wbuf, wbuf + 64, sources);
    SKIM_LAUNCH_CHECK();

    // ---- 3./4. windows
    uint64_t *words = A.alloc<uint64_t>(npairs);
    fill_u64(words, (uint64_t)kNoSrc, npairs, s);  // 0 ranks received, no visitor
    uint32_t *xcnt = A.alloc<uint32_t>(n + 1);
    uint32_t *xadd = A.alloc<uint32_t>(n + 1);
    fill_u32(xcnt, 0, n + 1, s);
    fill_u32(xadd, 0, n + 1, s);
    Ctl *ctl = A.alloc<Ctl>(1);
    fill_u64((uint64_t *)ctl, 0, sizeof(Ctl) / 8, s);

    uint64_t rec_cap = std::max<uint64_t>(1ull << 20, (uint64_t)n * k + (uint64_t)n * 4);
    uint64_t *rec = A.alloc<uint64_t>(rec_cap);
    uint64_t items_cap = 0, hcap = 0;
    uint64_t *items = nullptr, *hset = nullptr;
    uint64_t total_items = 0, total_scans = 0, windows_done = 0;
    uint64_t prev_items = 0, prev_hash = 0;
    constexpr uint64_t kTail = 16384;  // frontiers this small go to the one-workgroup loop
    Ctl h;

    for (uint32_t w = 0; w < W; ++w) {
        const uint32_t ws = (uint32_t)wb[w], we = (uint32_t)wb[w + 1];
        if (ws == we) continue;
        read_back(&h, ctl, sizeof h, s);
        if (h.full >= n) break;  // every sketch holds k ranks: later ranks cannot enter
        const uint64_t nw = we - ws;
        // windows double in size: predict from the previous one
        uint64_t want_items = std::max<uint64_t>({1ull << 16, 3 * nw, 3 * prev_items});
        uint64_t want_hash = next_pow2(std::max<uint64_t>({1ull << 14, nw / 2, 8 * prev_hash}));
        for (int attempt = 0;; ++attempt) {
            if (attempt >= 24) {
                set_error("window %u did not fit after %d attempts", w, attempt);
                throw Fail{SKIM_EDEVICE};
            }
            if (want_items > items_cap) {
                if (items) A.release(items);
                items_cap = want_items;
                items = A.alloc<uint64_t>(items_cap);
            }
            if (want_hash > hcap) {
                if (hset) A.release(hset);
                hcap = want_hash;
                hset = A.alloc<uint64_t>(hcap);
            }
            uint32_t logcap = 0;
            while ((1ull << logcap) < hcap) ++logcap;
            fill_u64(hset, kNone, hcap, s);
            k_ctl_begin<<<1, 1, 0, s>>>(ctl);
            SKIM_LAUNCH_CHECK();

            WinArgs WA{words, items, items_cap, hset, logcap, ws, we, k, ctl};
            {
                LaunchTimer t("k_seed_window", s);
                k_seed_window<<<grid_for(nw, kChunk, 4096), kBlock, 0, s>>>(WA, sources);
            }
            SKIM_LAUNCH_CHECK();
            k_seed_done<<<1, 1, 0, s>>>(ctl);
            SKIM_LAUNCH_CHECK();
            uint32_t level = 0;
            for (;;) {
                read_back(&h, ctl, sizeof h, s);
                if (h.flags) break;
                const uint64_t fa = h.lb[level & 3], fb = h.lb[(level + 1) & 3];
                if (fa == fb) break;  // empty frontier: window done
                if (fb - fa <= kTail) {
                    LaunchTimer t("k_expand_tail", s);
                    k_expand_tail<<<1, 1024, 0, s>>>(WA, lptr, lsrc, level, 4 * kTail);
                    SKIM_LAUNCH_CHECK();
                    read_back(&h, ctl, sizeof h, s);
                    level = h.level;
                    continue;
                }
                // big frontier: a few whole-grid levels before looking again
                for (int j = 0; j < 3; ++j, ++level) {
                    const unsigned grid = j == 0 ? grid_for(fb - fa, kChunk, 2048) : 2048;
                    LaunchTimer t("k_expand", s);
                    k_expand<<<grid, kBlock, 0, s>>>(WA, lptr, lsrc, level);
                    SKIM_LAUNCH_CHECK();
                }
            }
            if (h.flags & (kOvfItems | kOvfHash)) {
                k_unclaim<<<grid_for(npairs, kBlock, 8192), kBlock, 0, s>>>(words, npairs, ws, we);
                SKIM_LAUNCH_CHECK();
                if (h.flags & kOvfItems) want_items = std::max<uint64_t>(2 * items_cap, h.count + nw);
                if (h.flags & kOvfHash) want_hash = 2 * hcap;
                continue;
            }
            break;
        }
        const uint64_t count = h.count;
        prev_items = count;
        prev_hash = h.hinserts;
        total_items += count;
        total_scans += h.scans;
        // records of nodes that held fewer than k ranks at the window start
        const uint64_t rec_before = h.records;
        for (int attempt = 0;; ++attempt) {
            if (attempt >= 8) {
                set_error("record buffer did not fit");
                throw Fail{SKIM_EDEVICE};
            }
            {
                LaunchTimer t("k_records", s);
                k_records<<<grid_for(count, kChunk, 4096), kBlock, 0, s>>>(items, count, xcnt, xadd,
                                                                           k, rec, rec_cap, ctl);
            }
            SKIM_LAUNCH_CHECK();
            read_back(&h, ctl, sizeof h, s);
            if (!(h.flags & kOvfRecords)) break;
            // grow the record buffer, keep what earlier windows wrote, retry
            const uint64_t need = h.records;
            uint64_t new_cap = std::max<uint64_t>(2 * rec_cap, need + need / 4);
            uint64_t *nrec = A.alloc<uint64_t>(new_cap);
            SKIM_HIP(hipMemcpyAsync(nrec, rec, rec_before * sizeof(uint64_t),
                                    hipMemcpyDeviceToDevice, s));
            A.release(rec);
            rec = nrec;
            rec_cap = new_cap;
            fill_u32(xadd, 0, n + 1, s);
            k_ctl_records<<<1, 1, 0, s>>>(ctl, rec_before);
            SKIM_LAUNCH_CHECK();
        }
        k_fold<<<grid_for(n, kBlock, 8192), kBlock, 0, s>>>(xcnt, xadd, n, k, ctl);
        SKIM_LAUNCH_CHECK();
        {
            LaunchTimer t("k_count_arrivals", s);
            k_count_arrivals<<<grid_for(count, kBlock, 16384), kBlock, 0, s>>>(items, count, words);
        }
        SKIM_LAUNCH_CHECK();
        ++windows_done;
    }
    read_back(&h, ctl, sizeof h, s);
    const uint64_t nrec = h.records;

    // ---- 5. merge: group records by node, keep the k smallest
    A.release(words);
    if (items) A.release(items);
    if (hset) A.release(hset);
    uint64_t *goff = A.alloc<uint64_t>((uint64_t)n + 1);
    exclusive_scan_u32(xcnt, goff, n, A);
    uint64_t *seg = A.alloc<uint64_t>(nrec ? nrec : 1);
    fill_u32(xadd, 0, n + 1, s);
    if (nrec) {
        LaunchTimer t("k_group", s);
        k_group<<<grid_for(nrec, kBlock, 16384), kBlock, 0, s>>>(rec, nrec, sources, seed, goff, xadd,
                                                                 seg);
        SKIM_LAUNCH_CHECK();
    }
    {
        LaunchTimer t("k_select", s);
        k_select<<<grid_for(n, 1, 65536), 64, 0, s>>>(goff, seg, n, k, ranks_out, size_out);
    }
    SKIM_LAUNCH_CHECK();
    if (est_out) launch_estimates(ranks_out, size_out, n, k, ell, est_out, s);
    SKIM_HIP(hipStreamSynchronize(s));
    timing_resolve();
    if (work) {
        work[0] = total_items;
        work[1] = total_scans;
        work[2] = nrec;
        work[3] = windows_done;
    }
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
