// skim_greedy.hip -- SKIM greedy seed selection (Section 4, Algorithm 1).
//
// State on the device: live reverse and forward lists of every pair, the
// pairs sorted by rank, covered[pair], size[node], and the inverted index
// (for every processed pair, the nodes its reverse search reached).
//
// One persistent workgroup runs the selection loop (the loop is sequential
// per seed); residual searches that grow large continue on the whole grid:
//  * scan: the next B pairs in rank order each run their complete reverse
//    search in parallel (one thread per pair; an uncovered pair never reaches
//    a covered one, so the searches are independent of each other's
//    increments).  If some node's size reaches k with all B pairs, the first
//    prefix length T at which one does is the smallest position at which a
//    filling node receives its (k - size)-th entry, found from the entries
//    of the filling nodes alone (binary search over prefixes when there are
//    too many); pairs [0, T) are committed (size increments, index entries),
//    the rest are re-scanned later.  The nodes that reached k all sit in
//    pair T-1's search; the smallest id among them is the seed.  Batches
//    with a long search spread the per-entry work over the block by flat
//    position instead of per thread.
//  * exhaustion: with every rank processed, the unselected node with the
//    largest size (smallest id on ties) is the seed.
//  * records: before the residual update, the rank tau of the pair that filled
//    the seed's sketch and the second largest sketch k' (largest size among
//    the other unselected nodes, one less for nodes in that pair's search)
//    are stored per seed for the adaptive error estimate (Section 4).
//  * residual: a level-synchronous forward search from the seed over all
//    instances at once (each level's frontier of pairs shared by the block)
//    over live out-edges, not entering covered pairs; every newly covered
//    pair counts towards the seed's gain and decrements the size of every
//    node in its index entry, which is then erased.  A level of more than
//    kSkimHandoff pairs, or a seed with more than kSkimHandoffEdges live
//    out-edges, ends the workgroup's launch; the host runs the rest of that
//    search level by level on the whole grid (k_resid_level; pairs of long
//    out-lists are expanded edge-balanced by the next level's launch) and then
//    relaunches the loop; a search whose next level there is small again is
//    handed back, and the relaunched loop resumes it at that level.
//
// The adaptive error estimate itself (skim_discrepancy_tail) bounds each
// seed's discrepancy with eq. (chernoff) on a grid of discrepancy values and
// convolves the per-seed distributions pairwise in a tree of launches.
#include "skim_internal.h"

#include <mutex>

#include <rocprim/device/device_radix_sort.hpp>

#include <algorithm>
#include <cstring>
#include <memory>
#include <utility>

namespace skim {

namespace {

constexpr int kSkimBlock = 1024;
constexpr uint32_t kSkimLdsNodes = 20480;  // graphs up to this size keep size[] in LDS
constexpr uint32_t kSkimPairListNodes = 1u << 17;  // from this size, in-lists as pair words
constexpr uint32_t kSkimLdsWords = kSkimLdsNodes / 2;
constexpr uint32_t kFlagPool = 1u;
// Items whose search, index entry or out-list is at most this long are
// walked by their own thread; a batch or level with a longer one spreads
// its work over the block by flat position.
constexpr uint32_t kSkimSerial = 32;
// ... and a wave whose items all have at most this many walks them lane by
// lane; with a longer one the wave lays them end to end.
constexpr uint32_t kSkimFlat = 4;
// A residual level with more pairs than this continues on the whole grid.
constexpr uint64_t kSkimHandoff = 4096;
// ... and so does a seed whose own live out-edges are more than this.
constexpr uint64_t kSkimHandoffEdges = 65536;
// A search on the grid whose next level has at most this many pairs goes
// back to the workgroup (a level there costs less than two launches).
constexpr uint64_t kSkimHandBack = 2048;
// On the grid, pairs with more live out-edges than this are deferred to the
// next level's launch, which spreads their edges over every workgroup before
// it takes its own frontier (their heads join the level after it: the
// covered set does not depend on the order of the expansions).  At most
// kHeavyItems per level; more are expanded where they are.
constexpr uint64_t kSplitEdges = 1024;
constexpr uint32_t kHeavyItems = 1u << 16;
// Entries of the nodes that fill within a batch, kept to find the filling
// prefix directly (more: binary search over prefixes).
constexpr uint32_t kSkimCand = 1024;
// The first kSkimLdsFront entries of a residual level in the workgroup live
// in LDS (the rest in the queue area): small levels never go through global
// memory between one level and the next.
constexpr uint32_t kSkimLdsFront = 2048;
constexpr int kResidBlock = 256;
constexpr uint32_t kResidGrid = 512;

struct SkCtl {
    unsigned long long cursor;     // next position in the rank order
    unsigned long long pool_used;  // index entries in use
    unsigned long long need;       // pool entries a failed batch needed
    uint32_t done;                 // seeds completed by the last launch
    uint32_t flags;
    // A residual search handed to the whole grid (its frontier outgrew the
    // workgroup): the seed, the frontier buffer of its current level, the
    // pairs covered so far, and the level sizes (each counter on a line of
    // its own; level L reads rsize[L % 3], appends to rsize[(L + 1) % 3]).
    uint32_t pend, px, rcur, pad;
    unsigned long long rgain;
    unsigned long long pad2[10];
    unsigned long long rsize[3 * 16];
    unsigned long long hsize[3 * 16];  // pairs level L deferred: hsize[16 (L % 3)]
};

struct SkArgs {
    uint32_t n, ell, k;
    uint64_t nsrc;
    // live in-lists: on large graphs the words of the sketch build ([64 n],
    // rlive, with rsrc), else a CSR over pairs (rptr [64 n + 1], radj)
    const uint64_t *rlive;
    const uint32_t *rsrc;
    const uint64_t *rptr;
    const uint32_t *radj;
    const uint64_t *fptr;
    const uint32_t *fadj;
    const uint32_t *order;  // pair ids by increasing rank
    uint32_t *covered;      // [64 n] 0/1
    uint32_t *size;         // [2 ceil(n / 4)] packed 16-bit counters
    uint32_t *sel;          // [n] 0/1
    uint64_t *idx;          // [64 n] first pool entry << 32 | entries, 0 = no entry
    uint32_t *pool;
    uint64_t pool_cap;
    uint32_t *bcnt;         // [2 ceil(n / 4)] per-batch increment counters, packed
    uint32_t *queues;       // [kSkimBlock * n]
    uint64_t *heavy;        // [3][2 kHeavyItems] grid residual, deferred (pair, count), first out-edge
    uint32_t *vis;          // [kSkimBlock * vis_words] per-thread visited bitmaps, kept zero
    uint32_t vis_words;     // ceil(n / 32)
    SkCtl *ctl;
    uint64_t seed;
    uint64_t *rec_tau;      // [n] per selected seed: rank that filled its sketch
    uint32_t *rec_second;   // [n] per selected seed: second largest sketch
};

// A thread's reverse search marks the nodes it has queued in its own bitmap
// (test and set: one load and at most one store per scanned edge, instead of
// a scan of the queue) and clears the words it touched when it is done.
__device__ __forceinline__ bool mark_new(uint32_t *V, uint32_t w) {
    const uint32_t bit = 1u << (w & 31u), word = V[w >> 5];
    if (word & bit) return false;
    V[w >> 5] = word | bit;
    return true;
}

// size[] and the batch counters are 16-bit halves of 32-bit words (sizes
// never exceed k <= 256, batch counts never exceed one batch of 1024 pairs),
// so twice as many nodes fit in LDS.  Adds and subtracts never carry across
// halves.
__device__ __forceinline__ uint32_t half_shift(uint32_t v) { return (v & 1u) << 4; }

// State shared between the block's threads goes through agent-scope atomic
// loads and stores, so no thread reads a stale cached copy of it.
template <class T> __device__ __forceinline__ T ld(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ void st(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint32_t cget(const uint32_t *c, uint32_t v) {
    return (ld(c + (v >> 1)) >> half_shift(v)) & 0xFFFFu;
}
__device__ __forceinline__ void cadd(uint32_t *c, uint32_t v, uint32_t d) {
    atomicAdd(c + (v >> 1), d << half_shift(v));
}
__device__ __forceinline__ void csub(uint32_t *c, uint32_t v, uint32_t d) {
    atomicSub(c + (v >> 1), d << half_shift(v));
}
__device__ __forceinline__ void czero(uint32_t *c, uint32_t v) {
    atomicAnd(c + (v >> 1), ~(0xFFFFu << half_shift(v)));
}

// Exclusive prefix sum of v over the block (NT threads, called by all of
// them) and the block total; wsum holds one word per wave.
template <uint32_t NT>
__device__ __forceinline__ uint64_t block_excl_scan(uint64_t v, uint64_t *wsum, uint64_t &total) {
    const uint32_t lane = threadIdx.x & 63u, wave = threadIdx.x >> 6;
    uint64_t x = v;
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t lo = __shfl_up((uint32_t)x, off), hi = __shfl_up((uint32_t)(x >> 32), off);
        if (lane >= off) x += ((uint64_t)hi << 32) | lo;
    }
    __syncthreads();  // earlier readers of wsum are done
    if (lane == 63u) wsum[wave] = x;
    __syncthreads();
    uint64_t before = 0, tot = 0;
    for (uint32_t w = 0; w < NT / 64; ++w) {
        const uint64_t s = wsum[w];
        before += w < wave ? s : 0;
        tot += s;
    }
    total = tot;
    return before + x - v;
}

// The run that holds flat position t: the largest r with ex[r] <= t, for
// exclusive prefix sums ex[0..NT] (runs of length zero are never returned
// for t below the total).
template <uint32_t NT>
__device__ __forceinline__ uint32_t run_of(const uint64_t *ex, uint64_t t) {
    uint32_t lo = 0, hi = NT;  // ex[lo] <= t < ex[hi]
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) >> 1;
        if (ex[mid] <= t) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Inclusive prefix sum over the wave's 64 lanes, and the lane whose range
// holds flat position j of the wave's items laid end to end (binary lifting
// over the prefix sums; j below the wave's total).
__device__ __forceinline__ uint32_t wave_incl(uint32_t v) {
    const uint32_t lane = threadIdx.x & 63u;
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(v, off);
        if (lane >= off) v += y;
    }
    return v;
}
__device__ __forceinline__ uint32_t wave_owner(uint32_t incl, uint32_t j) {
    uint32_t r = 0;
#pragma unroll
    for (uint32_t step = 32; step > 0; step >>= 1) {
        const uint32_t v = (uint32_t)__shfl((int)incl, (int)(r + step - 1));
        if (v <= j) r += step;
    }
    return r & 63u;
}

// Work that depends on the length of a search or of an adjacency list is
// spread over the whole block by flat position (prefix sums over the
// block's items, then a binary search per position), so one long item
// does not hold up a level.
template <uint32_t NT> struct FlatShared {
    uint64_t ex[NT + 1];   // scan: queue lengths; residual: out-edges
    uint64_t ex2[NT + 1];  // residual: index entries
    uint64_t f0[NT];       // residual: first out-edge
    uint32_t q[NT];        // residual: the pair
    uint32_t o[NT];        // residual: first index entry
    uint64_t wsum[NT / 64];
};

// Appends of a grid-wide residual level, staged in LDS and reserved in
// global memory once per chunk (one counter serves the whole grid).
struct ResidStage {
    uint32_t buf[8 * kResidBlock];
    uint32_t n;
    unsigned long long base;
};

struct ScanShared {
    uint64_t cand[kSkimCand];  // (pair position << 32) | node, nodes that fill
    uint32_t ncand, tmin;
};

// One chunk of a residual level: frontier entries [base, base + NT) of
// Fin (fc entries).  Each newly covered pair's index entry is erased (its
// nodes lose one from their sizes), and its live out-edges cover the pairs
// they reach in the same instance, appended to Fout (counted in *next).
// Called by all NT threads of the block.
// Precheck: read a pair's covered flag before the CAS (fewer atomics when
// many targets are covered already; one more step of latency).
template <uint32_t NT, bool Precheck>
__device__ __forceinline__ void resid_chunk(const SkArgs &A, uint32_t *SZ, const uint32_t *Fin,
                                            uint32_t *Fout, uint64_t fc, uint64_t base,
                                            FlatShared<NT> &X, unsigned long long *next,
                                            ResidStage *stage, unsigned long long *hcount,
                                            uint64_t *hbuf, const uint32_t *lfin = nullptr,
                                            uint32_t *lfout = nullptr) {
    const uint32_t tid = threadIdx.x;
    // one wave's newly covered pairs: to the stage (when there is one) or
    // straight to Fout
    auto push = [&](bool add, uint32_t qw) {
        if (!stage) {
            const uint64_t slot = wave_reserve(next, add);
            if (add) {
                if (lfout && slot < kSkimLdsFront) lfout[slot] = qw;
                else st(Fout + slot, qw);
            }
            return;
        }
        const unsigned long long m = __ballot(add);
        if (!m) return;
        const int leader = __ffsll((long long)m) - 1;
        const uint32_t lane = lane_id();
        uint32_t pos0 = 0;
        if ((int)lane == leader) pos0 = atomicAdd(&stage->n, (uint32_t)__popcll(m));
        const uint32_t pos = (uint32_t)__shfl((int)pos0, leader) +
                             (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
        if (!add) return;
        if (pos < 8 * kResidBlock) stage->buf[pos] = qw;
        else Fout[atomicAdd(next, 1ull)] = qw;  // stage full
    };
    auto flush = [&]() {
        if (!stage) return;
        __syncthreads();
        const uint32_t ns = stage->n < 8 * kResidBlock ? stage->n : 8 * kResidBlock;
        if (tid == 0 && ns) stage->base = atomicAdd(next, (unsigned long long)ns);
        __syncthreads();
        const unsigned long long b = stage->base;
        for (uint32_t j = tid; j < ns; j += NT) Fout[b + j] = stage->buf[j];
        __syncthreads();
        if (tid == 0) stage->n = 0;  // before the next chunk's first barrier
    };
    const uint64_t e = base + tid;
    uint32_t q = 0, o = 0, c = 0;
    uint64_t f0 = 0, deg = 0;
    if (e < fc) {
        q = lfin && e < kSkimLdsFront ? lfin[e] : Fin[e];
        const uint64_t ix = ld(A.idx + q);
        c = (uint32_t)ix;
        if (c) {
            o = (uint32_t)(ix >> 32);
            st(A.idx + q, (uint64_t)0);
        }
        f0 = A.fptr[q];
        deg = A.fptr[q + 1] - f0;
        if (hcount && deg > kSplitEdges) {  // deferred to the next level's launch
            const unsigned long long slot = atomicAdd(hcount, 1ull);
            if (slot < kHeavyItems) {
                hbuf[2 * slot] = ((uint64_t)q << 32) | (uint32_t)deg;
                hbuf[2 * slot + 1] = f0;
                deg = 0;
            }
        }
    }
    const bool light = __syncthreads_or(c > kSkimSerial || deg > kSkimSerial) == 0;
    if (light) {
        // each wave lays its 64 items' index entries, then their out-edges,
        // end to end and takes them 64 at a time
        const uint32_t lane = tid & 63u;
        if (!__any(c > kSkimFlat)) {  // short everywhere: each lane its own
            for (uint32_t j = 0; j < c; ++j) csub(SZ, ld(A.pool + o + j), 1u);
        } else {
            const uint32_t incl = wave_incl(c), total = (uint32_t)__shfl((int)incl, 63);
            for (uint32_t base = 0; base < total; base += 64) {
                const uint32_t j = base + lane, r = wave_owner(incl, j);
                const uint32_t first = (uint32_t)__shfl((int)incl, (int)r) -
                                       (uint32_t)__shfl((int)c, (int)r);
                const uint32_t ro = (uint32_t)__shfl((int)o, (int)r);
                if (j < total) csub(SZ, ld(A.pool + ro + (j - first)), 1u);
            }
        }
        const uint32_t d = (uint32_t)deg;  // <= kSkimSerial here
        if (!__any(d > kSkimFlat)) {  // short everywhere: each lane its own
            for (uint64_t x2 = f0; x2 < f0 + d; ++x2) {
                const uint32_t qw = A.fadj[x2] * kPairStride + q % kPairStride;
                const bool add = (!Precheck || !ld(A.covered + qw)) &&
                                 atomicCAS(A.covered + qw, 0u, 1u) == 0u;
                push(add, qw);
            }
            flush();
            return;
        }
        const uint32_t incl = wave_incl(d), total = (uint32_t)__shfl((int)incl, 63);
        for (uint32_t base = 0; base < total; base += 64) {
            const uint32_t j = base + lane, r = wave_owner(incl, j);
            const uint32_t first = (uint32_t)__shfl((int)incl, (int)r) -
                                   (uint32_t)__shfl((int)d, (int)r);
            const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)f0, (int)r);
            const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(f0 >> 32), (int)r);
            const uint32_t rq = (uint32_t)__shfl((int)q, (int)r);
            bool add = false;
            uint32_t qw = 0;
            if (j < total) {
                qw = A.fadj[(((uint64_t)hi << 32) | lo) + (j - first)] * kPairStride +
                     rq % kPairStride;
                add = (!Precheck || !ld(A.covered + qw)) &&
                      atomicCAS(A.covered + qw, 0u, 1u) == 0u;
            }
            push(add, qw);
        }
        flush();
        return;
    }
    uint64_t ctot, dtot;
    const uint64_t cex = block_excl_scan<NT>(c, X.wsum, ctot);
    const uint64_t dex = block_excl_scan<NT>(deg, X.wsum, dtot);
    X.ex2[tid] = cex;
    X.ex[tid] = dex;
    X.q[tid] = q;
    X.o[tid] = o;
    X.f0[tid] = f0;
    if (tid == 0) {
        X.ex2[NT] = ctot;
        X.ex[NT] = dtot;
    }
    __syncthreads();
    for (uint64_t t = tid; t < ctot; t += NT) {
        const uint32_t r = run_of<NT>(X.ex2, t);
        csub(SZ, ld(A.pool + X.o[r] + (t - X.ex2[r])), 1u);
    }
    for (uint64_t t = tid; t < dtot; t += NT) {
        const uint32_t r = run_of<NT>(X.ex, t);
        const uint32_t qw = A.fadj[X.f0[r] + (t - X.ex[r])] * kPairStride + X.q[r] % kPairStride;
        const bool add =
            (!Precheck || !ld(A.covered + qw)) && atomicCAS(A.covered + qw, 0u, 1u) == 0u;
        push(add, qw);
    }
    flush();
    __syncthreads();  // the chunk's LDS arrays are reused
}

__global__ void __launch_bounds__(kSkimBlock) k_skim(SkArgs A, uint32_t goal, uint64_t handoff,
                                                     uint32_t *seeds, uint64_t *gains,
                                                     double *gain_d, uint64_t *rec_tau,
                                                     uint32_t *rec_second) {
    __shared__ unsigned long long s_cursor, s_pool, s_gain, s_best, s_tau, s_fcnt[2];
    __shared__ int s_x, s_filler;
    __shared__ uint32_t s_found, s_stop, s_fill_cnt, s_second, s_xmin, s_resume, s_rcur;
    // size[] and the batch counters live in LDS when the graph is small
    // enough: every pair's search adds to them, and device atomics from
    // different waves on one cache line are serialised.
    __shared__ __align__(8) uint32_t s_size[kSkimLdsWords];
    __shared__ __align__(8) uint32_t s_bcnt[kSkimLdsWords];
    __shared__ FlatShared<kSkimBlock> X;
    __shared__ ScanShared C;
    __shared__ uint32_t s_front[2][kSkimLdsFront];
    const uint32_t tid = threadIdx.x;
    const uint32_t n = A.n, k = A.k;
    const bool in_lds = n <= kSkimLdsNodes;
    uint32_t *SZ = in_lds ? s_size : A.size;
    uint32_t *BC = in_lds ? s_bcnt : A.bcnt;
    if (in_lds)
        for (uint32_t w = tid; w < kSkimLdsWords; w += kSkimBlock) {
            s_size[w] = w < (n + 1) / 2 ? ld(A.size + w) : 0u;
            s_bcnt[w] = 0;
        }
    uint32_t *Q = A.queues + (uint64_t)tid * n;
    uint32_t *V = A.vis + (uint64_t)tid * A.vis_words;
    if (tid == 0) {
        s_cursor = A.ctl->cursor;
        s_pool = A.ctl->pool_used;
        s_stop = 0;
        s_found = 0;
        C.ncand = 0;
        // a residual search the grid handed back (its frontier got small):
        // the launch starts by finishing that seed
        s_resume = A.ctl->pend == 2;
        if (s_resume) {
            A.ctl->pend = 0;
            s_x = (int)A.ctl->px;
            s_rcur = A.ctl->rcur;
            s_gain = A.ctl->rgain;
            s_fcnt[s_rcur] = A.ctl->rsize[0];
        }
    }
    __syncthreads();
    // entry t of the batch's searches, laid end to end in thread order
    auto entry = [&](uint64_t t) {
        const uint32_t r = run_of<kSkimBlock>(X.ex, t);
        return ld(A.queues + (uint64_t)r * n + (t - X.ex[r]));
    };
    uint32_t done = 0;
    for (uint32_t it = 0; it < goal; ++it) {
        const bool resumed = it == 0 && s_resume;  // uniform
        if (!resumed) {
        if (tid == 0) {
            s_x = -1;
            s_filler = -1;
        }
        __syncthreads();
        // ------------------------------------------------ scan pairs by rank
        while (s_x < 0 && s_cursor < A.nsrc) {
            const uint64_t cursor = s_cursor;
            const uint64_t left = A.nsrc - cursor;
            const uint32_t B = left < (uint64_t)kSkimBlock ? (uint32_t)left : (uint32_t)kSkimBlock;
            uint32_t cnt = 0, p = 0;
            if (tid < B) {
                p = A.order[cursor + tid];
                if (!ld(A.covered + p)) {
                    const uint32_t i = p % kPairStride;
                    Q[0] = p / kPairStride;
                    mark_new(V, Q[0]);
                    cnt = 1;
                    for (uint32_t head = 0; head < cnt; ++head) {
                        const uint32_t q = Q[head] * kPairStride + i;
                        if (!A.rlive) {
                            for (uint64_t e = A.rptr[q]; e < A.rptr[q + 1]; ++e) {
                                const uint32_t w = A.radj[e];
                                if (mark_new(V, w)) Q[cnt++] = w;
                            }
                            continue;
                        }
                        const uint64_t lw = A.rlive[q];
                        if (lw & kLiveOne) {
                            const uint32_t w = (uint32_t)lw;
                            if (mark_new(V, w)) Q[cnt++] = w;
                        } else {
                            const uint64_t e0 = lw >> kLiveCountBits;
                            const uint64_t e1 = e0 + (lw & ((1u << kLiveCountBits) - 1));
                            for (uint64_t e = e0; e < e1; ++e) {
                                const uint32_t w = A.rsrc[e];
                                if (mark_new(V, w)) Q[cnt++] = w;
                            }
                        }
                    }
                    for (uint32_t j = 0; j < cnt; ++j) V[Q[j] >> 5] = 0u;  // back to zero
                }
            }
            {
                uint64_t tot;
                const uint64_t ex = block_excl_scan<kSkimBlock>(cnt, X.wsum, tot);
                X.ex[tid] = ex;
                if (tid == 0) X.ex[kSkimBlock] = tot;
            }
            const bool heavy = __syncthreads_or(cnt > kSkimSerial) != 0;
            // Does some node reach k within the first T pairs?  Sizes are
            // below k at the start of a batch and grow by one per pair.  The
            // whole batch is tried first; if some node fills, the entries of
            // every such node are kept, and the first filling prefix is the
            // smallest position at which one of them receives its
            // (k - size)-th entry (a search holds a node at most once).  With
            // too many such entries, the prefix is found by binary search.
            bool filled = false;
            uint32_t lo = 0, hi = B, T = B;
            for (;;) {
                const uint64_t end = X.ex[T];
                bool cand = false;
                auto keep = [&](uint32_t r, uint32_t v) {
                    if (T != B) return;
                    const uint32_t slot = atomicAdd(&C.ncand, 1u);
                    if (slot < kSkimCand) C.cand[slot] = ((uint64_t)r << 32) | v;
                };
                if (heavy) {
                    for (uint64_t t = tid; t < end; t += kSkimBlock) cadd(BC, entry(t), 1u);
                    __syncthreads();
                    for (uint64_t t = tid; t < end; t += kSkimBlock) {
                        const uint32_t v = entry(t);
                        if (cget(SZ, v) + cget(BC, v) >= k) {
                            cand = true;
                            keep(run_of<kSkimBlock>(X.ex, t), v);
                        }
                    }
                } else {
                    if (tid < T)
                        for (uint32_t j = 0; j < cnt; ++j) cadd(BC, Q[j], 1u);
                    __syncthreads();
                    if (tid < T)
                        for (uint32_t j = 0; j < cnt; ++j)
                            if (cget(SZ, Q[j]) + cget(BC, Q[j]) >= k) {
                                cand = true;
                                keep(tid, Q[j]);
                            }
                }
                if (__any(cand) && (tid & 63u) == 0) atomicOr(&s_found, 1u);
                __syncthreads();
                const bool f = s_found != 0;
                if (heavy) {
                    for (uint64_t t = tid; t < end; t += kSkimBlock) czero(BC, entry(t));
                } else if (tid < T) {
                    for (uint32_t j = 0; j < cnt; ++j) czero(BC, Q[j]);
                }
                __syncthreads();
                if (tid == 0) s_found = 0;
                __syncthreads();
                if (T == B) {
                    filled = f;
                    if (!f) break;
                    const uint32_t nc = C.ncand;
                    if (nc <= kSkimCand) {
                        if (tid == 0) C.tmin = 0xFFFFFFFFu;
                        __syncthreads();
                        for (uint32_t c = tid; c < nc; c += kSkimBlock) {
                            const uint64_t e = C.cand[c];
                            const uint32_t r = (uint32_t)(e >> 32), v = (uint32_t)e;
                            uint32_t before = 0;  // entries of v at earlier positions
                            for (uint32_t c2 = 0; c2 < nc; ++c2) {
                                const uint64_t e2 = C.cand[c2];
                                before += (uint32_t)e2 == v && (uint32_t)(e2 >> 32) < r;
                            }
                            if (before + 1 == k - cget(SZ, v)) atomicMin(&C.tmin, r);
                        }
                        __syncthreads();
                        hi = C.tmin + 1;
                        break;
                    }
                } else if (f) {
                    hi = T;
                } else {
                    lo = T;
                }
                if (hi - lo <= 1) break;
                T = lo + (hi - lo) / 2;
            }
            T = hi;  // B when nothing fills; else the first filling prefix
            // does the committed prefix fit in the index pool?
            const uint64_t need = X.ex[T], pbase = s_pool;
            if (pbase + need > A.pool_cap) {
                if (tid == 0) {
                    A.ctl->flags |= kFlagPool;
                    A.ctl->need = pbase + need;
                    s_stop = 1;
                }
                __syncthreads();
                break;
            }
            // commit pairs [0, T): index entries in pair order, sizes
            if (heavy) {
                for (uint64_t t = tid; t < need; t += kSkimBlock) {
                    const uint32_t v = entry(t);
                    st(A.pool + pbase + t, v);
                    cadd(SZ, v, 1u);
                }
            } else if (tid < T) {
                for (uint32_t j = 0; j < cnt; ++j) {
                    st(A.pool + pbase + X.ex[tid] + j, Q[j]);
                    cadd(SZ, Q[j], 1u);
                }
            }
            if (tid < T && cnt) {
                st(A.idx + p, ((pbase + X.ex[tid]) << 32) | cnt);
            }
            if (tid == 0) s_xmin = 0xFFFFFFFFu;
            __syncthreads();
            if (filled) {
                // the nodes that just reached k are in pair T - 1's search;
                // the seed is the smallest of them
                if (heavy) {
                    for (uint64_t t = X.ex[T - 1] + tid; t < need; t += kSkimBlock) {
                        const uint32_t v = entry(t);
                        if (cget(SZ, v) >= k) atomicMin(&s_xmin, v);
                    }
                } else if (tid == T - 1) {
                    for (uint32_t j = 0; j < cnt; ++j)
                        if (cget(SZ, Q[j]) >= k) atomicMin(&s_xmin, Q[j]);
                }
                if (tid == T - 1) {
                    s_filler = (int)tid;
                    s_fill_cnt = cnt;
                    s_tau = pair_rank(A.seed, p);
                }
                __syncthreads();
                if (tid == 0) s_x = s_xmin == 0xFFFFFFFFu ? -1 : (int)s_xmin;
            }
            if (tid == 0) {
                s_cursor = cursor + T;
                s_pool = pbase + need;
                C.ncand = 0;
            }
            __syncthreads();
        }
        if (s_stop) break;
        // --------------------------------------------------- exhaustion rule
        if (s_x < 0) {
            if (tid == 0) s_best = 0;
            __syncthreads();
            unsigned long long best = 0;
            for (uint32_t v = tid; v < n; v += kSkimBlock)
                if (!ld(A.sel + v)) {
                    const unsigned long long key =
                        ((unsigned long long)cget(SZ, v) << 32) | (0xFFFFFFFFu - v);
                    best = key > best ? key : best;
                }
            atomicMax(&s_best, best);
            __syncthreads();
            // an unselected node always exists (the host checks s); keep the
            // index in range regardless
            if (tid == 0) {
                const uint32_t v = 0xFFFFFFFFu - (uint32_t)s_best;
                s_x = (s_best && v < n) ? (int)v : 0;
            }
            __syncthreads();
        }
        const uint32_t xs = (uint32_t)s_x;  // the seed
        // ------------------------------------ records for the error estimate
        // The filling pair's search is still in its thread's queue; the batch
        // counters are all zero here and mark it while the sizes are scanned.
        const uint32_t *Qf = s_filler >= 0 ? A.queues + (uint64_t)s_filler * n : nullptr;
        const uint32_t fcnt = s_filler >= 0 ? s_fill_cnt : 0u;
        for (uint32_t j = tid; j < fcnt; j += kSkimBlock) cadd(BC, ld(Qf + j), 1u);
        if (tid == 0) s_second = 0;
        __syncthreads();
        {
            // Selected nodes need no test: every pair a seed reaches is
            // covered, so its size is 0 from then on and no later search
            // reaches it.  Four nodes per 64-bit load (the arrays are padded
            // to whole pairs of words).
            uint32_t best2 = 0;
            const uint64_t *SZ2 = reinterpret_cast<const uint64_t *>(SZ);
            const uint64_t *BC2 = reinterpret_cast<const uint64_t *>(BC);
            // four words per thread in flight at once (a loop of single
            // loads waits for each: 0.1 ms per seed on 10^6 nodes)
            const uint32_t nw = (n + 3) / 4;
            for (uint32_t w0 = tid; w0 < nw; w0 += 4 * kSkimBlock) {
                uint64_t a[4], b[4];
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) {
                    const uint32_t w2 = w0 + u * kSkimBlock;
                    a[u] = w2 < nw ? ld(SZ2 + w2) : 0ull;
                    b[u] = w2 < nw ? ld(BC2 + w2) : 0ull;
                }
#pragma unroll
                for (uint32_t u = 0; u < 4; ++u) {
#pragma unroll
                    for (uint32_t h = 0; h < 4; ++h) {
                        const uint32_t v = 4 * (w0 + u * kSkimBlock) + h;
                        const uint32_t sz = (uint32_t)((a[u] >> (16 * h)) & 0xFFFFu) -
                                            (uint32_t)((b[u] >> (16 * h)) & 0xFFFFu);
                        if (v < n && v != xs && sz > best2) best2 = sz;
                    }
                }
            }
            // one LDS atomic per wave: lanes on one address are serialised
            for (int off = 32; off > 0; off >>= 1) {
                const uint32_t o = (uint32_t)__shfl_xor((int)best2, off);
                best2 = o > best2 ? o : best2;
            }
            if ((tid & 63) == 0 && best2) atomicMax(&s_second, best2);
        }
        __syncthreads();
        for (uint32_t j = tid; j < fcnt; j += kSkimBlock) czero(BC, ld(Qf + j));
        if (tid == 0) {
            rec_tau[it] = s_filler >= 0 ? (uint64_t)s_tau : ~0ull;
            rec_second[it] = s_second;
        }
        }  // !resumed
        const uint32_t x = (uint32_t)s_x;
        // ------------------------------------------------- residual problem
        // Level-synchronous over all instances at once: a frontier of pairs
        // (64 v + i) in two halves of the queue area (free here: the scan's
        // searches are done and the filler's queue has been read).  A pair is
        // claimed by the CAS that covers it; its index entry is erased then.
        // A level with more than `handoff` pairs (0: none) and the rest of
        // the search go to the whole grid (k_resid_level); the host then
        // completes the seed.
        uint32_t *F[2] = {A.queues, A.queues + (uint64_t)A.n * kPairStride};
        if (!resumed) {
        if (tid == 0) {
            s_gain = 0;
            s_fcnt[0] = 0;
        }
        __syncthreads();
        {
            bool add = false;
            uint32_t px = 0;
            if (tid < A.ell) {
                px = x * kPairStride + tid;
                add = atomicCAS(A.covered + px, 0u, 1u) == 0u;
            }
            if (tid < 64) {  // the first wave holds every instance (l <= 64)
                const uint64_t slot = wave_reserve(&s_fcnt[0], add);
                if (add) s_front[0][slot] = px;
            }
        }
        } else {
            // the grid left the pending level in the queue area
            const uint64_t fc = s_fcnt[s_rcur];
            for (uint32_t e = tid; e < fc && e < kSkimLdsFront; e += kSkimBlock)
                s_front[s_rcur][e] = F[s_rcur][e];
        }
        bool handed = false;
        const uint64_t seed_edges = A.fptr[(uint64_t)x * kPairStride + kPairStride] -
                                    A.fptr[(uint64_t)x * kPairStride];
        // a resumed search continues at its pending level (not level 0)
        for (uint32_t cur = resumed ? s_rcur : 0u, level = resumed ? 1u : 0u;;
             cur ^= 1u, ++level) {
            __syncthreads();
            // (the counter reset below is of the next level's counter, read
            // by nobody in this level)
            const uint64_t fc = s_fcnt[cur];
            if (fc == 0) break;
            if (handoff && (fc > handoff || (level == 0 && seed_edges > kSkimHandoffEdges))) {
                // the grid reads the level from the queue area
                for (uint32_t e = tid; e < fc && e < kSkimLdsFront; e += kSkimBlock)
                    st(F[cur] + e, s_front[cur][e]);
                if (tid == 0) {
                    A.ctl->pend = 1;
                    A.ctl->px = x;
                    A.ctl->rcur = cur;
                    A.ctl->rsize[0] = fc;
                    A.ctl->rsize[16] = 0;
                    A.ctl->rsize[32] = 0;
                    A.ctl->hsize[0] = A.ctl->hsize[16] = A.ctl->hsize[32] = 0;
                    A.ctl->rgain = s_gain;
                }
                handed = true;
                break;
            }
            if (tid == 0) {
                s_fcnt[cur ^ 1u] = 0;
                s_gain += fc;
            }
            for (uint64_t base = 0; base < fc; base += kSkimBlock)
                resid_chunk<kSkimBlock, false>(A, SZ, F[cur], F[cur ^ 1u], fc, base, X,
                                               &s_fcnt[cur ^ 1u], nullptr, nullptr, nullptr,
                                               s_front[cur], s_front[cur ^ 1u]);
        }
        if (handed) break;  // uniform
        __syncthreads();
        if (tid == 0) {
            st(A.sel + x, 1u);
            seeds[it] = x;
            gains[it] = s_gain;
            if (gain_d) gain_d[it] = (double)s_gain / (double)A.ell;
        }
        ++done;
        __syncthreads();
    }
    if (in_lds) {
        __syncthreads();
        for (uint32_t w = tid; w < (n + 1) / 2; w += kSkimBlock) st(A.size + w, s_size[w]);
    }
    if (tid == 0) {
        A.ctl->cursor = s_cursor;
        A.ctl->pool_used = s_pool;
        A.ctl->done = done;
    }
}

// Level L of a residual search handed over by k_skim, on the whole grid:
// frontier buffer (r0 + L) & 1 of the queue area, sizes in global memory.
// First the pairs level L - 1 deferred (long out-lists), their edges laid end
// to end and split evenly over every workgroup, kResidBlock pairs at a time;
// then the level's own frontier.  Both append to level L + 1.  A launch with
// nothing to do returns at once, so the host launches levels in batches and
// reads the sizes back after each batch.
__global__ void __launch_bounds__(kResidBlock) k_resid_level(SkArgs A, uint32_t L, uint32_t r0) {
    __shared__ FlatShared<kResidBlock> X;
    __shared__ ResidStage S;
    __shared__ unsigned long long s_fc, s_nh;
    const uint32_t tid = threadIdx.x;
    if (tid == 0) {
        S.n = 0;
        s_fc = ld(&A.ctl->rsize[16 * (L % 3)]);
        s_nh = ld(&A.ctl->hsize[16 * ((L + 2) % 3)]);  // deferred by level L - 1
        if (blockIdx.x == 0) {
            A.ctl->rsize[16 * ((L + 2) % 3)] = 0;  // level L + 1 appends there
            A.ctl->hsize[16 * ((L + 1) % 3)] = 0;  // and defers there
            A.ctl->rgain += s_fc;
        }
    }
    __syncthreads();
    const uint64_t fc = s_fc;
    const uint32_t nh = s_nh < kHeavyItems ? (uint32_t)s_nh : kHeavyItems;
    if (fc == 0 && nh == 0) return;  // uniform
    const uint32_t cur = (r0 + L) & 1u;
    const uint64_t half = (uint64_t)A.n * kPairStride;
    const uint32_t *Fin = A.queues + cur * half;
    uint32_t *Fout = A.queues + (cur ^ 1u) * half;
    unsigned long long *next = &A.ctl->rsize[16 * ((L + 1) % 3)];
    const uint64_t *hin = A.heavy + 2 * (uint64_t)kHeavyItems * ((L + 2) % 3);
    for (uint32_t h0 = 0; h0 < nh; h0 += kResidBlock) {
        uint64_t deg = 0, f0 = 0;
        uint32_t q = 0;
        if (h0 + tid < nh) {
            const uint64_t w = hin[2 * (h0 + tid)];
            q = (uint32_t)(w >> 32);
            deg = (uint32_t)w;
            f0 = hin[2 * (h0 + tid) + 1];
        }
        uint64_t tot;
        const uint64_t e = block_excl_scan<kResidBlock>(deg, X.wsum, tot);
        X.ex[tid] = e;
        X.q[tid] = q;
        X.f0[tid] = f0;
        if (tid == 0) X.ex[kResidBlock] = tot;
        __syncthreads();
        const uint64_t a = tot * blockIdx.x / gridDim.x, b = tot * (blockIdx.x + 1) / gridDim.x;
        for (uint64_t base = a; base < b; base += kResidBlock) {
            const uint64_t t = base + tid;
            bool add = false;
            uint32_t qw = 0;
            if (t < b) {
                const uint32_t r = run_of<kResidBlock>(X.ex, t);
                qw = A.fadj[X.f0[r] + (t - X.ex[r])] * kPairStride + X.q[r] % kPairStride;
                add = !ld(A.covered + qw) && atomicCAS(A.covered + qw, 0u, 1u) == 0u;
            }
            const unsigned long long m = __ballot(add);
            if (m) {
                const int leader = __ffsll((long long)m) - 1;
                const uint32_t lane = lane_id();
                uint32_t pos0 = 0;
                if ((int)lane == leader) pos0 = atomicAdd(&S.n, (uint32_t)__popcll(m));
                const uint32_t pos = (uint32_t)__shfl((int)pos0, leader) +
                                     (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
                if (add) {
                    if (pos < 8 * kResidBlock) S.buf[pos] = qw;
                    else Fout[atomicAdd(next, 1ull)] = qw;
                }
            }
            __syncthreads();
            const uint32_t ns = S.n < 8 * kResidBlock ? S.n : 8 * kResidBlock;
            __syncthreads();  // every thread has read S.n: the test below is uniform
            if (ns > 7 * kResidBlock || base + kResidBlock >= b) {
                if (tid == 0 && ns) S.base = atomicAdd(next, (unsigned long long)ns);
                __syncthreads();
                for (uint32_t j = tid; j < ns; j += kResidBlock) Fout[S.base + j] = S.buf[j];
                __syncthreads();
                if (tid == 0) S.n = 0;
                __syncthreads();
            }
        }
        __syncthreads();  // X is reused
    }
    uint64_t *hout = A.heavy + 2 * (uint64_t)kHeavyItems * (L % 3);
    for (uint64_t base = (uint64_t)blockIdx.x * kResidBlock; base < fc;
         base += (uint64_t)gridDim.x * kResidBlock)
        resid_chunk<kResidBlock, true>(A, A.size, Fin, Fout, fc, base, X, next, &S,
                                       &A.ctl->hsize[16 * (L % 3)], hout);
}

// The handed-over search's next level (L) is small: k_skim finishes it.
__global__ void k_resid_handback(SkArgs A, uint32_t L, uint32_t r0) {
    A.ctl->rsize[0] = A.ctl->rsize[16 * (L % 3)];
    A.ctl->rcur = (r0 + L) & 1u;
    A.ctl->pend = 2;
}

// The handed-over seed is complete: outputs, and the node leaves the
// candidates.
__global__ void k_resid_finish(SkArgs A, uint32_t *seeds, uint64_t *gains, double *gain_d) {
    const uint32_t x = A.ctl->px;
    const unsigned long long g = A.ctl->rgain;
    A.sel[x] = 1u;
    seeds[0] = x;
    gains[0] = g;
    if (gain_d) gain_d[0] = (double)g / (double)A.ell;
    A.ctl->pend = 0;
}

__global__ void k_pair_keys(uint32_t n, uint32_t ell, uint64_t seed, uint64_t *keys,
                            uint32_t *vals) {
    const uint64_t total = (uint64_t)n * ell;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < total;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p = (uint32_t)(t / ell) * kPairStride + (uint32_t)(t % ell);
        keys[t] = pair_rank(seed, p);
        vals[t] = p;
    }
}

// The pairs are radix-sorted on the high halves of their ranks only (four
// passes instead of eight).  Equal high halves are rare (about (n l)^2 / 2^33
// pairs of pairs for uniform ranks); the thread at the start of each such run
// puts it in full-rank order by a stable insertion sort, which gives exactly
// the order of a full sort (by rank, then by pair as listed).  Within a run
// the high halves are all equal, so the other threads' run tests read the
// same values whatever the owners are moving.
constexpr uint64_t kHalfSortPairs = 1ull << 21;
__global__ void k_rank_ties(uint64_t *keys, uint32_t *vals, uint64_t count) {
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t + 1 < count;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t hi = (uint32_t)(keys[t] >> 32);
        if ((uint32_t)(keys[t + 1] >> 32) != hi) continue;   // no tie follows
        if (t > 0 && (uint32_t)(keys[t - 1] >> 32) == hi) continue;  // not the run's start
        uint64_t e = t + 2;
        while (e < count && (uint32_t)(keys[e] >> 32) == hi) ++e;
        for (uint64_t i = t + 1; i < e; ++i) {
            const uint64_t key = keys[i];
            const uint32_t val = vals[i];
            uint64_t j = i;
            for (; j > t && keys[j - 1] > key; --j) {
                keys[j] = keys[j - 1];
                vals[j] = vals[j - 1];
            }
            keys[j] = key;
            vals[j] = val;
        }
    }
}

// ------------------------------------------------ adaptive error estimate
// Section 4 (adaptive error estimation), eq. (chernoff).  Discrepancies are
// counted on a grid of step h = max_rel_error * I / bins pairs, I the sum of
// the gains; every distribution is held as its survival function
// S[j] = P[D >= j h], j = 0..bins, with everything at or beyond bins * h kept
// in the last cell.

constexpr uint32_t kTailMaxBins = 1u << 16;
constexpr uint64_t kTailMaxCells = 1ull << 30;  // seeds * (bins + 1)
constexpr int kTailBlock = 256;

__global__ void __launch_bounds__(kTailBlock) k_tail_total(uint32_t s, const uint64_t *gain,
                                                           uint64_t *total) {
    __shared__ unsigned long long acc;
    if (threadIdx.x == 0) acc = 0;
    __syncthreads();
    unsigned long long t = 0;
    for (uint32_t r = threadIdx.x; r < s; r += kTailBlock) t += gain[r];
    atomicAdd(&acc, t);
    __syncthreads();
    if (threadIdx.x == 0) *total = acc;
}

// eq. (chernoff) with Z = z and nu = 1 - z / mu, in logarithms:
// (e^-nu / (1 - nu)^(1 - nu))^mu = exp(z - mu + z ln(mu / z)); 1 when z >= mu.
__device__ __forceinline__ double chernoff_bound(double mu, double z) {
    if (z >= mu) return 1.0;
    if (z == 0.0) return exp(-mu);
    return exp(z - mu + z * log(mu / z));
}

// S_r[j] >= P[D_r > (j-1) h] for record r: a seed whose sketch filled at rank
// tau with second largest sketch k' and gain Delta has
// P[D > eps Delta] <= bound(mu = rho(tau) Delta (1 + eps), k').  An exhaustion
// seed (tau = all ones) is exact (D = 0); a filled record with no gain gives
// no bound (S = 1).
__global__ void __launch_bounds__(kTailBlock) k_tail_survival(
    uint32_t s, const uint64_t *tau, const uint32_t *second, const uint64_t *gain,
    const uint64_t *total, uint32_t bins, double max_rel, double *S) {
    const uint64_t W = (uint64_t)bins + 1, work = (uint64_t)s * W;
    const uint64_t I = *total;
    const double h = max_rel * (double)I / (double)bins;
    for (uint64_t t = blockIdx.x * (uint64_t)kTailBlock + threadIdx.x; t < work;
         t += (uint64_t)gridDim.x * kTailBlock) {
        const uint64_t r = t / W;
        const uint32_t j = (uint32_t)(t - r * W);
        double v;
        if (j == 0) {
            v = 1.0;
        } else if (I == 0 || tau[r] == ~0ull) {
            v = 0.0;
        } else if (gain[r] == 0) {
            v = 1.0;
        } else {
            const double d = (double)gain[r];
            const double rho = (double)((tau[r] >> 11) + 1) * 0x1p-53;
            const double eps = (double)(j - 1) * h / d;
            const double mu = rho * d * (1.0 + eps);
            v = fmin(1.0, chernoff_bound(mu, (double)second[r]));
        }
        S[t] = v;
    }
}

// One level of the pairwise tree: out[p] = the capped sum of rows 2p and
// 2p+1 of in (an odd last row is copied).  With a[i] = Sa[i] - Sa[i+1],
//   Sc[j] = P[A + B >= j] = Sa[j+1] + sum_{i <= j} a[i] Sb[j-i],  Sa[bins+1] = 0.
// A workgroup owns kTailOut consecutive outputs j0.. of one pair; each of its
// kTailGroups waves takes the i tiles g, g + kTailGroups, ... of kTailI
// values, and lane l of a wave keeps the partial sums of the kTailPer
// consecutive outputs j0 + kTailPer l + c.  As i steps by one, the Sb values
// those outputs need slide by one place, so a lane holds them in registers
// and reads one new value per step.  A tile's a[i] and the Sb values it
// meets, Sb[j0 - i0 - kTailI + u] for u = 0 .. kTailOut + kTailI - 1 (zero
// outside 0 .. bins: below 0 this drops the terms with i > j), sit in the
// wave's LDS with u interleaved by u mod kTailPer, so the lanes of a wave
// read consecutive words.  The waves' partial sums are added in a fixed order
// at the end, so the result does not depend on scheduling.
constexpr int kTailGroups = 8, kTailPairBlock = 64 * kTailGroups;
constexpr int kTailPer = 4, kTailOut = 64 * kTailPer, kTailI = 256;
constexpr int kTailSpan = kTailOut + kTailI, kTailStride = kTailSpan / kTailPer;

__device__ __forceinline__ int tail_pos(int u) { return (u % kTailPer) * kTailStride + u / kTailPer; }

__global__ void __launch_bounds__(kTailPairBlock) k_tail_pair(const double *in, double *out,
                                                              uint32_t rows, uint32_t bins) {
    __shared__ double s_a[kTailGroups][kTailI];
    __shared__ double s_b[kTailGroups][kTailSpan];
    const uint64_t W = (uint64_t)bins + 1;
    const uint64_t outs = ((uint64_t)rows + 1) / 2;
    const uint64_t chunks = (W + kTailOut - 1) / kTailOut, nblk = outs * chunks;
    const int g = (int)threadIdx.x / 64, lane = (int)threadIdx.x % 64;
    for (uint64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
        const uint64_t p = blk / chunks;
        const int64_t j0 = (int64_t)(blk - p * chunks) * kTailOut;
        const int64_t j1 = j0 + kTailOut < (int64_t)W ? j0 + kTailOut : (int64_t)W;
        const double *a = in + 2 * p * W;
        double *o = out + p * W;
        if (2 * p + 1 >= rows) {
            for (int64_t j = j0 + threadIdx.x; j < j1; j += kTailPairBlock) o[j] = a[j];
            continue;
        }
        const double *b = a + W;
        double acc[kTailPer];
#pragma unroll
        for (int c = 0; c < kTailPer; ++c) acc[c] = 0.0;
        const int64_t tiles = (j1 + kTailI - 1) / kTailI;  // tiles with i0 < j1
        for (int64_t round = 0; round * kTailGroups < tiles; ++round) {
            const int64_t i0 = (round * kTailGroups + g) * kTailI;
            const bool active = i0 < j1;
            __syncthreads();  // the previous tiles are consumed
            if (active) {
                for (int t = lane; t < kTailI; t += 64) {
                    const int64_t i = i0 + t;
                    s_a[g][t] =
                        i < (int64_t)W ? a[i] - (i + 1 < (int64_t)W ? a[i + 1] : 0.0) : 0.0;
                }
                const int64_t base = j0 - i0 - kTailI;
                for (int u = lane; u < kTailSpan; u += 64) {
                    const int64_t q = base + u;
                    s_b[g][tail_pos(u)] = q >= 0 && q < (int64_t)W ? b[q] : 0.0;
                }
            }
            __syncthreads();
            if (active) {
                // output j0 + kTailPer lane + c at step t needs u = kTailPer lane + c + kTailI - t
                const double *sa = s_a[g];
                const double *sb = s_b[g];
                double w[kTailPer];
#pragma unroll
                for (int c = 0; c < kTailPer; ++c) w[c] = sb[tail_pos(kTailPer * lane + c + kTailI)];
#pragma unroll 8
                for (int t = 0; t < kTailI; ++t) {
                    const double at = sa[t];
#pragma unroll
                    for (int c = 0; c < kTailPer; ++c) acc[c] += at * w[c];
#pragma unroll
                    for (int c = kTailPer - 1; c > 0; --c) w[c] = w[c - 1];
                    w[0] = sb[tail_pos(kTailPer * lane + kTailI - 1 - t)];
                }
            }
        }
        // fixed-order reduction over the waves, through the staging LDS
        __syncthreads();
        double *red = &s_b[0][0];
#pragma unroll
        for (int c = 0; c < kTailPer; ++c) red[g * kTailOut + kTailPer * lane + c] = acc[c];
        __syncthreads();
        for (int jj = threadIdx.x; jj < kTailOut; jj += kTailPairBlock) {
            const int64_t j = j0 + jj;
            if (j < j1) {
                double v = j + 1 < (int64_t)W ? a[j + 1] : 0.0;
                for (int q = 0; q < kTailGroups; ++q) v += red[q * kTailOut + jj];
                o[j] = v;
            }
        }
        __syncthreads();  // LDS is reused by the next block of the stride
    }
}

}  // namespace

}  // namespace skim

struct skim_greedy_state {
    int device = 0;
    std::unique_ptr<skim::Arena> mem;
    uint32_t n = 0, ell = 0, k = 0;
    uint64_t seed = 0, m = 0;
    const uint64_t *row_ptr = nullptr;
    const uint32_t *col = nullptr;
    const uint32_t *thr = nullptr;
    uint32_t selected = 0;
    skim::SkArgs args{};
};

namespace skim {

skim_greedy_state *greedy_create(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed,
                                        hipStream_t s) {
    SKIM_REQUIRE(ell >= 1 && ell <= 64, "l must be in [1, 64]");
    // sizes and batch counters are 16-bit halves of words
    SKIM_REQUIRE(k >= 2 && k <= 65535, "k must be in [2, 65535]");
    SKIM_REQUIRE(g != nullptr, "graph is NULL");
    if ((uint64_t)g->n > (1ull << 22)) {
        set_error("skim_greedy supports n <= 4194304 (per-thread search queues of n entries)");
        throw Fail{SKIM_EUNSUPPORTED};
    }
    auto st = std::make_unique<skim_greedy_state>();
    SKIM_HIP(hipGetDevice(&st->device));
    st->mem = std::make_unique<Arena>(s, /*persistent=*/true);
    Arena &M = *st->mem;
    const uint32_t n = g->n;
    {
        Arena T(s);
        uint32_t *esrc = T.alloc<uint32_t>(g->m ? g->m : 1);
        validate_graph(g, esrc, T);
        // on large graphs the in-lists as the sketch build makes them and the
        // out-lists by the same chunked passes (no atomic per entry, scratch
        // in T); on small ones both from one coin pass (fewer launches)
        LiveLists fwd;
        if (n >= kSkimPairListNodes) {
            const PairLists rev = build_pair_lists(g, ell, seed, esrc, T, &M);
            fwd = build_out_lists(g, ell, seed, esrc, T, &M);
            st->args.rlive = rev.live;
            st->args.rsrc = rev.adj;
        } else {
            const LiveLists rev = build_live_lists(g, ell, seed, esrc, /*forward=*/false, M, &fwd);
            st->args.rptr = rev.ptr;
            st->args.radj = rev.adj;
        }
        st->args.fptr = fwd.ptr;
        st->args.fadj = fwd.adj;
        // pairs by increasing rank
        const uint64_t nsrc = (uint64_t)n * ell;
        uint64_t *keys = T.alloc<uint64_t>(nsrc);
        uint64_t *keys2 = T.alloc<uint64_t>(nsrc);
        uint32_t *vals = T.alloc<uint32_t>(nsrc);
        uint32_t *order = M.alloc<uint32_t>(nsrc);
        k_pair_keys<<<grid_for(nsrc, 256, 8192), 256, 0, s>>>(n, ell, seed, keys, vals);
        SKIM_LAUNCH_CHECK();
        size_t tmp_bytes = 0;
        // large sorts on the high halves (then k_rank_ties); small ones go to
        // another rocPRIM algorithm, which on the high halves alone did not
        // order the pairs of a 1000-node graph, and are cheap: the whole rank
        const unsigned begin_bit = nsrc > kHalfSortPairs ? 32u : 0u;
        SKIM_HIP(rocprim::radix_sort_pairs(nullptr, tmp_bytes, keys, keys2, vals, order, (size_t)nsrc,
                                           begin_bit, 64u, s));
        void *tmp = T.get(tmp_bytes);
        SKIM_HIP(rocprim::radix_sort_pairs(tmp, tmp_bytes, keys, keys2, vals, order, (size_t)nsrc,
                                           begin_bit, 64u, s));
        if (begin_bit) {
            k_rank_ties<<<grid_for(nsrc, 256, 8192), 256, 0, s>>>(keys2, order, nsrc);
            SKIM_LAUNCH_CHECK();
        }
        SKIM_HIP(hipStreamSynchronize(s));
        st->args.order = order;
        st->args.nsrc = nsrc;
    }
    const uint64_t npairs = (uint64_t)n * kPairStride;
    SkArgs &A = st->args;
    A.n = n;
    A.ell = ell;
    A.k = k;
    A.covered = M.alloc<uint32_t>(npairs);
    const uint64_t cwords = 2 * (((uint64_t)n + 3) / 4);  // whole 64-bit words
    A.size = M.alloc<uint32_t>(cwords);
    A.sel = M.alloc<uint32_t>(n);
    A.idx = M.alloc<uint64_t>(npairs);
    A.heavy = M.alloc<uint64_t>(3 * 2 * (uint64_t)kHeavyItems);
    A.bcnt = M.alloc<uint32_t>(cwords);
    A.queues = M.alloc<uint32_t>((uint64_t)kSkimBlock * n);
    A.vis_words = (n + 31) / 32;
    A.vis = M.alloc<uint32_t>((uint64_t)kSkimBlock * A.vis_words);
    fill_u32(A.vis, 0, (uint64_t)kSkimBlock * A.vis_words, s);
    A.pool_cap = std::max<uint64_t>(1ull << 16, 2 * A.nsrc);
    A.pool = M.alloc<uint32_t>(A.pool_cap);
    A.ctl = M.alloc<SkCtl>(1);
    A.seed = seed;
    A.rec_tau = M.alloc<uint64_t>(n);
    A.rec_second = M.alloc<uint32_t>(n);
    fill_u32(A.covered, 0, npairs, s);
    fill_u32(A.size, 0, cwords, s);
    fill_u32(A.sel, 0, n, s);
    fill_u64(A.idx, 0, npairs, s);
    fill_u32(A.bcnt, 0, cwords, s);
    fill_u64((uint64_t *)A.ctl, 0, sizeof(SkCtl) / 8, s);
    st->n = n;
    st->ell = ell;
    st->k = k;
    st->seed = seed;
    st->m = g->m;
    st->row_ptr = g->row_ptr;
    st->col = g->col;
    st->thr = g->thr;
    SKIM_HIP(hipStreamSynchronize(s));
    return st.release();
}

void greedy_run(skim_greedy_state *st, uint32_t s_goal, uint32_t *seeds, uint64_t *gains,
                       double *gain_d, hipStream_t s) {
    SkArgs &A = st->args;
    uint32_t done = 0;
    int growths = 0;
    while (done < s_goal) {
        k_skim<<<1, kSkimBlock, 0, s>>>(A, s_goal - done, kSkimHandoff, seeds + done,
                                        gains + done, gain_d ? gain_d + done : nullptr,
                                        A.rec_tau + st->selected, A.rec_second + st->selected);
        SKIM_LAUNCH_CHECK();
        SkCtl c;
        read_back(&c, A.ctl, sizeof c, s);
        done += c.done;
        st->selected += c.done;
        if (c.flags & kFlagPool) {
            SKIM_REQUIRE(++growths < 40, "SKIM index pool did not converge");
            // grow the inverted-index pool, keep its contents, continue
            const uint64_t cap = std::max<uint64_t>(2 * A.pool_cap, c.need + c.need / 2);
            uint32_t *np = st->mem->alloc<uint32_t>(cap);
            SKIM_HIP(hipMemcpyAsync(np, A.pool, c.pool_used * sizeof(uint32_t),
                                    hipMemcpyDeviceToDevice, s));
            st->mem->release(A.pool);
            A.pool = np;
            A.pool_cap = cap;
            fill_u32(&A.ctl->flags, 0, 1, s);
        } else if (c.pend) {
            // the seed's residual search continues on the whole grid, levels
            // in batches (an empty level's launch does nothing); every level
            // covers at least one new pair
            const uint64_t max_levels = (uint64_t)A.n * kPairStride + 1;
            const uint32_t r0 = c.rcur;
            uint32_t L = 0;
            bool back = false;
            for (;;) {
                for (int j = 0; j < 8; ++j, ++L) {
                    k_resid_level<<<kResidGrid, kResidBlock, 0, s>>>(A, L, r0);
                    SKIM_LAUNCH_CHECK();
                }
                read_back(&c, A.ctl, sizeof c, s);
                // level L's frontier, and the pairs level L - 1 deferred
                const uint64_t f = c.rsize[16 * (L % 3)], h = c.hsize[16 * ((L + 2) % 3)];
                if (f == 0 && h == 0) break;
                if (h == 0 && f <= kSkimHandBack) {  // k_skim resumes the search at level L
                    k_resid_handback<<<1, 1, 0, s>>>(A, L, r0);
                    SKIM_LAUNCH_CHECK();
                    back = true;
                    break;
                }
                SKIM_REQUIRE(L < max_levels, "SKIM residual search did not end");
            }
            if (back) continue;
            k_resid_finish<<<1, 1, 0, s>>>(A, seeds + done, gains + done,
                                           gain_d ? gain_d + done : nullptr);
            SKIM_LAUNCH_CHECK();
            ++done;
            ++st->selected;
        } else if (done < s_goal) {
            set_error("SKIM stopped early");
            throw Fail{SKIM_EDEVICE};
        }
    }
}

}  // namespace skim

extern "C" skim_status skim_greedy(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed,
                                   uint32_t s, uint32_t *seeds, uint64_t *gain_pairs, double *gain,
                                   skim_greedy_state **state, void *stream) {
    skim::clear_error();
    hipStream_t hs = (hipStream_t)stream;
    skim_greedy_state *own = nullptr;
    try {
        SKIM_REQUIRE(s == 0 || (seeds && gain_pairs), "seeds/gain_pairs is NULL");
        skim_greedy_state *st = state ? *state : nullptr;
        if (st) {
            SKIM_REQUIRE(g && g->n == st->n && g->m == st->m && g->row_ptr == st->row_ptr &&
                             g->col == st->col && g->thr == st->thr && ell == st->ell &&
                             k == st->k && seed == st->seed,
                         "resumed state belongs to a different graph or parameters");
        } else {
            st = skim::greedy_create(g, ell, k, seed, hs);
            own = st;
        }
        SKIM_REQUIRE(s <= st->n - st->selected, "s exceeds the number of unselected nodes");
        if (s) skim::greedy_run(st, s, seeds, gain_pairs, gain, hs);
        SKIM_HIP(hipStreamSynchronize(hs));
        if (state) *state = st;
        else delete st;
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        if (own && !(state && *state == own)) delete own;
        return f.st;
    }
}

extern "C" void skim_greedy_state_free(skim_greedy_state *state) { delete state; }

extern "C" uint32_t skim_greedy_state_selected(const skim_greedy_state *state) {
    return state ? state->selected : 0;
}

// ------------------------------------------------- suspend / resume a run
// A saved state: a header, then the run's progress arrays, each at an
// offset rounded up to 8 bytes.
namespace skim {
namespace {

constexpr char kImageMagic[8] = {'S', 'K', 'I', 'M', 'G', 'R', 'D', '1'};

struct ImageHeader {
    char magic[8];
    uint32_t n, ell, k, pad;
    uint64_t m, seed, selected, cursor, pool_used;
};

struct ImageLayout {
    uint64_t covered, size, sel, idx, pool, tau, second, total;
};

uint64_t round8(uint64_t x) { return (x + 7) & ~7ull; }

ImageLayout image_layout(uint32_t n, uint64_t selected, uint64_t pool_used) {
    const uint64_t npairs = (uint64_t)n * kPairStride, cwords = 2 * (((uint64_t)n + 3) / 4);
    ImageLayout L;
    L.covered = round8(sizeof(ImageHeader));
    L.size = round8(L.covered + npairs * 4);
    L.sel = round8(L.size + cwords * 4);
    L.idx = round8(L.sel + (uint64_t)n * 4);
    L.pool = round8(L.idx + npairs * 8);
    L.tau = round8(L.pool + pool_used * 4);
    L.second = round8(L.tau + selected * 8);
    L.total = round8(L.second + selected * 4);
    return L;
}

}  // namespace
}  // namespace skim

extern "C" skim_status skim_greedy_state_save(const skim_greedy_state *state, void *buf,
                                              uint64_t *bytes, void *stream) {
    skim::clear_error();
    hipStream_t hs = (hipStream_t)stream;
    try {
        SKIM_REQUIRE(state != nullptr && bytes != nullptr, "state or bytes is NULL");
        const skim::SkArgs &A = state->args;
        skim::SkCtl c;
        skim::read_back(&c, A.ctl, sizeof c, hs);
        const skim::ImageLayout L = skim::image_layout(state->n, state->selected, c.pool_used);
        if (!buf) {
            *bytes = L.total;
            return SKIM_OK;
        }
        SKIM_REQUIRE(*bytes >= L.total, "buffer of %llu bytes; the state needs %llu",
                     (unsigned long long)*bytes, (unsigned long long)L.total);
        uint8_t *b = (uint8_t *)buf;
        skim::ImageHeader h{};
        std::memcpy(h.magic, skim::kImageMagic, sizeof h.magic);
        h.n = state->n;
        h.ell = state->ell;
        h.k = state->k;
        h.m = state->m;
        h.seed = state->seed;
        h.selected = state->selected;
        h.cursor = c.cursor;
        h.pool_used = c.pool_used;
        std::memcpy(b, &h, sizeof h);
        const uint64_t npairs = (uint64_t)state->n * skim::kPairStride;
        const uint64_t cwords = 2 * (((uint64_t)state->n + 3) / 4);
        const struct {
            uint64_t off;
            const void *src;
            uint64_t len;
        } parts[] = {{L.covered, A.covered, npairs * 4},
                     {L.size, A.size, cwords * 4},
                     {L.sel, A.sel, (uint64_t)state->n * 4},
                     {L.idx, A.idx, npairs * 8},
                     {L.pool, A.pool, c.pool_used * 4},
                     {L.tau, A.rec_tau, (uint64_t)state->selected * 8},
                     {L.second, A.rec_second, (uint64_t)state->selected * 4}};
        for (const auto &pt : parts)
            if (pt.len)
                SKIM_HIP(hipMemcpyAsync(b + pt.off, pt.src, pt.len, hipMemcpyDeviceToHost, hs));
        SKIM_HIP(hipStreamSynchronize(hs));
        *bytes = L.total;
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        return f.st;
    }
}

extern "C" skim_status skim_greedy_state_load(const skim_graph *g, uint32_t ell, uint32_t k,
                                              uint64_t seed, const void *buf, uint64_t bytes,
                                              skim_greedy_state **state, void *stream) {
    skim::clear_error();
    hipStream_t hs = (hipStream_t)stream;
    skim_greedy_state *st = nullptr;
    try {
        SKIM_REQUIRE(g != nullptr && buf != nullptr && state != nullptr,
                     "graph, buffer or state is NULL");
        SKIM_REQUIRE(bytes >= sizeof(skim::ImageHeader), "buffer too small for a saved state");
        skim::ImageHeader h;
        std::memcpy(&h, buf, sizeof h);
        SKIM_REQUIRE(std::memcmp(h.magic, skim::kImageMagic, sizeof h.magic) == 0,
                     "not a saved SKIM state");
        SKIM_REQUIRE(h.n == g->n && h.m == g->m && h.ell == ell && h.k == k && h.seed == seed,
                     "the saved state belongs to another graph or parameters");
        SKIM_REQUIRE(h.selected <= h.n && h.cursor <= (uint64_t)h.n * ell,
                     "saved state is inconsistent");
        const skim::ImageLayout L = skim::image_layout(h.n, h.selected, h.pool_used);
        SKIM_REQUIRE(bytes >= L.total, "saved state truncated (%llu of %llu bytes)",
                     (unsigned long long)bytes, (unsigned long long)L.total);
        st = skim::greedy_create(g, ell, k, seed, hs);
        skim::SkArgs &A = st->args;
        if (h.pool_used > A.pool_cap) {
            const uint64_t cap = h.pool_used + h.pool_used / 2;
            uint32_t *np = st->mem->alloc<uint32_t>(cap);
            st->mem->release(A.pool);
            A.pool = np;
            A.pool_cap = cap;
        }
        const uint8_t *b = (const uint8_t *)buf;
        const uint64_t npairs = (uint64_t)h.n * skim::kPairStride;
        const uint64_t cwords = 2 * (((uint64_t)h.n + 3) / 4);
        const struct {
            void *dst;
            uint64_t off, len;
        } parts[] = {{A.covered, L.covered, npairs * 4},
                     {A.size, L.size, cwords * 4},
                     {A.sel, L.sel, (uint64_t)h.n * 4},
                     {A.idx, L.idx, npairs * 8},
                     {A.pool, L.pool, h.pool_used * 4},
                     {A.rec_tau, L.tau, h.selected * 8},
                     {A.rec_second, L.second, h.selected * 4}};
        for (const auto &pt : parts)
            if (pt.len)
                SKIM_HIP(hipMemcpyAsync(pt.dst, b + pt.off, pt.len, hipMemcpyHostToDevice, hs));
        skim::SkCtl c{};
        c.cursor = h.cursor;
        c.pool_used = h.pool_used;
        SKIM_HIP(hipMemcpyAsync(A.ctl, &c, sizeof c, hipMemcpyHostToDevice, hs));
        SKIM_HIP(hipStreamSynchronize(hs));
        st->selected = (uint32_t)h.selected;
        *state = st;
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        delete st;
        return f.st;
    }
}

extern "C" skim_status skim_greedy_records(const skim_greedy_state *state, uint32_t first,
                                           uint32_t count, uint64_t *tau, uint32_t *second,
                                           void *stream) {
    skim::clear_error();
    hipStream_t hs = (hipStream_t)stream;
    try {
        SKIM_REQUIRE(state != nullptr, "state is NULL");
        SKIM_REQUIRE(first <= state->selected && count <= state->selected - first,
                     "records [%u, %u) outside the %u selected seeds", first, first + count,
                     state->selected);
        SKIM_REQUIRE(count == 0 || tau || second, "tau and second are both NULL");
        if (count && tau)
            SKIM_HIP(hipMemcpyAsync(tau, state->args.rec_tau + first, count * sizeof(uint64_t),
                                    hipMemcpyDeviceToDevice, hs));
        if (count && second)
            SKIM_HIP(hipMemcpyAsync(second, state->args.rec_second + first,
                                    count * sizeof(uint32_t), hipMemcpyDeviceToDevice, hs));
        SKIM_HIP(hipStreamSynchronize(hs));
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        return f.st;
    }
}

// ------------------------------------------- the tail without allocation
// skim_discrepancy_tail_noalloc: the same kernels, with their scratch (the
// gain total, the per-seed survival functions and one level of the pairwise
// convolution tree) in a file-scope device array instead of memory the call
// allocates.  Each GPU holds its own copy of `scratch` at its own address,
// looked up once per device with hipGetSymbolAddress; host code only ever
// uses that address.
namespace skim {
namespace {

// seeds * (bins + 1) at most; the words hold the gain total (one 256-byte
// slot), s (bins + 1) survival values and ceil(s / 2) (bins + 1) values of
// a tree level (at most half the cells plus half a row): about 12.3 MiB.
constexpr uint64_t kNoAllocCells = 1ull << 20;
constexpr uint64_t kNoAllocWords = 32 + kNoAllocCells + kNoAllocCells / 2 + 32800;

}  // namespace
}  // namespace skim

static __device__ __align__(256) double scratch[skim::kNoAllocWords];

namespace skim {
namespace {

std::mutex g_scratch_mu;
double *g_scratch_ptr[64] = {};

double *scratch_on_device(int dev) {
    SKIM_REQUIRE(dev >= 0 && dev < 64, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        SKIM_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = (double *)ptr;
    }
    return g_scratch_ptr[dev];
}

}  // namespace
}  // namespace skim

extern "C" skim_status skim_discrepancy_tail_noalloc(uint32_t s, const uint64_t *tau,
                                                     const uint32_t *second,
                                                     const uint64_t *gain_pairs, uint32_t bins,
                                                     double max_rel_error, double *tail,
                                                     void *stream) {
    using namespace skim;
    clear_error();
    hipStream_t hs = (hipStream_t)stream;
    try {
        SKIM_REQUIRE(bins >= 1 && bins <= kTailMaxBins, "bins must be in [1, %u]", kTailMaxBins);
        SKIM_REQUIRE(max_rel_error > 0.0 && max_rel_error <= 1e300,
                     "max_rel_error must be positive and finite");
        SKIM_REQUIRE(tail != nullptr, "tail is NULL");
        SKIM_REQUIRE(s == 0 || (tau && second && gain_pairs), "tau/second/gain_pairs is NULL");
        const uint64_t W = (uint64_t)bins + 1;
        if ((uint64_t)s * W > kNoAllocCells) {
            set_error("seeds * (bins + 1) = %llu exceeds the %llu cells of the no-allocation "
                      "scratch", (unsigned long long)((uint64_t)s * W),
                      (unsigned long long)kNoAllocCells);
            throw Fail{SKIM_EUNSUPPORTED};
        }
        if (s == 0) {  // the empty sum is 0 with certainty
            fill_u64((uint64_t *)tail, 0, W, hs);
            fill_u64((uint64_t *)tail, 0x3FF0000000000000ull, 1, hs);  // 1.0
            return SKIM_OK;
        }
        int dev = 0;
        SKIM_HIP(hipGetDevice(&dev));
        double *base = scratch_on_device(dev);
        // layout: gain total (one 256-byte slot), survival functions, tree level
        uint64_t *total = (uint64_t *)base;
        double *bufA = base + 32;
        double *bufB = bufA + (uint64_t)s * W;
        k_tail_total<<<1, kTailBlock, 0, hs>>>(s, gain_pairs, total);
        SKIM_LAUNCH_CHECK();
        k_tail_survival<<<grid_for((uint64_t)s * W, kTailBlock), kTailBlock, 0, hs>>>(
            s, tau, second, gain_pairs, total, bins, max_rel_error, bufA);
        SKIM_LAUNCH_CHECK();
        double *in = bufA, *out = bufB;
        for (uint32_t rows = s; rows > 1; rows = (rows + 1) / 2) {
            const uint64_t blocks = ((uint64_t)rows + 1) / 2 * ((W + kTailOut - 1) / kTailOut);
            k_tail_pair<<<(unsigned)std::min<uint64_t>(blocks, 65536), kTailPairBlock, 0, hs>>>(
                in, out, rows, bins);
            SKIM_LAUNCH_CHECK();
            std::swap(in, out);
        }
        SKIM_HIP(hipMemcpyAsync(tail, in, W * sizeof(double), hipMemcpyDeviceToDevice, hs));
        return SKIM_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}

extern "C" skim_status skim_discrepancy_tail(uint32_t s, const uint64_t *tau,
                                             const uint32_t *second, const uint64_t *gain_pairs,
                                             uint32_t bins, double max_rel_error, double *tail,
                                             void *stream) {
    using namespace skim;
    clear_error();
    hipStream_t hs = (hipStream_t)stream;
    try {
        SKIM_REQUIRE(bins >= 1 && bins <= kTailMaxBins, "bins must be in [1, %u]", kTailMaxBins);
        SKIM_REQUIRE(max_rel_error > 0.0 && max_rel_error <= 1e300,
                     "max_rel_error must be positive and finite");
        SKIM_REQUIRE(tail != nullptr, "tail is NULL");
        SKIM_REQUIRE(s == 0 || (tau && second && gain_pairs), "tau/second/gain_pairs is NULL");
        const uint64_t W = (uint64_t)bins + 1;
        if ((uint64_t)s * W > kTailMaxCells) {
            set_error("seeds * (bins + 1) exceeds %llu", (unsigned long long)kTailMaxCells);
            throw Fail{SKIM_EUNSUPPORTED};
        }
        if (s == 0) {  // the empty sum is 0 with certainty
            fill_u64((uint64_t *)tail, 0, W, hs);
            fill_u64((uint64_t *)tail, 0x3FF0000000000000ull, 1, hs);  // 1.0
            SKIM_HIP(hipStreamSynchronize(hs));
            return SKIM_OK;
        }
        Arena T(hs);
        uint64_t *total = T.alloc<uint64_t>(1);
        double *bufA = T.alloc<double>((uint64_t)s * W);
        double *bufB = T.alloc<double>(((uint64_t)s + 1) / 2 * W);
        k_tail_total<<<1, kTailBlock, 0, hs>>>(s, gain_pairs, total);
        SKIM_LAUNCH_CHECK();
        k_tail_survival<<<grid_for((uint64_t)s * W, kTailBlock), kTailBlock, 0, hs>>>(
            s, tau, second, gain_pairs, total, bins, max_rel_error, bufA);
        SKIM_LAUNCH_CHECK();
        double *in = bufA, *out = bufB;
        for (uint32_t rows = s; rows > 1; rows = (rows + 1) / 2) {
            const uint64_t blocks = ((uint64_t)rows + 1) / 2 * ((W + kTailOut - 1) / kTailOut);
            k_tail_pair<<<(unsigned)std::min<uint64_t>(blocks, 65536), kTailPairBlock, 0, hs>>>(
                in, out, rows, bins);
            SKIM_LAUNCH_CHECK();
            std::swap(in, out);
        }
        SKIM_HIP(hipMemcpyAsync(tail, in, W * sizeof(double), hipMemcpyDeviceToDevice, hs));
        SKIM_HIP(hipStreamSynchronize(hs));
        return SKIM_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}
