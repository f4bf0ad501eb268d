// skim_eval.hip -- exact influence of seed sets over l live-edge instances
// (Section 2, eqs. (Inf) and (timedinf): l Inf({G^(i)}, S) = sum_i |reach_i(S)|).
//
// This is the evaluator of a quality harness: it scores seed sets (SKIM's,
// or any other) on the instances of a given seed, typically fresh ones that
// the sketches never saw.
//
// One coin pass builds the live out-list of every node-instance pair
// (64 v + i), so the searches never evaluate a coin.  Each query is then a
// breadth-first search over pairs run by one 1024-thread workgroup: a visited
// bitmap of 64 bits per node and an append-only queue of pair ids (every pair
// enters at most once, so the queue never overflows).  The queue is consumed
// in chunks of one pair per thread; appends reserve queue slots with one LDS
// atomic per wave.  The number of pairs appended is the query's answer.  The
// workgroup then clears the words its pairs set, so the next query on the
// same slot starts from a clean bitmap at a cost proportional to what was
// visited.  Queries run in parallel, one per workgroup slot.
//
// Exact greedy (skim_greedy_exact, the reference of a quality harness) reuses
// the search with a bitmap of covered pairs: the pairs the seeds so far
// reach.  That set is closed under reachability, so a search that skips
// covered pairs counts exactly a node's marginal gain.  Each step scores every
// node this way (n singleton queries), takes the largest gain on the device
// (smallest id on ties, among unselected nodes), searches once more from the
// winner and adds the pairs it reached to the covered bitmap.
#include "skim_internal.h"

#include <algorithm>

namespace skim {

namespace {

constexpr int kEvalBlock = 1024;
constexpr uint64_t kEvalSlotBudget = 2ull << 30;  // bytes of bitmaps + queues
constexpr uint32_t kEvalMaxSlots = 1024;

struct EvalArgs {
    uint32_t n, ell;
    const uint64_t *fptr;  // [64 n + 1] live out-lists per pair
    const uint32_t *fadj;
    uint64_t q;
    const uint64_t *qoff;
    const uint32_t *qnodes;
    uint64_t *reach;       // [q] out
    int32_t *status;       // [q] out, may be NULL
    uint32_t *bitmaps;     // [slots][2 n]
    uint32_t *queues;      // [slots][qcap]
    uint64_t qcap;         // l n
    const uint32_t *covered;  // [2 n] pairs not to enter, or NULL
};

template <class T> __device__ __forceinline__ T ld(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ void st(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// err = 1 unless qoff[0] = 0 and qoff is non-decreasing.
__global__ void k_eval_offsets(const uint64_t *qoff, uint64_t q, uint32_t *err) {
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j <= q;
         j += (uint64_t)gridDim.x * blockDim.x) {
        const bool bad = j == 0 ? qoff[0] != 0 : qoff[j - 1] > qoff[j];
        if (bad) atomicOr(err, 1u);
    }
}

// Marks pair p visited; true if this call set its bit.
__device__ __forceinline__ bool mark(uint32_t *bm, uint64_t p) {
    const uint32_t bit = 1u << (p & 31);
    return (atomicOr(bm + (p >> 5), bit) & bit) == 0;
}

__device__ __forceinline__ bool is_covered(const uint32_t *cov, uint64_t p) {
    return cov != nullptr && ((cov[p >> 5] >> (p & 31)) & 1u) != 0;
}

__global__ void __launch_bounds__(kEvalBlock) k_eval(EvalArgs A) {
    __shared__ unsigned long long s_tail;
    __shared__ uint32_t s_bad;
    const uint32_t tid = threadIdx.x;
    uint32_t *bm = A.bitmaps + (uint64_t)blockIdx.x * 2 * A.n;
    uint32_t *Q = A.queues + (uint64_t)blockIdx.x * A.qcap;
    for (uint64_t j = blockIdx.x; j < A.q; j += gridDim.x) {
        const uint64_t b = A.qoff[j], e = A.qoff[j + 1];  // validated by the host
        if (tid == 0) {
            s_tail = 0;
            s_bad = 0;
        }
        __syncthreads();
        if (s_bad == 0)
            for (uint64_t t = b + tid; t < e; t += kEvalBlock)
                if (A.qnodes[t] >= A.n) s_bad = 1u;  // any writer: same value
        __syncthreads();
        if (s_bad) {
            if (tid == 0) {
                A.reach[j] = 0;
                if (A.status) A.status[j] = -(int32_t)s_bad;
            }
            __syncthreads();
            continue;
        }
        // seeds: every (s, i) with s in S, i < l (duplicates in S act once)
        const uint64_t seeds = (e - b) * A.ell;
        for (uint64_t t0 = 0; t0 < seeds; t0 += kEvalBlock) {
            const uint64_t t = t0 + tid;
            bool add = false;
            uint64_t p = 0;
            if (t < seeds) {
                p = (uint64_t)A.qnodes[b + t / A.ell] * kPairStride + t % A.ell;
                add = !is_covered(A.covered, p) && mark(bm, p);
            }
            const uint64_t slot = wave_reserve(&s_tail, add);
            if (add) st(Q + slot, (uint32_t)p);
        }
        __syncthreads();
        // breadth-first over pairs; the queue only grows
        uint64_t head = 0;
        for (;;) {
            const uint64_t tail = s_tail;
            __syncthreads();  // every thread has the same tail before any append
            if (head >= tail) break;
            const uint64_t chunk = tail - head < (uint64_t)kEvalBlock ? tail - head : kEvalBlock;
            if (tid < chunk) {
                const uint32_t p = ld(Q + head + tid);
                const uint32_t i = p % kPairStride;
                const uint64_t e0 = A.fptr[p], e1 = A.fptr[p + 1];
                for (uint64_t x = e0; x < e1; ++x) {
                    const uint64_t pw = (uint64_t)A.fadj[x] * kPairStride + i;
                    const bool add = !is_covered(A.covered, pw) && mark(bm, pw);
                    const unsigned long long mask = __ballot(add);
                    if (mask) {
                        const int leader = __ffsll((long long)mask) - 1;
                        unsigned long long base = 0;
                        if ((int)lane_id() == leader)
                            base = atomicAdd(&s_tail, (unsigned long long)__popcll(mask));
                        base = ((unsigned long long)__shfl((uint32_t)(base >> 32), leader) << 32) |
                               __shfl((uint32_t)base, leader);
                        if (add)
                            st(Q + base + __popcll(mask & ((1ull << lane_id()) - 1ull)),
                               (uint32_t)pw);
                    }
                }
            }
            head += chunk;
            __syncthreads();  // appends of this chunk are in the queue and s_tail
        }
        const uint64_t total = s_tail;
        if (tid == 0) {
            A.reach[j] = total;
            if (A.status) A.status[j] = 0;
        }
        // clean the bitmap words this query set
        for (uint64_t t = tid; t < total; t += kEvalBlock) st(bm + (ld(Q + t) >> 5), 0u);
        __syncthreads();
    }
}

// The next exact-greedy seed: the largest gain among unselected nodes,
// smallest id on ties (one workgroup).
__global__ void __launch_bounds__(kEvalBlock) k_exact_pick(uint32_t n, const uint64_t *gain,
                                                           uint32_t *sel, uint32_t *x_out,
                                                           uint32_t *seed_out) {
    __shared__ unsigned long long best;
    if (threadIdx.x == 0) best = 0;
    __syncthreads();
    unsigned long long mine = 0;
    for (uint32_t v = threadIdx.x; v < n; v += kEvalBlock)
        if (!sel[v]) {
            // gains are at most 64 n < 2^32
            const unsigned long long key = (gain[v] << 32) | (0xFFFFFFFFu - v);
            mine = key > mine ? key : mine;
        }
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)mine, off);
        const uint32_t hi = __shfl_xor((uint32_t)(mine >> 32), off);
        const unsigned long long o = ((unsigned long long)hi << 32) | lo;
        mine = o > mine ? o : mine;
    }
    if ((threadIdx.x & 63) == 0) atomicMax(&best, mine);
    __syncthreads();
    if (threadIdx.x == 0) {
        // an unselected node always exists (the host checks s)
        const uint32_t v = 0xFFFFFFFFu - (uint32_t)best;
        const uint32_t x = (best != 0 && v < n) ? v : 0;
        sel[x] = 1;
        *x_out = x;
        *seed_out = x;
    }
}

// Adds the pairs of one finished search (its queue) to the covered bitmap.
__global__ void k_exact_cover(const uint32_t *Q, const uint64_t *count, uint32_t *covered) {
    const uint64_t c = *count;
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < c;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p = Q[t];
        atomicOr(covered + (p >> 5), 1u << (p & 31));
    }
}

__global__ void k_iota(uint32_t n, uint64_t *off, uint32_t *nodes) {
    for (uint32_t v = blockIdx.x * blockDim.x + threadIdx.x; v <= n; v += gridDim.x * blockDim.x) {
        off[v] = v;
        if (v < n) nodes[v] = v;
    }
}

}  // namespace

}  // namespace skim

extern "C" skim_status skim_greedy_exact(const skim_graph *g, uint32_t ell, uint64_t seed,
                                         uint32_t s, uint32_t *seeds, uint64_t *gain_pairs,
                                         void *stream) {
    using namespace skim;
    clear_error();
    hipStream_t hs = (hipStream_t)stream;
    try {
        SKIM_REQUIRE(g != nullptr, "graph is NULL");
        SKIM_REQUIRE(ell >= 1 && ell <= 64, "l must be in [1, 64]");
        SKIM_REQUIRE(s <= g->n, "s exceeds n");
        SKIM_REQUIRE(s == 0 || (seeds && gain_pairs), "seeds/gain_pairs is NULL");
        Arena T(hs);
        uint32_t *esrc = T.alloc<uint32_t>(g->m ? g->m : 1);
        validate_graph(g, esrc, T);
        if (s == 0) return SKIM_OK;
        const uint32_t n = g->n;
        LiveLists fwd = build_live_lists(g, ell, seed, esrc, /*forward=*/true, T);
        const uint64_t qcap = (uint64_t)ell * n;
        const uint64_t per_slot = (2ull * n + qcap) * sizeof(uint32_t);
        uint64_t slots = std::max<uint64_t>(1, kEvalSlotBudget / per_slot);
        slots = std::min<uint64_t>(std::min<uint64_t>(slots, kEvalMaxSlots), n);
        EvalArgs A{};
        A.n = n;
        A.ell = ell;
        A.fptr = fwd.ptr;
        A.fadj = fwd.adj;
        A.bitmaps = T.alloc<uint32_t>(slots * 2 * n);
        A.queues = T.alloc<uint32_t>(slots * qcap);
        A.qcap = qcap;
        A.status = nullptr;
        uint32_t *covered = T.alloc<uint32_t>(2ull * n);
        uint32_t *sel = T.alloc<uint32_t>(n);
        uint64_t *gain = T.alloc<uint64_t>(n);
        uint64_t *all_off = T.alloc<uint64_t>((uint64_t)n + 1);
        uint32_t *all_nodes = T.alloc<uint32_t>(n);
        uint64_t *one_off = T.alloc<uint64_t>(2);
        uint32_t *x = T.alloc<uint32_t>(1);
        fill_u32(A.bitmaps, 0, slots * 2 * n, hs);
        fill_u32(covered, 0, 2ull * n, hs);
        fill_u32(sel, 0, n, hs);
        k_iota<<<grid_for((uint64_t)n + 1, 256, 4096), 256, 0, hs>>>(n, all_off, all_nodes);
        SKIM_LAUNCH_CHECK();
        k_iota<<<1, 256, 0, hs>>>(1, one_off, x);  // one_off = {0, 1}
        SKIM_LAUNCH_CHECK();
        A.covered = covered;
        for (uint32_t step = 0; step < s; ++step) {
            // every node's marginal gain: a search that does not enter covered pairs
            A.q = n;
            A.qoff = all_off;
            A.qnodes = all_nodes;
            A.reach = gain;
            k_eval<<<(unsigned)slots, kEvalBlock, 0, hs>>>(A);
            SKIM_LAUNCH_CHECK();
            k_exact_pick<<<1, kEvalBlock, 0, hs>>>(n, gain, sel, x, seeds + step);
            SKIM_LAUNCH_CHECK();
            // the winner's search again, on slot 0, then cover what it reached
            A.q = 1;
            A.qoff = one_off;
            A.qnodes = x;
            A.reach = gain_pairs + step;
            k_eval<<<1, kEvalBlock, 0, hs>>>(A);
            SKIM_LAUNCH_CHECK();
            k_exact_cover<<<grid_for(qcap, 256, 4096), 256, 0, hs>>>(A.queues, gain_pairs + step,
                                                                    covered);
            SKIM_LAUNCH_CHECK();
        }
        SKIM_HIP(hipStreamSynchronize(hs));
        return SKIM_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}

extern "C" skim_status skim_influence_batch(const skim_graph *g, uint32_t ell, uint64_t seed,
                                            uint64_t q, const uint64_t *qoff,
                                            const uint32_t *qnodes, uint64_t *reach_pairs,
                                            int32_t *qstatus, void *stream) {
    using namespace skim;
    clear_error();
    hipStream_t hs = (hipStream_t)stream;
    try {
        SKIM_REQUIRE(g != nullptr, "graph is NULL");
        SKIM_REQUIRE(ell >= 1 && ell <= 64, "l must be in [1, 64]");
        SKIM_REQUIRE(q == 0 || (qoff && reach_pairs), "qoff/reach_pairs is NULL");
        Arena T(hs);
        uint32_t *esrc = T.alloc<uint32_t>(g->m ? g->m : 1);
        validate_graph(g, esrc, T);
        if (q == 0) return SKIM_OK;
        uint32_t *err = T.alloc<uint32_t>(1);
        fill_u32(err, 0, 1, hs);
        k_eval_offsets<<<grid_for(q + 1, 256, 4096), 256, 0, hs>>>(qoff, q, err);
        SKIM_LAUNCH_CHECK();
        uint32_t herr = 0;
        read_back(&herr, err, sizeof herr, hs);
        SKIM_REQUIRE(herr == 0, "qoff must start at 0 and be non-decreasing");
        uint64_t total = 0;
        read_back(&total, qoff + q, sizeof total, hs);
        SKIM_REQUIRE(total == 0 || qnodes, "qnodes is NULL");
        const uint32_t n = g->n;
        LiveLists fwd = build_live_lists(g, ell, seed, esrc, /*forward=*/true, T);
        const uint64_t qcap = (uint64_t)ell * n;
        const uint64_t per_slot = (2ull * n + qcap) * sizeof(uint32_t);
        uint64_t slots = std::max<uint64_t>(1, kEvalSlotBudget / per_slot);
        slots = std::min<uint64_t>(std::min<uint64_t>(slots, kEvalMaxSlots), q);
        EvalArgs A{};
        A.n = n;
        A.ell = ell;
        A.fptr = fwd.ptr;
        A.fadj = fwd.adj;
        A.q = q;
        A.qoff = qoff;
        A.qnodes = qnodes;  // never read when every set is empty
        A.reach = reach_pairs;
        A.status = qstatus;
        A.bitmaps = T.alloc<uint32_t>(slots * 2 * n);
        A.queues = T.alloc<uint32_t>(slots * qcap);
        A.qcap = qcap;
        A.covered = nullptr;
        fill_u32(A.bitmaps, 0, slots * 2 * n, hs);
        {
            LaunchTimer t("k_eval", hs);
            k_eval<<<(unsigned)slots, kEvalBlock, 0, hs>>>(A);
            SKIM_LAUNCH_CHECK();
        }
        SKIM_HIP(hipStreamSynchronize(hs));
        return SKIM_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}
