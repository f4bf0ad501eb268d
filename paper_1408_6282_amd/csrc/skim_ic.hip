// skim_ic.hip -- sketches for the IC model itself (Section 3, "Sketches for
// an IC model"), with structured permutation ranks (Section 3, "Structured
// permutation ranks") in the limit of infinitely many instances.
//
// Positions t = 1 .. k n come in k chunks of n; each chunk holds every node
// once, in the order of a SplitMix64 hash (a rocPRIM segmented radix sort per
// chunk).  Every position has an instance of its own, so the sketch of u is
// the k smallest positions t whose node v_t u reaches in instance t, and the
// influence estimate is n (k - 1) / (T - 1) with T the k-th smallest.  Nothing
// prunes a search here (an instance has one source), so:
//  * one thread per position runs the complete reverse search from v_t over
//    the in-edges whose coin in instance t is live (coins on the fly from a
//    per-edge SplitMix64 stream), deduplicating with a visited bitmap of its
//    own and clearing only the bits it set; a search that grows beyond
//    kIcLight nodes is handed to a workgroup (the heavy searches of hubs
//    would otherwise serialise in one thread);
//  * a first pass counts the nodes each search reaches, a scan gives every
//    position its record range, and a second pass writes the records
//    (node << 32 | t) there, so no record needs an atomic;
//  * the records are radix-sorted; every node holds at least k of them (it
//    reaches itself in every chunk) and keeps its first k.
#include "skim_internal.h"

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include <algorithm>

namespace skim {

namespace {

constexpr uint64_t kIcChunk = 1ull << 63;                  // counters of the chunk hashes
constexpr uint64_t kIcEdge = (1ull << 63) | (1ull << 62);  // counters of the per-edge streams
constexpr int kIcBlock = 256;
constexpr uint64_t kIcStateBudget = 8ull << 30;            // bytes of per-thread search state
constexpr uint32_t kIcLight = 1024;   // a thread's search hands over beyond this many nodes
constexpr int kIcHeavyBlock = 1024;   // one workgroup per handed-over search
constexpr uint64_t kIcHeavyBudget = 2ull << 30;            // bytes of per-workgroup state
constexpr uint64_t kIcRecordCap = 1ull << 28;  // records of the single pass (2 GiB)

// Coin of edge (u -> w) in the instance of position t (>= 1): the high
// (t - 1 even) or low (t - 1 odd) half of output floor((t - 1) / 2) of the
// stream seeded with SM(seed, kIcEdge + u n + w).
__device__ __forceinline__ bool ic_live(uint64_t seed, uint32_t n, uint32_t u, uint32_t w,
                                        uint32_t t, uint32_t thr) {
    const uint64_t edge_seed = sm_at(seed, kIcEdge + (uint64_t)u * n + w);
    const uint64_t h = sm_at(edge_seed, (t - 1) / 2);
    const uint32_t coin = ((t - 1) & 1u) == 0 ? (uint32_t)(h >> 32) : (uint32_t)h;
    return coin <= thr;
}

__global__ void k_ic_indeg(const uint32_t *col, uint64_t m, uint32_t *indeg) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x)
        atomicAdd(indeg + col[e], 1u);
}

// In-edges grouped by head: source and threshold (order within a head is
// immaterial: a search's reached set does not depend on it).
__global__ void k_ic_rfill(const uint32_t *esrc, const uint32_t *col, const uint32_t *thr,
                           uint64_t m, const uint64_t *rptr, uint32_t *cursor, uint32_t *rsrc,
                           uint32_t *rthr) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t w = col[e];
        const uint64_t at = rptr[w] + atomicAdd(cursor + w, 1u);
        rsrc[at] = esrc[e];
        rthr[at] = thr[e];
    }
}

__global__ void k_ic_hash(uint32_t n, uint32_t k, uint64_t seed, uint64_t *keys, uint32_t *vals,
                          uint32_t *offs) {
    const uint64_t total = (uint64_t)n * k;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total;
         x += (uint64_t)gridDim.x * blockDim.x) {
        keys[x] = sm_at(seed, kIcChunk + x);  // x = c n + v
        vals[x] = (uint32_t)(x % n);
        if (x % n == 0) offs[x / n] = (uint32_t)x;
        if (x == 0) offs[k] = (uint32_t)total;
    }
}

struct IcArgs {
    uint32_t n, k;
    uint64_t seed;
    const uint64_t *rptr;
    const uint32_t *rsrc, *rthr;
    const uint32_t *node_at;  // [k n] node at position t = index + 1
    uint32_t *counts;         // [k n] pass 0 out
    const uint64_t *offsets;  // [k n + 1] pass 1 in
    uint64_t *records;        // pass 1 out (pass 2: appended, up to rcap)
    unsigned long long *rcount;  // pass 2: records appended
    uint64_t rcap;
    uint32_t *ovf;            // pass 2: the records outgrew rcap
    uint32_t *bitmaps;        // [threads][(n + 31) / 32]
    uint32_t *queues;         // [threads][kIcLight]
    uint32_t *heavy;          // positions handed to the workgroup search
    unsigned long long *nheavy;
    uint32_t *hbitmaps;       // [workgroups][(n + 31) / 32]
    uint32_t *hqueues;        // [workgroups][n]
};

template <class T> __device__ __forceinline__ T ic_ld(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <class T> __device__ __forceinline__ void ic_st(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Inclusive prefix sum over the wave's lanes, and the lane whose range holds
// flat position j of the lanes' items laid end to end (binary lifting).
__device__ __forceinline__ uint32_t ic_wave_incl(uint32_t v, uint32_t lane) {
#pragma unroll
    for (uint32_t off = 1; off < 64; off <<= 1) {
        const uint32_t y = __shfl_up(v, off);
        if (lane >= off) v += y;
    }
    return v;
}
__device__ __forceinline__ uint32_t ic_wave_owner(uint32_t incl, uint32_t j) {
    uint32_t r = 0;
#pragma unroll
    for (uint32_t step = 32; step > 0; step >>= 1) {
        const uint32_t v = (uint32_t)__shfl((int)incl, (int)(r + step - 1));
        if (v <= j) r += step;
    }
    return r & 63u;
}

// One search per position, one position per thread.  The 64 searches of a
// wave advance together: at each step every lane takes the next node of its
// own queue, and the wave lays those nodes' in-edges end to end and tests
// them 64 at a time, so a lane whose node is a hub (thousands of in-edges,
// each a coin) does not hold the other 63.  A node that passes its coin and
// is new to its search (an atomic OR on that search's bitmap) is appended
// to its queue at its rank among that search's new nodes of the round.  A
// search that would reach more than kIcLight nodes stops, clears what it
// marked and hands the position to the workgroup search (first pass:
// appended to the heavy list; second pass: skipped, its count being above
// kIcLight).  Pass 2 is the single pass used when the records fit a buffer
// sized up front: the heavy list as in pass 0, and every other search's
// records appended at a place reserved once per wave.
template <int kPass>
__global__ void __launch_bounds__(kIcBlock) k_ic_search(IcArgs A) {
    const uint64_t tid = blockIdx.x * (uint64_t)kIcBlock + threadIdx.x;
    const uint64_t threads = (uint64_t)gridDim.x * kIcBlock;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave0 = tid - lane;  // thread id of the wave's lane 0
    const uint32_t words = (A.n + 31) / 32;
    uint32_t *bm = A.bitmaps + tid * words;
    uint32_t *Q = A.queues + tid * kIcLight;
    const uint64_t total = (uint64_t)A.n * A.k;
    for (uint64_t x0 = 0; x0 < total; x0 += threads) {
        const uint64_t x = x0 + tid;
        const bool mine = x < total && !(kPass == 1 && A.counts[x] > kIcLight);
        const uint32_t t = (uint32_t)(x + 1);
        bool heavy = false;
        uint32_t cnt = 0, head = 0;
        if (mine) {
            const uint32_t v = A.node_at[x];
            Q[0] = v;
            atomicOr(bm + (v >> 5), 1u << (v & 31));
            cnt = 1;
        }
        for (;;) {
            const bool act = mine && !heavy && head < cnt;
            if (!__any(act)) break;  // uniform over the wave
            uint32_t y = 0, d = 0;
            uint64_t e0 = 0;
            if (act) {
                y = Q[head++];
                e0 = A.rptr[y];
                d = (uint32_t)(A.rptr[y + 1] - e0);
            }
            const uint32_t incl = ic_wave_incl(d, lane);
            const uint32_t tot = (uint32_t)__shfl((int)incl, 63);
            const uint32_t mine_first = incl - d;  // this lane's items: [mine_first, incl)
            for (uint32_t base = 0; base < tot; base += 64) {
                const uint32_t j = base + lane, r = ic_wave_owner(incl, j);
                const uint32_t first = (uint32_t)__shfl((int)incl, (int)r) -
                                       (uint32_t)__shfl((int)d, (int)r);
                const uint32_t ry = (uint32_t)__shfl((int)y, (int)r);
                const uint32_t rt = (uint32_t)__shfl((int)t, (int)r);
                const uint32_t elo = (uint32_t)__shfl((int)(uint32_t)e0, (int)r);
                const uint32_t ehi = (uint32_t)__shfl((int)(uint32_t)(e0 >> 32), (int)r);
                const uint32_t rcnt = (uint32_t)__shfl((int)cnt, (int)r);
                uint32_t u = 0;
                bool add = false;
                if (j < tot) {
                    const uint64_t e = (((uint64_t)ehi << 32) | elo) + (j - first);
                    u = A.rsrc[e];
                    if (ic_live(A.seed, A.n, u, ry, rt, A.rthr[e])) {
                        const uint32_t bit = 1u << (u & 31);
                        uint32_t *rbm = A.bitmaps + (wave0 + r) * words + (u >> 5);
                        add = (atomicOr(rbm, bit) & bit) == 0;
                    }
                }
                // rank among the same search's new nodes of this round (its
                // positions are consecutive lanes, from lane first - base on)
                const unsigned long long m = __ballot(add);
                const uint32_t lo = first > base ? first - base : 0u;
                const unsigned long long below =
                    m & ((1ull << lane) - 1ull) & ~((1ull << lo) - 1ull);
                if (add) {
                    const uint32_t idx = rcnt + (uint32_t)__popcll(below);
                    if (idx < kIcLight) {
                        A.queues[(wave0 + r) * kIcLight + idx] = u;
                    } else {  // the search overflows: unmark, it goes to a workgroup
                        atomicAnd(A.bitmaps + (wave0 + r) * words + (u >> 5),
                                  ~(1u << (u & 31)));
                    }
                }
                // this lane's search counts its own new nodes of the round
                if (mine_first < base + 64 && incl > base) {
                    const uint32_t a = mine_first > base ? mine_first - base : 0u;
                    const uint32_t b = incl < base + 64 ? incl - base : 64u;
                    const unsigned long long range =
                        (b >= 64 ? ~0ull : ((1ull << b) - 1ull)) & ~((1ull << a) - 1ull);
                    cnt += (uint32_t)__popcll(m & range);
                }
            }
            if (cnt > kIcLight) heavy = true;
        }
        if (mine) {
            const uint32_t kept = cnt < kIcLight ? cnt : kIcLight;
            if (kPass == 0) {
                A.counts[x] = heavy ? 0u : cnt;
            } else if (kPass == 2) {
                A.counts[x] = 0u;  // a heavy search's count comes from the workgroup pass
            } else if (!heavy) {
                uint64_t *out = A.records + A.offsets[x];
                for (uint32_t j = 0; j < kept; ++j) out[j] = ((uint64_t)Q[j] << 32) | t;
            }
            for (uint32_t j = 0; j < kept; ++j) atomicAnd(bm + (Q[j] >> 5), 0u);
        }
        if (kPass == 2) {  // every lane of the wave takes part
            const uint32_t nrec = mine && !heavy ? (cnt < kIcLight ? cnt : kIcLight) : 0u;
            const uint32_t incl = ic_wave_incl(nrec, lane);
            const uint32_t wtot = (uint32_t)__shfl((int)incl, 63);
            unsigned long long base = 0;
            if (lane == 0 && wtot) base = atomicAdd(A.rcount, (unsigned long long)wtot);
            base = ((unsigned long long)(uint32_t)__shfl((int)(uint32_t)(base >> 32), 0) << 32) |
                   (uint32_t)__shfl((int)(uint32_t)base, 0);
            if (nrec) {
                if (base + wtot <= A.rcap) {
                    uint64_t *out = A.records + base + (incl - nrec);
                    for (uint32_t j = 0; j < nrec; ++j) out[j] = ((uint64_t)Q[j] << 32) | t;
                } else {
                    atomicOr(A.ovf, 1u);
                }
            }
        }
        if (kPass != 1) {  // every lane of the wave takes part in the reservation
            const uint64_t slot = wave_reserve(A.nheavy, heavy);
            if (heavy) A.heavy[slot] = (uint32_t)x;
        }
    }
}

// One workgroup per handed-over position: the breadth-first search takes up
// to kIcHeavyBlock queue entries per round, one per thread; new nodes are
// marked in the workgroup's bitmap with an atomic OR and appended with one
// LDS atomic per wave.
template <int kPass>
__global__ void __launch_bounds__(kIcHeavyBlock) k_ic_heavy(IcArgs A, uint64_t nheavy) {
    __shared__ unsigned long long s_tail;
    const uint32_t tid = threadIdx.x;
    const uint32_t words = (A.n + 31) / 32;
    uint32_t *bm = A.hbitmaps + (uint64_t)blockIdx.x * words;
    uint32_t *Q = A.hqueues + (uint64_t)blockIdx.x * A.n;
    for (uint64_t h = blockIdx.x; h < nheavy; h += gridDim.x) {
        const uint64_t x = A.heavy[h];
        const uint32_t t = (uint32_t)(x + 1);
        if (tid == 0) {
            const uint32_t v = A.node_at[x];
            atomicOr(bm + (v >> 5), 1u << (v & 31));
            ic_st(Q, v);
            s_tail = 1;
        }
        __syncthreads();
        uint64_t head = 0;
        for (;;) {
            const uint64_t tail = s_tail;
            __syncthreads();  // every thread has the same tail before any append
            if (head >= tail) break;
            const uint64_t chunk = tail - head < (uint64_t)kIcHeavyBlock ? tail - head : kIcHeavyBlock;
            if (tid < chunk) {
                const uint32_t y = ic_ld(Q + head + tid);
                for (uint64_t e = A.rptr[y]; e < A.rptr[y + 1]; ++e) {
                    const uint32_t u = A.rsrc[e];
                    const uint32_t bit = 1u << (u & 31);
                    bool add = (ic_ld(bm + (u >> 5)) & bit) == 0 &&
                               ic_live(A.seed, A.n, u, y, t, A.rthr[e]);
                    if (add) add = (atomicOr(bm + (u >> 5), bit) & bit) == 0;
                    const uint64_t slot = wave_reserve(&s_tail, add);
                    if (add) ic_st(Q + slot, u);
                }
            }
            head += chunk;
            __syncthreads();  // this round's appends are in the queue and s_tail
        }
        const uint64_t cnt = s_tail;
        if (kPass == 0) {
            if (tid == 0) A.counts[x] = (uint32_t)cnt;
        } else {
            uint64_t *out = A.records + A.offsets[x];
            for (uint64_t j = tid; j < cnt; j += kIcHeavyBlock)
                out[j] = ((uint64_t)ic_ld(Q + j) << 32) | t;
        }
        for (uint64_t j = tid; j < cnt; j += kIcHeavyBlock) ic_st(bm + (ic_ld(Q + j) >> 5), 0u);
        __syncthreads();  // the bitmap is clean before the next position
    }
}

// start[u] = index of u's first record (every node has records).
__global__ void k_ic_starts(const uint64_t *rec, uint64_t R, uint64_t *start) {
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j < R;
         j += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t node = (uint32_t)(rec[j] >> 32);
        if (j == 0 || (uint32_t)(rec[j - 1] >> 32) != node) start[node] = j;
    }
}

__global__ void k_ic_select(const uint64_t *rec, const uint64_t *start, uint32_t n, uint32_t k,
                            uint32_t *pos, double *est) {
    for (uint64_t u = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; u < n;
         u += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t s = start[u];
        for (uint32_t j = 0; j < k; ++j) pos[u * k + j] = (uint32_t)rec[s + j];
        if (est) {
            const uint32_t T = (uint32_t)rec[s + k - 1];
            est[u] = ((double)n * (double)(k - 1)) / (double)(T - 1);
        }
    }
}

// ------------------------------------------------------------ union queries
// One wave per query; each lane keeps the current heads and thresholds of
// its members in registers, so a step of the k-way merge reads global memory
// only for the members holding the current minimum.
constexpr uint32_t kIcMaxMembers = 1024;
constexpr uint32_t kIcNoPos = 0xFFFFFFFFu;

__global__ void k_icq_offsets(const uint64_t *qoff, uint64_t q, uint32_t *err) {
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j <= q;
         j += (uint64_t)gridDim.x * blockDim.x) {
        const bool bad = j == 0 ? qoff[0] != 0 : qoff[j - 1] > qoff[j];
        if (bad) atomicOr(err, 1u);
    }
}

__device__ __forceinline__ uint32_t wave_min_u32(uint32_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t y = __shfl_xor(x, off);
        x = y < x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t y = __shfl_xor(x, off);
        x = y > x ? y : x;
    }
    return x;
}

// The k-way merge over S members with R >= S / 64 register slots per lane:
// lane l keeps the current head and threshold of members l + 64 r.
template <int R>
__device__ __forceinline__ void ic_merge(const uint32_t *pos, uint32_t n, uint32_t k,
                                         uint32_t estimator, uint32_t S, const uint32_t *mnode,
                                         uint32_t &T, double &sum) {
    const uint32_t lane = threadIdx.x;
    const uint32_t lim = estimator == 1 ? k - 1 : k;  // CK leaves out each threshold
    uint32_t head[R], thr[R], at[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t t = lane + 64u * r;
        head[r] = kIcNoPos;
        thr[r] = 0;
        at[r] = 0;
        if (t < S) {
            const uint64_t row = (uint64_t)mnode[t] * k;
            head[r] = pos[row];
            thr[r] = pos[row + k - 1];
        }
    }
    uint32_t d = 0;
    for (;;) {
        uint32_t lmin = kIcNoPos;
#pragma unroll
        for (int r = 0; r < R; ++r) lmin = head[r] < lmin ? head[r] : lmin;
        const uint32_t g = wave_min_u32(lmin);
        if (g == kIcNoPos) break;
        uint32_t tmax = 0;
#pragma unroll
        for (int r = 0; r < R; ++r)
            if (head[r] == g) {
                const uint32_t p = ++at[r];
                head[r] = p < lim ? pos[(uint64_t)mnode[lane + 64u * r] * k + p] : kIcNoPos;
                tmax = thr[r] > tmax ? thr[r] : tmax;
            }
        if (estimator == 1) {
            tmax = wave_max_u32(tmax);
            if (lane == 0) sum += (double)n / (double)(tmax - 1);
        } else if (++d == k) {
            T = g;
            break;
        }
    }
}

__global__ void __launch_bounds__(64) k_ic_query(const uint32_t *pos, uint32_t n, uint32_t k,
                                                 uint64_t q, const uint64_t *qoff,
                                                 const uint32_t *qnodes, uint32_t estimator,
                                                 double *est, int32_t *qstatus) {
    __shared__ uint32_t mnode[kIcMaxMembers];
    const uint32_t lane = threadIdx.x;
    for (uint64_t j = blockIdx.x; j < q; j += gridDim.x) {
        const uint64_t a = qoff[j], b = qoff[j + 1], S = b - a;
        bool bad = false;
        for (uint64_t t = a + lane; t < b; t += 64) bad |= qnodes[t] >= n;
        bad = __ballot(bad) != 0;
        if (bad || S == 0 || S > kIcMaxMembers) {
            if (lane == 0) {
                est[j] = 0.0;
                if (qstatus) qstatus[j] = bad ? -1 : (S == 0 ? 0 : -2);
            }
            continue;
        }
        for (uint32_t t = lane; t < S; t += 64) mnode[t] = qnodes[a + t];
        __syncthreads();
        uint32_t T = 0;
        double sum = 0.0;
        if (S <= 64)
            ic_merge<1>(pos, n, k, estimator, (uint32_t)S, mnode, T, sum);
        else if (S <= 256)
            ic_merge<4>(pos, n, k, estimator, (uint32_t)S, mnode, T, sum);
        else
            ic_merge<kIcMaxMembers / 64>(pos, n, k, estimator, (uint32_t)S, mnode, T, sum);
        if (lane == 0) {
            est[j] = estimator == 1 ? sum : ((double)n * (double)(k - 1)) / (double)(T - 1);
            if (qstatus) qstatus[j] = 0;
        }
        __syncthreads();  // LDS is reused by the next query of the stride
    }
}

}  // namespace

}  // namespace skim

extern "C" skim_status skim_ic_query_batch(const uint32_t *positions, uint32_t n, uint32_t k,
                                           uint64_t q, const uint64_t *qoff,
                                           const uint32_t *qnodes, uint32_t estimator,
                                           double *est, int32_t *qstatus, void *stream) {
    using namespace skim;
    clear_error();
    hipStream_t hs = (hipStream_t)stream;
    try {
        SKIM_REQUIRE(k >= 2 && k <= 256, "k must be in [2, 256]");
        SKIM_REQUIRE(n >= 1 && (uint64_t)n * k < (1ull << 32), "n must be >= 1 with k n < 2^32");
        SKIM_REQUIRE(estimator <= 1, "estimator must be 0 (bottom-k) or 1 (Cohen-Kaplan)");
        SKIM_REQUIRE(positions != nullptr, "positions is NULL");
        if (q == 0) return SKIM_OK;
        SKIM_REQUIRE(qoff && est, "qoff/est is NULL");
        Arena T(hs);
        uint32_t *err = T.alloc<uint32_t>(1);
        fill_u32(err, 0, 1, hs);
        k_icq_offsets<<<grid_for(q + 1, 256, 4096), 256, 0, hs>>>(qoff, q, err);
        SKIM_LAUNCH_CHECK();
        uint32_t herr = 0;
        read_back(&herr, err, sizeof herr, hs);
        SKIM_REQUIRE(herr == 0, "qoff must start at 0 and be non-decreasing");
        uint64_t total = 0;
        read_back(&total, qoff + q, sizeof total, hs);
        SKIM_REQUIRE(total == 0 || qnodes, "qnodes is NULL");
        {
            LaunchTimer t("k_ic_query", hs);
            k_ic_query<<<(unsigned)std::min<uint64_t>(q, 16384), 64, 0, hs>>>(
                positions, n, k, q, qoff, qnodes, estimator, est, qstatus);
            SKIM_LAUNCH_CHECK();
        }
        SKIM_HIP(hipStreamSynchronize(hs));
        return SKIM_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}

extern "C" skim_status skim_build_ic_sketches(const skim_graph *g, uint32_t k, uint64_t seed,
                                              uint32_t *positions, double *est, void *stream) {
    using namespace skim;
    clear_error();
    hipStream_t hs = (hipStream_t)stream;
    try {
        SKIM_REQUIRE(g != nullptr, "graph is NULL");
        SKIM_REQUIRE(k >= 2 && k <= 256, "k must be in [2, 256]");
        SKIM_REQUIRE(positions != nullptr, "positions is NULL");
        SKIM_REQUIRE((uint64_t)g->n * k < (1ull << 32), "k n must be below 2^32");
        Arena T(hs);
        const uint32_t n = g->n;
        const uint64_t m = g->m;
        uint32_t *esrc = T.alloc<uint32_t>(m ? m : 1);
        validate_graph(g, esrc, T);
        // reverse graph with thresholds
        uint32_t *indeg = T.alloc<uint32_t>(n);
        fill_u32(indeg, 0, n, hs);
        if (m) {
            k_ic_indeg<<<grid_for(m, 256, 16384), 256, 0, hs>>>(g->col, m, indeg);
            SKIM_LAUNCH_CHECK();
        }
        uint64_t *rptr = T.alloc<uint64_t>((uint64_t)n + 1);
        exclusive_scan_u32(indeg, rptr, n, T);
        uint32_t *rsrc = T.alloc<uint32_t>(m ? m : 1);
        uint32_t *rthr = T.alloc<uint32_t>(m ? m : 1);
        fill_u32(indeg, 0, n, hs);  // reused as per-head cursors
        if (m) {
            k_ic_rfill<<<grid_for(m, 256, 16384), 256, 0, hs>>>(esrc, g->col, g->thr, m, rptr,
                                                               indeg, rsrc, rthr);
            SKIM_LAUNCH_CHECK();
        }
        // the structured permutation: chunk c orders the nodes by their hash
        const uint64_t total = (uint64_t)n * k;
        uint64_t *hkeys = T.alloc<uint64_t>(total);
        uint64_t *hkeys2 = T.alloc<uint64_t>(total);
        uint32_t *hvals = T.alloc<uint32_t>(total);
        uint32_t *node_at = T.alloc<uint32_t>(total);
        uint32_t *offs = T.alloc<uint32_t>((uint64_t)k + 1);
        k_ic_hash<<<grid_for(total, 256, 16384), 256, 0, hs>>>(n, k, seed, hkeys, hvals, offs);
        SKIM_LAUNCH_CHECK();
        size_t tmp_bytes = 0;
        SKIM_HIP(rocprim::segmented_radix_sort_pairs(nullptr, tmp_bytes, hkeys, hkeys2, hvals,
                                                     node_at, (unsigned)total, k, offs, offs + 1,
                                                     0, 64, hs));
        void *tmp = T.get(tmp_bytes);
        SKIM_HIP(rocprim::segmented_radix_sort_pairs(tmp, tmp_bytes, hkeys, hkeys2, hvals,
                                                     node_at, (unsigned)total, k, offs, offs + 1,
                                                     0, 64, hs));
        T.release(tmp);
        T.release(hkeys);
        T.release(hkeys2);
        T.release(hvals);
        // per-thread search state within the budget
        const uint32_t words = (n + 31) / 32;
        const uint64_t per_thread = ((uint64_t)words + kIcLight) * sizeof(uint32_t);
        uint64_t threads = std::max<uint64_t>(kIcBlock, kIcStateBudget / per_thread);
        threads = std::min<uint64_t>(threads, (total + kIcBlock - 1) / kIcBlock * kIcBlock);
        threads = std::min<uint64_t>(threads, 1ull << 19);  // enough to fill the chip
        threads = threads / kIcBlock * kIcBlock;
        IcArgs A{};
        A.n = n;
        A.k = k;
        A.seed = seed;
        A.rptr = rptr;
        A.rsrc = rsrc;
        A.rthr = rthr;
        A.node_at = node_at;
        A.bitmaps = T.alloc<uint32_t>(threads * words);
        A.queues = T.alloc<uint32_t>(threads * kIcLight);
        fill_u32(A.bitmaps, 0, threads * words, hs);
        A.counts = T.alloc<uint32_t>(total);
        A.heavy = T.alloc<uint32_t>(total);
        A.nheavy = T.alloc<unsigned long long>(1);
        fill_u64((uint64_t *)A.nheavy, 0, 1, hs);
        const unsigned grid = (unsigned)(threads / kIcBlock);
        // One pass when the light searches' records fit a buffer sized up
        // front (32 per position, at most kIcRecordCap): they are appended
        // as the searches end.  Otherwise, or for the handed-over searches,
        // a counting pass, a scan and a writing pass.
        uint64_t rcap = std::min<uint64_t>(std::max<uint64_t>(total * 32, 1u << 20), kIcRecordCap);
        if (take_fault(kFaultIcRecords)) rcap = 1;  // tests of the counting path
        uint64_t *recbuf = T.alloc<uint64_t>(rcap);
        A.records = recbuf;
        A.rcap = rcap;
        A.rcount = T.alloc<unsigned long long>(1);
        A.ovf = T.alloc<uint32_t>(1);
        fill_u64((uint64_t *)A.rcount, 0, 1, hs);
        fill_u32(A.ovf, 0, 1, hs);
        {
            LaunchTimer t("k_ic_search", hs);
            k_ic_search<2><<<grid, kIcBlock, 0, hs>>>(A);
            SKIM_LAUNCH_CHECK();
        }
        uint32_t ovf = 0;
        uint64_t rlight = 0;
        read_back(&ovf, A.ovf, sizeof ovf, hs);
        read_back(&rlight, A.rcount, sizeof rlight, hs);
        if (ovf) {  // back to counting first
            rlight = 0;
            fill_u64((uint64_t *)A.nheavy, 0, 1, hs);
            LaunchTimer t("k_ic_search", hs);
            k_ic_search<0><<<grid, kIcBlock, 0, hs>>>(A);
            SKIM_LAUNCH_CHECK();
        }
        uint64_t nheavy = 0;
        read_back(&nheavy, A.nheavy, sizeof nheavy, hs);
        unsigned hgrid = 1;
        if (nheavy) {
            const uint64_t per_block = ((uint64_t)words + n) * sizeof(uint32_t);
            uint64_t blocks = std::max<uint64_t>(1, kIcHeavyBudget / per_block);
            blocks = std::min<uint64_t>(std::min<uint64_t>(blocks, 1024), nheavy);
            hgrid = (unsigned)blocks;
            A.hbitmaps = T.alloc<uint32_t>(blocks * words);
            A.hqueues = T.alloc<uint32_t>(blocks * n);
            fill_u32(A.hbitmaps, 0, blocks * words, hs);
            LaunchTimer t("k_ic_heavy", hs);
            k_ic_heavy<0><<<hgrid, kIcHeavyBlock, 0, hs>>>(A, nheavy);
            SKIM_LAUNCH_CHECK();
        }
        // offsets of what is still to be written: every search after a
        // counting pass, the handed-over ones after the single pass
        uint64_t *offsets = T.alloc<uint64_t>(total + 1);
        exclusive_scan_u32(A.counts, offsets, total, T);
        uint64_t rrest = 0;
        read_back(&rrest, offsets + total, sizeof rrest, hs);
        A.offsets = offsets;
        const uint64_t R = rlight + rrest;
        uint64_t *records = recbuf;
        if (R > rcap) {  // room for the rest after the appended records
            records = T.alloc<uint64_t>(R);
            if (rlight)
                SKIM_HIP(hipMemcpyAsync(records, recbuf, rlight * sizeof(uint64_t),
                                        hipMemcpyDeviceToDevice, hs));
            T.release(recbuf);
        }
        A.records = records + rlight;
        if (ovf) {
            LaunchTimer t("k_ic_search", hs);
            k_ic_search<1><<<grid, kIcBlock, 0, hs>>>(A);
            SKIM_LAUNCH_CHECK();
        }
        if (nheavy) {
            LaunchTimer t("k_ic_heavy", hs);
            k_ic_heavy<1><<<hgrid, kIcHeavyBlock, 0, hs>>>(A, nheavy);
            SKIM_LAUNCH_CHECK();
        }
        A.records = records;
        T.release(A.bitmaps);
        T.release(A.queues);
        if (nheavy) {
            T.release(A.hbitmaps);
            T.release(A.hqueues);
        }
        // records by (node, position); every node keeps its first k
        uint64_t *sorted = T.alloc<uint64_t>(R);
        // the keys' high bits above the node id are zero: large sorts skip
        // them (small ones take the whole key)
        int node_bits = 1;
        while (node_bits < 32 && (1ull << node_bits) < n) ++node_bits;
        const unsigned end_bit = R > (1ull << 21) ? 32u + (unsigned)node_bits : 64u;
        tmp_bytes = 0;
        SKIM_HIP(rocprim::radix_sort_keys(nullptr, tmp_bytes, A.records, sorted, (size_t)R, 0u,
                                          end_bit, hs));
        tmp = T.get(tmp_bytes);
        SKIM_HIP(rocprim::radix_sort_keys(tmp, tmp_bytes, A.records, sorted, (size_t)R, 0u, end_bit,
                                          hs));
        uint64_t *start = T.alloc<uint64_t>(n);
        k_ic_starts<<<grid_for(R, 256, 16384), 256, 0, hs>>>(sorted, R, start);
        SKIM_LAUNCH_CHECK();
        k_ic_select<<<grid_for(n, 256, 4096), 256, 0, hs>>>(sorted, start, n, k, positions, est);
        SKIM_LAUNCH_CHECK();
        SKIM_HIP(hipStreamSynchronize(hs));
        return SKIM_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}
