// skim_query.hip -- influence queries from the sketches (Section 5.1).
//
// One wave per query.  The member sketches are sorted, so the distinct ranks
// of their union come out in increasing order from a k-way merge: each step
// takes the minimum head over the members (lane-local minimum, then a wave
// minimum), then advances every member whose head equals it.
//  * bottom-k estimator: stop at the k-th distinct value tau (or when the
//    union runs out), estimate as for a single sketch;
//  * Cohen-Kaplan (eq. unionest): run over every distinct non-threshold
//    value; its weight is 1/rho(max tau_u over the members holding it), a
//    non-full member counting as rho = 1; lane 0 adds the weights in
//    increasing order of the value.
// Each lane keeps its members' current heads in registers, so a merge step
// touches global memory only for the members that advance.
// The batched path is one persistent launch whose waves pull queries from a
// device counter; the plain path launches the same device code once per
// query.
#include "skim_internal.h"

#include <atomic>
#include <memory>

namespace skim {

namespace {

constexpr uint32_t kMaxMembers = 1024;  // members per query (LDS state)
constexpr int kQBlock = 64;             // one wave per block
constexpr int kPerLane = kMaxMembers / 64;

using QArgs = QueryArgs;

__device__ __forceinline__ uint64_t wave_min_u64(uint64_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)x, off);
        const uint32_t hi = __shfl_xor((uint32_t)(x >> 32), off);
        const uint64_t y = ((uint64_t)hi << 32) | lo;
        x = y < x ? y : x;
    }
    return x;
}

__device__ __forceinline__ uint64_t wave_max_u64(uint64_t x) {
    for (int off = 32; off > 0; off >>= 1) {
        const uint32_t lo = __shfl_xor((uint32_t)x, off);
        const uint32_t hi = __shfl_xor((uint32_t)(x >> 32), off);
        const uint64_t y = ((uint64_t)hi << 32) | lo;
        x = y > x ? y : x;
    }
    return x;
}

// The k-way merge over S members (R >= S / 64 register slots per lane).
// Each lane keeps the current head of its members t = lane + 64 r in
// registers; a step reads global memory only for the members that advance.
// Bottom-k stops at the k-th distinct value (d, tau); Cohen-Kaplan adds each
// distinct value's weight in increasing order on lane 0 (sum).
template <int R>
__device__ __forceinline__ void merge_members(const QArgs &Q, uint64_t S, uint32_t k,
                                              const uint32_t *mnode, uint16_t *mpos,
                                              const uint16_t *mlim, uint32_t &d, uint64_t &tau,
                                              double &sum) {
    const uint32_t lane = lane_id();
    uint64_t head[R];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const uint32_t t = lane + 64u * r;
        head[r] = kNone;
        if (t < S && mlim[t] > 0) head[r] = Q.ranks[(uint64_t)mnode[t] * k];
    }
    for (;;) {
        uint64_t lmin = kNone;
#pragma unroll
        for (int r = 0; r < R; ++r) lmin = head[r] < lmin ? head[r] : lmin;
        const uint64_t g = wave_min_u64(lmin);
        if (g == kNone) break;
        // advance the holders of g; for CK also find their largest threshold
        uint64_t tmax = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (head[r] == g) {
                const uint32_t t = lane + 64u * r;
                const uint32_t u = mnode[t];
                const uint32_t p = mpos[t] + 1u;
                mpos[t] = (uint16_t)p;
                head[r] = p < mlim[t] ? Q.ranks[(uint64_t)u * k + p] : kNone;
                if (Q.estimator == 1) {
                    const uint64_t tu = Q.size[u] >= k ? Q.ranks[(uint64_t)u * k + k - 1] : kNone;
                    tmax = tu > tmax ? tu : tmax;
                }
            }
        }
        if (Q.estimator == 1) {
            tmax = wave_max_u64(tmax);
            // the weight 1/r of the largest holder threshold: r = rho(T) for
            // hashed ranks, (T - 1)/(l n - 1) for permutation positions
            if (lane == 0)
                sum += tmax == kNone ? 1.0
                       : Q.perm_d    ? ((double)Q.perm_d - 1.0) / (double)(tmax - 1)
                                     : 1.0 / rank_real(tmax);
        } else {
            ++d;
            if (d == k) {
                tau = g;
                break;
            }
        }
    }
}

// Answer query j with the calling wave (all 64 lanes, converged).
__device__ void answer_query(const QArgs &Q, uint64_t j, uint32_t *mnode, uint16_t *mpos,
                             uint16_t *mlim) {
    const uint32_t lane = lane_id();
    const uint64_t a = Q.qoff[j], b = Q.qoff[j + 1];
    const uint32_t k = Q.k;
    // Offsets are validated before a batch; a replayed plan re-checks its
    // own set here (non-decreasing, within qoff[q]) and never reads outside.
    if (b < a || b > Q.qoff[Q.q] || b > Q.nodes_cap || (j == 0 && a != 0)) {
        if (lane == 0) {
            Q.est[j] = 0.0;
            if (Q.qstatus) Q.qstatus[j] = -3;
        }
        return;
    }
    const uint64_t S = b - a;
    // membership checks (node ids are validated per query)
    bool bad = false;
    for (uint64_t t = a + lane; t < b; t += 64) bad |= Q.qnodes[t] >= Q.n;
    bad = __ballot(bad) != 0;
    if (bad || S > kMaxMembers) {
        if (lane == 0) {
            Q.est[j] = 0.0;
            if (Q.qstatus) Q.qstatus[j] = bad ? -1 : -2;
        }
        return;
    }
    if (S == 0) {
        if (lane == 0) {
            Q.est[j] = 0.0;
            if (Q.qstatus) Q.qstatus[j] = 0;
        }
        return;
    }
    if (S == 1 && Q.estimator == 0) {
        if (lane == 0) {
            const uint32_t u = Q.qnodes[a];
            const uint32_t sz = Q.size[u];
            const uint64_t T = sz >= k ? Q.ranks[(uint64_t)u * k + k - 1] : 0;
            Q.est[j] = Q.perm_d ? perm_estimate(sz, T, k, Q.ell, Q.perm_d)
                                : bottomk_estimate(sz, T, k, Q.ell);
            if (Q.qstatus) Q.qstatus[j] = 0;
        }
        return;
    }
    // member state: node, next position, usable length
    for (uint32_t t = lane; t < S; t += 64) {
        const uint32_t u = Q.qnodes[a + t];
        const uint32_t sz = Q.size[u];
        mnode[t] = u;
        mpos[t] = 0;
        // CK ignores the threshold element of a full sketch
        mlim[t] = (uint16_t)(Q.estimator == 1 && sz >= k ? k - 1 : (sz < k ? sz : k));
    }
    __syncthreads();
    uint32_t d = 0;
    uint64_t tau = 0;
    double sum = 0.0;
    if (S <= 64)
        merge_members<1>(Q, S, k, mnode, mpos, mlim, d, tau, sum);
    else if (S <= 256)
        merge_members<4>(Q, S, k, mnode, mpos, mlim, d, tau, sum);
    else
        merge_members<kPerLane>(Q, S, k, mnode, mpos, mlim, d, tau, sum);
    if (lane == 0) {
        Q.est[j] = Q.estimator == 1 ? sum / (double)Q.ell
                   : Q.perm_d          ? perm_estimate(d, tau, k, Q.ell, Q.perm_d)
                                       : bottomk_estimate(d, tau, k, Q.ell);
        if (Q.qstatus) Q.qstatus[j] = 0;
    }
    __syncthreads();
}

__global__ void __launch_bounds__(kQBlock) k_query_persistent(QArgs Q, uint64_t q,
                                                               unsigned long long *next) {
    __shared__ uint32_t mnode[kMaxMembers];
    __shared__ uint16_t mpos[kMaxMembers];
    __shared__ uint16_t mlim[kMaxMembers];
    __shared__ unsigned long long jcur;
    // Queries are taken in runs that shrink as the batch drains (at most 32,
    // about a quarter of an even share of what is left): takes from
    // different waves on the one counter are serialised by the hardware, so
    // one query per take would cap the batch at the counter's rate.
    const uint64_t share = 4ull * gridDim.x;
    uint64_t g = q / share;
    g = g < 1 ? 1 : g > 32 ? 32 : g;
    for (;;) {
        if (threadIdx.x == 0) jcur = atomicAdd(next, (unsigned long long)g);
        __syncthreads();
        const uint64_t j0 = jcur;
        __syncthreads();
        if (j0 >= q) break;
        const uint64_t j1 = j0 + g < q ? j0 + g : q;
        for (uint64_t j = j0; j < j1; ++j) answer_query(Q, j, mnode, mpos, mlim);
        g = (q - j1) / share;
        g = g < 1 ? 1 : g > 32 ? 32 : g;
    }
}

__global__ void __launch_bounds__(kQBlock) k_query_one(QArgs Q, uint64_t j) {
    __shared__ uint32_t mnode[kMaxMembers];
    __shared__ uint16_t mpos[kMaxMembers];
    __shared__ uint16_t mlim[kMaxMembers];
    answer_query(Q, j, mnode, mpos, mlim);
}

__global__ void k_check_offsets(const uint64_t *qoff, uint64_t q, uint32_t *err) {
    for (uint64_t j = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; j <= q;
         j += (uint64_t)gridDim.x * blockDim.x) {
        if (j == 0 && qoff[0] != 0) atomicOr(err, 1u);
        if (j < q && qoff[j + 1] < qoff[j]) atomicOr(err, 2u);
    }
}

}  // namespace

unsigned query_grid(uint64_t q) {
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        cus = 256;
        if (hipGetDevice(&dev) == hipSuccess)
            (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        (void)hipGetLastError();
    }
    const uint64_t want = (uint64_t)cus * 16;
    return (unsigned)(q < want ? (q ? q : 1) : want);
}

void launch_queries_async(const QueryArgs &Q, uint64_t q, unsigned long long *next, hipStream_t s) {
    fill_u64((uint64_t *)next, 0, 1, s);
    k_query_persistent<<<query_grid(q), kQBlock, 0, s>>>(Q, q, next);
    SKIM_LAUNCH_CHECK();
}

static void query_batch(const uint64_t *ranks, const uint32_t *size, uint32_t n, uint32_t k,
                        uint32_t ell, uint64_t q, const uint64_t *qoff, const uint32_t *qnodes,
                        uint32_t estimator, uint32_t mode, double *est, int32_t *qstatus,
                        hipStream_t s, bool permutation = false) {
    SKIM_REQUIRE(ranks && size, "sketches are NULL");
    SKIM_REQUIRE(n >= 1 && k >= 2 && k <= 256 && ell >= 1 && ell <= 64,
                 "need n >= 1, 2 <= k <= 256, 1 <= l <= 64");
    SKIM_REQUIRE(estimator <= 1, "estimator must be 0 (bottom-k) or 1 (Cohen-Kaplan)");
    SKIM_REQUIRE(mode <= 1, "mode must be 0 (batched) or 1 (one launch per query)");
    if (q == 0) return;
    SKIM_REQUIRE(qoff && est, "qoff/est is NULL");
    Arena A(s);
    uint32_t *err = A.alloc<uint32_t>(1);
    fill_u32(err, 0, 1, s);
    k_check_offsets<<<grid_for(q + 1, 256, 4096), 256, 0, s>>>(qoff, q, err);
    SKIM_LAUNCH_CHECK();
    uint32_t herr = 0;
    read_back(&herr, err, sizeof herr, s);
    SKIM_REQUIRE(herr == 0, "qoff must start at 0 and be non-decreasing");
    uint64_t total = 0;
    read_back(&total, qoff + q, sizeof total, s);
    SKIM_REQUIRE(total == 0 || qnodes, "qnodes is NULL");
    QArgs Q{ranks, size, n, k, ell, q, qoff, qnodes, est, qstatus, estimator};
    if (permutation) Q.perm_d = (uint64_t)n * ell;
    if (mode == 0) {
        unsigned long long *next = A.alloc<unsigned long long>(1);
        LaunchTimer t("k_query_persistent", s);
        launch_queries_async(Q, q, next, s);
    } else {
        for (uint64_t j = 0; j < q; ++j) {
            k_query_one<<<1, kQBlock, 0, s>>>(Q, j);
            SKIM_LAUNCH_CHECK();
        }
    }
    SKIM_HIP(hipStreamSynchronize(s));
    timing_resolve();
}

}  // namespace skim

extern "C" skim_status skim_query_batch(const uint64_t *ranks, const uint32_t *size, uint32_t n,
                                        uint32_t k, uint32_t ell, uint64_t q, const uint64_t *qoff,
                                        const uint32_t *qnodes, uint32_t estimator, uint32_t mode,
                                        double *est, int32_t *qstatus, void *stream) {
    skim::clear_error();
    try {
        skim::query_batch(ranks, size, n, k, ell, q, qoff, qnodes, estimator, mode, est, qstatus,
                          (hipStream_t)stream);
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        return f.st;
    }
}

extern "C" skim_status skim_perm_query_batch(const uint64_t *ranks, const uint32_t *size,
                                             uint32_t n, uint32_t k, uint32_t ell, uint64_t q,
                                             const uint64_t *qoff, const uint32_t *qnodes,
                                             uint32_t estimator, double *est, int32_t *qstatus,
                                             void *stream) {
    skim::clear_error();
    try {
        skim::query_batch(ranks, size, n, k, ell, q, qoff, qnodes, estimator, 0, est, qstatus,
                          (hipStream_t)stream, true);
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        return f.st;
    }
}

// ------------------------------------------------------------ query plans
// A plan is the batched launch (counter reset by a fill kernel, then the
// persistent query kernel) captured once into a HIP graph; launching the plan
// replays the graph on the caller's stream.
struct skim_query_plan {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long *next = nullptr;
    uint64_t q = 0;
    int device = 0;
};

namespace skim {

static void plan_free(skim_query_plan *p) {
    if (!p) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (have) (void)hipSetDevice(p->device);
    if (p->exec) (void)hipGraphExecDestroy(p->exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    if (p->next) (void)hipFree(p->next);
    if (have) (void)hipSetDevice(cur);
    (void)hipGetLastError();
    delete p;
}

static skim_query_plan *plan_create(const uint64_t *ranks, const uint32_t *size, uint32_t n,
                                    uint32_t k, uint32_t ell, uint64_t q, const uint64_t *qoff,
                                    const uint32_t *qnodes, uint32_t estimator, double *est,
                                    int32_t *qstatus, hipStream_t s) {
    SKIM_REQUIRE(ranks && size, "sketches are NULL");
    SKIM_REQUIRE(n >= 1 && k >= 2 && k <= 256 && ell >= 1 && ell <= 64,
                 "need n >= 1, 2 <= k <= 256, 1 <= l <= 64");
    SKIM_REQUIRE(estimator <= 1, "estimator must be 0 (bottom-k) or 1 (Cohen-Kaplan)");
    SKIM_REQUIRE(q >= 1, "a plan needs q >= 1 sets");
    SKIM_REQUIRE(qoff && est, "qoff/est is NULL");
    {   // the offsets as they are now
        Arena A(s);
        uint32_t *err = A.alloc<uint32_t>(1);
        fill_u32(err, 0, 1, s);
        k_check_offsets<<<grid_for(q + 1, 256, 4096), 256, 0, s>>>(qoff, q, err);
        SKIM_LAUNCH_CHECK();
        uint32_t herr = 0;
        read_back(&herr, err, sizeof herr, s);
        SKIM_REQUIRE(herr == 0, "qoff must start at 0 and be non-decreasing");
        uint64_t total = 0;
        read_back(&total, qoff + q, sizeof total, s);
        SKIM_REQUIRE(total == 0 || qnodes, "qnodes is NULL");
    }
    std::unique_ptr<skim_query_plan, void (*)(skim_query_plan *)> p(new skim_query_plan,
                                                                   plan_free);
    SKIM_HIP(hipGetDevice(&p->device));
    p->q = q;
    SKIM_HIP(hipMalloc(&p->next, sizeof(unsigned long long)));
    hipStream_t cs = nullptr;
    SKIM_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
    QArgs Q{ranks, size, n, k, ell, q, qoff, qnodes, est, qstatus, estimator};
    hipError_t e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (e == hipSuccess) {
        try {
            launch_queries_async(Q, q, p->next, cs);
        } catch (const Fail &) {
            hipGraph_t g = nullptr;
            (void)hipStreamEndCapture(cs, &g);
            if (g) (void)hipGraphDestroy(g);
            (void)hipStreamDestroy(cs);
            throw;
        }
        e = hipStreamEndCapture(cs, &p->graph);
    }
    (void)hipStreamDestroy(cs);
    SKIM_HIP(e);
    SKIM_HIP(hipGraphInstantiate(&p->exec, p->graph, nullptr, nullptr, 0));
    return p.release();
}

}  // namespace skim

extern "C" skim_status skim_query_plan_create(const uint64_t *ranks, const uint32_t *size,
                                              uint32_t n, uint32_t k, uint32_t ell, uint64_t q,
                                              const uint64_t *qoff, const uint32_t *qnodes,
                                              uint32_t estimator, double *est, int32_t *qstatus,
                                              void *stream, skim_query_plan **plan) {
    skim::clear_error();
    if (!plan) {
        skim::set_error("plan is NULL");
        return SKIM_EINVAL;
    }
    *plan = nullptr;
    try {
        *plan = skim::plan_create(ranks, size, n, k, ell, q, qoff, qnodes, estimator, est, qstatus,
                                  (hipStream_t)stream);
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        return f.st;
    }
}

extern "C" skim_status skim_query_plan_launch(skim_query_plan *plan, void *stream) {
    skim::clear_error();
    if (!plan) {
        skim::set_error("plan is NULL");
        return SKIM_EINVAL;
    }
    try {
        skim::LaunchTimer t("k_query_persistent", (hipStream_t)stream);
        SKIM_HIP(hipGraphLaunch(plan->exec, (hipStream_t)stream));
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        return f.st;
    }
}

extern "C" void skim_query_plan_free(skim_query_plan *plan) { skim::plan_free(plan); }

// -------------------------------------------------------- resident sketches
// A library-owned copy of a sketch table (ranks, sizes, per-node estimates)
// answering union queries with one enqueue-only launch: no host check of the
// offsets (the query kernel checks every set on the device, status -3) and
// no wait, so the call can be captured into a HIP graph.  The persistent
// kernel's work counter is reset by a fill kernel on the stream (no memset
// node) and comes from a ring of per-handle counters, or from a workspace the
// caller passes.
struct skim_sketches {
    int device = 0;
    uint32_t n = 0, k = 0, ell = 0;
    uint64_t *ranks = nullptr;
    uint32_t *size = nullptr;
    double *est = nullptr;
    unsigned long long *counters = nullptr;  // kRing counters, one 128-byte line each
    std::atomic<uint32_t> turn{0};
};

namespace skim {

constexpr uint32_t kRing = 64;

static void sketches_free(skim_sketches *h) {
    if (!h) return;
    int cur = 0;
    const bool have = hipGetDevice(&cur) == hipSuccess;
    if (have) (void)hipSetDevice(h->device);
    (void)hipDeviceSynchronize();  // no queued work may still use the buffers
    (void)hipFree(h->ranks);
    (void)hipFree(h->size);
    (void)hipFree(h->est);
    (void)hipFree(h->counters);
    if (have) (void)hipSetDevice(cur);
    (void)hipGetLastError();
    delete h;
}

static skim_sketches *sketches_alloc(uint32_t n, uint32_t k, uint32_t ell) {
    SKIM_REQUIRE(n >= 1 && k >= 2 && k <= 256 && ell >= 1 && ell <= 64,
                 "need n >= 1, 2 <= k <= 256, 1 <= l <= 64");
    if (take_fault(kFaultAlloc)) {
        set_error("device allocation for resident sketches failed: injected failure");
        throw Fail{SKIM_ENOMEM};
    }
    std::unique_ptr<skim_sketches, void (*)(skim_sketches *)> h(new skim_sketches,
                                                                sketches_free);
    SKIM_HIP(hipGetDevice(&h->device));
    h->n = n;
    h->k = k;
    h->ell = ell;
    SKIM_HIP(hipMalloc(&h->ranks, (size_t)n * k * sizeof(uint64_t)));
    SKIM_HIP(hipMalloc(&h->size, (size_t)n * sizeof(uint32_t)));
    SKIM_HIP(hipMalloc(&h->est, (size_t)n * sizeof(double)));
    SKIM_HIP(hipMalloc(&h->counters, (size_t)kRing * 128));
    return h.release();
}

}  // namespace skim

extern "C" skim_status skim_sketches_create(const uint64_t *ranks, const uint32_t *size,
                                            uint32_t n, uint32_t k, uint32_t ell, void *stream,
                                            skim_sketches **out) {
    skim::clear_error();
    if (!out) {
        skim::set_error("out is NULL");
        return SKIM_EINVAL;
    }
    *out = nullptr;
    try {
        SKIM_REQUIRE(ranks && size, "sketches are NULL");
        skim_sketches *h = skim::sketches_alloc(n, k, ell);
        hipStream_t s = (hipStream_t)stream;
        try {
            SKIM_HIP(hipMemcpyAsync(h->ranks, ranks, (size_t)n * k * 8, hipMemcpyDeviceToDevice, s));
            SKIM_HIP(hipMemcpyAsync(h->size, size, (size_t)n * 4, hipMemcpyDeviceToDevice, s));
            skim::launch_estimates(h->ranks, h->size, n, k, ell, h->est, s);
        } catch (const skim::Fail &) {
            skim::sketches_free(h);
            throw;
        }
        *out = h;
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        return f.st;
    }
}

extern "C" skim_status skim_build_sketches_resident(const skim_graph *g, uint32_t ell, uint32_t k,
                                                    uint64_t seed, uint64_t *work, void *stream,
                                                    skim_sketches **out) {
    skim::clear_error();
    if (!out || !g) {
        skim::set_error("NULL argument");
        return SKIM_EINVAL;
    }
    *out = nullptr;
    skim_sketches *h = nullptr;
    try {
        h = skim::sketches_alloc(g->n, k, ell);
    } catch (const skim::Fail &f) {
        return f.st;
    }
    const skim_status st =
        skim_build_sketches(g, ell, k, seed, h->ranks, h->size, h->est, work, stream);
    if (st != SKIM_OK) {
        skim::sketches_free(h);
        return st;
    }
    *out = h;
    return SKIM_OK;
}

extern "C" skim_status skim_sketches_data(const skim_sketches *h, const uint64_t **ranks,
                                          const uint32_t **size, const double **est, uint32_t *n,
                                          uint32_t *k, uint32_t *ell) {
    skim::clear_error();
    if (!h) {
        skim::set_error("handle is NULL");
        return SKIM_EINVAL;
    }
    if (ranks) *ranks = h->ranks;
    if (size) *size = h->size;
    if (est) *est = h->est;
    if (n) *n = h->n;
    if (k) *k = h->k;
    if (ell) *ell = h->ell;
    return SKIM_OK;
}

extern "C" skim_status skim_sketches_query(const skim_sketches *hc, uint64_t q, const uint64_t *qoff,
                                           const uint32_t *qnodes, uint64_t nnodes,
                                           uint32_t estimator, double *est, int32_t *qstatus,
                                           void *workspace, void *stream) {
    skim::clear_error();
    skim_sketches *h = const_cast<skim_sketches *>(hc);
    if (!h) {
        skim::set_error("handle is NULL");
        return SKIM_EINVAL;
    }
    try {
        SKIM_REQUIRE(estimator <= 1, "estimator must be 0 (bottom-k) or 1 (Cohen-Kaplan)");
        if (q == 0) return SKIM_OK;
        SKIM_REQUIRE(qoff && est, "qoff/est is NULL");
        SKIM_REQUIRE(nnodes == 0 || qnodes, "qnodes is NULL");
        skim::QueryArgs Q{h->ranks, h->size, h->n, h->k, h->ell, q, qoff, qnodes, est, qstatus,
                          estimator, nnodes};
        unsigned long long *next =
            workspace ? (unsigned long long *)workspace
                      : h->counters + 16 * (h->turn.fetch_add(1) % skim::kRing);
        skim::launch_queries_async(Q, q, next, (hipStream_t)stream);
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        return f.st;
    }
}

extern "C" void skim_sketches_free(skim_sketches *h) { skim::sketches_free(h); }
