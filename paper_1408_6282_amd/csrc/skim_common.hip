// skim_common.hip -- host plumbing shared by every entry point: errors,
// cached scratch allocation, fills, exclusive scan, graph validation, and the
// per-node estimate entry point.
#include "skim_internal.h"

#include <atomic>

#include <chrono>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <string>

namespace skim {

namespace {
thread_local char g_err[512] = "";

}  // namespace

void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof g_err, fmt, ap);
    va_end(ap);
}

void clear_error() { g_err[0] = 0; }

// ----------------------------------------------------- scratch allocation
// Calls take their scratch from a per-device cache of device blocks: a block
// is allocated once (hipMalloc) and reused by later calls, so a build does
// not map ~20 GB afresh.  (The runtime's stream-ordered pool was measured to
// get slower with every call in a long-running process.)  An arena
// synchronises its stream (a persistent one, whose state calls on any stream
// may use, its device) before its blocks go back to the cache, so a cached
// block is never still in use by a queued kernel; blocks a call arena
// releases in the middle of the call are reused only by that arena (same
// stream).
namespace {
struct DeviceCache {
    std::multimap<size_t, void *> free;  // block size -> block
    size_t cached = 0;                   // bytes held in `free`
    size_t limit = 0;                    // most bytes to keep cached
};
std::mutex g_cache_mu;
DeviceCache g_cache[64];

// Size class: at most 1/8 above the request (256-byte granularity below 2 KiB).
size_t size_class(size_t bytes) {
    if (bytes < 2048) return (bytes + 255) & ~(size_t)255;
    int lg = 63 - __builtin_clzll((unsigned long long)bytes);
    const size_t step = (size_t)1 << (lg - 3);
    return (bytes + step - 1) & ~(step - 1);
}

int current_device() {
    int dev = 0;
    SKIM_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) {
        set_error("device index %d out of range", dev);
        throw Fail{SKIM_EUNSUPPORTED};
    }
    return dev;
}

// Free cached blocks of `dev` (largest first) until at most `keep` bytes stay.
void trim_cache(int dev, size_t keep) {
    DeviceCache &C = g_cache[dev];
    while (C.cached > keep && !C.free.empty()) {
        auto it = std::prev(C.free.end());
        C.cached -= it->first;
        (void)hipFree(it->second);
        C.free.erase(it);
    }
    (void)hipGetLastError();
}
}  // namespace

Arena::Arena(hipStream_t s, bool persistent) : s_(s), persistent_(persistent) {
    dev_ = current_device();
}

// Wait until nothing queued on the arena's device can still use its blocks:
// its stream, or for a persistent arena (state used by calls on any stream)
// the whole device.
static void quiesce(int dev, hipStream_t s, bool whole_device) {
    if (!whole_device) {
        (void)hipStreamSynchronize(s);
        (void)hipGetLastError();
        return;
    }
    int cur = dev;
    (void)hipGetDevice(&cur);
    if (cur != dev) (void)hipSetDevice(dev);
    (void)hipDeviceSynchronize();
    if (cur != dev) (void)hipSetDevice(cur);
    (void)hipGetLastError();
}

Arena::~Arena() {
    bool any = false;
    for (auto &b : bufs_) any |= b.p != nullptr;
    for (auto &b : spare_) any |= b.p != nullptr;
    if (!any) return;
    quiesce(dev_, s_, persistent_);
    std::lock_guard<std::mutex> lk(g_cache_mu);
    DeviceCache &C = g_cache[dev_];
    if (!C.limit) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) == hipSuccess && tot) C.limit = tot / 10 * 7;
        else C.limit = (size_t)64 << 30;
        (void)hipGetLastError();
    }
    for (auto *list : {&bufs_, &spare_})
        for (auto &b : *list)
            if (b.p) {
                C.free.emplace(b.bytes, b.p);
                C.cached += b.bytes;
                b.p = nullptr;
            }
    if (C.cached > C.limit) trim_cache(dev_, C.limit);
}

std::atomic<uint32_t> g_fault[4];

bool take_fault(FaultKind what) {
    std::atomic<uint32_t> &c = g_fault[what];
    uint32_t v = c.load();
    while (v && !c.compare_exchange_weak(v, v - 1)) {
    }
    return v != 0;
}

void *Arena::get(size_t bytes) {
    if (take_fault(kFaultAlloc)) {
        set_error("device allocation of %zu bytes failed: injected failure", bytes);
        throw Fail{SKIM_ENOMEM};
    }
    if (bytes == 0) bytes = 8;
    const size_t cls = size_class(bytes);
    void *p = nullptr;
    size_t got = cls;
    // a block this arena released earlier (same stream: ordered; persistent
    // arenas hand released blocks back to the cache instead)
    for (auto &b : spare_)
        if (b.p && b.bytes >= cls && b.bytes <= cls + cls / 4) {
            bufs_.push_back(b);
            b.p = nullptr;
            return bufs_.back().p;
        }
    {   // a cached block of this size class (or at most a quarter larger)
        std::lock_guard<std::mutex> lk(g_cache_mu);
        DeviceCache &C = g_cache[dev_];
        auto it = C.free.lower_bound(cls);
        if (it != C.free.end() && it->first <= cls + cls / 4) {
            p = it->second;
            got = it->first;
            C.cached -= it->first;
            C.free.erase(it);
        }
    }
    if (!p) {
        static const bool trace = std::getenv("SKIM_TRACE_ALLOC") != nullptr;
        const auto t0 = std::chrono::steady_clock::now();
        hipError_t e = hipMalloc(&p, cls);
        if (e != hipSuccess || !p) {  // give the cache back to the device and try once more
            (void)hipGetLastError();
            {
                std::lock_guard<std::mutex> lk(g_cache_mu);
                trim_cache(dev_, 0);
            }
            p = nullptr;
            e = hipMalloc(&p, cls);
        }
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            set_error("device allocation of %zu bytes failed: %s", cls, hipGetErrorString(e));
            throw Fail{SKIM_ENOMEM};
        }
        if (trace) {
            size_t held = 0, spare = 0;
            for (auto &b : bufs_) held += b.p ? b.bytes : 0;
            for (auto &b : spare_) spare += b.p ? b.bytes : 0;
            std::fprintf(stderr, "skim alloc %.3f GB in %.1f ms (arena holds %.3f GB, %.3f GB spare)\n",
                         cls / 1e9,
                         std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0)
                             .count(),
                         held / 1e9, spare / 1e9);
        }
    }
    bufs_.push_back({p, got});
    return p;
}

void Arena::release(void *p) {
    if (!p) return;
    for (auto &b : bufs_)
        if (b.p == p) {
            if (persistent_) {  // to the cache, once nothing can still use it
                quiesce(dev_, s_, true);
                std::lock_guard<std::mutex> lk(g_cache_mu);
                g_cache[dev_].free.emplace(b.bytes, b.p);
                g_cache[dev_].cached += b.bytes;
            } else {
                spare_.push_back(b);  // reusable by this arena's later allocations
            }
            b.p = nullptr;
        }
}

void *pinned_scratch(size_t bytes) {
    thread_local void *buf = nullptr;
    thread_local size_t cap = 0;
    if (bytes > cap) {
        if (buf) (void)hipHostFree(buf);
        buf = nullptr;
        cap = 0;
        size_t want = bytes < 4096 ? 4096 : bytes;
        SKIM_HIP(hipHostMalloc(&buf, want, hipHostMallocDefault));
        cap = want;
    }
    return buf;
}

void read_back(void *host, const void *dev, size_t bytes, hipStream_t s) {
    void *pin = pinned_scratch(bytes);
    SKIM_HIP(hipMemcpyAsync(pin, dev, bytes, hipMemcpyDeviceToHost, s));
    SKIM_HIP(hipStreamSynchronize(s));
    std::memcpy(host, pin, bytes);
}

// ------------------------------------------------------------ kernel timing
namespace {
std::mutex g_time_mu;
std::string g_time_kernel;  // ",name,name," of the kernels timed; empty = timing off
struct TimeAcc {
    double ms = 0;
    uint64_t launches = 0;
};
std::map<std::string, TimeAcc> g_time_acc;
struct PendingTime {
    std::string name;
    hipEvent_t a, b;
};
thread_local std::vector<PendingTime> g_pending;
// Events are reused (creating and destroying two per launch costs more host
// time than the launch); one free list per device.
thread_local std::map<int, std::vector<hipEvent_t>> g_free_events;

hipEvent_t take_event() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return nullptr;
    auto &pool = g_free_events[dev];
    if (!pool.empty()) {
        hipEvent_t e = pool.back();
        pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void give_event(hipEvent_t e) {
    int dev = 0;
    if (!e) return;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipEventDestroy(e);
        return;
    }
    g_free_events[dev].push_back(e);
}
}  // namespace

LaunchTimer::LaunchTimer(const char *kernel, hipStream_t s) : s_(s), name_(kernel) {
    {
        std::lock_guard<std::mutex> lk(g_time_mu);
        if (g_time_kernel.empty() ||
            g_time_kernel.find("," + std::string(kernel) + ",") == std::string::npos)
            return;
    }
    a_ = take_event();
    if (a_ && hipEventRecord(a_, s_) != hipSuccess) {
        (void)hipGetLastError();
        give_event(a_);
        a_ = nullptr;
    }
}

LaunchTimer::~LaunchTimer() {
    if (!a_) return;
    hipEvent_t b = take_event();
    if (b && hipEventRecord(b, s_) == hipSuccess) {
        g_pending.push_back({name_, a_, b});
    } else {
        (void)hipGetLastError();
        give_event(a_);
        give_event(b);
    }
}

void timing_resolve() {
    for (auto &p : g_pending) {
        float ms = 0;
        if (hipEventSynchronize(p.b) == hipSuccess && hipEventElapsedTime(&ms, p.a, p.b) == hipSuccess) {
            std::lock_guard<std::mutex> lk(g_time_mu);
            auto &acc = g_time_acc[p.name];
            acc.ms += ms;
            acc.launches += 1;
        }
        (void)hipGetLastError();
        give_event(p.a);
        give_event(p.b);
    }
    g_pending.clear();
}

// ------------------------------------------------------------------- fills
__global__ void k_fill_u32(uint32_t *p, uint32_t v, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}
__global__ void k_fill_u64(uint64_t *p, uint64_t v, uint64_t n) {
    for (uint64_t i = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

void fill_u32(uint32_t *p, uint32_t value, uint64_t count, hipStream_t s) {
    if (!count) return;
    k_fill_u32<<<grid_for(count, 256, 8192), 256, 0, s>>>(p, value, count);
    SKIM_LAUNCH_CHECK();
}
void fill_u64(uint64_t *p, uint64_t value, uint64_t count, hipStream_t s) {
    if (!count) return;
    k_fill_u64<<<grid_for(count, 256, 8192), 256, 0, s>>>(p, value, count);
    SKIM_LAUNCH_CHECK();
}

// -------------------------------------------------------------------- scan
// Three phases: per-tile sums, scan of the tile sums, per-tile scan + offset.
constexpr int kScanBlock = 256;
constexpr int kScanPer = 16;
constexpr uint64_t kScanTile = (uint64_t)kScanBlock * kScanPer;

__device__ __forceinline__ uint64_t block_excl_scan(uint64_t x, uint64_t *sh, uint64_t *total) {
    // inclusive Hillis-Steele in shared memory, then shift
    const int t = threadIdx.x;
    sh[t] = x;
    __syncthreads();
    for (int off = 1; off < kScanBlock; off <<= 1) {
        uint64_t y = t >= off ? sh[t - off] : 0;
        __syncthreads();
        sh[t] += y;
        __syncthreads();
    }
    uint64_t incl = sh[t];
    *total = sh[kScanBlock - 1];
    __syncthreads();
    return incl - x;
}

__global__ void k_scan_tiles(const uint32_t *in, uint64_t n, uint64_t *tile_sum) {
    __shared__ uint64_t sh[kScanBlock];
    const uint64_t base = blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPer;
    uint64_t s = 0;
    for (int j = 0; j < kScanPer; ++j) {
        uint64_t i = base + j;
        if (i < n) s += in[i];
    }
    uint64_t tot;
    block_excl_scan(s, sh, &tot);
    if (threadIdx.x == 0) tile_sum[blockIdx.x] = tot;
}

__global__ void k_scan_sums(uint64_t *tile_sum, uint64_t ntiles) {
    __shared__ uint64_t sh[kScanBlock];
    __shared__ uint64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (uint64_t b = 0; b < ntiles; b += kScanBlock) {
        uint64_t i = b + threadIdx.x;
        uint64_t x = i < ntiles ? tile_sum[i] : 0;
        uint64_t tot;
        uint64_t ex = block_excl_scan(x, sh, &tot);
        if (i < ntiles) tile_sum[i] = ex + carry;
        __syncthreads();
        if (threadIdx.x == 0) carry += tot;
        __syncthreads();
    }
    if (threadIdx.x == 0) tile_sum[ntiles] = carry;
}

__global__ void k_scan_apply(const uint32_t *in, uint64_t n, const uint64_t *tile_sum,
                             uint64_t *out) {
    __shared__ uint64_t sh[kScanBlock];
    const uint64_t base = blockIdx.x * kScanTile + (uint64_t)threadIdx.x * kScanPer;
    uint32_t v[kScanPer];
    uint64_t s = 0;
    for (int j = 0; j < kScanPer; ++j) {
        uint64_t i = base + j;
        v[j] = i < n ? in[i] : 0;
        s += v[j];
    }
    uint64_t tot;
    uint64_t run = block_excl_scan(s, sh, &tot) + tile_sum[blockIdx.x];
    for (int j = 0; j < kScanPer; ++j) {
        uint64_t i = base + j;
        if (i < n) out[i] = run;
        run += v[j];
    }
}

__global__ void k_scan_total(uint64_t *out, uint64_t n, const uint64_t *tile_sum, uint64_t ntiles) {
    out[n] = tile_sum[ntiles];
}

void exclusive_scan_u32(const uint32_t *in, uint64_t *out, uint64_t n, Arena &a) {
    hipStream_t s = a.stream();
    const uint64_t ntiles = (n + kScanTile - 1) / kScanTile;
    uint64_t *ts = a.alloc<uint64_t>(ntiles + 1);
    if (ntiles) {
        if (ntiles > 0x7FFFFFFFull) {
            set_error("scan too large");
            throw Fail{SKIM_EUNSUPPORTED};
        }
        k_scan_tiles<<<(unsigned)ntiles, kScanBlock, 0, s>>>(in, n, ts);
        SKIM_LAUNCH_CHECK();
    }
    k_scan_sums<<<1, kScanBlock, 0, s>>>(ts, ntiles);
    SKIM_LAUNCH_CHECK();
    if (ntiles) {
        k_scan_apply<<<(unsigned)ntiles, kScanBlock, 0, s>>>(in, n, ts, out);
        SKIM_LAUNCH_CHECK();
    }
    k_scan_total<<<1, 1, 0, s>>>(out, n, ts, ntiles);
    SKIM_LAUNCH_CHECK();
    a.release(ts);
}

// --------------------------------------------------------------- validation
__global__ void k_check_rows(const uint64_t *rp, uint32_t n, uint64_t m, uint32_t *err) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t a = rp[v], b = rp[v + 1];
        uint32_t bad = 0;
        if (a > b || b > m) bad |= 1u;
        if (v == 0 && a != 0) bad |= 2u;
        if (v == n - 1 && b != m) bad |= 4u;
        if (bad) atomicOr(err, bad);
    }
}

// Source of every edge by binary search on row_ptr (indices stay in range
// even when row_ptr is invalid; such a graph is rejected anyway).
__global__ void k_check_edges(const uint64_t *rp, const uint32_t *col, uint32_t n, uint64_t m,
                              uint32_t *esrc, uint32_t *err) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint32_t lo = 0, hi = n;  // largest u with rp[u] <= e
        while (hi - lo > 1) {
            uint32_t mid = lo + (hi - lo) / 2;
            if (rp[mid] <= e) lo = mid;
            else hi = mid;
        }
        const uint32_t u = lo;
        const uint32_t v = col[e];
        uint32_t bad = 0;
        if (v >= n) bad |= 8u;
        if (v == u) bad |= 16u;
        if (e + 1 < m && e + 1 < rp[u + 1] && !(v < col[e + 1])) bad |= 32u;
        if (bad) atomicOr(err, bad);
        if (esrc) esrc[e] = u;
    }
}

void validate_graph(const skim_graph *g, uint32_t *esrc, Arena &a) {
    SKIM_REQUIRE(g != nullptr, "graph is NULL");
    SKIM_REQUIRE(g->n >= 1, "n must be >= 1");
    SKIM_REQUIRE((uint64_t)g->n * kPairStride < 0xFFFFFFFFull, "n too large (need 64 n < 2^32)");
    SKIM_REQUIRE(g->row_ptr != nullptr, "row_ptr is NULL");
    SKIM_REQUIRE(g->m == 0 || (g->col != nullptr && g->thr != nullptr), "col/thr is NULL");
    hipStream_t s = a.stream();
    uint32_t *err = a.alloc<uint32_t>(1);
    fill_u32(err, 0, 1, s);
    k_check_rows<<<grid_for(g->n, 256, 4096), 256, 0, s>>>(g->row_ptr, g->n, g->m, err);
    SKIM_LAUNCH_CHECK();
    if (g->m) {
        k_check_edges<<<grid_for(g->m, 256, 16384), 256, 0, s>>>(g->row_ptr, g->col, g->n, g->m,
                                                                 esrc, err);
        SKIM_LAUNCH_CHECK();
    }
    uint32_t herr = 0;
    read_back(&herr, err, sizeof herr, s);
    a.release(err);
    if (herr) {
        std::string why;
        if (herr & 7u) why += " row_ptr not a valid offset array;";
        if (herr & 8u) why += " head id >= n;";
        if (herr & 16u) why += " self-loop;";
        if (herr & 32u) why += " heads not strictly increasing within a row (unsorted or duplicate);";
        set_error("invalid graph:%s", why.c_str());
        throw Fail{SKIM_EINVAL};
    }
}

// ---------------------------------------------------------------- estimates
// perm_d = 0: hashed ranks, the bottom-k estimator; else sketches of
// structured permutation positions over perm_d = n l pairs.
__global__ void k_estimates(const uint64_t *ranks, const uint32_t *size, uint32_t n, uint32_t k,
                            uint32_t ell, double *est, uint64_t perm_d) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t sz = size[v];
        const uint64_t tau = sz >= k ? ranks[v * k + (k - 1)] : 0;
        est[v] = perm_d ? perm_estimate(sz, tau, k, ell, perm_d) : bottomk_estimate(sz, tau, k, ell);
    }
}

void launch_estimates(const uint64_t *ranks, const uint32_t *size, uint32_t n, uint32_t k,
                      uint32_t ell, double *est, hipStream_t s, uint64_t perm_d) {
    k_estimates<<<grid_for(n, 256, 8192), 256, 0, s>>>(ranks, size, n, k, ell, est, perm_d);
    SKIM_LAUNCH_CHECK();
}

}  // namespace skim

using namespace skim;

extern "C" uint32_t skim_abi_version(void) { return SKIM_ABI_VERSION; }

extern "C" skim_status skim_debug_inject(uint32_t what, uint32_t count) {
    skim::clear_error();
    if (what != SKIM_FAULT_ALLOC && what != SKIM_FAULT_SERVE && what != SKIM_FAULT_IC_RECORDS) {
        skim::set_error("unknown fault kind %u", what);
        return SKIM_EINVAL;
    }
    skim::g_fault[what].store(count);
    return SKIM_OK;
}

extern "C" void skim_timing_enable(const char *kernel) {
    std::lock_guard<std::mutex> lk(g_time_mu);
    g_time_kernel = kernel && *kernel ? "," + std::string(kernel) + "," : "";
}

extern "C" void skim_timing_reset(void) {
    std::lock_guard<std::mutex> lk(g_time_mu);
    g_time_acc.clear();
}

extern "C" int skim_timing_read(const char *kernel, double *total_ms, uint64_t *launches) {
    std::lock_guard<std::mutex> lk(g_time_mu);
    auto it = g_time_acc.find(kernel ? kernel : "");
    if (it == g_time_acc.end()) {
        if (total_ms) *total_ms = 0;
        if (launches) *launches = 0;
        return 0;
    }
    if (total_ms) *total_ms = it->second.ms;
    if (launches) *launches = it->second.launches;
    return 1;
}

extern "C" const char *skim_last_error(void) { return g_err; }

extern "C" skim_status skim_estimates(const uint64_t *ranks, const uint32_t *size, uint32_t n,
                                      uint32_t k, uint32_t ell, double *est, void *stream) {
    clear_error();
    try {
        SKIM_REQUIRE(ranks && size && est, "NULL pointer argument");
        SKIM_REQUIRE(n >= 1 && k >= 2 && k <= 256 && ell >= 1 && ell <= 64,
                     "need n >= 1, 2 <= k <= 256, 1 <= l <= 64");
        hipStream_t s = (hipStream_t)stream;
        launch_estimates(ranks, size, n, k, ell, est, s);
        SKIM_HIP(hipStreamSynchronize(s));
        return SKIM_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}
