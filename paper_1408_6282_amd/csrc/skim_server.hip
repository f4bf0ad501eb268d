// skim_server.cpp -- serving loop: resident sketches, memory-budget admission,
// continuous batching of union queries over several HIP streams, and
// incremental SKIM requests that overlap with them on the device.
//
// Requests enter a FIFO when their bytes fit the remaining budget (else the
// caller is told SKIM_EBUSY).  A worker thread keeps up to `streams` batches
// in flight: whenever a stream slot is free it packs every waiting query that
// fits the slot into one persistent launch (staging in pinned memory, H2D,
// kernel, D2H, event), and it retires batches as their events complete.  A
// second worker runs SKIM requests in order on their own stream, resuming one
// device-resident SKIM state.  Latency runs from the request's arrival to the
// moment the host observes its batch complete.
//
// Failures never leave a slot busy: a batch whose copy, launch or
// completion event reports an error completes with status -5 for every
// request in it, and its slot is freed, so skim_server_destroy always
// returns.  Requests can be cancelled (status -6).
#include "skim_internal.h"

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cstring>
#include <condition_variable>
#include <deque>
#include <memory>
#include <mutex>
#include <thread>
#include <unordered_map>

namespace skim {
skim_greedy_state *greedy_create(const skim_graph *g, uint32_t ell, uint32_t k, uint64_t seed,
                                 hipStream_t s);
void greedy_run(skim_greedy_state *st, uint32_t s_goal, uint32_t *seeds, uint64_t *gains,
                double *gain_d, hipStream_t s);
}  // namespace skim

using Clock = std::chrono::steady_clock;

namespace {

struct QueryReq {
    uint64_t ticket;
    std::vector<uint32_t> nodes;
    Clock::time_point t0;
    size_t bytes;
};

struct GreedyReq {
    uint64_t ticket;
    uint32_t s;
    Clock::time_point t0;
    size_t bytes;
};

struct QueryDone {
    double est;
    int32_t status;
    double lat_us;
};

struct GreedyDone {
    std::vector<uint32_t> seeds;
    std::vector<uint64_t> gains;
    double lat_us;
    skim_status status;
};

// A batch of q queries moves in one copy each way: in = q + 1 offsets
// (8 B) followed by the member nodes (4 B), out = q estimates (8 B)
// followed by q statuses (4 B).
struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    uint8_t *h_in = nullptr, *d_in = nullptr;    // pinned / device
    uint8_t *h_out = nullptr, *d_out = nullptr;  // pinned / device
    unsigned long long *d_next = nullptr;
    uint32_t cap_q = 0;
    uint64_t cap_nodes = 0;
    bool busy = false;
    std::vector<QueryReq> reqs;
};

size_t query_bytes(size_t count) { return count * 4 + 8 + 8 + 4; }
size_t greedy_bytes(uint32_t s) { return (size_t)s * 12 + 64; }

constexpr int32_t kStatusFailed = -5, kStatusCancelled = -6;

}  // namespace

struct skim_server {
    int device = 0;
    skim_server_config cfg{};
    skim::QueryArgs base{};
    std::vector<Slot> slots;

    std::mutex mu;
    // Each worker sleeps on its own condition variable; a submission wakes the
    // query worker only while it sleeps (a wake-up per request, and waking
    // the other worker too, cost more than the work of a small request).
    std::condition_variable cv_q, cv_g;
    bool q_sleeping = false;  // under mu
    std::deque<QueryReq> pending;
    std::deque<GreedyReq> gpending;
    std::unordered_map<uint64_t, QueryDone> done;
    std::unordered_map<uint64_t, GreedyDone> gdone;
    std::unordered_map<uint64_t, int> live;  // ticket -> 1 query, 2 greedy
    std::unordered_map<uint64_t, bool> cancelled;  // in a batch on the GPU, result dropped
    uint64_t next_ticket = 1;
    size_t inflight_bytes = 0;
    std::atomic<bool> stop{false};
    std::thread worker, gworker;

    // SKIM over the server
    skim_graph g{};
    uint32_t g_ell = 0, g_k = 0;
    uint64_t g_seed = 0;
    bool has_graph = false;
    skim_greedy_state *gstate = nullptr;
    hipStream_t gstream = nullptr;

    void run_queries();
    void run_greedy();
    bool launch_batch(Slot &sl);
    void retire(Slot &sl);
    void fail_batch(Slot &sl);
};

void skim_server::retire(Slot &sl) {
    const auto now = Clock::now();
    std::lock_guard<std::mutex> lk(mu);
    const size_t q = sl.reqs.size();
    const double *est = (const double *)sl.h_out;
    const int32_t *st = (const int32_t *)(sl.h_out + q * 8);
    for (size_t j = 0; j < q; ++j) {
        auto &r = sl.reqs[j];
        const double lat = std::chrono::duration<double, std::micro>(now - r.t0).count();
        if (cancelled.erase(r.ticket)) done[r.ticket] = {0.0, kStatusCancelled, lat};
        else done[r.ticket] = {est[j], st[j], lat};
        inflight_bytes -= r.bytes;
    }
    sl.reqs.clear();
    sl.busy = false;
}

// The batch's copy, launch or completion failed: every request in it
// completes with status -5 and the slot is free again.  The stream is
// synchronised first (its error, if any, is only reported) so that no copy
// into the slot's buffers is still queued when the slot is reused.
void skim_server::fail_batch(Slot &sl) {
    (void)hipStreamSynchronize(sl.stream);
    (void)hipGetLastError();
    const size_t q = sl.reqs.size();
    for (size_t j = 0; j < q; ++j) {
        ((double *)sl.h_out)[j] = 0.0;
        ((int32_t *)(sl.h_out + q * 8))[j] = kStatusFailed;
    }
    retire(sl);
}

bool skim_server::launch_batch(Slot &sl) {
    {
        std::lock_guard<std::mutex> lk(mu);
        uint64_t nn = 0;
        while (!pending.empty() && sl.reqs.size() < sl.cap_q &&
               nn + pending.front().nodes.size() <= sl.cap_nodes) {
            nn += pending.front().nodes.size();
            sl.reqs.push_back(std::move(pending.front()));
            pending.pop_front();
        }
    }
    if (sl.reqs.empty()) return false;
    const uint64_t q = sl.reqs.size();
    uint64_t *h_off = (uint64_t *)sl.h_in;
    uint32_t *h_nodes = (uint32_t *)(sl.h_in + (q + 1) * 8);
    uint64_t o = 0;
    for (uint64_t j = 0; j < q; ++j) {
        h_off[j] = o;
        const auto &nd = sl.reqs[j].nodes;
        if (!nd.empty()) std::memcpy(h_nodes + o, nd.data(), nd.size() * 4);
        o += nd.size();
    }
    h_off[q] = o;
    hipStream_t s = sl.stream;
    if (skim::take_fault(skim::kFaultServe) ||
        hipMemcpyAsync(sl.d_in, sl.h_in, (q + 1) * 8 + o * 4, hipMemcpyHostToDevice, s) !=
            hipSuccess) {
        fail_batch(sl);
        return true;
    }
    skim::QueryArgs Q = base;
    Q.q = q;
    Q.qoff = (const uint64_t *)sl.d_in;
    Q.qnodes = (const uint32_t *)(sl.d_in + (q + 1) * 8);
    Q.est = (double *)sl.d_out;
    Q.qstatus = (int32_t *)(sl.d_out + q * 8);
    try {
        skim::launch_queries_async(Q, q, sl.d_next, s);
    } catch (const skim::Fail &) {
        fail_batch(sl);
        return true;
    }
    if (hipMemcpyAsync(sl.h_out, sl.d_out, q * 12, hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipEventRecord(sl.ev, s) != hipSuccess) {
        fail_batch(sl);
        return true;
    }
    sl.busy = true;
    return true;
}

void skim_server::run_queries() {
    (void)hipSetDevice(device);
    while (true) {
        bool progressed = false;
        for (auto &sl : slots)
            if (sl.busy) {
                const hipError_t q = hipEventQuery(sl.ev);
                (void)hipGetLastError();  // "not ready" is not a failure
                if (q == hipSuccess) {
                    retire(sl);
                    progressed = true;
                } else if (q != hipErrorNotReady) {  // the batch failed on the device
                    fail_batch(sl);
                    progressed = true;
                }
            }
        for (auto &sl : slots)
            if (!sl.busy && launch_batch(sl)) progressed = true;
        if (progressed) continue;
        bool any_busy = false;
        for (auto &sl : slots) any_busy |= sl.busy;
        std::unique_lock<std::mutex> lk(mu);
        if (stop && pending.empty() && !any_busy) break;
        if (!any_busy && pending.empty()) {
            q_sleeping = true;
            cv_q.wait_for(lk, std::chrono::milliseconds(1));
            q_sleeping = false;
        }
        else if (any_busy) {
            lk.unlock();
            std::this_thread::yield();
        }
    }
}

void skim_server::run_greedy() {
    (void)hipSetDevice(device);
    while (true) {
        GreedyReq r;
        {
            std::unique_lock<std::mutex> lk(mu);
            cv_g.wait_for(lk, std::chrono::milliseconds(1), [&] { return stop || !gpending.empty(); });
            if (gpending.empty()) {
                if (stop) break;
                continue;
            }
            r = gpending.front();
            gpending.pop_front();
        }
        GreedyDone d;
        d.status = SKIM_OK;
        try {
            if (!gstate) gstate = skim::greedy_create(&g, g_ell, g_k, g_seed, gstream);
            skim::Arena A(gstream);
            uint32_t *ds = A.alloc<uint32_t>(r.s ? r.s : 1);
            uint64_t *dg = A.alloc<uint64_t>(r.s ? r.s : 1);
            if (r.s) skim::greedy_run(gstate, r.s, ds, dg, nullptr, gstream);
            d.seeds.resize(r.s);
            d.gains.resize(r.s);
            if (r.s) {
                SKIM_HIP(hipMemcpyAsync(d.seeds.data(), ds, r.s * 4, hipMemcpyDeviceToHost, gstream));
                SKIM_HIP(hipMemcpyAsync(d.gains.data(), dg, r.s * 8, hipMemcpyDeviceToHost, gstream));
            }
            SKIM_HIP(hipStreamSynchronize(gstream));
        } catch (const skim::Fail &f) {
            d.status = f.st;
        }
        d.lat_us = std::chrono::duration<double, std::micro>(Clock::now() - r.t0).count();
        std::lock_guard<std::mutex> lk(mu);
        inflight_bytes -= r.bytes;
        gdone[r.ticket] = std::move(d);
    }
}

namespace {

skim_status submit_query(skim_server *sv, const uint32_t *nodes, uint32_t count, uint64_t *ticket,
                         Clock::time_point t0) {
    const size_t b = query_bytes(count);
    if (b > sv->cfg.budget_bytes || count > sv->slots[0].cap_nodes) {
        skim::set_error("request of %u nodes can never fit the budget or a batch", count);
        return SKIM_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->inflight_bytes + b > sv->cfg.budget_bytes) return SKIM_EBUSY;
    sv->inflight_bytes += b;
    QueryReq r;
    r.ticket = sv->next_ticket++;
    r.nodes.assign(nodes, nodes + count);
    r.t0 = t0;
    r.bytes = b;
    *ticket = r.ticket;
    sv->live[r.ticket] = 1;
    sv->pending.push_back(std::move(r));
    if (sv->q_sleeping) sv->cv_q.notify_one();
    return SKIM_OK;
}

}  // namespace

extern "C" skim_status skim_server_create(const uint64_t *ranks, const uint32_t *size, uint32_t n,
                                          uint32_t k, uint32_t ell, const skim_server_config *cfg,
                                          skim_server **out) {
    skim::clear_error();
    try {
        SKIM_REQUIRE(out && ranks && size && cfg, "NULL argument");
        SKIM_REQUIRE(n >= 1 && k >= 2 && k <= 256 && ell >= 1 && ell <= 64,
                     "need n >= 1, 2 <= k <= 256, 1 <= l <= 64");
        SKIM_REQUIRE(cfg->estimator <= 1, "estimator must be 0 or 1");
        SKIM_REQUIRE(cfg->streams >= 1 && cfg->streams <= 16, "streams must be in [1, 16]");
        SKIM_REQUIRE(cfg->max_batch >= 1, "max_batch must be >= 1");
        SKIM_REQUIRE(cfg->budget_bytes >= 4096, "budget too small");
        auto sv = std::make_unique<skim_server>();
        SKIM_HIP(hipGetDevice(&sv->device));
        sv->cfg = *cfg;
        sv->base = skim::QueryArgs{ranks, size, n, k, ell, 0, nullptr, nullptr, nullptr, nullptr,
                                   cfg->estimator};
        const uint64_t cap_nodes = std::max<uint64_t>(1024, cfg->budget_bytes / 4 / cfg->streams);
        sv->slots.resize(cfg->streams);
        for (auto &sl : sv->slots) {
            sl.cap_q = cfg->max_batch;
            sl.cap_nodes = cap_nodes;
            SKIM_HIP(hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking));
            SKIM_HIP(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
            const size_t in_bytes = ((size_t)sl.cap_q + 1) * 8 + cap_nodes * 4;
            const size_t out_bytes = (size_t)sl.cap_q * 12;
            SKIM_HIP(hipHostMalloc((void **)&sl.h_in, in_bytes, hipHostMallocDefault));
            SKIM_HIP(hipHostMalloc((void **)&sl.h_out, out_bytes, hipHostMallocDefault));
            SKIM_HIP(hipMalloc((void **)&sl.d_in, in_bytes));
            SKIM_HIP(hipMalloc((void **)&sl.d_out, out_bytes));
            SKIM_HIP(hipMalloc((void **)&sl.d_next, 8));
        }
        SKIM_HIP(hipStreamCreateWithFlags(&sv->gstream, hipStreamNonBlocking));
        skim_server *raw = sv.get();
        sv->worker = std::thread([raw] { raw->run_queries(); });
        sv->gworker = std::thread([raw] { raw->run_greedy(); });
        *out = sv.release();
        return SKIM_OK;
    } catch (const skim::Fail &f) {
        return f.st;
    }
}

extern "C" void skim_server_destroy(skim_server *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
    }
    sv->cv_q.notify_all();
    sv->cv_g.notify_all();
    if (sv->worker.joinable()) sv->worker.join();
    if (sv->gworker.joinable()) sv->gworker.join();
    for (auto &sl : sv->slots) {
        if (sl.stream) (void)hipStreamSynchronize(sl.stream);
        (void)hipFree(sl.d_in);
        (void)hipFree(sl.d_out);
        (void)hipFree(sl.d_next);
        (void)hipHostFree(sl.h_in);
        (void)hipHostFree(sl.h_out);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    if (sv->gstate) skim_greedy_state_free(sv->gstate);
    if (sv->gstream) (void)hipStreamDestroy(sv->gstream);
    delete sv;
}

extern "C" skim_status skim_server_submit(skim_server *sv, const uint32_t *nodes, uint32_t count,
                                          uint64_t *ticket) {
    skim::clear_error();
    if (!sv || !ticket || (count && !nodes)) {
        skim::set_error("NULL argument");
        return SKIM_EINVAL;
    }
    return submit_query(sv, nodes, count, ticket, Clock::now());
}

extern "C" skim_status skim_server_poll(skim_server *sv, uint64_t ticket, double *est,
                                        int32_t *status, double *latency_us) {
    if (!sv) return SKIM_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->done.find(ticket);
    if (it == sv->done.end()) {
        auto lv = sv->live.find(ticket);
        if (lv == sv->live.end() || lv->second != 1) {
            skim::set_error("unknown query ticket");
            return SKIM_EINVAL;
        }
        return SKIM_EBUSY;
    }
    if (est) *est = it->second.est;
    if (status) *status = it->second.status;
    if (latency_us) *latency_us = it->second.lat_us;
    sv->done.erase(it);
    sv->live.erase(ticket);
    return SKIM_OK;
}

extern "C" skim_status skim_server_cancel(skim_server *sv, uint64_t ticket) {
    skim::clear_error();
    if (!sv) {
        skim::set_error("NULL argument");
        return SKIM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    auto lv = sv->live.find(ticket);
    if (lv == sv->live.end() || lv->second != 1 || sv->done.count(ticket)) {
        skim::set_error("unknown or finished query ticket");
        return SKIM_EINVAL;
    }
    for (auto it = sv->pending.begin(); it != sv->pending.end(); ++it)
        if (it->ticket == ticket) {  // not in a batch yet: withdraw it
            const double lat =
                std::chrono::duration<double, std::micro>(Clock::now() - it->t0).count();
            sv->inflight_bytes -= it->bytes;
            sv->pending.erase(it);
            sv->done[ticket] = {0.0, kStatusCancelled, lat};
            return SKIM_OK;
        }
    sv->cancelled[ticket] = true;  // on the GPU: drop its result when the batch retires
    return SKIM_OK;
}

extern "C" skim_status skim_server_set_graph(skim_server *sv, const skim_graph *g, uint32_t ell,
                                             uint32_t k, uint64_t seed) {
    skim::clear_error();
    if (!sv || !g) {
        skim::set_error("NULL argument");
        return SKIM_EINVAL;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    if (sv->has_graph) {
        skim::set_error("the server already holds a SKIM graph");
        return SKIM_EINVAL;
    }
    sv->g = *g;
    sv->g_ell = ell;
    sv->g_k = k;
    sv->g_seed = seed;
    sv->has_graph = true;
    return SKIM_OK;
}

extern "C" skim_status skim_server_submit_greedy(skim_server *sv, uint32_t s, uint64_t *ticket) {
    skim::clear_error();
    if (!sv || !ticket) {
        skim::set_error("NULL argument");
        return SKIM_EINVAL;
    }
    const size_t b = greedy_bytes(s);
    if (b > sv->cfg.budget_bytes) {
        skim::set_error("SKIM request of %u seeds can never fit the budget", s);
        return SKIM_EUNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(sv->mu);
    if (!sv->has_graph) {
        skim::set_error("no SKIM graph: call skim_server_set_graph first");
        return SKIM_EINVAL;
    }
    if (sv->inflight_bytes + b > sv->cfg.budget_bytes) return SKIM_EBUSY;
    sv->inflight_bytes += b;
    GreedyReq r{sv->next_ticket++, s, Clock::now(), b};
    *ticket = r.ticket;
    sv->live[r.ticket] = 2;
    sv->gpending.push_back(r);
    sv->cv_g.notify_one();
    return SKIM_OK;
}

extern "C" skim_status skim_server_poll_greedy(skim_server *sv, uint64_t ticket, uint32_t *seeds,
                                               uint64_t *gain_pairs, double *latency_us) {
    if (!sv) return SKIM_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->gdone.find(ticket);
    if (it == sv->gdone.end()) {
        auto lv = sv->live.find(ticket);
        if (lv == sv->live.end() || lv->second != 2) {
            skim::set_error("unknown SKIM ticket");
            return SKIM_EINVAL;
        }
        return SKIM_EBUSY;
    }
    const GreedyDone &d = it->second;
    const skim_status st = d.status;
    if (st == SKIM_OK) {
        if (seeds && !d.seeds.empty()) std::memcpy(seeds, d.seeds.data(), d.seeds.size() * 4);
        if (gain_pairs && !d.gains.empty())
            std::memcpy(gain_pairs, d.gains.data(), d.gains.size() * 8);
    }
    if (latency_us) *latency_us = d.lat_us;
    sv->gdone.erase(it);
    sv->live.erase(ticket);
    return st;
}

extern "C" skim_status skim_server_replay(skim_server *sv, uint64_t q, const uint64_t *offsets,
                                          const uint32_t *nodes, const double *arrival_s,
                                          double *est, int32_t *status, double *latency_us,
                                          uint64_t *busy_retries) {
    skim::clear_error();
    if (!sv || (q && (!offsets || !arrival_s || !est))) {
        skim::set_error("NULL argument");
        return SKIM_EINVAL;
    }
    std::vector<uint64_t> tickets(q, 0);
    uint64_t retries = 0;
    const auto start = Clock::now();
    uint64_t next_poll = 0;
    auto poll_some = [&](bool block) {
        while (next_poll < q && tickets[next_poll]) {
            double e, l;
            int32_t st;
            const skim_status r = skim_server_poll(sv, tickets[next_poll], &e, &st, &l);
            if (r == SKIM_EBUSY) {
                if (!block) return;
                std::this_thread::yield();
                continue;
            }
            est[next_poll] = r == SKIM_OK ? e : 0.0;
            if (status) status[next_poll] = r == SKIM_OK ? st : -4;
            if (latency_us) latency_us[next_poll] = l;
            ++next_poll;
        }
    };
    for (uint64_t j = 0; j < q; ++j) {
        const auto t0 = start + std::chrono::duration_cast<Clock::duration>(
                                    std::chrono::duration<double>(arrival_s[j]));
        while (Clock::now() < t0) {
            poll_some(false);
            std::this_thread::yield();
        }
        const uint64_t a = offsets[j], b = offsets[j + 1];
        for (;;) {
            const skim_status r = submit_query(sv, nodes + a, (uint32_t)(b - a), &tickets[j], t0);
            if (r == SKIM_OK) break;
            if (r != SKIM_EBUSY) return r;
            ++retries;
            poll_some(false);
            std::this_thread::yield();
        }
    }
    poll_some(true);
    if (busy_retries) *busy_retries = retries;
    return SKIM_OK;
}
