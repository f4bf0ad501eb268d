// skim_tune_cache.hip -- a persistent cache of the build autotuner's
// choices, keyed by the device and the configuration.
//
// The key is a 64-bit FNV-1a hash of: the number of fields of
// skim_build_params (so lines of an older field set never match); the
// device's architecture name and compute-unit count; n, m, l, k and the
// seed; and 64 evenly spaced samples each of row_ptr, col and thr, gathered
// on the device by one small kernel.  The cache is a text file with one line
// per key:
//   <key hex> <small_frontier> <small_batch> <large_batch> <thread_frontier>
//   <heavy_visits> <sort_frontier> <window_span> <first_span> <pull_frontier>
//   <best_ms>
// A hit applies the stored launch shapes (skim_set_build_params) without
// timing anything; a miss runs skim_tune_build and appends its choice.
// Lines that do not parse, or whose shapes the library refuses, are skipped.
#include "skim_internal.h"

#include <cstring>
#include <fstream>
#include <mutex>
#include <sstream>
#include <string>

namespace skim {

namespace {

constexpr uint32_t kTuneSamples = 64;

__global__ void k_tune_sample(const uint64_t *row_ptr, const uint32_t *col, const uint32_t *thr,
                              uint32_t n, uint64_t m, uint64_t *out) {
    const uint32_t j = threadIdx.x;
    if (j >= kTuneSamples) return;
    out[j] = row_ptr[(uint64_t)n * j / (kTuneSamples - 1)];
    const uint64_t e = m ? (m - 1) * j / (kTuneSamples - 1) : 0;
    out[kTuneSamples + j] = m ? col[e] : 0;
    out[2 * kTuneSamples + j] = m ? thr[e] : 0;
}

uint64_t fnv1a(uint64_t h, const void *p, size_t bytes) {
    const unsigned char *c = (const unsigned char *)p;
    for (size_t i = 0; i < bytes; ++i) {
        h ^= c[i];
        h *= 0x100000001B3ull;
    }
    return h;
}

std::mutex g_file_mu;

}  // namespace

}  // namespace skim

extern "C" skim_status skim_tune_build_cached(const skim_graph *g, uint32_t ell, uint32_t k,
                                              uint64_t seed, uint64_t *ranks, uint32_t *size,
                                              uint32_t reps, const char *cache_path,
                                              skim_build_params *best, double *best_ms,
                                              double *start_ms, uint32_t *hit, void *stream) {
    using namespace skim;
    clear_error();
    hipStream_t hs = (hipStream_t)stream;
    try {
        SKIM_REQUIRE(g != nullptr && g->row_ptr != nullptr, "graph is NULL");
        SKIM_REQUIRE(cache_path != nullptr && cache_path[0] != 0, "cache_path is empty");
        SKIM_REQUIRE(best != nullptr && hit != nullptr, "best/hit is NULL");
        SKIM_REQUIRE(g->n >= 1 && (g->m == 0 || (g->col && g->thr)), "graph arrays are NULL");
        int dev = 0;
        SKIM_HIP(hipGetDevice(&dev));
        hipDeviceProp_t prop;
        SKIM_HIP(hipGetDeviceProperties(&prop, dev));
        uint64_t h = 0xCBF29CE484222325ull;
        const uint32_t nfields = sizeof(skim_build_params) / sizeof(uint32_t);
        h = fnv1a(h, &nfields, sizeof nfields);
        h = fnv1a(h, prop.gcnArchName, strnlen(prop.gcnArchName, sizeof prop.gcnArchName));
        h = fnv1a(h, &prop.multiProcessorCount, sizeof prop.multiProcessorCount);
        const uint64_t cfg[5] = {g->n, g->m, ell, k, seed};
        h = fnv1a(h, cfg, sizeof cfg);
        {
            Arena T(hs);
            uint64_t *d = T.alloc<uint64_t>(3 * kTuneSamples);
            k_tune_sample<<<1, kTuneSamples, 0, hs>>>(g->row_ptr, g->col, g->thr, g->n, g->m, d);
            SKIM_LAUNCH_CHECK();
            uint64_t hsamp[3 * kTuneSamples];
            read_back(hsamp, d, sizeof hsamp, hs);
            h = fnv1a(h, hsamp, sizeof hsamp);
        }
        char key[17];
        snprintf(key, sizeof key, "%016llx", (unsigned long long)h);
        std::lock_guard<std::mutex> lock(g_file_mu);
        {
            std::ifstream in(cache_path);
            std::string line;
            while (in && std::getline(in, line)) {
                std::istringstream ls(line);
                std::string k2;
                skim_build_params p{};
                double ms = 0;
                if (!(ls >> k2 >> p.small_frontier >> p.small_batch >> p.large_batch >>
                      p.thread_frontier >> p.heavy_visits >> p.sort_frontier >> p.window_span >>
                      p.first_span >> p.pull_frontier >> ms))
                    continue;
                if (k2 != key) continue;
                if (skim_set_build_params(&p) != SKIM_OK) continue;  // refused: tune again
                *best = p;
                if (best_ms) *best_ms = ms;
                if (start_ms) *start_ms = 0.0;
                *hit = 1;
                return SKIM_OK;
            }
        }
        double bms = 0, sms = 0;
        const skim_status st = skim_tune_build(g, ell, k, seed, ranks, size, reps, best, &bms, &sms,
                                               stream);
        if (st != SKIM_OK) return st;
        std::ofstream out(cache_path, std::ios::app);
        if (!out) {
            set_error("cannot append to the tuning cache %s", cache_path);
            return SKIM_EINVAL;
        }
        out << key << ' ' << best->small_frontier << ' ' << best->small_batch << ' '
            << best->large_batch << ' ' << best->thread_frontier << ' ' << best->heavy_visits << ' '
            << best->sort_frontier << ' ' << best->window_span << ' ' << best->first_span << ' '
            << best->pull_frontier << ' ' << bms << '\n';
        if (best_ms) *best_ms = bms;
        if (start_ms) *start_ms = sms;
        *hit = 0;
        return SKIM_OK;
    } catch (const Fail &f) {
        return f.st;
    }
}
