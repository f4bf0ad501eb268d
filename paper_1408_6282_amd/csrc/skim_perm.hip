// skim_perm.hip -- structured permutation ranks for finite l (Section 3.1).
//
// The n l node-instance pairs get positions 1 .. n l in l chunks of n
// positions.  Chunk c holds every node exactly once, ordered by the hash
// h_c(v) = SM(seed, 2^63 + c n + v) (the chunk order of the IC-model
// sketches).  The instance a node takes in chunk c is drawn from those it
// has not taken in earlier chunks, which makes its instances a uniform
// permutation over the chunks: instance i goes to the chunk given by the
// place of g_v(i) = SM(seed, 2^61 + 64 v + i) among g_v(0 .. l-1).
//
//  1. one segmented radix sort orders every chunk by h_c (rocPRIM);
//  2. the place of every node in every chunk is scattered from the order;
//  3. one wave per node gives lane i instance i, ranks its key among the
//     lanes (the chunk), and writes the pair's position.
// The sketch build then uses these positions as its ranks (a table lookup
// instead of the hashed rank), the estimator 1 + (k-1)(n l - 1)/(T - 1)
// divided by l, and queries read T as r = (T - 1)/(l n - 1) for
// Cohen-Kaplan (Section 5.1, last paragraph).
#include "skim_internal.h"

#include <rocprim/device/device_segmented_radix_sort.hpp>

namespace skim {

namespace {

constexpr uint64_t kPermChunk = 1ull << 63;  // counters of the chunk hashes h_c(v)
constexpr uint64_t kPermInst = 1ull << 61;   // counters of the instance keys g_v(i)

__global__ void k_perm_hash(uint32_t n, uint32_t ell, uint64_t seed, uint64_t *keys,
                            uint32_t *vals, uint32_t *offs) {
    const uint64_t total = (uint64_t)n * ell;
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total;
         x += (uint64_t)gridDim.x * blockDim.x) {
        keys[x] = sm_at(seed, kPermChunk + x);  // x = c n + v
        vals[x] = (uint32_t)(x % n);
        if (x % n == 0) offs[x / n] = (uint32_t)x;
        if (x == 0) offs[ell] = (uint32_t)total;
    }
}

// place[c n + v] = j where node v is the j-th of chunk c
__global__ void k_perm_place(const uint32_t *node_at, uint32_t n, uint64_t total,
                             uint32_t *place) {
    for (uint64_t x = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; x < total;
         x += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t c = x / n;
        place[c * n + node_at[x]] = (uint32_t)(x - c * n);
    }
}

// One wave per node; lane i holds instance i.
__global__ void __launch_bounds__(256) k_perm_assign(uint32_t n, uint32_t ell, uint64_t seed,
                                                     const uint32_t *place, uint64_t *table) {
    const uint32_t lane = lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    for (uint64_t v = blockIdx.x * (uint64_t)(blockDim.x / 64) + threadIdx.x / 64; v < n;
         v += waves) {
        const uint64_t key = lane < ell ? sm_at(seed, kPermInst + v * kPairStride + lane) : ~0ull;
        uint32_t c = 0;  // keys of the other instances below this lane's
        for (uint32_t j = 0; j < ell; ++j) {
            const uint32_t lo = __shfl((uint32_t)key, (int)j), hi = __shfl((uint32_t)(key >> 32), (int)j);
            const uint64_t other = ((uint64_t)hi << 32) | lo;
            c += other < key;
        }
        table[v * kPairStride + lane] =
            lane < ell ? (uint64_t)c * n + place[(uint64_t)c * n + v] + 1 : kNone;
    }
}

}  // namespace

void perm_positions(uint32_t n, uint32_t ell, uint64_t seed, uint64_t *table, Arena &a) {
    hipStream_t s = a.stream();
    const uint64_t total = (uint64_t)n * ell;
    SKIM_REQUIRE(total < (1ull << 32), "n l must be below 2^32 for permutation positions");
    uint64_t *keys = a.alloc<uint64_t>(total), *keys2 = a.alloc<uint64_t>(total);
    uint32_t *vals = a.alloc<uint32_t>(total), *node_at = a.alloc<uint32_t>(total);
    uint32_t *offs = a.alloc<uint32_t>((uint64_t)ell + 1);
    k_perm_hash<<<grid_for(total, 256, 16384), 256, 0, s>>>(n, ell, seed, keys, vals, offs);
    SKIM_LAUNCH_CHECK();
    size_t tb = 0;
    SKIM_HIP(rocprim::segmented_radix_sort_pairs(nullptr, tb, keys, keys2, vals, node_at,
                                                 (unsigned)total, ell, offs, offs + 1, 0, 64, s));
    void *tmp = a.get(tb ? tb : 1);
    SKIM_HIP(rocprim::segmented_radix_sort_pairs(tmp, tb, keys, keys2, vals, node_at,
                                                 (unsigned)total, ell, offs, offs + 1, 0, 64, s));
    a.release(tmp);
    a.release(keys);
    a.release(keys2);
    a.release(vals);
    uint32_t *place = a.alloc<uint32_t>(total);
    k_perm_place<<<grid_for(total, 256, 16384), 256, 0, s>>>(node_at, n, total, place);
    SKIM_LAUNCH_CHECK();
    a.release(node_at);
    k_perm_assign<<<grid_for(n, 4, 65536), 256, 0, s>>>(n, ell, seed, place, table);
    SKIM_LAUNCH_CHECK();
    a.release(place);
    a.release(offs);
}

}  // namespace skim
