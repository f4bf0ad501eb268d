// skim_live.hip -- live-edge lists of the l Monte-Carlo instances.
//
// Binary IC (Section 1; Section 2, eq. timedinf): instance G^(i) keeps edge
// (u -> v) iff its coin for instance i fires.  One coalesced pass over the
// edges evaluates all l coins of each edge (half a SplitMix64 output per
// instance) into a 64-bit instance mask.  Two builders group the live edges
// by pair p = 64 v + i:
//  * build_pair_lists (the sketch build): edges sorted by head, then one
//    wave per node writes the live lists of its 64 pairs (two passes: count,
//    then place); no atomics.
//  * build_live_lists (SKIM, which also needs out-lists): per-pair counts,
//    a scan and a scatter into one CSR over pair ids.
// Searches then read only the live edges of their own instance.
#include "skim_internal.h"

#include <rocprim/device/device_radix_sort.hpp>

namespace skim {

namespace {

__global__ void k_live_masks(const uint32_t *esrc, const uint32_t *col, const uint32_t *thr,
                             uint64_t m, uint32_t n, uint32_t ell, uint64_t seed, uint64_t *masks,
                             uint32_t *rcnt, uint32_t *fcnt) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t u = esrc[e], v = col[e];
        uint64_t mask = live_mask(seed, n, u, v, thr[e], ell);
        masks[e] = mask;
        uint32_t *rrow = rcnt ? rcnt + (uint64_t)v * kPairStride : nullptr;
        uint32_t *frow = fcnt ? fcnt + (uint64_t)u * kPairStride : nullptr;
        while (mask) {
            const int i = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            if (rrow) atomicAdd(rrow + i, 1u);
            if (frow) atomicAdd(frow + i, 1u);
        }
    }
}

// Scatter: reverse lists hold sources (in-edges of v), forward lists heads.
__global__ void k_live_fill(const uint32_t *esrc, const uint32_t *col, const uint64_t *masks,
                            uint64_t m, const uint64_t *rptr, uint32_t *rcnt, uint32_t *radj,
                            const uint64_t *fptr, uint32_t *fcnt, uint32_t *fadj) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t mask = masks[e];
        if (!mask) continue;
        const uint32_t u = esrc[e], v = col[e];
        while (mask) {
            const int i = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            if (radj) {
                const uint64_t p = (uint64_t)v * kPairStride + i;
                const uint32_t c = atomicSub(rcnt + p, 1u);
                radj[rptr[p] + c - 1] = u;
            }
            if (fadj) {
                const uint64_t p = (uint64_t)u * kPairStride + i;
                const uint32_t c = atomicSub(fcnt + p, 1u);
                fadj[fptr[p] + c - 1] = v;
            }
        }
    }
}

// Pair lists without atomics, grouped by node.  Edges are keyed
// (head << 32 | source) with their coin masks as values and radix-sorted on
// the head bits: the in-edges of every node become one run, in source order
// (the sort is stable and the forward CSR lists sources in order).  One wave
// per node then turns its run into the live lists of its 64 pairs, lane i
// taking instance i: a first pass counts each pair's live in-edges (the
// lanes' bits of 64 masks at a time are gathered by ballots), a scan over
// the nodes places every list, and a second pass writes the sources.  Lists
// of one source live in the pair's word itself, so only longer lists take
// room in the source array.
__global__ void k_edge_keys(const uint32_t *esrc, const uint32_t *col, const uint32_t *thr,
                            uint64_t m, uint32_t n, uint32_t ell, uint64_t seed, uint64_t *key,
                            uint64_t *mask) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t u = esrc[e], v = col[e];
        key[e] = ((uint64_t)v << 32) | u;
        mask[e] = live_mask(seed, n, u, v, thr[e], ell);
    }
}

// Run [beg[v], end[v]) of node v's in-edges in the sorted keys (both arrays
// zero for a node without in-edges).
__global__ void k_in_runs(const uint64_t *key, uint64_t m, uint64_t *beg, uint64_t *end) {
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < m;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t v = (uint32_t)(key[t] >> 32);
        if (t == 0 || (uint32_t)(key[t - 1] >> 32) != v) beg[v] = t;
        if (t + 1 == m || (uint32_t)(key[t + 1] >> 32) != v) end[v] = t + 1;
    }
}

// Bits of instance `lane` among the 64 masks held by the wave's lanes
// (lane j holds edge j of the chunk): bit j of the result is set when edge j
// is live in the lane's instance.
__device__ __forceinline__ uint64_t column_bits(uint64_t mask, uint32_t ell, uint32_t lane) {
    uint64_t mine = 0;
    for (uint32_t i = 0; i < ell; ++i) {
        const uint64_t b = __ballot((mask >> i) & 1ull);
        if (lane == i) mine = b;
    }
    return mine;
}

// Pass 1: live in-edges of every pair (kept in live[p] until pass 2) and,
// per node, the source-array room its lists of two or more take.
__global__ void __launch_bounds__(256) k_pair_count(const uint64_t *mask, const uint64_t *beg,
                                                    const uint64_t *end, uint32_t n, uint32_t ell,
                                                    uint64_t *live, uint32_t *room,
                                                    uint32_t *too_long) {
    const uint32_t lane = lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    for (uint64_t v = blockIdx.x * (uint64_t)(blockDim.x / 64) + threadIdx.x / 64; v < n;
         v += waves) {
        const uint64_t b = beg[v], e = end[v];
        uint64_t c = 0;
        for (uint64_t j0 = b; j0 < e; j0 += 64) {
            const uint64_t mk = j0 + lane < e ? mask[j0 + lane] : 0;
            c += (uint64_t)__popcll(column_bits(mk, ell, lane));
        }
        if (c >> kLiveCountBits) atomicOr(too_long, 1u);
        live[v * kPairStride + lane] = c;
        uint64_t r = c >= 2 ? c : 0;
        for (int off = 32; off > 0; off >>= 1) r += __shfl_xor(r, off);
        if (lane == 0) room[v] = (uint32_t)r;
    }
}

// Pass 2: sources of every list of two or more at its place (node base from
// the scan, then the lanes' lists in instance order); the pair's word.
__global__ void __launch_bounds__(256) k_pair_emit(const uint64_t *key, const uint64_t *mask,
                                                   const uint64_t *beg, const uint64_t *end,
                                                   const uint64_t *node_off, uint32_t n,
                                                   uint32_t ell, uint64_t *live, uint32_t *adj) {
    __shared__ uint32_t src[256];
    const uint32_t lane = lane_id(), wbase = threadIdx.x & ~63u;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    for (uint64_t v = blockIdx.x * (uint64_t)(blockDim.x / 64) + threadIdx.x / 64; v < n;
         v += waves) {
        const uint64_t b = beg[v], e = end[v];
        const uint64_t c = live[v * kPairStride + lane];
        const uint64_t mine = c >= 2 ? c : 0;
        uint64_t incl = mine;  // inclusive scan of the list lengths over the lanes
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t x = __shfl_up(incl, off);
            if ((int)lane >= off) incl += x;
        }
        uint64_t at = node_off[v] + incl - mine;
        const uint64_t first = at;
        uint32_t single = 0;
        for (uint64_t j0 = b; j0 < e; j0 += 64) {
            const bool in = j0 + lane < e;
            const uint64_t mk = in ? mask[j0 + lane] : 0;
            src[wbase + lane] = in ? (uint32_t)key[j0 + lane] : 0;
            uint64_t bits = column_bits(mk, ell, lane);
            // the lanes' sources are read by other lanes of the same wave
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            while (bits) {
                const int j = __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                const uint32_t u = src[wbase + j];
                if (c >= 2) adj[at++] = u;
                else single = u;
            }
            __builtin_amdgcn_wave_barrier();
        }
        live[v * kPairStride + lane] =
            c == 0 ? 0ull : c == 1 ? (kLiveOne | single) : ((first << kLiveCountBits) | c);
    }
}

}  // namespace

PairLists build_pair_lists(const skim_graph *g, uint32_t ell, uint64_t seed, const uint32_t *esrc,
                           Arena &a) {
    hipStream_t s = a.stream();
    const uint32_t n = g->n;
    const uint64_t m = g->m;
    const uint64_t npairs = (uint64_t)n * kPairStride;
    PairLists L;
    L.live = a.alloc<uint64_t>(npairs);
    if (!m) {
        fill_u64(L.live, 0, npairs, s);
        L.adj = a.alloc<uint32_t>(1);
        return L;
    }
    // coin masks of every edge, keyed by (head, source)
    uint64_t *key = a.alloc<uint64_t>(m), *mask = a.alloc<uint64_t>(m);
    {
        LaunchTimer t("k_edge_keys", s);
        k_edge_keys<<<grid_for(m, 256, 32768), 256, 0, s>>>(esrc, g->col, g->thr, m, n, ell, seed,
                                                            key, mask);
    }
    SKIM_LAUNCH_CHECK();
    int head_bits = 1;
    while (head_bits < 32 && (1ull << head_bits) < n) ++head_bits;
    uint64_t *skey = a.alloc<uint64_t>(m), *smask = a.alloc<uint64_t>(m);
    size_t tb = 0;
    SKIM_HIP(rocprim::radix_sort_pairs(nullptr, tb, key, skey, mask, smask, (size_t)m, 32,
                                       32 + head_bits, s));
    void *tmp = a.get(tb ? tb : 1);
    SKIM_HIP(rocprim::radix_sort_pairs(tmp, tb, key, skey, mask, smask, (size_t)m, 32,
                                       32 + head_bits, s));
    a.release(tmp);
    a.release(key);
    a.release(mask);
    // in-edge runs per node
    uint64_t *beg = a.alloc<uint64_t>(n), *end = a.alloc<uint64_t>(n);
    fill_u64(beg, 0, n, s);
    fill_u64(end, 0, n, s);
    k_in_runs<<<grid_for(m, 256, 65536), 256, 0, s>>>(skey, m, beg, end);
    SKIM_LAUNCH_CHECK();
    // pass 1: counts; the room of every node's lists; scan over the nodes
    uint32_t *room = a.alloc<uint32_t>(n);
    uint32_t *too_long = a.alloc<uint32_t>(1);
    fill_u32(too_long, 0, 1, s);
    const unsigned wgrid = grid_for(n, 4, 65536);  // four waves (nodes) per block
    {
        LaunchTimer t("k_pair_count", s);
        k_pair_count<<<wgrid, 256, 0, s>>>(smask, beg, end, n, ell, L.live, room, too_long);
    }
    SKIM_LAUNCH_CHECK();
    uint64_t *node_off = a.alloc<uint64_t>((uint64_t)n + 1);
    exclusive_scan_u32(room, node_off, n, a);
    a.release(room);
    uint64_t tot = 0;
    uint32_t bad = 0;
    read_back(&tot, node_off + n, sizeof tot, s);
    read_back(&bad, too_long, sizeof bad, s);
    if (bad) {
        set_error("a pair has 2^%u or more live in-edges", kLiveCountBits);
        throw Fail{SKIM_EUNSUPPORTED};
    }
    L.nlive = tot;
    L.adj = a.alloc<uint32_t>(tot ? tot : 1);
    {
        LaunchTimer t("k_pair_emit", s);
        k_pair_emit<<<wgrid, 256, 0, s>>>(skey, smask, beg, end, node_off, n, ell, L.live, L.adj);
    }
    SKIM_LAUNCH_CHECK();
    a.release(node_off);
    a.release(beg);
    a.release(end);
    a.release(skey);
    a.release(smask);
    return L;
}

LiveLists build_live_lists(const skim_graph *g, uint32_t ell, uint64_t seed, const uint32_t *esrc,
                           bool forward, Arena &a, LiveLists *also_other) {
    hipStream_t s = a.stream();
    const uint32_t n = g->n;
    const uint64_t m = g->m;
    const uint64_t npairs = (uint64_t)n * kPairStride;
    // `forward` selects the list returned; `also_other` (optional) receives
    // the opposite direction from the same coin pass.
    const bool want_rev = !forward || also_other;
    const bool want_fwd = forward || also_other;
    uint32_t *rcnt = want_rev ? a.alloc<uint32_t>(npairs) : nullptr;
    uint32_t *fcnt = want_fwd ? a.alloc<uint32_t>(npairs) : nullptr;
    if (rcnt) fill_u32(rcnt, 0, npairs, s);
    if (fcnt) fill_u32(fcnt, 0, npairs, s);
    uint64_t *masks = nullptr;
    const unsigned grid = grid_for(m, 256, 32768);
    if (m) {
        masks = a.alloc<uint64_t>(m);
        LaunchTimer t("k_live_masks", s);
        k_live_masks<<<grid, 256, 0, s>>>(esrc, g->col, g->thr, m, n, ell, seed, masks, rcnt, fcnt);
        SKIM_LAUNCH_CHECK();
    }
    LiveLists rev, fwd;
    uint64_t tot = 0;
    if (want_rev) {
        rev.ptr = a.alloc<uint64_t>(npairs + 1);
        exclusive_scan_u32(rcnt, rev.ptr, npairs, a);
        read_back(&tot, rev.ptr + npairs, sizeof tot, s);
        rev.nlive = tot;
        rev.adj = a.alloc<uint32_t>(tot ? tot : 1);
    }
    if (want_fwd) {
        fwd.ptr = a.alloc<uint64_t>(npairs + 1);
        exclusive_scan_u32(fcnt, fwd.ptr, npairs, a);
        read_back(&tot, fwd.ptr + npairs, sizeof tot, s);
        fwd.nlive = tot;
        fwd.adj = a.alloc<uint32_t>(tot ? tot : 1);
    }
    if (m) {
        LaunchTimer t("k_live_fill", s);
        k_live_fill<<<grid, 256, 0, s>>>(esrc, g->col, masks, m, rev.ptr, rcnt, rev.adj, fwd.ptr,
                                         fcnt, fwd.adj);
        SKIM_LAUNCH_CHECK();
        a.release(masks);
    }
    if (rcnt) a.release(rcnt);
    if (fcnt) a.release(fcnt);
    if (also_other) *also_other = forward ? rev : fwd;
    return forward ? fwd : rev;
}

}  // namespace skim
