// skim_live.hip -- live-edge lists of the l Monte-Carlo instances.
//
// Binary IC (Section 1; Section 2, eq. timedinf): instance G^(i) keeps edge
// (u -> v) iff its coin for instance i fires.  One coalesced pass over the
// edges evaluates all l coins of each edge (half a SplitMix64 output per
// instance) into a 64-bit instance mask.  Two builders group the live edges
// by pair p = 64 v + i:
//  * build_pair_lists (the sketch build): each edge writes its live (pair,
//    source) entries at its prefix offset, a radix sort groups them by pair
//    and each pair's run is located; no atomics.
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

// Pair lists without atomics: each edge's live (pair, source) entries are
// written at its prefix offset, sorted by pair (a stable radix sort keeps
// the sources of a pair in edge order), and every pair's run is located.
__global__ void k_live_pc(const uint32_t *esrc, const uint32_t *col, const uint32_t *thr,
                          uint64_t m, uint32_t n, uint32_t ell, uint64_t seed, uint64_t *masks,
                          uint32_t *pc) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t mask = live_mask(seed, n, esrc[e], col[e], thr[e], ell);
        masks[e] = mask;
        pc[e] = (uint32_t)__popcll(mask);
    }
}

__global__ void k_live_emit(const uint32_t *esrc, const uint32_t *col, const uint64_t *masks,
                            const uint64_t *off, uint64_t m, uint64_t *ent) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        uint64_t mask = masks[e];
        if (!mask) continue;
        const uint64_t u = esrc[e], p0 = (uint64_t)col[e] * kPairStride;
        uint64_t o = off[e];
        while (mask) {
            const int i = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            ent[o++] = ((p0 + (uint64_t)i) << 32) | u;
        }
    }
}

// Runs of the sorted entries: the first entry of a pair's run leaves its
// index in live[p], the last one turns it into the pair's live-list word.
__global__ void k_live_run_starts(const uint64_t *ent, uint64_t nlive, uint64_t *live,
                                  uint32_t *adj) {
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < nlive;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t x = ent[t];
        const uint32_t p = (uint32_t)(x >> 32);
        adj[t] = (uint32_t)x;
        if (t == 0 || (uint32_t)(ent[t - 1] >> 32) != p) live[p] = t;
    }
}

__global__ void k_live_run_ends(const uint64_t *ent, uint64_t nlive, uint64_t *live,
                                uint32_t *too_long) {
    for (uint64_t t = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; t < nlive;
         t += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t p = (uint32_t)(ent[t] >> 32);
        if (t + 1 < nlive && (uint32_t)(ent[t + 1] >> 32) == p) continue;
        const uint64_t b = live[p], c = t + 1 - b;
        if (c >> kLiveCountBits) atomicOr(too_long, 1u);
        live[p] = c == 1 ? kLiveOne | (uint32_t)ent[t] : (b << kLiveCountBits) | c;
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
    fill_u64(L.live, 0, npairs, s);
    if (!m) {
        L.adj = a.alloc<uint32_t>(1);
        return L;
    }
    const unsigned grid = grid_for(m, 256, 32768);
    uint64_t *masks = a.alloc<uint64_t>(m);
    uint32_t *pc = a.alloc<uint32_t>(m);
    {
        LaunchTimer t("k_live_pc", s);
        k_live_pc<<<grid, 256, 0, s>>>(esrc, g->col, g->thr, m, n, ell, seed, masks, pc);
    }
    SKIM_LAUNCH_CHECK();
    uint64_t *off = a.alloc<uint64_t>(m + 1);
    exclusive_scan_u32(pc, off, m, a);
    a.release(pc);
    uint64_t tot = 0;
    read_back(&tot, off + m, sizeof tot, s);
    L.nlive = tot;
    L.adj = a.alloc<uint32_t>(tot ? tot : 1);
    if (!tot) {
        a.release(masks);
        a.release(off);
        return L;
    }
    uint64_t *ent = a.alloc<uint64_t>(tot);
    k_live_emit<<<grid, 256, 0, s>>>(esrc, g->col, masks, off, m, ent);
    SKIM_LAUNCH_CHECK();
    a.release(masks);
    a.release(off);
    int pair_bits = 1;
    while (pair_bits < 32 && (1ull << pair_bits) < npairs) ++pair_bits;
    uint64_t *sorted = a.alloc<uint64_t>(tot);
    size_t tb = 0;
    SKIM_HIP(rocprim::radix_sort_keys(nullptr, tb, ent, sorted, (size_t)tot, 32, 32 + pair_bits, s));
    void *tmp = a.get(tb ? tb : 1);
    SKIM_HIP(rocprim::radix_sort_keys(tmp, tb, ent, sorted, (size_t)tot, 32, 32 + pair_bits, s));
    a.release(tmp);
    a.release(ent);
    uint32_t *too_long = a.alloc<uint32_t>(1);
    fill_u32(too_long, 0, 1, s);
    k_live_run_starts<<<grid_for(tot, 256, 65536), 256, 0, s>>>(sorted, tot, L.live, L.adj);
    SKIM_LAUNCH_CHECK();
    k_live_run_ends<<<grid_for(tot, 256, 65536), 256, 0, s>>>(sorted, tot, L.live, too_long);
    SKIM_LAUNCH_CHECK();
    a.release(sorted);
    uint32_t bad = 0;
    read_back(&bad, too_long, sizeof bad, s);
    if (bad) {
        set_error("a pair has 2^%u or more live in-edges", kLiveCountBits);
        throw Fail{SKIM_EUNSUPPORTED};
    }
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
