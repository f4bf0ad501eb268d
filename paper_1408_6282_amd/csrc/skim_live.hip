// skim_live.hip -- live-edge lists of the l Monte-Carlo instances.
//
// Binary IC (Section 1; Section 2, eq. timedinf): instance G^(i) keeps edge
// (u -> v) iff its coin for instance i fires.  One coalesced pass over the
// edges evaluates all l coins of each edge (half a SplitMix64 output per
// instance) into a 64-bit instance mask, counts the live edges of every
// pair p = 64 v + i, and a second pass scatters them into one CSR over pair
// ids.  Searches then read only the live edges of their own instance.
#include "skim_internal.h"

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

}  // namespace

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
