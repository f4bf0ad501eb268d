// skim_live.hip -- live-edge lists of the l Monte-Carlo instances.
//
// Binary IC (Section 1; Section 2, eq. timedinf): instance G^(i) keeps edge
// (u -> v) iff its coin for instance i fires.  One coalesced pass over the
// edges evaluates all l coins of each edge (half a SplitMix64 output per
// instance) into a 64-bit instance mask.  Two builders group the live edges
// by pair p = 64 v + i:
//  * build_pair_lists (the sketch build): edges sorted by head, then one
//    wave per chunk of at most 1024 in-edges of a node writes the chunk's
//    part of the live lists of the node's 64 pairs (passes: count, room,
//    place); atomics only for the counts of nodes of several chunks.
//  * build_out_lists (SKIM's out-lists on large graphs, and levels taken by
//    pull): the same passes over the forward CSR's rows, which need no
//    sort, writing one CSR over pair ids.
//  * build_live_lists (SKIM on small graphs, where one pass serves both
//    directions): per-pair counts, a scan and a scatter into one CSR over
//    pair ids.
// Searches then read only the live edges of their own instance.
#include "skim_internal.h"

#include <rocprim/device/device_radix_sort.hpp>

namespace skim {

namespace {

// A wave whose 64 edges share one source (the out-edges of a hub: the
// forward CSR lists them consecutively) adds the forward counts of each
// instance once, from a ballot, instead of once per live edge: atomics from
// different waves on the hub's counters are serialised.
__device__ __forceinline__ bool wave_one_source(bool valid, uint32_t u, uint32_t &u0) {
    const unsigned long long act = __ballot(valid);
    if (!act) return false;
    const int leader = __ffsll((long long)act) - 1;
    u0 = (uint32_t)__shfl((int)u, leader);
    return __all(!valid || u == u0);
}

__global__ void k_live_masks(const uint32_t *esrc, const uint32_t *col, const uint32_t *thr,
                             uint64_t m, uint32_t n, uint32_t ell, uint64_t seed, uint64_t *masks,
                             uint32_t *rcnt, uint32_t *fcnt) {
    const uint32_t lane = lane_id();
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x; base < m;
         base += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = base + threadIdx.x;
        const bool valid = e < m;
        const uint32_t u = valid ? esrc[e] : 0u, v = valid ? col[e] : 0u;
        uint64_t mask = valid ? live_mask(seed, n, u, v, thr[e], ell) : 0ull;
        if (valid) masks[e] = mask;
        uint32_t u0 = 0;
        const bool one = fcnt && wave_one_source(valid, u, u0);
        if (one) {
            for (uint32_t i = 0; i < ell; ++i) {
                const unsigned long long b = __ballot((mask >> i) & 1ull);
                if (lane == i && b) atomicAdd(fcnt + (uint64_t)u0 * kPairStride + i,
                                              (uint32_t)__popcll(b));
            }
        }
        uint32_t *rrow = rcnt ? rcnt + (uint64_t)v * kPairStride : nullptr;
        uint32_t *frow = fcnt && !one ? fcnt + (uint64_t)u * kPairStride : nullptr;
        while (mask) {
            const int i = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            if (rrow) atomicAdd(rrow + i, 1u);
            if (frow) atomicAdd(frow + i, 1u);
        }
    }
}

// Scatter: reverse lists hold sources (in-edges of v), forward lists heads.
// Lists fill from their end (each entry takes the place its atomic returns);
// a one-source wave reserves each instance's entries with one atomic.
__global__ void k_live_fill(const uint32_t *esrc, const uint32_t *col, const uint64_t *masks,
                            uint64_t m, uint32_t ell, const uint64_t *rptr, uint32_t *rcnt,
                            uint32_t *radj, const uint64_t *fptr, uint32_t *fcnt, uint32_t *fadj) {
    const uint32_t lane = lane_id();
    for (uint64_t base = blockIdx.x * (uint64_t)blockDim.x; base < m;
         base += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t e = base + threadIdx.x;
        const bool valid = e < m;
        uint64_t mask = valid ? masks[e] : 0ull;
        const uint32_t u = valid ? esrc[e] : 0u, v = valid ? col[e] : 0u;
        uint32_t u0 = 0;
        const bool one = fadj && wave_one_source(valid, u, u0);
        if (one) {
            for (uint32_t i = 0; i < ell; ++i) {
                const unsigned long long b = __ballot((mask >> i) & 1ull);
                if (!b) continue;  // uniform
                const int leader = __ffsll((long long)b) - 1;
                const uint64_t p = (uint64_t)u0 * kPairStride + i;
                const uint32_t c = (uint32_t)__popcll(b);
                uint32_t old = 0;
                if ((int)lane == leader) old = atomicSub(fcnt + p, c);
                old = (uint32_t)__shfl((int)old, leader);
                if ((mask >> i) & 1ull)
                    fadj[fptr[p] + old - c + (uint32_t)__popcll(b & ((1ull << lane) - 1ull))] = v;
            }
        }
        while (mask) {
            const int i = __ffsll((long long)mask) - 1;
            mask &= mask - 1;
            if (radj) {
                const uint64_t p = (uint64_t)v * kPairStride + i;
                const uint32_t c = atomicSub(rcnt + p, 1u);
                radj[rptr[p] + c - 1] = u;
            }
            if (fadj && !one) {
                const uint64_t p = (uint64_t)u * kPairStride + i;
                const uint32_t c = atomicSub(fcnt + p, 1u);
                fadj[fptr[p] + c - 1] = v;
            }
        }
    }
}

// Pair lists without atomics per entry, grouped by node.  Edges are keyed
// (head << 32 | source) with their coin masks as values and radix-sorted on
// the head bits: the in-edges of every node become one run, in source order
// (the sort is stable and the forward CSR lists sources in order).  Each run
// is cut into chunks of at most kChunkEdges in-edges (a node without
// in-edges gets one empty chunk), and one wave per chunk turns its edges
// into the live lists of the node's 64 pairs, lane i taking instance i (the
// lanes' bits of 64 masks at a time are gathered by ballots):
//  1. count: per chunk and instance; the node's totals (atomics only for
//     nodes of several chunks, the in-degree hubs);
//  2. room: per node, the source-array room of its lists of two or more,
//     then a scan over the nodes;
//  3. chunk offsets: for nodes of several chunks, each chunk's place inside
//     each list (a prefix over the node's chunks);
//  4. write: the sources at their places and every pair's word, written
//     once (by the node's first chunk, or for a list of one by the chunk that
//     holds its source, the source itself being the word).
// Cutting hubs into chunks keeps every wave's work short: one wave per whole
// node left a 180,000-in-edge hub to a single wave.
constexpr uint32_t kChunkEdges = 1024;

// Key (run node << 32 | list entry): (head << 32 | source) for in-lists, or
// (source << 32 | head) for out-lists, which are already in run order.
__global__ void k_edge_keys(const uint32_t *esrc, const uint32_t *col, const uint32_t *thr,
                            uint64_t m, uint32_t n, uint32_t ell, uint64_t seed, bool forward,
                            uint64_t *key, uint64_t *mask) {
    for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < m;
         e += (uint64_t)gridDim.x * blockDim.x) {
        const uint32_t u = esrc[e], v = col[e];
        key[e] = forward ? (((uint64_t)u << 32) | v) : (((uint64_t)v << 32) | u);
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

__global__ void k_chunks_per_node(const uint64_t *beg, const uint64_t *end, uint32_t n,
                                  uint32_t *nch) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * blockDim.x) {
        const uint64_t d = end[v] - beg[v];
        nch[v] = d ? (uint32_t)((d + kChunkEdges - 1) / kChunkEdges) : 1u;
    }
}

__global__ void k_chunk_nodes(const uint64_t *choff, uint32_t n, uint32_t *chnode) {
    for (uint64_t v = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; v < n;
         v += (uint64_t)gridDim.x * blockDim.x)
        for (uint64_t c = choff[v]; c < choff[v + 1]; ++c) chnode[c] = (uint32_t)v;
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

struct ChunkArgs {
    const uint64_t *key, *mask, *beg, *end, *choff;
    const uint32_t *chnode;
    uint64_t nchunks;
    uint32_t ell;
};

// Edges [j0, j1) of chunk c of node v.
__device__ __forceinline__ void chunk_range(const ChunkArgs &C, uint64_t c, uint32_t &v,
                                            uint64_t &j0, uint64_t &j1, bool &multi) {
    v = C.chnode[c];
    const uint64_t first = C.choff[v];
    multi = C.choff[v + 1] - first > 1;
    j0 = C.beg[v] + (c - first) * kChunkEdges;
    const uint64_t e = C.end[v];
    j1 = j0 + kChunkEdges < e ? j0 + kChunkEdges : e;
    if (j0 > j1) j0 = j1;  // a node without in-edges: one empty chunk
}

// 1. count
__global__ void __launch_bounds__(256) k_pair_count(ChunkArgs C, uint32_t *ccnt, uint32_t *pcnt) {
    const uint32_t lane = lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    for (uint64_t c = blockIdx.x * (uint64_t)(blockDim.x / 64) + threadIdx.x / 64; c < C.nchunks;
         c += waves) {
        uint32_t v;
        uint64_t j0, j1;
        bool multi;
        chunk_range(C, c, v, j0, j1, multi);
        uint32_t cnt = 0;
        for (uint64_t j = j0; j < j1; j += 64) {
            const uint64_t mk = j + lane < j1 ? C.mask[j + lane] : 0;
            cnt += (uint32_t)__popcll(column_bits(mk, C.ell, lane));
        }
        ccnt[c * kPairStride + lane] = cnt;
        if (!multi) pcnt[(uint64_t)v * kPairStride + lane] = cnt;
        else if (cnt) atomicAdd(pcnt + (uint64_t)v * kPairStride + lane, cnt);
    }
}

// 2. room per node (lists of two or more; every list for a CSR), a flag for
// a list too long for the pair word's count field (flags[0]) and the longest
// list (flags[1])
__global__ void k_pair_room(const uint32_t *pcnt, uint32_t n, bool csr, uint32_t *room,
                            uint32_t *flags) {
    const uint32_t lane = lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    for (uint64_t v = blockIdx.x * (uint64_t)(blockDim.x / 64) + threadIdx.x / 64; v < n;
         v += waves) {
        const uint32_t c = pcnt[v * kPairStride + lane];
        if (!csr && (c >> kLiveCountBits)) atomicOr(flags, 1u);
        uint32_t r = c >= 2 || csr ? c : 0, mx = c;
        for (int off = 32; off > 0; off >>= 1) {
            r += __shfl_xor(r, off);
            const uint32_t o = (uint32_t)__shfl_xor((int)mx, off);
            mx = o > mx ? o : mx;
        }
        if (lane == 0) room[v] = r;
        if (lane == 0 && mx > 16) atomicMax(flags + 1, mx);  // short lists need no report
    }
}

// 3. for nodes of several chunks: ccnt becomes each chunk's exclusive prefix
// within each of the node's lists
__global__ void k_chunk_prefix(const uint64_t *choff, uint32_t n, uint32_t *ccnt) {
    const uint32_t lane = lane_id();
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    for (uint64_t v = blockIdx.x * (uint64_t)(blockDim.x / 64) + threadIdx.x / 64; v < n;
         v += waves) {
        const uint64_t c0 = choff[v], c1 = choff[v + 1];
        if (c1 - c0 < 2) continue;
        uint32_t run = 0;
        for (uint64_t c = c0; c < c1; ++c) {
            const uint32_t x = ccnt[c * kPairStride + lane];
            ccnt[c * kPairStride + lane] = run;
            run += x;
        }
    }
}

// 4. write (csr: every entry goes to adj and the node's first chunk writes
// each pair's start into live, which is then the CSR's offset array)
__global__ void __launch_bounds__(256) k_pair_emit(ChunkArgs C, const uint32_t *ccnt,
                                                   const uint32_t *pcnt, const uint64_t *node_off,
                                                   bool csr, uint64_t *live, uint32_t *adj) {
    __shared__ uint32_t src[256];
    const uint32_t lane = lane_id(), wbase = threadIdx.x & ~63u;
    const uint64_t waves = (uint64_t)gridDim.x * (blockDim.x / 64);
    for (uint64_t c = blockIdx.x * (uint64_t)(blockDim.x / 64) + threadIdx.x / 64; c < C.nchunks;
         c += waves) {
        uint32_t v;
        uint64_t j0, j1;
        bool multi;
        chunk_range(C, c, v, j0, j1, multi);
        const uint64_t cnt = pcnt[(uint64_t)v * kPairStride + lane];
        const uint64_t mine = cnt >= 2 || csr ? cnt : 0;
        uint64_t incl = mine;  // inclusive scan of the list lengths over the lanes
        for (int off = 1; off < 64; off <<= 1) {
            const uint64_t x = __shfl_up(incl, off);
            if ((int)lane >= off) incl += x;
        }
        const uint64_t first = node_off[v] + incl - mine;  // the list's start
        uint64_t at = first + (multi ? ccnt[c * kPairStride + lane] : 0);
        bool have_single = false;
        uint32_t single = 0;
        for (uint64_t j = j0; j < j1; j += 64) {
            const bool in = j + lane < j1;
            const uint64_t mk = in ? C.mask[j + lane] : 0;
            src[wbase + lane] = in ? (uint32_t)C.key[j + lane] : 0;
            uint64_t bits = column_bits(mk, C.ell, lane);
            // the lanes' sources are read by other lanes of the same wave
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
            while (bits) {
                const int b = __ffsll((long long)bits) - 1;
                bits &= bits - 1;
                const uint32_t u = src[wbase + b];
                if (cnt >= 2 || csr) {
                    adj[at++] = u;
                } else {
                    single = u;
                    have_single = true;
                }
            }
            __builtin_amdgcn_wave_barrier();
        }
        const bool head = c == C.choff[v];  // the node's first chunk
        if (csr) {
            if (head) live[(uint64_t)v * kPairStride + lane] = first;
        } else if (cnt == 1 ? have_single : head)
            live[(uint64_t)v * kPairStride + lane] =
                cnt == 0 ? 0ull : cnt == 1 ? (kLiveOne | single) : ((first << kLiveCountBits) | cnt);
    }
}

}  // namespace

namespace {
// The chunked builder: in-lists as pair words (csr false, live = [64 n]
// words), or out-lists as a CSR over pair ids (csr true, live = [64 n + 1]
// offsets).
struct ChunkedLists {
    uint64_t *live = nullptr;
    uint32_t *adj = nullptr;
    uint64_t nlive = 0;
    uint32_t maxlen = 0;
};

ChunkedLists chunked_lists(const skim_graph *g, uint32_t ell, uint64_t seed, const uint32_t *esrc,
                           bool csr, Arena &a, Arena &o) {
    hipStream_t s = a.stream();
    const uint32_t n = g->n;
    const uint64_t m = g->m;
    const uint64_t npairs = (uint64_t)n * kPairStride;
    ChunkedLists L;
    L.live = o.alloc<uint64_t>(csr ? npairs + 1 : npairs);
    if (!m) {
        fill_u64(L.live, 0, csr ? npairs + 1 : npairs, s);
        L.adj = o.alloc<uint32_t>(1);
        return L;
    }
    // coin masks of every edge, keyed by (run node, entry)
    uint64_t *key = a.alloc<uint64_t>(m), *mask = a.alloc<uint64_t>(m);
    {
        LaunchTimer t("k_edge_keys", s);
        k_edge_keys<<<grid_for(m, 256, 32768), 256, 0, s>>>(esrc, g->col, g->thr, m, n, ell, seed,
                                                            csr, key, mask);
    }
    SKIM_LAUNCH_CHECK();
    uint64_t *skey = key, *smask = mask;
    if (!csr) {  // in-lists: runs by head (out-lists are in source order already)
        int head_bits = 1;
        while (head_bits < 32 && (1ull << head_bits) < n) ++head_bits;
        skey = a.alloc<uint64_t>(m);
        smask = a.alloc<uint64_t>(m);
        size_t tb = 0;
        SKIM_HIP(rocprim::radix_sort_pairs(nullptr, tb, key, skey, mask, smask, (size_t)m, 32,
                                           32 + head_bits, s));
        void *tmp = a.get(tb ? tb : 1);
        SKIM_HIP(rocprim::radix_sort_pairs(tmp, tb, key, skey, mask, smask, (size_t)m, 32,
                                           32 + head_bits, s));
        a.release(tmp);
        a.release(key);
        a.release(mask);
    }
    // runs and their chunks
    uint64_t *beg = a.alloc<uint64_t>(n), *end = a.alloc<uint64_t>(n);
    fill_u64(beg, 0, n, s);
    fill_u64(end, 0, n, s);
    k_in_runs<<<grid_for(m, 256, 65536), 256, 0, s>>>(skey, m, beg, end);
    SKIM_LAUNCH_CHECK();
    uint32_t *nch = a.alloc<uint32_t>(n);
    k_chunks_per_node<<<grid_for(n, 256, 65536), 256, 0, s>>>(beg, end, n, nch);
    SKIM_LAUNCH_CHECK();
    uint64_t *choff = a.alloc<uint64_t>((uint64_t)n + 1);
    exclusive_scan_u32(nch, choff, n, a);
    a.release(nch);
    uint64_t nchunks = 0;
    read_back(&nchunks, choff + n, sizeof nchunks, s);
    uint32_t *chnode = a.alloc<uint32_t>(nchunks);
    k_chunk_nodes<<<grid_for(n, 256, 65536), 256, 0, s>>>(choff, n, chnode);
    SKIM_LAUNCH_CHECK();
    const ChunkArgs C{skey, smask, beg, end, choff, chnode, nchunks, ell};
    // 1. counts per chunk and per pair
    uint32_t *ccnt = a.alloc<uint32_t>(nchunks * kPairStride);
    uint32_t *pcnt = a.alloc<uint32_t>(npairs);
    fill_u32(pcnt, 0, npairs, s);
    const unsigned cgrid = grid_for(nchunks, 4, 65536);  // four waves (chunks) per block
    {
        LaunchTimer t("k_pair_count", s);
        k_pair_count<<<cgrid, 256, 0, s>>>(C, ccnt, pcnt);
    }
    SKIM_LAUNCH_CHECK();
    // 2. room per node, scan over the nodes
    uint32_t *room = a.alloc<uint32_t>(n);
    uint32_t *flags = a.alloc<uint32_t>(2);
    fill_u32(flags, 0, 2, s);
    k_pair_room<<<grid_for(n, 4, 65536), 256, 0, s>>>(pcnt, n, csr, room, flags);
    SKIM_LAUNCH_CHECK();
    uint64_t *node_off = a.alloc<uint64_t>((uint64_t)n + 1);
    exclusive_scan_u32(room, node_off, n, a);
    a.release(room);
    // 3. chunk places within the hubs' lists
    k_chunk_prefix<<<grid_for(n, 4, 65536), 256, 0, s>>>(choff, n, ccnt);
    SKIM_LAUNCH_CHECK();
    uint64_t tot = 0;
    uint32_t fl[2] = {0, 0};
    read_back(&tot, node_off + n, sizeof tot, s);
    read_back(fl, flags, sizeof fl, s);
    L.maxlen = fl[1];
    if (fl[0]) {
        set_error("a pair has 2^%u or more live in-edges", kLiveCountBits);
        throw Fail{SKIM_EUNSUPPORTED};
    }
    L.nlive = tot;
    L.adj = o.alloc<uint32_t>(tot ? tot : 1);
    // 4. entries and pair words (or offsets)
    {
        LaunchTimer t("k_pair_emit", s);
        k_pair_emit<<<cgrid, 256, 0, s>>>(C, ccnt, pcnt, node_off, csr, L.live, L.adj);
    }
    SKIM_LAUNCH_CHECK();
    if (csr) fill_u64(L.live + npairs, tot, 1, s);
    for (void *p : {(void *)node_off, (void *)beg, (void *)end, (void *)skey, (void *)smask,
                    (void *)choff, (void *)chnode, (void *)ccnt, (void *)pcnt})
        a.release(p);
    return L;
}
}  // namespace

PairLists build_pair_lists(const skim_graph *g, uint32_t ell, uint64_t seed, const uint32_t *esrc,
                           Arena &a, Arena *out) {
    const ChunkedLists c = chunked_lists(g, ell, seed, esrc, /*csr=*/false, a, out ? *out : a);
    PairLists L;
    L.live = c.live;
    L.adj = c.adj;
    L.nlive = c.nlive;
    L.maxlen = c.maxlen;
    return L;
}

LiveLists build_out_lists(const skim_graph *g, uint32_t ell, uint64_t seed, const uint32_t *esrc,
                          Arena &a, Arena *out) {
    const ChunkedLists c = chunked_lists(g, ell, seed, esrc, /*csr=*/true, a, out ? *out : a);
    LiveLists L;
    L.ptr = c.live;
    L.adj = c.adj;
    L.nlive = c.nlive;
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
        k_live_fill<<<grid, 256, 0, s>>>(esrc, g->col, masks, m, ell, rev.ptr, rcnt, rev.adj,
                                         fwd.ptr, fcnt, fwd.adj);
        SKIM_LAUNCH_CHECK();
        a.release(masks);
    }
    if (rcnt) a.release(rcnt);
    if (fcnt) a.release(fcnt);
    if (also_other) *also_other = forward ? rev : fwd;
    return forward ? fwd : rev;
}

}  // namespace skim
