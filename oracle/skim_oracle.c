/*
 * skim_oracle.c -- plain, slow, obviously-correct CPU oracle for
 * sketch-based influence computation (Cohen, Delling, Pajor, Werneck,
 * "Sketch-based Influence Maximization and Computation", 2014).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the reference the HIP library is
 * checked against.  Only the test suite, the smoke check and the bench's CPU
 * baseline may load it.  It shares no code, header or table with the HIP
 * path; the two meet only by comparing outputs.
 *
 * Conventions fixed here (the paper leaves them open; both sides implement
 * them independently):
 *
 *  - Randomness is SplitMix64 (Steele, Lea, Flood, OOPSLA 2014): output c
 *    (c = 0, 1, ...) of the stream seeded with s is mix64(s + (c+1)*GAMMA),
 *    GAMMA = 0x9E3779B97F4A7C15, where mix64 is Stafford's "variant 13"
 *    finaliser (xor-shift 30, multiply, xor-shift 27, multiply, xor-shift 31).
 *  - Rank of node-instance pair (v, i): r(v,i) = SM(seed, 64*v + i), a uint64.
 *    mix64 is a bijection and GAMMA is odd, so all ranks are distinct; the
 *    paper's U[0,1] rank (Section 3) is the real reading of this integer.
 *  - Live edge (u -> v) in instance i (binary IC, Section 1 and 2):
 *    h = SM(seed, 2^62 + 32*(u*n + v) + floor(i/2)); the 32-bit coin is the
 *    high half of h for even i and the low half for odd i; the edge is live
 *    iff coin <= thr, so P[live] = (thr + 1) / 2^32.
 *  - Estimate from threshold rank T: rho(T) = ((T >> 11) + 1) * 2^-53.
 *
 * Functions and the passages they follow:
 *   or_sm64, or_rank, or_live ............. Section 3 (random ranks), Section 1
 *                                          (binary IC live edges)
 *   or_influence .......................... Section 2, eq. (Inf) and (timedinf)
 *   or_sketch_brute ....................... Section 3, eq. (combinedrs): the
 *                                          plain definition, by forward search
 *   or_build_alg2 ......................... Section 5.2, Algorithm 2
 *   or_estimates .......................... Section 3, eq. (combinedthresh) and
 *                                          the bottom-k estimator; Section 5.1
 *                                          (divide by l)
 *   or_union_query ........................ Section 5.1, bottom-k of the union
 *   or_ck_query ........................... Section 5.1, eq. (unionest)
 *   or_ic_live, or_ic_order, or_ic_sketches  Section 3, structured permutation
 *                                          ranks and sketches for an IC model
 *                                          (the l -> infinity limit)
 *   or_ic_union_query ..................... Section 3 and 5.1: bottom-k and
 *                                          Cohen-Kaplan unions of IC-model
 *                                          sketches (permutation ranks)
 *   or_perm_positions, or_build_alg2_table, or_sketch_brute_table,
 *   or_perm_estimates, or_perm_union_query  Section 3.1, structured
 *                                          permutation ranks for finite l:
 *                                          positions, sketches of positions
 *                                          (Algorithm 2 and the definition),
 *                                          the permutation estimator, and
 *                                          bottom-k and Cohen-Kaplan unions
 *                                          (Section 5.1, last paragraph)
 *   or_skim ............................... Section 4, Algorithm 1; per-seed
 *                                          records for the adaptive error
 *                                          estimate (Section 4, adaptive error
 *                                          estimation: tau and the second
 *                                          largest sketch k')
 *
 * Parameter limits: 1 <= l <= 64, k >= 1, n < 2^27.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <pthread.h>

#define OR_GAMMA 0x9E3779B97F4A7C15ULL
#define OR_EDGE_BASE (1ULL << 62)
#define OR_NONE UINT64_MAX

/* ---------------------------------------------------------------- random */

static uint64_t or_mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t or_sm64(uint64_t seed, uint64_t counter)
{
    return or_mix64(seed + (counter + 1) * OR_GAMMA);
}

uint64_t or_rank(uint64_t seed, uint32_t v, uint32_t i)
{
    return or_sm64(seed, (uint64_t)v * 64 + i);
}

int or_live(uint64_t seed, uint32_t n, uint32_t u, uint32_t v, uint32_t i, uint32_t thr)
{
    uint64_t key = (uint64_t)u * n + v;
    uint64_t h = or_sm64(seed, OR_EDGE_BASE + key * 32 + (i >> 1));
    uint32_t coin = (i & 1) ? (uint32_t)h : (uint32_t)(h >> 32);
    return coin <= thr;
}

/* All ranks, node-major: out[v*l + i] = r(v, i). */
void or_ranks(uint64_t seed, uint32_t n, uint32_t ell, uint64_t *out)
{
    for (uint32_t v = 0; v < n; v++)
        for (uint32_t i = 0; i < ell; i++) out[(uint64_t)v * ell + i] = or_rank(seed, v, i);
}

/* Ranks of arbitrary pair ids p = 64 v + i: out[j] = r(v, i). */
void or_pair_ranks(uint64_t seed, uint64_t cnt, const uint64_t *pairs, uint64_t *out)
{
    for (uint64_t j = 0; j < cnt; j++) out[j] = or_sm64(seed, pairs[j]);
}

/* Live-edge coins for a batch of (u, v, i, thr) tuples. */
void or_live_batch(uint64_t seed, uint32_t n, uint64_t cnt, const uint32_t *u,
                   const uint32_t *v, const uint32_t *inst, const uint32_t *thr, uint8_t *out)
{
    for (uint64_t j = 0; j < cnt; j++) out[j] = (uint8_t)or_live(seed, n, u[j], v[j], inst[j], thr[j]);
}

/* ---------------------------------------------------------------- graph */

typedef struct {
    uint32_t n;
    const uint64_t *row_ptr; /* [n+1] forward CSR */
    const uint32_t *col;     /* heads */
    const uint32_t *thr;     /* thresholds aligned with col */
} or_graph;

/* ------------------------------------------- influence by forward search */

/* Nodes reached from the set S in instance i (Section 2: u in S counts),
 * scanning at most *budget out-edges (the budget is decremented by the edges
 * scanned).  Returns UINT64_MAX, with `seen` cleared, when the search would
 * scan more; otherwise the reached nodes are in queue[0..returned). */
static uint64_t reach_count_budget(const or_graph *g, uint64_t seed, uint32_t i,
                                   const uint32_t *S, uint64_t ns, uint8_t *seen,
                                   uint32_t *queue, uint64_t *budget)
{
    uint64_t head = 0, tail = 0, aborted = 0;
    for (uint64_t j = 0; j < ns; j++) {
        uint32_t s = S[j];
        if (!seen[s]) { seen[s] = 1; queue[tail++] = s; }
    }
    while (head < tail && !aborted) {
        uint32_t u = queue[head++];
        uint64_t deg = g->row_ptr[u + 1] - g->row_ptr[u];
        if (deg > *budget) { aborted = 1; break; }
        *budget -= deg;
        for (uint64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; e++) {
            uint32_t v = g->col[e];
            if (!seen[v] && or_live(seed, g->n, u, v, i, g->thr[e])) {
                seen[v] = 1;
                queue[tail++] = v;
            }
        }
    }
    for (uint64_t j = 0; j < tail; j++) seen[queue[j]] = 0;
    return aborted ? UINT64_MAX : tail;
}

static uint64_t reach_count(const or_graph *g, uint64_t seed, uint32_t i,
                            const uint32_t *S, uint64_t ns, uint8_t *seen, uint32_t *queue)
{
    uint64_t unlimited = UINT64_MAX;
    return reach_count_budget(g, seed, i, S, ns, seen, queue, &unlimited);
}

/* sum over instances of |reach_i(S)|, i.e. l * Inf({G^(i)}, S); per-instance
 * counts go to per_inst[l] when it is not NULL.  Returns 0 on bad input. */
uint64_t or_influence(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                      const uint32_t *thr, uint64_t seed, uint32_t ell,
                      const uint32_t *S, uint64_t ns, uint64_t *per_inst)
{
    or_graph g = {n, row_ptr, col, thr};
    for (uint64_t j = 0; j < ns; j++) if (S[j] >= n) return 0;
    uint8_t *seen = calloc(n ? n : 1, 1);
    uint32_t *queue = malloc(sizeof(uint32_t) * (n ? n : 1));
    uint64_t total = 0;
    for (uint32_t i = 0; i < ell; i++) {
        uint64_t c = reach_count(&g, seed, i, S, ns, seen, queue);
        if (per_inst) per_inst[i] = c;
        total += c;
    }
    free(seen);
    free(queue);
    return total;
}

/* ------------------------------------------------ sketches by definition */

static int cmp_u64(const void *a, const void *b)
{
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

/* X_u = the k smallest ranks r(v,i) over all (v,i) with u ~>_i v
 * (eq. combinedrs), computed by a full forward search in every instance.
 * out_ranks[j*k .. j*k+k) ascending, padded with UINT64_MAX; out_size[j] =
 * min(k, |R_u|); out_reach[j] (may be NULL) = |R_u|.  With a finite
 * `budget`, a node whose searches would scan more out-edges in total is
 * left out: out_ok[j] = 0 and its outputs are not written (out_ok may be
 * NULL when the budget is UINT64_MAX).  Nodes are split over `threads`
 * POSIX threads. */
typedef struct {
    or_graph g;
    uint64_t seed, budget;
    uint32_t ell, k;
    const uint32_t *nodes;
    uint64_t nq, first, step;
    uint64_t *out_ranks, *out_reach;
    uint32_t *out_size;
    uint8_t *out_ok;
    const uint64_t *rank_table;  /* [64 n] ranks of the pairs, or NULL: r(v, i) */
} brute_job;

static void *brute_worker(void *arg)
{
    brute_job *J = arg;
    uint8_t *seen = calloc(J->g.n ? J->g.n : 1, 1);
    uint32_t *queue = malloc(sizeof(uint32_t) * (J->g.n ? J->g.n : 1));
    uint64_t cap = 1024, cnt;
    uint64_t *all = malloc(sizeof(uint64_t) * cap);
    for (uint64_t j = J->first; j < J->nq; j += J->step) {
        uint32_t u = J->nodes[j];
        uint64_t budget = J->budget;
        int ok = 1;
        cnt = 0;
        for (uint32_t i = 0; i < J->ell && ok; i++) {
            uint64_t reached = reach_count_budget(&J->g, J->seed, i, &u, 1, seen, queue, &budget);
            if (reached == UINT64_MAX) { ok = 0; break; }
            if (cnt + reached > cap) {
                while (cnt + reached > cap) cap *= 2;
                all = realloc(all, sizeof(uint64_t) * cap);
            }
            for (uint64_t t = 0; t < reached; t++)
                all[cnt++] = J->rank_table ? J->rank_table[(uint64_t)queue[t] * 64 + i]
                                           : or_rank(J->seed, queue[t], i);
        }
        if (J->out_ok) J->out_ok[j] = (uint8_t)ok;
        if (!ok) continue;
        qsort(all, cnt, sizeof(uint64_t), cmp_u64);
        uint32_t s = (uint32_t)(cnt < J->k ? cnt : J->k);
        for (uint32_t t = 0; t < J->k; t++) J->out_ranks[j * J->k + t] = t < s ? all[t] : OR_NONE;
        J->out_size[j] = s;
        if (J->out_reach) J->out_reach[j] = cnt;
    }
    free(seen);
    free(queue);
    free(all);
    return NULL;
}

void or_sketch_brute_budget(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                            const uint32_t *thr, uint64_t seed, uint32_t ell, uint32_t k,
                            const uint32_t *nodes, uint64_t nq, uint64_t budget,
                            uint32_t threads, uint64_t *out_ranks, uint32_t *out_size,
                            uint64_t *out_reach, uint8_t *out_ok)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    brute_job jobs[256];
    pthread_t tid[256];
    for (uint32_t t = 0; t < threads; t++) {
        brute_job J = {{n, row_ptr, col, thr}, seed, budget, ell, k, nodes, nq, t, threads,
                       out_ranks, out_reach, out_size, out_ok, NULL};
        jobs[t] = J;
    }
    for (uint32_t t = 1; t < threads; t++) pthread_create(&tid[t], NULL, brute_worker, &jobs[t]);
    brute_worker(&jobs[0]);
    for (uint32_t t = 1; t < threads; t++) pthread_join(tid[t], NULL);
}

/* The definition with the ranks of a table (rank_table[64 v + i] for pair
 * (v, i)) in place of r(v, i): structured permutation positions. */
void or_sketch_brute_table(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                           const uint32_t *thr, uint64_t seed, uint32_t ell, uint32_t k,
                           const uint64_t *rank_table, const uint32_t *nodes, uint64_t nq,
                           uint64_t *out_ranks, uint32_t *out_size)
{
    brute_job J = {{n, row_ptr, col, thr}, seed, UINT64_MAX, ell, k, nodes, nq, 0, 1,
                   out_ranks, NULL, out_size, NULL, rank_table};
    brute_worker(&J);
}

void or_sketch_brute(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                     const uint32_t *thr, uint64_t seed, uint32_t ell, uint32_t k,
                     const uint32_t *nodes, uint64_t nq,
                     uint64_t *out_ranks, uint32_t *out_size, uint64_t *out_reach)
{
    or_sketch_brute_budget(n, row_ptr, col, thr, seed, ell, k, nodes, nq, UINT64_MAX, 1,
                           out_ranks, out_size, out_reach, NULL);
}

/* --------------------------------------------------- Algorithm 2 (5.2) */

typedef struct {
    uint64_t n_ins;   /* sum_{v,i} min(k, |R_i(v)|): rank insertions      */
    uint64_t w_live;  /* sum_{v,i} min(k,|R_i(v)|) * live indeg_i(v)     */
    uint64_t n_exp;   /* sum_v max_i min(k, |R_i(v)|)                     */
    uint64_t c_min;   /* sum_v max_i min(k, |R_i(v)|) * indeg(v)          */
} or_build_counters;

typedef struct {
    const or_graph *g;
    uint64_t seed;
    uint32_t ell, k;
    const uint64_t *rank_table;  /* [64 n] pair ranks, or NULL: r(v, i) */
    uint64_t *X;          /* [n*k] global sketches */
    uint32_t *Xs;         /* [n]   global sizes    */
    uint16_t *emax;       /* [n]   max_i E_{v,i} (under lock) */
    pthread_mutex_t *locks;
    uint32_t nlocks;
    uint32_t next_inst;   /* work counter (under qlock) */
    pthread_mutex_t qlock;
    uint64_t n_ins, w_live;  /* under qlock */
} alg2_ctx;

typedef struct { uint64_t r; uint32_t v; } rank_node;

static int cmp_rank_node(const void *a, const void *b)
{
    uint64_t x = ((const rank_node *)a)->r, y = ((const rank_node *)b)->r;
    return (x > y) - (x < y);
}

static void *alg2_worker(void *arg)
{
    alg2_ctx *c = arg;
    const or_graph *g = c->g;
    uint32_t n = g->n, k = c->k;
    uint64_t m = g->row_ptr[n];
    /* instance-local buffers */
    uint8_t *live = malloc(m ? m : 1);
    uint64_t *lptr = malloc(sizeof(uint64_t) * (n + 1));
    uint32_t *lsrc = malloc(sizeof(uint32_t) * (m ? m : 1));
    uint64_t *fill = malloc(sizeof(uint64_t) * (n + 1));
    rank_node *order = malloc(sizeof(rank_node) * n);
    uint32_t *cnt = malloc(sizeof(uint32_t) * n);
    uint32_t *stamp = malloc(sizeof(uint32_t) * n);
    uint32_t *queue = malloc(sizeof(uint32_t) * n);
    uint64_t rcap = (uint64_t)n * 4 + 16, nrec;
    uint32_t *rec_v = malloc(sizeof(uint32_t) * rcap);   /* records in the   */
    uint64_t *rec_r = malloc(sizeof(uint64_t) * rcap);   /* order they occur */
    uint64_t *sorted = NULL;
    uint64_t scap = 0;
    uint64_t *merged = malloc(sizeof(uint64_t) * k);

    for (;;) {
        pthread_mutex_lock(&c->qlock);
        uint32_t i = c->next_inst++;
        pthread_mutex_unlock(&c->qlock);
        if (i >= c->ell) break;

        /* The live reverse graph of instance i: in-lists of live edges. */
        memset(lptr, 0, sizeof(uint64_t) * (n + 1));
        for (uint32_t u = 0; u < n; u++)
            for (uint64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; e++) {
                live[e] = (uint8_t)or_live(c->seed, n, u, g->col[e], i, g->thr[e]);
                if (live[e]) lptr[g->col[e] + 1]++;
            }
        for (uint32_t v = 0; v < n; v++) lptr[v + 1] += lptr[v];
        memcpy(fill, lptr, sizeof(uint64_t) * (n + 1));
        for (uint32_t u = 0; u < n; u++)
            for (uint64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; e++)
                if (live[e]) lsrc[fill[g->col[e]]++] = u;

        /* Pairs (u, i) of this instance by increasing rank. */
        for (uint32_t u = 0; u < n; u++) {
            order[u].r = c->rank_table ? c->rank_table[(uint64_t)u * 64 + i]
                                       : or_rank(c->seed, u, i);
            order[u].v = u;
        }
        qsort(order, n, sizeof(rank_node), cmp_rank_node);
        for (uint32_t v = 0; v < n; v++) { cnt[v] = 0; stamp[v] = UINT32_MAX; }
        nrec = 0;

        /* Pruned reverse searches: a scanned node whose local sketch already
         * holds k ranks is pruned (not recorded, not expanded). */
        for (uint32_t t = 0; t < n; t++) {
            uint32_t u = order[t].v;
            uint64_t r = order[t].r;
            uint64_t head = 0, tail = 0;
            stamp[u] = t;
            if (cnt[u] == k) continue;
            queue[tail++] = u;
            while (head < tail) {
                uint32_t v = queue[head++];
                /* v is scanned and not pruned: record r in local[v] */
                cnt[v]++;
                if (nrec == rcap) {
                    rcap *= 2;
                    rec_v = realloc(rec_v, sizeof(uint32_t) * rcap);
                    rec_r = realloc(rec_r, sizeof(uint64_t) * rcap);
                }
                rec_v[nrec] = v;
                rec_r[nrec] = r;
                nrec++;
                for (uint64_t e = lptr[v]; e < lptr[v + 1]; e++) {
                    uint32_t w = lsrc[e];
                    if (stamp[w] == t) continue;
                    stamp[w] = t;
                    if (cnt[w] == k) continue;
                    queue[tail++] = w;
                }
            }
        }

        /* Group the records by node, keeping their order: sources went by
         * increasing rank, so every local sketch comes out sorted. */
        if (nrec > scap) {
            scap = nrec;
            sorted = realloc(sorted, sizeof(uint64_t) * scap);
        }
        fill[0] = 0;
        for (uint32_t v = 0; v < n; v++) fill[v + 1] = fill[v] + cnt[v];
        for (uint64_t t = 0; t < nrec; t++) sorted[fill[rec_v[t]]++] = rec_r[t];

        /* Merge local sketches into the global sketches and trim to k. */
        uint64_t ins = 0, wl = 0, base = 0;
        for (uint32_t v = 0; v < n; v++) {
            uint32_t lc = cnt[v];
            const uint64_t *L = sorted + base;
            base += lc;
            ins += lc;
            wl += (uint64_t)lc * (lptr[v + 1] - lptr[v]);
            if (lc == 0) continue;
            pthread_mutex_t *lk = &c->locks[v % c->nlocks];
            pthread_mutex_lock(lk);
            uint64_t *X = c->X + (uint64_t)v * k;
            uint32_t a = 0, b = 0, o = 0, xs = c->Xs[v];
            while (o < k && (a < xs || b < lc)) {
                if (b >= lc || (a < xs && X[a] < L[b])) merged[o++] = X[a++];
                else merged[o++] = L[b++];
            }
            memcpy(X, merged, sizeof(uint64_t) * o);
            c->Xs[v] = o;
            if (lc > c->emax[v]) c->emax[v] = (uint16_t)lc;
            pthread_mutex_unlock(lk);
        }
        pthread_mutex_lock(&c->qlock);
        c->n_ins += ins;
        c->w_live += wl;
        pthread_mutex_unlock(&c->qlock);
    }
    free(live); free(lptr); free(lsrc); free(fill); free(order); free(cnt); free(stamp);
    free(queue); free(rec_v); free(rec_r); free(sorted); free(merged);
    return NULL;
}

/* Combined bottom-k sketches of every node by Algorithm 2.
 * out_ranks[n*k] ascending with UINT64_MAX padding, out_size[n].
 * Returns 0 on success, -1 on bad arguments. */
static int build_alg2(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                      const uint32_t *thr, uint64_t seed, uint32_t ell, uint32_t k,
                      const uint64_t *rank_table, uint32_t nthreads, uint64_t *out_ranks,
                      uint32_t *out_size, or_build_counters *counters)
{
    if (ell < 1 || ell > 64 || k < 1 || k > 65535 || n == 0) return -1;
    or_graph g = {n, row_ptr, col, thr};
    alg2_ctx c;
    memset(&c, 0, sizeof c);
    c.g = &g; c.seed = seed; c.ell = ell; c.k = k; c.rank_table = rank_table;
    c.X = out_ranks; c.Xs = out_size;
    for (uint64_t j = 0; j < (uint64_t)n * k; j++) out_ranks[j] = OR_NONE;
    for (uint32_t v = 0; v < n; v++) out_size[v] = 0;
    c.emax = calloc(n, sizeof(uint16_t));
    c.nlocks = 4096;
    c.locks = malloc(sizeof(pthread_mutex_t) * c.nlocks);
    for (uint32_t j = 0; j < c.nlocks; j++) pthread_mutex_init(&c.locks[j], NULL);
    pthread_mutex_init(&c.qlock, NULL);
    if (nthreads < 1) nthreads = 1;
    if (nthreads > ell) nthreads = ell;
    pthread_t *th = malloc(sizeof(pthread_t) * nthreads);
    for (uint32_t t = 0; t < nthreads; t++) pthread_create(&th[t], NULL, alg2_worker, &c);
    for (uint32_t t = 0; t < nthreads; t++) pthread_join(th[t], NULL);
    if (counters) {
        counters->n_ins = c.n_ins;
        counters->w_live = c.w_live;
        counters->n_exp = 0;
        counters->c_min = 0;
        for (uint32_t v = 0; v < n; v++) counters->n_exp += c.emax[v];
        uint64_t *indeg = calloc(n, sizeof(uint64_t));
        for (uint64_t e = 0; e < row_ptr[n]; e++) indeg[col[e]]++;
        for (uint32_t v = 0; v < n; v++) counters->c_min += (uint64_t)c.emax[v] * indeg[v];
        free(indeg);
    }
    for (uint32_t j = 0; j < c.nlocks; j++) pthread_mutex_destroy(&c.locks[j]);
    pthread_mutex_destroy(&c.qlock);
    free(c.locks); free(c.emax); free(th);
    return 0;
}

int or_build_alg2(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                  const uint32_t *thr, uint64_t seed, uint32_t ell, uint32_t k,
                  uint32_t nthreads, uint64_t *out_ranks, uint32_t *out_size,
                  or_build_counters *counters)
{
    return build_alg2(n, row_ptr, col, thr, seed, ell, k, NULL, nthreads, out_ranks, out_size,
                      counters);
}

/* Algorithm 2 with the ranks of a table (rank_table[64 v + i]): the same
 * searches, pairs taken in increasing order of their table rank. */
int or_build_alg2_table(uint32_t n, const uint64_t *row_ptr, const uint32_t *col,
                        const uint32_t *thr, uint64_t seed, uint32_t ell, uint32_t k,
                        const uint64_t *rank_table, uint32_t nthreads, uint64_t *out_ranks,
                        uint32_t *out_size, or_build_counters *counters)
{
    if (!rank_table) return -1;
    return build_alg2(n, row_ptr, col, thr, seed, ell, k, rank_table, nthreads, out_ranks,
                      out_size, counters);
}

/* ------------------------------------------------------------ estimates */

static double or_rho(uint64_t T)
{
    return (double)((T >> 11) + 1) * 0x1p-53;
}

/* Bottom-k cardinality estimate divided by l: |X|/l when |X| < k, else
 * ((k-1)/rho(tau))/l with tau the k-th smallest rank. */
static double or_estimate_one(uint64_t size, uint64_t tau, uint32_t k, uint32_t ell)
{
    if (size < k) return (double)size / (double)ell;
    return ((double)(k - 1) / or_rho(tau)) / (double)ell;
}

void or_estimates(uint32_t n, uint32_t k, uint32_t ell, const uint64_t *ranks,
                  const uint32_t *size, double *out_est)
{
    for (uint32_t v = 0; v < n; v++)
        out_est[v] = or_estimate_one(size[v], ranks[(uint64_t)v * k + k - 1], k, ell);
}

/* ---------------------------------------------------- union queries 5.1 */

/* For each seed set S_q = nodes[offsets[q] .. offsets[q+1]): the k smallest
 * distinct ranks of the union of the sketches of S_q; estimate by the same
 * bottom-k rule.  Duplicate nodes act once; an empty set gives 0; a node id
 * >= n gives status -1 and estimate 0 for that query only. */
void or_union_query(uint32_t n, uint32_t k, uint32_t ell, const uint64_t *ranks,
                    const uint32_t *size, uint64_t Q, const uint64_t *offsets,
                    const uint32_t *nodes, double *out_est, int32_t *out_status)
{
    uint64_t cap = 1024;
    uint64_t *buf = malloc(sizeof(uint64_t) * cap);
    for (uint64_t q = 0; q < Q; q++) {
        uint64_t a = offsets[q], b = offsets[q + 1], cnt = 0;
        int bad = 0;
        for (uint64_t j = a; j < b; j++) if (nodes[j] >= n) bad = 1;
        if (bad) { out_est[q] = 0.0; if (out_status) out_status[q] = -1; continue; }
        if ((b - a) * k > cap) {
            while ((b - a) * k > cap) cap *= 2;
            buf = realloc(buf, sizeof(uint64_t) * cap);
        }
        for (uint64_t j = a; j < b; j++) {
            uint32_t u = nodes[j];
            for (uint32_t t = 0; t < size[u]; t++) buf[cnt++] = ranks[(uint64_t)u * k + t];
        }
        qsort(buf, cnt, sizeof(uint64_t), cmp_u64);
        uint64_t d = 0;
        for (uint64_t t = 0; t < cnt; t++)
            if (d == 0 || buf[t] != buf[d - 1]) buf[d++] = buf[t];
        out_est[q] = or_estimate_one(d < k ? d : k, d >= k ? buf[k - 1] : 0, k, ell);
        if (out_status) out_status[q] = 0;
    }
    free(buf);
}

/* Cohen-Kaplan union estimator, eq. (unionest), divided by l.  Each node's
 * threshold tau_u is its k-th rank when the sketch is full, and 1 (the top
 * of the rank range) otherwise; the tau element itself is excluded from a
 * full sketch.  Every distinct remaining rank z contributes
 * 1 / rho(max tau_u over the sketches holding z as a non-tau element); a
 * non-full holder contributes weight exactly 1.  Contributions are summed in
 * increasing order of z.  Status as in or_union_query. */
void or_ck_query(uint32_t n, uint32_t k, uint32_t ell, const uint64_t *ranks,
                 const uint32_t *size, uint64_t Q, const uint64_t *offsets,
                 const uint32_t *nodes, double *out_est, int32_t *out_status)
{
    uint64_t cap = 1024;
    uint64_t *buf = malloc(sizeof(uint64_t) * cap * 2);
    for (uint64_t q = 0; q < Q; q++) {
        uint64_t a = offsets[q], b = offsets[q + 1], cnt = 0;
        int bad = 0;
        for (uint64_t j = a; j < b; j++) if (nodes[j] >= n) bad = 1;
        if (bad) { out_est[q] = 0.0; if (out_status) out_status[q] = -1; continue; }
        if ((b - a) * k > cap) {
            while ((b - a) * k > cap) cap *= 2;
            buf = realloc(buf, sizeof(uint64_t) * cap * 2);
        }
        /* (rank, holder's threshold) pairs; a non-full holder's threshold is
         * encoded as UINT64_MAX, meaning rho = 1. */
        for (uint64_t j = a; j < b; j++) {
            uint32_t u = nodes[j];
            uint32_t s = size[u];
            int full = (s == k);
            uint64_t tau = full ? ranks[(uint64_t)u * k + k - 1] : OR_NONE;
            uint32_t lim = full ? k - 1 : s;
            for (uint32_t t = 0; t < lim; t++) {
                buf[2 * cnt] = ranks[(uint64_t)u * k + t];
                buf[2 * cnt + 1] = tau;
                cnt++;
            }
        }
        qsort(buf, cnt, 2 * sizeof(uint64_t), cmp_u64); /* by rank (first word) */
        double sum = 0.0;
        uint64_t x = 0;
        while (x < cnt) {
            uint64_t r = buf[2 * x], tmax = buf[2 * x + 1];
            uint64_t y = x + 1;
            while (y < cnt && buf[2 * y] == r) {
                if (buf[2 * y + 1] > tmax) tmax = buf[2 * y + 1];
                y++;
            }
            sum += (tmax == OR_NONE) ? 1.0 : 1.0 / or_rho(tmax);
            x = y;
        }
        out_est[q] = sum / (double)ell;
        if (out_status) out_status[q] = 0;
    }
    free(buf);
}

/* ------------------------------------------------------ Algorithm 1 (4) */

typedef struct {
    uint64_t insertions;   /* size[v]++ operations (rank insertions)       */
    uint64_t pairs_scanned;/* pairs taken from the rank order               */
    uint64_t reverse_bfs;  /* reverse searches run (uncovered pairs)        */
    uint64_t covered;      /* pairs covered by the residual updates         */
    uint64_t decrements;   /* size[w]-- operations                          */
    uint64_t fallback;     /* seeds chosen by the exhaustion argmax         */
} or_skim_counters;

/* Per-instance live adjacency: forward and reverse CSR of live edges. */
typedef struct { uint64_t *fptr, *rptr; uint32_t *fadj, *radj; } live_inst;

static void build_live(const or_graph *g, uint64_t seed, uint32_t i, live_inst *L)
{
    uint32_t n = g->n;
    uint64_t m = g->row_ptr[n];
    L->fptr = calloc(n + 1, sizeof(uint64_t));
    L->rptr = calloc(n + 1, sizeof(uint64_t));
    uint8_t *live = malloc(m ? m : 1);
    uint64_t cntl = 0;
    for (uint32_t u = 0; u < n; u++)
        for (uint64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; e++) {
            live[e] = (uint8_t)or_live(seed, n, u, g->col[e], i, g->thr[e]);
            if (live[e]) { L->fptr[u + 1]++; L->rptr[g->col[e] + 1]++; cntl++; }
        }
    for (uint32_t v = 0; v < n; v++) { L->fptr[v + 1] += L->fptr[v]; L->rptr[v + 1] += L->rptr[v]; }
    L->fadj = malloc(sizeof(uint32_t) * (cntl ? cntl : 1));
    L->radj = malloc(sizeof(uint32_t) * (cntl ? cntl : 1));
    uint64_t *rf = calloc(n, sizeof(uint64_t));
    uint64_t fo = 0;
    for (uint32_t u = 0; u < n; u++)
        for (uint64_t e = g->row_ptr[u]; e < g->row_ptr[u + 1]; e++)
            if (live[e]) {
                uint32_t v = g->col[e];
                L->fadj[fo++] = v;
                L->radj[L->rptr[v] + rf[v]++] = u;
            }
    free(rf);
    free(live);
}

/* SKIM (Algorithm 1) for s seeds.  Ties: among the nodes whose size reaches
 * k during the reverse search of one pair, the smallest id is selected; the
 * exhaustion fallback takes the largest size among unselected nodes,
 * smallest id on ties.  out_seeds[s], out_gain[s] = newly covered pairs
 * (l times the marginal influence).
 *
 * Records for the adaptive error estimate (may be NULL), taken at the moment
 * the seed is chosen, before its residual update:
 *   out_tau[s]    the rank of the pair whose reverse search filled the seed's
 *                 sketch; OR_NONE for a seed of the exhaustion rule;
 *   out_second[s] the second largest sketch: the largest size among the other
 *                 unselected nodes, not counting the pair of rank tau (a node
 *                 that pair's search reached counts one less), so it is at
 *                 most k-1; for an exhaustion seed, the largest size among
 *                 the other unselected nodes.
 * Returns 0, or -1 on bad arguments, or -2 if the reverse search of an
 * uncovered pair met a covered pair (an internal invariant; cannot happen). */
int or_skim(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, const uint32_t *thr,
            uint64_t seed, uint32_t ell, uint32_t k, uint32_t s,
            uint32_t *out_seeds, uint64_t *out_gain, uint64_t *out_tau, uint32_t *out_second,
            or_skim_counters *counters)
{
    if (ell < 1 || ell > 64 || k < 1 || s > n || n == 0) return -1;
    or_graph g = {n, row_ptr, col, thr};
    uint64_t npairs = (uint64_t)n * ell;
    live_inst *L = malloc(sizeof(live_inst) * ell);
    for (uint32_t i = 0; i < ell; i++) build_live(&g, seed, i, &L[i]);

    /* "shuffle the n*l pairs": the random order is increasing rank */
    rank_node *pairs = malloc(sizeof(rank_node) * npairs);
    for (uint32_t u = 0; u < n; u++)
        for (uint32_t i = 0; i < ell; i++) {
            pairs[(uint64_t)u * ell + i].r = or_rank(seed, u, i);
            pairs[(uint64_t)u * ell + i].v = u * 64 + i; /* packed (u, i) */
        }
    qsort(pairs, npairs, sizeof(rank_node), cmp_rank_node);

    uint8_t *covered = calloc(npairs, 1);           /* [u*ell + i] */
    uint32_t *size = calloc(n, sizeof(uint32_t));
    uint8_t *selected = calloc(n, 1);
    /* index[(u,i)]: nodes whose partial sketch holds r(u,i) */
    uint32_t **idx = calloc(npairs, sizeof(uint32_t *));
    uint32_t *idxn = calloc(npairs, sizeof(uint32_t));
    uint64_t *stamp = malloc(sizeof(uint64_t) * n);
    uint32_t *queue = malloc(sizeof(uint32_t) * n);
    uint8_t *seen = calloc(n, 1);
    for (uint32_t v = 0; v < n; v++) stamp[v] = 0;
    or_skim_counters cc;
    memset(&cc, 0, sizeof cc);
    uint64_t cursor = 0;
    int rc = 0;

    for (uint32_t it = 0; it < s; it++) {
        int64_t x = -1;
        uint64_t tau = OR_NONE, last_tag = 0;
        /* Build sketches: pairs by increasing rank, skipping covered ones. */
        while (x < 0 && cursor < npairs) {
            uint32_t packed = pairs[cursor].v;
            uint32_t u = packed / 64, i = packed % 64;
            uint64_t pid = (uint64_t)u * ell + i;
            cursor++;
            cc.pairs_scanned++;
            if (covered[pid]) continue;
            cc.reverse_bfs++;
            /* complete reverse search from u in G^(i) */
            uint64_t head = 0, tail = 0;
            uint64_t tag = cursor; /* >= 1 and distinct per search */
            stamp[u] = tag;
            queue[tail++] = u;
            while (head < tail) {
                uint32_t v = queue[head++];
                for (uint64_t e = L[i].rptr[v]; e < L[i].rptr[v + 1]; e++) {
                    uint32_t w = L[i].radj[e];
                    if (stamp[w] != tag) { stamp[w] = tag; queue[tail++] = w; }
                }
            }
            idx[pid] = malloc(sizeof(uint32_t) * tail);
            idxn[pid] = (uint32_t)tail;
            for (uint64_t t = 0; t < tail; t++) {
                uint32_t v = queue[t];
                if (covered[(uint64_t)v * ell + i]) { rc = -2; goto done; }
                size[v]++;
                cc.insertions++;
                idx[pid][t] = v;
                if (size[v] == k && (x < 0 || v < (uint32_t)x)) x = v;
            }
            if (x >= 0) { tau = pairs[cursor - 1].r; last_tag = tag; }
        }
        if (x < 0) {
            /* every rank processed: largest partial sketch, unselected */
            uint32_t best = 0;
            for (uint32_t v = 0; v < n; v++) {
                if (selected[v]) continue;
                if (x < 0 || size[v] > best) { best = size[v]; x = v; }
            }
            cc.fallback++;
        }
        /* second largest sketch, without the pair of rank tau (whose search
         * carries the stamp last_tag; 0 when the seed came from exhaustion) */
        uint32_t second = 0;
        for (uint32_t v = 0; v < n; v++) {
            if (selected[v] || v == (uint32_t)x) continue;
            uint32_t sz = size[v] - (last_tag && stamp[v] == last_tag ? 1u : 0u);
            if (sz > second) second = sz;
        }
        if (out_tau) out_tau[it] = tau;
        if (out_second) out_second[it] = second;
        /* Residual problem: cover what x reaches in every instance. */
        uint64_t gain = 0;
        for (uint32_t i = 0; i < ell; i++) {
            if (covered[(uint64_t)x * ell + i]) continue;
            uint64_t head = 0, tail = 0;
            seen[x] = 1;
            queue[tail++] = (uint32_t)x;
            while (head < tail) {
                uint32_t v = queue[head++];
                uint64_t pid = (uint64_t)v * ell + i;
                covered[pid] = 1;
                gain++;
                for (uint32_t t = 0; t < idxn[pid]; t++) { size[idx[pid][t]]--; cc.decrements++; }
                free(idx[pid]);
                idx[pid] = NULL;
                idxn[pid] = 0;
                for (uint64_t e = L[i].fptr[v]; e < L[i].fptr[v + 1]; e++) {
                    uint32_t w = L[i].fadj[e];
                    if (!seen[w] && !covered[(uint64_t)w * ell + i]) { seen[w] = 1; queue[tail++] = w; }
                }
            }
            for (uint64_t t = 0; t < tail; t++) seen[queue[t]] = 0;
        }
        cc.covered += gain;
        selected[x] = 1;
        out_seeds[it] = (uint32_t)x;
        out_gain[it] = gain;
    }
done:
    if (counters) *counters = cc;
    for (uint64_t p = 0; p < npairs; p++) free(idx[p]);
    free(idx); free(idxn); free(stamp); free(queue); free(seen);
    free(covered); free(size); free(selected); free(pairs);
    for (uint32_t i = 0; i < ell; i++) { free(L[i].fptr); free(L[i].rptr); free(L[i].fadj); free(L[i].radj); }
    free(L);
    return rc;
}

/* ------------------------------------- IC-model sketches (Section 3, 4) */
/* Sketches for the IC model itself (Section 3, "Sketches for an IC model"),
 * with structured permutation ranks (Section 3, "Structured permutation
 * ranks") in the limit l -> infinity, where every rank position is a node in
 * an instance of its own.  Conventions fixed here:
 *  - chunk c (0 <= c < k) holds positions c n + 1 .. (c + 1) n, each node
 *    once: node v takes position c n + 1 + |{w : h_c(w) < h_c(v)}| with
 *    h_c(v) = SM(seed, 2^63 + c n + v) (distinct: SM is a bijection);
 *  - position t has instance t; the coin of edge (u -> w) in instance t is
 *    the high (t - 1 even) or low (t - 1 odd) half of
 *    SM(SM(seed, 2^63 + 2^62 + u n + w), floor((t - 1) / 2)), live iff
 *    coin <= thr, so P[live] = (thr + 1) / 2^32 independently per instance;
 *  - X_u = the k smallest positions t such that u reaches v_t (the node at
 *    position t) in instance t.  Only positions up to k n matter: u holds one
 *    position of its own in every chunk;
 *  - the influence estimate is n (k - 1) / (T - 1), T the k-th smallest
 *    position (the limit of the permutation-rank estimator divided by l). */
#define OR_IC_CHUNK (1ULL << 63)
#define OR_IC_EDGE ((1ULL << 63) | (1ULL << 62))

int or_ic_live(uint64_t seed, uint32_t n, uint32_t u, uint32_t w, uint64_t t, uint32_t thr)
{
    uint64_t edge_seed = or_sm64(seed, OR_IC_EDGE + (uint64_t)u * n + w);
    uint64_t h = or_sm64(edge_seed, (t - 1) / 2);
    uint32_t coin = ((t - 1) % 2 == 0) ? (uint32_t)(h >> 32) : (uint32_t)h;
    return coin <= thr;
}

/* node_at[t - 1] = the node at position t, for t = 1 .. k n */
void or_ic_order(uint64_t seed, uint32_t n, uint32_t k, uint32_t *node_at)
{
    rank_node *tmp = malloc(sizeof(rank_node) * (n ? n : 1));
    for (uint32_t c = 0; c < k; c++) {
        for (uint32_t v = 0; v < n; v++) {
            tmp[v].r = or_sm64(seed, OR_IC_CHUNK + (uint64_t)c * n + v);
            tmp[v].v = v;
        }
        qsort(tmp, n, sizeof(rank_node), cmp_rank_node);
        for (uint32_t j = 0; j < n; j++) node_at[(uint64_t)c * n + j] = tmp[j].v;
    }
    free(tmp);
}

/* out_pos[n k]: X_u ascending (1-based positions); out_est[n] (may be NULL);
 * *out_visits (may be NULL) = sum over positions of the nodes reached.
 * Returns 0, -1 on bad arguments, -2 if a node ended with fewer than k
 * positions (cannot happen: every node reaches itself in every chunk). */
int or_ic_sketches(uint32_t n, const uint64_t *row_ptr, const uint32_t *col, const uint32_t *thr,
                   uint32_t k, uint64_t seed, uint32_t *out_pos, double *out_est,
                   uint64_t *out_visits)
{
    if (n == 0 || k < 2 || (uint64_t)k * n >= (1ULL << 32)) return -1;
    uint64_t m = row_ptr[n];
    /* reverse graph: in-edges of every node with their source and threshold */
    uint64_t *rptr = calloc((size_t)n + 1, sizeof(uint64_t));
    uint32_t *rsrc = malloc(sizeof(uint32_t) * (m ? m : 1));
    uint32_t *rthr = malloc(sizeof(uint32_t) * (m ? m : 1));
    uint64_t *fill = calloc(n, sizeof(uint64_t));
    for (uint64_t e = 0; e < m; e++) rptr[col[e] + 1]++;
    for (uint32_t v = 0; v < n; v++) rptr[v + 1] += rptr[v];
    for (uint32_t u = 0; u < n; u++)
        for (uint64_t e = row_ptr[u]; e < row_ptr[u + 1]; e++) {
            uint32_t w = col[e];
            uint64_t at = rptr[w] + fill[w]++;
            rsrc[at] = u;
            rthr[at] = thr[e];
        }
    uint64_t total = (uint64_t)k * n;
    uint32_t *node_at = malloc(sizeof(uint32_t) * total);
    or_ic_order(seed, n, k, node_at);
    uint32_t *cnt = calloc(n, sizeof(uint32_t));
    uint32_t *stamp = calloc(n, sizeof(uint32_t));
    uint32_t *queue = malloc(sizeof(uint32_t) * n);
    uint64_t visits = 0;
    for (uint64_t t = 1; t <= total; t++) {
        /* reverse search from v_t in instance t: every node that reaches v_t */
        uint32_t v = node_at[t - 1];
        uint64_t head = 0, tail = 0;
        stamp[v] = (uint32_t)t;
        queue[tail++] = v;
        while (head < tail) {
            uint32_t x = queue[head++];
            for (uint64_t e = rptr[x]; e < rptr[x + 1]; e++) {
                uint32_t u = rsrc[e];
                if (stamp[u] != (uint32_t)t && or_ic_live(seed, n, u, x, t, rthr[e])) {
                    stamp[u] = (uint32_t)t;
                    queue[tail++] = u;
                }
            }
        }
        visits += tail;
        for (uint64_t j = 0; j < tail; j++) {
            uint32_t y = queue[j];
            if (cnt[y] < k) out_pos[(uint64_t)y * k + cnt[y]++] = (uint32_t)t;
        }
    }
    int rc = 0;
    for (uint32_t y = 0; y < n; y++) {
        if (cnt[y] != k) { rc = -2; break; }
        if (out_est)
            out_est[y] = ((double)n * (double)(k - 1)) /
                         (double)(out_pos[(uint64_t)y * k + k - 1] - 1);
    }
    if (out_visits) *out_visits = visits;
    free(rptr); free(rsrc); free(rthr); free(fill); free(node_at);
    free(cnt); free(stamp); free(queue);
    return rc;
}

static int cmp_u32(const void *a, const void *b)
{
    uint32_t x = *(const uint32_t *)a, y = *(const uint32_t *)b;
    return x < y ? -1 : x > y;
}

/* Union queries over IC-model sketches (Section 3 and 5.1 with structured
 * permutation ranks in the l -> infinity limit).  pos[n k]: each row
 * ascending, always k positions.  Set j = qnodes[qoff[j] .. qoff[j+1]).
 *   estimator 0 (bottom-k): T = the k-th smallest distinct position of the
 *     union of the members' sketches; est = n (k - 1) / (T - 1).
 *   estimator 1 (Cohen-Kaplan, eq. unionest with permutation ranks): every
 *     distinct position z held by some member u outside u's own threshold
 *     position T_u = X_u[k-1] weighs n / (T_max(z) - 1), T_max(z) the largest
 *     T_u over those members; the weights are added in increasing z.
 * Duplicate members act once; an empty set gives 0; a node >= n gives
 * status -1 and est 0. */
void or_ic_union_query(uint32_t n, uint32_t k, const uint32_t *pos, uint64_t q,
                       const uint64_t *qoff, const uint32_t *qnodes, uint32_t estimator,
                       double *out_est, int32_t *out_status)
{
    for (uint64_t j = 0; j < q; j++) {
        uint64_t a = qoff[j], b = qoff[j + 1], S = b - a;
        int bad = 0;
        for (uint64_t t = a; t < b; t++) if (qnodes[t] >= n) bad = 1;
        out_est[j] = 0.0;
        if (out_status) out_status[j] = bad ? -1 : 0;
        if (bad || S == 0) continue;
        uint32_t *vals = malloc(sizeof(uint32_t) * S * k);
        uint64_t c = 0;
        for (uint64_t t = a; t < b; t++) {
            const uint32_t *row = pos + (uint64_t)qnodes[t] * k;
            uint32_t lim = estimator == 1 ? k - 1 : k;
            for (uint32_t x = 0; x < lim; x++) vals[c++] = row[x];
        }
        qsort(vals, c, sizeof(uint32_t), cmp_u32);
        if (estimator == 0) {
            uint32_t d = 0, T = 0;
            for (uint64_t x = 0; x < c && d < k; x++)
                if (x == 0 || vals[x] != vals[x - 1]) { d++; T = vals[x]; }
            out_est[j] = ((double)n * (double)(k - 1)) / (double)(T - 1);
        } else {
            /* (value, holder's threshold) pairs sorted by value: each run of
             * one value gives its largest holder threshold */
            uint64_t *pairs = malloc(sizeof(uint64_t) * S * k);
            uint64_t cp = 0;
            for (uint64_t t = a; t < b; t++) {
                const uint32_t *row = pos + (uint64_t)qnodes[t] * k;
                for (uint32_t y = 0; y + 1 < k; y++)
                    pairs[cp++] = ((uint64_t)row[y] << 32) | row[k - 1];
            }
            qsort(pairs, cp, sizeof(uint64_t), cmp_u64);
            double sum = 0.0;
            for (uint64_t x = 0; x < cp; x++) {
                uint32_t z = (uint32_t)(pairs[x] >> 32);
                if (x + 1 < cp && (uint32_t)(pairs[x + 1] >> 32) == z) continue;  /* last = max */
                uint32_t Tmax = (uint32_t)pairs[x];
                sum += (double)n / (double)(Tmax - 1);
            }
            out_est[j] = sum;
            free(pairs);
        }
        free(vals);
    }
}

/* ------------------------------- structured permutation ranks (3.1) -----
 * Finite-l structured permutation ranks: the n l node-instance pairs are
 * placed at positions 1 .. n l in l chunks of n positions; chunk c holds
 * every node exactly once, in the order of h_c(v) = SM(seed, 2^63 + c n + v)
 * (the chunk order the IC-model sketches use), and the instance a node takes
 * in chunk c is drawn from the instances it has not taken in earlier chunks.
 * The draw without replacement is a uniform permutation of the node's l
 * instances: instance i goes to the chunk given by the place of
 * g_v(i) = SM(seed, 2^61 + 64 v + i) among g_v(0 .. l-1).
 * out[64 v + i] = the position of pair (v, i) (1-based), 0 for i >= l.
 * Only the first min(k, l) n positions can enter a sketch. */
#define OR_PERM_INST (1ULL << 61)

void or_perm_positions(uint64_t seed, uint32_t n, uint32_t ell, uint64_t *out)
{
    rank_node *tmp = malloc(sizeof(rank_node) * (n ? n : 1));
    uint32_t *place = malloc(sizeof(uint32_t) * (uint64_t)ell * (n ? n : 1));  /* [c n + v] */
    memset(out, 0, sizeof(uint64_t) * (uint64_t)n * 64);
    for (uint32_t c = 0; c < ell; c++) {  /* the node order of every chunk */
        for (uint32_t v = 0; v < n; v++) {
            tmp[v].r = or_sm64(seed, OR_IC_CHUNK + (uint64_t)c * n + v);
            tmp[v].v = v;
        }
        qsort(tmp, n, sizeof(rank_node), cmp_rank_node);
        for (uint32_t j = 0; j < n; j++) place[(uint64_t)c * n + tmp[j].v] = j;
    }
    for (uint32_t v = 0; v < n; v++) {  /* the instance of every chunk */
        rank_node inst[64];
        for (uint32_t i = 0; i < ell; i++) {
            inst[i].r = or_sm64(seed, OR_PERM_INST + (uint64_t)v * 64 + i);
            inst[i].v = i;
        }
        qsort(inst, ell, sizeof(rank_node), cmp_rank_node);
        for (uint32_t c = 0; c < ell; c++)
            out[(uint64_t)v * 64 + inst[c].v] = (uint64_t)c * n + place[(uint64_t)c * n + v] + 1;
    }
    free(tmp);
    free(place);
}

/* Influence estimate from permutation ranks (Section 3.1): with T the k-th
 * smallest position of X_v and D = n l, the cardinality estimate is
 * 1 + (k - 1)(D - 1)/(T - 1), divided by l (Section 3.2 gives the same
 * form: 1/l + (k - 1)(n l - 1)/(l (T - 1))); |X_v| / l when |X_v| < k.
 * Computed as (1 + ((k-1)(D-1)) / (T-1)) / l in IEEE double. */
static double or_perm_estimate_one(uint64_t size, uint64_t T, uint32_t k, uint32_t n, uint32_t ell)
{
    if (size < k) return (double)size / (double)ell;
    const double D = (double)n * (double)ell;
    return (1.0 + ((double)(k - 1) * (D - 1.0)) / (double)(T - 1)) / (double)ell;
}

void or_perm_estimates(uint32_t n, uint32_t k, uint32_t ell, const uint64_t *ranks,
                       const uint32_t *size, double *out_est)
{
    for (uint32_t v = 0; v < n; v++)
        out_est[v] = or_perm_estimate_one(size[v], size[v] >= k ? ranks[(uint64_t)v * k + k - 1] : 0,
                                          k, n, ell);
}

/* Union queries over sketches of permutation positions.
 *   estimator 0: the k smallest distinct positions of the union of the
 *     members' sketches; the estimate above with T = the k-th of them.
 *   estimator 1: Cohen-Kaplan (eq. unionest) with the permutation rank T of
 *     a threshold read as the uniform rank r = (T - 1)/(l n - 1) (Section
 *     5.1): each distinct position z held by a member outside its own
 *     threshold element weighs 1/r of the largest threshold among those
 *     members, (l n - 1)/(T_max - 1); a non-full member has threshold 1
 *     (weight 1); the weights are added in increasing z and divided by l.
 * Duplicates act once; an empty set gives 0; a node >= n gives status -1. */
void or_perm_union_query(uint32_t n, uint32_t k, uint32_t ell, const uint64_t *ranks,
                         const uint32_t *size, uint64_t Q, const uint64_t *offsets,
                         const uint32_t *nodes, uint32_t estimator, double *out_est,
                         int32_t *out_status)
{
    const double Dm1 = (double)n * (double)ell - 1.0;
    for (uint64_t q = 0; q < Q; q++) {
        uint64_t a = offsets[q], b = offsets[q + 1], cnt = 0;
        int bad = 0;
        for (uint64_t j = a; j < b; j++) if (nodes[j] >= n) bad = 1;
        out_est[q] = 0.0;
        if (out_status) out_status[q] = bad ? -1 : 0;
        if (bad || a == b) continue;
        uint64_t *buf = malloc(sizeof(uint64_t) * 2 * (b - a) * k);
        for (uint64_t j = a; j < b; j++) {
            uint32_t u = nodes[j], s = size[u];
            int full = s == k;
            uint64_t tau = full ? ranks[(uint64_t)u * k + k - 1] : OR_NONE;
            uint32_t lim = estimator == 1 && full ? k - 1 : s;
            for (uint32_t t = 0; t < lim; t++) {
                buf[2 * cnt] = ranks[(uint64_t)u * k + t];
                buf[2 * cnt + 1] = tau;
                cnt++;
            }
        }
        qsort(buf, cnt, 2 * sizeof(uint64_t), cmp_u64); /* by position (first word) */
        if (estimator == 0) {
            uint64_t d = 0, T = 0;
            for (uint64_t x = 0; x < cnt && d < k; x++)
                if (x == 0 || buf[2 * x] != buf[2 * (x - 1)]) { d++; T = buf[2 * x]; }
            out_est[q] = or_perm_estimate_one(d, T, k, n, ell);
        } else {
            double sum = 0.0;
            uint64_t x = 0;
            while (x < cnt) {
                uint64_t z = buf[2 * x], tmax = buf[2 * x + 1], y = x + 1;
                while (y < cnt && buf[2 * y] == z) {
                    if (buf[2 * y + 1] > tmax) tmax = buf[2 * y + 1];
                    y++;
                }
                sum += tmax == OR_NONE ? 1.0 : Dm1 / (double)(tmax - 1);
                x = y;
            }
            out_est[q] = sum / (double)ell;
        }
        free(buf);
    }
}
