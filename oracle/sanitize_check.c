/*
 * sanitize_check.c -- a standalone driver that runs every oracle function on
 * small seeded graphs, for AddressSanitizer and UndefinedBehaviorSanitizer
 * builds of the oracle (test infrastructure, like the oracle itself).
 *
 * It compiles the oracle into the same translation unit and checks, on
 * random graphs: Algorithm 2 (one and several threads) against the plain
 * definition, with hashed ranks and with structured permutation positions;
 * the estimates and the union estimators on every singleton;
 * SKIM to the full permutation (its gains add up to every pair); the
 * IC-model sketches and their unions.  Exit status 0 when every check
 * holds; the sanitizers abort on the first memory or undefined-behaviour
 * error.
 *
 *   gcc -O1 -g -fsanitize=address,undefined -fno-sanitize-recover=all \
 *       -pthread oracle/sanitize_check.c -o sanitize_check && ./sanitize_check
 */
#include "skim_oracle.c"

#include <stdio.h>

static uint64_t lcg(uint64_t *s)
{
    *s = *s * 6364136223846793005ULL + 1442695040888963407ULL;
    return *s >> 33;
}

/* A simple random graph: m distinct edges u -> v, u != v, as a forward CSR
 * with heads ascending per row. */
static void random_graph(uint32_t n, uint32_t m, uint64_t gs, uint32_t thr_div,
                         uint64_t **rp, uint32_t **col, uint32_t **thr)
{
    uint8_t *adj = calloc((size_t)n * n, 1);
    uint32_t made = 0;
    while (made < m) {
        uint32_t u = (uint32_t)(lcg(&gs) % n), v = (uint32_t)(lcg(&gs) % n);
        if (u == v || adj[(size_t)u * n + v]) continue;
        adj[(size_t)u * n + v] = 1;
        made++;
    }
    *rp = calloc(n + 1, sizeof(uint64_t));
    *col = malloc(sizeof(uint32_t) * (m ? m : 1));
    *thr = malloc(sizeof(uint32_t) * (m ? m : 1));
    uint64_t e = 0;
    for (uint32_t u = 0; u < n; u++) {
        for (uint32_t v = 0; v < n; v++)
            if (adj[(size_t)u * n + v]) {
                (*col)[e] = v;
                (*thr)[e] = thr_div ? UINT32_MAX / thr_div : UINT32_MAX;
                e++;
            }
        (*rp)[u + 1] = e;
    }
    free(adj);
}

static int fail(const char *what, uint32_t n, uint32_t ell, uint32_t k)
{
    fprintf(stderr, "sanitize_check: %s differs (n=%u l=%u k=%u)\n", what, n, ell, k);
    return 1;
}

int main(void)
{
    const uint32_t cases[][5] = {  /* n, m, thr divisor, l, k */
        {40, 120, 2, 8, 6}, {60, 240, 5, 16, 16}, {30, 0, 1, 4, 4},
        {50, 300, 1, 2, 3}, {70, 200, 3, 64, 64}, {25, 80, 2, 1, 2},
    };
    for (size_t c = 0; c < sizeof cases / sizeof cases[0]; c++) {
        uint32_t n = cases[c][0], m = cases[c][1], div = cases[c][2];
        uint32_t ell = cases[c][3], k = cases[c][4];
        uint64_t seed = 11 + c, *rp;
        uint32_t *col, *thr;
        random_graph(n, m, 1000 + c, div, &rp, &col, &thr);

        uint64_t *R1 = malloc(sizeof(uint64_t) * n * k), *R4 = malloc(sizeof(uint64_t) * n * k);
        uint64_t *RB = malloc(sizeof(uint64_t) * n * k), *reach = malloc(sizeof(uint64_t) * n);
        uint32_t *S1 = malloc(sizeof(uint32_t) * n), *S4 = malloc(sizeof(uint32_t) * n);
        uint32_t *SB = malloc(sizeof(uint32_t) * n), *nodes = malloc(sizeof(uint32_t) * n);
        or_build_counters cnt;
        if (or_build_alg2(n, rp, col, thr, seed, ell, k, 1, R1, S1, &cnt) != 0) return 1;
        if (or_build_alg2(n, rp, col, thr, seed, ell, k, 4, R4, S4, NULL) != 0) return 1;
        for (uint32_t v = 0; v < n; v++) nodes[v] = v;
        or_sketch_brute(n, rp, col, thr, seed, ell, k, nodes, n, RB, SB, reach);
        if (memcmp(R1, R4, sizeof(uint64_t) * n * k) || memcmp(S1, S4, sizeof(uint32_t) * n))
            return fail("threaded Algorithm 2", n, ell, k);
        if (memcmp(R1, RB, sizeof(uint64_t) * n * k) || memcmp(S1, SB, sizeof(uint32_t) * n))
            return fail("Algorithm 2 vs the definition", n, ell, k);

        double *est = malloc(sizeof(double) * n), *qe = malloc(sizeof(double) * n);
        double *ce = malloc(sizeof(double) * n);
        int32_t *qs = malloc(sizeof(int32_t) * n);
        uint64_t *off = malloc(sizeof(uint64_t) * (n + 1));
        for (uint32_t v = 0; v <= n; v++) off[v] = v;
        or_estimates(n, k, ell, R1, S1, est);
        or_union_query(n, k, ell, R1, S1, n, off, nodes, qe, qs);
        or_ck_query(n, k, ell, R1, S1, n, off, nodes, ce, qs);
        for (uint32_t v = 0; v < n; v++) {
            if (qe[v] != est[v]) return fail("singleton union", n, ell, k);
            double d = ce[v] - est[v];
            if (d > 1e-9 * est[v] || d < -1e-9 * est[v]) return fail("singleton CK", n, ell, k);
        }

        uint32_t s = n;
        uint32_t *seeds = malloc(sizeof(uint32_t) * s), *second = malloc(sizeof(uint32_t) * s);
        uint64_t *gain = malloc(sizeof(uint64_t) * s), *tau = malloc(sizeof(uint64_t) * s);
        or_skim_counters sc;
        if (or_skim(n, rp, col, thr, seed, ell, k, s, seeds, gain, tau, second, &sc) != 0)
            return fail("SKIM status", n, ell, k);
        uint64_t total = 0;
        for (uint32_t j = 0; j < s; j++) total += gain[j];
        if (total != (uint64_t)n * ell) return fail("SKIM gains of the full permutation", n, ell, k);

        uint32_t *pos = malloc(sizeof(uint32_t) * n * k);
        double *ice = malloc(sizeof(double) * n);
        uint64_t visits = 0;
        if (k >= 2 && or_ic_sketches(n, rp, col, thr, k, seed, pos, ice, &visits) != 0)
            return fail("IC-model sketches", n, ell, k);
        if (k >= 2) {
            double *ie = malloc(sizeof(double) * n);
            int32_t *is = malloc(sizeof(int32_t) * n);
            or_ic_union_query(n, k, pos, n, off, nodes, 0, ie, is);
            for (uint32_t v = 0; v < n; v++)
                if (ie[v] != ice[v]) return fail("IC singleton union", n, ell, k);
            or_ic_union_query(n, k, pos, n, off, nodes, 1, ie, is);
            free(ie);
            free(is);
        }
        /* structured permutation positions as ranks */
        uint64_t *ppos = malloc(sizeof(uint64_t) * n * 64);
        or_perm_positions(seed, n, ell, ppos);
        if (build_alg2(n, rp, col, thr, seed, ell, k, ppos, 3, R1, S1, NULL) != 0) return 1;
        or_sketch_brute_table(n, rp, col, thr, seed, ell, k, ppos, nodes, n, RB, SB);
        if (memcmp(R1, RB, sizeof(uint64_t) * n * k) || memcmp(S1, SB, sizeof(uint32_t) * n))
            return fail("permutation sketches vs the definition", n, ell, k);
        or_perm_estimates(n, k, ell, R1, S1, est);
        or_perm_union_query(n, k, ell, R1, S1, n, off, nodes, 0, qe, qs);
        for (uint32_t v = 0; v < n; v++)
            if (qe[v] != est[v]) return fail("permutation singleton union", n, ell, k);
        or_perm_union_query(n, k, ell, R1, S1, n, off, nodes, 1, ce, qs);
        free(ppos);

        free(R1); free(R4); free(RB); free(reach); free(S1); free(S4); free(SB); free(nodes);
        free(est); free(qe); free(ce); free(qs); free(off);
        free(seeds); free(second); free(gain); free(tau); free(pos); free(ice);
        free(rp); free(col); free(thr);
    }
    printf("sanitize_check: all oracle checks passed\n");
    return 0;
}
