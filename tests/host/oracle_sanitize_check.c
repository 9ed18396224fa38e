/* Every entry point of the CPU oracle (oracle/oracle.c) run on small graphs,
 * for a build with AddressSanitizer and UndefinedBehaviorSanitizer (the
 * sanitizers report any out-of-bounds access, use after free, leak, signed
 * overflow or misaligned access and end the process).  The graphs: K4 and
 * K5, a star, two triangles sharing an edge with a pendant vertex, an empty
 * and an edgeless graph, and seeded random graphs (n = 10..14 with brute
 * force, n = 60 and 200 without).  On every graph and mode (edges,
 * triangles; the FW iteration also over 4-cliques) the run goes through
 * listing, core numbers,
 * exact and FP64 Frank-Wolfe, sort / prefix, stable groups, the exact
 * decomposition, LDS from compact numbers, one k-core and one superlevel set.
 * Two cross-checks keep the run honest: the load numerators sum to
 * (patterns) x D_N (each pattern's shares sum to D_N), and for n <= 14 the
 * compact numbers of the decomposition equal those of brute force.
 * Prints "ok" and exits 0 when every run completes and both checks hold. */
#include "../../oracle/oracle.c"

#include <stdio.h>

/* test input only: a 64-bit linear congruential sequence (Knuth's MMIX
 * constants), high bits used */
static uint64_t lcg_state;
static uint32_t lcg_next(void) {
    lcg_state = lcg_state * 6364136223846793005ull + 1442695040888963407ull;
    return (uint32_t)(lcg_state >> 33);
}

static int failures = 0;
#define CHECK(cond, what)                                             \
    do {                                                              \
        if (!(cond)) {                                                \
            fprintf(stderr, "FAILED %s (%s:%d)\n", what, __FILE__, __LINE__); \
            ++failures;                                               \
        }                                                             \
    } while (0)

static void *xmalloc(size_t bytes) {
    void *p = malloc(bytes > 0 ? bytes : 1);
    if (!p) {
        fprintf(stderr, "out of memory\n");
        exit(2);
    }
    return p;
}

static int64_t patterns_of(const orc_graph *g, int mode) {
    if (mode == 2) return orc_graph_m(g);
    if (mode == 3) return orc_triangles(g, NULL, NULL);
    return orc_cliques4(g, NULL, NULL);
}

static void run_mode(const orc_graph *g, int mode, int iters) {
    const int64_t n = orc_graph_n(g);
    const int64_t np = patterns_of(g, mode);
    CHECK(np >= 0, "pattern count");
    uint64_t *A = (uint64_t *)xmalloc((size_t)n * sizeof(uint64_t));
    uint64_t *split = (uint64_t *)xmalloc((size_t)np * mode * sizeof(uint64_t));
    double *gap = (double *)xmalloc((size_t)iters * sizeof(double));
    double *lb = (double *)xmalloc((size_t)iters * sizeof(double));
    CHECK(orc_fw_exact(g, mode, iters, A, split, gap, lb) == 0, "fw_exact");
    u128 sum = 0;
    for (int64_t u = 0; u < n; ++u) sum += A[u];
    CHECK(sum == (u128)np * denom(mode, iters), "sum of load numerators = patterns x D");
    double *r = (double *)xmalloc((size_t)n * sizeof(double));
    double *alpha = (double *)xmalloc((size_t)np * mode * sizeof(double));
    CHECK(orc_fw_literal(g, mode, iters, r, alpha) == 0, "fw_literal");
    free(r);
    free(alpha);
    if (mode == 4) {
        free(A);
        free(split);
        free(gap);
        free(lb);
        return;
    }
    int64_t *core = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    CHECK(orc_core_numbers(g, mode, core) == 0, "core numbers");
    int32_t *order = (int32_t *)xmalloc((size_t)n * sizeof(int32_t));
    int64_t *E = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    uint8_t *inI = (uint8_t *)xmalloc((size_t)n);
    CHECK(orc_sort_prefix(g, mode, A, order, E, inI) == 0, "sort_prefix");
    int64_t ng = 0;
    int64_t *gs = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    int64_t *ge = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    int64_t *lo = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    int64_t *hi = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    CHECK(orc_extract_sg(g, mode, A, split, denom(mode, iters), &ng, gs, ge, lo, hi) == 0, "extract_sg");
    int64_t *pn = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    int64_t *pd = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    CHECK(orc_decompose(g, mode, pn, pd) >= 0, "decompose");
    int64_t *comp = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    int64_t *rn = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    int64_t *rd = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    int64_t *mv = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    CHECK(orc_lds_from_phi(g, pn, pd, comp, rn, rd, mv) >= 0, "lds_from_phi");
    uint8_t *mask = (uint8_t *)xmalloc((size_t)n);
    CHECK(orc_kcore(g, mode, 2, mask) >= 0, "kcore");
    CHECK(orc_superlevel(g, mode, 1, 1, mask) >= 0, "superlevel");
    if (n <= 14) {
        const size_t cap = (size_t)1 << n;
        int64_t *bn = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
        int64_t *bd = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
        uint32_t *masks = (uint32_t *)xmalloc(cap * sizeof(uint32_t));
        int64_t *ln = (int64_t *)xmalloc(cap * sizeof(int64_t));
        int64_t *ld = (int64_t *)xmalloc(cap * sizeof(int64_t));
        CHECK(orc_brute(g, mode, bn, bd, masks, ln, ld) >= 0, "brute");
        for (int64_t u = 0; u < n; ++u)
            CHECK((__int128)pn[u] * bd[u] == (__int128)bn[u] * pd[u], "decompose = brute force");
        free(bn);
        free(bd);
        free(masks);
        free(ln);
        free(ld);
    }
    free(A);
    free(split);
    free(gap);
    free(lb);
    free(core);
    free(order);
    free(E);
    free(inI);
    free(gs);
    free(ge);
    free(lo);
    free(hi);
    free(pn);
    free(pd);
    free(comp);
    free(rn);
    free(rd);
    free(mv);
    free(mask);
}

static void run_graph(int64_t n, int64_t np, const int32_t *s, const int32_t *d) {
    orc_graph *g = orc_graph_new(n, np, s, d);
    CHECK(g != NULL, "graph");
    if (!g) return;
    const int64_t m = orc_graph_m(g);
    int32_t *eu = (int32_t *)xmalloc((size_t)m * sizeof(int32_t));
    int32_t *ev = (int32_t *)xmalloc((size_t)m * sizeof(int32_t));
    orc_graph_edges(g, eu, ev);
    int64_t *deg = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    orc_graph_degrees(g, deg);
    const int64_t T = orc_triangles(g, NULL, NULL);
    int32_t *tri = (int32_t *)xmalloc((size_t)T * 3 * sizeof(int32_t));
    int64_t *tc = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    CHECK(orc_triangles(g, tri, tc) == T, "triangles");
    const int64_t Q = orc_cliques4(g, NULL, NULL);
    int32_t *q = (int32_t *)xmalloc((size_t)Q * 4 * sizeof(int32_t));
    int64_t *qc = (int64_t *)xmalloc((size_t)n * sizeof(int64_t));
    CHECK(orc_cliques4(g, q, qc) == Q, "4-cliques");
    run_mode(g, 2, 30);
    run_mode(g, 3, 30);
    run_mode(g, 4, 10);
    free(eu);
    free(ev);
    free(deg);
    free(tri);
    free(tc);
    free(q);
    free(qc);
    orc_graph_free(g);
}

static void run_list(int64_t n, const int32_t (*e)[2], int64_t ne) {
    int32_t *s = (int32_t *)xmalloc((size_t)ne * sizeof(int32_t));
    int32_t *d = (int32_t *)xmalloc((size_t)ne * sizeof(int32_t));
    for (int64_t i = 0; i < ne; ++i) {
        s[i] = e[i][0];
        d[i] = e[i][1];
    }
    run_graph(n, ne, s, d);
    free(s);
    free(d);
}

static void run_random(int64_t n, uint32_t p_percent, uint64_t seed) {
    lcg_state = seed;
    int64_t cap = n * (n - 1), ne = 0;
    int32_t *s = (int32_t *)xmalloc((size_t)cap * sizeof(int32_t));
    int32_t *d = (int32_t *)xmalloc((size_t)cap * sizeof(int32_t));
    for (int32_t u = 0; u < n; ++u)
        for (int32_t v = u + 1; v < n; ++v)
            if (lcg_next() % 100 < p_percent) {
                /* either orientation, and now and then the pair again the
                   other way round (ingest keeps one) */
                s[ne] = (lcg_next() & 1) ? u : v;
                d[ne] = s[ne] == u ? v : u;
                ++ne;
                if (lcg_next() % 16 == 0) {
                    s[ne] = d[ne - 1];
                    d[ne] = s[ne - 1];
                    ++ne;
                }
            }
    run_graph(n, ne, s, d);
    free(s);
    free(d);
}

int main(void) {
    static const int32_t k4[][2] = {{0, 1}, {0, 2}, {0, 3}, {1, 2}, {1, 3}, {2, 3}};
    static const int32_t k5[][2] = {{0, 1}, {0, 2}, {0, 3}, {0, 4}, {1, 2}, {1, 3}, {1, 4}, {2, 3}, {2, 4}, {3, 4}};
    static const int32_t star[][2] = {{0, 1}, {0, 2}, {0, 3}, {0, 4}, {0, 5}};
    static const int32_t bowtie[][2] = {{0, 1}, {0, 2}, {1, 2}, {1, 3}, {2, 3}, {3, 4}, {4, 4}, {2, 1}};
    run_list(4, k4, 6);
    run_list(5, k5, 10);
    run_list(6, star, 5);
    run_list(5, bowtie, 8);
    run_list(0, k4, 0);
    run_list(7, k4, 0);
    for (uint64_t seed = 1; seed <= 4; ++seed) run_random(10 + (int64_t)seed, 45, seed);
    run_random(60, 15, 99);
    run_random(200, 8, 7);
    if (failures) {
        fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    printf("ok\n");
    return 0;
}
