/*
 * CPU ORACLE for the convex-programming LDS / LTDS method (arXiv 2504.10937).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this library.  It shares no code,
 * header, table or helper with the GPU implementation; it is a plain, slow,
 * obviously-correct transcription of the paper's definitions and algorithms:
 *
 *   graph ingest ........ simple undirected graph (Section 3): self-loops and
 *                         duplicate pairs are dropped
 *   triangles ........... the set T used by Eq. (trcp) / Alg. 6 (the paper
 *                         does not say how it is listed; forward algorithm
 *                         over a degree orientation, then sorted)
 *   cliques4 ............ the 4-clique set of the h-clique program that
 *                         Eq. trcp generalises (h = 4; Section 2 / Section 6
 *                         cite the k-clique density line of work): every
 *                         4-clique once, sorted
 *   fw_exact ............ Alg. 1 (edges, Eq. cp) and Alg. 6 (triangles,
 *                         Eq. trcp) with gamma_i = 2/(i+2), decisions on the
 *                         exact rational loads r = A / D_i (A integer); the
 *                         same iteration over 4-cliques (mode 4)
 *   fw_literal .......... Alg. 1 / Alg. 6 in plain FP64 (alpha, r doubles)
 *   sort_prefix ......... Alg. 2, sort and prefix step (sort by r, prefix densities,
 *                         index set I of suffix argmaxima, ties -> larger j)
 *   extract_sg .......... Alg. 2, stable-group scan, with Def. 5 / Def. trsg
 *   decompose ........... exact compact numbers (Def. 4 / Def. trcn) via
 *                         Thm. 1 / Thm. cp: nested maximal maximisers,
 *                         Dinkelbach iteration on Goldberg-style min cuts
 *   lds_from_phi ........ LDS / LTDS sets from compact numbers (Lemmas
 *                         lds-in-phi, lds-out-phi; Thm. cnltds)
 *   brute ............... Defs. 1-4 and 7-10 by enumeration (n <= 16)
 *   kcore ............... one k-core (k-tr-core) by repeated deletion, the
 *                         bound phi(u) <= core(u) of Section 4.3 in set form
 *   superlevel .......... {u : phi(u) >= p/q} as the maximal maximiser of
 *                         q |P(U)| - p |U| (one min cut; Thm. 1 / Thm. cp)
 *
 * Readings of silent/ambiguous passages (kept identical on both sides):
 *   - FW ties (Alg. 1, Alg. 6): exact ties in r go to the endpoint with the
 *     larger original id (Alg. 1's "else" branch with edges written as
 *     (smaller id, larger id)); Alg. 6's undefined x is the argmin-r vertex.
 *   - exact arithmetic: with gamma_i = 2/(i+2) all loads share the
 *     denominator D_i = (i+1)(i+2) (edges) or 3(i+1)(i+2) (triangles); the
 *     numerators are integers: A^(i) = A^(i-1) + 2(i+1) b (edges),
 *     A^(i) = A^(i-1) + 6(i+1) b (triangles), b = units won in iteration i.
 *     For 4-cliques D_i = 2(i+1)(i+2), D_0 = 4 holds the initial quarter
 *     shares as numerator 1, and A^(i) = A^(i-1) + 4(i+1) b.
 *   - sort ties (the sort of Alg. 2): original id ascending.
 *   - restriction in ExtractSG: every pattern (edge / triangle) touching the
 *     tested group gives weight only to its vertices in the lowest group it
 *     touches; shares freed from higher vertices go to the lowest-r vertex of
 *     that lowest group.  Restrictions of accepted groups persist.  Bounds are
 *     the restricted min / max of each accepted group; an unaccepted tail gets
 *     no bounds.
 *   - LDS / LTDS of density 0 are not reported.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef unsigned __int128 u128;

/* ================================================================ graph == */
typedef struct {
    int64_t n, m;
    int32_t *eu, *ev;  /* canonical edges eu < ev, sorted lexicographically */
    int64_t *off;      /* adjacency offsets (n+1) */
    int32_t *adj;      /* neighbour ids, ascending within each vertex */
    int64_t *eid;      /* canonical edge index of each adjacency slot */
} orc_graph;

static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

void orc_graph_free(orc_graph *g) {
    if (!g) return;
    free(g->eu); free(g->ev); free(g->off); free(g->adj); free(g->eid); free(g);
}

/* Simple undirected graph from arbitrary pairs: drop self-loops, merge
 * duplicates (Section 3 assumes simple graphs).  Returns NULL on bad ids. */
orc_graph *orc_graph_new(int64_t n, int64_t npairs, const int32_t *src, const int32_t *dst) {
    if (n < 0 || npairs < 0) return NULL;
    uint64_t *key = (uint64_t *)malloc((size_t)(npairs > 0 ? npairs : 1) * sizeof(uint64_t));
    orc_graph *g = (orc_graph *)calloc(1, sizeof(orc_graph));
    if (!key || !g) { free(key); free(g); return NULL; }
    int64_t k = 0;
    for (int64_t e = 0; e < npairs; e++) {
        int64_t a = src[e], b = dst[e];
        if (a < 0 || b < 0 || a >= n || b >= n) { free(key); free(g); return NULL; }
        if (a == b) continue;
        if (a > b) { int64_t t = a; a = b; b = t; }
        key[k++] = ((uint64_t)a << 32) | (uint64_t)b;
    }
    qsort(key, (size_t)k, sizeof(uint64_t), cmp_u64);
    int64_t m = 0;
    for (int64_t i = 0; i < k; i++)
        if (i == 0 || key[i] != key[i - 1]) key[m++] = key[i];
    g->n = n;
    g->m = m;
    g->eu = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    g->ev = (int32_t *)malloc((size_t)(m > 0 ? m : 1) * sizeof(int32_t));
    g->off = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    g->adj = (int32_t *)malloc((size_t)(2 * m > 0 ? 2 * m : 1) * sizeof(int32_t));
    g->eid = (int64_t *)malloc((size_t)(2 * m > 0 ? 2 * m : 1) * sizeof(int64_t));
    if (!g->eu || !g->ev || !g->off || !g->adj || !g->eid) { free(key); orc_graph_free(g); return NULL; }
    for (int64_t e = 0; e < m; e++) {
        g->eu[e] = (int32_t)(key[e] >> 32);
        g->ev[e] = (int32_t)(key[e] & 0xffffffffu);
    }
    free(key);
    for (int64_t e = 0; e < m; e++) { g->off[g->eu[e] + 1]++; g->off[g->ev[e] + 1]++; }
    for (int64_t u = 0; u < n; u++) g->off[u + 1] += g->off[u];
    int64_t *fill = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!fill) { orc_graph_free(g); return NULL; }
    memcpy(fill, g->off, (size_t)n * sizeof(int64_t));
    /* edges are sorted by (eu, ev): scanning them in order writes each
     * adjacency list in ascending neighbour order */
    for (int64_t e = 0; e < m; e++) {
        int32_t u = g->eu[e], v = g->ev[e];
        int64_t s = fill[v]++;
        g->adj[s] = u; g->eid[s] = e;
    }
    for (int64_t e = 0; e < m; e++) {
        int32_t u = g->eu[e], v = g->ev[e];
        int64_t s = fill[u]++;
        g->adj[s] = v; g->eid[s] = e;
    }
    free(fill);
    /* lists hold smaller neighbours first (from the first pass, ascending)
     * then larger ones (second pass, ascending): already sorted */
    return g;
}

int64_t orc_graph_n(const orc_graph *g) { return g->n; }
int64_t orc_graph_m(const orc_graph *g) { return g->m; }
void orc_graph_edges(const orc_graph *g, int32_t *u, int32_t *v) {
    memcpy(u, g->eu, (size_t)g->m * sizeof(int32_t));
    memcpy(v, g->ev, (size_t)g->m * sizeof(int32_t));
}
void orc_graph_degrees(const orc_graph *g, int64_t *deg) {
    for (int64_t u = 0; u < g->n; u++) deg[u] = g->off[u + 1] - g->off[u];
}

/* ============================================================ triangles == */
typedef struct { int32_t a, b, c; } tri_t;
static int cmp_tri(const void *x, const void *y) {
    const tri_t *p = (const tri_t *)x, *q = (const tri_t *)y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    if (p->c != q->c) return p->c < q->c ? -1 : 1;
    return 0;
}

/* Orientation u -> v when (deg u, u) < (deg v, v): acyclic, so every
 * triangle is found exactly once at its lowest-ranked vertex. */
static int rank_less(const orc_graph *g, int32_t u, int32_t v) {
    int64_t du = g->off[u + 1] - g->off[u], dv = g->off[v + 1] - g->off[v];
    return du < dv || (du == dv && u < v);
}

/* Lists all triangles as ascending triples (a<b<c), sorted lexicographically.
 * Returns |T| (or -1 on allocation failure).  `tri` (3|T| ints) and `tcount`
 * (n counts) may be NULL. */
int64_t orc_triangles(const orc_graph *g, int32_t *tri, int64_t *tcount) {
    int64_t n = g->n;
    /* out-lists: neighbours of higher rank */
    int64_t *ooff = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *oadj = (int32_t *)malloc((size_t)(g->m > 0 ? g->m : 1) * sizeof(int32_t));
    uint8_t *mark = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!ooff || !oadj || !mark) { free(ooff); free(oadj); free(mark); return -1; }
    for (int32_t u = 0; u < n; u++) {
        ooff[u + 1] = ooff[u];
        for (int64_t s = g->off[u]; s < g->off[u + 1]; s++)
            if (rank_less(g, u, g->adj[s])) oadj[ooff[u + 1]++] = g->adj[s];
    }
    int64_t cnt = 0, cap = 0;
    tri_t *buf = NULL;
    if (tcount) memset(tcount, 0, (size_t)n * sizeof(int64_t));
    for (int32_t u = 0; u < n; u++) {
        for (int64_t s = ooff[u]; s < ooff[u + 1]; s++) mark[oadj[s]] = 1;
        for (int64_t s = ooff[u]; s < ooff[u + 1]; s++) {
            int32_t v = oadj[s];
            for (int64_t q = ooff[v]; q < ooff[v + 1]; q++) {
                int32_t w = oadj[q];
                if (!mark[w]) continue;
                /* triangle {u, v, w}: u -> v -> w and u -> w */
                if (tcount) { tcount[u]++; tcount[v]++; tcount[w]++; }
                if (tri) {
                    if (cnt == cap) {
                        int64_t nc = cap ? 2 * cap : 1024;
                        tri_t *nb = (tri_t *)realloc(buf, (size_t)nc * sizeof(tri_t));
                        if (!nb) { free(buf); free(mark); free(ooff); free(oadj); return -1; }
                        buf = nb; cap = nc;
                    }
                    int32_t x[3] = {u, v, w};
                    for (int i = 0; i < 3; i++)
                        for (int j = i + 1; j < 3; j++)
                            if (x[j] < x[i]) { int32_t t = x[i]; x[i] = x[j]; x[j] = t; }
                    buf[cnt].a = x[0]; buf[cnt].b = x[1]; buf[cnt].c = x[2];
                }
                cnt++;
            }
        }
        for (int64_t s = ooff[u]; s < ooff[u + 1]; s++) mark[oadj[s]] = 0;
    }
    free(mark); free(ooff); free(oadj);
    if (tri) {
        if (cnt > 0) qsort(buf, (size_t)cnt, sizeof(tri_t), cmp_tri); /* buf is NULL without triangles */
        for (int64_t t = 0; t < cnt; t++) {
            tri[3 * t] = buf[t].a; tri[3 * t + 1] = buf[t].b; tri[3 * t + 2] = buf[t].c;
        }
        free(buf);
    }
    return cnt;
}

/* ============================================================ 4-cliques == */
static int adjacent(const orc_graph *g, int32_t u, int32_t v) {
    int64_t lo = g->off[u], hi = g->off[u + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) / 2;
        if (g->adj[mid] < v) lo = mid + 1; else hi = mid;
    }
    return lo < g->off[u + 1] && g->adj[lo] == v;
}

/* Lists all 4-cliques as ascending quadruples (a<b<c<d), sorted
 * lexicographically: every triangle a<b<c (sorted) is extended by each
 * d > c adjacent to a, b and c, in ascending order of d, so each 4-clique
 * appears once, from its three smallest vertices.  Returns the count (or -1).
 * `q` (4 per clique) and `qcount` (n) may be NULL. */
int64_t orc_cliques4(const orc_graph *g, int32_t *q, int64_t *qcount) {
    int64_t T = orc_triangles(g, NULL, NULL);
    if (T < 0) return -1;
    int32_t *tri = (int32_t *)malloc((size_t)(3 * T > 0 ? 3 * T : 1) * sizeof(int32_t));
    if (!tri) return -1;
    if (orc_triangles(g, tri, NULL) != T) { free(tri); return -1; }
    if (qcount) memset(qcount, 0, (size_t)g->n * sizeof(int64_t));
    int64_t cnt = 0;
    for (int64_t t = 0; t < T; t++) {
        int32_t a = tri[3 * t], b = tri[3 * t + 1], c = tri[3 * t + 2];
        for (int64_t s = g->off[c]; s < g->off[c + 1]; s++) {
            int32_t d = g->adj[s];
            if (d <= c || !adjacent(g, a, d) || !adjacent(g, b, d)) continue;
            if (q) { q[4 * cnt] = a; q[4 * cnt + 1] = b; q[4 * cnt + 2] = c; q[4 * cnt + 3] = d; }
            if (qcount) { qcount[a]++; qcount[b]++; qcount[c]++; qcount[d]++; }
            cnt++;
        }
    }
    free(tri);
    return cnt;
}

/* patterns (edges, triangles or 4-cliques) as flat vertex tuples */
typedef struct { int h; int64_t np; int32_t *v; } patterns;
static int get_patterns(const orc_graph *g, int mode, patterns *P) {
    P->h = mode;
    if (mode == 2) {
        P->np = g->m;
        P->v = (int32_t *)malloc((size_t)(2 * g->m > 0 ? 2 * g->m : 1) * sizeof(int32_t));
        if (!P->v) return -1;
        for (int64_t e = 0; e < g->m; e++) { P->v[2 * e] = g->eu[e]; P->v[2 * e + 1] = g->ev[e]; }
        return 0;
    }
    if (mode == 3) {
        int64_t T = orc_triangles(g, NULL, NULL);
        if (T < 0) return -1;
        P->np = T;
        P->v = (int32_t *)malloc((size_t)(3 * T > 0 ? 3 * T : 1) * sizeof(int32_t));
        if (!P->v) return -1;
        if (orc_triangles(g, P->v, NULL) != T) { free(P->v); return -1; }
        return 0;
    }
    if (mode == 4) {
        int64_t Q = orc_cliques4(g, NULL, NULL);
        if (Q < 0) return -1;
        P->np = Q;
        P->v = (int32_t *)malloc((size_t)(4 * Q > 0 ? 4 * Q : 1) * sizeof(int32_t));
        if (!P->v) return -1;
        if (orc_cliques4(g, P->v, NULL) != Q) { free(P->v); return -1; }
        return 0;
    }
    return -1;
}

/* ====================================================== core numbers == */
/* Core numbers (edges) and tr-core numbers (triangles), used by Pruning
 * (Alg. 3) and as the initial bounds of the compact numbers: core(u) is the
 * largest k such that u belongs to the k-core, the largest vertex set in
 * which every vertex lies in at least k patterns (edges or triangles) whose
 * vertices are all in the set.  The k-cores are nested, so the k-core is
 * obtained from the (k-1)-core by deleting, until none is left, vertices
 * that lie in fewer than k patterns of the remaining set (counted afresh on
 * every pass).  core[u] = 0 for vertices outside the 1-core.  Returns 0, or -1. */
int orc_core_numbers(const orc_graph *g, int mode, int64_t *core) {
    patterns P;
    if (get_patterns(g, mode, &P)) return -1;
    const int64_t n = g->n, h = P.h;
    char *in = (char *)malloc((size_t)(n > 0 ? n : 1));
    int64_t *cnt = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!in || !cnt) { free(in); free(cnt); free(P.v); return -1; }
    for (int64_t u = 0; u < n; u++) { in[u] = 1; core[u] = 0; }
    int64_t left = n;
    for (int64_t k = 1; left > 0; k++) {
        int changed = 1;
        while (changed) {
            changed = 0;
            for (int64_t u = 0; u < n; u++) cnt[u] = 0;
            for (int64_t p = 0; p < P.np; p++) {
                int all = 1;
                for (int64_t j = 0; j < h; j++) all = all && in[P.v[h * p + j]];
                if (all)
                    for (int64_t j = 0; j < h; j++) cnt[P.v[h * p + j]]++;
            }
            for (int64_t u = 0; u < n; u++)
                if (in[u] && cnt[u] < k) { in[u] = 0; left--; changed = 1; }
        }
        for (int64_t u = 0; u < n; u++)
            if (in[u]) core[u] = k;
    }
    free(in); free(cnt); free(P.v);
    return 0;
}

/* ============================================================ FW exact == */
/* Denominator of the loads after iteration i (exact form of gamma_i =
 * 2/(i+2)): (i+1)(i+2) for edges, 3(i+1)(i+2) for triangles, 2(i+1)(i+2)
 * for 4-cliques (D_0 = 2, 6, 4: the initial 1/h shares are integers). */
static uint64_t denom(int mode, int64_t i) {
    const uint64_t c = mode == 3 ? 3 : (mode == 4 ? 2 : 1);
    return c * (uint64_t)(i + 1) * (uint64_t)(i + 2);
}

/* Alg. 1 / Alg. 6 (and the 4-clique iteration, mode 4).  Outputs after
 * `iters` iterations:
 *   A[u]      numerator of r_u (r_u = A[u] / D_iters)
 *   split[h*p+j] numerator of alpha_{x_j, p} for pattern p's j-th vertex
 *             (patterns in canonical order: edges (u<v) sorted, triangles
 *             (a<b<c) and 4-cliques (a<b<c<d) sorted); the h numerators of
 *             a pattern sum to D_iters
 *   gap[i-1]  FW duality gap at r^(i-1): 2 (sum r^2 - sum_p min_{x in p} r_x)
 *   lb[i-1]   the matching lower bound on the optimum, sum r^2 - gap
 * Any output pointer may be NULL.  Returns 0, or -1 (allocation / mode). */
int orc_fw_exact(const orc_graph *g, int mode, int iters, uint64_t *A_out, uint64_t *split_out,
                 double *gap_out, double *lb_out) {
    patterns P;
    if ((mode < 2 || mode > 4) || iters < 0 || get_patterns(g, mode, &P)) return -1;
    int h = P.h;
    int64_t n = g->n, np = P.np;
    uint64_t *A = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    uint64_t *b = (uint64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint64_t));
    uint64_t *sp = (uint64_t *)malloc((size_t)(h * np > 0 ? h * np : 1) * sizeof(uint64_t));
    if (!A || !b || !sp) { free(A); free(b); free(sp); free(P.v); return -1; }
    /* initial split: 1/h of each pattern to each vertex; D_0 = 2 (edges), 6
     * (triangles) or 4 (4-cliques), so the numerator is D_0 / h = 1, 2 or 1 */
    uint64_t a0 = denom(mode, 0) / (uint64_t)h;
    for (int64_t p = 0; p < np; p++)
        for (int j = 0; j < h; j++) { sp[h * p + j] = a0; A[P.v[h * p + j]] += a0; }
    for (int64_t i = 1; i <= iters; i++) {
        uint64_t Dprev = denom(mode, i - 1);
        uint64_t inc = denom(mode, i) - Dprev; /* 2(i+1), 6(i+1) or 4(i+1) */
        memset(b, 0, (size_t)n * sizeof(uint64_t));
        u128 summin = 0;
        for (int64_t p = 0; p < np; p++) {
            /* the vertex with the smallest r^(i-1) receives the unit;
             * ties -> larger original id */
            int best = 0;
            for (int j = 1; j < h; j++) {
                int32_t x = P.v[h * p + j], y = P.v[h * p + best];
                if (A[x] < A[y] || (A[x] == A[y] && x > y)) best = j;
            }
            int32_t w = P.v[h * p + best];
            b[w]++;
            summin += A[w];
            sp[h * p + best] += inc;
        }
        if (gap_out || lb_out) {
            u128 sq = 0;
            for (int64_t u = 0; u < n; u++) sq += (u128)A[u] * A[u];
            /* with D = D_{i-1}:  (D^2 / 2) g = sum A^2 - D sum_p min A  (exact,
             * non-negative since min <= every split-weighted average) */
            u128 num = sq - (u128)Dprev * summin;
            long double D = (long double)Dprev;
            long double gap = 2.0L * (long double)num / (D * D);
            long double S2 = (long double)sq / (D * D);
            if (gap_out) gap_out[i - 1] = (double)gap;
            if (lb_out) lb_out[i - 1] = (double)(S2 - gap);
        }
        for (int64_t u = 0; u < n; u++) A[u] += inc * b[u];
    }
    if (A_out) memcpy(A_out, A, (size_t)n * sizeof(uint64_t));
    if (split_out) memcpy(split_out, sp, (size_t)(h * np) * sizeof(uint64_t));
    free(A); free(b); free(sp); free(P.v);
    return 0;
}

/* ========================================================== FW literal == */
/* Alg. 1 / Alg. 6 exactly as printed, in FP64: alpha^(i) =
 * (1-gamma) alpha^(i-1) + gamma alpha_hat, r = sum alpha.  Decisions on the
 * FP64 loads (ties -> larger original id).  Outputs r (n) and alpha (h*np). */
int orc_fw_literal(const orc_graph *g, int mode, int iters, double *r_out, double *alpha_out) {
    patterns P;
    if ((mode < 2 || mode > 4) || iters < 0 || get_patterns(g, mode, &P)) return -1;
    int h = P.h;
    int64_t n = g->n, np = P.np;
    double *r = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *al = (double *)malloc((size_t)(h * np > 0 ? h * np : 1) * sizeof(double));
    int *win = (int *)malloc((size_t)(np > 0 ? np : 1) * sizeof(int));
    if (!r || !al || !win) { free(r); free(al); free(win); free(P.v); return -1; }
    for (int64_t p = 0; p < np; p++)
        for (int j = 0; j < h; j++) al[h * p + j] = 1.0 / h;
    for (int64_t p = 0; p < np; p++)
        for (int j = 0; j < h; j++) r[P.v[h * p + j]] += al[h * p + j];
    for (int64_t i = 1; i <= iters; i++) {
        double gam = 2.0 / (double)(i + 2);
        for (int64_t p = 0; p < np; p++) {
            int best = 0;
            for (int j = 1; j < h; j++) {
                int32_t x = P.v[h * p + j], y = P.v[h * p + best];
                if (r[x] < r[y] || (r[x] == r[y] && x > y)) best = j;
            }
            win[p] = best;
        }
        for (int64_t p = 0; p < np; p++)
            for (int j = 0; j < h; j++)
                al[h * p + j] = (1.0 - gam) * al[h * p + j] + gam * (j == win[p] ? 1.0 : 0.0);
        memset(r, 0, (size_t)n * sizeof(double));
        for (int64_t p = 0; p < np; p++)
            for (int j = 0; j < h; j++) r[P.v[h * p + j]] += al[h * p + j];
    }
    if (r_out) memcpy(r_out, r, (size_t)n * sizeof(double));
    if (alpha_out) memcpy(alpha_out, al, (size_t)(h * np) * sizeof(double));
    free(r); free(al); free(win); free(P.v);
    return 0;
}

/* ======================================================== sort / prefix == */
static const uint64_t *g_sortA;
static int cmp_rdesc(const void *x, const void *y) {
    int32_t a = *(const int32_t *)x, b = *(const int32_t *)y;
    if (g_sortA[a] != g_sortA[b]) return g_sortA[a] > g_sortA[b] ? -1 : 1;
    return (a > b) - (a < b);
}

/* Alg. 2: sort by r and prefix densities.  order[j] = vertex at 0-based position j (r descending,
 * ties: original id ascending).  E[j] = number of patterns whose vertices all
 * lie in the first j+1 positions (edge count of G[V[1:j+1]], or triangle
 * count).  inI[j] = 1 iff position j+1 (1-based) is argmax_{k >= j+1} of
 * E_k / k with ties to the larger k, i.e. a strict suffix maximum. */
int orc_sort_prefix(const orc_graph *g, int mode, const uint64_t *A, int32_t *order, int64_t *E,
                    uint8_t *inI) {
    patterns P;
    if ((mode != 2 && mode != 3) || get_patterns(g, mode, &P)) return -1;
    int64_t n = g->n;
    int32_t *ord = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t *pos = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *c = (int64_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(int64_t));
    if (!ord || !pos || !c) { free(ord); free(pos); free(c); free(P.v); return -1; }
    for (int64_t u = 0; u < n; u++) ord[u] = (int32_t)u;
    g_sortA = A;
    qsort(ord, (size_t)n, sizeof(int32_t), cmp_rdesc);
    for (int64_t j = 0; j < n; j++) pos[ord[j]] = j;
    for (int64_t p = 0; p < P.np; p++) {
        int64_t last = -1;
        for (int j = 0; j < P.h; j++) if (pos[P.v[P.h * p + j]] > last) last = pos[P.v[P.h * p + j]];
        c[last]++;
    }
    int64_t run = 0;
    for (int64_t j = 0; j < n; j++) { run += c[j]; c[j] = run; }
    /* backwards: best suffix density so far as a fraction bestE / bestK */
    int64_t bestE = 0, bestK = 0;
    for (int64_t j = n - 1; j >= 0; j--) {
        int64_t k = j + 1;
        int in = 0;
        if (bestK == 0) in = 1;
        else if ((__int128)c[j] * bestK > (__int128)bestE * k) in = 1;
        if (in) { bestE = c[j]; bestK = k; }
        if (inI) inI[j] = (uint8_t)in;
    }
    if (order) memcpy(order, ord, (size_t)n * sizeof(int32_t));
    if (E) memcpy(E, c, (size_t)n * sizeof(int64_t));
    free(ord); free(pos); free(c); free(P.v);
    return 0;
}

/* =========================================================== extract_sg == */
/* Alg. 2 with Def. 5 (edges) / Def. trsg (triangles) under the restriction
 * reading stated in the file header.  Inputs: loads A (numerators over
 * D = D_iters), pattern splits (as produced by orc_fw_exact), D.
 * Outputs:
 *   ngroups            number of accepted stable groups
 *   gstart[k], gend[k] 0-based position range [start, end) of group k in the
 *                      sorted order (orc_sort_prefix), top group first
 *   lo[u], hi[u]       restricted min / max numerator of u's group (over D);
 *                      -1 when u lies in the unaccepted tail
 * gstart/gend need room for n entries.  Returns 0 or -1. */
int orc_extract_sg(const orc_graph *g, int mode, const uint64_t *A, const uint64_t *split, uint64_t D,
                   int64_t *ngroups, int64_t *gstart, int64_t *gend, int64_t *lo, int64_t *hi) {
    patterns P;
    if ((mode != 2 && mode != 3) || get_patterns(g, mode, &P)) return -1;
    int h = P.h;
    int64_t n = g->n, np = P.np;
    int32_t *ord = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t *pos = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *E = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    uint8_t *inI = (uint8_t *)malloc((size_t)(n > 0 ? n : 1));
    int64_t *grp = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *rp = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int ok = ord && pos && E && inI && grp && rp;
    if (!ok || orc_sort_prefix(g, mode, A, ord, E, inI)) {
        free(ord); free(pos); free(E); free(inI); free(grp); free(rp); free(P.v);
        return -1;
    }
    for (int64_t j = 0; j < n; j++) pos[ord[j]] = j;
    for (int64_t u = 0; u < n; u++) { lo[u] = -1; hi[u] = -1; }
    int64_t ng = 0, S0 = 0; /* pending group starts at position S0 */
    int64_t minH = -1;      /* min restricted load of the last accepted group */
    /* group rank of a vertex at position x when testing [S0, S1):
     * accepted groups keep their index (0..ng-1), S gets ng, L gets ng+1 */
    for (int64_t j = 0; j < n; j++) {
        if (!inI[j]) continue;
        int64_t S1 = j + 1;
        for (int64_t x = S0; x < n; x++) grp[ord[x]] = (x < S1) ? ng : ng + 1;
        for (int64_t x = S0; x < n; x++) rp[ord[x]] = 0;
        for (int64_t p = 0; p < np; p++) {
            const int32_t *vv = P.v + h * p;
            const uint64_t *aa = split + h * p;
            int64_t gl = -1;
            for (int q = 0; q < h; q++) if (grp[vv[q]] > gl) gl = grp[vv[q]];
            if (gl < ng) continue; /* pattern inside accepted groups: final */
            int64_t freed = 0;
            int recv = -1;
            for (int q = 0; q < h; q++) {
                if (grp[vv[q]] < gl) freed += (int64_t)aa[q];
                else if (recv < 0 || pos[vv[q]] > pos[vv[recv]]) recv = q;
            }
            for (int q = 0; q < h; q++)
                if (grp[vv[q]] == gl) rp[vv[q]] += (int64_t)aa[q] + (q == recv ? freed : 0);
        }
        int64_t mnS = INT64_MAX, mxS = -1, mxL = -1;
        for (int64_t x = S0; x < n; x++) {
            int64_t v = rp[ord[x]];
            if (x < S1) { if (v < mnS) mnS = v; if (v > mxS) mxS = v; }
            else if (v > mxL) mxL = v;
        }
        int accept = 1;
        if (ng > 0 && !(mxS < minH)) accept = 0;
        if (S1 < n && !(mxL < mnS)) accept = 0;
        if (accept) {
            for (int64_t x = S0; x < S1; x++) {
                grp[ord[x]] = ng;
                lo[ord[x]] = mnS;
                hi[ord[x]] = mxS;
            }
            gstart[ng] = S0; gend[ng] = S1;
            ng++;
            minH = mnS;
            S0 = S1;
        }
    }
    *ngroups = ng;
    (void)D;
    free(ord); free(pos); free(E); free(inI); free(grp); free(rp); free(P.v);
    return 0;
}

/* ============================================================ max-flow == */
/* Dinic's algorithm on an explicit residual graph with int64 capacities. */
typedef struct {
    int64_t nn, na, cap_a;
    int64_t *head, *nxt, *to, *cap; /* arcs in pairs (a, a^1) */
    int64_t *level, *it, *queue;
} flownet;

static int fn_init(flownet *f, int64_t nn, int64_t arcs_hint) {
    memset(f, 0, sizeof(*f));
    f->nn = nn;
    f->head = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
    f->level = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
    f->it = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
    f->queue = (int64_t *)malloc((size_t)nn * sizeof(int64_t));
    f->cap_a = arcs_hint > 16 ? arcs_hint : 16;
    f->nxt = (int64_t *)malloc((size_t)f->cap_a * sizeof(int64_t));
    f->to = (int64_t *)malloc((size_t)f->cap_a * sizeof(int64_t));
    f->cap = (int64_t *)malloc((size_t)f->cap_a * sizeof(int64_t));
    if (!f->head || !f->level || !f->it || !f->queue || !f->nxt || !f->to || !f->cap) return -1;
    for (int64_t i = 0; i < nn; i++) f->head[i] = -1;
    return 0;
}
static void fn_free(flownet *f) {
    free(f->head); free(f->level); free(f->it); free(f->queue);
    free(f->nxt); free(f->to); free(f->cap);
}
static int fn_arc1(flownet *f, int64_t a, int64_t b, int64_t c) {
    if (f->na == f->cap_a) {
        int64_t nc = f->cap_a * 2;
        int64_t *x = (int64_t *)realloc(f->nxt, (size_t)nc * sizeof(int64_t));
        if (!x) return -1;
        f->nxt = x;
        x = (int64_t *)realloc(f->to, (size_t)nc * sizeof(int64_t));
        if (!x) return -1;
        f->to = x;
        x = (int64_t *)realloc(f->cap, (size_t)nc * sizeof(int64_t));
        if (!x) return -1;
        f->cap = x;
        f->cap_a = nc;
    }
    f->to[f->na] = b; f->cap[f->na] = c; f->nxt[f->na] = f->head[a]; f->head[a] = f->na; f->na++;
    return 0;
}
static int fn_arc(flownet *f, int64_t a, int64_t b, int64_t c) {
    return fn_arc1(f, a, b, c) || fn_arc1(f, b, a, 0);
}
static int fn_bfs(flownet *f, int64_t s, int64_t t) {
    for (int64_t i = 0; i < f->nn; i++) f->level[i] = -1;
    int64_t qh = 0, qt = 0;
    f->level[s] = 0; f->queue[qt++] = s;
    while (qh < qt) {
        int64_t x = f->queue[qh++];
        for (int64_t a = f->head[x]; a >= 0; a = f->nxt[a])
            if (f->cap[a] > 0 && f->level[f->to[a]] < 0) {
                f->level[f->to[a]] = f->level[x] + 1;
                f->queue[qt++] = f->to[a];
            }
    }
    return f->level[t] >= 0;
}
/* iterative DFS for one augmenting path within the level graph */
static int64_t fn_dfs(flownet *f, int64_t s, int64_t t, int64_t *stk_node, int64_t *stk_arc) {
    int64_t top = 0;
    stk_node[0] = s;
    for (;;) {
        int64_t x = stk_node[top];
        if (x == t) {
            int64_t push = INT64_MAX;
            for (int64_t k = 0; k < top; k++) if (f->cap[stk_arc[k]] < push) push = f->cap[stk_arc[k]];
            for (int64_t k = 0; k < top; k++) { f->cap[stk_arc[k]] -= push; f->cap[stk_arc[k] ^ 1] += push; }
            return push;
        }
        int advanced = 0;
        for (; f->it[x] >= 0; f->it[x] = f->nxt[f->it[x]]) {
            int64_t a = f->it[x], y = f->to[a];
            if (f->cap[a] > 0 && f->level[y] == f->level[x] + 1) {
                stk_arc[top] = a;
                stk_node[++top] = y;
                advanced = 1;
                break;
            }
        }
        if (!advanced) {
            if (top == 0) return 0;
            f->level[x] = -1; /* dead end */
            top--;
            int64_t px = stk_node[top];
            f->it[px] = f->nxt[f->it[px]];
        }
    }
}
static int64_t fn_maxflow(flownet *f, int64_t s, int64_t t) {
    int64_t flow = 0;
    int64_t *sn = (int64_t *)malloc((size_t)(f->nn + 1) * sizeof(int64_t));
    int64_t *sa = (int64_t *)malloc((size_t)(f->nn + 1) * sizeof(int64_t));
    if (!sn || !sa) { free(sn); free(sa); return -1; }
    while (fn_bfs(f, s, t)) {
        for (int64_t i = 0; i < f->nn; i++) f->it[i] = f->head[i];
        int64_t pushed;
        while ((pushed = fn_dfs(f, s, t, sn, sa)) > 0) flow += pushed;
    }
    free(sn); free(sa);
    return flow;
}
/* maximal source side of a min cut: nodes that cannot reach t in the
 * residual graph */
static void fn_maximal_source_side(flownet *f, int64_t t, uint8_t *src_side) {
    /* reverse BFS from t over arcs with residual capacity (x -> y with cap>0
     * means x can reach y) */
    for (int64_t i = 0; i < f->nn; i++) { src_side[i] = 1; f->level[i] = -1; }
    int64_t qh = 0, qt = 0;
    f->level[t] = 0; f->queue[qt++] = t; src_side[t] = 0;
    while (qh < qt) {
        int64_t y = f->queue[qh++];
        for (int64_t a = f->head[y]; a >= 0; a = f->nxt[a]) {
            /* arc a: y -> x ; its twin a^1: x -> y */
            int64_t x = f->to[a];
            if (f->cap[a ^ 1] > 0 && f->level[x] < 0) {
                f->level[x] = 0; src_side[x] = 0; f->queue[qt++] = x;
            }
        }
    }
}

/* ===================================================== exact decompose == */
/* max over U with B ⊆ U of  q*(|P(U)| - |P(B)|) - p*(|U| - |B|), where P(U)
 * are the patterns (edges/triangles) inside U.  Returns the maximal
 * maximiser in `inU` (which always contains B) and its pattern gain and size
 * gain.  Network: s -> pattern (cap q), pattern -> each vertex of it outside
 * B (infinite), vertex outside B -> t (cap p); patterns with all vertices in
 * B are left out (they are in P(B)). */
static int best_superset(const orc_graph *g, const patterns *P, const uint8_t *inB, int64_t p, int64_t q,
                         uint8_t *inU, int64_t *dpat, int64_t *dsize) {
    int64_t n = g->n, h = P->h;
    int64_t s = P->np + n, t = s + 1;
    flownet f;
    if (fn_init(&f, P->np + n + 2, 4 * P->np + 2 * n + 16)) { fn_free(&f); return -1; }
    const int64_t INF = INT64_MAX / 4;
    for (int64_t k = 0; k < P->np; k++) {
        int outside = 0;
        for (int j = 0; j < h; j++) if (!inB[P->v[h * k + j]]) outside = 1;
        if (!outside) continue;
        if (fn_arc(&f, s, k, q)) { fn_free(&f); return -1; }
        for (int j = 0; j < h; j++) {
            int32_t x = P->v[h * k + j];
            if (!inB[x] && fn_arc(&f, k, P->np + x, INF)) { fn_free(&f); return -1; }
        }
    }
    for (int64_t x = 0; x < n; x++)
        if (!inB[x] && fn_arc(&f, P->np + x, t, p)) { fn_free(&f); return -1; }
    if (fn_maxflow(&f, s, t) < 0) { fn_free(&f); return -1; }
    uint8_t *side = (uint8_t *)malloc((size_t)f.nn);
    if (!side) { fn_free(&f); return -1; }
    fn_maximal_source_side(&f, t, side);
    int64_t dp = 0, ds = 0;
    for (int64_t x = 0; x < n; x++) {
        inU[x] = inB[x] || side[P->np + x];
        if (!inB[x] && inU[x]) ds++;
    }
    for (int64_t k = 0; k < P->np; k++) {
        int all = 1, outside = 0;
        for (int j = 0; j < h; j++) {
            if (!inU[P->v[h * k + j]]) all = 0;
            if (!inB[P->v[h * k + j]]) outside = 1;
        }
        if (all && outside) dp++;
    }
    free(side);
    fn_free(&f);
    *dpat = dp; *dsize = ds;
    return 0;
}

static int64_t gcd64(int64_t a, int64_t b) {
    while (b) { int64_t t = a % b; a = b; b = t; }
    return a < 0 ? -a : a;
}

/* Exact compact numbers (Def. 4, Def. trcn) as reduced fractions.
 * By Thm. 1 / Thm. cp they equal r* of Eq. (cp) / Eq. (trcp), whose level
 * sets are nested: the top level B_1 is the maximal set of maximum
 * density, and each next level adds the maximal U ⊋ B maximising
 * (|P(U)| - |P(B)|) / (|U| - |B|).  Each level is found by Dinkelbach
 * iteration, each step one min cut.  Isolated / pattern-free vertices end
 * with phi = 0.  Returns the number of levels, or -1. */
int64_t orc_decompose(const orc_graph *g, int mode, int64_t *phi_num, int64_t *phi_den) {
    patterns P;
    if ((mode != 2 && mode != 3) || get_patterns(g, mode, &P)) return -1;
    int64_t n = g->n;
    uint8_t *inB = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    uint8_t *inU = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!inB || !inU) { free(inB); free(inU); free(P.v); return -1; }
    int64_t sizeB = 0, patB = 0, levels = 0;
    while (sizeB < n) {
        /* start from U = V */
        int64_t num = P.np - patB, den = n - sizeB;
        for (;;) {
            int64_t dp, ds;
            int64_t gg = gcd64(num, den);
            int64_t pp = gg ? num / gg : 0, qq = gg ? den / gg : 1;
            if (best_superset(g, &P, inB, pp, qq, inU, &dp, &ds)) { free(inB); free(inU); free(P.v); return -1; }
            /* value of the maximiser at lambda = num/den */
            __int128 val = (__int128)qq * dp - (__int128)pp * ds;
            if (val > 0 && ds > 0) { num = dp; den = ds; continue; }
            /* lambda optimal; the maximal maximiser has value 0 */
            if (ds == 0) {
                /* no strict superset reaches lambda: happens only when the
                 * remaining vertices carry no pattern (lambda = 0) */
                for (int64_t x = 0; x < n; x++) inU[x] = 1;
                ds = n - sizeB; dp = P.np - patB; num = 0; den = 1;
            }
            int64_t g2 = gcd64(num, den);
            int64_t rn = g2 ? num / g2 : 0, rd = g2 ? den / g2 : 1;
            for (int64_t x = 0; x < n; x++)
                if (inU[x] && !inB[x]) { phi_num[x] = rn; phi_den[x] = rd; inB[x] = 1; }
            sizeB += ds; patB += dp; levels++;
            break;
        }
    }
    free(inB); free(inU); free(P.v);
    return levels;
}

/* ================================================ large-graph helpers == */
/* The k-core (mode 2) or k-tr-core (mode 3): the largest vertex set in which
 * every vertex lies in at least k patterns (edges / triangles) whose
 * vertices are all in the set, as used by Pruning (Alg. 3) and the bounds of
 * Section 4.3.  Obtained from V by deleting, one at a time until none is
 * left, a vertex that lies in fewer than k patterns of the remaining set;
 * a deletion removes every pattern through the vertex.  The result does not
 * depend on the deletion order (the k-core is the union of all vertex sets
 * with that property).  A vertex u with phi(u) >= rho > 0 lies in a
 * rho-compact set, where it has at least rho patterns (removing u alone
 * loses at least rho), so it lies in the ceil(rho)-core: the k-core holds
 * {u : phi(u) >= lambda} for k = ceil(lambda).  in_core[u] = 1 inside.
 * Returns the core size, or -1. */
int64_t orc_kcore(const orc_graph *g, int mode, int64_t k, uint8_t *in_core) {
    patterns P;
    if ((mode != 2 && mode != 3) || get_patterns(g, mode, &P)) return -1;
    const int64_t n = g->n, h = P.h, np = P.np;
    /* patterns through each vertex (CSR) */
    int64_t *cnt = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *po = (int64_t *)calloc((size_t)(n + 1), sizeof(int64_t));
    int64_t *pl = (int64_t *)malloc((size_t)(h * np > 0 ? h * np : 1) * sizeof(int64_t));
    uint8_t *palive = (uint8_t *)malloc((size_t)(np > 0 ? np : 1));
    int64_t *queue = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    uint8_t *queued = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!cnt || !po || !pl || !palive || !queue || !queued) {
        free(cnt); free(po); free(pl); free(palive); free(queue); free(queued); free(P.v);
        return -1;
    }
    for (int64_t p = 0; p < h * np; p++) po[P.v[p] + 1]++;
    for (int64_t u = 0; u < n; u++) po[u + 1] += po[u];
    for (int64_t p = 0; p < np; p++) {
        palive[p] = 1;
        for (int64_t j = 0; j < h; j++) {
            const int32_t x = P.v[h * p + j];
            pl[po[x] + cnt[x]] = p;
            cnt[x]++;
        }
    }
    int64_t qh = 0, qt = 0;
    for (int64_t u = 0; u < n; u++) {
        in_core[u] = 1;
        if (cnt[u] < k) { queue[qt++] = u; queued[u] = 1; }
    }
    int64_t left = n;
    while (qh < qt) {
        const int64_t u = queue[qh++];
        in_core[u] = 0;
        left--;
        for (int64_t e = po[u]; e < po[u + 1]; e++) {
            const int64_t p = pl[e];
            if (!palive[p]) continue;
            palive[p] = 0;
            for (int64_t j = 0; j < h; j++) {
                const int32_t w = P.v[h * p + j];
                if (w == u) continue;
                cnt[w]--;
                if (!queued[w] && cnt[w] < k) { queue[qt++] = w; queued[w] = 1; }
            }
        }
    }
    free(cnt); free(po); free(pl); free(palive); free(queue); free(queued); free(P.v);
    return left;
}

/* {u : phi(u) >= p/q} (p >= 0, q >= 1): the maximal maximiser of
 * q |P(U)| - p |U| over all vertex sets U.  By Thm. 1 / Thm. cp the compact
 * numbers are the levels of the nested maximal maximisers found by
 * orc_decompose; at lambda = p/q every level with density >= lambda adds a
 * non-negative amount and every lower level a negative one, so the maximal
 * maximiser is the union of the levels with density >= lambda.  One min cut
 * (best_superset with B empty).  Returns |U|, or -1. */
int64_t orc_superlevel(const orc_graph *g, int mode, int64_t p, int64_t q, uint8_t *inU) {
    patterns P;
    if ((mode != 2 && mode != 3) || p < 0 || q < 1 || get_patterns(g, mode, &P)) return -1;
    const int64_t n = g->n;
    uint8_t *inB = (uint8_t *)calloc((size_t)(n > 0 ? n : 1), 1);
    if (!inB) { free(P.v); return -1; }
    int64_t dp = 0, ds = 0;
    const int rc = best_superset(g, &P, inB, p, q, inU, &dp, &ds);
    free(inB); free(P.v);
    return rc ? -1 : ds;
}

/* LDS (mode 2) / LTDS (mode 3) from exact compact numbers: the connected
 * components C of G[{u : phi(u) = rho}] none of whose neighbours has
 * phi > rho (Lemmas lds-in-phi, lds-out-phi; Thm. cnltds), rho > 0.
 * comp[u] = index of u's LDS or -1; rho_num/rho_den per LDS.  Returns the
 * number of LDSs; LDS indices are sorted by (rho desc, min vertex id asc). */
int64_t orc_lds_from_phi(const orc_graph *g, const int64_t *pn, const int64_t *pd, int64_t *comp,
                         int64_t *rho_num, int64_t *rho_den, int64_t *minv) {
    int64_t n = g->n;
    int64_t *lab = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    int64_t *queue = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!lab || !queue) { free(lab); free(queue); return -1; }
    for (int64_t u = 0; u < n; u++) { lab[u] = -1; comp[u] = -1; }
    int64_t nc = 0;
    int64_t *tmpn = NULL, *tmpd = NULL, *tmpm = NULL;
    for (int64_t u0 = 0; u0 < n; u0++) {
        if (lab[u0] >= 0 || pn[u0] == 0) continue;
        /* BFS over neighbours with equal phi */
        int64_t qh = 0, qt = 0, good = 1, mv = u0;
        lab[u0] = u0; queue[qt++] = u0;
        while (qh < qt) {
            int64_t x = queue[qh++];
            if (x < mv) mv = x;
            for (int64_t s = g->off[x]; s < g->off[x + 1]; s++) {
                int32_t y = g->adj[s];
                __int128 l = (__int128)pn[y] * pd[x], r = (__int128)pn[x] * pd[y];
                if (l > r) good = 0;
                else if (l == r && lab[y] < 0) { lab[y] = u0; queue[qt++] = y; }
            }
        }
        if (!good) continue;
        int64_t *a = (int64_t *)realloc(tmpn, (size_t)(nc + 1) * sizeof(int64_t));
        int64_t *b = a ? (int64_t *)realloc(tmpd, (size_t)(nc + 1) * sizeof(int64_t)) : NULL;
        if (a) tmpn = a;
        if (b) tmpd = b;
        int64_t *c = (a && b) ? (int64_t *)realloc(tmpm, (size_t)(nc + 1) * sizeof(int64_t)) : NULL;
        if (!c) { free(tmpn); free(tmpd); free(tmpm); free(lab); free(queue); return -1; }
        tmpm = c;
        for (int64_t k = 0; k < qt; k++) comp[queue[k]] = nc;
        tmpn[nc] = pn[u0]; tmpd[nc] = pd[u0]; tmpm[nc] = mv;
        nc++;
    }
    /* order by (rho desc, min id asc) */
    int64_t *perm = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    int64_t *inv = (int64_t *)malloc((size_t)(nc > 0 ? nc : 1) * sizeof(int64_t));
    if (!perm || !inv) { free(perm); free(inv); free(tmpn); free(tmpd); free(tmpm); free(lab); free(queue); return -1; }
    for (int64_t i = 0; i < nc; i++) perm[i] = i;
    for (int64_t i = 1; i < nc; i++) { /* insertion sort: nc is small */
        int64_t x = perm[i], j = i - 1;
        while (j >= 0) {
            int64_t y = perm[j];
            __int128 l = (__int128)tmpn[x] * tmpd[y], r = (__int128)tmpn[y] * tmpd[x];
            int before = (l > r) || (l == r && tmpm[x] < tmpm[y]);
            if (!before) break;
            perm[j + 1] = y; j--;
        }
        perm[j + 1] = x;
    }
    for (int64_t i = 0; i < nc; i++) inv[perm[i]] = i;
    for (int64_t u = 0; u < n; u++) if (comp[u] >= 0) comp[u] = inv[comp[u]];
    for (int64_t i = 0; i < nc; i++) {
        if (rho_num) rho_num[i] = tmpn[perm[i]];
        if (rho_den) rho_den[i] = tmpd[perm[i]];
        if (minv) minv[i] = tmpm[perm[i]];
    }
    free(perm); free(inv); free(tmpn); free(tmpd); free(tmpm); free(lab); free(queue);
    return nc;
}

/* ========================================================= brute force == */
/* For n <= 16: compactness by enumeration (Def. 1 / Def. compact): a
 * connected G[S] is rho-compact iff removing any nonempty Q ⊆ S removes at
 * least rho|Q| patterns, so its best rho is min_Q removed(Q)/|Q|.
 * Outputs:
 *   phi_num/phi_den[u]  compact number (Def. 4 / Def. trcn), reduced
 *   lds_mask[k]         vertex bitmask of each LDS / LTDS with density > 0
 *                       (Def. 3 / Def. ltds), sorted by (density desc,
 *                       lowest vertex asc); returns their number (or -1). */
int64_t orc_brute(const orc_graph *g, int mode, int64_t *phi_num, int64_t *phi_den, uint32_t *lds_mask,
                  int64_t *lds_num, int64_t *lds_den) {
    int64_t n = g->n;
    if (n > 16 || (mode != 2 && mode != 3)) return -1;
    patterns P;
    if (get_patterns(g, mode, &P)) return -1;
    uint32_t full = (n == 0) ? 0 : (uint32_t)((1u << n) - 1);
    uint32_t *pm = (uint32_t *)malloc((size_t)(P.np > 0 ? P.np : 1) * sizeof(uint32_t));
    int64_t *cnt = (int64_t *)calloc((size_t)full + 1, sizeof(int64_t));     /* |P(S)| */
    uint8_t *conn = (uint8_t *)calloc((size_t)full + 1, 1);
    int64_t *kn = (int64_t *)calloc((size_t)full + 1, sizeof(int64_t));      /* compactness num */
    int64_t *kd = (int64_t *)calloc((size_t)full + 1, sizeof(int64_t));      /* compactness den */
    uint32_t *nb = (uint32_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(uint32_t));
    if (!pm || !cnt || !conn || !kn || !kd || !nb) {
        free(pm); free(cnt); free(conn); free(kn); free(kd); free(nb); free(P.v); return -1;
    }
    for (int64_t k = 0; k < P.np; k++) {
        pm[k] = 0;
        for (int j = 0; j < P.h; j++) pm[k] |= 1u << P.v[P.h * k + j];
    }
    for (int64_t e = 0; e < g->m; e++) { nb[g->eu[e]] |= 1u << g->ev[e]; nb[g->ev[e]] |= 1u << g->eu[e]; }
    for (uint32_t S = 1; S <= full && full; S++) {
        int64_t c = 0;
        for (int64_t k = 0; k < P.np; k++) if ((pm[k] & S) == pm[k]) c++;
        cnt[S] = c;
        /* connectivity by flood fill inside S */
        uint32_t seen = S & (~S + 1), frontier = seen;
        while (frontier) {
            uint32_t nx = 0;
            for (int u = 0; u < n; u++) if (frontier >> u & 1) nx |= nb[u];
            nx &= S & ~seen;
            seen |= nx; frontier = nx;
        }
        conn[S] = (seen == S);
    }
    for (uint32_t S = 1; S <= full && full; S++) {
        if (!conn[S]) continue;
        int64_t bn = -1, bd = 1;
        /* nonempty Q ⊆ S: removing Q leaves S\Q */
        for (uint32_t Q = S; Q; Q = (Q - 1) & S) {
            int64_t rem = cnt[S] - cnt[S & ~Q];
            int64_t q = __builtin_popcount(Q);
            if (bn < 0 || (__int128)rem * bd < (__int128)bn * q) { bn = rem; bd = q; }
        }
        int64_t gg = gcd64(bn, bd);
        kn[S] = gg ? bn / gg : 0; kd[S] = gg ? bd / gg : 1;
    }
    for (int64_t u = 0; u < n; u++) {
        int64_t bn = 0, bd = 1;
        for (uint32_t S = 1; S <= full; S++) {
            if (!(S >> u & 1) || !conn[S]) continue;
            if ((__int128)kn[S] * bd > (__int128)bn * kd[S]) { bn = kn[S]; bd = kd[S]; }
        }
        phi_num[u] = bn; phi_den[u] = bd;
    }
    /* LDS: density(S)-compact (compactness == density) and no connected
     * proper superset is density(S)-compact */
    int64_t nl = 0;
    for (uint32_t S = 1; S <= full && full; S++) {
        if (!conn[S] || cnt[S] == 0) continue;
        int64_t dn = cnt[S], dd = __builtin_popcount(S);
        if ((__int128)kn[S] * dd != (__int128)dn * kd[S]) continue;
        int maximal = 1;
        /* proper supersets T of S, in increasing order */
        for (uint32_t T = (S + 1) | S; T <= full && maximal; T = (T + 1) | S) {
            if (!conn[T]) continue;
            if ((__int128)kn[T] * dd >= (__int128)dn * kd[T]) maximal = 0;
        }
        if (!maximal) continue;
        int64_t gg = gcd64(dn, dd);
        if (lds_mask) lds_mask[nl] = S;
        if (lds_num) lds_num[nl] = dn / gg;
        if (lds_den) lds_den[nl] = dd / gg;
        nl++;
    }
    /* sort (density desc, lowest vertex asc) */
    for (int64_t i = 1; i < nl && lds_mask && lds_num && lds_den; i++) {
        uint32_t xm = lds_mask[i]; int64_t xn = lds_num[i], xd = lds_den[i];
        int64_t j = i - 1;
        while (j >= 0) {
            __int128 l = (__int128)xn * lds_den[j], r = (__int128)lds_num[j] * xd;
            int before = (l > r) || (l == r && __builtin_ctz(xm) < __builtin_ctz(lds_mask[j]));
            if (!before) break;
            lds_mask[j + 1] = lds_mask[j]; lds_num[j + 1] = lds_num[j]; lds_den[j + 1] = lds_den[j];
            j--;
        }
        lds_mask[j + 1] = xm; lds_num[j + 1] = xn; lds_den[j + 1] = xd;
    }
    free(pm); free(cnt); free(conn); free(kn); free(kd); free(nb); free(P.v);
    return nl;
}
