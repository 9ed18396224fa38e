/*
 * Seeded synthetic graph generators shared by the GPU path's tests/bench and
 * by the CPU oracle.  This file holds NO arithmetic of the densest-subgraph
 * method: it only produces undirected edge lists (COO pairs) and query
 * streams.  Everything is deterministic given the seed (xoshiro256** seeded
 * through splitmix64, both from their published definitions by Vigna /
 * Blackman-Vigna), so the same graph can be rebuilt on any machine.
 *
 * Output edge lists may contain duplicate pairs (a planted block overlapping
 * the background) and arbitrary (src,dst) orientation; self-loops are never
 * emitted.  Consumers are expected to canonicalise (the paper assumes simple
 * undirected graphs, Section 3).
 *
 * Generators:
 *   - Chung-Lu power law (expected-degree model) sampled exactly with the
 *     Miller-Hagberg skipping method, optionally with planted G(s,p) blocks
 *     on disjoint random vertex sets;
 *   - Holme-Kim preferential attachment with triad formation;
 *   - Erdos-Renyi G(n,p) for small tests;
 *   - batch / serving-pool members and a Poisson query stream.
 * A final random permutation of vertex ids removes any id/degree correlation.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------ RNG -- */
typedef struct { uint64_t s[4]; } rng_t;

static uint64_t splitmix64(uint64_t *x) {
    uint64_t z = (*x += 0x9E3779B97F4A7C15ull);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
static void rng_seed(rng_t *r, uint64_t seed, uint64_t stream) {
    uint64_t x = seed * 0x9E3779B97F4A7C15ull ^ (stream + 0x632BE59BD9B4E019ull);
    for (int i = 0; i < 4; i++) r->s[i] = splitmix64(&x);
}
static inline uint64_t rotl(uint64_t x, int k) { return (x << k) | (x >> (64 - k)); }
static inline uint64_t rng_next(rng_t *r) {
    uint64_t *s = r->s;
    uint64_t out = rotl(s[1] * 5, 7) * 9;
    uint64_t t = s[1] << 17;
    s[2] ^= s[0]; s[3] ^= s[1]; s[1] ^= s[2]; s[0] ^= s[3];
    s[2] ^= t; s[3] = rotl(s[3], 45);
    return out;
}
/* uniform in (0,1] */
static inline double rng_u01(rng_t *r) { return ((rng_next(r) >> 11) + 1) * 0x1.0p-53; }
/* uniform integer in [0, k) (k > 0), Lemire-free simple rejection */
static inline uint64_t rng_below(rng_t *r, uint64_t k) {
    uint64_t lim = UINT64_MAX - UINT64_MAX % k;
    uint64_t x;
    do { x = rng_next(r); } while (x >= lim);
    return x % k;
}
static inline double rng_normal(rng_t *r) {
    double u1 = rng_u01(r), u2 = rng_u01(r);
    return sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

/* ----------------------------------------------------------- edge buffer -- */
typedef struct {
    int64_t n, m, cap;
    int32_t *src, *dst;
} graph_t;

static int g_push(graph_t *g, int64_t u, int64_t v) {
    if (g->m == g->cap) {
        int64_t nc = g->cap ? g->cap * 2 : 1024;
        int32_t *a = (int32_t *)realloc(g->src, nc * sizeof(int32_t));
        if (!a) return -1;
        g->src = a;
        int32_t *b = (int32_t *)realloc(g->dst, nc * sizeof(int32_t));
        if (!b) return -1;
        g->dst = b;
        g->cap = nc;
    }
    g->src[g->m] = (int32_t)u;
    g->dst[g->m] = (int32_t)v;
    g->m++;
    return 0;
}
static graph_t *g_new(int64_t n, int64_t cap_hint) {
    graph_t *g = (graph_t *)calloc(1, sizeof(graph_t));
    if (!g) return NULL;
    g->n = n;
    if (cap_hint > 0) {
        g->src = (int32_t *)malloc(cap_hint * sizeof(int32_t));
        g->dst = (int32_t *)malloc(cap_hint * sizeof(int32_t));
        if (!g->src || !g->dst) { free(g->src); free(g->dst); free(g); return NULL; }
        g->cap = cap_hint;
    }
    return g;
}

/* Fisher-Yates permutation of [0,n) */
static int32_t *random_perm(int64_t n, rng_t *r) {
    int32_t *p = (int32_t *)malloc((n > 0 ? n : 1) * sizeof(int32_t));
    if (!p) return NULL;
    for (int64_t i = 0; i < n; i++) p[i] = (int32_t)i;
    for (int64_t i = n - 1; i > 0; i--) {
        int64_t j = (int64_t)rng_below(r, (uint64_t)(i + 1));
        int32_t t = p[i]; p[i] = p[j]; p[j] = t;
    }
    return p;
}

/* relabel all ids by a random permutation and flip each pair's orientation
 * with probability 1/2 */
static int finish(graph_t *g, uint64_t seed) {
    rng_t r;
    rng_seed(&r, seed, 0xF1);
    int32_t *p = random_perm(g->n, &r);
    if (!p) return -1;
    for (int64_t e = 0; e < g->m; e++) {
        int32_t a = p[g->src[e]], b = p[g->dst[e]];
        if (rng_next(&r) >> 63) { int32_t t = a; a = b; b = t; }
        g->src[e] = a; g->dst[e] = b;
    }
    free(p);
    return 0;
}

/* --------------------------------------------------------- Chung-Lu ----- */
/* Expected degrees w_i = c*(i+1)^(-1/(beta-1)), rescaled to the requested
 * mean and capped at sqrt(sum w) (so every pair probability is <= 1);
 * capping and rescaling alternate a few times until the mean is met. */
static double *chung_lu_weights(int64_t n, double beta, double avg_deg) {
    double *w = (double *)malloc((n > 0 ? n : 1) * sizeof(double));
    if (!w) return NULL;
    double ex = -1.0 / (beta - 1.0);
    for (int64_t i = 0; i < n; i++) w[i] = pow((double)(i + 1), ex);
    double target = avg_deg * (double)n;
    for (int it = 0; it < 8; it++) {
        double s = 0;
        for (int64_t i = 0; i < n; i++) s += w[i];
        double sc = target / s;
        for (int64_t i = 0; i < n; i++) w[i] *= sc;
        double cap = sqrt(target);
        for (int64_t i = 0; i < n; i++) if (w[i] > cap) w[i] = cap;
    }
    return w;
}

/* Miller-Hagberg exact O(n+m) sampling: edge (u,v) independently with
 * probability min(w_u w_v / S, 1), w sorted non-increasing. */
static int chung_lu_sample(graph_t *g, const double *w, int64_t n, rng_t *r) {
    double S = 0;
    for (int64_t i = 0; i < n; i++) S += w[i];
    if (S <= 0) return 0;
    for (int64_t u = 0; u + 1 < n; u++) {
        int64_t v = u + 1;
        double p = w[u] * w[v] / S;
        if (p > 1) p = 1;
        while (v < n && p > 0) {
            if (p < 1) {
                double x = rng_u01(r);
                double skip = floor(log(x) / log1p(-p));
                if (skip >= (double)(n - v)) break;
                v += (int64_t)skip;
            }
            if (v < n) {
                double q = w[u] * w[v] / S;
                if (q > 1) q = 1;
                if (rng_u01(r) <= q / p)
                    if (g_push(g, u, v)) return -1;
                p = q;
                v++;
            }
        }
    }
    return 0;
}

/* G(s,p) on the vertex list vs[0..s) with geometric skipping over pairs */
static int planted_block(graph_t *g, const int32_t *vs, int64_t s, double p, rng_t *r) {
    if (s < 2 || p <= 0) return 0;
    int64_t npairs = s * (s - 1) / 2;
    int64_t i = 0, j = 1, rowstart = 0; /* pair index of (i, i+1) */
    int64_t k = -1;
    for (;;) {
        if (p < 1) {
            double x = rng_u01(r);
            double skip = floor(log(x) / log1p(-p));
            if (skip >= (double)(npairs - k - 1)) break;
            k += (int64_t)skip + 1;
        } else {
            k += 1;
        }
        if (k >= npairs) break;
        /* advance (i,j) to pair index k; rows have s-1-i pairs */
        while (k >= rowstart + (s - 1 - i)) { rowstart += s - 1 - i; i++; }
        j = i + 1 + (k - rowstart);
        if (g_push(g, vs[i], vs[j])) return -1;
    }
    return 0;
}

static graph_t *gen_powerlaw_planted(int64_t n, double beta, double avg_deg, int32_t n_blocks,
                                     int32_t s_lo, int32_t s_hi, double p_block, uint64_t seed) {
    graph_t *g = g_new(n, (int64_t)(avg_deg * (double)n * 0.55) + 1024);
    if (!g) return NULL;
    rng_t r;
    rng_seed(&r, seed, 0xC1);
    double *w = chung_lu_weights(n, beta, avg_deg);
    if (!w) goto fail;
    if (chung_lu_sample(g, w, n, &r)) { free(w); goto fail; }
    free(w);
    if (n_blocks > 0) {
        rng_t rb;
        rng_seed(&rb, seed, 0xB1);
        int32_t *perm = random_perm(n, &rb);
        if (!perm) goto fail;
        int64_t off = 0;
        for (int32_t b = 0; b < n_blocks; b++) {
            int64_t s = s_lo + (int64_t)rng_below(&rb, (uint64_t)(s_hi - s_lo + 1));
            if (off + s > n) s = n - off;
            if (s < 2) break;
            if (planted_block(g, perm + off, s, p_block, &rb)) { free(perm); goto fail; }
            off += s;
        }
        free(perm);
    }
    if (finish(g, seed)) goto fail;
    return g;
fail:
    free(g->src); free(g->dst); free(g);
    return NULL;
}

/* -------------------------------------------------------- Holme-Kim ----- */
typedef struct { int32_t *a; int32_t n, cap; } ivec;
static int iv_push(ivec *v, int32_t x) {
    if (v->n == v->cap) {
        int32_t nc = v->cap ? v->cap * 2 : 8;
        int32_t *p = (int32_t *)realloc(v->a, (size_t)nc * sizeof(int32_t));
        if (!p) return -1;
        v->a = p; v->cap = nc;
    }
    v->a[v->n++] = x;
    return 0;
}

/* Preferential attachment with triad formation: each new vertex adds mper
 * edges; the first goes to a degree-proportional target, each further one
 * with probability pt to a random neighbour of the last preferential target
 * (triad formation), else preferentially.  Seed graph: K_{mper+1}. */
static graph_t *gen_holme_kim(int64_t n, int32_t mper, double pt, uint64_t seed) {
    int64_t n0 = mper + 1;
    if (n < n0) n0 = n;
    int64_t mtot = n0 * (n0 - 1) / 2 + (n - n0) * (int64_t)mper;
    graph_t *g = g_new(n, mtot + 16);
    if (!g) return NULL;
    ivec *adj = (ivec *)calloc((size_t)(n > 0 ? n : 1), sizeof(ivec));
    int32_t *ends = (int32_t *)malloc((size_t)(2 * mtot + 16) * sizeof(int32_t));
    int32_t *tg = (int32_t *)malloc((size_t)(mper + 1) * sizeof(int32_t));
    int64_t ne = 0;
    rng_t r;
    rng_seed(&r, seed, 0xA1);
    if (!adj || !ends || !tg) goto fail;
    for (int64_t a = 0; a < n0; a++)
        for (int64_t b = a + 1; b < n0; b++) {
            if (g_push(g, a, b) || iv_push(&adj[a], (int32_t)b) || iv_push(&adj[b], (int32_t)a)) goto fail;
            ends[ne++] = (int32_t)a; ends[ne++] = (int32_t)b;
        }
    for (int64_t v = n0; v < n; v++) {
        int nt = 0;
        int32_t last_pa = -1;
        for (int k = 0; k < mper; k++) {
            int32_t t = -1;
            if (k > 0 && last_pa >= 0 && rng_u01(&r) <= pt) {
                ivec *nb = &adj[last_pa];
                for (int tries = 0; tries < 4 && nb->n > 0; tries++) {
                    int32_t c = nb->a[rng_below(&r, (uint64_t)nb->n)];
                    int dup = (c == v);
                    for (int q = 0; q < nt && !dup; q++) dup = (tg[q] == c);
                    if (!dup) { t = c; break; }
                }
            }
            if (t < 0) {
                for (;;) {
                    int32_t c = ends[rng_below(&r, (uint64_t)ne)];
                    int dup = 0;
                    for (int q = 0; q < nt && !dup; q++) dup = (tg[q] == c);
                    if (!dup) { t = c; break; }
                }
                last_pa = t;
            }
            tg[nt++] = t;
        }
        for (int q = 0; q < nt; q++) {
            if (g_push(g, v, tg[q]) || iv_push(&adj[v], tg[q]) || iv_push(&adj[tg[q]], (int32_t)v)) goto fail;
            ends[ne++] = (int32_t)v; ends[ne++] = tg[q];
        }
    }
    for (int64_t i = 0; i < n; i++) free(adj[i].a);
    free(adj); free(ends); free(tg);
    if (finish(g, seed)) { free(g->src); free(g->dst); free(g); return NULL; }
    return g;
fail:
    if (adj) { for (int64_t i = 0; i < n; i++) free(adj[i].a); free(adj); }
    free(ends); free(tg);
    free(g->src); free(g->dst); free(g);
    return NULL;
}

/* ----------------------------------------------------- Erdos-Renyi ------ */
static graph_t *gen_erdos_renyi(int64_t n, double p, uint64_t seed) {
    graph_t *g = g_new(n, 0);
    if (!g) return NULL;
    rng_t r;
    rng_seed(&r, seed, 0xE1);
    int32_t *ids = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    if (!ids) { free(g); return NULL; }
    for (int64_t i = 0; i < n; i++) ids[i] = (int32_t)i;
    if (planted_block(g, ids, n, p, &r)) { free(ids); free(g->src); free(g->dst); free(g); return NULL; }
    free(ids);
    if (finish(g, seed)) { free(g->src); free(g->dst); free(g); return NULL; }
    return g;
}

/* ------------------------------------------ batch / serving-pool members -- */
/* One member of a batch of uneven graphs: n log-uniform in [n_lo, n_hi],
 * average degree uniform in [6,20], Chung-Lu beta 2.3, 1-5 planted G(s,0.5)
 * blocks with s uniform in [8, max(8, min(60, n/4))]. */
static graph_t *gen_batch_member(int64_t index, uint64_t base_seed, double n_lo, double n_hi) {
    rng_t r;
    uint64_t seed = base_seed + (uint64_t)index;
    rng_seed(&r, seed, 0xD1);
    double ln = log(n_lo) + (log(n_hi) - log(n_lo)) * (rng_u01(&r));
    int64_t n = (int64_t)llround(exp(ln));
    if (n < (int64_t)n_lo) n = (int64_t)n_lo;
    if (n > (int64_t)n_hi) n = (int64_t)n_hi;
    double deg = 6.0 + 14.0 * rng_u01(&r);
    int32_t nb = 1 + (int32_t)rng_below(&r, 5);
    int64_t shi = n / 4 < 60 ? n / 4 : 60;
    if (shi < 8) shi = 8;
    return gen_powerlaw_planted(n, 2.3, deg, nb, 8, (int32_t)shi, 0.5, seed);
}

/* Serving pool member: n lognormal (median `median`, sigma `sigma`) clipped
 * to [50, n_max]; member 0 is pinned at n_max; otherwise as a batch member. */
static graph_t *gen_pool_member(int64_t index, uint64_t base_seed, double median, double sigma,
                                int64_t n_max) {
    rng_t r;
    uint64_t seed = base_seed * 1000003ull + (uint64_t)index;
    rng_seed(&r, seed, 0xD2);
    int64_t n;
    if (index == 0) n = n_max;
    else {
        double x = exp(log(median) + sigma * rng_normal(&r));
        n = (int64_t)llround(x);
        if (n < 50) n = 50;
        if (n > n_max) n = n_max;
    }
    double deg = 6.0 + 14.0 * rng_u01(&r);
    int32_t nb = 1 + (int32_t)rng_below(&r, 5);
    int64_t shi = n / 4 < 60 ? n / 4 : 60;
    if (shi < 8) shi = 8;
    return gen_powerlaw_planted(n, 2.3, deg, nb, 8, (int32_t)shi, 0.5, seed);
}

/* ------------------------------------------------------------ C API ----- */
void *synth_powerlaw_planted(int64_t n, double beta, double avg_deg, int32_t n_blocks,
                             int32_t s_lo, int32_t s_hi, double p_block, uint64_t seed) {
    if (n < 0 || n > 2147483647LL || s_lo > s_hi || beta <= 1.0) return NULL;
    return gen_powerlaw_planted(n, beta, avg_deg, n_blocks, s_lo, s_hi, p_block, seed);
}
void *synth_holme_kim(int64_t n, int32_t mper, double pt, uint64_t seed) {
    if (n < 0 || n > 2147483647LL || mper < 1) return NULL;
    return gen_holme_kim(n, mper, pt, seed);
}
void *synth_erdos_renyi(int64_t n, double p, uint64_t seed) {
    if (n < 0 || n > 100000) return NULL;
    return gen_erdos_renyi(n, p, seed);
}
void *synth_batch_member(int64_t index, uint64_t base_seed, double n_lo, double n_hi) {
    if (n_lo < 2 || n_hi < n_lo) return NULL;
    return gen_batch_member(index, base_seed, n_lo, n_hi);
}
void *synth_pool_member(int64_t index, uint64_t base_seed, double median, double sigma, int64_t n_max) {
    if (n_max < 50) return NULL;
    return gen_pool_member(index, base_seed, median, sigma, n_max);
}
int64_t synth_num_vertices(void *h) { return h ? ((graph_t *)h)->n : -1; }
int64_t synth_num_pairs(void *h) { return h ? ((graph_t *)h)->m : -1; }
void synth_copy(void *h, int32_t *src, int32_t *dst) {
    graph_t *g = (graph_t *)h;
    if (!g) return;
    if (g->m) {
        memcpy(src, g->src, (size_t)g->m * sizeof(int32_t));
        memcpy(dst, g->dst, (size_t)g->m * sizeof(int32_t));
    }
}
void synth_free(void *h) {
    graph_t *g = (graph_t *)h;
    if (!g) return;
    free(g->src); free(g->dst); free(g);
}

/* Poisson query stream: exponential inter-arrival gaps at `qps`, graph
 * uniform over [0,pool), mode 2 (edge) or 3 (triangle) with probability 1/2,
 * k uniform in [1,kmax].  Writes `count` entries. */
void synth_queries(int64_t count, double qps, int32_t pool, int32_t kmax, uint64_t seed,
                   double *t_arrive, int32_t *graph, int32_t *mode, int32_t *k) {
    rng_t r;
    rng_seed(&r, seed, 0x51);
    double t = 0;
    for (int64_t i = 0; i < count; i++) {
        t += -log(rng_u01(&r)) / qps;
        t_arrive[i] = t;
        graph[i] = (int32_t)rng_below(&r, (uint64_t)pool);
        mode[i] = (rng_next(&r) >> 63) ? 3 : 2;
        k[i] = 1 + (int32_t)rng_below(&r, (uint64_t)kmax);
    }
}
