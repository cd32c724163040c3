/*
 * Seeded synthetic network generators for the planted-community workloads.
 *
 * This file only draws random graphs; it holds none of the community
 * integration arithmetic.  Both the FP64 oracle and the HIP path consume
 * what it produces (a symmetric CSR adjacency with sorted rows, no
 * self-loops and no duplicates, plus planted community labels).
 *
 * Random numbers come from splitmix64 (Steele, Lea, Flood, "Fast splittable
 * pseudorandom number generators", OOPSLA 2014), one independent stream per
 * community so that generation is deterministic under any thread count.
 *
 * Graph model (stochastic block model with planted labels):
 *   - every unordered pair of distinct nodes inside community c is an edge
 *     with probability p_in[c], independently;
 *   - cross pairs (different communities, or at least one node with label -1)
 *     are either Bernoulli(p_out) each, or exactly n_inter distinct pairs
 *     drawn uniformly among all cross pairs.
 * Within a community, node ids increase with the local index, so sorted
 * local-index lists map to sorted user-id lists; the label sequence itself is
 * a uniformly shuffled multiset (done by the caller).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t sm64(uint64_t *s) {
    uint64_t z = (*s += GOLDEN);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
/* uniform double in (0,1] */
static inline double u01(uint64_t *s) { return ((sm64(s) >> 11) + 1) * 0x1.0p-53; }

/* number of failures before the first success of Bernoulli(q) trials */
static inline int64_t geom_skip(uint64_t *s, double log1mq) {
    double u = u01(s);
    double k = floor(log(u) / log1mq);
    if (k > 9.0e18) return INT64_MAX / 4;
    return (int64_t)k;
}

typedef struct gen_sbm {
    int64_t n;
    int32_t ncomm;
    int32_t *label;       /* [n] user order, -1 = no community */
    int32_t *local;       /* [n] index of the node inside its community */
    int64_t *comm_off;    /* [ncomm+1] offsets into members */
    int32_t *members;     /* user ids grouped by community, increasing */
    int64_t *miss_ptr;    /* [n+1] missing intra partners (local index) */
    int32_t *miss;
    int64_t *inter_ptr;   /* [n+1] cross-community neighbours (user id) */
    int32_t *inter;
    int64_t nnz;
} gen_sbm;

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}
static int cmp_u64(const void *a, const void *b) {
    uint64_t x = *(const uint64_t *)a, y = *(const uint64_t *)b;
    return (x > y) - (x < y);
}

static inline int is_cross(const int32_t *label, int64_t u, int64_t v) {
    return u != v && !(label[u] >= 0 && label[u] == label[v]);
}

void gen_sbm_free(gen_sbm *g) {
    if (!g) return;
    free(g->label); free(g->local); free(g->comm_off); free(g->members);
    free(g->miss_ptr); free(g->miss); free(g->inter_ptr); free(g->inter);
    free(g);
}

/* Build the cross-pair list: packed (u<<32 | v) with u < v, sorted, unique. */
static uint64_t *draw_cross_pairs(const int32_t *label, int64_t n, double p_out,
                                  int64_t n_inter, uint64_t seed, int64_t *count) {
    uint64_t s = seed ^ 0xC0FFEE1234567ULL;
    int64_t cap = 1024, cnt = 0;
    uint64_t *pairs = (uint64_t *)malloc(sizeof(uint64_t) * cap);
    if (p_out > 0.0) {
        /* geometric skipping over the upper triangle, row-major */
        if (p_out >= 1.0) p_out = 1.0;
        double l1q = log1p(-p_out);
        int64_t u = 0, v = 1;
        if (n < 2) { *count = 0; return pairs; }
        for (;;) {
            int64_t skip = (p_out >= 1.0) ? 0 : geom_skip(&s, l1q);
            /* advance (u,v) by skip positions */
            while (skip > 0 && u < n - 1) {
                int64_t rem = n - v;
                if (skip < rem) { v += skip; skip = 0; }
                else { skip -= rem; u++; v = u + 1; }
            }
            if (u >= n - 1) break;
            if (is_cross(label, u, v)) {
                if (cnt == cap) { cap *= 2; pairs = (uint64_t *)realloc(pairs, sizeof(uint64_t) * cap); }
                pairs[cnt++] = ((uint64_t)u << 32) | (uint64_t)v;
            }
            v++;
            if (v >= n) { u++; v = u + 1; }
            if (u >= n - 1) break;
        }
    } else if (n_inter > 0) {
        /* exactly n_inter distinct uniform cross pairs; never more than exist */
        int64_t *csz = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
        for (int64_t u = 0; u < n; u++) if (label[u] >= 0 && label[u] < n) csz[label[u]]++;
        double avail = 0.5 * (double)n * (double)(n - 1);
        for (int64_t c = 0; c < n; c++) avail -= 0.5 * (double)csz[c] * (double)(csz[c] - 1);
        free(csz);
        if ((double)n_inter > avail) n_inter = (int64_t)avail;
        cap = n_inter + 16;
        pairs = (uint64_t *)realloc(pairs, sizeof(uint64_t) * cap);
        while (cnt < n_inter) {
            while (cnt < n_inter) {
                int64_t u = (int64_t)(sm64(&s) % (uint64_t)n);
                int64_t v = (int64_t)(sm64(&s) % (uint64_t)n);
                if (!is_cross(label, u, v)) continue;
                if (u > v) { int64_t t = u; u = v; v = t; }
                pairs[cnt++] = ((uint64_t)u << 32) | (uint64_t)v;
            }
            qsort(pairs, (size_t)cnt, sizeof(uint64_t), cmp_u64);
            int64_t w = 0;
            for (int64_t i = 0; i < cnt; i++)
                if (w == 0 || pairs[i] != pairs[w - 1]) pairs[w++] = pairs[i];
            cnt = w;
        }
    }
    *count = cnt;
    return pairs;
}

/*
 * Create the generator state.  labels: [n] user order, -1 = no community,
 * community ids dense in [0, ncomm).  p_in: [ncomm].  Returns NULL on a bad
 * argument or allocation failure.
 */
gen_sbm *gen_sbm_create(int64_t n, const int32_t *labels, int32_t ncomm,
                        const double *p_in, double p_out, int64_t n_inter,
                        uint64_t seed) {
    if (n <= 0 || n > 0x7fffffff || ncomm < 0) return NULL;
    gen_sbm *g = (gen_sbm *)calloc(1, sizeof(gen_sbm));
    g->n = n; g->ncomm = ncomm;
    g->label = (int32_t *)malloc(sizeof(int32_t) * n);
    g->local = (int32_t *)malloc(sizeof(int32_t) * n);
    g->comm_off = (int64_t *)calloc((size_t)ncomm + 1, sizeof(int64_t));
    g->members = (int32_t *)malloc(sizeof(int32_t) * n);
    memcpy(g->label, labels, sizeof(int32_t) * n);
    for (int64_t u = 0; u < n; u++) {
        int32_t c = labels[u];
        if (c >= ncomm) { gen_sbm_free(g); return NULL; }
        if (c >= 0) g->comm_off[c + 1]++;
    }
    for (int32_t c = 0; c < ncomm; c++) g->comm_off[c + 1] += g->comm_off[c];
    {
        int64_t *fill = (int64_t *)calloc((size_t)ncomm + 1, sizeof(int64_t));
        for (int64_t u = 0; u < n; u++) {
            int32_t c = labels[u];
            if (c < 0) { g->local[u] = -1; continue; }
            g->local[u] = (int32_t)fill[c];
            g->members[g->comm_off[c] + fill[c]] = (int32_t)u;
            fill[c]++;
        }
        free(fill);
    }

    /* ---- intra-community missing pairs, one RNG stream per community ---- */
    g->miss_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    uint64_t **cpairs = (uint64_t **)calloc((size_t)ncomm + 1, sizeof(uint64_t *));
    int64_t *cnpairs = (int64_t *)calloc((size_t)ncomm + 1, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t c = 0; c < ncomm; c++) {
        int64_t lam = g->comm_off[c + 1] - g->comm_off[c];
        double q = 1.0 - p_in[c];
        if (lam < 2 || q <= 0.0) continue;
        uint64_t s = seed ^ (GOLDEN * (uint64_t)(c + 1)) ^ 0x5EED5EED5EEDULL;
        int64_t cap = 64, cnt = 0;
        uint64_t *pp = (uint64_t *)malloc(sizeof(uint64_t) * cap);
        double l1q = (q >= 1.0) ? 0.0 : log1p(-q);
        int64_t a = 0, b = 1;
        for (;;) {
            int64_t skip = (q >= 1.0) ? 0 : geom_skip(&s, l1q);
            while (skip > 0 && a < lam - 1) {
                int64_t rem = lam - b;
                if (skip < rem) { b += skip; skip = 0; }
                else { skip -= rem; a++; b = a + 1; }
            }
            if (a >= lam - 1) break;
            if (cnt == cap) { cap *= 2; pp = (uint64_t *)realloc(pp, sizeof(uint64_t) * cap); }
            pp[cnt++] = ((uint64_t)a << 32) | (uint64_t)b;
            b++;
            if (b >= lam) { a++; b = a + 1; }
            if (a >= lam - 1) break;
        }
        cpairs[c] = pp; cnpairs[c] = cnt;
        const int32_t *mem = g->members + g->comm_off[c];
        for (int64_t t = 0; t < cnt; t++) {
            int64_t la = (int64_t)(pp[t] >> 32), lb = (int64_t)(pp[t] & 0xffffffffULL);
            g->miss_ptr[mem[la] + 1]++;
            g->miss_ptr[mem[lb] + 1]++;
        }
    }
    for (int64_t u = 0; u < n; u++) g->miss_ptr[u + 1] += g->miss_ptr[u];
    g->miss = (int32_t *)malloc(sizeof(int32_t) * (g->miss_ptr[n] + 1));
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t c = 0; c < ncomm; c++) {
        if (!cpairs[c]) continue;
        const int32_t *mem = g->members + g->comm_off[c];
        /* generation order is row-major over (a<b): appending in that order
           leaves every row sorted by local index */
        for (int64_t t = 0; t < cnpairs[c]; t++) {
            int64_t la = (int64_t)(cpairs[c][t] >> 32), lb = (int64_t)(cpairs[c][t] & 0xffffffffULL);
            int32_t ua = mem[la], ub = mem[lb];
            g->miss[g->miss_ptr[ua]++] = (int32_t)lb;
            g->miss[g->miss_ptr[ub]++] = (int32_t)la;
        }
        free(cpairs[c]);
    }
    /* miss_ptr[u] now holds the end of row u; shift back */
    for (int64_t u = n; u > 0; u--) g->miss_ptr[u] = g->miss_ptr[u - 1];
    g->miss_ptr[0] = 0;
    free(cpairs); free(cnpairs);

    /* ---- cross pairs ---- */
    int64_t ncross = 0;
    uint64_t *cross = draw_cross_pairs(g->label, n, p_out, n_inter, seed, &ncross);
    g->inter_ptr = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t t = 0; t < ncross; t++) {
        g->inter_ptr[(cross[t] >> 32) + 1]++;
        g->inter_ptr[(cross[t] & 0xffffffffULL) + 1]++;
    }
    for (int64_t u = 0; u < n; u++) g->inter_ptr[u + 1] += g->inter_ptr[u];
    g->inter = (int32_t *)malloc(sizeof(int32_t) * (g->inter_ptr[n] + 1));
    {
        int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
        memcpy(pos, g->inter_ptr, sizeof(int64_t) * (n + 1));
        for (int64_t t = 0; t < ncross; t++) {
            int64_t u = (int64_t)(cross[t] >> 32), v = (int64_t)(cross[t] & 0xffffffffULL);
            g->inter[pos[u]++] = (int32_t)v;
            g->inter[pos[v]++] = (int32_t)u;
        }
        free(pos);
    }
    free(cross);
#pragma omp parallel for schedule(dynamic, 4096)
    for (int64_t u = 0; u < n; u++) {
        int64_t b = g->inter_ptr[u], e = g->inter_ptr[u + 1];
        if (e - b > 1) qsort(g->inter + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
    }

    int64_t nnz = 0;
    for (int64_t u = 0; u < n; u++) {
        int32_t c = g->label[u];
        int64_t d = g->inter_ptr[u + 1] - g->inter_ptr[u];
        if (c >= 0) d += (g->comm_off[c + 1] - g->comm_off[c]) - 1 - (g->miss_ptr[u + 1] - g->miss_ptr[u]);
        nnz += d;
    }
    g->nnz = nnz;
    return g;
}

int64_t gen_sbm_nnz(const gen_sbm *g) { return g->nnz; }
int64_t gen_sbm_n_missing(const gen_sbm *g) { return g->miss_ptr[g->n]; }
int64_t gen_sbm_n_cross(const gen_sbm *g) { return g->inter_ptr[g->n]; }

/* Write the CSR: row_ptr [n+1], col [nnz]; rows sorted by user id. */
void gen_sbm_fill(const gen_sbm *g, int64_t *row_ptr, int32_t *col) {
    int64_t n = g->n;
    row_ptr[0] = 0;
    for (int64_t u = 0; u < n; u++) {
        int32_t c = g->label[u];
        int64_t d = g->inter_ptr[u + 1] - g->inter_ptr[u];
        if (c >= 0) d += (g->comm_off[c + 1] - g->comm_off[c]) - 1 - (g->miss_ptr[u + 1] - g->miss_ptr[u]);
        row_ptr[u + 1] = row_ptr[u] + d;
    }
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t u = 0; u < n; u++) {
        int32_t c = g->label[u];
        int32_t *out = col + row_ptr[u];
        const int32_t *it = g->inter + g->inter_ptr[u];
        const int32_t *ie = g->inter + g->inter_ptr[u + 1];
        if (c < 0) {
            while (it < ie) *out++ = *it++;
            continue;
        }
        int64_t lam = g->comm_off[c + 1] - g->comm_off[c];
        const int32_t *mem = g->members + g->comm_off[c];
        const int32_t *mt = g->miss + g->miss_ptr[u];
        const int32_t *me = g->miss + g->miss_ptr[u + 1];
        int32_t self = g->local[u];
        for (int64_t b = 0; b < lam; b++) {
            if (b == self) continue;
            if (mt < me && *mt == b) { mt++; continue; }
            int32_t v = mem[b];
            while (it < ie && *it < v) *out++ = *it++;
            *out++ = v;
        }
        while (it < ie) *out++ = *it++;
    }
}

/*
 * Distinct random triples {u,v,w} that are not all inside one community,
 * packed as three int32 per triple with u < v < w, sorted and unique.
 * Returns the number written (== count unless the space is too small).
 */
int64_t gen_cross_triangles(int64_t n, const int32_t *labels, int64_t count,
                            uint64_t seed, int32_t *out /* [3*count] */) {
    if (n < 3 || count <= 0) return 0;
    if (n >= (1 << 21)) return -1;
    uint64_t s = seed ^ 0x7121A9C1E5ULL;
    int64_t cnt = 0;
    /* draw, sort, dedupe, repeat */
    typedef struct { int32_t a, b, c; } tri_t;
    tri_t *t = (tri_t *)malloc(sizeof(tri_t) * (size_t)count);
    while (cnt < count) {
        while (cnt < count) {
            int32_t x[3];
            for (int k = 0; k < 3; k++) x[k] = (int32_t)(sm64(&s) % (uint64_t)n);
            if (x[0] == x[1] || x[1] == x[2] || x[0] == x[2]) continue;
            if (labels[x[0]] >= 0 && labels[x[0]] == labels[x[1]] && labels[x[1]] == labels[x[2]]) continue;
            /* sort three */
            if (x[0] > x[1]) { int32_t q = x[0]; x[0] = x[1]; x[1] = q; }
            if (x[1] > x[2]) { int32_t q = x[1]; x[1] = x[2]; x[2] = q; }
            if (x[0] > x[1]) { int32_t q = x[0]; x[0] = x[1]; x[1] = q; }
            t[cnt].a = x[0]; t[cnt].b = x[1]; t[cnt].c = x[2]; cnt++;
        }
        /* sort lexicographically via packed keys (n < 2^21 required for packing) */
        uint64_t *key = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)cnt);
        for (int64_t i = 0; i < cnt; i++)
            key[i] = ((uint64_t)t[i].a << 42) | ((uint64_t)t[i].b << 21) | (uint64_t)t[i].c;
        qsort(key, (size_t)cnt, sizeof(uint64_t), cmp_u64);
        int64_t w = 0;
        for (int64_t i = 0; i < cnt; i++)
            if (w == 0 || key[i] != key[w - 1]) key[w++] = key[i];
        for (int64_t i = 0; i < w; i++) {
            t[i].a = (int32_t)(key[i] >> 42);
            t[i].b = (int32_t)((key[i] >> 21) & 0x1FFFFF);
            t[i].c = (int32_t)(key[i] & 0x1FFFFF);
        }
        free(key);
        cnt = w;
    }
    for (int64_t i = 0; i < cnt; i++) { out[3 * i] = t[i].a; out[3 * i + 1] = t[i].b; out[3 * i + 2] = t[i].c; }
    free(t);
    return cnt;
}
