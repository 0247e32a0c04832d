/*
 * Seeded synthetic graph generators shared by the tests, the benchmark and the
 * oracle's golden-value script.  This module holds none of the counting
 * method's arithmetic: it only draws simple undirected graphs and writes them
 * as symmetric CSR (rows sorted by vertex id, no self-loops, no duplicates).
 *
 * Randomness: splitmix64 (Steele, Lea, Flood, "Fast splittable pseudorandom
 * number generators", OOPSLA 2014).  Every independent stream is keyed by
 * (seed, stream index), so results do not depend on thread count.
 *
 * Generators:
 *   - Erdos-Renyi G(n,p) by geometric skipping over the lower triangle
 *     (Batagelj and Brandes, "Efficient generation of large random networks",
 *     Phys. Rev. E 71, 2005).
 *   - Chung-Lu expected-degree graphs, p_uv = min(1, w_u w_v / sum(w)), sampled
 *     in O(n+m) (Miller and Hagberg, "Efficient generation of networks with
 *     given expected degrees", WAW 2011).  Power-law weights
 *     w_i = c (i + 1 + i0)^(-1/(gamma-1)) with (c, i0) chosen so that
 *     w_0 = d_max and mean(w) = d_bar.
 * After generation the vertex ids are shuffled by a seeded permutation so that
 * id order says nothing about degree.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

static inline uint64_t sm64_next(uint64_t *s) {
    uint64_t z = (*s += 0x9E3779B97F4A7C15ULL);
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Public helper: one splitmix64 output for (seed, index); used to derive
 * per-graph seeds for batches and request streams. */
uint64_t synth_mix(uint64_t seed, uint64_t index) {
    uint64_t s = seed ^ (index * 0xD1B54A32D192ED03ULL);
    sm64_next(&s);
    return sm64_next(&s);
}

static inline uint64_t stream_init(uint64_t seed, uint64_t stream) {
    uint64_t s = synth_mix(seed, stream + 0x5bd1e995ULL);
    return s;
}

/* uniform double in (0,1), never 0 or 1 */
static inline double u01(uint64_t *s) {
    return ((double)(sm64_next(s) >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

typedef struct { int32_t u, v; } edge_t;

typedef struct {
    edge_t *e;
    int64_t len, cap;
} edgevec;

static int ev_push(edgevec *ev, int32_t u, int32_t v) {
    if (ev->len == ev->cap) {
        int64_t nc = ev->cap ? ev->cap * 2 : 1024;
        edge_t *ne = (edge_t *)realloc(ev->e, (size_t)nc * sizeof(edge_t));
        if (!ne) return -1;
        ev->e = ne; ev->cap = nc;
    }
    ev->e[ev->len].u = u; ev->e[ev->len].v = v; ev->len++;
    return 0;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Shuffle ids with a seeded permutation and build symmetric sorted CSR.
 * row_ptr has n+1 entries (int64 so very large graphs are representable),
 * col has 2*len entries.  Returns 0 on success. */
static int to_csr(int32_t n, const edgevec *ev, uint64_t seed,
                  int64_t **row_ptr_out, int32_t **col_out) {
    int32_t *perm = (int32_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int32_t));
    int64_t *rp = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    int32_t *col = (int32_t *)malloc((size_t)(ev->len > 0 ? 2 * ev->len : 1) * sizeof(int32_t));
    int64_t *fill = (int64_t *)malloc((size_t)(n > 0 ? n : 1) * sizeof(int64_t));
    if (!perm || !rp || !col || !fill) { free(perm); free(rp); free(col); free(fill); return -1; }
    for (int32_t i = 0; i < n; i++) perm[i] = i;
    uint64_t s = stream_init(seed, 0xFFFFFFFFull);
    for (int32_t i = n - 1; i > 0; i--) {
        int32_t j = (int32_t)(sm64_next(&s) % (uint64_t)(i + 1));
        int32_t t = perm[i]; perm[i] = perm[j]; perm[j] = t;
    }
    for (int64_t k = 0; k < ev->len; k++) {
        rp[perm[ev->e[k].u] + 1]++;
        rp[perm[ev->e[k].v] + 1]++;
    }
    for (int32_t i = 0; i < n; i++) rp[i + 1] += rp[i];
    for (int32_t i = 0; i < n; i++) fill[i] = rp[i];
    for (int64_t k = 0; k < ev->len; k++) {
        int32_t a = perm[ev->e[k].u], b = perm[ev->e[k].v];
        col[fill[a]++] = b;
        col[fill[b]++] = a;
    }
    for (int32_t i = 0; i < n; i++)
        qsort(col + rp[i], (size_t)(rp[i + 1] - rp[i]), sizeof(int32_t), cmp_i32);
    free(perm); free(fill);
    *row_ptr_out = rp; *col_out = col;
    return 0;
}

void synth_free(void *p) { free(p); }

/* G(n,p).  Returns number of undirected edges, or -1 on allocation failure. */
int64_t synth_er(int32_t n, double p, uint64_t seed,
                 int64_t **row_ptr_out, int32_t **col_out) {
    edgevec ev = {0, 0, 0};
    if (n >= 2 && p > 0.0) {
        if (p >= 1.0) {
            for (int32_t v = 1; v < n; v++)
                for (int32_t w = 0; w < v; w++)
                    if (ev_push(&ev, v, w)) { free(ev.e); return -1; }
        } else {
            uint64_t s = stream_init(seed, 0);
            double lq = log1p(-p);
            int64_t v = 1, w = -1;
            while (v < n) {
                double r = u01(&s);
                double sk = floor(log(1.0 - r) / lq);
                if (sk >= (double)n * (double)n) break;
                w = w + 1 + (int64_t)sk;
                while (w >= v && v < n) { w -= v; v++; }
                if (v < n && ev_push(&ev, (int32_t)v, (int32_t)w)) { free(ev.e); return -1; }
            }
        }
    }
    int rc = to_csr(n, &ev, seed, row_ptr_out, col_out);
    int64_t m = ev.len;
    free(ev.e);
    return rc ? -1 : m;
}

/* Power-law weights: w_i = c (i+1+i0)^(-a), a = 1/(gamma-1), w_0 = dmax,
 * mean(w) = dbar.  mean is increasing in i0 at fixed w_0, so bisect on
 * log(1+i0).  Degenerate requests (dbar >= dmax) get constant weights. */
static void powerlaw_weights(int32_t n, double gamma, double dbar, double dmax, double *w) {
    double a = 1.0 / (gamma - 1.0);
    if (dbar >= dmax) {
        for (int32_t i = 0; i < n; i++) w[i] = dmax;
        return;
    }
    double lo = -20.0, hi = 40.0;   /* bounds on log(1+i0) */
    for (int it = 0; it < 64; it++) {
        double mid = 0.5 * (lo + hi);
        double base = exp(mid);     /* 1+i0 */
        double acc = 0.0;
        for (int32_t i = 0; i < n; i++) acc += pow(base / (base + (double)i), a);
        double mean = dmax * acc / (double)n;
        if (mean < dbar) lo = mid; else hi = mid;
    }
    double base = exp(0.5 * (lo + hi));
    for (int32_t i = 0; i < n; i++) w[i] = dmax * pow(base / (base + (double)i), a);
}

static int cl_row(int32_t u, int32_t n, const double *w, double S, uint64_t seed, edgevec *ev, int64_t *count) {
    uint64_t s = stream_init(seed, (uint64_t)u + 1);
    int64_t v = (int64_t)u + 1;
    if (v >= n) return 0;
    double p = w[u] * w[v] / S;
    if (p > 1.0) p = 1.0;
    while (v < n && p > 0.0) {
        if (p != 1.0) {
            double r = u01(&s);
            double sk = floor(log(r) / log1p(-p));
            if (sk >= (double)n) v = n; else v += (int64_t)sk;
        }
        if (v < n) {
            double q = w[u] * w[v] / S;
            if (q > 1.0) q = 1.0;
            double r = u01(&s);
            if (r < q / p) {
                if (ev) { if (ev_push(ev, u, (int32_t)v)) return -1; }
                else (*count)++;
            }
            p = q;
            v++;
        }
    }
    return 0;
}

/* Chung-Lu with power-law weights.  Returns number of undirected edges. */
int64_t synth_chung_lu(int32_t n, double gamma, double dbar, double dmax, uint64_t seed,
                       int64_t **row_ptr_out, int32_t **col_out) {
    edgevec ev = {0, 0, 0};
    double *w = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    if (!w) return -1;
    if (n > 0) powerlaw_weights(n, gamma, dbar, dmax, w);
    double S = 0.0;
    for (int32_t i = 0; i < n; i++) S += w[i];
    if (n >= 2 && S > 0.0) {
        for (int32_t u = 0; u + 1 < n; u++)
            if (cl_row(u, n, w, S, seed, &ev, NULL)) { free(w); free(ev.e); return -1; }
    }
    free(w);
    int rc = to_csr(n, &ev, seed, row_ptr_out, col_out);
    int64_t m = ev.len;
    free(ev.e);
    return rc ? -1 : m;
}
