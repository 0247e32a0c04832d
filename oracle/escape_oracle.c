/*
 * ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, CPU implementation of the counting method of Pinar, Seshadhri
 * and Vishal, "ESCAPE: Efficiently Counting All 5-Vertex Subgraphs"
 * (arXiv 1610.09411).  Only the test-suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this file's library; the product
 * path never does.  It shares no code with the GPU library.
 *
 * Every count is an exact integer.  Per-item counters are uint64, global sums
 * are unsigned 128-bit.  Loops over source vertices run under OpenMP with
 * per-thread partial sums, so the result does not depend on thread count.
 *
 * The steps follow the paper's order:
 *   1. degree order and DAG                          (Sec. 2.2, notation)
 *   2. triangles, per-vertex / per-edge triangle counts and per-edge
 *      triangle lists                                (Thm 4vertex-tri)
 *   3. 4-cycles, total and per edge                  (Thm 4cycle)
 *   4. 4-cliques per vertex / edge / triangle        (Thm 4clique)
 *   5. the sums behind the 5-vertex cut formulas     (Thms 5cutvertex,
 *      5cutedge, 5cuttri, 5cutwed, 5formula)
 *   6. 5-cycles through directed 3-paths             (Thm 5cycle)
 *   7. 5-cliques through directed bipyramids         (Thm 5clique)
 * The Python side (oracle/__init__.py) turns these sums into non-induced
 * counts, adds the disconnected patterns (Appendix A) and applies the
 * induced/non-induced transform (Appendix B).
 *
 * Readings where the printed paper is ambiguous or wrong are listed next to
 * the step that uses them and pinned by brute-force tests.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

typedef unsigned __int128 u128;
typedef uint64_t u64;

/* Timing sample for the CPU baseline: with g_sample = s > 1 the loops after
 * the triangle stage visit only sources (and edges) whose id plus g_offset
 * is a multiple of s; the sums are then meaningless and only the elapsed time
 * is used.  With s = 1 (every test) nothing is skipped. */
static int g_sample = 1;
static int g_offset = 0;
#define SAMPLED(x) (g_sample > 1 && (((int64_t)(x) + g_offset) % g_sample) != 0)

/* offset of the next sampled run (timing only) */
void oracle_set_sample_offset(int offset) { g_offset = offset > 0 ? offset : 0; }

/* ------------------------------------------------------------------ graph */

typedef struct {
    int32_t n;
    int64_t m;            /* undirected edges */
    const int32_t *rp;    /* n+1 */
    const int32_t *ci;    /* 2m, rows sorted by id */
    int64_t *rank;        /* position of each vertex in the total order */
    int64_t *deg;
    int64_t *eid;         /* per arc: id of its undirected edge */
    int32_t *eu, *ev;     /* per edge: endpoints, eu precedes ev */
    /* triangles */
    u128 T;
    u64 *tv, *te;         /* t(v), t(e) */
    int64_t *aoff;        /* per edge: offset of its triangle list (apex vertices) */
    int32_t *apex;        /* third vertices, sorted by id within each list */
    int64_t *atri;        /* triangle id of each apex entry */
    int64_t ntri;
    /* 4-cycles and 4-cliques */
    u128 C4, K4;
    u64 *c4e, *c4v;
    u64 *k4e, *k4v, *k4t;
} graph;

static inline int prec(const graph *g, int32_t a, int32_t b) { return g->rank[a] < g->rank[b]; }

/* position of v in the sorted row of u, or -1 */
static int64_t find_arc(const graph *g, int32_t u, int32_t v) {
    int64_t lo = g->rp[u], hi = g->rp[u + 1];
    while (lo < hi) {
        int64_t mid = (lo + hi) >> 1;
        if (g->ci[mid] < v) lo = mid + 1; else hi = mid;
    }
    return (lo < g->rp[u + 1] && g->ci[lo] == v) ? lo : -1;
}

static inline int64_t edge_of(const graph *g, int32_t u, int32_t v) { return g->eid[find_arc(g, u, v)]; }

static inline int adjacent(const graph *g, int32_t u, int32_t v) { return find_arc(g, u, v) >= 0; }

static inline u64 ch2(u64 x) { return x < 2 ? 0 : x * (x - 1) / 2; }
static inline u128 ch3(u64 x) { return x < 3 ? 0 : (u128)x * (x - 1) * (x - 2) / 6; }
static inline u128 ch4(u64 x) { return x < 4 ? 0 : (u128)x * (x - 1) * (x - 2) / 6 * (x - 3) / 4; }

/* Step 1: degree order (Sec. 2.2): i precedes j when d(i) < d(j), ties by id.
 * A caller may pass any other total order in `order_rank` (used by tests: all
 * counts must be independent of it). */
static int setup(graph *g, int32_t n, const int32_t *rp, const int32_t *ci, const int64_t *order_rank) {
    memset(g, 0, sizeof(*g));
    g->n = n; g->rp = rp; g->ci = ci; g->m = (int64_t)rp[n] / 2;
    g->deg = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    g->rank = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    g->eid = (int64_t *)malloc(sizeof(int64_t) * (rp[n] + 1));
    g->eu = (int32_t *)malloc(sizeof(int32_t) * (g->m + 1));
    g->ev = (int32_t *)malloc(sizeof(int32_t) * (g->m + 1));
    if (!g->deg || !g->rank || !g->eid || !g->eu || !g->ev) return -1;
    for (int32_t v = 0; v < n; v++) g->deg[v] = rp[v + 1] - rp[v];
    if (order_rank) {
        for (int32_t v = 0; v < n; v++) g->rank[v] = order_rank[v];
    } else {
        /* rank = number of vertices strictly before v in (degree, id) order:
         * counting sort on degree, stable in id */
        int64_t maxd = 0;
        for (int32_t v = 0; v < n; v++) if (g->deg[v] > maxd) maxd = g->deg[v];
        int64_t *cnt = (int64_t *)calloc((size_t)maxd + 2, sizeof(int64_t));
        if (!cnt) return -1;
        for (int32_t v = 0; v < n; v++) cnt[g->deg[v] + 1]++;
        for (int64_t d = 0; d <= maxd; d++) cnt[d + 1] += cnt[d];
        for (int32_t v = 0; v < n; v++) g->rank[v] = cnt[g->deg[v]]++;
        free(cnt);
    }
    /* undirected edge ids: one per pair, endpoints stored low-to-high in the order */
    int64_t e = 0;
    for (int32_t u = 0; u < n; u++)
        for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
            int32_t v = ci[p];
            if (u < v) {
                g->eid[p] = e;
                if (prec(g, u, v)) { g->eu[e] = u; g->ev[e] = v; } else { g->eu[e] = v; g->ev[e] = u; }
                e++;
            }
        }
    for (int32_t u = 0; u < n; u++)
        for (int64_t p = rp[u]; p < rp[u + 1]; p++) {
            int32_t v = ci[p];
            if (v < u) g->eid[p] = g->eid[find_arc(g, v, u)];
        }
    return 0;
}

/* Step 2: triangles (Thm 4vertex-tri, classic out-wedge enumeration).  For an
 * arc a->b, every c adjacent to both with a before b before c closes exactly
 * one triangle.  Also stores, for each edge, the list of third vertices of its
 * triangles (the paper keeps these lists; they are reused by later steps). */
static int triangles(graph *g) {
    int32_t n = g->n;
    int64_t m = g->m;
    g->tv = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    g->te = (u64 *)calloc((size_t)m + 1, sizeof(u64));
    if (!g->tv || !g->te) return -1;
    u128 T = 0;
    #pragma omp parallel for schedule(dynamic, 256) reduction(+:T)
    for (int32_t a = 0; a < n; a++)
        for (int64_t p = g->rp[a]; p < g->rp[a + 1]; p++) {
            int32_t b = g->ci[p];
            if (!prec(g, a, b)) continue;
            /* third vertices c with b before c, adjacent to a and b */
            int64_t x = g->rp[a], y = g->rp[b];
            while (x < g->rp[a + 1] && y < g->rp[b + 1]) {
                int32_t ca = g->ci[x], cb = g->ci[y];
                if (ca < cb) x++;
                else if (ca > cb) y++;
                else {
                    if (prec(g, b, ca)) {
                        T++;
                        __atomic_fetch_add(&g->tv[a], 1, __ATOMIC_RELAXED);
                        __atomic_fetch_add(&g->tv[b], 1, __ATOMIC_RELAXED);
                        __atomic_fetch_add(&g->tv[ca], 1, __ATOMIC_RELAXED);
                        __atomic_fetch_add(&g->te[g->eid[p]], 1, __ATOMIC_RELAXED);
                        __atomic_fetch_add(&g->te[g->eid[x]], 1, __ATOMIC_RELAXED);
                        __atomic_fetch_add(&g->te[g->eid[y]], 1, __ATOMIC_RELAXED);
                    }
                    x++; y++;
                }
            }
        }
    g->T = T;
    /* per-edge triangle lists = common neighbours of the endpoints (sorted) */
    g->aoff = (int64_t *)malloc(sizeof(int64_t) * (m + 1));
    if (!g->aoff) return -1;
    g->aoff[0] = 0;
    for (int64_t e = 0; e < m; e++) g->aoff[e + 1] = g->aoff[e] + (int64_t)g->te[e];
    g->apex = (int32_t *)malloc(sizeof(int32_t) * (g->aoff[m] + 1));
    g->atri = (int64_t *)malloc(sizeof(int64_t) * (g->aoff[m] + 1));
    if (!g->apex || !g->atri) return -1;
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t e = 0; e < m; e++) {
        int32_t u = g->eu[e], v = g->ev[e];
        int64_t x = g->rp[u], y = g->rp[v], k = g->aoff[e];
        while (x < g->rp[u + 1] && y < g->rp[v + 1]) {
            if (g->ci[x] < g->ci[y]) x++;
            else if (g->ci[x] > g->ci[y]) y++;
            else { g->apex[k++] = g->ci[x]; x++; y++; }
        }
    }
    /* triangle ids: a triangle is owned by the edge of its two earliest vertices */
    g->ntri = 0;
    for (int64_t e = 0; e < m; e++)
        for (int64_t k = g->aoff[e]; k < g->aoff[e + 1]; k++)
            if (prec(g, g->ev[e], g->apex[k])) g->atri[k] = g->ntri++;
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t e = 0; e < m; e++)
        for (int64_t k = g->aoff[e]; k < g->aoff[e + 1]; k++) {
            int32_t u = g->eu[e], v = g->ev[e], w = g->apex[k];
            if (prec(g, v, w)) continue;
            /* here v is the latest of the three, so the owner edge is {u,w}
             * and its list holds v */
            int64_t f = edge_of(g, u, w);
            int64_t lo = g->aoff[f], hi = g->aoff[f + 1];
            while (lo < hi) { int64_t mid = (lo + hi) >> 1; if (g->apex[mid] < v) lo = mid + 1; else hi = mid; }
            g->atri[k] = g->atri[lo];
        }
    return 0;
}

/* triangle id of {a,b,c} (a triangle) */
static int64_t tri_id(const graph *g, int32_t a, int32_t b, int32_t c) {
    int64_t f = edge_of(g, a, b);
    int64_t lo = g->aoff[f], hi = g->aoff[f + 1];
    while (lo < hi) { int64_t mid = (lo + hi) >> 1; if (g->apex[mid] < c) lo = mid + 1; else hi = mid; }
    return g->atri[lo];
}

/* Step 3: 4-cycles (Thm 4cycle).  Every 4-cycle has a latest vertex i; with j
 * the opposite vertex, both middle vertices precede i.  So with
 * c(i,j) = #{k adjacent to i and j, k before i} the number of 4-cycles is the
 * sum over pairs j before i of C(c(i,j),2).  Per edge: a 4-cycle with top i,
 * opposite j and middles {k,k'} contains the edges ik, kj, ik', k'j, so every
 * wedge i-k-j with k in the middle set lies on c(i,j)-1 of them.
 * (Reading: the printed per-edge expression omits common neighbours that lie
 * above both endpoints of the edge; the attribution above is the plain
 * per-edge version of the same decomposition and is pinned by brute force.) */
static int four_cycles(graph *g) {
    int32_t n = g->n;
    int64_t m = g->m;
    g->c4e = (u64 *)calloc((size_t)m + 1, sizeof(u64));
    g->c4v = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    if (!g->c4e || !g->c4v) return -1;
    u128 C4 = 0;
    #pragma omp parallel reduction(+:C4)
    {
        u64 *cnt = (u64 *)calloc((size_t)n + 1, sizeof(u64));
        int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
        #pragma omp for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; i++) {
            if (SAMPLED(i)) continue;
            int64_t nt = 0;
            for (int64_t p = g->rp[i]; p < g->rp[i + 1]; p++) {
                int32_t k = g->ci[p];
                if (!prec(g, k, i)) continue;
                for (int64_t q = g->rp[k]; q < g->rp[k + 1]; q++) {
                    int32_t j = g->ci[q];
                    if (j == i || !prec(g, j, i)) continue;
                    if (cnt[j]++ == 0) touched[nt++] = j;
                }
            }
            for (int64_t t = 0; t < nt; t++) C4 += ch2(cnt[touched[t]]);
            for (int64_t p = g->rp[i]; p < g->rp[i + 1]; p++) {
                int32_t k = g->ci[p];
                if (!prec(g, k, i)) continue;
                for (int64_t q = g->rp[k]; q < g->rp[k + 1]; q++) {
                    int32_t j = g->ci[q];
                    if (j == i || !prec(g, j, i)) continue;
                    u64 c = cnt[j] - 1;
                    if (c) {
                        __atomic_fetch_add(&g->c4e[g->eid[p]], c, __ATOMIC_RELAXED);
                        __atomic_fetch_add(&g->c4e[g->eid[q]], c, __ATOMIC_RELAXED);
                    }
                }
            }
            for (int64_t t = 0; t < nt; t++) cnt[touched[t]] = 0;
        }
        free(cnt); free(touched);
    }
    g->C4 = C4;
    /* each 4-cycle through v uses two edges at v */
    for (int64_t e = 0; e < m; e++) { g->c4v[g->eu[e]] += g->c4e[e]; g->c4v[g->ev[e]] += g->c4e[e]; }
    for (int32_t v = 0; v < n; v++) g->c4v[v] /= 2;
    return 0;
}

/* Step 4: 4-cliques (Thm 4clique).  Each 4-clique has one directed diamond:
 * its earliest vertex i and latest vertex j form the diagonal, and the two
 * others lie strictly between them, adjacent to both.  For every arc i->j take
 * L = {l adjacent to i and j, i before l before j}; every adjacent pair in L
 * closes one 4-clique, found exactly once. */
static int four_cliques(graph *g) {
    int32_t n = g->n;
    int64_t m = g->m;
    g->k4e = (u64 *)calloc((size_t)m + 1, sizeof(u64));
    g->k4v = (u64 *)calloc((size_t)n + 1, sizeof(u64));
    g->k4t = (u64 *)calloc((size_t)g->ntri + 1, sizeof(u64));
    if (!g->k4e || !g->k4v || !g->k4t) return -1;
    u128 K4 = 0;
    #pragma omp parallel reduction(+:K4)
    {
        int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
        #pragma omp for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; i++)
            for (int64_t p = g->rp[i]; p < g->rp[i + 1]; p++) {
                if (SAMPLED(i)) break;
                int32_t j = g->ci[p];
                if (!prec(g, i, j)) continue;
                int64_t nl = 0;
                int64_t x = g->rp[i], y = g->rp[j];
                while (x < g->rp[i + 1] && y < g->rp[j + 1]) {
                    if (g->ci[x] < g->ci[y]) x++;
                    else if (g->ci[x] > g->ci[y]) y++;
                    else {
                        int32_t l = g->ci[x];
                        if (prec(g, i, l) && prec(g, l, j)) L[nl++] = l;
                        x++; y++;
                    }
                }
                for (int64_t s = 0; s < nl; s++)
                    for (int64_t t = s + 1; t < nl; t++) {
                        int32_t a = L[s], b = L[t];
                        if (!adjacent(g, a, b)) continue;
                        K4++;
                        int32_t q[4] = {i, a, b, j};
                        for (int u = 0; u < 4; u++) __atomic_fetch_add(&g->k4v[q[u]], 1, __ATOMIC_RELAXED);
                        for (int u = 0; u < 4; u++)
                            for (int w = u + 1; w < 4; w++)
                                __atomic_fetch_add(&g->k4e[edge_of(g, q[u], q[w])], 1, __ATOMIC_RELAXED);
                        for (int u = 0; u < 4; u++) {
                            int32_t r[3]; int c = 0;
                            for (int w = 0; w < 4; w++) if (w != u) r[c++] = q[w];
                            __atomic_fetch_add(&g->k4t[tri_id(g, r[0], r[1], r[2])], 1, __ATOMIC_RELAXED);
                        }
                    }
            }
        free(L);
    }
    g->K4 = K4;
    return 0;
}

/* ----------------------------------------------------- result structure */

/* Indices of the exported 128-bit sums.  The Python side documents each one. */
enum {
    S_N, S_M, S_W, S_T, S_TT, S_D, S_C4, S_K4,
    S_3STAR, S_EDGEPAIR,                       /* sum C(d,3); sum_e (d(u)-1)(d(v)-1) */
    S_N1, S_N2, S_N3, S_N4, S_N5, S_N6, S_N7, S_N8, S_N9, S_N10,
    S_N11, S_N12, S_N13, S_N14, S_N15, S_N16, S_N17, S_N18, S_N19, S_N20, S_N21,
    S_DP, S_DBP,          /* work counts of Thm fivevertex: directed 3-paths, directed bipyramids */
    S_COUNT
};

/* signed helpers: the cut formulas subtract shrinkage terms; every such
 * difference is a non-negative count, so it is formed once the full sum is
 * known. */
static u128 sub(u128 a, u128 b) { return a - b; }

/* Step 5-7.  Returns 0 on success.  `out` holds S_COUNT little-endian u128s. */
static int five_vertex(graph *g, u128 *S) {
    int32_t n = g->n;
    int64_t m = g->m;
    u64 *d = (u64 *)g->deg;   /* degrees are non-negative */

    u128 W = 0, s3 = 0, s4 = 0;
    for (int32_t v = 0; v < n; v++) { W += ch2(d[v]); s3 += ch3(d[v]); s4 += ch4(d[v]); }
    u128 TT = 0;                                  /* tailed triangles (Thm 4vertex-easy) */
    for (int32_t v = 0; v < n; v++) if (g->tv[v]) TT += (u128)g->tv[v] * (d[v] - 2);
    u128 D = 0;                                   /* diamonds = sum_e C(t(e),2) */
    for (int64_t e = 0; e < m; e++) D += ch2(g->te[e]);
    u128 ep = 0;
    for (int64_t e = 0; e < m; e++) ep += (u128)(d[g->eu[e]] - 1) * (d[g->ev[e]] - 1);

    S[S_N] = (u128)n; S[S_M] = (u128)m; S[S_W] = W; S[S_T] = g->T; S[S_TT] = TT; S[S_D] = D;
    S[S_C4] = g->C4; S[S_K4] = g->K4; S[S_3STAR] = s3; S[S_EDGEPAIR] = ep;

    /* ---- cut is a vertex (Thm 5cutvertex) */
    S[S_N1] = s4;
    /* N3, path of 5 vertices centred at 1: choose the centre i and two
     * neighbours j,k; each extends by one further neighbour.  Shrinkages: the
     * two ends meet (4-cycle, 4 ways), an end closes a triangle with the other
     * middle vertex (tailed triangle, 2 ways), both close (triangle, 3 ways).
     * (Reading: the printed first term sums over single neighbours; the pair
     * sum below is what the cut lemma gives for this pattern.) */
    {
        u128 acc = 0;
        #pragma omp parallel for reduction(+:acc) schedule(dynamic, 1024)
        for (int32_t i = 0; i < n; i++) {
            if (SAMPLED(i)) continue;
            u128 a = 0, b = 0;
            for (int64_t p = g->rp[i]; p < g->rp[i + 1]; p++) {
                u64 x = d[g->ci[p]] - 1;
                a += x; b += (u128)x * x;
            }
            acc += (a * a - b) / 2;
        }
        S[S_N3] = sub(sub(sub(acc, 4 * g->C4), 2 * TT), 3 * g->T);
    }
    /* N4 (cricket): a triangle at i and two more neighbours of i.
     * (Reading: printed as t(i)(d(i)-2), which is the tailed triangle.) */
    {
        u128 acc = 0;
        for (int32_t i = 0; i < n; i++) if (g->tv[i] && d[i] >= 4) acc += (u128)g->tv[i] * ch2(d[i] - 2);
        S[S_N4] = acc;
    }
    /* N7: a 4-cycle at i and one more neighbour of i; N9: two triangles at i;
     * N15: a 4-clique at i and one more neighbour. */
    {
        u128 a7 = 0, a9 = 0, a15 = 0;
        for (int32_t i = 0; i < n; i++) {
            if (d[i] >= 2) a7 += (u128)g->c4v[i] * (d[i] - 2);
            a9 += ch2(g->tv[i]);
            if (d[i] >= 3) a15 += (u128)g->k4v[i] * (d[i] - 3);
        }
        S[S_N7] = sub(a7, 2 * D);
        S[S_N9] = sub(a9, 2 * D);
        S[S_N15] = a15;
    }

    /* ---- cut is an edge (Thm 5cutedge); <i,j> ranges over both orientations */
    {
        u128 a2 = 0, a5 = 0, a6 = 0, a11 = 0, a12 = 0, a14 = 0, a19 = 0;
        for (int64_t e = 0; e < m; e++) {
            if (SAMPLED(e)) continue;
            int32_t u = g->eu[e], v = g->ev[e];
            u64 te = g->te[e];
            for (int side = 0; side < 2; side++) {
                int32_t i = side ? v : u, j = side ? u : v;
                /* N2: edge (i,j), two more neighbours at i, one more at j */
                a2 += (u128)(d[j] - 1) * ch2(d[i] - 1);
                /* N5 (triangle + 2-path tail): a triangle at j not using i, and a
                 * further neighbour of i.  (Reading: printed (d(i)-1)(d(j)-T(e)).) */
                a5 += (u128)(d[i] - 1) * (g->tv[j] - te);
                /* N11: two triangles on the edge and one more neighbour at i */
                if (d[i] >= 3) a11 += (u128)ch2(te) * (d[i] - 3);
            }
            if (te && d[u] >= 2 && d[v] >= 2) a6 += (u128)te * (d[u] - 2) * (d[v] - 2);
            a12 += (u128)g->c4e[e] * te;
            a14 += ch3(te);
            if (te >= 2) a19 += (u128)g->k4e[e] * (te - 2);
        }
        S[S_N2] = sub(a2, 2 * TT);
        S[S_N5] = sub(a5, 4 * D);
        S[S_N6] = sub(a6, 2 * D);
        S[S_N11] = a11;
        S[S_N12] = sub(a12, 4 * D);
        S[S_N14] = a14;
        S[S_N19] = a19;
    }

    /* ---- cut is a triangle (Thm 5cuttri).  Loop over triangles through the
     * triangle lists, each triangle once (from the edge of its two earliest
     * vertices).
     * N10 (diamond + pendant at a tip): for each vertex k of the triangle, a
     * second triangle on the opposite edge and a further neighbour of k.
     * Shrinkage: the pendant lands on the second apex (4-clique, 12 ways).
     * (Reading: printed with d(k)-1 and 4 K4.)
     * N16 (gem): two further triangles on two edges of t meeting at i.
     * Shrinkage: both apexes coincide (12 ways).  (Reading: printed without it.)
     * N20: two 4-cliques sharing t.  (Reading: printed with a -4 K4 term.) */
    {
        u128 a10 = 0, a16 = 0, a20 = 0;
        #pragma omp parallel for reduction(+:a10, a16, a20) schedule(dynamic, 1024)
        for (int64_t e = 0; e < m; e++) {
            if (SAMPLED(e)) continue;
            int32_t a = g->eu[e], b = g->ev[e];
            for (int64_t k = g->aoff[e]; k < g->aoff[e + 1]; k++) {
                int32_t c = g->apex[k];
                if (!prec(g, b, c)) continue;
                u64 tab = g->te[e], tac = g->te[edge_of(g, a, c)], tbc = g->te[edge_of(g, b, c)];
                /* vertex k opposite edge {i,j} */
                a10 += (u128)(tbc - 1) * (d[a] - 2) + (u128)(tac - 1) * (d[b] - 2) + (u128)(tab - 1) * (d[c] - 2);
                a16 += (u128)(tab - 1) * (tac - 1) + (u128)(tab - 1) * (tbc - 1) + (u128)(tac - 1) * (tbc - 1);
                a20 += ch2(g->k4t[g->atri[k]]);
            }
        }
        S[S_N10] = sub(a10, 12 * g->K4);
        S[S_N16] = sub(a16, 12 * g->K4);
        S[S_N20] = a20;
    }

    /* ---- cut is a pair or wedge (Thm 5cutwed, algorithm of Thm 5formula).
     * W(i,j) = common neighbours of i and j (2-step search from i);
     * D(i,j) = edges inside the common neighbourhood of i and j, i.e. diamonds
     * whose two degree-2 tips are i and j (reading of the garbled definition),
     * generated from triangles (i,k,l) followed by triangles (k,l,j).
     * N13 = sum over pairs C(W,3);  N17 = sum over pairs (W-2) D.
     * Pairs are unordered: j < i by id. */
    {
        u128 a13 = 0, a17 = 0;
        #pragma omp parallel reduction(+:a13, a17)
        {
            u64 *Wc = (u64 *)calloc((size_t)n + 1, sizeof(u64));
            u64 *Dc = (u64 *)calloc((size_t)n + 1, sizeof(u64));
            int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
            #pragma omp for schedule(dynamic, 256)
            for (int32_t i = 0; i < n; i++) {
                if (SAMPLED(i)) continue;
                int64_t nt = 0;
                for (int64_t p = g->rp[i]; p < g->rp[i + 1]; p++) {
                    int32_t k = g->ci[p];
                    for (int64_t q = g->rp[k]; q < g->rp[k + 1]; q++) {
                        int32_t j = g->ci[q];
                        if (j >= i) break;
                        if (Wc[j]++ == 0) touched[nt++] = j;
                    }
                }
                /* triangles (i,k,l) with k < l by id, then apexes j of edge (k,l) */
                for (int64_t p = g->rp[i]; p < g->rp[i + 1]; p++) {
                    int32_t k = g->ci[p];
                    int64_t eik = g->eid[p];
                    for (int64_t t = g->aoff[eik]; t < g->aoff[eik + 1]; t++) {
                        int32_t l = g->apex[t];
                        if (l <= k) continue;
                        int64_t ekl = edge_of(g, k, l);
                        for (int64_t s = g->aoff[ekl]; s < g->aoff[ekl + 1]; s++) {
                            int32_t j = g->apex[s];
                            if (j >= i) break;
                            Dc[j]++;
                        }
                    }
                }
                for (int64_t t = 0; t < nt; t++) {
                    int32_t j = touched[t];
                    a13 += ch3(Wc[j]);
                    if (Dc[j]) a17 += (u128)(Wc[j] - 2) * Dc[j];
                    Wc[j] = 0; Dc[j] = 0;
                }
            }
            free(Wc); free(Dc); free(touched);
        }
        S[S_N13] = a13;
        S[S_N17] = a17;
    }
    /* N18 (wheel, hub h): for each hub h and unordered pair {i,k} in N(h), the
     * rim vertices adjacent to h, i and k number c_h(i,k); every two of them
     * close a wheel.  Each wheel has two rim diagonals, hence the 1/2.
     * (Reading: the printed sum lacks this normalisation.)  Enumerated as
     * triangles (h,i,l) followed by triangles (h,l,k). */
    {
        u128 a18 = 0;
        #pragma omp parallel reduction(+:a18)
        {
            u64 *cnt = (u64 *)calloc((size_t)n + 1, sizeof(u64));
            int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
            #pragma omp for schedule(dynamic, 64)
            for (int32_t h = 0; h < n; h++)
                for (int64_t p = g->rp[h]; p < g->rp[h + 1]; p++) {
                    if (SAMPLED(h)) break;
                    int32_t i = g->ci[p];
                    int64_t ehi = g->eid[p];
                    int64_t nt = 0;
                    for (int64_t t = g->aoff[ehi]; t < g->aoff[ehi + 1]; t++) {
                        int32_t l = g->apex[t];
                        int64_t ehl = edge_of(g, h, l);
                        for (int64_t s = g->aoff[ehl]; s < g->aoff[ehl + 1]; s++) {
                            int32_t k = g->apex[s];
                            if (k >= i) break;
                            if (cnt[k]++ == 0) touched[nt++] = k;
                        }
                    }
                    for (int64_t t = 0; t < nt; t++) { a18 += ch2(cnt[touched[t]]); cnt[touched[t]] = 0; }
                }
            free(cnt); free(touched);
        }
        S[S_N18] = a18 / 2;
    }

    /* ---- 5-cycles (Thm 5cycle).
     * P(i,j) = directed 3-paths i <- a -> b -> j (a, b, i, j distinct).
     * Wnt(i,j) = common neighbours c of i and j with c not after both.
     * N8 = sum over ordered (i,j) of P(i,j) Wnt(i,j), minus the tuples where c
     * coincides with a or b (directed tailed triangles), which number
     * Z = sum over triangles x<y<z of d+(x) + d+(y) + d+(z) - 3.
     * (Readings: the printed sum over i before j misses the acyclic 5-cycle
     * orientations whose 3-path splits as 1+4, so ordered pairs are used; and
     * the tailed triangle correction has three directed shapes, not one.) */
    {
        u128 acc = 0, npaths = 0;
        #pragma omp parallel reduction(+:acc, npaths)
        {
            u64 *P = (u64 *)calloc((size_t)n + 1, sizeof(u64));
            u64 *Wn = (u64 *)calloc((size_t)n + 1, sizeof(u64));
            int32_t *touched = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
            #pragma omp for schedule(dynamic, 64)
            for (int32_t i = 0; i < n; i++) {
                if (SAMPLED(i)) continue;
                int64_t nt = 0;
                for (int64_t p = g->rp[i]; p < g->rp[i + 1]; p++) {
                    int32_t a = g->ci[p];
                    if (!prec(g, a, i)) continue;
                    for (int64_t q = g->rp[a]; q < g->rp[a + 1]; q++) {
                        int32_t b = g->ci[q];
                        if (b == i || !prec(g, a, b)) continue;
                        for (int64_t r = g->rp[b]; r < g->rp[b + 1]; r++) {
                            int32_t j = g->ci[r];
                            if (j == i || !prec(g, b, j)) continue;
                            npaths++;   /* one directed 3-path i <- a -> b -> j */
                            if (P[j]++ == 0) touched[nt++] = j;
                        }
                    }
                }
                if (nt) {
                    for (int64_t p = g->rp[i]; p < g->rp[i + 1]; p++) {
                        int32_t c = g->ci[p];
                        for (int64_t q = g->rp[c]; q < g->rp[c + 1]; q++) {
                            int32_t j = g->ci[q];
                            if (j == i || !P[j]) continue;
                            if (prec(g, i, c) && prec(g, j, c)) continue;
                            Wn[j]++;
                        }
                    }
                }
                for (int64_t t = 0; t < nt; t++) {
                    int32_t j = touched[t];
                    acc += (u128)P[j] * Wn[j];
                    P[j] = 0; Wn[j] = 0;
                }
            }
            free(P); free(Wn); free(touched);
        }
        u128 Z = 0;
        u64 *dp = (u64 *)calloc((size_t)n + 1, sizeof(u64));
        for (int64_t e = 0; e < m; e++) dp[g->eu[e]]++;
        for (int64_t e = 0; e < m; e++)
            for (int64_t k = g->aoff[e]; k < g->aoff[e + 1]; k++) {
                int32_t x = g->eu[e], y = g->ev[e], z = g->apex[k];
                if (!prec(g, y, z)) continue;
                Z += (u128)dp[x] + dp[y] + dp[z] - 3;
            }
        free(dp);
        S[S_N8] = sub(acc, Z);
        S[S_DP] = npaths;
    }

    /* ---- 5-cliques (Thm 5clique).  For a triangle t, the other triangles on
     * its last edge give third vertices l; those after all of t and adjacent to
     * its first vertex complete the directed configuration, and every adjacent
     * pair of them closes a 5-clique.  Each 5-clique is found once, from the
     * triangle of its three earliest vertices.  (Reading: the drawn bipyramid
     * contains a directed cycle, impossible in a DAG; the configuration used is
     * the one that makes the count exact.) */
    {
        u128 K5 = 0, pairs = 0;
        #pragma omp parallel reduction(+:K5, pairs)
        {
            int32_t *L = (int32_t *)malloc(sizeof(int32_t) * (n + 1));
            #pragma omp for schedule(dynamic, 1024)
            for (int64_t e = 0; e < m; e++) {
                if (SAMPLED(e)) continue;
                int32_t a = g->eu[e], b = g->ev[e];
                for (int64_t k = g->aoff[e]; k < g->aoff[e + 1]; k++) {
                    int32_t c = g->apex[k];
                    if (!prec(g, b, c)) continue;
                    int64_t ebc = edge_of(g, b, c);
                    int64_t nl = 0;
                    for (int64_t s = g->aoff[ebc]; s < g->aoff[ebc + 1]; s++) {
                        int32_t l = g->apex[s];
                        if (prec(g, c, l) && adjacent(g, a, l)) L[nl++] = l;
                    }
                    pairs += (u128)nl * (nl > 0 ? nl - 1 : 0) / 2;   /* directed bipyramids tried */
                    for (int64_t x = 0; x < nl; x++)
                        for (int64_t y = x + 1; y < nl; y++)
                            if (adjacent(g, L[x], L[y])) K5++;
                }
            }
            free(L);
        }
        S[S_N21] = K5;
        S[S_DBP] = pairs;
    }
    return 0;
}

static void release(graph *g) {
    free(g->deg); free(g->rank); free(g->eid); free(g->eu); free(g->ev);
    free(g->tv); free(g->te); free(g->aoff); free(g->apex); free(g->atri);
    free(g->c4e); free(g->c4v); free(g->k4e); free(g->k4v); free(g->k4t);
}

int oracle_num_sums(void) { return S_COUNT; }

/* Full pipeline.  k = 4 stops after the 4-vertex quantities (the 5-vertex
 * entries are left zero).  `order_rank` may be NULL (degree order).  Optional
 * per-item outputs (any may be NULL): t(v), C4(v), K4(v) [n] and, per arc of
 * the input CSR, t(e), C4(e), K4(e) of that arc's edge [2m].
 * out: S_COUNT x 2 uint64 (lo, hi).  Returns 0 or -1 (allocation failure). */
int oracle_run(int32_t n, const int32_t *rp, const int32_t *ci, int k, const int64_t *order_rank,
               int threads, uint64_t *out,
               uint64_t *tv, uint64_t *c4v, uint64_t *k4v,
               uint64_t *te_arc, uint64_t *c4e_arc, uint64_t *k4e_arc,
               int sample, double *seconds /* [2]: setup + triangles, the rest; may be NULL */) {
    if (threads > 0) omp_set_num_threads(threads);
    g_sample = sample > 1 ? sample : 1;
    graph g;
    u128 S[S_COUNT];
    memset(S, 0, sizeof(S));
    double t0 = omp_get_wtime();
    int rc = setup(&g, n, rp, ci, order_rank);
    if (!rc) rc = triangles(&g);
    double t1 = omp_get_wtime();
    if (!rc) rc = four_cycles(&g);
    if (!rc) rc = four_cliques(&g);
    if (!rc) {
        if (k >= 5) rc = five_vertex(&g, S);
        else {
            /* 4-vertex sums only */
            u64 *d = (u64 *)g.deg;
            u128 W = 0, s3 = 0, TT = 0, D = 0, ep = 0;
            for (int32_t v = 0; v < n; v++) { W += ch2(d[v]); s3 += ch3(d[v]); if (g.tv[v]) TT += (u128)g.tv[v] * (d[v] - 2); }
            for (int64_t e = 0; e < g.m; e++) { D += ch2(g.te[e]); ep += (u128)(d[g.eu[e]] - 1) * (d[g.ev[e]] - 1); }
            S[S_N] = (u128)n; S[S_M] = (u128)g.m; S[S_W] = W; S[S_T] = g.T; S[S_TT] = TT; S[S_D] = D;
            S[S_C4] = g.C4; S[S_K4] = g.K4; S[S_3STAR] = s3; S[S_EDGEPAIR] = ep;
        }
    }
    double t2 = omp_get_wtime();
    if (seconds) { seconds[0] = t1 - t0; seconds[1] = t2 - t1; }
    g_sample = 1;
    if (!rc) {
        for (int s = 0; s < S_COUNT; s++) { out[2 * s] = (uint64_t)S[s]; out[2 * s + 1] = (uint64_t)(S[s] >> 64); }
        for (int32_t v = 0; v < n; v++) {
            if (tv) tv[v] = g.tv[v];
            if (c4v) c4v[v] = g.c4v[v];
            if (k4v) k4v[v] = g.k4v[v];
        }
        for (int64_t p = 0; p < (int64_t)rp[n]; p++) {
            if (te_arc) te_arc[p] = g.te[g.eid[p]];
            if (c4e_arc) c4e_arc[p] = g.c4e[g.eid[p]];
            if (k4e_arc) k4e_arc[p] = g.k4e[g.eid[p]];
        }
    }
    release(&g);
    return rc;
}
