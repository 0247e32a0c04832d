// 4-cliques per triangle (Thm 4clique) and 5-cliques (Thm 5clique).
//
// K4(t) for every triangle t = {a<b<c} is the number of common neighbours of
// a, b and c.  The triangle list of arc (a,b) is the common neighbourhood of
// a and b, stored as positions in the row of a; the list of arc (a,c) is the
// common neighbourhood of a and c in the same coordinates.  One wave takes
// an edge (a,b), marks its list in an LDS bitmap over the row of a, and each
// lane counts, for one triangle (a,b,c) with c after b, the marked entries of
// the list of (a,c).  From K4(t): K4(e) (scattered to the three edges),
// sum C(K4(t),2) (pattern 20), the triangle-cut sums of patterns 10 and 16 and
// the 5-cycle correction term of each triangle.
//
// 5-cliques: a 5-clique is found once, from its earliest vertex a, as a
// 4-clique of H_a = G[N+(a)].  Direct count: for every out-arc (c,x) a bitmap
// over the positions of N+(c) marks N+(c) & N+(x) (read off the triangle list
// of (c,x)); with these rows, for a and b<c<x in N+(a):
//   S = row(a,b) & row(a,c)           (common out-neighbours of a, b, c)
//   5-cliques += popcount(S & row(a,x)) for every x in S.
// That visits every 4-clique of H_a, which is too much when H_a is nearly
// complete (hub cores of heavy-tailed graphs).  Such a vertex is counted
// through the complement Hc of H_a instead: a 4-set of H_a is a clique when
// it spans no edge of Hc, so by the sign rule of the inverse of A (App. B)
// applied to the empty pattern, K4(H_a) = sum over the 11 four-vertex
// patterns j of (-1)^e(j) N_j(Hc), the non-induced counts of Hc given by
// the 4-vertex formulas (Thm 4vertex-easy, Thm 4cycle, Thm 4clique) with
// the disconnected patterns in closed form (App. A).
#include <vector>
#include "device.h"
#include "ctx.h"
#include "tiles.h"

#define BM_WORDS 512   // LDS bitmap per wave: rows of up to 16384 vertices

// merge-count of two sorted id lists (rows too long for the bitmap)
__device__ inline uint32_t count_common(const int32_t *av, const int32_t *adj, const uint32_t *aa, int64_t x,
                                        int64_t xe, int64_t y, int64_t ye, uint64_t &nvis) {
    const int64_t x0 = x, y0 = y;
    uint32_t c = 0;
    while (x < xe && y < ye) {
        const int32_t p = apex_at(av, adj, aa, x), q = apex_at(av, adj, aa, y);
        c += (p == q);
        x += (p <= q);
        y += (q <= p);
    }
    nvis += (x - x0) + (y - y0);
    return c;
}

template <bool IDS>
__global__ void __launch_bounds__(256) k_k4_triangles(int64_t m, const int32_t *off, const int32_t *adj,
                                                      const int32_t *split, const int32_t *rev,
                                                      const int32_t *arc_eid, const int32_t *earc,
                                                      const int32_t *elo, const uint32_t *te, const int64_t *aoff,
                                                      const uint32_t *aa, const int32_t *av,
                                                      unsigned long long *k4e, GMap gm, int small,
                                                      unsigned long long *acc, unsigned long long *visits,
                                                      const uint8_t *kdense) {
    __shared__ uint32_t bm_all[4][BM_WORDS];
    __shared__ u128 red[5 * 4];
    __shared__ int64_t wsa[4][64];
    __shared__ int32_t wse[4][64], wsi[4][64];
    __shared__ uint32_t wcn[4][64];
    const int ids[5] = {AC_K4X4, AC_N20, AC_N10, AC_N16, AC_Z};
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    uint32_t *bm = bm_all[wid];
    for (int w = lane; w < BM_WORDS; w += 64) bm[w] = 0;
    wave_sync();
    const int64_t wave = (int64_t)blockIdx.x * 4 + wid;
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    // one graph: edges strided over the waves; a batch: one contiguous block
    // of edges per wave, so that its per-graph sums change graph rarely
    const bool batched = gm.vg != nullptr;
    const int64_t per = (m + nwaves - 1) / nwaves;
    const int64_t e_first = batched ? wave * per : wave;
    const int64_t e_end = batched ? (e_first + per < m ? e_first + per : m) : m;
    const int64_t e_step = batched ? 1 : nwaves;
    u128 s[5] = {0, 0, 0, 0, 0};
    int gcur = -1;
    uint64_t nvis = 0;
    // the terms of triangle (a,b,c) whose list entry is k in the list of edge
    // e = (a,b) (c after b), given K4 of the triangle
    auto triangle_terms = [&](int64_t e, int32_t a, int32_t b, int64_t l0, int64_t r0, int64_t k, uint32_t k4) {
        const int32_t cc = apex_at<IDS>(av, adj, aa, k);
        const int32_t pac = (int32_t)aa[k];                  // arc (a,c) in row a
        const int32_t pbc = (int32_t)aa[r0 + (k - l0)];      // arc (b,c) in row b
        const int32_t eac = arc_eid[pac], ebc = arc_eid[pbc];
        const uint64_t tab = te[e], tac = te[eac], tbc = te[ebc];
        const uint64_t da = off[a + 1] - off[a], db = off[b + 1] - off[b], dc = off[cc + 1] - off[cc];
        const uint64_t dpa = off[a + 1] - split[a], dpb = off[b + 1] - split[b], dpc = off[cc + 1] - split[cc];
        if (k4) {
            atomicAdd(&k4e[e], (unsigned long long)k4);
            atomicAdd(&k4e[eac], (unsigned long long)k4);
            atomicAdd(&k4e[ebc], (unsigned long long)k4);
        }
        s[0] += k4;
        s[1] += c2(k4);
        s[2] += (u128)(tbc - 1) * (da - 2) + (u128)(tac - 1) * (db - 2) + (u128)(tab - 1) * (dc - 2);
        s[3] += (u128)(tab - 1) * (tac - 1) + (u128)(tab - 1) * (tbc - 1) + (u128)(tac - 1) * (tbc - 1);
        s[4] += dpa + dpb + dpc - 3;
    };
    if (small) {
        // a batch of small graphs, whose lists are short: the triangles of 64
        // consecutive edges of one graph are numbered in one run, a lane
        // takes one and merges the two sorted lists (a,b) and (a,c) for K4
        for (int64_t eb = e_first; eb < e_end;) {
            const int g0 = gm.graph(elo[eb]);
            const int64_t e = eb + lane;
            const bool in = e < e_end && gm.graph(elo[e < e_end ? e : eb]) == g0;
            const uint64_t inb = __ballot(in);
            const int nb = inb == ~0ull ? 64 : __ffsll((long long)~inb) - 1;   // edges of this run
            if (g0 != gcur) {
                if (gcur >= 0) wave_flush_runs<5>(s, gcur, acc, ACC_STRIDE, ids);
                gcur = g0;
            }
            int cnt = 0;
            int64_t lo = 0;
            if (lane < nb) {
                const int32_t p = earc[e];
                const int64_t l0 = aoff[p], l1 = aoff[p + 1];
                int64_t hi = l1;   // first apex after b = adj[p]: the first arc of row a after p
                lo = l0;
                while (lo < hi) { int64_t mid = (lo + hi) >> 1; if (aa[mid] <= (uint32_t)p) lo = mid + 1; else hi = mid; }
                cnt = (int)(l1 - lo);
            }
            int incl = cnt;
            for (int o = 1; o < 64; o <<= 1) {
                const int y = __shfl_up(incl, o);
                if (lane >= o) incl += y;
            }
            const int total = __shfl(incl, 63);
            wsa[wid][lane] = lo;
            wsi[wid][lane] = incl;
            wave_sync();
            int y = 0;
            for (int t = lane; t < total; t += 64) {
                while (wsi[wid][y] <= t) y++;
                const int64_t ey = eb + y;
                const int32_t p = earc[ey];
                const int32_t a = elo[ey], b = adj[p];
                const int64_t l0 = aoff[p], l1 = aoff[p + 1];
                const int64_t k = wsa[wid][y] + (t - (wsi[wid][y] - (int)(l1 - wsa[wid][y])));
                const int32_t pac = (int32_t)aa[k];
                int64_t x = l0, q = aoff[pac];
                const int64_t qe = aoff[pac + 1];
                uint32_t k4 = 0;
                while (x < l1 && q < qe) {   // positions in the row of a, both sorted
                    const uint32_t u = aa[x], v = aa[q];
                    k4 += u == v;
                    x += u <= v;
                    q += v <= u;
                }
                nvis += (uint64_t)(l1 - l0) + (uint64_t)(qe - aoff[pac]);
                triangle_terms(ey, a, b, l0, aoff[rev[p]], k, k4);
            }
            wave_sync();   // the run arrays are rewritten by the next run
            eb += nb;
        }
        if (gcur >= 0) wave_flush_runs<5>(s, gcur, acc, ACC_STRIDE, ids);
        flush_count(nvis, visits);
        return;
    }
    for (int64_t e = e_first; e < e_end; e += e_step) {
        if (batched) {
            const int g = gm.graph(elo[e]);   // wave-uniform
            if (g != gcur) {
                if (gcur >= 0) wave_flush_runs<5>(s, gcur, acc, ACC_STRIDE, ids);
                gcur = g;
            }
        }
        const int32_t p = earc[e];
        const int64_t l0 = aoff[p], l1 = aoff[p + 1];
        if (l1 == l0) continue;
        const int32_t a = elo[e], b = adj[p];
        if (kdense && kdense[a]) continue;   // its triangles take the product (below)
        int64_t lo = l0, hi = l1;   // first apex after b: the list holds arcs (a,c) of row a, after p
        while (lo < hi) { int64_t mid = (lo + hi) >> 1; if (aa[mid] <= (uint32_t)p) lo = mid + 1; else hi = mid; }
        if (lo == l1) continue;
        const int32_t oa = off[a];
        const int32_t da_i = off[a + 1] - oa;
        const bool use_bm = da_i <= BM_WORDS * 32;
        if (use_bm) {
            for (int64_t k = l0 + lane; k < l1; k += 64) {
                int32_t pos = (int32_t)aa[k] - oa;
                atomicOr(&bm[pos >> 5], 1u << (pos & 31));
            }
            wave_sync();
        }
        const int64_t r0 = aoff[rev[p]];
        const uint64_t da = da_i, db = off[b + 1] - off[b];
        const uint64_t dpa = off[a + 1] - split[a], dpb = off[b + 1] - split[b];
        const uint64_t tab = te[e];
        // 64 triangles (a,b,c), c after b, at a time: lane = triangle; K4 of
        // the triangle = entries of list(a,c) marked in the bitmap, counted
        // by the whole wave across the 64 lists
        for (int64_t kb = lo; kb < l1; kb += 64) {
            const int64_t k = kb + lane;
            const bool ok = k < l1;
            int32_t cc = 0, pac = 0, pbc = 0;
            int64_t q0 = 0, q1 = 0;
            if (ok) {
                cc = apex_at<IDS>(av, adj, aa, k);
                pac = (int32_t)aa[k];                  // arc (a,c) in row a
                pbc = (int32_t)aa[r0 + (k - l0)];      // arc (b,c) in row b
                q0 = aoff[pac];
                q1 = aoff[pac + 1];
            }
            uint32_t k4 = 0;
            if (use_bm) {
                k4 = wave_count(q0, q1, wsa[wid], wse[wid], wsi[wid], wcn[wid],
                                [&](int64_t q) { return (int32_t)aa[q] - oa; },
                                [&](int32_t pos) { return (bm[pos >> 5] >> (pos & 31)) & 1u; });
                nvis += q1 - q0;
            } else if (ok) {
                k4 = count_common(av, adj, aa, l0, l1, q0, q1, nvis);
            }
            if (!ok) continue;
            const int32_t eac = arc_eid[pac], ebc = arc_eid[pbc];
            const uint64_t tac = te[eac], tbc = te[ebc];
            const uint64_t dc = off[cc + 1] - off[cc], dpc = off[cc + 1] - split[cc];
            if (k4) {
                atomicAdd(&k4e[e], (unsigned long long)k4);
                atomicAdd(&k4e[eac], (unsigned long long)k4);
                atomicAdd(&k4e[ebc], (unsigned long long)k4);
            }
            s[0] += k4;
            s[1] += c2(k4);
            s[2] += (u128)(tbc - 1) * (da - 2) + (u128)(tac - 1) * (db - 2) + (u128)(tab - 1) * (dc - 2);
            s[3] += (u128)(tab - 1) * (tac - 1) + (u128)(tab - 1) * (tbc - 1) + (u128)(tac - 1) * (tbc - 1);
            s[4] += dpa + dpb + dpc - 3;
        }
        if (use_bm) {
            wave_sync();
            for (int64_t k = l0 + lane; k < l1; k += 64) {
                int32_t pos = (int32_t)aa[k] - oa;
                bm[pos >> 5] = 0;
            }
            wave_sync();
        }
    }
    if (batched) wave_flush_runs<5>(s, gcur, acc, ACC_STRIDE, ids);
    else block_flush_u128<5>(s, red, acc, ids);
    flush_count(nvis, visits);
}

// ------------------------------------------------- 4-cliques, dense rows
//
// For a vertex a, K4 of every triangle (a,b,c) with a earliest is
// |N(a) & N(b) & N(c)| = (B_a B_a^T)(b,c), B_a the 0/1 matrix with a row per
// out-neighbour b (its position in N+(a)) and a column per neighbour w of a
// (its position in N(a)): B_a(b,w) = [b ~ w], read off the triangle list of
// arc (a,b).  When N+(a) is large and dense (the core of a heavy-tailed
// graph) the walk of Thm 4clique visits t(a,c) entries per triangle while
// the product costs d+(a)^2 d(a) / 2 multiply-adds in all; such vertices
// take the product on the matrix cores (tiles.h) and their triangles read K4 from
// it.  A batch of them: vertex va[q], B_a at bo[q] (dpp[q] x dk[q] bytes:
// d+ rounded up to HUB_T rows, d rounded up to HUB_K columns), C_a at co[q]
// (dpp[q] x dpp[q] int32, the tiles on and above the diagonal), rows
// numbered from rp[q], out-arcs from ap[q], product patches from pp[q].

// row i of B_a (one workgroup per row)
__global__ void __launch_bounds__(256) k_k4_rows(const int32_t *off, const int32_t *split, const int64_t *aoff,
                                                 const uint32_t *aa, int32_t nq, const int32_t *va,
                                                 const int32_t *dpp, const int32_t *dk, const int64_t *rp,
                                                 const int64_t *bo, uint8_t *yb) {
    extern __shared__ uint32_t rowb[];
    int lo = 0, hi = nq - 1;   // last vertex whose first row is <= blockIdx.x
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (rp[mid] <= (int64_t)blockIdx.x) lo = mid; else hi = mid - 1;
    }
    const int32_t a = va[lo], kb = dk[lo];
    const int64_t i = (int64_t)blockIdx.x - rp[lo];
    const int32_t oa = off[a], sa = split[a], dplus = off[a + 1] - sa;
    for (int q = threadIdx.x; q < kb / 4; q += blockDim.x) rowb[q] = 0;
    __syncthreads();
    if (i < dplus) {
        const int64_t x0 = aoff[sa + i], x1 = aoff[sa + i + 1];
        for (int64_t x = x0 + threadIdx.x; x < x1; x += blockDim.x) {
            fp4_set_one(rowb, (int32_t)aa[x] - oa);   // column: the position of w in N(a)
        }
    }
    __syncthreads();
    uint4 *dst = (uint4 *)(yb + bo[lo] + i * (int64_t)kb);
    const uint4 *src = (const uint4 *)rowb;
    for (int q = threadIdx.x; q < kb / 16; q += blockDim.x) dst[q] = src[q];
}

// C_a = B_a B_a^T on the tiles on and above the diagonal
__global__ void __launch_bounds__(64 * HUB_WAVES) k_k4_gemm(const uint8_t *yb, int32_t nq, const int32_t *dpp,
                                                 const int32_t *dk, const int64_t *bo, const int64_t *co,
                                                 const int32_t *pp, int32_t *cm) {
    extern __shared__ __attribute__((aligned(16))) uint8_t hub_lds[];
    const int local = (int)(blockIdx.x >> 3), xcd = (int)(blockIdx.x & 7);
    const int P = (local / (HUB_PR * HUB_PC)) * 8 + xcd;
    if (P >= pp[nq]) return;   // the whole workgroup leaves
    int lo = 0, hi = nq - 1;   // vertex of patch P
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (pp[mid] <= P) lo = mid; else hi = mid - 1;
    }
    const int32_t rows = dpp[lo];
    int ti, tj;
    if (!hub_patch_tile(rows / HUB_T, P - pp[lo], local % (HUB_PR * HUB_PC), &ti, &tj)) return;
    hub_v4f cacc[8][HUB_BC];
    hub_tile((lds_u8 *)hub_lds, yb + bo[lo], dk[lo], ti, tj, cacc);
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    int32_t *out = cm + co[lo];
#pragma unroll
    for (int a = 0; a < 8; a++)
#pragma unroll
        for (int b = 0; b < HUB_BC; b++)
#pragma unroll
            for (int r = 0; r < 4; r++) {
                const int64_t i = (int64_t)ti * HUB_T + hub_acc_row(wid, lane, a, r);
                const int64_t j = (int64_t)tj * HUB_T + hub_acc_col(wid, lane, b);
                out[i * rows + j] = (int32_t)cacc[a][b][r];   // exact integer count
            }
}

// The triangles (a,b,c), c after b, of the batch's vertices with K4 read
// from C_a, and every per-triangle term of the walk kernel: one wave per
// out-arc (a,b), a lane per triangle.
template <bool IDS>
__global__ void __launch_bounds__(256) k_k4_lookup(const int32_t *off, const int32_t *adj, const int32_t *split,
                                                   const int32_t *rev, const int32_t *arc_eid, const uint32_t *te,
                                                   const int64_t *aoff, const uint32_t *aa, const int32_t *av,
                                                   int32_t nq, const int32_t *va, const int32_t *dpp,
                                                   const int64_t *ap, const int64_t *co, const int32_t *cm,
                                                   unsigned long long *k4e, unsigned long long *acc,
                                                   unsigned long long *visits) {
    __shared__ u128 red[5 * 4];
    const int ids[5] = {AC_K4X4, AC_N20, AC_N10, AC_N16, AC_Z};
    const int lane = threadIdx.x & 63;
    const int64_t w0 = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6, nwv = ((int64_t)gridDim.x * blockDim.x) >> 6;
    u128 s[5] = {0, 0, 0, 0, 0};
    uint64_t nvis = 0;
    for (int64_t w = w0; w < ap[nq]; w += nwv) {
        int lo = 0, hi = nq - 1;   // vertex of out-arc w
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (ap[mid] <= w) lo = mid; else hi = mid - 1;
        }
        const int32_t a = va[lo], rows = dpp[lo];
        const int64_t i = w - ap[lo];
        const int32_t sa = split[a], p = sa + (int32_t)i, b = adj[p];
        const int64_t l0 = aoff[p], l1 = aoff[p + 1];
        int64_t kl = l0, kh = l1;   // first apex after b: the first arc of row a after p
        while (kl < kh) { const int64_t mid = (kl + kh) >> 1; if (aa[mid] <= (uint32_t)p) kl = mid + 1; else kh = mid; }
        if (kl == l1) continue;
        nvis += (uint64_t)(l1 - kl);
        const int32_t e = arc_eid[p];
        const int64_t r0 = aoff[rev[p]];
        const uint64_t da = off[a + 1] - off[a], db = off[b + 1] - off[b];
        const uint64_t dpa = off[a + 1] - sa, dpb = off[b + 1] - split[b];
        const uint64_t tab = te[e];
        const int32_t *crow = cm + co[lo] + i * rows;
        uint64_t k4sum = 0;
        for (int64_t k = kl + lane; k < l1; k += 64) {
            const int32_t cc = apex_at<IDS>(av, adj, aa, k);
            const int32_t pac = (int32_t)aa[k];                  // arc (a,c) in row a
            const int32_t pbc = (int32_t)aa[r0 + (k - l0)];      // arc (b,c) in row b
            const uint32_t k4 = (uint32_t)crow[pac - sa];
            const int32_t eac = arc_eid[pac], ebc = arc_eid[pbc];
            const uint64_t tac = te[eac], tbc = te[ebc];
            const uint64_t dc = off[cc + 1] - off[cc], dpc = off[cc + 1] - split[cc];
            if (k4) {
                atomicAdd(&k4e[eac], (unsigned long long)k4);
                atomicAdd(&k4e[ebc], (unsigned long long)k4);
            }
            k4sum += k4;
            s[0] += k4;
            s[1] += c2(k4);
            s[2] += (u128)(tbc - 1) * (da - 2) + (u128)(tac - 1) * (db - 2) + (u128)(tab - 1) * (dc - 2);
            s[3] += (u128)(tab - 1) * (tac - 1) + (u128)(tab - 1) * (tbc - 1) + (u128)(tac - 1) * (tbc - 1);
            s[4] += dpa + dpb + dpc - 3;
        }
        // the edge (a,b) takes the K4 of all its triangles after b at once
        const uint64_t ksum = wave_sum_u64(k4sum);
        if (lane == 0 && ksum) atomicAdd(&k4e[e], (unsigned long long)ksum);
    }
    block_flush_u128<5>(s, red, acc, ids);
    flush_count(nvis, visits);
}

// candidates: out-degree at least dmin, degree at most K4_MAX_DEG (a row of
// B_a in LDS); listed as (vertex, d+, d)
#define K4_MAX_DEG 65536
__global__ void k_k4_pick(int32_t n, const int32_t *off, const int32_t *split, int32_t dmin, int32_t *list,
                          int *cnt) {
    for (int32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < n; a += gridDim.x * blockDim.x) {
        const int32_t dp = off[a + 1] - split[a], d = off[a + 1] - off[a];
        if (dp >= dmin && d <= K4_MAX_DEG) {
            const int q = atomicAdd(cnt, 1);
            list[3 * q] = a;
            list[3 * q + 1] = dp;
            list[3 * q + 2] = d;
        }
    }
}

__global__ void k_k4_flags(int32_t nq, const int32_t *list, uint8_t *flag) {
    for (int32_t q = blockIdx.x * blockDim.x + threadIdx.x; q < nq; q += gridDim.x * blockDim.x) flag[list[q]] = 1;
}

// ---------------------------------------------------------------- 5-cliques

// Vertices of the direct pass with at most `light` (<= 64) out-neighbours
// (one-word rows) are counted a wave each, lane = b, after the units of the
// others; heavier ones with rows of at most `wave_words` (<= K5_WAVE_WORDS)
// words take a wave per b.
#define K5_LIGHT 64
#define K5_LIGHT_RUN 32    // consecutive light vertices per wave at a time
#define K5_WAVE_WORDS 8    // most words of a row held in registers by the wave path
#define K5_DENSE_HMAX 4096 // largest out-degree counted through the complement

// Classification, one wave per vertex a with h = d+(a): e(H_a) = sum over b
// in N+(a) of the apexes of list(a,b) after b (the entries whose arc index
// in the row of a lies after b's).  a is dense when light < h <=
// K5_DENSE_HMAX and e(H_a) >= dense_pct % of C(h,2); a dense vertex gets no
// rows (len = 0) and is appended to the dense list.
__global__ void k_k5_classify(int32_t n, const int32_t *off, const int32_t *split, const int64_t *aoff,
                              const uint32_t *aa, int light, int dense_pct, int64_t *len, int32_t *dlist,
                              int *ndense) {
    const int lane = threadIdx.x & 63;
    const int32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int32_t a = wave; a < n; a += nwaves) {
        const int32_t sa = split[a], ea = off[a + 1];
        const int64_t dp = ea - sa;
        bool dense = false;
        if (dp > light && dp <= K5_DENSE_HMAX && dense_pct <= 100) {
            uint64_t e = 0;
            for (int32_t p = sa + lane; p < ea; p += 64) {
                int64_t lo = aoff[p], hi = aoff[p + 1];
                const int64_t l1 = hi;
                while (lo < hi) { const int64_t mid = (lo + hi) >> 1; if ((int32_t)aa[mid] <= p) lo = mid + 1; else hi = mid; }
                e += (uint64_t)(l1 - lo);
            }
            e = wave_sum_u64(e);
            dense = 200 * e >= (uint64_t)dense_pct * (uint64_t)(dp * (dp - 1));
        }
        if (lane == 0) {
            len[a] = dense ? 0 : dp * ((dp + 63) >> 6);
            if (dense) dlist[atomicAdd(ndense, 1)] = a;
        }
    }
}

// one wave per vertex c, a lane per out-arc (c,x): the row of (c,x) marks
// the apexes of its triangle list that come after x, by position in N+(c)
// (entries with an arc index in the row of c after x's, a suffix of the
// list).  Dense vertices have no rows.
__global__ void k_ob_rows(int32_t n, const int32_t *off, const int32_t *split, const int64_t *aoff,
                          const uint32_t *aa, const int64_t *ob_off, unsigned long long *ob) {
    const int lane = threadIdx.x & 63;
    const int32_t wave = (blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int32_t nwaves = (gridDim.x * blockDim.x) >> 6;
    for (int32_t c = wave; c < n; c += nwaves) {
        if (ob_off[c + 1] == ob_off[c]) continue;
        const int32_t sc = split[c], ec = off[c + 1];
        const int32_t dp = ec - sc;
        const int wc = (dp + 63) >> 6;
        for (int32_t p = sc + lane; p < ec; p += 64) {
            unsigned long long *row = ob + ob_off[c] + (int64_t)(p - sc) * wc;
            const int64_t k1 = aoff[p + 1];
            int64_t k = aoff[p], hi = k1;
            while (k < hi) { const int64_t mid = (k + hi) >> 1; if ((int32_t)aa[mid] <= p) k = mid + 1; else hi = mid; }
            for (; k < k1; k++) {
                int32_t pos = (int32_t)aa[k] - sc;
                row[pos >> 6] |= 1ull << (pos & 63);
            }
        }
    }
}

__device__ inline int nth_set_bit(const unsigned long long *row, int words, int r) {
    for (int w = 0; w < words; w++) {
        unsigned long long x = row[w];
        int c = __popcll(x);
        if (r < c) {
            for (int t = 0; t < r; t++) x &= x - 1;
            return w * 64 + __ffsll((long long)x) - 1;
        }
        r -= c;
    }
    return -1;
}

// Work of vertex a grows like d+(a)^3 / 64 word operations, so a is split
// into units of ch out-neighbours b, ch = min(256, 2^lg / d+(a)^2) (lg = 20
// unless tuned): a hub spreads over many workgroups.
__device__ inline int k5_chunk(int32_t dp, int lg) {
    const int64_t q = ((int64_t)1 << lg) / ((int64_t)dp * dp);
    return q >= 256 ? 256 : (q < 1 ? 1 : (int)q);
}

// units of the direct pass: none for light vertices (their own loop) and
// for dense ones (no rows)
__global__ void k_k5_units(int32_t n, const int32_t *off, const int32_t *split, const int64_t *ob_off, int lg,
                           int light, int64_t *len) {
    for (int32_t a = blockIdx.x * blockDim.x + threadIdx.x; a < n; a += gridDim.x * blockDim.x) {
        const int32_t dp = off[a + 1] - split[a];
        const bool rows = ob_off[a + 1] > ob_off[a];
        len[a] = dp <= light || !rows ? 0 : (dp + k5_chunk(dp, lg) - 1) / k5_chunk(dp, lg);
    }
}

// one workgroup per unit (a, block of out-neighbours b); items = pairs
// (b, c) with c in row(a,b); units are taken latest vertex first
__global__ void __launch_bounds__(256) k_k5(int32_t n, const int32_t *off, const int32_t *split,
                                            const int64_t *ob_off, const unsigned long long *ob,
                                            const int64_t *uoff, const int32_t *uown, int64_t nunits, int lg,
                                            int light, int wave_words, int *task, GMap gm,
                                            unsigned long long *acc, unsigned long long *visits,
                                            unsigned long long *dbp_out) {
    __shared__ int pref[257], tmp[8];
    __shared__ int64_t beg[257];
    __shared__ int64_t s_u;
    __shared__ int32_t s_a;
    __shared__ u128 red[4];
    const int ids[1] = {AC_K5};
    u128 k5[1] = {0};
    int gcur = -1;
    uint64_t nvis = 0;
    // directed bipyramids (work counter of Thm 5clique): C(|S|,2) for each
    // triangle a < b < c, S its common out-neighbours
    uint64_t dbp = 0;
    for (;;) {
        if (threadIdx.x == 0) {
            const int64_t t = atomicAdd(task, 1);
            s_u = t < nunits ? nunits - 1 - t : -1;
            if (s_u >= 0) s_a = uown[s_u];
        }
        __syncthreads();
        const int64_t u = s_u;
        const int32_t a = s_a;
        __syncthreads();   // s_u, s_a are read by every thread before they are taken again
        if (u < 0) break;
        block_switch_graph<1>(k5, gcur, gm.graph(a), red, acc, ACC_STRIDE, ids);
        const int32_t dpa = off[a + 1] - split[a];
        const int ch = k5_chunk(dpa, lg);
        const int32_t ib0 = (int32_t)(u - uoff[a]) * ch;
        const int32_t ib1 = ib0 + ch < dpa ? ib0 + ch : dpa;
        const int wa = (dpa + 63) >> 6;
        const unsigned long long *rows = ob + ob_off[a];
        if (wa <= wave_words) {
            // rows of at most wave_words words: one wave per b, the row of
            // b in registers; lane l takes the c = 64 w + l of row(a,b), ANDs
            // the two rows once and counts, for each x of the result, the y
            // adjacent to all of b, c, x
            const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nwv = blockDim.x >> 6;
            for (int ib = ib0 + wid; ib < ib1; ib += nwv) {
                const unsigned long long *rb = rows + (int64_t)ib * wa;
                unsigned long long bw[K5_WAVE_WORDS];
#pragma unroll
                for (int w = 0; w < K5_WAVE_WORDS; w++) bw[w] = w < wa ? rb[w] : 0ull;
                uint64_t cnt = 0;
#pragma unroll
                for (int w = 0; w < K5_WAVE_WORDS; w++) {
                    if (w >= wa || !((bw[w] >> lane) & 1ull)) continue;
                    const unsigned long long *rc = rows + (int64_t)(w * 64 + lane) * wa;
                    unsigned long long sc[K5_WAVE_WORDS];
#pragma unroll
                    for (int w2 = 0; w2 < K5_WAVE_WORDS; w2++) sc[w2] = w2 < wa ? (bw[w2] & rc[w2]) : 0ull;
                    uint32_t ns = 0;
#pragma unroll
                    for (int w2 = 0; w2 < K5_WAVE_WORDS; w2++) ns += (uint32_t)__popcll(sc[w2]);
                    dbp += c2(ns);
#pragma unroll
                    for (int w2 = 0; w2 < K5_WAVE_WORDS; w2++) {
                        unsigned long long xs = sc[w2];
                        while (xs) {
                            const int x = w2 * 64 + __ffsll((long long)xs) - 1;
                            xs &= xs - 1;
                            const unsigned long long *rx = rows + (int64_t)x * wa;
#pragma unroll
                            for (int w3 = 0; w3 < K5_WAVE_WORDS; w3++)
                                if (w3 < wa) cnt += (uint64_t)__popcll(sc[w3] & rx[w3]);
                            nvis += wa;
                        }
                    }
                }
                k5[0] += cnt;
            }
            continue;
        }
        for (int ib = ib0; ib < ib1; ib += blockDim.x) {
            int i = ib + threadIdx.x;
            int len = 0;
            if (i < ib1)
                for (int w = 0; w < wa; w++) len += __popcll(rows[(int64_t)i * wa + w]);
            lbs_batch(0, len, pref, beg, tmp, [&](int s, int64_t r) {
                const unsigned long long *rb = rows + (int64_t)(ib + s) * wa;
                const int j = nth_set_bit(rb, wa, (int)r);
                const unsigned long long *rc = rows + (int64_t)j * wa;
                uint32_t ns = 0;
                for (int w = 0; w < wa; w++) {
                    unsigned long long sw = rb[w] & rc[w];
                    ns += (uint32_t)__popcll(sw);
                    while (sw) {
                        const int x = w * 64 + __ffsll((long long)sw) - 1;
                        sw &= sw - 1;
                        const unsigned long long *rx = rows + (int64_t)x * wa;
                        for (int w2 = 0; w2 < wa; w2++) k5[0] += __popcll(rb[w2] & rc[w2] & rx[w2]);
                        nvis += wa;
                    }
                }
                dbp += c2(ns);
            });
        }
    }
    if (gcur >= 0) block_flush_u128<1>(k5, red, acc + (size_t)gcur * ACC_STRIDE, ids);
    // light vertices: runs of K5_LIGHT_RUN consecutive vertices dealt to the
    // waves in turn; lane b walks the c after b adjacent to b, then the x
    // after c adjacent to both, and counts the y adjacent to all three
    const int lane = threadIdx.x & 63;
    const int64_t nwv = (int64_t)gridDim.x * (blockDim.x >> 6);
    const int64_t wv = (int64_t)blockIdx.x * (blockDim.x >> 6) + (threadIdx.x >> 6);
    u128 s = 0;
    int wg = -1;
    for (int64_t r0 = wv * K5_LIGHT_RUN; r0 < n; r0 += nwv * K5_LIGHT_RUN) {
        const int32_t r1 = (int32_t)(r0 + K5_LIGHT_RUN < n ? r0 + K5_LIGHT_RUN : n);
        for (int32_t a = (int32_t)r0; a < r1; a++) {
            const int32_t dp = off[a + 1] - split[a];
            if (dp < 4 || dp > light) continue;
            const int g = gm.graph(a);
            if (g != wg) {
                if (wg >= 0) wave_flush_u128(s, acc + (size_t)wg * ACC_STRIDE + 2 * AC_K5);
                wg = g;
            }
            const unsigned long long *rows = ob + ob_off[a];   // one word per row
            if (lane < dp) {
                const unsigned long long rb = rows[lane];
                unsigned long long cs = rb;
                while (cs) {
                    const int ci = __ffsll((long long)cs) - 1;
                    cs &= cs - 1;
                    const unsigned long long sw = rb & rows[ci];
                    dbp += c2((uint64_t)__popcll(sw));
                    unsigned long long xs = sw;
                    while (xs) {
                        const int x = __ffsll((long long)xs) - 1;
                        xs &= xs - 1;
                        s += (uint64_t)__popcll(sw & rows[x]);
                        nvis++;
                    }
                }
            }
        }
    }
    if (wg >= 0) wave_flush_u128(s, acc + (size_t)wg * ACC_STRIDE + 2 * AC_K5);
    flush_count(nvis, visits);
    flush_count(dbp, dbp_out);
}

// Dense vertices, one workgroup per vertex a (h = d+(a), taken from the
// dense list): the 4-cliques of H_a through its complement Hc.
//  1. Rows of Hc over the positions 0..h-1 of N+(a): N(v) & N+(a) is the
//     suffix of list(a,v) whose arc indices in the row of a come after a's
//     in-arcs; its complement (without v itself) is the row.  Rows are
//     stored word-major (T[w * h + v]) so that lanes taking consecutive v
//     read consecutive words; dc(v) = complement degree.
//  2. Terms of the degrees alone (thread 0): C(h,4) - e C(h-2,2) + W (h-3)
//     + C(e,2) - W - S with e, W, S the edges, wedges and 3-stars of Hc
//     (App. A: one edge, a wedge or a matching, a 3-star with the rest of
//     the 4-set free).
//  3. One wave per vertex u, a lane per v > u, with c = common Hc
//     neighbours after u: + C(c,2), each 4-cycle of Hc once, from its
//     earliest vertex u and the opposite vertex v (Thm 4cycle).  For an Hc
//     edge u-v with t common neighbours (Thm 4vertex-tri): - (dc(u)-1)
//     (dc(v)-1) - C(t,2) (3-paths of the edge, diamonds on it); for each Hc
//     triangle u<v<x: + dc(u)+dc(v)+dc(x) - h (its -(h-3) for triangle+point,
//     +3 undoing the 3-path count's triangles, the tailed triangles at its
//     three vertices); + the Hc 4-cliques u<v<x<y (Thm 4clique).
// The signed terms add up modulo 2^128; their total, the 5-cliques, is a
// count in range.
template <bool IDS>
__global__ void __launch_bounds__(256) k_k5_dense(const int32_t *off, const int32_t *split, const int64_t *aoff,
                                                  const uint32_t *aa, const int32_t *dlist, const int *ndense,
                                                  unsigned long long *scr_all, int64_t scr_words, int32_t hcap,
                                                  int32_t vbc, int *task, GMap gm, unsigned long long *acc,
                                                  unsigned long long *visits, unsigned long long *dbp_out) {
    extern __shared__ unsigned long long tl[];   // a block of vbc columns of T, word-major
    __shared__ unsigned long long fu[4][K5_DENSE_HMAX / 64];
    __shared__ int fsum[4][K5_DENSE_HMAX / 64 + 1];   // popcounts of fu[w..] per wave
    __shared__ int s_t;
    __shared__ u128 red[3 * 4];
    const int ids[1] = {AC_K5};
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6, nwv = blockDim.x >> 6;
    unsigned long long *T = scr_all + (size_t)blockIdx.x * scr_words;
    int64_t *los = (int64_t *)(T + (size_t)hcap * (hcap / 64));
    int32_t *dc = (int32_t *)(los + hcap);
    int32_t *dch = dc + hcap;   // complement neighbours after the vertex
    const int nd = *ndense;
    u128 k5[1] = {0};
    int gcur = -1;
    uint64_t nvis = 0, dbp = 0;
    for (;;) {
        if (threadIdx.x == 0) s_t = atomicAdd(task, 1);
        __syncthreads();
        const int t = s_t;
        __syncthreads();   // s_t is read by every thread before it is taken again
        if (t >= nd) break;
        const int32_t a = dlist[t];
        block_switch_graph<1>(k5, gcur, gm.graph(a), red, acc, ACC_STRIDE, ids);
        const int32_t sa = split[a];
        const int h = off[a + 1] - sa;
        const int wa = (h + 63) >> 6;
        // 1. complement rows; first the start of each list's suffix in N+(a)
        for (int v = threadIdx.x; v < h; v += blockDim.x) {
            int64_t lo = aoff[sa + v], hi = aoff[sa + v + 1];
            while (lo < hi) { const int64_t mid = (lo + hi) >> 1; if ((int32_t)aa[mid] < sa) lo = mid + 1; else hi = mid; }
            los[v] = lo;
        }
        __syncthreads();
        for (int v = wid; v < h; v += nwv) {
            unsigned long long *row = fu[wid];
            for (int w = lane; w < wa; w += 64) row[w] = 0;
            wave_sync();
            const int64_t l0 = los[v], l1 = aoff[sa + v + 1];
            // four entries per lane in flight
            for (int64_t q = l0 + lane; q < l1; q += 256) {
                int32_t p4[4];
#pragma unroll
                for (int r = 0; r < 4; r++) p4[r] = q + 64 * r < l1 ? (int32_t)aa[q + 64 * r] - sa : -1;
#pragma unroll
                for (int r = 0; r < 4; r++)
                    if (p4[r] >= 0) atomicOr(&row[p4[r] >> 6], 1ull << (p4[r] & 63));
            }
            nvis += (uint64_t)(l1 - l0);
            wave_sync();
            int d = 0, dh = 0;
            for (int w = lane; w < wa; w += 64) {
                unsigned long long x = ~row[w];
                const int top = h - 64 * w;   // positions of this word below h
                if (top < 64) x &= (1ull << top) - 1ull;
                if (w == (v >> 6)) x &= ~(1ull << (v & 63));
                T[(size_t)w * h + v] = x;
                d += __popcll(x);
                if (w > (v >> 6)) dh += __popcll(x);
                else if (w == (v >> 6) && (v & 63) != 63) dh += __popcll(x & (~0ull << ((v & 63) + 1)));
            }
            d = (int)wave_sum_u64((uint64_t)d);
            dh = (int)wave_sum_u64((uint64_t)dh);
            if (lane == 0) { dc[v] = d; dch[v] = dh; }
            wave_sync();   // the row buffer is reused by the wave's next row
        }
        __syncthreads();
        // 2. degree terms
        {
            u128 e2 = 0, w2 = 0, s3 = 0;
            for (int v = threadIdx.x; v < h; v += blockDim.x) {
                const uint64_t d = (uint64_t)dc[v];
                e2 += d;
                w2 += c2(d);
                s3 += c3(d);
            }
            e2 = wave_sum_u128(e2);
            w2 = wave_sum_u128(w2);
            s3 = wave_sum_u128(s3);
            if (lane == 0) { red[wid] = e2; red[4 + wid] = w2; red[8 + wid] = s3; }
            __syncthreads();
            if (threadIdx.x == 0) {
                u128 E = 0, W = 0, S = 0;
                for (int w = 0; w < nwv; w++) { E += red[w]; W += red[4 + w]; S += red[8 + w]; }
                E >>= 1;
                const u128 hh = (u128)h;
                k5[0] += c4((uint64_t)h);
                k5[0] -= E * (u128)c2((uint64_t)(h - 2));
                k5[0] += W * (hh - 3);
                k5[0] += (u128)c2((uint64_t)E);
                k5[0] -= W;
                k5[0] -= S;
            }
            __syncthreads();   // red is reused by the flushes
        }
        // 3. pairs u < v, the columns v in blocks of vbc staged in LDS (tl),
        //    so that T is read from memory once per block, not once per u
        for (int vb = 0; vb < h; vb += vbc) {
            const int ve = vb + vbc < h ? vb + vbc : h;
            __syncthreads();   // the previous block is read by every wave
            for (int q = threadIdx.x; q < wa * vbc; q += blockDim.x) {
                const int w = q / vbc, vv = q - w * vbc;
                tl[q] = vb + vv < h ? T[(size_t)w * h + vb + vv] : 0ull;
            }
            __syncthreads();
            for (int u = wid; u < ve - 1; u += nwv) {
            for (int w = lane; w < wa; w += 64) fu[wid][w] = T[(size_t)w * h + u];
            wave_sync();
            if (lane == 0) {
                int acc_p = 0;
                fsum[wid][wa] = 0;
                for (int w = wa - 1; w >= 0; w--) { acc_p += __popcll(fu[wid][w]); fsum[wid][w] = acc_p; }
            }
            wave_sync();
            const uint64_t du = (uint64_t)dc[u];
            const int w0 = (u + 1) >> 6;
            const unsigned long long m0 = ~0ull << ((u + 1) & 63);   // positions after u in word w0
            for (int v = (u + 1 > vb ? u + 1 : vb) + lane; v < ve; v += 64) {
                // w0 < wa: v <= h - 1 lies in the last word at the latest
                const unsigned long long *tv = tl + (v - vb);   // column v: tv[w * vbc]
                uint32_t cnt = (uint32_t)__popcll(fu[wid][w0] & tv[w0 * vbc] & m0);
                int w = w0 + 1;
                for (; w + 8 <= wa; w += 8) {
                    unsigned long long x[8];
#pragma unroll
                    for (int r = 0; r < 8; r++) x[r] = tv[(w + r) * vbc];
#pragma unroll
                    for (int r = 0; r < 8; r++) cnt += (uint32_t)__popcll(fu[wid][w + r] & x[r]);
                }
                for (; w < wa; w++) cnt += (uint32_t)__popcll(fu[wid][w] & tv[w * vbc]);
                nvis += (uint64_t)(wa - w0);
                k5[0] += c2(cnt);
                if (!((fu[wid][v >> 6] >> (v & 63)) & 1ull)) {
                    // an edge u-v of H_a: its common neighbours in H_a after v
                    // (the positions after v less the Hc neighbours of u or v
                    // there) close C(s,2) directed bipyramids
                    const int wv = v >> 6;
                    const unsigned long long mg = (v & 63) == 63 ? 0ull : ~0ull << ((v & 63) + 1);
                    uint32_t chi = (uint32_t)__popcll(fu[wid][wv] & tv[wv * vbc] & mg);
                    for (int w = wv + 1; w < wa; w++) chi += (uint32_t)__popcll(fu[wid][w] & tv[w * vbc]);
                    const int duh = __popcll(fu[wid][wv] & mg) + fsum[wid][wv + 1];
                    const int sh = (h - 1 - v) - duh - dch[v] + (int)chi;
                    dbp += c2((uint64_t)sh);
                    continue;
                }
                // an edge of Hc
                uint32_t tf = cnt;
                for (int w = 0; w <= w0 && w < wa; w++) {
                    unsigned long long x = fu[wid][w] & tv[w * vbc];
                    if (w == w0) x &= ~m0;
                    tf += (uint32_t)__popcll(x);
                }
                const uint64_t dv = (uint64_t)dc[v];
                k5[0] -= (u128)((du - 1) * (dv - 1)) + (u128)c2(tf);
                const int wv = v >> 6;
                for (int w = wv; w < wa; w++) {
                    unsigned long long sx = fu[wid][w] & tv[w * vbc];
                    if (w == wv) sx &= (v & 63) == 63 ? 0ull : ~0ull << ((v & 63) + 1);
                    while (sx) {
                        const int x = w * 64 + __ffsll((long long)sx) - 1;
                        sx &= sx - 1;
                        k5[0] += (u128)(du + dv + (uint64_t)dc[x]);
                        k5[0] -= (u128)h;
                        const int wx = x >> 6;
                        for (int w2 = wx; w2 < wa; w2++) {
                            unsigned long long y = fu[wid][w2] & tv[w2 * vbc] & T[(size_t)w2 * h + x];
                            if (w2 == wx) y &= (x & 63) == 63 ? 0ull : ~0ull << ((x & 63) + 1);
                            k5[0] += (uint64_t)__popcll(y);
                        }
                        nvis += (uint64_t)(wa - wx);
                    }
                }
            }
            wave_sync();   // fu is reused by the wave's next u
            }
        }
        __syncthreads();   // T, los and dc are rewritten for the next vertex
    }
    if (gcur >= 0) block_flush_u128<1>(k5, red, acc + (size_t)gcur * ACC_STRIDE, ids);
    flush_count(nvis, visits);
    flush_count(dbp, dbp_out);
}

// ------------------------------------------------------------------- stages

// Vertices whose triangles take the product: out-degree at least
// k4_dense_dplus, their B_a and C_a within the memory the buffer can have.
// Sets B_K4_FLAG and lists them (vertex, d+, d) in *dense.
static esc_status k4_dense_select(esc_ctx *c, std::vector<int32_t> *dense) {
    const int32_t n = c->n;
    hipStream_t st = c->stream;
    if (c->G || c->k4_dense_dplus <= 0 || c->maxdplus < c->k4_dense_dplus) return ESC_OK;
    if ((size_t)c->max_lds < 4 * (size_t)HUB_T * HUB_K + 1024) return ESC_OK;
    int32_t *list = (int32_t *)ctx_buf(c, B_K4_LIST, sizeof(int32_t) * 3 * (size_t)(n + 1));
    int *cnt = (int *)ctx_buf(c, B_K4_CNT, sizeof(int) * 4);
    uint8_t *flag = (uint8_t *)ctx_buf(c, B_K4_FLAG, (size_t)n + 1);
    if (!list || !cnt || !flag) return ESC_ENOMEM;
    HIP_TRY(hipMemsetAsync(cnt, 0, sizeof(int) * 4, st));
    HIP_TRY(hipMemsetAsync(flag, 0, (size_t)n + 1, st));
    k_k4_pick<<<grid_cap(c, n, 256), 256, 0, st>>>(n, (const int32_t *)c->buf[B_OFF], (const int32_t *)c->buf[B_SPLIT],
                                                   c->k4_dense_dplus, list, cnt);
    HIP_TRY(hipGetLastError());
    // the count with the first K4_READ candidates in one read-back (more: a second)
    const int32_t K4_READ = 16384;
    const size_t first = (size_t)(n + 1 < K4_READ ? n + 1 : K4_READ);
    std::vector<int32_t> all(3 * first);
    int h = 0;
    HIP_TRY(hipMemcpyAsync(&h, cnt, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipMemcpyAsync(all.data(), list, sizeof(int32_t) * 3 * first, hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    if (h == 0) return ESC_OK;
    if ((size_t)h > first) {
        all.resize(3 * (size_t)h);
        HIP_TRY(hipMemcpyAsync(all.data() + 3 * first, list + 3 * first, sizeof(int32_t) * 3 * ((size_t)h - first),
                               hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
    }
    size_t free_b = 0;
    ESC_TRY(ctx_free_bytes(c, &free_b));
    const size_t room = ctx_held(c, B_K4_Y) +
                        (free_b > ((size_t)2 << 30) ? (free_b - ((size_t)2 << 30)) / 2 : 0);
    size_t total = 0, biggest = 0;
    std::vector<int32_t> &ids = c->k4_ids;   // kept until the next call: the copy below reads it
    ids.clear();
    for (int q = 0; q < h; q++) {
        const size_t dpp = ((size_t)all[3 * q + 1] + HUB_T - 1) / HUB_T * HUB_T;
        const size_t dk = (((size_t)all[3 * q + 2] + 1) / 2 + HUB_K - 1) / HUB_K * HUB_K;   // bytes
        const size_t bytes = dpp * dk + 4 * dpp * dpp;
        if (bytes > room) continue;
        dense->insert(dense->end(), {all[3 * q], all[3 * q + 1], all[3 * q + 2]});
        ids.push_back(all[3 * q]);
        total += bytes;
        biggest = bytes > biggest ? bytes : biggest;
    }
    if (ids.empty()) return ESC_OK;
    size_t cap = total < ((size_t)8 << 30) ? total : ((size_t)8 << 30);
    if (cap < biggest) cap = biggest;
    if (cap > room) cap = room;
    c->k4_cap = cap;
    HIP_TRY(hipMemcpyAsync(list, ids.data(), sizeof(int32_t) * ids.size(), hipMemcpyHostToDevice, st));
    k_k4_flags<<<grid_cap(c, (int64_t)ids.size(), 256), 256, 0, st>>>((int32_t)ids.size(), list, flag);
    HIP_TRY(hipGetLastError());
    return ESC_OK;
}

// The chosen vertices in batches through the B and C buffers: rows of B_a,
// the products C_a, then their triangles.
static esc_status k4_dense_product(esc_ctx *c, const std::vector<int32_t> &dense) {
    const size_t nd = dense.size() / 3;
    if (nd == 0) return ESC_OK;
    hipStream_t st = c->stream;
    // the B and C parts of a batch share the cap: B bytes first, C after
    const size_t cap = c->k4_cap;
    uint8_t *yb = (uint8_t *)ctx_buf(c, B_K4_Y, cap + 256);   // C starts 16-byte aligned after B
    int64_t *meta = (int64_t *)ctx_buf(c, B_K4_META, sizeof(int64_t) * 8 * (nd + 1));
    if (!yb || !meta) return ESC_ENOMEM;
    std::vector<int32_t> va(nd + 1), dpp(nd + 1), dk(nd + 1), pp(nd + 1);
    std::vector<int64_t> rp(nd + 1), ap(nd + 1), bo(nd + 1), co(nd + 1);
    const size_t lds = 4 * (size_t)HUB_T * HUB_K;
    int32_t *d_va = (int32_t *)meta, *d_dpp = d_va + (nd + 1), *d_dk = d_dpp + (nd + 1), *d_pp = d_dk + (nd + 1);
    int64_t *d_rp = meta + 2 * (nd + 1), *d_ap = d_rp + (nd + 1), *d_bo = d_ap + (nd + 1), *d_co = d_bo + (nd + 1);
    size_t q0 = 0;
    while (q0 < nd) {
        size_t q1 = q0;
        size_t bbytes = 0, cbytes = 0;
        int64_t rows = 0, arcs = 0;
        int32_t patches = 0, maxk = 0;
        while (q1 < nd) {
            const int32_t dplus = dense[3 * q1 + 1];
            const int64_t r = ((int64_t)dplus + HUB_T - 1) / HUB_T * HUB_T;
            const int64_t k = (((int64_t)dense[3 * q1 + 2] + 1) / 2 + HUB_K - 1) / HUB_K * HUB_K;   // bytes
            if (q1 > q0 && bbytes + cbytes + (size_t)(r * k + 4 * r * r) > cap) break;
            const size_t j = q1 - q0;
            va[j] = dense[3 * q1];
            dpp[j] = (int32_t)r;
            dk[j] = (int32_t)k;
            rp[j] = rows;
            ap[j] = arcs;
            bo[j] = (int64_t)bbytes;
            co[j] = (int64_t)(cbytes / 4);
            pp[j] = patches;
            rows += r;
            arcs += dplus;
            bbytes += (size_t)(r * k);
            cbytes += (size_t)(4 * r * r);
            patches += hub_npatches((int)(r / HUB_T));
            maxk = (int32_t)k > maxk ? (int32_t)k : maxk;
            c->prod_macs[STAGE_K4] += (uint64_t)((r / HUB_T) * (r / HUB_T + 1) / 2) * HUB_T * HUB_T * 2 * (uint64_t)k;
            q1++;
        }
        const int32_t nq = (int32_t)(q1 - q0);
        rp[nq] = rows;
        ap[nq] = arcs;
        bo[nq] = (int64_t)bbytes;
        co[nq] = (int64_t)(cbytes / 4);
        pp[nq] = patches;
        // C after the B part, 16-byte aligned
        const size_t cstart = (bbytes + 15) & ~(size_t)15;
        int32_t *cm = (int32_t *)(yb + cstart);
        HIP_TRY(hipMemcpyAsync(d_va, va.data(), sizeof(int32_t) * (nq + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_dpp, dpp.data(), sizeof(int32_t) * (nq + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_dk, dk.data(), sizeof(int32_t) * (nq + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_pp, pp.data(), sizeof(int32_t) * (nq + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_rp, rp.data(), sizeof(int64_t) * (nq + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_ap, ap.data(), sizeof(int64_t) * (nq + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_bo, bo.data(), sizeof(int64_t) * (nq + 1), hipMemcpyHostToDevice, st));
        HIP_TRY(hipMemcpyAsync(d_co, co.data(), sizeof(int64_t) * (nq + 1), hipMemcpyHostToDevice, st));
        k_k4_rows<<<(unsigned)rows, 256, (size_t)maxk, st>>>((const int32_t *)c->buf[B_OFF],
                                                            (const int32_t *)c->buf[B_SPLIT],
                                                            (const int64_t *)c->buf[B_AOFF],
                                                            (const uint32_t *)c->buf[B_AA], nq, d_va, d_dpp, d_dk,
                                                            d_rp, d_bo, yb);
        HIP_TRY(hipGetLastError());
        const int nwg = 8 * HUB_PR * HUB_PC * ((patches + 7) / 8);
        k_k4_gemm<<<nwg, 64 * HUB_WAVES, lds, st>>>(yb, nq, d_dpp, d_dk, d_bo, d_co, d_pp, cm);
        HIP_TRY(hipGetLastError());
        auto look = c->av ? k_k4_lookup<true> : k_k4_lookup<false>;
        look<<<grid_cap(c, arcs * 64, 256, 8), 256, 0, st>>>(
            (const int32_t *)c->buf[B_OFF], (const int32_t *)c->buf[B_ADJ], (const int32_t *)c->buf[B_SPLIT],
            (const int32_t *)c->buf[B_REV], (const int32_t *)c->buf[B_ARC_EID], (const uint32_t *)c->buf[B_TE],
            (const int64_t *)c->buf[B_AOFF], (const uint32_t *)c->buf[B_AA], c->av, nq, d_va, d_dpp, d_ap, d_co,
            cm, (unsigned long long *)c->buf[B_K4E], (unsigned long long *)c->buf[B_ACC],
            (unsigned long long *)c->buf[B_WORK] + WORK_VISITS + 3);
        HIP_TRY(hipGetLastError());
        HIP_TRY(hipStreamSynchronize(st));   // the host arrays are rewritten by the next batch
        q0 = q1;
    }
    return ESC_OK;
}

esc_status stage_k4_triangles(esc_ctx *c) {
    hipStream_t st = c->stream;
    const int64_t m = c->m;
    unsigned long long *k4e = (unsigned long long *)ctx_buf(c, B_K4E, sizeof(uint64_t) * (size_t)(m + 1));
    if (!k4e) return ESC_ENOMEM;
    HIP_TRY(hipMemsetAsync(k4e, 0, sizeof(uint64_t) * (size_t)(m + 1), st));
    if (m == 0 || c->narcs_apex == 0) return ESC_OK;
    std::vector<int32_t> dense;
    ESC_TRY(k4_dense_select(c, &dense));
    const uint8_t *kflag = dense.empty() ? nullptr : (const uint8_t *)c->buf[B_K4_FLAG];
    auto kern = c->av ? k_k4_triangles<true> : k_k4_triangles<false>;
    kern<<<grid_cap(c, m * 64, 256, 8), 256, 0, st>>>(
        m, (const int32_t *)c->buf[B_OFF], (const int32_t *)c->buf[B_ADJ], (const int32_t *)c->buf[B_SPLIT],
        (const int32_t *)c->buf[B_REV], (const int32_t *)c->buf[B_ARC_EID], (const int32_t *)c->buf[B_EARC],
        (const int32_t *)c->buf[B_ELO], (const uint32_t *)c->buf[B_TE], (const int64_t *)c->buf[B_AOFF],
        (const uint32_t *)c->buf[B_AA], c->av, k4e, gmap_of(c), c->G && c->tab_n <= 4096 ? 1 : 0,
        (unsigned long long *)c->buf[B_ACC],
        (unsigned long long *)c->buf[B_WORK] + WORK_VISITS + 3, kflag);
    HIP_TRY(hipGetLastError());
    ESC_TRY(mark_walk_end(c, STAGE_K4));
    ESC_TRY(k4_dense_product(c, dense));
    return ctx_release_if_short(c, {B_K4_Y});
}

esc_status stage_k5(esc_ctx *c) {
    hipStream_t st = c->stream;
    const int32_t n = c->n;
    if (n == 0 || c->narcs_apex == 0) return ESC_OK;
    const int32_t *off = (const int32_t *)c->buf[B_OFF], *split = (const int32_t *)c->buf[B_SPLIT];
    const int64_t *aoff = (const int64_t *)c->buf[B_AOFF];
    const uint32_t *aa = (const uint32_t *)c->buf[B_AA];
    int64_t *len = (int64_t *)ctx_buf(c, B_EOFF, sizeof(int64_t) * (size_t)(n + 2));
    int64_t *ob_off = (int64_t *)ctx_buf(c, B_OB_OFF, sizeof(int64_t) * (size_t)(n + 2));
    int32_t *dlist = (int32_t *)ctx_buf(c, B_K5_DENSE, sizeof(int32_t) * (size_t)(n + 1));
    int *task = (int *)ctx_buf(c, B_TASK, sizeof(int) * 16);
    if (!len || !ob_off || !dlist || !task) return ESC_ENOMEM;
    // task[3]: units of the direct pass, task[5]: dense vertices listed,
    // task[6]: dense vertices taken
    HIP_TRY(hipMemsetAsync(task + 3, 0, 4 * sizeof(int), st));
    k_k5_classify<<<grid_cap(c, (int64_t)n * 64, 256), 256, 0, st>>>(n, off, split, aoff, aa, c->k5_light,
                                                                     c->k5_dense_pct, len, dlist, task + 5);
    HIP_TRY(hipGetLastError());
    ESC_TRY(dev_exclusive_scan_i64(c, len, ob_off, n));
    int64_t words = 0;
    HIP_TRY(hipMemcpyAsync(&words, ob_off + n, sizeof(int64_t), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    unsigned long long *ob = (unsigned long long *)ctx_buf(c, B_OB, sizeof(uint64_t) * (size_t)(words + 1));
    if (!ob) return ESC_ENOMEM;
    HIP_TRY(hipMemsetAsync(ob, 0, sizeof(uint64_t) * (size_t)(words + 1), st));
    k_ob_rows<<<grid_cap(c, (int64_t)n * 64, 256), 256, 0, st>>>(n, off, split, aoff, aa, ob_off, ob);
    HIP_TRY(hipGetLastError());
    // units of work of the direct pass (see k5_chunk): per-vertex counts, then offsets
    int64_t *uoff = (int64_t *)ctx_buf(c, B_K5_UNITS, sizeof(int64_t) * (size_t)(n + 2));
    if (!uoff) return ESC_ENOMEM;
    k_k5_units<<<grid_cap(c, n, 256), 256, 0, st>>>(n, off, split, ob_off, c->k5_work_log2, c->k5_light, len);
    HIP_TRY(hipGetLastError());
    ESC_TRY(dev_exclusive_scan_i64(c, len, uoff, n));
    int64_t nunits = 0;
    int32_t *uown = nullptr;
    ESC_TRY(dev_task_owner(c, n, uoff, &nunits, &uown));
    unsigned long long *acc = (unsigned long long *)c->buf[B_ACC];
    unsigned long long *vis = (unsigned long long *)c->buf[B_WORK] + WORK_VISITS + 4;
    unsigned long long *dbp = (unsigned long long *)c->buf[B_WORK] + WORK_DBP;
    k_k5<<<c->num_cu * 4, 256, 0, st>>>(n, off, split, ob_off, ob, uoff, uown, nunits, c->k5_work_log2,
                                        c->k5_light, c->k5_wave_words, task + 3, gmap_of(c), acc, vis, dbp);
    HIP_TRY(hipGetLastError());
    if (c->maxdplus > c->k5_light && c->k5_dense_pct <= 100) {
        // dense vertices: per-workgroup scratch for the complement rows of
        // the largest out-neighbourhood, its list starts and degrees
        int32_t hmax = c->maxdplus < K5_DENSE_HMAX ? c->maxdplus : K5_DENSE_HMAX;
        const int32_t hcap = (hmax + 63) & ~63;
        const int64_t per_wg = (int64_t)hcap * (hcap / 64) + hcap + hcap;   // rows, list starts, two degree arrays
        int nwg = 4 * c->num_cu;   // 113 VGPRs: four 4-wave workgroups per CU are resident
        while (nwg > c->num_cu && (size_t)nwg * (size_t)per_wg * 8 > c->dev_mem / 16) nwg -= c->num_cu;
        // a block of vbc columns of the complement rows in LDS: about 32 KB
        // (four workgroups a CU), 64 to 256 columns
        const int32_t wa_cap = hcap / 64;
        int32_t vbc = (int32_t)(32768 / (8 * wa_cap)) & ~63;
        if (vbc > 256) vbc = 256;
        if (vbc < 64) vbc = 64;
        const size_t tl_bytes = sizeof(uint64_t) * (size_t)wa_cap * vbc;
        unsigned long long *scr = (unsigned long long *)ctx_buf(c, B_K5_DENSE_SCR, sizeof(uint64_t) * (size_t)per_wg * nwg);
        if (!scr) return ESC_ENOMEM;
        auto kern = c->av ? k_k5_dense<true> : k_k5_dense<false>;
        kern<<<nwg, 256, tl_bytes, st>>>(off, split, aoff, aa, dlist, task + 5, scr, per_wg, hcap, vbc, task + 6,
                                         gmap_of(c), acc, vis, dbp);
        HIP_TRY(hipGetLastError());
    }
    return ESC_OK;
}
