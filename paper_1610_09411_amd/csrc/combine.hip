// Final combination on the device: the 128-bit sums become non-induced counts
// of every pattern (the cut formulas of Secs. 5-6 with their shrinkage
// corrections; disconnected patterns in closed form, Appendix A), then
// induced counts through the inverse of the matrix of Appendix B.
//
// The matrix is built here from the pattern drawings: A[i][j] = number of
// edge subsets of pattern j that form pattern i, and by inclusion-exclusion
// over edge sets its inverse is (-1)^(e(j)-e(i)) A[i][j].
#include <string.h>
#include <vector>
#include <algorithm>
#include <stdlib.h>
#include "device.h"
#include "ctx.h"

// ----------------------------------------------------- pattern table (host)

struct Pat { int k; int ne; int e[10][2]; };

// vertex labels as drawn, 1-based
static const Pat kPatterns[45] = {
    // 4-vertex connected: 3-star, 3-path, tailed triangle, 4-cycle, diamond, 4-clique
    {4, 3, {{1, 2}, {1, 3}, {1, 4}}},
    {4, 3, {{1, 2}, {1, 3}, {2, 4}}},
    {4, 4, {{1, 2}, {1, 3}, {1, 4}, {2, 4}}},
    {4, 4, {{1, 2}, {1, 3}, {2, 4}, {3, 4}}},
    {4, 5, {{1, 2}, {1, 3}, {1, 4}, {2, 4}, {3, 4}}},
    {4, 6, {{1, 2}, {1, 3}, {1, 4}, {2, 3}, {2, 4}, {3, 4}}},
    // 4-vertex disconnected: independent set, edge, matching, wedge, triangle
    {4, 0, {}},
    {4, 1, {{1, 2}}},
    {4, 2, {{1, 2}, {3, 4}}},
    {4, 2, {{1, 2}, {2, 3}}},
    {4, 3, {{1, 2}, {1, 3}, {2, 3}}},
    // 5-vertex connected, patterns 1..21
    {5, 4, {{1, 2}, {1, 3}, {1, 4}, {1, 5}}},
    {5, 4, {{1, 2}, {1, 3}, {1, 4}, {2, 5}}},
    {5, 4, {{1, 2}, {1, 3}, {2, 4}, {3, 5}}},
    {5, 5, {{1, 2}, {1, 3}, {2, 3}, {3, 4}, {3, 5}}},
    {5, 5, {{1, 2}, {1, 3}, {2, 3}, {2, 4}, {4, 5}}},
    {5, 5, {{1, 2}, {1, 3}, {2, 3}, {2, 4}, {3, 5}}},
    {5, 5, {{1, 2}, {2, 4}, {3, 4}, {1, 3}, {3, 5}}},
    {5, 5, {{1, 2}, {1, 3}, {2, 4}, {3, 5}, {4, 5}}},
    {5, 6, {{1, 2}, {1, 3}, {2, 3}, {3, 4}, {3, 5}, {4, 5}}},
    {5, 6, {{1, 2}, {2, 4}, {3, 4}, {1, 3}, {3, 5}, {1, 4}}},
    {5, 6, {{1, 2}, {2, 4}, {3, 4}, {1, 3}, {3, 5}, {2, 3}}},
    {5, 6, {{1, 2}, {2, 4}, {3, 4}, {1, 3}, {3, 5}, {4, 5}}},
    {5, 6, {{1, 2}, {2, 5}, {1, 3}, {3, 5}, {1, 4}, {4, 5}}},
    {5, 7, {{1, 2}, {2, 5}, {1, 3}, {3, 5}, {1, 4}, {4, 5}, {1, 5}}},
    {5, 7, {{1, 2}, {2, 4}, {3, 4}, {1, 3}, {3, 5}, {1, 4}, {2, 3}}},
    {5, 7, {{1, 2}, {2, 4}, {3, 4}, {1, 3}, {3, 5}, {2, 3}, {4, 5}}},
    {5, 7, {{1, 2}, {1, 3}, {1, 4}, {2, 3}, {2, 4}, {3, 5}, {4, 5}}},
    {5, 8, {{1, 2}, {1, 3}, {1, 4}, {1, 5}, {2, 3}, {3, 5}, {4, 5}, {2, 4}}},
    {5, 8, {{1, 2}, {2, 4}, {3, 4}, {1, 3}, {3, 5}, {2, 3}, {4, 5}, {1, 4}}},
    {5, 9, {{1, 3}, {1, 4}, {1, 5}, {2, 3}, {2, 4}, {2, 5}, {3, 4}, {3, 5}, {4, 5}}},
    {5, 10, {{1, 2}, {1, 3}, {1, 4}, {1, 5}, {2, 3}, {2, 4}, {2, 5}, {3, 4}, {3, 5}, {4, 5}}},
    // 5-vertex disconnected (1)..(11), then wedge+edge, triangle+edge
    {5, 0, {}},
    {5, 1, {{1, 2}}},
    {5, 2, {{1, 2}, {3, 4}}},
    {5, 2, {{1, 2}, {1, 3}}},
    {5, 3, {{1, 2}, {1, 3}, {2, 3}}},
    {5, 3, {{1, 2}, {1, 3}, {1, 4}}},
    {5, 3, {{1, 2}, {1, 3}, {3, 4}}},
    {5, 4, {{1, 2}, {2, 3}, {1, 3}, {3, 4}}},
    {5, 4, {{1, 2}, {2, 4}, {3, 4}, {1, 3}}},
    {5, 5, {{1, 2}, {2, 4}, {3, 4}, {1, 4}, {1, 3}}},
    {5, 6, {{1, 2}, {2, 3}, {3, 4}, {1, 4}, {2, 4}, {1, 3}}},
    {5, 3, {{1, 2}, {1, 3}, {4, 5}}},
    {5, 4, {{1, 2}, {1, 3}, {2, 3}, {4, 5}}},
};

static int pair_index(int k, int a, int b) {   // 0-based a < b
    int idx = 0;
    for (int x = 0; x < k; x++)
        for (int y = x + 1; y < k; y++) {
            if (x == a && y == b) return idx;
            idx++;
        }
    return -1;
}

static unsigned mask_of(const Pat &p) {
    unsigned m = 0;
    for (int i = 0; i < p.ne; i++) {
        int a = p.e[i][0] - 1, b = p.e[i][1] - 1;
        if (a > b) std::swap(a, b);
        m |= 1u << pair_index(p.k, a, b);
    }
    return m;
}

// smallest relabelled mask over all vertex permutations
static unsigned canonical(int k, unsigned m) {
    int perm[5] = {0, 1, 2, 3, 4};
    unsigned best = ~0u;
    do {
        unsigned x = 0;
        for (int a = 0; a < k; a++)
            for (int b = a + 1; b < k; b++)
                if (m >> pair_index(k, a, b) & 1) {
                    int pa = perm[a], pb = perm[b];
                    if (pa > pb) std::swap(pa, pb);
                    x |= 1u << pair_index(k, pa, pb);
                }
        best = std::min(best, x);
    } while (std::next_permutation(perm, perm + k));
    return best;
}

// signed inverse of A for one pattern size: rows/cols in output order
static void build_inverse(int k, int first, int count, std::vector<int32_t> &inv) {
    std::vector<unsigned> canon(count);
    for (int j = 0; j < count; j++) canon[j] = canonical(k, mask_of(kPatterns[first + j]));
    std::vector<int32_t> A((size_t)count * count, 0);
    for (int j = 0; j < count; j++) {
        const Pat &p = kPatterns[first + j];
        unsigned m = mask_of(p);
        int bits[10], nb = 0;
        for (int b = 0; b < k * (k - 1) / 2; b++) if (m >> b & 1) bits[nb++] = b;
        for (unsigned sub = 0; sub < (1u << nb); sub++) {
            unsigned x = 0;
            for (int t = 0; t < nb; t++) if (sub >> t & 1) x |= 1u << bits[t];
            unsigned cx = canonical(k, x);
            for (int i = 0; i < count; i++)
                if (canon[i] == cx) { A[(size_t)i * count + j]++; break; }
        }
    }
    inv.assign((size_t)count * count, 0);
    for (int i = 0; i < count; i++)
        for (int j = 0; j < count; j++) {
            int s = ((kPatterns[first + j].ne - kPatterns[first + i].ne) & 1) ? -1 : 1;
            inv[(size_t)i * count + j] = s * A[(size_t)i * count + j];
        }
}

esc_status combine_tables(int32_t *host_inv4 /*121*/, int32_t *host_inv5 /*1156*/) {
    std::vector<int32_t> a4, a5;
    build_inverse(4, 0, 11, a4);
    build_inverse(5, 11, 34, a5);
    memcpy(host_inv4, a4.data(), sizeof(int32_t) * 121);
    memcpy(host_inv5, a5.data(), sizeof(int32_t) * 1156);
    return ESC_OK;
}

// ------------------------------------------------------------ device side

__device__ inline uint32_t gcd_u32(uint32_t a, uint32_t b) {
    while (b) { const uint32_t t = a % b; a = b; b = t; }
    return a;
}

__device__ inline u128 binom(u128 n, int k) {
    // C(n,k), 0 when n < k.  Step i turns r = C(n,i) into C(n,i+1) =
    // r (n-i) / (i+1) dividing first: with g = gcd(r, i+1), (i+1)/g divides
    // n-i, so (r/g) ((n-i) / ((i+1)/g)) is exact and no intermediate exceeds
    // the result (r (n-i) itself would pass 2^128 for C(n,5) from n near 9.6e7)
    if (n < (u128)k) return 0;
    u128 r = 1;
    for (int i = 0; i < k; i++) {
        const uint32_t d = (uint32_t)(i + 1);
        const uint32_t g = gcd_u32(d, (uint32_t)(r % (u128)d));
        r = (r / (u128)g) * ((n - (u128)i) / (u128)(d / g));
    }
    return r;
}

__device__ inline u128 apply_inv(const int32_t *inv, int count, int row, const u128 *N) {
    u128 s = 0;   // arithmetic modulo 2^128; the true value lies in [0, 2^128)
    for (int j = 0; j < count; j++) {
        int32_t a = inv[row * count + j];
        if (a > 0) s += (u128)a * N[j];
        else if (a < 0) s -= (u128)(-a) * N[j];
    }
    return s;
}

// One graph: its AC_COUNT sums, n and m -> out[0..44] induced counts,
// out[45..89] non-induced counts (the first 11 of each when k = 4),
// out[90..93] induced 3-vertex counts (no edge, one edge, path, triangle).
#define COMBINE_ROW 96
__device__ void combine_one(const unsigned long long *acc, const int32_t *inv4, const int32_t *inv5, int64_t nv,
                            int64_t me, int k, u128 *out) {
    u128 S[AC_COUNT];
    for (int s = 0; s < AC_COUNT; s++) S[s] = ((u128)acc[2 * s + 1] << 64) | acc[2 * s];
    const u128 n = (u128)nv, m = (u128)me;
    const u128 T = S[AC_T3] / 3, K4 = S[AC_K4X4] / 4;
    const u128 W = S[AC_W], TT = S[AC_TT], D = S[AC_D], C4 = S[AC_C4];
    // connected 4-vertex (Thm 4vertex-easy, Thm 4cycle, Thm 4clique)
    u128 N4[11];
    N4[0] = S[AC_S3];
    N4[1] = S[AC_EP] - 3 * T;
    N4[2] = TT;
    N4[3] = C4;
    N4[4] = D;
    N4[5] = K4;
    // disconnected 4-vertex: choose the missing vertices freely
    const u128 pairs_m = binom(m, 2);
    N4[6] = binom(n, 4);
    N4[7] = m * binom(n >= 2 ? n - 2 : 0, 2);
    N4[8] = pairs_m - W;                 // edge pairs not sharing a vertex
    N4[9] = n >= 3 ? W * (n - 3) : 0;
    N4[10] = n >= 3 ? T * (n - 3) : 0;
    for (int i = 0; i < 11; i++) out[i] = apply_inv(inv4, 11, i, N4);
    for (int i = 0; i < 11; i++) out[45 + i] = N4[i];
    // 3-vertex subsets: triangles T, induced paths W - 3T; the m (n-2) pairs
    // (edge, third vertex) meet a one-edge set once, a path twice, a
    // triangle three times
    const u128 P3 = W - 3 * T;
    const u128 E1 = n >= 2 ? m * (n - 2) - 2 * P3 - 3 * T : 0;
    out[90] = binom(n, 3) - E1 - P3 - T;
    out[91] = E1;
    out[92] = P3;
    out[93] = T;
    if (k < 5) return;
    u128 N5[34];
    N5[0] = S[AC_S4];
    N5[1] = S[AC_N2] - 2 * TT;
    N5[2] = S[AC_N3] - 4 * C4 - 2 * TT - 3 * T;
    N5[3] = S[AC_N4];
    N5[4] = S[AC_N5] - 4 * D;
    N5[5] = S[AC_N6] - 2 * D;
    N5[6] = S[AC_N7X2] / 2 - 2 * D;
    N5[7] = S[AC_CYC] - S[AC_Z];
    N5[8] = S[AC_N9] - 2 * D;
    N5[9] = S[AC_N10] - 12 * K4;
    N5[10] = S[AC_N11];
    N5[11] = S[AC_N12] - 4 * D;
    N5[12] = S[AC_N13];
    N5[13] = S[AC_N14];
    N5[14] = S[AC_N15];
    N5[15] = S[AC_N16] - 12 * K4;
    N5[16] = S[AC_N17];
    // dense hubs: every rim 4-cycle was counted at both its diagonals
    N5[17] = S[AC_N18] + (S[AC_WD2] >> 1);
    N5[18] = S[AC_N19];
    N5[19] = S[AC_N20];
    N5[20] = S[AC_K5];
    // disconnected 5-vertex
    const u128 n3 = n >= 3 ? n - 3 : 0, n4 = n >= 4 ? n - 4 : 0;
    N5[21] = binom(n, 5);
    N5[22] = m * binom(n >= 2 ? n - 2 : 0, 3);
    N5[23] = (pairs_m - W) * n4;
    N5[24] = W * binom(n3, 2);
    N5[25] = T * binom(n3, 2);
    for (int x = 0; x < 6; x++) N5[26 + x] = N4[x] * n4;
    // wedge + disjoint edge: all (wedge, edge) pairs minus those where the edge
    // touches the wedge's vertices; an edge touching it is counted once per
    // endpoint degree, edges inside the 3 vertices (2 per wedge, plus 1 for each
    // closed wedge, 3 T in all) once too often
    N5[32] = W * m - S[AC_SW] + 2 * W + 3 * T;
    // triangle + disjoint edge
    N5[33] = T * m - S[AC_TD] + 3 * T;
    for (int i = 0; i < 34; i++) out[11 + i] = apply_inv(inv5, 34, i, N5);
    for (int i = 0; i < 34; i++) out[56 + i] = N5[i];
}

__global__ void k_combine(const unsigned long long *acc, const int32_t *inv4, const int32_t *inv5, int64_t nv,
                          int64_t me, int k, u128 *out) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    combine_one(acc, inv4, inv5, nv, me, k, out);
}

// One thread per graph of a batch: exact 128-bit combination, then the
// induced counts as uint64 with a per-graph flag when one does not fit.
// Also adds the graphs' W, 3T and D into the work counters.
__global__ void k_combine_batched(int32_t G, const unsigned long long *acc, const int32_t *inv4, const int32_t *inv5,
                                  const int64_t *voff, const int64_t *aoff, int k, u128 *tmp, uint64_t *out,
                                  uint8_t *ovf, unsigned long long *work) {
    const int cnt = k == 4 ? 11 : 45;
    for (int32_t g = blockIdx.x * blockDim.x + threadIdx.x; g < G; g += gridDim.x * blockDim.x) {
        const unsigned long long *a = acc + (size_t)g * ACC_STRIDE;
        u128 *o = tmp + (size_t)g * COMBINE_ROW;
        combine_one(a, inv4, inv5, voff[g + 1] - voff[g], (aoff[g + 1] - aoff[g]) / 2, k, o);
        uint8_t f = 0;
        for (int i = 0; i < cnt; i++) {
            out[(size_t)g * cnt + i] = (uint64_t)o[i];
            f |= (o[i] >> 64) != 0;
        }
        ovf[g] = f;
        atomicAdd(&work[12], a[2 * AC_W]);
        atomicAdd(&work[13], a[2 * AC_T3]);
        atomicAdd(&work[14], a[2 * AC_D]);
    }
}

esc_status stage_combine(esc_ctx *c, esc_u128 *host_out, const int32_t *d_inv4, const int32_t *d_inv5) {
    u128 *dout = (u128 *)ctx_buf(c, B_OUT, sizeof(u128) * COMBINE_ROW);
    if (!dout) return ESC_ENOMEM;
    k_combine<<<1, 64, 0, c->stream>>>((const unsigned long long *)c->buf[B_ACC], d_inv4, d_inv5, c->n, c->m, c->k,
                                       dout);
    HIP_TRY(hipGetLastError());
    u128 h[COMBINE_ROW];
    int cnt = c->k == 4 ? 11 : 45;
    HIP_TRY(hipMemcpyAsync(h, dout, sizeof(u128) * COMBINE_ROW, hipMemcpyDeviceToHost, c->stream));
    HIP_TRY(hipStreamSynchronize(c->stream));
    for (int i = 0; i < cnt; i++) {
        host_out[i].lo = (uint64_t)h[i];
        host_out[i].hi = (uint64_t)(h[i] >> 64);
        c->noninduced[i].lo = (uint64_t)h[45 + i];
        c->noninduced[i].hi = (uint64_t)(h[45 + i] >> 64);
    }
    for (int i = 0; i < 4; i++) {
        c->three[i].lo = (uint64_t)h[90 + i];
        c->three[i].hi = (uint64_t)(h[90 + i] >> 64);
    }
    return ESC_OK;
}

// Device side of a batched combine: exact rows (COMBINE_ROW u128 per graph:
// 45 induced, 45 non-induced, 4 three-vertex) in B_OUT, uint64 rows and
// overflow flags in B_BOUT.
esc_status stage_combine_batched(esc_ctx *c) {
    const int32_t G = c->G;
    const int cnt = c->k == 4 ? 11 : 45;
    u128 *tmp = (u128 *)ctx_buf(c, B_OUT, sizeof(u128) * COMBINE_ROW * (size_t)G);
    uint8_t *bout = (uint8_t *)ctx_buf(c, B_BOUT, (sizeof(uint64_t) * cnt + 1) * (size_t)G);
    if (!tmp || !bout) return ESC_ENOMEM;
    uint64_t *dout = (uint64_t *)bout;
    uint8_t *dovf = bout + sizeof(uint64_t) * cnt * (size_t)G;
    const int64_t *voff = (const int64_t *)c->buf[B_GOFF];
    int blocks = (G + 63) / 64;
    if (blocks > c->num_cu * 8) blocks = c->num_cu * 8;
    k_combine_batched<<<blocks, 64, 0, c->stream>>>(G, (const unsigned long long *)c->buf[B_ACC], c->d_inv4, c->d_inv5,
                                                    voff, voff + G + 1, c->k, tmp, dout, dovf,
                                                    (unsigned long long *)c->buf[B_WORK]);
    HIP_TRY(hipGetLastError());
    return ESC_OK;
}

esc_status batched_copy_u64(esc_ctx *c, uint64_t *host_out, uint8_t *host_overflow, int *any_overflow) {
    const int32_t G = c->G;
    const int cnt = c->k == 4 ? 11 : 45;
    const uint64_t *dout = (const uint64_t *)c->buf[B_BOUT];
    const uint8_t *dovf = (const uint8_t *)c->buf[B_BOUT] + sizeof(uint64_t) * cnt * (size_t)G;
    HIP_TRY(hipMemcpyAsync(host_out, dout, sizeof(uint64_t) * cnt * (size_t)G, hipMemcpyDeviceToHost, c->stream));
    uint8_t *flags = host_overflow;
    uint8_t *own = nullptr;
    if (!flags) {
        own = (uint8_t *)malloc((size_t)G);
        if (!own) return ESC_ENOMEM;
        flags = own;
    }
    esc_status st = ESC_OK;
    if (hipMemcpyAsync(flags, dovf, (size_t)G, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        st = ESC_EDEVICE;
    int any = 0;
    if (st == ESC_OK)
        for (int32_t g = 0; g < G; g++) any |= flags[g];
    free(own);
    *any_overflow = any;
    return st;
}

esc_status batched_copy_u128(esc_ctx *c, esc_u128 *host_out) {
    const int32_t G = c->G;
    const int cnt = c->k == 4 ? 11 : 45;
    u128 *h = (u128 *)malloc(sizeof(u128) * COMBINE_ROW * (size_t)G);
    if (!h) return ESC_ENOMEM;
    esc_status st = ESC_OK;
    if (hipMemcpyAsync(h, c->buf[B_OUT], sizeof(u128) * COMBINE_ROW * (size_t)G, hipMemcpyDeviceToHost, c->stream) != hipSuccess ||
        hipStreamSynchronize(c->stream) != hipSuccess)
        st = ESC_EDEVICE;
    if (st == ESC_OK)
        for (int32_t g = 0; g < G; g++)
            for (int i = 0; i < cnt; i++) {
                const u128 x = h[(size_t)g * COMBINE_ROW + i];
                host_out[(size_t)g * cnt + i].lo = (uint64_t)x;
                host_out[(size_t)g * cnt + i].hi = (uint64_t)(x >> 64);
            }
    free(h);
    return st;
}
